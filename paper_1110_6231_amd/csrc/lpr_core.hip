// Library-wide pieces of the C ABI: error text, version, event timing and
// fill kernels (used instead of hipMemsetAsync so that every clear is an
// ordinary kernel node).
#include <cstdio>
#include <cstring>

#include "lpr_internal.h"

namespace lpr {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

EventTimer::~EventTimer() {
    for (hipEvent_t e : ev_) (void)hipEventDestroy(e);
}

lpr_status EventTimer::ensure(size_t pairs) {
    while (ev_.size() < 2 * pairs) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) {
            set_error("hipEventCreate failed: %s", hipGetErrorString(r));
            return LPR_EDEVICE;
        }
        ev_.push_back(e);
    }
    return LPR_OK;
}

int EventTimer::begin() {
    if (!enabled_ || err_ != LPR_OK) return -1;
    if (ensure(used_ + 1) != LPR_OK) {
        err_ = LPR_EDEVICE;
        return -1;
    }
    int slot = int(used_++);
    if (hipEventRecord(ev_[2 * slot], stream_) != hipSuccess) err_ = LPR_EDEVICE;
    return slot;
}

void EventTimer::end(int slot) {
    if (slot < 0) return;
    if (hipEventRecord(ev_[2 * slot + 1], stream_) != hipSuccess)
        err_ = LPR_EDEVICE;
}

lpr_status EventTimer::harvest(double *acc) {
    if (!enabled_) return LPR_OK;
    if (err_ != LPR_OK) {
        set_error("event timing failed");
        return err_;
    }
    for (size_t i = 0; i < used_; ++i) {
        float ms = 0.f;
        hipError_t r = hipEventElapsedTime(&ms, ev_[2 * i], ev_[2 * i + 1]);
        if (r != hipSuccess) {
            set_error("hipEventElapsedTime failed: %s", hipGetErrorString(r));
            return LPR_EDEVICE;
        }
        *acc += ms;
    }
    used_ = 0;
    return LPR_OK;
}

CallTimer::CallTimer(hipStream_t s) : s_(s) {
    if (hipEventCreate(&a_) != hipSuccess) a_ = nullptr;
    if (hipEventCreate(&b_) != hipSuccess) b_ = nullptr;
}

CallTimer::~CallTimer() {
    if (a_) (void)hipEventDestroy(a_);
    if (b_) (void)hipEventDestroy(b_);
}

void CallTimer::start() {
    if (a_) (void)hipEventRecord(a_, s_);
}

lpr_status CallTimer::stop_ms(double *ms) {
    if (!a_ || !b_) return LPR_OK;
    LPR_TRY_HIP(hipEventRecord(b_, s_));
    LPR_TRY_HIP(hipEventSynchronize(b_));
    float f = 0.f;
    LPR_TRY_HIP(hipEventElapsedTime(&f, a_, b_));
    *ms = f;
    return LPR_OK;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

static int fill_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    return int(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

lpr_status fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return LPR_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
    LPR_TRY_HIP(hipGetLastError());
    return LPR_OK;
}

lpr_status fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return LPR_OK;
    hipLaunchKernelGGL(k_fill_i64, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
    LPR_TRY_HIP(hipGetLastError());
    return LPR_OK;
}

lpr_status side_stream(hipStream_t *side, hipEvent_t *fork, hipEvent_t *join) {
    struct Side {
        int dev;
        hipStream_t s;
        hipEvent_t fork, join;
    };
    static thread_local std::vector<Side> cache;
    int dev = 0;
    LPR_TRY_HIP(hipGetDevice(&dev));
    for (const Side &c : cache)
        if (c.dev == dev) {
            *side = c.s;
            *fork = c.fork;
            *join = c.join;
            return LPR_OK;
        }
    Side c{dev, nullptr, nullptr, nullptr};
    LPR_TRY_HIP(hipStreamCreateWithFlags(&c.s, hipStreamNonBlocking));
    LPR_TRY_HIP(hipEventCreateWithFlags(&c.fork, hipEventDisableTiming));
    LPR_TRY_HIP(hipEventCreateWithFlags(&c.join, hipEventDisableTiming));
    cache.push_back(c);
    *side = c.s;
    *fork = c.fork;
    *join = c.join;
    return LPR_OK;
}

}  // namespace lpr

extern "C" const char *lpr_last_error(void) { return lpr::g_err; }

extern "C" const char *lpr_version(void) { return "lpr 0.1.0 gfx950"; }
