// Internal helpers shared by the library's translation units: error
// reporting, workspace carving, HIP-event timing and small device utilities.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/lpr.h"

namespace lpr {

// Thread-local error text behind lpr_last_error().
void set_error(const char *fmt, ...);
void clear_error();

#define LPR_TRY_HIP(call)                                                   \
    do {                                                                    \
        hipError_t lpr_e_ = (call);                                         \
        if (lpr_e_ != hipSuccess) {                                         \
            ::lpr::set_error("%s failed: %s", #call,                        \
                             hipGetErrorString(lpr_e_));                    \
            return LPR_EDEVICE;                                             \
        }                                                                   \
    } while (0)

#define LPR_TRY(expr)                                                       \
    do {                                                                    \
        lpr_status lpr_s_ = (expr);                                         \
        if (lpr_s_ != LPR_OK) return lpr_s_;                                \
    } while (0)

// Bump allocator over the caller's workspace; every carve is 256-B aligned.
struct Carver {
    uintptr_t base = 0, cur = 0, end = 0;
    bool dry = true;  // sizing pass: no base pointer
    Carver() = default;
    Carver(void *p, size_t bytes)
        : base(reinterpret_cast<uintptr_t>(p)),
          cur(reinterpret_cast<uintptr_t>(p)),
          end(reinterpret_cast<uintptr_t>(p) + bytes),
          dry(p == nullptr) {}
    template <typename T>
    T *take(size_t count) {
        cur = (cur + 255) & ~uintptr_t(255);
        T *out = reinterpret_cast<T *>(cur);
        cur += count * sizeof(T);
        return dry ? nullptr : out;
    }
    size_t used() const { return (cur - base) + 256; }
    bool fits() const { return cur <= end; }
};

// Pairs of HIP events bracketing launches on one stream; the durations are
// harvested once the stream has been synchronised.
class EventTimer {
  public:
    explicit EventTimer(hipStream_t s) : stream_(s) {}
    ~EventTimer();
    bool enabled() const { return enabled_; }
    void enable() { enabled_ = true; }
    // Returns slot index or -1 if disabled.
    int begin();
    void end(int slot);
    // Sum (ms) of completed pairs of the given tag since the last harvest;
    // call only after the stream has been synchronised.
    lpr_status harvest(double *acc);

  private:
    hipStream_t stream_;
    bool enabled_ = false;
    std::vector<hipEvent_t> ev_;
    size_t used_ = 0;
    lpr_status err_ = LPR_OK;
    lpr_status ensure(size_t pairs);
};

// Scope timer of the whole call (two events).
class CallTimer {
  public:
    explicit CallTimer(hipStream_t s);
    ~CallTimer();
    void start();
    lpr_status stop_ms(double *ms);  // after sync

  private:
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Device utilities
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n);
__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n);

lpr_status fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
lpr_status fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);

// A second stream of the current device for this thread (default priority,
// non-blocking) with two events for forking work onto it and joining it
// back; created on the first call and kept until the process ends.
lpr_status side_stream(hipStream_t *side, hipEvent_t *fork, hipEvent_t *join);

namespace assign {
// The batched dense solve (lpr_assign_solve_batched) with its instance
// tables, counters and cost copies enqueued on `side` after `fork` (an event
// the caller recorded on `stream`), and the solve kernel on `stream` after
// them (through `join`).
lpr_status run_forked(int32_t B, const int32_t *n, const int64_t *cost_offset,
                      const int32_t *costs, int32_t maximize, int32_t *row_to_col,
                      int64_t *totals, int64_t *col_prices, const lpr_assign_opts *opts,
                      lpr_assign_stats *stats, void *workspace, size_t ws_bytes,
                      void *stream, hipStream_t side, hipEvent_t fork, hipEvent_t join);
}  // namespace assign

}  // namespace lpr
