// Measurement helper, not part of the method: the rate of non-returning
// device-scope 32-bit atomic adds to scattered addresses, the empirical
// ceiling against which the push updates of the grid solver are compared
// (no vendor figure exists for it).
#include "lpr_internal.h"

namespace lpr {

// Every thread adds 1 to `per_thread` counters chosen by its own xorshift32
// sequence (seeded from its global index); the adds return nothing.
__global__ __launch_bounds__(256) void k_atomic_probe(int32_t *cnt, uint32_t mask,
                                                      int32_t per_thread) {
    uint32_t s = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + 1u;
    for (int k = 0; k < per_thread; ++k) {
        s ^= s << 13;
        s ^= s >> 17;
        s ^= s << 5;
        atomicAdd(&cnt[s & mask], 1);
    }
}

}  // namespace lpr

extern "C" lpr_status lpr_atomic_probe(int32_t *counters, int32_t log2_counters,
                                       int32_t blocks, int32_t per_thread,
                                       double *ms, void *stream) {
    lpr::clear_error();
    if (!counters || !ms || log2_counters < 6 || log2_counters > 28 || blocks < 1 ||
        blocks > (1 << 20) || per_thread < 1 || per_thread > 4096) {
        lpr::set_error("invalid atomic probe arguments");
        return LPR_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    lpr::CallTimer call(s);
    call.start();
    hipLaunchKernelGGL(lpr::k_atomic_probe, dim3(blocks), dim3(256), 0, s, counters,
                       (uint32_t(1) << log2_counters) - 1u, per_thread);
    LPR_TRY_HIP(hipGetLastError());
    *ms = 0;
    LPR_TRY(call.stop_ms(ms));
    return LPR_OK;
}
