// Form 2: dense assignment by cost scaling with a lock-free refine, gfx950.
//
// Method (Section 5).  The assignment instance becomes a min-cost flow
// problem (arcs (x,y) with u = 1 and cost c(x,y), reverses (y,x) with u = 0
// and cost -c(x,y); excess +1 on X and -1 on Y).  The Min-Cost loop of
// Algorithm 5.0 runs Refine at eps <- max(1, floor(eps/alpha)) on costs scaled
// by S = 2n+1 until the refine at eps = 1 has run.  Refine is Algorithm 5.2:
// unmatch everything, set p(x) = -min_y {c'_p(x,y) + eps}, then apply the
// push/relabel operation of Algorithm 5.4 to active nodes until none is left:
// an active node scans its residual arcs for the least part-reduced cost
// c'_p(v,w) = c(v,w) - p(w); if c'_p + p(v) < 0 it pushes one unit along that
// arc with atomic excess updates, otherwise it relabels p(v) = -(c'_p + eps).
//
// GPU design.  One 1024-thread workgroup owns an instance for the whole
// solve; prices, excesses and the matching live in LDS, the cost matrix stays
// in global memory (L2 / MALL resident for the sizes served).  Active nodes
// are processed in alternating X and Y phases separated by workgroup
// barriers -- one admissible schedule of the lock-free method that keeps the
// prices a node reads fixed while it scans:
//   X phase: one wavefront per active x scans its cost row (lane-strided,
//     coalesced) and reduces (c'_p, y) to the minimum with the smallest y on
//     ties; it relabels if the best arc is not admissible (after which it is)
//     and pushes its unit: mate[x] = y~, atomic prepend of x to y~'s list of
//     matched rows, atomic increment of e(y~).
//   Y phase: one thread per y that became active (e(y) >= 1) applies the same
//     operation to y until e(y) = 0: its residual arcs are the reverses (y,x)
//     of its matched rows, the least c'_p(y,x) = -c(x,y) - p(x) is pushed back
//     (x unmatched, e(x) = 1) after a relabel when not admissible.
// The refine's initialisation and the first X phase share one scan of every
// row: after p(x) = -(min + eps) the minimising arc is admissible.
#include <algorithm>
#include <climits>
#include <numeric>
#include <vector>

#include "lpr_internal.h"

namespace lpr {
namespace assign {

constexpr int NT = 1024;
constexpr int NW = NT / 64;

struct AInst {
    int64_t cost_off;  // first cost entry of the instance
    int32_t n;
    int32_t row_off;   // offset of the instance in packed per-row outputs
};

struct AArgs {
    const AInst *inst;
    const int32_t *order;
    const int32_t *costs;
    int32_t sign;      // +1 minimise c, -1 maximise (solve with c = -w)
    int32_t alpha;
    int64_t eps0;      // 0: max|c| * S
    const int64_t *init_prices;
    int32_t *row_to_col;
    int64_t *totals;
    int64_t *col_prices;
    int64_t max_ops;
    uint64_t max_ticks;            // wall-clock budget in wall_clock64 ticks
    unsigned long long *counters;  // refines, phases, pushes, relabels, scans
    int32_t *status;  // per instance: 0 ok, 1 budget, 2 range, 3 internal
};

// Least (value, index) over one cost row: c'_p(x,y) = S*sign*c(x,y) - p(y),
// ties broken towards the smallest y.  Result valid in every lane.
__device__ inline void row_min(const int32_t *__restrict__ row,
                               const int64_t *py, int n, int64_t sgnS,
                               int lane, int64_t &best, int &arg) {
    int64_t b = LLONG_MAX;
    int a = INT_MAX;
    int y = lane;
    for (; y + 192 < n; y += 256) {
        const int32_t c0 = row[y], c1 = row[y + 64], c2 = row[y + 128],
                      c3 = row[y + 192];
        const int64_t v0 = int64_t(c0) * sgnS - py[y];
        const int64_t v1 = int64_t(c1) * sgnS - py[y + 64];
        const int64_t v2 = int64_t(c2) * sgnS - py[y + 128];
        const int64_t v3 = int64_t(c3) * sgnS - py[y + 192];
        if (v0 < b) { b = v0; a = y; }
        if (v1 < b) { b = v1; a = y + 64; }
        if (v2 < b) { b = v2; a = y + 128; }
        if (v3 < b) { b = v3; a = y + 192; }
    }
    for (; y < n; y += 64) {
        const int64_t v = int64_t(row[y]) * sgnS - py[y];
        if (v < b) { b = v; a = y; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t ob = __shfl_xor(b, o, 64);
        const int oa = __shfl_xor(a, o, 64);
        if (ob < b || (ob == b && oa < a)) {
            b = ob;
            a = oa;
        }
    }
    best = b;
    arg = a;
}

__global__ __launch_bounds__(NT) void k_assign(AArgs A) {
    const int slot = A.order[blockIdx.x];
    const AInst I = A.inst[slot];
    const int n = I.n;
    const int32_t *__restrict__ C = A.costs + I.cost_off;
    extern __shared__ __align__(16) unsigned char smem[];
    int64_t *py = reinterpret_cast<int64_t *>(smem);
    int64_t *px = py + n;
    int32_t *ey = reinterpret_cast<int32_t *>(px + n);
    int32_t *head = ey + n;
    int32_t *nxt = head + n;
    int32_t *mate = nxt + n;
    int32_t *xl = mate + n;  // rows pushed back in the last Y phase
    int32_t *yl = xl + n;    // columns made active in the last X phase
    __shared__ int s_nx, s_ny, s_stop;
    __shared__ unsigned long long s_cnt[5];
    __shared__ unsigned s_red[NW];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t t_start = wall_clock64();
    const int64_t S = 2 * int64_t(n) + 1;
    const int64_t sgnS = int64_t(A.sign) * S;

    // C = max |c| (Algorithm 5.0 starts at eps = C, here in scaled units)
    unsigned cmax = 0;
    const int64_t nn = int64_t(n) * n;
    for (int64_t k = tid; k < nn; k += NT) {
        const int32_t c = C[k];
        cmax = max(cmax, c < 0 ? 0u - unsigned(c) : unsigned(c));
    }
    for (int o = 32; o > 0; o >>= 1) cmax = max(cmax, (unsigned)__shfl_xor((int)cmax, o, 64));
    if (lane == 0) s_red[wave] = cmax;
    if (tid < 5) s_cnt[tid] = 0;
    if (tid == 0) {
        s_nx = 0;
        s_ny = 0;
        s_stop = 0;
    }
    for (int y = tid; y < n; y += NT)
        py[y] = A.init_prices ? A.init_prices[I.row_off + y] : 0;
    __syncthreads();
    cmax = 0;
    for (int i = 0; i < NW; ++i) cmax = max(cmax, s_red[i]);
    if (cmax > unsigned(LPR_ASSIGN_MAX_COST)) {
        if (tid == 0) A.status[slot] = 2;
        return;
    }
    int64_t eps = A.eps0 > 0 ? A.eps0 : (cmax > 0 ? int64_t(cmax) * S : 1);
    const int64_t alpha = A.alpha;

    for (;;) {
        eps = eps / alpha;
        if (eps < 1) eps = 1;
        // ---- Refine init (Algorithm 5.2): f <- 0, e(x) = 1, e(y) = -1 ----
        for (int y = tid; y < n; y += NT) {
            head[y] = -1;
            ey[y] = -1;
        }
        __syncthreads();
        // p(x) = -min_y {c'_p(x,y) + eps}; the minimising arc is then
        // admissible (c_p = -eps), so x pushes its unit along it at once.
        for (int x = wave; x < n; x += NW) {
            int64_t best;
            int arg;
            row_min(C + int64_t(x) * n, py, n, sgnS, lane, best, arg);
            if (lane == 0) {
                px[x] = -(best + eps);
                mate[x] = arg;
                nxt[x] = atomicExch(&head[arg], x);
                if (atomicAdd(&ey[arg], 1) == 0) yl[atomicAdd(&s_ny, 1)] = arg;
            }
        }
        if (tid == 0) {
            atomicAdd(&s_cnt[0], 1ull);
            atomicAdd(&s_cnt[2], (unsigned long long)n);
            atomicAdd(&s_cnt[4], (unsigned long long)n);
        }
        __syncthreads();
        for (;;) {
            // ---- Y phase: active columns push surplus rows back ----
            const int ny = s_ny;
            unsigned long long my_push = 0, my_rel = 0;
            for (int j = tid; j < ny; j += NT) {
                const int y = yl[j];
                const int64_t *pxc = px;
                while (ey[y] >= 1) {
                    int prev = -1, cur = head[y], bprev = -1, bx = -1;
                    int64_t bb = LLONG_MIN;
                    while (cur >= 0) {
                        // c'_p(y,x) = -c(x,y) - p(x); minimum <=> max b(x)
                        const int64_t b = int64_t(C[int64_t(cur) * n + y]) * sgnS + pxc[cur];
                        if (b > bb || (b == bb && cur < bx)) {
                            bb = b;
                            bx = cur;
                            bprev = prev;
                        }
                        prev = cur;
                        cur = nxt[cur];
                    }
                    if (bx < 0) {  // cannot happen: e(y) >= 1 means >= 2 rows
                        atomicOr(&s_stop, 2);
                        break;
                    }
                    if (!(bb > py[y])) {  // not admissible: relabel
                        py[y] = bb - eps;
                        ++my_rel;
                    }
                    if (bprev < 0) head[y] = nxt[bx];
                    else nxt[bprev] = nxt[bx];
                    mate[bx] = -1;
                    ey[y] -= 1;
                    ++my_push;
                    xl[atomicAdd(&s_nx, 1)] = bx;
                }
            }
            if (my_push) atomicAdd(&s_cnt[2], my_push);
            if (my_rel) atomicAdd(&s_cnt[3], my_rel);
            __syncthreads();
            const int nx = s_nx;
            if (tid == 0) {
                s_ny = 0;
                atomicAdd(&s_cnt[1], 1ull);
                if ((long long)(s_cnt[2] + s_cnt[3]) > A.max_ops ||
                    wall_clock64() - t_start > A.max_ticks)
                    s_stop = 1;
            }
            __syncthreads();
            const bool stop = s_stop != 0;
            if (tid == 0) s_nx = 0;
            if (nx == 0 || stop) break;
            // ---- X phase: every pushed-back row bids again ----
            unsigned long long x_rel = 0, x_ops = 0;
            for (int i = wave; i < nx; i += NW) {
                ++x_ops;
                const int x = xl[i];
                int64_t best;
                int arg;
                row_min(C + int64_t(x) * n, py, n, sgnS, lane, best, arg);
                if (lane == 0) {
                    if (best + px[x] >= 0) {  // relabel, then the arc is admissible
                        px[x] = -(best + eps);
                        ++x_rel;
                    }
                    mate[x] = arg;
                    nxt[x] = atomicExch(&head[arg], x);
                    if (atomicAdd(&ey[arg], 1) == 0) yl[atomicAdd(&s_ny, 1)] = arg;
                }
            }
            if (lane == 0 && x_ops) {
                atomicAdd(&s_cnt[4], x_ops);  // row scans
                atomicAdd(&s_cnt[2], x_ops);  // one push per scan
                if (x_rel) atomicAdd(&s_cnt[3], x_rel);
            }
            __syncthreads();
        }
        if (s_stop) break;
        if (eps == 1) break;
        __syncthreads();
    }
    __syncthreads();
    if (s_stop) {
        if (tid == 0) A.status[slot] = (s_stop & 2) ? 3 : 1;
    } else {
        long long part = 0;
        for (int x = tid; x < n; x += NT) {
            const int y = mate[x];
            A.row_to_col[I.row_off + x] = y;
            part += C[int64_t(x) * n + y];
        }
        if (A.col_prices)
            for (int y = tid; y < n; y += NT) A.col_prices[I.row_off + y] = py[y];
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
        __shared__ long long s_tot[NW];
        if (lane == 0) s_tot[wave] = part;
        __syncthreads();
        if (tid == 0) {
            long long tot = 0;
            for (int i = 0; i < NW; ++i) tot += s_tot[i];
            A.totals[slot] = tot;
            A.status[slot] = 0;
        }
    }
    if (tid < 5 && s_cnt[tid]) atomicAdd(&A.counters[tid], s_cnt[tid]);
}

static size_t lds_bytes(int nmax) { return size_t(nmax) * 44 + 64; }

struct Layout {
    AInst *inst;
    int32_t *order, *status;
    unsigned long long *counters;
};

static Carver carve(Carver cv, int B, Layout *L) {
    L->inst = cv.take<AInst>(size_t(B));
    L->order = cv.take<int32_t>(size_t(B));
    L->status = cv.take<int32_t>(size_t(B));
    L->counters = cv.take<unsigned long long>(8);
    return cv;
}

static size_t workspace_bytes(int B) {
    Layout L;
    return carve(Carver(), B, &L).used();
}

static lpr_status run(int32_t B, const int32_t *n, const int64_t *cost_offset,
                      const int32_t *costs, int32_t maximize,
                      int32_t *row_to_col, int64_t *totals, int64_t *col_prices,
                      const lpr_assign_opts *opts, lpr_assign_stats *stats,
                      void *workspace, size_t ws_bytes, void *stream) {
    clear_error();
    if (B < 1 || !n || !cost_offset || !costs || !row_to_col || !totals ||
        !workspace) {
        set_error("invalid arguments (NULL pointer or B < 1)");
        return LPR_EINVAL;
    }
    if (cost_offset[0] != 0) {
        set_error("cost_offset[0] must be 0");
        return LPR_EINVAL;
    }
    int nmax = 0;
    std::vector<AInst> insts(B);
    int64_t rows = 0;
    for (int b = 0; b < B; ++b) {
        if (n[b] < 1 || n[b] > LPR_ASSIGN_MAX_N) {
            set_error("instance %d: n = %d outside [1, %d]", b, n[b], LPR_ASSIGN_MAX_N);
            return LPR_EINVAL;
        }
        if (cost_offset[b + 1] != cost_offset[b] + int64_t(n[b]) * n[b]) {
            set_error("cost_offset is not the prefix sum of n^2 at %d", b);
            return LPR_EINVAL;
        }
        insts[b].cost_off = cost_offset[b];
        insts[b].n = n[b];
        insts[b].row_off = int32_t(rows);
        rows += n[b];
        nmax = std::max(nmax, n[b]);
    }
    if (rows >= (int64_t(1) << 31)) {
        set_error("too many rows");
        return LPR_EINVAL;
    }
    int32_t alpha = 8;
    int64_t eps0 = 0, max_ops = 64 * int64_t(nmax) * nmax + (int64_t(1) << 20);
    int64_t max_ms = 20000;
    const int64_t *init = nullptr;
    bool timing = false;
    if (opts) {
        if (opts->alpha) alpha = opts->alpha;
        eps0 = opts->eps0;
        init = opts->init_col_prices;
        if (opts->max_ops) max_ops = opts->max_ops;
        if (opts->max_ms) max_ms = opts->max_ms;
        timing = (opts->flags & LPR_ASSIGN_TIME_KERNELS) != 0;
    }
    if (alpha < 2 || eps0 < 0 || max_ops < 0 || max_ms < 0) {
        set_error("invalid lpr_assign_opts");
        return LPR_EINVAL;
    }
    if (ws_bytes < workspace_bytes(B)) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, workspace_bytes(B));
        return LPR_ENOMEM;
    }
    Layout L;
    carve(Carver(workspace, ws_bytes), B, &L);
    std::vector<int32_t> order(B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return n[a] > n[b]; });
    hipStream_t s = static_cast<hipStream_t>(stream);
    CallTimer call(s);
    call.start();
    LPR_TRY_HIP(hipMemcpyAsync(L.inst, insts.data(), sizeof(AInst) * B,
                               hipMemcpyHostToDevice, s));
    LPR_TRY_HIP(hipMemcpyAsync(L.order, order.data(), sizeof(int32_t) * B,
                               hipMemcpyHostToDevice, s));
    LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(L.counters), 0, 8, s));
    LPR_TRY(fill_i32(L.status, -1, B, s));
    AArgs A;
    A.inst = L.inst;
    A.order = L.order;
    A.costs = costs;
    A.sign = maximize ? -1 : 1;
    A.alpha = alpha;
    A.eps0 = eps0;
    A.init_prices = init;
    A.row_to_col = row_to_col;
    A.totals = totals;
    A.col_prices = col_prices;
    A.max_ops = max_ops;
    {
        int dev = 0, khz = 0;
        LPR_TRY_HIP(hipGetDevice(&dev));
        LPR_TRY_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        if (khz <= 0) khz = 100000;
        A.max_ticks = uint64_t(max_ms) * uint64_t(khz);
    }
    A.counters = L.counters;
    A.status = L.status;
    const size_t lds = lds_bytes(nmax);
    LPR_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_assign),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    int(lds)));
    EventTimer tk(s);
    if (timing) tk.enable();
    int ev = tk.begin();
    hipLaunchKernelGGL(k_assign, dim3(B), dim3(NT), lds, s, A);
    tk.end(ev);
    LPR_TRY_HIP(hipGetLastError());
    std::vector<int32_t> status(B);
    unsigned long long cnt[8];
    LPR_TRY_HIP(hipMemcpyAsync(status.data(), L.status, sizeof(int32_t) * B,
                               hipMemcpyDeviceToHost, s));
    LPR_TRY_HIP(hipMemcpyAsync(cnt, L.counters, sizeof(cnt),
                               hipMemcpyDeviceToHost, s));
    LPR_TRY_HIP(hipStreamSynchronize(s));
    double kms = 0, tms = 0;
    LPR_TRY(tk.harvest(&kms));
    LPR_TRY(call.stop_ms(&tms));
    if (stats) {
        stats->refines = int64_t(cnt[0]);
        stats->phases = int64_t(cnt[1]);
        stats->pushes = int64_t(cnt[2]);
        stats->relabels = int64_t(cnt[3]);
        stats->scans = int64_t(cnt[4]);
        stats->kernel_ms = kms;
        stats->total_ms = tms;
    }
    for (int b = 0; b < B; ++b) {
        if (status[b] == 2) {
            set_error("instance %d: |cost| exceeds LPR_ASSIGN_MAX_COST", b);
            return LPR_ERANGE;
        }
        if (status[b] == 1) {
            set_error("instance %d: operation or time budget exhausted", b);
            return LPR_EBUDGET;
        }
        if (status[b] == 3) {
            set_error("instance %d: internal inconsistency in the Y phase", b);
            return LPR_EDEVICE;
        }
        if (status[b] != 0) {
            set_error("instance %d: solver did not report completion", b);
            return LPR_EDEVICE;
        }
    }
    return LPR_OK;
}

}  // namespace assign
}  // namespace lpr

using namespace lpr;

extern "C" size_t lpr_assign_workspace(int32_t n) {
    if (n < 1) return 0;
    return assign::workspace_bytes(1);
}

extern "C" size_t lpr_assign_batched_workspace(int32_t B, const int32_t *n) {
    if (B < 1 || !n) return 0;
    return assign::workspace_bytes(B);
}

extern "C" lpr_status lpr_assign_solve(int32_t n, const int32_t *cost,
                                       int32_t maximize, int32_t *row_to_col,
                                       int64_t *total, int64_t *col_prices,
                                       const lpr_assign_opts *opts,
                                       lpr_assign_stats *stats, void *workspace,
                                       size_t workspace_bytes, void *stream) {
    if (n < 1 || n > LPR_ASSIGN_MAX_N) {
        clear_error();
        set_error("n = %d outside [1, %d]", n, LPR_ASSIGN_MAX_N);
        return LPR_EINVAL;
    }
    const int64_t off[2] = {0, int64_t(n) * n};
    return assign::run(1, &n, off, cost, maximize, row_to_col, total, col_prices,
                       opts, stats, workspace, workspace_bytes, stream);
}

extern "C" lpr_status lpr_assign_solve_batched(
    int32_t B, const int32_t *n, const int64_t *cost_offset,
    const int32_t *costs, int32_t maximize, int32_t *row_to_col,
    int64_t *totals, int64_t *col_prices, const lpr_assign_opts *opts,
    lpr_assign_stats *stats, void *workspace, size_t workspace_bytes,
    void *stream) {
    return assign::run(B, n, cost_offset, costs, maximize, row_to_col, totals,
                       col_prices, opts, stats, workspace, workspace_bytes,
                       stream);
}
