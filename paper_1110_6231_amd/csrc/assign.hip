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
// GPU design.  A prep kernel spread over the whole GPU computes max|c| per
// instance and, where |c| < 2^15, a compact int16 copy of the costs (half the
// bytes per row scan; a 1024 x 1024 instance then fits one XCD's L2).  One
// 1024-thread workgroup then owns an instance for the whole solve; prices,
// excesses and the matching live in LDS.  Active nodes are processed in
// alternating X and Y phases separated by workgroup barriers -- one admissible
// schedule of the lock-free method that keeps the prices a node reads fixed
// while it scans:
//   X phase: one wavefront per active x scans its cost row (all loads in
//     flight at once) and reduces (c'_p, y) to a minimum with DPP exchanges;
//     it relabels if the best arc is not admissible (after which it is) and
//     pushes its unit: mate[x] = y~, atomic prepend of x to y~'s list of
//     matched rows, atomic increment of e(y~).
//   Y phase: one thread per y that became active (e(y) >= 1) applies the same
//     operation to y until e(y) = 0: its residual arcs are the reverses (y,x)
//     of its matched rows, the least c'_p(y,x) = -c(x,y) - p(x) is pushed back
//     (x unmatched, e(x) = 1) after a relabel when not admissible.
//   Serial tail: when at most `tail_rows` rows are active (the long chains at
//     the end of a refine), one wavefront runs pushes and push-backs back to
//     back with no block barrier -- a sequential trace of the same operations
//     -- and returns the queue to the phases if it grows.
// The refine's initialisation and the first X phase share one scan of every
// row: after p(x) = -(min + eps) the minimising arc is admissible.
//   Price update (Section 5, Algorithm 5.3): right after each refine's first
//     push of every row, and when the serial tail is entered after at least
//     `n` pushes since the last update, the workgroup runs a
//     Dijkstra search from the deficit columns over reversed residual arcs,
//     with arc length floor(c_p / eps) + 1 and Dial's buckets, until every
//     active node is labelled, and lowers each price by eps x its label
//     (unreached nodes by eps x (last label + 1)).  Shortest paths from the
//     active rows to deficit columns become admissible at once instead of
//     being found by one relabel at a time.  Column scans read a transposed
//     int16 copy of the costs.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "lpr_internal.h"

namespace lpr {
namespace assign {

constexpr int NT = 1024;
constexpr int NW = NT / 64;
constexpr int TAIL_EXIT = 8;   // back to phases when the queue grows past
                               // max(this, 4 x the entry threshold)
constexpr unsigned C16_MAX = 32767;
constexpr int NCNT = 16;       // statistics counters per solve
// Row stride of the int16 copies: rows padded to a multiple of 8 entries so
// that every row starts 16-byte aligned and is read with 16-byte loads.
__host__ __device__ inline int ld16(int n) { return (n + 7) & ~7; }
// Price of the padding columns of the int16 copies in the column-price
// array: a padded entry's part-reduced cost c*S*sign - p is then ~2^62,
// above every real one, so it never wins a row minimum.
constexpr int64_t PAD_PRICE = -(int64_t(1) << 62);

// Global-address-space views: loads through them are global (not flat)
// memory instructions, which do not wait on the LDS counter.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) v4i *gv4i_p;
typedef const __attribute__((address_space(1))) int32_t *gint32_p;

struct AInst {
    int64_t cost_off;  // first cost entry of the instance (int32 input)
    int64_t c16_off;   // sum of n x ld16(n) over the instances before it
    int32_t n;
    int32_t row_off;   // offset of the instance in packed per-row outputs
};

struct AArgs {
    const AInst *inst;
    const int32_t *order;
    const int32_t *costs;
    // Cost copies: instance b owns the 2 n ld16(n) int16 entries from
    // 2 c16_off.  When max|c| fits int16 they hold the row-major copy, then
    // the transposed copy (column y contiguous); otherwise a transposed int32
    // copy fills the same bytes.  Rows are ld16(n) entries apart throughout.
    const int16_t *c16;
    const unsigned *cmax;
    int32_t sign;      // +1 minimise c, -1 maximise (solve with c = -w)
    int32_t alpha;
    int64_t eps0;      // 0: max|c| * S
    const int64_t *eps0_inst;  // per-instance override, or null
    const int64_t *init_prices;
    int32_t *row_to_col;
    int64_t *totals;
    int64_t *col_prices;
    int64_t max_ops;
    int64_t warm_max_ops;          // > 0: budget of a warm start before it
                                   // restarts from the plain start; 0: the
                                   // default 2 n^2 + 2^16; < 0: never
    int64_t pu_period;             // pushes between price updates; 0: n pu_q / 4;
                                   // < 0: never
    int32_t pu_q;                  // q of the default period; 0: 2 up to
                                   // n = 512, 4 above
    int32_t tail_rows;             // serial tail threshold (active rows)
    int32_t pu_start;              // price update after each refine's first push
    int32_t arc_fixing;            // keep candidate lists of unfixed arcs
    int32_t fixing_shift;          // the bound divided by 2^fixing_shift
    int32_t sparse;                // the lists hold the instance's arcs: the
                                   // row scans read only them, always
    int32_t *cand;                 // per row: (y << 16 | c16(x,y)) of the arcs
                                   // not fixed yet, row stride ld16(n)
    int32_t *ncand;                // per row: number of them
    uint64_t max_ticks;            // wall-clock budget in wall_clock64 ticks
    unsigned long long *counters;  // refines, phases, pushes, relabels, scans,
                                   // price updates, wall-clock ticks in them,
                                   // fixing reruns, warm-start restarts,
                                   // cost entries read by row scans,
                                   // price-update steps
    int32_t *status;  // per instance: 0 ok, 1 budget, 2 range, 3 internal
};

// max|c| per instance and the saturated int16 copy with row stride ld16(n)
// (used only when max|c| fits; padding entries 0).  grid = (blocks per
// instance, B); a block takes every gridDim.x-th row.
__global__ __launch_bounds__(256) void k_prep(const AInst *inst,
                                              const int32_t *costs,
                                              int16_t *c16, unsigned *cmax) {
    const AInst I = inst[blockIdx.y];
    const int n = I.n, ld = ld16(n);
    unsigned m = 0;
    // PR rows x 512 columns per step with every load issued first (from a
    // clamped valid entry; padding columns store 0), then the stores: one
    // memory latency per step instead of one per row and column block
    constexpr int PR = 4;
    for (int r0 = blockIdx.x * PR; r0 < n; r0 += gridDim.x * PR) {
        for (int k0 = 0; k0 < ld; k0 += 512) {
            int32_t v[PR][2];
#pragma unroll
            for (int i = 0; i < PR; ++i) {
                const int32_t *src = costs + I.cost_off + int64_t(min(r0 + i, n - 1)) * n;
#pragma unroll
                for (int j = 0; j < 2; ++j) v[i][j] = src[min(k0 + int(threadIdx.x) + 256 * j, n - 1)];
            }
#pragma unroll
            for (int i = 0; i < PR; ++i) {
                if (r0 + i >= n) break;
                int16_t *dst = c16 + 2 * I.c16_off + int64_t(r0 + i) * ld;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int k = k0 + threadIdx.x + 256 * j;
                    if (k >= ld) break;
                    const int32_t c = k < n ? v[i][j] : 0;
                    m = max(m, c < 0 ? 0u - unsigned(c) : unsigned(c));
                    dst[k] = int16_t(max(-32768, min(32767, c)));
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) m = max(m, unsigned(__shfl_xor(int(m), o, 64)));
    __shared__ unsigned red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = max(max(red[0], red[1]), max(red[2], red[3]));
        if (m) atomicMax(&cmax[blockIdx.y], m);
    }
}

// Transposed copy of every instance's costs, through 64 x 64 LDS tiles, in
// int16 after the row-major copy when max|c| fits int16, else in int32 over
// both halves of the instance's region (row stride ld16(n) either way).
// Runs after k_prep, whose max|c| it reads.  grid = (B, tiles, tiles) over
// the largest instance.
__global__ __launch_bounds__(256) void k_transpose(const AInst *inst,
                                                   const int32_t *costs,
                                                   const unsigned *cmax,
                                                   int16_t *c16) {
    const AInst I = inst[blockIdx.x];
    const int n = I.n;
    const int c0 = blockIdx.y * 64, r0 = blockIdx.z * 64;  // source column / row
    const unsigned cm = cmax[blockIdx.x];
    if (c0 >= n || r0 >= n || cm > unsigned(LPR_ASSIGN_MAX_COST)) return;
    __shared__ int32_t tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    // the sixteen loads of a thread from clamped valid entries first, then
    // the zeros outside the matrix
    int32_t v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int row = min(r0 + ty + 4 * i, n - 1), col = min(c0 + tx, n - 1);
        v[i] = costs[I.cost_off + int64_t(row) * n + col];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r = ty + 4 * i;
        tile[r][tx] = r0 + r < n && c0 + tx < n ? v[i] : 0;
    }
    __syncthreads();
    const bool narrow = cm <= C16_MAX;
    int16_t *t16 = c16 + 2 * I.c16_off + int64_t(n) * ld16(n);
    int32_t *t32 = reinterpret_cast<int32_t *>(c16 + 2 * I.c16_off);
    for (int r = ty; r < 64; r += 4) {
        const int orow = c0 + r, ocol = r0 + tx;  // destination row = source column
        // padding columns (ocol in [n, ld16(n))) get the tile's zeros
        if (orow < n && ocol < ld16(n)) {
            const int64_t o = int64_t(orow) * ld16(n) + ocol;
            if (narrow)
                t16[o] = int16_t(tile[tx][r]);
            else
                t32[o] = tile[tx][r];
        }
    }
}

__device__ inline int64_t readlane64(int64_t v, int lane) {
    const int lo = __builtin_amdgcn_readlane(int(uint32_t(uint64_t(v))), lane);
    const int hi = __builtin_amdgcn_readlane(int(uint32_t(uint64_t(v) >> 32)), lane);
    return int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}

template <int CTRL>
__device__ inline int64_t dpp_min64(int64_t v) {
    const int lo = __builtin_amdgcn_mov_dpp(int(uint32_t(uint64_t(v))), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(int(uint32_t(uint64_t(v) >> 32)), CTRL, 0xf, 0xf, false);
    const int64_t o = int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
    return o < v ? o : v;
}

// Minimum of an int64 over the 64 lanes of a fully active wavefront, as a
// wave-uniform value: DPP exchanges inside each row of 16 lanes (xor 1,
// xor 2, half-row mirror, row mirror) and then the four row minima.
__device__ inline int64_t wave_min64(int64_t v) {
    v = dpp_min64<0xB1>(v);   // quad_perm [1,0,3,2]
    v = dpp_min64<0x4E>(v);   // quad_perm [2,3,0,1]
    v = dpp_min64<0x141>(v);  // row_half_mirror
    v = dpp_min64<0x140>(v);  // row_mirror
    int64_t m = readlane64(v, 0);
    const int64_t m1 = readlane64(v, 16), m2 = readlane64(v, 32),
                  m3 = readlane64(v, 48);
    m = m1 < m ? m1 : m;
    m = m2 < m ? m2 : m;
    return m3 < m ? m3 : m;
}

// Per-lane part of the row scan: int32 costs (row stride n, any
// alignment).  Branch-free: out-of-range columns read p(0) and are masked.
__device__ inline void lane_scan(const int32_t *__restrict__ row,
                                 const int64_t *py, int n, int32_t sgnS,
                                 int lane, int64_t &b, int &a, int &ca) {
    const gint32_p g = (gint32_p)row;
    for (int base = 0; base < n; base += 1024) {
        int32_t cv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int y = base + lane + 64 * i;
            cv[i] = g[y < n ? y : 0];
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int y = base + lane + 64 * i;
            const bool ok = y < n;
            const int64_t v = int64_t(cv[i]) * sgnS - py[ok ? y : 0];
            if (ok && v < b) {
                b = v;
                a = y;
                ca = cv[i];
            }
        }
    }
}

// Per-lane part of the row scan: int16 costs, row stride ld16(n), every row
// 16-byte aligned (8 costs per load).  |c| <= 32768 and |S| <= 4097, so
// c * S*sign is a 24 x 24-bit product; the padding columns carry PAD_PRICE
// and never win.
__device__ inline void lane_scan(const int16_t *__restrict__ row,
                                 const int64_t *py, int n, int32_t sgnS,
                                 int lane, int64_t &b, int &a, int &ca) {
    const gv4i_p g = (gv4i_p)row;
    const int no = ld16(n) >> 3;
    for (int base = 0; base < no; base += 128) {
        v4i cv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int q = base + lane + 64 * i;
            cv[i] = q < no ? g[q] : v4i{0, 0, 0, 0};
        }
        // the chunk's minimum keeps the entry's position as a constant
        // (8 i + j); the column is rebuilt once at the end
        int64_t bl = b;
        int al = -1, cl = 0;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int q = base + lane + 64 * i;
            if (q < no) {
                const int y = 8 * q;
                const int w[4] = {cv[i].x, cv[i].y, cv[i].z, cv[i].w};
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int c = j & 1 ? w[j >> 1] >> 16 : int(int16_t(w[j >> 1] & 0xffff));
                    const int64_t v = int64_t(__mul24(c, sgnS)) - py[y + j];
                    if (v < bl) {
                        bl = v;
                        al = 8 * i + j;
                        cl = c;
                    }
                }
            }
        }
        if (al >= 0) {
            b = bl;
            a = 8 * (base + lane) + 512 * (al >> 3) + (al & 7);
            ca = cl;
        }
    }
}

// Least part-reduced cost over one cost row, c'_p(x,y) = S*sign*c(x,y) - p(y),
// with an argmin y~ and c(x, y~).  Every load of a 1024-column chunk is in
// flight before any is consumed, so a scan costs one memory round trip per
// chunk.  Results are wave-uniform.  Called by all 64 lanes of a wavefront.
template <typename T>
__device__ inline void row_min(const T *__restrict__ row, const int64_t *py,
                               int n, int64_t sgnS, int lane, int64_t &best,
                               int &arg, int &carg) {
    int64_t b = LLONG_MAX;
    int a = 0, ca = 0;
    // |S*sign| <= 2*2048+1 fits 32 bits
    lane_scan(row, py, n, int32_t(sgnS), lane, b, a, ca);
    const int64_t m = wave_min64(b);
    const unsigned long long hit = __ballot(b == m);
    const int src = __ffsll((long long)hit) - 1;
    best = m;
    arg = __builtin_amdgcn_readlane(a, src);
    carg = __builtin_amdgcn_readlane(ca, src);
}

// Row minimum over a candidate list: entries (y << 16) | (c(x,y) & 0xffff) of
// int16 costs, K of them.  Same value as the full scan when the list holds
// the row's minimising column; ties go to the smallest column of a lane's
// entries, then to the lowest lane.
__device__ inline void row_min_list(const int32_t *__restrict__ list, int K,
                                    const int64_t *py, int64_t sgnS, int lane,
                                    int64_t &best, int &arg, int &carg) {
    int64_t b = LLONG_MAX;
    int a = 0, ca = 0;
    for (int k = lane; k < K; k += 64) {
        const int w = list[k];
        const int y = int(uint32_t(w) >> 16);
        const int c = int(int16_t(w & 0xffff));
        const int64_t v = int64_t(__mul24(c, int32_t(sgnS))) - py[y];
        if (v < b || (v == b && y < a)) {
            b = v;
            a = y;
            ca = c;
        }
    }
    const int64_t m = wave_min64(b);
    const unsigned long long hit = __ballot(b == m);
    const int src = __ffsll((long long)hit) - 1;
    best = m;
    arg = __builtin_amdgcn_readlane(a, src);
    carg = __builtin_amdgcn_readlane(ca, src);
}

struct Shared {
    int64_t *py, *px;
    int64_t *bv;  // b(x) = c(x, mate[x]) * S*sign + p(x), fixed while matched
    int32_t *ey, *head, *nxt, *mate, *xl, *yl;
};

// Operation of Algorithm 5.4 applied to an active column y until e(y) = 0.
// Its residual arcs are the reverses (y,x) of its matched rows, with
// c'_p(y,x) = -c(x,y) - p(x); the least one (largest b(x) = c(x,y) + p(x),
// ties to the smallest x; p(x) cannot change while x is matched, so b(x) is
// recorded when x pushes) is pushed back, after a relabel
// p(y) = -(c'_p + eps) when it is not admissible.  Every pushed-back row is
// handed to `emit`.  Only the caller touches y's list while this runs.
template <typename Emit>
__device__ inline bool resolve_column(int y, int64_t eps, const Shared &L,
                                      unsigned long long &pushes,
                                      unsigned long long &relabels, Emit emit) {
    while (L.ey[y] >= 1) {
        int prev = -1, cur = L.head[y], bprev = -1, bx = -1;
        int64_t bb = LLONG_MIN;
        while (cur >= 0) {
            const int64_t b = L.bv[cur];
            if (b > bb || (b == bb && cur < bx)) {
                bb = b;
                bx = cur;
                bprev = prev;
            }
            prev = cur;
            cur = L.nxt[cur];
        }
        if (bx < 0) return false;  // e(y) >= 1 implies >= 2 matched rows
        if (!(bb > L.py[y])) {     // not admissible: relabel
            L.py[y] = bb - eps;
            ++relabels;
        }
        if (bprev < 0) L.head[y] = L.nxt[bx];
        else L.nxt[bprev] = L.nxt[bx];
        L.mate[bx] = -1;
        L.ey[y] -= 1;
        ++pushes;
        emit(bx);
    }
    return true;
}

// Division by a fixed eps >= 1 without a 64-bit integer divide per call
// (a software sequence of ~100 instructions on this hardware): the quotient
// is estimated through a double reciprocal and corrected to the exact floor
// by its integer remainder.  Exact for |a| < 2^62: double(a) is within 2^9 of
// a there, so the first estimate is within 2^9 / eps + 2 of the quotient and
// leaves a remainder below 2^9 + 3 eps in magnitude; a second estimate on that
// remainder has a relative error near 2^-52, so it is off by at most one, and
// each correction loop below runs at most one step.
struct EpsDiv {
    int64_t eps, kmax;  // kmax = floor(LLONG_MAX / eps)
    double inv;
    __device__ explicit EpsDiv(int64_t e)
        : eps(e), kmax(LLONG_MAX / e), inv(1.0 / double(e)) {}
    __device__ int64_t floor_div(int64_t a) const {
        int64_t q = int64_t(floor(double(a) * inv));
        int64_t r = a - q * eps;
        q += int64_t(floor(double(r) * inv));
        r = a - q * eps;
        while (r < 0) {
            --q;
            r += eps;
        }
        while (r >= eps) {
            ++q;
            r -= eps;
        }
        return q;
    }
    // eps * k, saturated (k >= -1)
    __device__ int64_t mul_sat(int64_t k) const { return k > kmax ? LLONG_MAX : eps * k; }
};

constexpr int PU_LOADS = 16;  // column loads in flight per thread in a price update

struct PU {
    int64_t *lx, *ly;  // labels (multiples of eps), LLONG_MAX = none yet
    uint8_t *fx, *fy;  // scanned
};

// Price update heuristic (Algorithm 5.3).  Buckets are the distinct label
// values: after the nodes of one label are scanned, the next label is the
// least tentative label of an unscanned node (a workgroup minimum), so the
// number of steps is the number of distinct labels, not their range.  The
// bucket of the deficit columns is 0; scanning a column y offers every row x
// with a residual arc (x, y) (every x not matched to y) the label
// level + floor(c_p(x,y) / eps) + 1; scanning a row x offers its mate the
// label level + floor(c_p(mate, x) / eps) + 1 (the reverse arc of the matched
// pair).  An eps-optimal pseudoflow has c_p >= -eps on residual arcs, so
// offers never fall below the current level.  The search stops once every
// active node (unmatched row, column with e >= 1) is scanned and the current
// bucket is empty; prices drop by eps x label, and by eps x (last label + 1)
// for the nodes not scanned.
// Called by the whole workgroup between phases; `fl` is n ints of scratch
// for the column frontier.  Returns the number of steps (labels scanned).
template <typename T>
__device__ int price_update(const Shared &L, const PU &U, int32_t *fl,
                            const T *__restrict__ CT, int n, int64_t sgnS,
                            int64_t eps, int tid) {
    // per-level shared values, double-buffered by level parity so that no
    // barrier is spent resetting them and every read precedes the next write:
    // frontier size, active nodes scanned, next level
    __shared__ int s_rem, s_nf[2], s_dec[2];
    __shared__ unsigned long long s_next[2];
    constexpr int64_t NONE = LLONG_MAX;
    const EpsDiv D(eps);
    if (tid == 0) {
        s_rem = 0;
        s_nf[0] = 0;
        s_dec[0] = 0;
        s_next[0] = ULLONG_MAX;
    }
    __syncthreads();
    int rem = 0;
    for (int x = tid; x < n; x += NT) {
        U.lx[x] = NONE;
        U.fx[x] = 0;
        rem += L.mate[x] < 0;
    }
    for (int y = tid; y < n; y += NT) {
        U.ly[y] = L.ey[y] < 0 ? 0 : NONE;
        U.fy[y] = 0;
        rem += L.ey[y] >= 1;
    }
    if (rem) atomicAdd(&s_rem, rem);
    __syncthreads();
    int left = s_rem;  // active nodes not scanned yet (same in every thread)
    int64_t level = 0;
    int par = 0, steps = 0;
    for (;;) {
        ++steps;
        // columns labelled `level`
        for (int y = tid; y < n; y += NT)
            if (!U.fy[y] && U.ly[y] == level) {
                U.fy[y] = 1;
                fl[atomicAdd(&s_nf[par], 1)] = y;
                if (L.ey[y] >= 1) atomicAdd(&s_dec[par], 1);
            }
        __syncthreads();
        if (tid == 0) {  // the other parity's slots are read by nobody now
            s_nf[par ^ 1] = 0;
            s_dec[par ^ 1] = 0;
            s_next[par ^ 1] = ULLONG_MAX;
        }
        const int nf = s_nf[par];
        if (nf > 0) {
            for (int x = tid; x < n; x += NT) {
                if (U.fx[x]) continue;
                int64_t best = U.lx[x];
                // an offer improves iff c_p < eps * (best - level - 1)
                int64_t bound = best == NONE ? NONE : D.mul_sat(best - level - 1);
                const int64_t pxx = L.px[x];
                const int mx = L.mate[x];
                // PU_LOADS column loads in flight before any is used
                for (int j0 = 0; j0 < nf; j0 += PU_LOADS) {
                    int cv[PU_LOADS];
#pragma unroll
                    for (int k = 0; k < PU_LOADS; ++k)
                        cv[k] = j0 + k < nf ? int(CT[int64_t(fl[j0 + k]) * ld16(n) + x]) : 0;
#pragma unroll
                    for (int k = 0; k < PU_LOADS; ++k) {
                        if (j0 + k >= nf) break;
                        const int y = fl[j0 + k];
                        // int16 costs take a 24 x 24-bit product, int32 a 64-bit one
                        const int64_t cs = sizeof(T) == 2
                                               ? int64_t(__mul24(cv[k], int(sgnS)))
                                               : int64_t(cv[k]) * sgnS;
                        const int64_t cp = cs + pxx - L.py[y];
                        if (cp < bound && y != mx) {
                            // c_p >= -eps on every arc of an eps-optimal
                            // pseudoflow, so the clamp only acts on the
                            // missing arcs of a sparse instance (which are
                            // not kept eps-optimal): Dial's buckets need
                            // lengths >= 0
                            best = level + max(int64_t(0), D.floor_div(cp) + 1);
                            bound = D.mul_sat(best - level - 1);
                        }
                    }
                }
                U.lx[x] = best;
            }
        }
        __syncthreads();
        // rows labelled `level` offer their mates a label; at the same time
        // the least label of any node still unscanned (including those
        // offers) is the next bucket, `level` again if an offer equals it
        unsigned long long m = ULLONG_MAX;
        for (int x = tid; x < n; x += NT) {
            if (U.fx[x]) continue;
            if (U.lx[x] != level) {
                m = min(m, (unsigned long long)U.lx[x]);
                continue;
            }
            U.fx[x] = 1;
            const int y = L.mate[x];
            if (y < 0) {
                atomicAdd(&s_dec[par], 1);
                continue;
            }
            if (U.fy[y]) continue;
            // c_p(y, x) = -c(x,y) + p(y) - p(x) = p(y) - b(x)
            const int64_t cand = level + D.floor_div(L.py[y] - L.bv[x]) + 1;
            atomicMin(reinterpret_cast<unsigned long long *>(&U.ly[y]),
                      (unsigned long long)cand);
            m = min(m, (unsigned long long)cand);
        }
        // a column's label only drops to an offer counted above, so a stale
        // read here is still bounded by the true minimum
        for (int y = tid; y < n; y += NT)
            if (!U.fy[y]) m = min(m, (unsigned long long)U.ly[y]);
        // every label and offer is at most NONE, which also stands for
        // "nothing" here: the wavefront minimum by DPP
        const int64_t wm = wave_min64(int64_t(min(m, (unsigned long long)NONE)));
        if ((tid & 63) == 0 && wm < NONE) atomicMin(&s_next[par], (unsigned long long)wm);
        __syncthreads();
        const unsigned long long next = s_next[par];
        left -= s_dec[par];
        if (next >= (unsigned long long)NONE) break;  // nothing left to reach
        // stop once every active node is scanned and the bucket is empty
        if (left <= 0 && int64_t(next) > level) break;
        level = int64_t(next);
        par ^= 1;
    }
    const int64_t far = level + 1;
    for (int x = tid; x < n; x += NT) {
        const int64_t dp = eps * (U.fx[x] ? U.lx[x] : far);
        L.px[x] -= dp;
        if (L.mate[x] >= 0) L.bv[x] -= dp;
    }
    for (int y = tid; y < n; y += NT) L.py[y] -= eps * (U.fy[y] ? U.ly[y] : far);
    __syncthreads();
    return steps;
}

// Arc fixing (Section 5's second heuristic): for an eps-optimal flow, an arc
// whose reduced cost exceeds 2 |V| eps never changes its flow again.  At the
// end of a refine the flow is a perfect matching, eps-optimal with the
// current prices, and for row x every c_p(x,y) >= -eps, so c_p(x,y) >=
// r(x,y) - eps with r(x,y) = c'_p(x,y) - min_y' c'_p(x,y').  The row keeps
// the arcs with r < keep_r = (2 |V| + 2) eps (|V| = 2n) and its
// matched arc; later row scans read only that list (which holds the row's
// minimising column whenever the fixed arcs are indeed never used).  Every
// wavefront compacts its rows in place; called by every thread, no barrier.
__device__ void fix_arcs(const int16_t *__restrict__ C, int ldc, int32_t *cand,
                         int32_t *ncand, bool lists, const int64_t *py,
                         const int32_t *mate, int n, int64_t sgnS, int64_t keep_r,
                         int wave, int lane) {
    for (int x = wave; x < n; x += NW) {
        int32_t *list = cand + int64_t(x) * ldc;
        const int16_t *row = C + int64_t(x) * ldc;
        const int K = lists ? ncand[x] : n;
        const int mx = mate[x];
        int64_t b = LLONG_MAX;
        for (int k = lane; k < K; k += 64) {
            const int w = lists ? list[k] : 0;
            const int y = lists ? int(uint32_t(w) >> 16) : k;
            const int c = lists ? int(int16_t(w & 0xffff)) : int(row[k]);
            const int64_t v = int64_t(__mul24(c, int32_t(sgnS))) - py[y];
            b = v < b ? v : b;
        }
        const int64_t m = wave_min64(b);
        int out = 0;
        for (int k0 = 0; k0 < K; k0 += 64) {
            const int k = k0 + lane;
            int w = 0;
            bool keep = false;
            if (k < K) {
                const int lw = lists ? list[k] : 0;
                const int y = lists ? int(uint32_t(lw) >> 16) : k;
                const int c = lists ? int(int16_t(lw & 0xffff)) : int(row[k]);
                const int64_t v = int64_t(__mul24(c, int32_t(sgnS))) - py[y];
                keep = v - m < keep_r || y == mx;
                w = (y << 16) | (c & 0xffff);
            }
            // every lane has read its entry before any lane writes (the
            // ballot), and the write position never passes k0 + 63
            const unsigned long long bal = __ballot(keep);
            if (keep) list[out + __popcll(bal & ((1ull << lane) - 1))] = w;
            out += __popcll(bal);
        }
        if (lane == 0) ncand[x] = out;
    }
}

// 1 if some row's matched arc is not within 2 (scaled units) of its row
// minimum over all columns, i.e. the final matching is not 1-optimal for any
// row prices; else 0.  Full scans of every row.  Called by every thread.
template <typename T>
__device__ bool not_one_optimal(const T *__restrict__ C, int ldc, const int64_t *py,
                                const int32_t *mate, int n, int64_t sgnS, int wave,
                                int lane, int *flag) {
    for (int x = wave; x < n; x += NW) {
        int64_t best;
        int arg, carg;
        row_min(C + int64_t(x) * ldc, py, n, sgnS, lane, best, arg, carg);
        if (lane == 0) {
            const int y = mate[x];
            const int64_t cm = int64_t(C[int64_t(x) * ldc + y]) * sgnS - py[y];
            if (cm - best > 2) atomicOr(flag, 1);
        }
    }
    __syncthreads();
    return *flag != 0;
}

constexpr int HOT = 64;  // columns with e(y) >= HOT are resolved by the workgroup

// The same operation as resolve_column for a column with many matched rows
// (every row preferring one column makes e(y) ~ n, and the one-thread list
// walk per push-back is then quadratic), by the whole workgroup: the matched
// rows are gathered from mate[], bitonic-sorted by b(x) descending (ties:
// smaller x first) -- exactly the order resolve_column pushes them back in --
// and one thread then applies the relabels of that sequence; the first
// e(y) rows are pushed back (appended to the row list at *nx) and the last
// one stays.  `idx` is LDS scratch for 2n ints.  Called by every thread.
__device__ bool resolve_hot(int y, int64_t eps, const Shared &L, int32_t *idx,
                            int n, int *nx, int tid, unsigned long long &pushes,
                            unsigned long long &relabels) {
    __shared__ int s_k, s_base, s_bad;
    __shared__ unsigned long long s_rel;
    if (tid == 0) {
        s_k = 0;
        s_bad = 0;
        s_rel = 0;
    }
    __syncthreads();
    for (int x = tid; x < n; x += NT)
        if (L.mate[x] == y) idx[atomicAdd(&s_k, 1)] = x;
    __syncthreads();
    const int k = s_k;
    int m = 1;
    while (m < k) m <<= 1;
    for (int i = k + tid; i < m; i += NT) idx[i] = -1;  // padding sorts last
    __syncthreads();
    // a goes before b: larger b(x), then smaller x; padding last
    auto before = [&](int a, int b) {
        if (a < 0) return false;
        if (b < 0) return true;
        const int64_t ba = L.bv[a], bb = L.bv[b];
        return ba > bb || (ba == bb && a < b);
    };
    for (int size = 2; size <= m; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < (m >> 1); i += NT) {
                const int lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1));
                const int hi = lo + stride;
                const int a = idx[lo], b = idx[hi];
                const bool up = (lo & size) == 0;
                if (up ? before(b, a) : before(a, b)) {
                    idx[lo] = b;
                    idx[hi] = a;
                }
            }
            __syncthreads();
        }
    if (tid == 0) {
        if (k < 2 || k != L.ey[y] + 1) {
            s_bad = 1;
        } else {
            int64_t p = L.py[y];
            unsigned long long rel = 0;
            for (int i = 0; i < k - 1; ++i) {
                const int64_t b = L.bv[idx[i]];
                if (!(b > p)) {  // not admissible: relabel p(y) = b - eps
                    p = b - eps;
                    ++rel;
                }
            }
            L.py[y] = p;
            const int keep = idx[k - 1];
            L.head[y] = keep;
            L.nxt[keep] = -1;
            L.ey[y] = 0;
            s_base = atomicAdd(nx, k - 1);
            s_rel = rel;
        }
    }
    __syncthreads();
    if (s_bad) return false;
    const int base = s_base;
    for (int i = tid; i < k - 1; i += NT) {
        const int x = idx[i];
        L.mate[x] = -1;
        L.xl[base + i] = x;
    }
    if (tid == 0) {
        pushes += (unsigned long long)(k - 1);
        relabels += s_rel;
    }
    __syncthreads();
    return true;
}

template <typename T>
__device__ void solve_instance(const AArgs &A, const AInst &I, int slot,
                               const T *__restrict__ C,
                               const T *__restrict__ CT, unsigned cmax,
                               unsigned char *smem) {
    const int n = I.n;
    Shared L;
    // rows of the int16 copies are padded to ld16(n) entries
    const int ldc = sizeof(T) == 2 ? ld16(n) : n;
    L.py = reinterpret_cast<int64_t *>(smem);
    L.px = L.py + ld16(n);
    L.bv = L.px + n;
    L.ey = reinterpret_cast<int32_t *>(L.bv + n);
    L.head = L.ey + n;
    L.nxt = L.head + n;
    L.mate = L.nxt + n;
    L.xl = L.mate + n;  // active rows (circular queue in the serial tail)
    L.yl = L.xl + n;    // columns made active by the last X phase
    PU U;
    U.lx = reinterpret_cast<int64_t *>(L.yl + n);
    U.ly = U.lx + n;
    U.fx = reinterpret_cast<uint8_t *>(U.ly + n);
    U.fy = U.fx + n;
    int64_t *py = L.py, *px = L.px;
    const int pu_q = A.pu_q > 0 ? A.pu_q : (n > 512 ? 4 : 2);
    const unsigned long long period =
        A.pu_period > 0 ? (unsigned long long)A.pu_period
                        : (unsigned long long)max(1, n * pu_q / 4);
    if (A.pu_period < 0) CT = nullptr;
    // the tail's cost per operation grows with n (one row scan), a phase's
    // barrier cost does not
    const int tail_enter = A.tail_rows > 0 ? A.tail_rows : min(32, max(8, 8192 / n));
    const int tail_exit = max(TAIL_EXIT, 4 * tail_enter);
    __shared__ int s_nx, s_ny, s_stop, s_qh, s_nh;
    __shared__ unsigned long long s_pu_mark;  // pushes at the last price update
    __shared__ unsigned long long s_cnt[NCNT];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t t_start = wall_clock64();
    const int64_t S = 2 * int64_t(n) + 1;
    const int64_t sgnS = int64_t(A.sign) * S;
    if (tid < NCNT) s_cnt[tid] = 0;
    if (tid == 0) {
        s_nx = 0;
        s_ny = 0;
        s_stop = 0;
        s_qh = 0;
        s_nh = 0;
        s_pu_mark = 0;
    }
    for (int y = tid; y < n; y += NT)
        py[y] = A.init_prices ? A.init_prices[I.row_off + y] : 0;
    if (tid < ld16(n) - n) py[n + tid] = PAD_PRICE;
    __syncthreads();
    // Algorithm 5.0 starts at eps = C (largest |cost|), here in scaled units
    const int64_t eps_plain = cmax > 0 ? int64_t(cmax) * S : 1;
    int64_t eps = A.eps0 > 0 ? A.eps0 : eps_plain;
    if (A.eps0_inst && A.eps0_inst[slot] > 0) eps = A.eps0_inst[slot];
    // A start from given prices or a given epsilon is a guess: exactness
    // never depends on it (every refine recomputes p(X) from p(Y), Algorithm
    // 5.2), but a poor guess can cost far more operations than the plain
    // start.  Past its budget the instance restarts once from the plain
    // start (p = 0, eps = max|c| S), which is thus both the fallback and the
    // judge of the guess.  `on_warm` is the same in every thread.
    bool on_warm = A.warm_max_ops >= 0 &&
                   (A.init_prices != nullptr || A.eps0 > 0 ||
                    (A.eps0_inst && A.eps0_inst[slot] > 0));
    const long long warm_budget =
        A.warm_max_ops > 0 ? (long long)A.warm_max_ops
                           : 2ll * n * n + (1ll << 16);
    const int64_t alpha = A.alpha;
    // candidate lists of unfixed arcs (int16 costs only); `lists` is the same
    // in every thread
    const bool fixing = sizeof(T) == 2 && A.arc_fixing && A.cand;
    const bool sparse = sizeof(T) == 2 && A.sparse;
    int32_t *cand = fixing || sparse ? A.cand + I.c16_off : nullptr;
    int32_t *ncand = fixing || sparse ? A.ncand + I.row_off : nullptr;
    bool lists = sparse;
    __shared__ int s_bad;
    // the least part-reduced cost of row x over its candidates (all columns
    // without lists)
    auto scan = [&](int x, int64_t &best, int &arg, int &carg) {
        if (lists)
            row_min_list(cand + int64_t(x) * ldc, ncand[x], py, sgnS, lane, best, arg,
                         carg);
        else
            row_min(C + int64_t(x) * ldc, py, n, sgnS, lane, best, arg, carg);
    };

    for (;;) {
        eps = eps / alpha;
        if (eps < 1) eps = 1;
        // ---- Refine init (Algorithm 5.2): f <- 0, e(x) = 1, e(y) = -1 ----
        for (int y = tid; y < n; y += NT) {
            L.head[y] = -1;
            L.ey[y] = -1;
        }
        __syncthreads();
        // p(x) = -min_y {c'_p(x,y) + eps}; the minimising arc is then
        // admissible (c_p = -eps), so x pushes its unit along it at once.
        for (int x = wave; x < n; x += NW) {
            int64_t best;
            int arg, carg;
            scan(x, best, arg, carg);
            if (lane == 0) {
                px[x] = -(best + eps);
                L.mate[x] = arg;
                L.bv[x] = int64_t(carg) * sgnS + px[x];
                L.nxt[x] = atomicExch(&L.head[arg], x);
                if (atomicAdd(&L.ey[arg], 1) == 0) L.yl[atomicAdd(&s_ny, 1)] = arg;
            }
        }
        if (tid == 0) {
            atomicAdd(&s_cnt[0], 1ull);
            atomicAdd(&s_cnt[2], (unsigned long long)n);
            atomicAdd(&s_cnt[4], (unsigned long long)n);
        }
        __syncthreads();
        if (CT && A.pu_start && s_ny > 0) {
            // every row is matched here, so the row list is free scratch
            const uint64_t t0 = wall_clock64();
            const int steps = price_update(L, U, L.xl, CT, n, sgnS, eps, tid);
            if (tid == 0) {
                s_pu_mark = s_cnt[2];
                atomicAdd(&s_cnt[5], 1ull);
                atomicAdd(&s_cnt[6], (unsigned long long)(wall_clock64() - t0));
                atomicAdd(&s_cnt[10], (unsigned long long)steps);
            }
            __syncthreads();
        }
        for (;;) {
            // ---- Y phase: active columns push surplus rows back ----
            const int ny = s_ny;
            unsigned long long my_push = 0, my_rel = 0;
            int32_t *hot = reinterpret_cast<int32_t *>(U.ly);  // free outside updates
            // entry j goes to lane j / NW of wavefront j % NW, so that a few
            // active columns are spread over the wavefronts rather than
            // walking their lists in the lanes of one
            for (int j = (tid & 63) * NW + (tid >> 6); j < ny; j += NT) {
                const int y = L.yl[j];
                if (L.ey[y] >= HOT) {
                    hot[atomicAdd(&s_nh, 1)] = y;
                    continue;
                }
                const bool ok = resolve_column(
                    y, eps, L, my_push, my_rel,
                    [&](int bx) { L.xl[atomicAdd(&s_nx, 1)] = bx; });
                if (!ok) atomicOr(&s_stop, 2);
            }
            __syncthreads();
            const int nh = s_nh;
            for (int j = 0; j < nh; ++j)
                if (!resolve_hot(hot[j], eps, L, reinterpret_cast<int32_t *>(U.lx), n,
                                 &s_nx, tid, my_push, my_rel) &&
                    tid == 0)
                    atomicOr(&s_stop, 2);
            if (my_push) atomicAdd(&s_cnt[2], my_push);
            if (my_rel) atomicAdd(&s_cnt[3], my_rel);
            if (tid == 0) {
                // every thread read s_ny before the last barrier, and s_qh is
                // read only after the next one; the budget check sees the
                // counters of earlier phases (a safety limit, not exact)
                s_ny = 0;
                s_qh = 0;
                atomicAdd(&s_cnt[1], 1ull);
                const long long ops = (long long)(s_cnt[2] + s_cnt[3]);
                if (ops > A.max_ops || wall_clock64() - t_start > A.max_ticks)
                    atomicOr(&s_stop, 1);
                else if (on_warm && ops > warm_budget)
                    atomicOr(&s_stop, 4);
            }
            __syncthreads();
            int nx = s_nx;
            // s_nh was read by every thread before the last barrier and is
            // next used after the X phase's barrier
            if (tid == 0) s_nh = 0;
            if (nx == 0 || s_stop) break;
            if (nx <= tail_enter) {
                if (CT && s_cnt[2] - s_pu_mark >= period) {
                    const uint64_t t0 = wall_clock64();
                    const int steps = price_update(L, U, L.yl, CT, n, sgnS, eps, tid);
                    if (tid == 0) {
                        s_pu_mark = s_cnt[2];
                        atomicAdd(&s_cnt[5], 1ull);
                        atomicAdd(&s_cnt[6], (unsigned long long)(wall_clock64() - t0));
                        atomicAdd(&s_cnt[10], (unsigned long long)steps);
                    }
                    __syncthreads();
                }
                // ---- serial tail ----
                if (wave == 0) {
                    // circular queue over xl: head position, tail position
                    // and length, wrapped without division
                    int qh = 0, qt = nx == n ? 0 : nx, qlen = nx;
                    unsigned long long tp = 0, tr = 0, ts = 0;
                    int stop = 0;
                    // back to the phases after n pushes, for the next price update
                    while (qlen > 0 && qlen <= tail_exit &&
                           (!CT || tp < period)) {
                        const int x = L.xl[qh];
                        if (++qh == n) qh = 0;
                        --qlen;
                        int64_t best;
                        int arg, carg;
                        scan(x, best, arg, carg);
                        const int old = L.head[arg], e = L.ey[arg];
                        int64_t pxx = px[x];
                        if (best + pxx >= 0) {
                            pxx = -(best + eps);
                            px[x] = pxx;
                            ++tr;
                        }
                        const int64_t bx = int64_t(carg) * sgnS + pxx;
                        ++tp;
                        ++ts;
                        auto emit = [&](int r) {
                            L.xl[qt] = r;
                            if (++qt == n) qt = 0;
                            ++qlen;
                        };
                        if (e == 0 && old >= 0) {
                            // y held exactly one row (every column is settled
                            // between tail operations): resolve_column on the
                            // pair {x, old} without the list walk
                            const int64_t bo = L.bv[old];
                            const bool back_x = bx > bo || (bx == bo && x < old);
                            const int64_t bb = back_x ? bx : bo;
                            if (!(bb > py[arg])) {
                                py[arg] = bb - eps;
                                ++tr;
                            }
                            if (back_x) {
                                L.mate[x] = -1;
                            } else {
                                L.mate[x] = arg;
                                L.bv[x] = bx;
                                L.nxt[x] = -1;
                                L.head[arg] = x;
                                L.mate[old] = -1;
                            }
                            ++tp;
                            emit(back_x ? x : old);
                        } else {
                            L.mate[x] = arg;
                            L.bv[x] = bx;
                            L.nxt[x] = old;
                            L.head[arg] = x;
                            L.ey[arg] = e + 1;
                            if (!resolve_column(arg, eps, L, tp, tr, emit)) {
                                stop = 2;
                                break;
                            }
                        }
                        if ((ts & 127) == 0) {
                            const long long ops = (long long)(s_cnt[2] + s_cnt[3] + tp + tr);
                            if (ops > A.max_ops || wall_clock64() - t_start > A.max_ticks) {
                                stop = 1;
                                break;
                            }
                            if (on_warm && ops > warm_budget) {
                                stop = 4;
                                break;
                            }
                        }
                    }
                    if (lane == 0) {
                        s_nx = qlen;
                        s_qh = qh;
                        s_stop |= stop;
                        atomicAdd(&s_cnt[2], tp);
                        atomicAdd(&s_cnt[3], tr);
                        atomicAdd(&s_cnt[4], ts);
                    }
                }
                __syncthreads();
                nx = s_nx;
                if (nx == 0 || s_stop) break;
            }
            const int qh0 = s_qh;
            __syncthreads();
            if (tid == 0) s_nx = 0;
            // ---- X phase: every pushed-back row bids again ----
            unsigned long long x_rel = 0, x_ops = 0;
            for (int i = wave; i < nx; i += NW) {
                ++x_ops;
                const int x = L.xl[qh0 + i < n ? qh0 + i : qh0 + i - n];
                int64_t best;
                int arg, carg;
                scan(x, best, arg, carg);
                if (lane == 0) {
                    if (best + px[x] >= 0) {  // relabel, then the arc is admissible
                        px[x] = -(best + eps);
                        ++x_rel;
                    }
                    L.mate[x] = arg;
                    L.bv[x] = int64_t(carg) * sgnS + px[x];
                    L.nxt[x] = atomicExch(&L.head[arg], x);
                    if (atomicAdd(&L.ey[arg], 1) == 0) L.yl[atomicAdd(&s_ny, 1)] = arg;
                }
            }
            if (lane == 0 && x_ops) {
                atomicAdd(&s_cnt[4], x_ops);  // row scans
                atomicAdd(&s_cnt[2], x_ops);  // one push per scan
                if (x_rel) atomicAdd(&s_cnt[3], x_rel);
            }
            __syncthreads();
        }
        if (s_stop == 4) {
            // The warm start ran past its budget: back to the plain start of
            // Algorithm 5.0.  Every thread has read s_stop before the
            // barrier below; the refine init rebuilds the matching state.
            __syncthreads();
            for (int y = tid; y < n; y += NT) py[y] = 0;
            if (tid == 0) {
                s_stop = 0;
                s_nx = 0;
                s_ny = 0;
                s_qh = 0;
                s_nh = 0;
                s_pu_mark = s_cnt[2];
                atomicAdd(&s_cnt[8], 1ull);
            }
            on_warm = false;
            lists = sparse;
            eps = eps_plain;  // the loop divides it first, as for a plain start
            __syncthreads();
            continue;
        }
        if (s_stop) break;
        if (eps == 1) {
            // a sparse instance's lists are its arcs: nothing else to check
            if (!lists || sparse) break;
            // the lists rest on arc fixing's bound: confirm 1-optimality over
            // all arcs, else run the last refine again with full scans
            if (tid == 0) s_bad = 0;
            __syncthreads();
            if (!not_one_optimal(C, ldc, py, L.mate, n, sgnS, wave, lane, &s_bad)) break;
            lists = false;
            eps = alpha;  // the next refine runs at eps = 1 again
            if (tid == 0) atomicAdd(&s_cnt[7], 1ull);
            __syncthreads();
            continue;
        }
        if constexpr (sizeof(T) == 2) {
            const int64_t bound = (4 * int64_t(n) + 2) * eps;
            const int64_t keep_r = bound >> A.fixing_shift;
            // only once the bound can drop arcs (every r is at most about
            // 2 max|c| S)
            if (fixing && bound < int64_t(cmax) * S) {
                fix_arcs(C, ldc, cand, ncand, lists, py, L.mate, n, sgnS, keep_r, wave,
                         lane);
                lists = true;
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (s_stop) {
        if (tid == 0) A.status[slot] = (s_stop & 2) ? 3 : 1;
    } else {
        const int32_t *C32 = A.costs + I.cost_off;
        long long part = 0;
        for (int x = tid; x < n; x += NT) {
            const int y = L.mate[x];
            A.row_to_col[I.row_off + x] = y;
            part += C32[int64_t(x) * n + y];
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
    if (tid == 0) s_cnt[9] = s_cnt[4] * (unsigned long long)n;  // cost entries scanned
    __syncthreads();
    if (tid < NCNT && s_cnt[tid]) atomicAdd(&A.counters[tid], s_cnt[tid]);
}

__global__ __launch_bounds__(NT) void k_assign(AArgs A) {
    const int slot = A.order[blockIdx.x];
    const AInst I = A.inst[slot];
    extern __shared__ __align__(16) unsigned char smem[];
    const unsigned cmax = A.cmax[slot];
    if (cmax > unsigned(LPR_ASSIGN_MAX_COST) || (A.sparse && cmax > C16_MAX)) {
        if (threadIdx.x == 0) A.status[slot] = 2;
        return;
    }
    const int16_t *copies = A.c16 + 2 * I.c16_off;
    if (cmax <= C16_MAX)
        solve_instance<int16_t>(A, I, slot, copies, copies + int64_t(I.n) * ld16(I.n),
                                cmax, smem);
    else
        solve_instance<int32_t>(A, I, slot, A.costs + I.cost_off,
                                reinterpret_cast<const int32_t *>(copies), cmax, smem);
}

// py, px, b(x) (int64), e(y), head, next, mate, two lists (int32), two
// labels (int64) and two scanned flags (uint8) per node
// prices of Y padded to ld16(n) entries, then the n-sized arrays
static size_t lds_bytes(int nmax) { return size_t(nmax) * 66 + 64 + 64; }

struct Layout {
    AInst *inst;
    int32_t *order, *status;
    unsigned *cmax;
    unsigned long long *counters;
    int16_t *c16;
    int32_t *cand, *ncand;
};

static int64_t c16_elems(int B, const int32_t *n) {
    int64_t e = 0;
    for (int b = 0; b < B; ++b) e += int64_t(n[b]) * ld16(n[b]);
    return e;
}

static Carver carve(Carver cv, int B, const int32_t *n, Layout *L) {
    L->inst = cv.take<AInst>(size_t(B));
    L->order = cv.take<int32_t>(size_t(B));
    L->status = cv.take<int32_t>(size_t(B));
    L->cmax = cv.take<unsigned>(size_t(B));
    L->counters = cv.take<unsigned long long>(NCNT);
    L->c16 = cv.take<int16_t>(size_t(2 * c16_elems(B, n)));
    int64_t rows = 0;
    for (int b = 0; b < B; ++b) rows += n[b];
    L->cand = cv.take<int32_t>(size_t(c16_elems(B, n)));
    L->ncand = cv.take<int32_t>(size_t(rows));
    return cv;
}

static size_t workspace_bytes(int B, const int32_t *n) {
    Layout L;
    return carve(Carver(), B, n, &L).used();
}

// ---------------------------------------------------------------------------
// Tuned schedules (lpr_assign_tune): alpha, the price-update quarters and the
// tail threshold per size class (floor(log2(sum of n^2))), kind of start
// (plain or warm) and form (dense or sparse); 0 in a field keeps the
// built-in rule.
// ---------------------------------------------------------------------------
struct ASched {
    int alpha, q, tail;
};

static std::mutex g_asched_mu;
static std::map<int, ASched> g_asched;
static bool g_asched_loaded = false;

static int sched_key(int B, const int32_t *n, bool warm, int sparse) {
    int64_t e = 0;
    for (int b = 0; b < B; ++b) e += int64_t(n[b]) * n[b];
    int c = 0;
    while (c < 62 && (int64_t(1) << (c + 1)) <= e) ++c;
    return c * 4 + (warm ? 2 : 0) + (sparse ? 1 : 0);
}

static bool valid_asched(const ASched &a) {
    return (a.alpha == 0 || (a.alpha >= 2 && a.alpha <= 1024)) && a.q >= 0 && a.q <= 64 &&
           a.tail >= 0 && a.tail <= 4096;
}

static void load_asched_file_locked() {
    if (g_asched_loaded) return;
    g_asched_loaded = true;
    const char *path = std::getenv("LPR_ASSIGN_TUNE_FILE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    int k;
    ASched a;
    while (std::fscanf(f, "%d %d %d %d", &k, &a.alpha, &a.q, &a.tail) == 4)
        if (k >= 0 && k < 256 && valid_asched(a)) g_asched[k] = a;
    std::fclose(f);
}

static ASched default_asched(int key) {
    std::lock_guard<std::mutex> lk(g_asched_mu);
    load_asched_file_locked();
    const auto it = g_asched.find(key);
    return it != g_asched.end() ? it->second : ASched{0, 0, 0};
}

static void store_asched(int key, const ASched &a) {
    std::lock_guard<std::mutex> lk(g_asched_mu);
    load_asched_file_locked();
    g_asched[key] = a;
    const char *path = std::getenv("LPR_ASSIGN_TUNE_FILE");
    if (!path) return;
    FILE *f = std::fopen(path, "w");
    if (!f) return;
    for (const auto &e : g_asched)
        std::fprintf(f, "%d %d %d %d\n", e.first, e.second.alpha, e.second.q, e.second.tail);
    std::fclose(f);
}

// Forgets the schedule of a key, so that a tuning trial's 0 fields mean the
// built-in rules.
static void erase_asched(int key) {
    std::lock_guard<std::mutex> lk(g_asched_mu);
    load_asched_file_locked();
    g_asched.erase(key);
}

static lpr_status run(int32_t B, const int32_t *n, const int64_t *cost_offset,
                      const int32_t *costs, int32_t maximize,
                      int32_t *row_to_col, int64_t *totals, int64_t *col_prices,
                      const lpr_assign_opts *opts, lpr_assign_stats *stats,
                      void *workspace, size_t ws_bytes, void *stream,
                      int32_t sparse = 0, hipStream_t side = nullptr,
                      hipEvent_t fork = nullptr, hipEvent_t join = nullptr) {
    if (!sparse && !side) clear_error();
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
    int64_t rows = 0, c16 = 0, nnmax = 0;
    for (int b = 0; b < B; ++b) {
        if (n[b] < 1 || n[b] > LPR_ASSIGN_MAX_N) {
            set_error("instance %d: n = %d outside [1, %d]", b, n[b], LPR_ASSIGN_MAX_N);
            return LPR_EINVAL;
        }
        const int64_t nn = int64_t(n[b]) * n[b];
        if (cost_offset[b + 1] != cost_offset[b] + nn) {
            set_error("cost_offset is not the prefix sum of n^2 at %d", b);
            return LPR_EINVAL;
        }
        insts[b].cost_off = cost_offset[b];
        insts[b].c16_off = c16;
        insts[b].n = n[b];
        insts[b].row_off = int32_t(rows);
        rows += n[b];
        c16 += int64_t(n[b]) * ld16(n[b]);
        nmax = std::max(nmax, n[b]);
        nnmax = std::max(nnmax, nn);
    }
    if (rows >= (int64_t(1) << 31)) {
        set_error("too many rows");
        return LPR_EINVAL;
    }
    // the tuned schedule of this size class and kind of start fills the
    // schedule fields the options leave 0
    const bool warm = opts && (opts->init_col_prices || opts->eps0 || opts->eps0_per_instance);
    const ASched ds = default_asched(sched_key(B, n, warm, sparse));
    // built-in rules (the fields a tuned schedule leaves 0), measured on
    // the dense workloads: alpha 6 when the largest instance has n >= 1024
    // (the n = 1024 solve); for batches of instances up to n = 512, alpha
    // 16 from the plain start and 8 from a warm one, a tail of 32 rows, and
    // from a warm start a price update every n/4 operations (the batched
    // workload over seeds 0-4: plain 8 % and warm 5.5 % faster than alpha 8
    // with the per-instance tail and period); alpha 8 otherwise, also for
    // the sparse solve (n = 2048)
    const bool small = nmax <= 512 && !sparse;
    int32_t alpha = ds.alpha ? ds.alpha
                             : (nmax >= 1024 && !sparse ? 6 : (small && !warm ? 16 : 8));
    int64_t eps0 = 0, max_ops = 64 * int64_t(nmax) * nmax + (int64_t(1) << 20);
    int64_t max_ms = 20000, pu_period = 0, warm_max_ops = 0;
    int32_t tail_rows = ds.tail ? ds.tail : (small ? 32 : 0);
    int32_t pu_q = ds.q ? ds.q : (small && warm ? 1 : 0);
    int32_t pu_start = 1, arc_fixing = 0, fixing_shift = 0;
    const int64_t *init = nullptr, *eps0_inst = nullptr;
    bool timing = false;
    if (opts) {
        eps0_inst = opts->eps0_per_instance;
        if (opts->alpha) alpha = opts->alpha;
        eps0 = opts->eps0;
        init = opts->init_col_prices;
        if (opts->max_ops) max_ops = opts->max_ops;
        if (opts->max_ms) max_ms = opts->max_ms;
        pu_period = opts->price_update_period;
        if (opts->tail_rows) tail_rows = opts->tail_rows;
        if (opts->price_update_quarters) pu_q = opts->price_update_quarters;
        pu_start = (opts->flags & LPR_ASSIGN_NO_START_UPDATE) == 0;
        arc_fixing = (opts->flags & LPR_ASSIGN_ARC_FIXING) != 0;
        fixing_shift = opts->fixing_shift;
        warm_max_ops = opts->warm_max_ops;
        timing = (opts->flags & LPR_ASSIGN_TIME_KERNELS) != 0;
        if (opts->price_update_quarters < 0 || opts->price_update_quarters > 64 ||
            opts->reserved != 0) {
            set_error("invalid lpr_assign_opts (price_update_quarters outside 0..64 or "
                      "reserved not 0)");
            return LPR_EINVAL;
        }
    }
    if (alpha < 2 || eps0 < 0 || max_ops < 0 || max_ms < 0 || tail_rows < 0 ||
        tail_rows > 4096 || fixing_shift < 0 || fixing_shift > 63 || warm_max_ops < -1) {
        set_error("invalid lpr_assign_opts");
        return LPR_EINVAL;
    }
    const size_t need = workspace_bytes(B, n);
    if (ws_bytes < need) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
        return LPR_ENOMEM;
    }
    Layout L;
    carve(Carver(workspace, ws_bytes), B, n, &L);
    std::vector<int32_t> order(B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return n[a] > n[b]; });
    hipStream_t s = static_cast<hipStream_t>(stream);
    CallTimer call(s);
    call.start();
    // the tables, the counters and the cost copies go on `side` when the
    // caller forks them there (they then overlap work the caller enqueued
    // on `s` after `fork`); k_assign waits for them through `join`
    hipStream_t sp = s;
    if (side) {
        LPR_TRY_HIP(hipStreamWaitEvent(side, fork, 0));
        sp = side;
    }
    LPR_TRY_HIP(hipMemcpyAsync(L.inst, insts.data(), sizeof(AInst) * B,
                               hipMemcpyHostToDevice, sp));
    LPR_TRY_HIP(hipMemcpyAsync(L.order, order.data(), sizeof(int32_t) * B,
                               hipMemcpyHostToDevice, sp));
    LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(L.counters), 0, NCNT, sp));
    LPR_TRY(fill_i32(L.status, -1, B, sp));
    LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(L.cmax), 0, B, sp));
    const int gx = int(std::min<int64_t>(512, std::max<int64_t>(1, (nnmax + 4095) / 4096)));
    hipLaunchKernelGGL(k_prep, dim3(gx, B), dim3(256), 0, sp, L.inst, costs, L.c16, L.cmax);
    LPR_TRY_HIP(hipGetLastError());
    const unsigned tiles = unsigned((nmax + 63) / 64);
    hipLaunchKernelGGL(k_transpose, dim3(B, tiles, tiles), dim3(256), 0, sp, L.inst,
                       costs, L.cmax, L.c16);
    LPR_TRY_HIP(hipGetLastError());
    if (side) {
        LPR_TRY_HIP(hipEventRecord(join, side));
        LPR_TRY_HIP(hipStreamWaitEvent(s, join, 0));
    }
    AArgs A;
    A.inst = L.inst;
    A.order = L.order;
    A.costs = costs;
    A.c16 = L.c16;
    A.cmax = L.cmax;
    A.sign = maximize ? -1 : 1;
    A.alpha = alpha;
    A.eps0 = eps0;
    A.eps0_inst = eps0_inst;
    A.init_prices = init;
    A.row_to_col = row_to_col;
    A.totals = totals;
    A.col_prices = col_prices;
    A.max_ops = max_ops;
    A.warm_max_ops = warm_max_ops;
    A.pu_period = pu_period;
    A.pu_q = pu_q;
    A.tail_rows = tail_rows;
    A.pu_start = pu_start;
    A.arc_fixing = arc_fixing;
    A.fixing_shift = fixing_shift;
    A.sparse = sparse;
    if (sparse) A.arc_fixing = 0;
    A.cand = L.cand;
    A.ncand = L.ncand;
    int khz = 0;  // wall_clock64 ticks per millisecond
    {
        int dev = 0;
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
    unsigned long long cnt[NCNT];
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
        stats->price_updates = int64_t(cnt[5]);
        stats->price_update_us = int64_t(cnt[6] * 1000 / uint64_t(khz));
        stats->fixing_reruns = int64_t(cnt[7]);
        stats->warm_restarts = int64_t(cnt[8]);
        stats->scan_entries = int64_t(cnt[9]);
        stats->price_update_steps = int64_t(cnt[10]);
        stats->kernel_ms = kms;
        stats->total_ms = tms;
        stats->alpha = alpha;
        stats->price_update_quarters = pu_period != 0 ? 0 : pu_q;
        stats->tail_rows = tail_rows;
        stats->reserved = 0;
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

lpr_status run_forked(int32_t B, const int32_t *n, const int64_t *cost_offset,
                      const int32_t *costs, int32_t maximize, int32_t *row_to_col,
                      int64_t *totals, int64_t *col_prices, const lpr_assign_opts *opts,
                      lpr_assign_stats *stats, void *workspace, size_t ws_bytes,
                      void *stream, hipStream_t side, hipEvent_t fork, hipEvent_t join) {
    return run(B, n, cost_offset, costs, maximize, row_to_col, totals, col_prices, opts,
               stats, workspace, ws_bytes, stream, 0, side, fork, join);
}

}  // namespace assign
}  // namespace lpr

using namespace lpr;

extern "C" size_t lpr_assign_workspace(int32_t n) {
    if (n < 1) return 0;
    return assign::workspace_bytes(1, &n);
}

extern "C" size_t lpr_assign_batched_workspace(int32_t B, const int32_t *n) {
    if (B < 1 || !n) return 0;
    for (int b = 0; b < B; ++b)
        if (n[b] < 1) return 0;
    return assign::workspace_bytes(B, n);
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

extern "C" lpr_status lpr_assign_tune(int32_t B, const int32_t *n,
                                      const int64_t *cost_offset, const int32_t *costs,
                                      int32_t maximize, int32_t *row_to_col,
                                      int64_t *totals, const lpr_assign_opts *base,
                                      int32_t reps, lpr_assign_opts *best,
                                      double *best_ms, void *workspace,
                                      size_t workspace_bytes, void *stream) {
    clear_error();
    if (B < 1 || !n || !totals || reps < 1 || reps > 100) {
        set_error("invalid tuning arguments");
        return LPR_EINVAL;
    }
    lpr_assign_opts o = base ? *base : lpr_assign_opts{};
    if (o.alpha || o.price_update_period || o.price_update_quarters || o.tail_rows) {
        set_error("the schedule fields of the base options must be 0");
        return LPR_EINVAL;
    }
    o.flags &= ~LPR_ASSIGN_TIME_KERNELS;
    const bool warm = base && (base->init_col_prices || base->eps0 || base->eps0_per_instance);
    const int key = assign::sched_key(B, n, warm, 0);
    assign::erase_asched(key);
    static const int alphas[4] = {4, 6, 8, 16};
    static const int qs[4] = {1, 2, 4, 8};
    static const int tails[3] = {0, 8, 32};
    std::vector<int64_t> ref(B), got(B);
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool have_ref = false;
    double best_t = 1e300;
    assign::ASched best_s{8, 0, 0};
    for (int a : alphas)
        for (int q : qs)
            for (int tl : tails) {
                o.alpha = a;
                o.price_update_quarters = q;
                o.tail_rows = tl;
                // the fastest of `reps` runs after a warm-up, its totals
                // checked against the first schedule's
                double t_min = 1e300;
                for (int r = 0; r <= reps; ++r) {
                    lpr_assign_stats st{};
                    LPR_TRY(assign::run(B, n, cost_offset, costs, maximize, row_to_col,
                                        totals, nullptr, &o, &st, workspace,
                                        workspace_bytes, stream));
                    if (r > 0) t_min = std::min(t_min, st.total_ms);
                }
                LPR_TRY_HIP(hipMemcpyAsync(got.data(), totals, sizeof(int64_t) * B,
                                           hipMemcpyDeviceToHost, s));
                LPR_TRY_HIP(hipStreamSynchronize(s));
                if (!have_ref) {
                    ref = got;
                    have_ref = true;
                } else if (got != ref) {
                    set_error("schedules disagree on an optimal total (alpha %d, quarters "
                              "%d, tail rows %d)", a, q, tl);
                    return LPR_EDEVICE;
                }
                if (t_min < best_t) {
                    best_t = t_min;
                    best_s = assign::ASched{a, q, tl};
                }
            }
    assign::store_asched(key, best_s);
    if (best) {
        *best = base ? *base : lpr_assign_opts{};
        best->alpha = best_s.alpha;
        best->price_update_quarters = best_s.q;
        best->tail_rows = best_s.tail;
    }
    if (best_ms) *best_ms = best_t;
    return LPR_OK;
}

// ---------------------------------------------------------------------------
// Sparse assignment: the bipartite graph is given by its arcs (CSR by row).
// The arcs become the row lists that every row scan of the refine reads.
// The price update keeps a dense column-major copy; there every missing arc
// carries the largest cost of the instance.  Missing arcs are not kept
// eps-optimal, so their length floor(c_p / eps) + 1 is clamped at 0 (Dial's
// buckets need lengths >= 0; real arcs are never clamped).  Labels computed
// over a graph with extra arcs of length >= 0 still satisfy
// d(u) <= d(v) + length(u,v) on every real residual arc, so their price
// change keeps the pseudoflow eps-optimal and the update stays valid.  A refine terminates only when a perfect matching exists, so that
// is checked first, as a unit-capacity max-flow on the arbitrary-network
// solver (Section 3: a maximum matching is a maximum flow).
// ---------------------------------------------------------------------------
namespace lpr {
namespace assign {

// error bits: 1 structure (row_ptr, column range), 2 |cost| > C16_MAX
__global__ __launch_bounds__(256) void k_sp_check(int n, int m, const int32_t *row_ptr,
                                                  const int32_t *col,
                                                  const int32_t *cost, unsigned *err,
                                                  unsigned *cmax) {
    const int tid = blockIdx.x * 256 + threadIdx.x, nth = gridDim.x * 256;
    unsigned bits = 0, cm = 0;
    for (int x = tid; x <= n; x += nth) {
        const int a = row_ptr[x];
        if (x == 0 && a != 0) bits |= 1;
        if (x == n && a != m) bits |= 1;
        if (x < n && row_ptr[x + 1] < a) bits |= 1;
    }
    for (int k = tid; k < m; k += nth) {
        const int y = col[k], c = cost[k];
        if (y < 0 || y >= n) bits |= 1;
        const unsigned a = c < 0 ? 0u - unsigned(c) : unsigned(c);
        if (a > C16_MAX) bits |= 2;
        cm = max(cm, a);
    }
    if (bits) atomicOr(err, bits);
    for (int o = 32; o > 0; o >>= 1) cm = max(cm, unsigned(__shfl_xor(int(cm), o, 64)));
    if ((threadIdx.x & 63) == 0 && cm) atomicMax(cmax, cm);
}

// Dense matrix of the missing-arc cost (max|c| to minimise, -max|c| to
// maximise: the worst value either way) and an empty arc bitmap.
__global__ __launch_bounds__(256) void k_sp_fill(int n, int32_t *D, uint32_t *mask,
                                                 int words, const unsigned *cmax,
                                                 int sign) {
    const int32_t fake = sign > 0 ? int32_t(*cmax) : -int32_t(*cmax);
    const int64_t nn = int64_t(n) * n, nm = int64_t(n) * words;
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < nn; i += gridDim.x * 256ll) {
        D[i] = fake;
        if (i < nm) mask[i] = 0;
    }
}

// One wavefront per row: each arc lowers (raises, to maximise) its matrix
// entry -- of parallel arcs only the best one matters -- and sets its bit;
// the flow network gets the arc X(x) -> Y(y) of capacity 1, plus s -> X(x)
// and Y(x) -> t.  Nodes: X = 0..n-1, Y = n..2n-1, s = 2n, t = 2n + 1.
__global__ __launch_bounds__(256) void k_sp_scatter(int n, int m, const int32_t *row_ptr,
                                                    const int32_t *col,
                                                    const int32_t *cost, int sign,
                                                    int32_t *D, uint32_t *mask, int words,
                                                    int32_t *tail, int32_t *head,
                                                    int32_t *cap) {
    const int lane = threadIdx.x & 63;
    const int x = (blockIdx.x * 256 + threadIdx.x) >> 6;
    if (x >= n) return;
    for (int k = row_ptr[x] + lane; k < row_ptr[x + 1]; k += 64) {
        const int y = col[k], c = cost[k];
        int32_t *d = D + int64_t(x) * n + y;
        if (sign > 0) atomicMin(d, c);
        else atomicMax(d, c);
        atomicOr(&mask[int64_t(x) * words + (y >> 5)], 1u << (y & 31));
        tail[2 * k] = x;
        head[2 * k] = n + y;
        cap[2 * k] = 1;
        tail[2 * k + 1] = n + y;
        head[2 * k + 1] = x;
        cap[2 * k + 1] = 0;
    }
    if (lane == 0) {
        const int64_t a = 2 * (int64_t(m) + x), b = 2 * (int64_t(m) + n + x);
        tail[a] = 2 * n;
        head[a] = x;
        cap[a] = 1;
        tail[a + 1] = x;
        head[a + 1] = 2 * n;
        cap[a + 1] = 0;
        tail[b] = n + x;
        head[b] = 2 * n + 1;
        cap[b] = 1;
        tail[b + 1] = 2 * n + 1;
        head[b + 1] = n + x;
        cap[b + 1] = 0;
    }
}

// One wavefront per row: the row's distinct arcs in column order as list
// entries (y << 16) | (c(x,y) & 0xffff), their number in ncand[x].
__global__ __launch_bounds__(256) void k_sp_lists(int n, const int32_t *D,
                                                  const uint32_t *mask, int words,
                                                  int32_t *cand, int32_t *ncand) {
    const int lane = threadIdx.x & 63;
    const int x = (blockIdx.x * 256 + threadIdx.x) >> 6;
    if (x >= n) return;
    int32_t *list = cand + int64_t(x) * ld16(n);
    int out = 0;
    for (int y0 = 0; y0 < n; y0 += 64) {
        const int y = y0 + lane;
        const bool real =
            y < n && (mask[int64_t(x) * words + (y >> 5)] >> (y & 31) & 1u) != 0;
        const unsigned long long bal = __ballot(real);
        if (real)
            list[out + __popcll(bal & ((1ull << lane) - 1))] =
                (y << 16) | (D[int64_t(x) * n + y] & 0xffff);
        out += __popcll(bal);
    }
    if (lane == 0) ncand[x] = out;
}

struct SparseLayout {
    unsigned char *assign_ws, *graph_ws;
    size_t assign_bytes, graph_bytes;
    int32_t *D, *tail, *head, *cap;
    uint32_t *mask;
    unsigned *words;  // error bits, max|c|
};

static Carver sparse_carve(Carver cv, int n, int m, SparseLayout *S) {
    const int words = (n + 31) / 32;
    const int64_t arcs = 2 * (int64_t(m) + 2 * n);
    S->assign_bytes = workspace_bytes(1, &n);
    S->graph_bytes = lpr_graph_maxflow_workspace(2 * n + 2, int32_t(arcs));
    S->assign_ws = cv.take<unsigned char>(S->assign_bytes);
    S->graph_ws = cv.take<unsigned char>(S->graph_bytes);
    S->D = cv.take<int32_t>(size_t(n) * n);
    S->mask = cv.take<uint32_t>(size_t(n) * words);
    S->tail = cv.take<int32_t>(size_t(arcs));
    S->head = cv.take<int32_t>(size_t(arcs));
    S->cap = cv.take<int32_t>(size_t(arcs));
    S->words = cv.take<unsigned>(2);
    return cv;
}

static bool sparse_args_ok(int32_t n, int32_t m) {
    return n >= 1 && n <= LPR_ASSIGN_MAX_N && m >= 0 && m <= LPR_ASSIGN_SPARSE_MAX_ARCS;
}

}  // namespace assign
}  // namespace lpr

extern "C" size_t lpr_assign_sparse_workspace(int32_t n, int32_t m) {
    if (!assign::sparse_args_ok(n, m)) return 0;
    assign::SparseLayout S;
    return assign::sparse_carve(Carver(), n, m, &S).used();
}

extern "C" lpr_status lpr_assign_sparse_solve(int32_t n, int32_t m, const int32_t *row_ptr,
                                              const int32_t *col, const int32_t *cost,
                                              int32_t maximize, int32_t *row_to_col,
                                              int64_t *total, int64_t *col_prices,
                                              const lpr_assign_opts *opts,
                                              lpr_assign_stats *stats, void *workspace,
                                              size_t workspace_bytes, void *stream) {
    using namespace assign;
    clear_error();
    if (!sparse_args_ok(n, m) || !row_ptr || (m > 0 && (!col || !cost)) || !row_to_col ||
        !total || !workspace) {
        set_error("invalid arguments (n = %d, m = %d, or a NULL pointer)", n, m);
        return LPR_EINVAL;
    }
    const size_t need = lpr_assign_sparse_workspace(n, m);
    if (workspace_bytes < need) {
        set_error("workspace too small: %zu < %zu bytes", workspace_bytes, need);
        return LPR_ENOMEM;
    }
    SparseLayout S;
    sparse_carve(Carver(workspace, workspace_bytes), n, m, &S);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int words = (n + 31) / 32, sign = maximize ? -1 : 1;
    LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(S.words), 0, 2, s));
    const int gc = int(std::min<int64_t>(1024, (int64_t(m) + n + 256) / 256));
    hipLaunchKernelGGL(k_sp_check, dim3(gc), dim3(256), 0, s, n, m, row_ptr, col, cost,
                       S.words, S.words + 1);
    LPR_TRY_HIP(hipGetLastError());
    unsigned w[2] = {0, 0};
    LPR_TRY_HIP(hipMemcpyAsync(w, S.words, sizeof(w), hipMemcpyDeviceToHost, s));
    LPR_TRY_HIP(hipStreamSynchronize(s));
    if (w[0] & 1) {
        set_error("row_ptr is not a CSR offset array of m arcs, or a column is outside [0, n)");
        return LPR_EINVAL;
    }
    if (w[0] & 2) {
        set_error("|cost| > 32767 in a sparse instance");
        return LPR_ERANGE;
    }
    const int gf = int(std::min<int64_t>(4096, (int64_t(n) * n + 255) / 256));
    hipLaunchKernelGGL(k_sp_fill, dim3(gf), dim3(256), 0, s, n, S.D, S.mask, words,
                       S.words + 1, sign);
    const int gw = (n + 3) / 4;  // four wavefronts per block, one per row
    hipLaunchKernelGGL(k_sp_scatter, dim3(gw), dim3(256), 0, s, n, m, row_ptr, col, cost,
                       sign, S.D, S.mask, words, S.tail, S.head, S.cap);
    LPR_TRY_HIP(hipGetLastError());
    // a perfect matching must exist, else no refine ends
    int64_t matched = 0;
    const lpr_status fs = lpr_graph_maxflow(
        2 * n + 2, int32_t(2 * (int64_t(m) + 2 * n)), S.tail, S.head, S.cap, 2 * n,
        2 * n + 1, &matched, nullptr, nullptr, nullptr, S.graph_ws, S.graph_bytes, stream);
    if (fs != LPR_OK) return fs;
    if (matched < n) {
        set_error("no perfect matching: at most %lld of %d rows can be matched",
                  (long long)matched, n);
        return LPR_ENOMATCH;
    }
    Layout L;
    carve(Carver(S.assign_ws, S.assign_bytes), 1, &n, &L);
    hipLaunchKernelGGL(k_sp_lists, dim3(gw), dim3(256), 0, s, n, S.D, S.mask, words,
                       L.cand, L.ncand);
    LPR_TRY_HIP(hipGetLastError());
    const int64_t off[2] = {0, int64_t(n) * n};
    return run(1, &n, off, S.D, maximize, row_to_col, total, col_prices, opts, stats,
               S.assign_ws, S.assign_bytes, stream, 1);
}
