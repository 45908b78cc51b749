// Form 1: lock-free push-relabel maximum flow / minimum cut on 4-connected
// grid networks, for gfx950.
//
// Method (Section 4): Hong's lock-free push-relabel (Algorithm 4.5) -- every
// active pixel finds its lowest residual neighbour and either pushes
// min(e, u_f) to it with atomic updates of the two residuals and the two
// excesses, or relabels itself to that neighbour's height + 1 with a plain
// store (only the owner writes its height).  Phases of pushing alternate with
// an exact global relabel (backward BFS from t, Algorithm 4.4) followed by the
// gap step (unscanned pixels get h = |V|), as in the hybrid scheme of
// Algorithm 4.8 and Section 4.6.  The run stops when, right after a global
// relabel, no pixel has e > 0 and h < |V| (equivalent to e(s) + e(t) reaching
// ExcessTotal).  The maximum flow value is e(t) = sum_p (cap_snk - u_f(p,t));
// the minimal cut side is the residual closure of the pixels with excess.
//
// GPU design (not the paper's Fermi design):
//  * SoA state, one int32 array each for e, h, and the residuals of p->right,
//    p->left, p->down, p->up and p->t; the arc p->s is never used again after
//    the initial saturation (pixels with h >= |V| are never discharged).
//  * 64 x TH tiles, one 256-thread workgroup per tile.  A sweep launch loads a
//    tile into LDS and runs `local_iters` lock-free iterations there with LDS
//    atomics; pushes that cross the tile edge go straight to global memory
//    with device-scope atomics, and the tile's own edge values are merged back
//    by atomic deltas.  Every value a pixel reads of another pixel is a lower
//    bound of the true one (excess and residuals are only decreased by their
//    owner, heights only grow between global relabels), which is exactly the
//    staleness Hong's argument admits.
//  * Active-tile flags double-buffered across sweep launches so that quiet
//    tiles cost one flag read.
//  * The BFS (and the cut closure) is a Bellman-Ford style relaxation run to a
//    local fixpoint inside each LDS tile; tiles whose edge values changed mark
//    their neighbours dirty, and passes repeat until no tile is dirty.  The
//    least fixpoint is exactly the BFS level of every pixel.
//  * Batched solves share every launch: the tile table spans all instances,
//    and an instance whose count reaches zero retires from later rounds.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "lpr_internal.h"

namespace lpr {
namespace grid {

constexpr int TW = 64;        // tile width: one wavefront per tile row
constexpr int NT = 256;       // threads per tile workgroup
constexpr int RPP = NT / TW;  // tile rows covered per thread pass (4)
constexpr int MAX_PASS_SLOTS = 64;

// Element at a 32-bit byte offset from a wave-uniform base: every per-pixel
// array shares the offset, so the compiler keeps one VGPR per pixel instead of
// a 64-bit address per array (the batch holds fewer than 2^30 pixels).
template <class T>
__device__ __forceinline__ T &at(T *base, uint32_t byte_off) {
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off);
}

struct Inst {
    int64_t off;      // first pixel of the instance in the packed arrays
    int32_t H, W;
    int32_t tiles_x, tiles_y;
    int32_t tile_base;
    int32_t HV;       // |V| = H*W + 2, the gap height
};

struct Scalars {
    unsigned long long total_active;
    int32_t err;
    int32_t pad;
    int32_t pass_count[MAX_PASS_SLOTS];
};

struct Dev {
    int32_t *e, *h, *rr, *rl, *rd, *ru, *rs;
    const int32_t *cap_src, *cap_snk, *cap_r, *cap_l, *cap_d, *cap_u;
    const Inst *inst;
    const int32_t *tile_inst;
    unsigned long long *inst_active;  // per-instance active pixels (last count)
    int32_t *done;                    // per-instance: no active pixel left
    unsigned long long *counters;     // pushes, relabels, tiles swept,
                                      // tiles relaxed (BFS), tiles relaxed (cut)
    Scalars *sc;
    int32_t ntiles;
    int32_t ninst;
};

struct Geo {
    int inst, H, W, HV, y0, x0, tx, ty, tiles_x, tiles_y;
    int64_t off;
};

template <int TH>
__device__ inline Geo tile_geo(const Dev &D, int t) {
    Geo g;
    g.inst = D.tile_inst[t];
    const Inst I = D.inst[g.inst];
    g.H = I.H;
    g.W = I.W;
    g.HV = I.HV;
    g.off = I.off;
    g.tiles_x = I.tiles_x;
    g.tiles_y = I.tiles_y;
    int lt = t - I.tile_base;
    g.ty = lt / I.tiles_x;
    g.tx = lt - g.ty * I.tiles_x;
    g.y0 = g.ty * TH;
    g.x0 = g.tx * TW;
    return g;
}

// Loads the one-pixel halo of a tile's labels/heights into rows 0 and TH+1
// and columns 0 and TW+1 of `s` (|V| outside the grid); corners unused.
template <int TH>
__device__ inline void load_halo(const Dev &D, const Geo &g, int c,
                                 int32_t (*s)[TW + 2]) {
    const int tid = threadIdx.x;
    const int x = g.x0 + c;
    if (tid < TW) {
        int32_t v = g.HV;
        if (x < g.W && g.y0 > 0) v = D.h[g.off + int64_t(g.y0 - 1) * g.W + x];
        s[0][c + 1] = v;
    } else if (tid < 2 * TW) {
        int32_t v = g.HV;
        if (x < g.W && g.y0 + TH < g.H)
            v = D.h[g.off + int64_t(g.y0 + TH) * g.W + x];
        s[TH + 1][c + 1] = v;
    } else if (tid < 2 * TW + TH) {
        const int r = tid - 2 * TW, y = g.y0 + r;
        int32_t v = g.HV;
        if (y < g.H && g.x0 > 0) v = D.h[g.off + int64_t(y) * g.W + g.x0 - 1];
        s[r + 1][0] = v;
    } else if (tid < 2 * TW + 2 * TH) {
        const int r = tid - 2 * TW - TH, y = g.y0 + r;
        int32_t v = g.HV;
        if (y < g.H && g.x0 + TW < g.W)
            v = D.h[g.off + int64_t(y) * g.W + g.x0 + TW];
        s[r + 1][TW + 1] = v;
    }
}

__device__ inline unsigned long long block_sum_u64(unsigned long long v) {
    __shared__ unsigned long long red[NT / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    unsigned long long s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;  // valid in thread 0
}

// ---------------------------------------------------------------------------
// Init (Algorithm 4.5 / 4.7): u_f = u on pixel arcs and pixel->t, the source
// arcs saturated (e(p) = u(s,p)), h = 0.  Border arcs that would leave the
// grid get residual 0.  Capacities are validated on the way.
// ---------------------------------------------------------------------------
template <int TH>
__global__ __launch_bounds__(NT) void k_init(Dev D) {
    const Geo g = tile_geo<TH>(D, blockIdx.x);
    const int c = threadIdx.x & (TW - 1);
    int bad = 0;
#pragma unroll
    for (int k = 0; k < TH / RPP; ++k) {
        const int r = (threadIdx.x >> 6) + RPP * k;
        const int y = g.y0 + r, x = g.x0 + c;
        if (y >= g.H || x >= g.W) continue;
        const int64_t p = g.off + int64_t(y) * g.W + x;
        const int32_t src = D.cap_src[p], snk = D.cap_snk[p];
        const int32_t cr = (x + 1 < g.W) ? D.cap_r[p] : 0;
        const int32_t cl = (x > 0) ? D.cap_l[p] : 0;
        const int32_t cd = (y + 1 < g.H) ? D.cap_d[p] : 0;
        const int32_t cu = (y > 0) ? D.cap_u[p] : 0;
        const int32_t mn = min(min(min(src, snk), min(cr, cl)), min(cd, cu));
        const int32_t mx = max(max(max(src, snk), max(cr, cl)), max(cd, cu));
        if (mn < 0) bad |= 1;
        if (mx > LPR_GRID_MAX_CAP) bad |= 2;
        D.e[p] = src;
        D.rs[p] = snk;
        D.rr[p] = cr;
        D.rl[p] = cl;
        D.rd[p] = cd;
        D.ru[p] = cu;
        D.h[p] = 0;
    }
    if (bad) atomicOr(&D.sc->err, bad);
}

// ---------------------------------------------------------------------------
// Global relabel seed (Algorithm 4.4 from t): level 1 for pixels with a
// residual arc to t, |V| (= "not scanned") elsewhere.  Tiles of retired
// instances are left untouched and not marked.
// ---------------------------------------------------------------------------
template <int TH>
__global__ __launch_bounds__(NT) void k_bfs_seed(Dev D, int32_t *dirty_cur,
                                                 int32_t *dirty_next) {
    const int t = blockIdx.x;
    const Geo g = tile_geo<TH>(D, t);
    const bool retired = D.done[g.inst] != 0;
    if (threadIdx.x == 0) {
        dirty_cur[t] = retired ? 0 : 1;
        dirty_next[t] = 0;
    }
    if (retired) return;
    const int c = threadIdx.x & (TW - 1);
#pragma unroll
    for (int k = 0; k < TH / RPP; ++k) {
        const int r = (threadIdx.x >> 6) + RPP * k;
        const int y = g.y0 + r, x = g.x0 + c;
        if (y >= g.H || x >= g.W) continue;
        const int64_t p = g.off + int64_t(y) * g.W + x;
        D.h[p] = D.rs[p] > 0 ? 1 : g.HV;
    }
}

// Cut-closure seed: label 0 for pixels holding excess, |V| elsewhere.
template <int TH>
__global__ __launch_bounds__(NT) void k_cut_seed(Dev D, int32_t *dirty_cur,
                                                 int32_t *dirty_next) {
    const int t = blockIdx.x;
    const Geo g = tile_geo<TH>(D, t);
    if (threadIdx.x == 0) {
        dirty_cur[t] = 1;
        dirty_next[t] = 0;
    }
    const int c = threadIdx.x & (TW - 1);
#pragma unroll
    for (int k = 0; k < TH / RPP; ++k) {
        const int r = (threadIdx.x >> 6) + RPP * k;
        const int y = g.y0 + r, x = g.x0 + c;
        if (y >= g.H || x >= g.W) continue;
        const int64_t p = g.off + int64_t(y) * g.W + x;
        D.h[p] = D.e[p] > 0 ? 0 : g.HV;
    }
}

template <int TH>
__global__ __launch_bounds__(NT) void k_cut_write(Dev D, uint8_t *side) {
    const Geo g = tile_geo<TH>(D, blockIdx.x);
    const int c = threadIdx.x & (TW - 1);
#pragma unroll
    for (int k = 0; k < TH / RPP; ++k) {
        const int r = (threadIdx.x >> 6) + RPP * k;
        const int y = g.y0 + r, x = g.x0 + c;
        if (y >= g.H || x >= g.W) continue;
        const int64_t p = g.off + int64_t(y) * g.W + x;
        side[p] = D.h[p] < g.HV ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// Tile relaxation to a local fixpoint.
//   BFS (CUT = false): lab(p) = min(lab(p), lab(q) + 1) over arcs p->q with
//     u_f > 0 -- the backward BFS of Algorithm 4.4 from t; its least fixpoint
//     is the BFS level, |V| where t is unreachable (the gap of Section 4.2).
//   CUT (CUT = true):  lab(p) = min(lab(p), lab(q)) over arcs q->p with
//     u_f > 0 -- forward reachability from the excess pixels.
// One wavefront per 64 x TH tile, no block barrier: lane c owns column c of
// the tile in registers.  An iteration takes the horizontal neighbours'
// current labels by cross-lane shuffles (lanes 0 and 63 use the halo
// columns), then runs a downward and an upward pass along its column, which
// settles every vertical path inside the tile at once.  Iterations repeat
// until no label of the tile changes (a wavefront vote).  Labels only
// decrease and every value read from a neighbouring tile is an upper bound
// of its final value, so concurrent tiles reach the same least fixpoint.
// ---------------------------------------------------------------------------
template <int TH, bool CUT>
__global__ __launch_bounds__(256) void k_relax(Dev D, int32_t *dirty_cur,
                                              int32_t *dirty_next,
                                              int32_t *pass_count) {
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= D.ntiles) return;                // wave-uniform
    if (dirty_cur[t] == 0) return;            // wave-uniform (same address)
    if (lane == 0) dirty_cur[t] = 0;
    const Geo g = tile_geo<TH>(D, t);
    constexpr int INC = CUT ? 0 : 1;
    const int HV = g.HV;
    const int x = g.x0 + lane;
    const bool colv = x < g.W;
    int32_t d[TH], d0[TH];
    uint32_t mR = 0, mL = 0, mD = 0, mU = 0;  // bit r: arc usable in row r
#pragma unroll
    for (int r = 0; r < TH; ++r) {
        const int y = g.y0 + r;
        d[r] = HV;
        if (colv && y < g.H) {
            const int64_t p = g.off + int64_t(y) * g.W + x;
            d[r] = D.h[p];
            if (!CUT) {
                mR |= uint32_t(D.rr[p] > 0) << r;
                mL |= uint32_t(D.rl[p] > 0) << r;
                mD |= uint32_t(D.rd[p] > 0) << r;
                mU |= uint32_t(D.ru[p] > 0) << r;
            } else {
                if (x + 1 < g.W) mR |= uint32_t(D.rl[p + 1] > 0) << r;
                if (x > 0) mL |= uint32_t(D.rr[p - 1] > 0) << r;
                if (y + 1 < g.H) mD |= uint32_t(D.ru[p + g.W] > 0) << r;
                if (y > 0) mU |= uint32_t(D.rd[p - g.W] > 0) << r;
            }
        }
        d0[r] = d[r];
    }
    // halo: row above / below (every lane), column left (lane 0) / right (63)
    int32_t top = HV, bot = HV, hside[TH];
    if (colv && g.y0 > 0) top = D.h[g.off + int64_t(g.y0 - 1) * g.W + x];
    if (colv && g.y0 + TH < g.H) bot = D.h[g.off + int64_t(g.y0 + TH) * g.W + x];
    const int hx = lane == 0 ? g.x0 - 1 : g.x0 + 64;
#pragma unroll
    for (int r = 0; r < TH; ++r) {
        const int y = g.y0 + r;
        hside[r] = HV;
        if ((lane == 0 || lane == 63) && hx >= 0 && hx < g.W && y < g.H)
            hside[r] = D.h[g.off + int64_t(y) * g.W + hx];
    }
    for (;;) {
        bool changed = false;
#pragma unroll
        for (int r = 0; r < TH; ++r) {
            int32_t left = __shfl_up(d[r], 1, 64);
            int32_t right = __shfl_down(d[r], 1, 64);
            if (lane == 0) left = hside[r];
            if (lane == 63) right = hside[r];
            int32_t nd = d[r];
            if ((mL >> r) & 1u) nd = min(nd, left + INC);
            if ((mR >> r) & 1u) nd = min(nd, right + INC);
            changed |= nd < d[r];
            d[r] = nd;
        }
#pragma unroll
        for (int r = 0; r < TH; ++r) {
            const int32_t up = r == 0 ? top : d[r - 1];
            if ((mU >> r) & 1u) {
                const int32_t nd = min(d[r], up + INC);
                changed |= nd < d[r];
                d[r] = nd;
            }
        }
#pragma unroll
        for (int r = TH - 1; r >= 0; --r) {
            const int32_t dn = r == TH - 1 ? bot : d[r + 1];
            if ((mD >> r) & 1u) {
                const int32_t nd = min(d[r], dn + INC);
                changed |= nd < d[r];
                d[r] = nd;
            }
        }
        if (!__any(changed)) break;
    }
    bool ch_top = false, ch_bot = false, ch_col = false;
#pragma unroll
    for (int r = 0; r < TH; ++r) {
        if (d[r] == d0[r]) continue;
        D.h[g.off + int64_t(g.y0 + r) * g.W + x] = d[r];
        ch_col = true;
        if (r == 0) ch_top = true;
        if (r == TH - 1) ch_bot = true;
    }
    const bool e_top = __any(ch_top), e_bot = __any(ch_bot);
    const bool e_left = __any(lane == 0 && ch_col), e_right = __any(lane == 63 && ch_col);
    if (lane == 0) {
        atomicAdd(&D.counters[CUT ? 4 : 3], 1ull);
        int nb[4] = {-1, -1, -1, -1};
        if (e_right && g.tx + 1 < g.tiles_x) nb[0] = t + 1;
        if (e_left && g.tx > 0) nb[1] = t - 1;
        if (e_bot && g.ty + 1 < g.tiles_y) nb[2] = t + g.tiles_x;
        if (e_top && g.ty > 0) nb[3] = t - g.tiles_x;
        for (int i = 0; i < 4; ++i)
            if (nb[i] >= 0 && atomicExch(&dirty_next[nb[i]], 1) == 0)
                atomicAdd(pass_count, 1);
    }
}

// ---------------------------------------------------------------------------
// Count active pixels (e > 0, h < |V|) right after a global relabel; seeds
// the active-tile flags of the next push phase.
// ---------------------------------------------------------------------------
template <int TH>
__global__ __launch_bounds__(NT) void k_count(Dev D, int32_t *act_cur,
                                              int32_t *act_next) {
    const int t = blockIdx.x;
    const Geo g = tile_geo<TH>(D, t);
    unsigned long long cnt = 0;
    if (!D.done[g.inst]) {
        const int c = threadIdx.x & (TW - 1);
#pragma unroll
        for (int k = 0; k < TH / RPP; ++k) {
            const int r = (threadIdx.x >> 6) + RPP * k;
            const int y = g.y0 + r, x = g.x0 + c;
            if (y >= g.H || x >= g.W) continue;
            const int64_t p = g.off + int64_t(y) * g.W + x;
            cnt += (D.e[p] > 0 && D.h[p] < g.HV) ? 1 : 0;
        }
    }
    const unsigned long long s = block_sum_u64(cnt);
    if (threadIdx.x == 0) {
        act_cur[t] = s > 0 ? 1 : 0;
        act_next[t] = 0;
        if (s) atomicAdd(&D.inst_active[g.inst], s);
    }
}

// Retire instances with no active pixel and publish the total.  The count
// is exact only after the BFS reached its fixpoint: when `bfs_open` is given
// and nonzero (the last relaxation pass still marked tiles dirty), labels can
// still be |V| above their BFS level, so nothing is retired and the host
// finishes the BFS and counts again.
__global__ void k_count_finish(Dev D, const int32_t *bfs_open) {
    const bool exact = bfs_open == nullptr || *bfs_open == 0;
    unsigned long long tot = 0;
    for (int i = threadIdx.x; i < D.ninst; i += blockDim.x) {
        const unsigned long long a = D.inst_active[i];
        if (a == 0 && exact) D.done[i] = 1;
        tot += a;
    }
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
    __shared__ unsigned long long red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
        D.sc->total_active = s;
    }
}

// ---------------------------------------------------------------------------
// Push sweep: `L` lock-free push/relabel iterations of Algorithm 4.5 per
// active 64 x TH tile, one wavefront per tile, no block barrier.  Lane c owns
// column c of the tile in registers (e, h, the four neighbour residuals and
// the sink residual of each of its TH pixels).  An iteration walks the rows
// top to bottom: the lane reads its horizontal neighbours' current heights by
// cross-lane shuffles (lanes 0 and 63 use the halo heights), picks the lowest
// residual neighbour and pushes or relabels; a push inside the column updates
// the registers directly, a push to the lane on the left or right is handed
// over by a shuffle right after the row, and flow pushed across the tile edge
// is summed per pixel and applied to global memory with device-scope atomics
// when the visit ends (activating that tile) -- for the other tile the push
// is fulfilled a little later, which Hong's argument admits.  The tile's own
// excesses on its edge are merged back by atomic deltas, so pushes that other
// tiles make into it meanwhile are kept.  Every value read of another
// pixel is a lower bound of the true one (excess and residuals only shrink
// by their owner's pushes, heights only grow between global relabels), the
// staleness Hong's argument admits.
// ---------------------------------------------------------------------------
template <int TH>
__global__ __launch_bounds__(256) void k_sweep(Dev D, int32_t *act_cur,
                                              int32_t *act_next, int L) {
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= D.ntiles) return;           // wave-uniform
    if (act_cur[t] == 0) return;         // wave-uniform (same address)
    if (lane == 0) act_cur[t] = 0;
    const Geo g = tile_geo<TH>(D, t);
    const int HV = g.HV;
    const int x = g.x0 + lane;
    const bool colv = x < g.W;
    int32_t e[TH], h[TH], rs[TH], rr[TH], rl[TH], rd[TH], ru[TH];
    uint32_t valid = 0;
#pragma unroll
    for (int r = 0; r < TH; ++r) {
        const int y = g.y0 + r;
        e[r] = 0; h[r] = HV; rs[r] = 0; rr[r] = 0; rl[r] = 0; rd[r] = 0; ru[r] = 0;
        if (colv && y < g.H) {
            valid |= 1u << r;
            const uint32_t o = 4u * uint32_t(g.off + int64_t(y) * g.W + x);
            e[r] = at(D.e, o);
            h[r] = at(D.h, o);
            rs[r] = at(D.rs, o);
            rr[r] = at(D.rr, o);
            rl[r] = at(D.rl, o);
            rd[r] = at(D.rd, o);
            ru[r] = at(D.ru, o);
        }
    }
    // Excess at load time, for the delta merge of edge pixels.  Residuals of
    // arcs that leave the tile are decremented in global memory at push time
    // (other tiles only ever increase them there), so they are never written
    // back; everything else is stored plainly if it changed (bit per row).
    int32_t e0[TH];
#pragma unroll
    for (int r = 0; r < TH; ++r) e0[r] = e[r];
    uint32_t ch_h = 0, ch_rs = 0, ch_rr = 0, ch_rl = 0, ch_rd = 0, ch_ru = 0;
    // flow pushed out of the tile (lanes 0 / 63 sideways, rows 0 / TH-1
    // vertically), applied to the neighbouring tiles when the visit ends
    int32_t outH[TH];
#pragma unroll
    for (int r = 0; r < TH; ++r) outH[r] = 0;
    int32_t outU = 0, outD = 0;
    // halo heights (read once; heights only grow, so these are lower bounds)
    int32_t top = HV, bot = HV, hside[TH];
    const uint32_t o0 = 4u * uint32_t(g.off + int64_t(g.y0) * g.W + x);  // row 0
    const uint32_t ow = 4u * uint32_t(g.W);                                // one row
    if (colv && g.y0 > 0) top = at(D.h, o0 - ow);
    if (colv && g.y0 + TH < g.H) bot = at(D.h, o0 + TH * ow);
    const int hx = lane == 0 ? g.x0 - 1 : g.x0 + 64;
#pragma unroll
    for (int r = 0; r < TH; ++r) {
        const int y = g.y0 + r;
        hside[r] = HV;
        if ((lane == 0 || lane == 63) && hx >= 0 && hx < g.W && y < g.H)
            hside[r] = at(D.h, o0 + r * ow + 4u * uint32_t(hx - x));
    }
    unsigned pushes = 0, relabels = 0;
    bool touch_l = false, touch_r = false, touch_u = false, touch_d = false;
    for (int it = 0; it < L; ++it) {
        bool any = false;
#pragma unroll
        for (int r = 0; r < TH; ++r) {
            int32_t hl = __shfl_up(h[r], 1, 64);
            int32_t hr = __shfl_down(h[r], 1, 64);
            if (lane == 0) hl = hside[r];
            if (lane == 63) hr = hside[r];
            int32_t sendR = 0, sendL = 0;
            const int y = g.y0 + r;
            if (((valid >> r) & 1u) && e[r] > 0 && h[r] < HV) {
                any = true;
                // lowest residual neighbour; scan order t, right, left, down, up
                int32_t best = INT_MAX, cap = 0;
                int dir = -1;
                if (rs[r] > 0) { best = 0; dir = 0; cap = rs[r]; }
                if (rr[r] > 0 && x + 1 < g.W && hr < best) { best = hr; dir = 1; cap = rr[r]; }
                if (rl[r] > 0 && x > 0 && hl < best) { best = hl; dir = 2; cap = rl[r]; }
                const int32_t hd = r + 1 < TH ? h[r + 1] : bot;
                if (rd[r] > 0 && y + 1 < g.H && hd < best) { best = hd; dir = 3; cap = rd[r]; }
                const int32_t hu = r > 0 ? h[r - 1] : top;
                if (ru[r] > 0 && y > 0 && hu < best) { best = hu; dir = 4; cap = ru[r]; }
                if (dir >= 0 && h[r] > best) {
                    // PUSH delta = min(e', u_f(x, y~)) towards y~
                    const int32_t d = min(e[r], cap);
                    e[r] -= d;
                    if (dir == 0) {
                        rs[r] -= d;
                        ch_rs |= 1u << r;
                    } else if (dir == 1) {
                        rr[r] -= d;
                        if (lane < 63) {
                            sendR = d;
                            ch_rr |= 1u << r;
                        } else {
                            outH[r] += d;
                        }
                    } else if (dir == 2) {
                        rl[r] -= d;
                        if (lane > 0) {
                            sendL = d;
                            ch_rl |= 1u << r;
                        } else {
                            outH[r] += d;
                        }
                    } else if (dir == 3) {
                        rd[r] -= d;
                        if (r + 1 < TH) {
                            ru[r + 1] += d;
                            e[r + 1] += d;
                            ch_rd |= 1u << r;
                            ch_ru |= 1u << (r + 1);
                        } else {
                            outD += d;
                        }
                    } else {
                        ru[r] -= d;
                        if (r > 0) {
                            rd[r - 1] += d;
                            e[r - 1] += d;
                            ch_ru |= 1u << r;
                            ch_rd |= 1u << (r - 1);
                        } else {
                            outU += d;
                        }
                    }
                    ++pushes;
                } else {
                    // RELABEL h(x) = h~ + 1 (owner only); no residual arc or
                    // a height past |V| freezes the pixel (gap height)
                    h[r] = (dir < 0 || best >= HV - 1) ? HV : best + 1;
                    ch_h |= 1u << r;
                    ++relabels;
                }
            }
            // hand the horizontal pushes of this row to the neighbour lanes
            const int32_t fromL = __shfl_up(sendR, 1, 64);
            const int32_t fromR = __shfl_down(sendL, 1, 64);
            if (lane > 0 && fromL) {
                rl[r] += fromL;
                e[r] += fromL;
                ch_rl |= 1u << r;
            }
            if (lane < 63 && fromR) {
                rr[r] += fromR;
                e[r] += fromR;
                ch_rr |= 1u << r;
            }
        }
        if (!__any(any)) break;
    }
    // write back: plain stores where only this tile writes, an atomic delta
    // for the excess of pixels that other tiles can push into
    bool active_end = false;
#pragma unroll
    for (int r = 0; r < TH; ++r) {
        if (!((valid >> r) & 1u)) continue;
        const int y = g.y0 + r;
        const uint32_t o = o0 + r * ow;
        const bool edge = (lane == 63 && x + 1 < g.W) || (lane == 0 && x > 0) ||
                          (r == TH - 1 && y + 1 < g.H) || (r == 0 && y > 0);
        if (e[r] != e0[r]) {
            if (edge) atomicAdd(&at(D.e, o), e[r] - e0[r]);
            else at(D.e, o) = e[r];
        }
        const uint32_t b = 1u << r;
        if (ch_h & b) at(D.h, o) = h[r];
        if (ch_rs & b) at(D.rs, o) = rs[r];
        if (ch_rr & b) at(D.rr, o) = rr[r];
        if (ch_rl & b) at(D.rl, o) = rl[r];
        if (ch_rd & b) at(D.rd, o) = rd[r];
        if (ch_ru & b) at(D.ru, o) = ru[r];
        active_end |= e[r] > 0 && h[r] < HV;
        // pushes out of the tile: own residual down, neighbour's reverse
        // residual and excess up
        if (outH[r]) {
            if (lane == 63) {
                atomicSub(&at(D.rr, o), outH[r]);
                atomicAdd(&at(D.rl, o + 4), outH[r]);
                atomicAdd(&at(D.e, o + 4), outH[r]);
                touch_r = true;
            } else {
                atomicSub(&at(D.rl, o), outH[r]);
                atomicAdd(&at(D.rr, o - 4), outH[r]);
                atomicAdd(&at(D.e, o - 4), outH[r]);
                touch_l = true;
            }
        }
        if (r == 0 && outU) {
            atomicSub(&at(D.ru, o), outU);
            atomicAdd(&at(D.rd, o - ow), outU);
            atomicAdd(&at(D.e, o - ow), outU);
            touch_u = true;
        }
        if (r == TH - 1 && outD) {
            atomicSub(&at(D.rd, o), outD);
            atomicAdd(&at(D.ru, o + ow), outD);
            atomicAdd(&at(D.e, o + ow), outD);
            touch_d = true;
        }
    }
    const bool a_end = __any(active_end);
    const bool a_l = __any(touch_l), a_r = __any(touch_r);
    const bool a_u = __any(touch_u), a_d = __any(touch_d);
    unsigned long long np = pushes, nr = relabels;
    for (int o = 32; o > 0; o >>= 1) {
        np += __shfl_xor(np, o, 64);
        nr += __shfl_xor(nr, o, 64);
    }
    if (lane == 0) {
        if (a_end) act_next[t] = 1;
        if (a_l) act_next[t - 1] = 1;
        if (a_r) act_next[t + 1] = 1;
        if (a_u) act_next[t - g.tiles_x] = 1;
        if (a_d) act_next[t + g.tiles_x] = 1;
        if (np) atomicAdd(&D.counters[0], np);
        if (nr) atomicAdd(&D.counters[1], nr);
        atomicAdd(&D.counters[2], 1ull);
    }
}

// Flow value e(t) = sum_p (u(p,t) - u_f(p,t)) per instance (int64).
template <int TH>
__global__ __launch_bounds__(NT) void k_flow_value(Dev D, int64_t *flow) {
    const Geo g = tile_geo<TH>(D, blockIdx.x);
    const int c = threadIdx.x & (TW - 1);
    unsigned long long s = 0;
#pragma unroll
    for (int k = 0; k < TH / RPP; ++k) {
        const int r = (threadIdx.x >> 6) + RPP * k;
        const int y = g.y0 + r, x = g.x0 + c;
        if (y >= g.H || x >= g.W) continue;
        const int64_t p = g.off + int64_t(y) * g.W + x;
        s += (unsigned long long)(int64_t(D.cap_snk[p]) - D.rs[p]);
    }
    const unsigned long long tot = block_sum_u64(s);
    if (threadIdx.x == 0 && tot)
        atomicAdd(reinterpret_cast<unsigned long long *>(&flow[g.inst]), tot);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct Layout {
    int32_t *st[7];
    int32_t *tile_inst, *act[2], *dirty[2], *done;
    Inst *inst;
    unsigned long long *inst_active, *counters;
    Scalars *sc;
};

static Carver carve(Carver cv, int64_t N, int64_t T, int B, Layout *L) {
    for (int i = 0; i < 7; ++i) L->st[i] = cv.take<int32_t>(size_t(N));
    L->tile_inst = cv.take<int32_t>(size_t(T));
    L->act[0] = cv.take<int32_t>(size_t(T));
    L->act[1] = cv.take<int32_t>(size_t(T));
    L->dirty[0] = cv.take<int32_t>(size_t(T));
    L->dirty[1] = cv.take<int32_t>(size_t(T));
    L->inst = cv.take<Inst>(size_t(B));
    L->inst_active = cv.take<unsigned long long>(size_t(B));
    L->done = cv.take<int32_t>(size_t(B));
    L->counters = cv.take<unsigned long long>(8);
    L->sc = cv.take<Scalars>(1);
    return cv;
}

static int64_t tiles_for(int32_t H, int32_t W, int TH) {
    return int64_t(ceil_div(W, TW)) * ceil_div(H, TH);
}

static size_t workspace_bytes(int B, const int32_t *H, const int32_t *W) {
    int64_t N = 0, T = 0;
    for (int b = 0; b < B; ++b) {
        N += int64_t(H[b]) * W[b];
        T += tiles_for(H[b], W[b], 8);  // smallest tile height: most tiles
    }
    Layout L;
    Carver cv = carve(Carver(), N, T, B, &L);
    return cv.used();
}

template <int TH>
struct Kern {
    static void init(dim3 g, hipStream_t s, const Dev &D) {
        hipLaunchKernelGGL(k_init<TH>, g, dim3(NT), 0, s, D);
    }
    static void bfs_seed(dim3 g, hipStream_t s, const Dev &D, int32_t *a, int32_t *b) {
        hipLaunchKernelGGL(k_bfs_seed<TH>, g, dim3(NT), 0, s, D, a, b);
    }
    static void cut_seed(dim3 g, hipStream_t s, const Dev &D, int32_t *a, int32_t *b) {
        hipLaunchKernelGGL(k_cut_seed<TH>, g, dim3(NT), 0, s, D, a, b);
    }
    // one wavefront per tile, four tiles per 256-thread block
    static void relax(bool cut, dim3 g, hipStream_t s, const Dev &D, int32_t *a,
                      int32_t *b, int32_t *pc) {
        const dim3 gw((g.x + 3) / 4);
        if (cut) hipLaunchKernelGGL((k_relax<TH, true>), gw, dim3(NT), 0, s, D, a, b, pc);
        else hipLaunchKernelGGL((k_relax<TH, false>), gw, dim3(NT), 0, s, D, a, b, pc);
    }
    static void count(dim3 g, hipStream_t s, const Dev &D, int32_t *a, int32_t *b) {
        hipLaunchKernelGGL(k_count<TH>, g, dim3(NT), 0, s, D, a, b);
    }
    static void sweep(dim3 g, hipStream_t s, const Dev &D, int32_t *a, int32_t *b, int L) {
        hipLaunchKernelGGL(k_sweep<TH>, dim3((g.x + 3) / 4), dim3(NT), 0, s, D, a, b, L);
    }
    static void flow(dim3 g, hipStream_t s, const Dev &D, int64_t *f) {
        hipLaunchKernelGGL(k_flow_value<TH>, g, dim3(NT), 0, s, D, f);
    }
    static void cut_write(dim3 g, hipStream_t s, const Dev &D, uint8_t *side) {
        hipLaunchKernelGGL(k_cut_write<TH>, g, dim3(NT), 0, s, D, side);
    }
};

struct Params {
    int TH, L, K, max_rounds;
    bool timing;
};

// Runs relaxation passes until no tile is dirty.  Pass counters are cleared
// per batch; the last slot of a batch being 0 means the fixpoint is reached.
template <int TH>
static lpr_status relax_to_fixpoint(bool cut, hipStream_t s, const Dev &D,
                                    Layout &Lw, int *dirty_sel, dim3 grid,
                                    EventTimer &tm, int64_t *passes) {
    int batch = 8;
    const int64_t guard = 16 * int64_t(D.ntiles) + 1024;
    for (int64_t done_passes = 0;; done_passes += batch) {
        if (done_passes > guard) {
            set_error("relaxation did not reach its fixpoint within %lld passes",
                      (long long)guard);
            return LPR_EBUDGET;
        }
        LPR_TRY(fill_i32(Lw.sc->pass_count, 0, batch, s));
        const int ev = tm.begin();
        for (int i = 0; i < batch; ++i) {
            Kern<TH>::relax(cut, grid, s, D, Lw.dirty[*dirty_sel],
                            Lw.dirty[*dirty_sel ^ 1], Lw.sc->pass_count + i);
            *dirty_sel ^= 1;
        }
        tm.end(ev);
        LPR_TRY_HIP(hipGetLastError());
        *passes += batch;
        int32_t last = 0;
        LPR_TRY_HIP(hipMemcpyAsync(&last, Lw.sc->pass_count + batch - 1,
                                   sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LPR_TRY_HIP(hipStreamSynchronize(s));
        if (last == 0) return LPR_OK;
        batch = std::min(batch * 2, MAX_PASS_SLOTS);
    }
}

// Count active pixels (after an exact global relabel) into the scalars and
// seed the active-tile flags act[0] (read by the next sweep).
template <int TH>
static lpr_status enqueue_count(hipStream_t s, const Dev &D, Layout &Lw, dim3 grid,
                                int B, const int32_t *bfs_open) {
    LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(Lw.inst_active), 0, B, s));
    Kern<TH>::count(grid, s, D, Lw.act[0], Lw.act[1]);
    hipLaunchKernelGGL(k_count_finish, dim3(1), dim3(256), 0, s, D, bfs_open);
    LPR_TRY_HIP(hipGetLastError());
    return LPR_OK;
}

// One round of the hybrid scheme (Algorithm 4.8 with the heuristic on the
// device): K push sweeps, the global relabel seed, P BFS relaxation passes
// and the count.  K and P are even, so every double-buffer selection is back
// where it started and the same sequence (or its graph) serves every round.
template <int TH>
static lpr_status enqueue_round(hipStream_t s, const Dev &D, Layout &Lw, dim3 grid,
                                int B, int K, int L, int P, EventTimer *t_sweep,
                                EventTimer *t_bfs) {
    int ev = t_sweep ? t_sweep->begin() : -1;
    for (int k = 0; k < K; ++k)
        Kern<TH>::sweep(grid, s, D, Lw.act[k & 1], Lw.act[(k & 1) ^ 1], L);
    if (t_sweep) t_sweep->end(ev);
    Kern<TH>::bfs_seed(grid, s, D, Lw.dirty[0], Lw.dirty[1]);
    LPR_TRY(fill_i32(Lw.sc->pass_count, 0, P, s));
    ev = t_bfs ? t_bfs->begin() : -1;
    for (int i = 0; i < P; ++i)
        Kern<TH>::relax(false, grid, s, D, Lw.dirty[i & 1], Lw.dirty[(i & 1) ^ 1],
                        Lw.sc->pass_count + i);
    if (t_bfs) t_bfs->end(ev);
    LPR_TRY(enqueue_count<TH>(s, D, Lw, grid, B, Lw.sc->pass_count + P - 1));
    return LPR_OK;
}

// ---------------------------------------------------------------------------
// Round graphs: the kernels of one round captured once per (buffers, shape,
// schedule) and replayed with a single launch per round.
// ---------------------------------------------------------------------------
struct GraphKey {
    int device;
    const void *ws;
    const void *caps[6];
    int64_t N;
    int B, T, TH, K, L, P;
    bool operator==(const GraphKey &o) const {
        return device == o.device && ws == o.ws && N == o.N && B == o.B &&
               T == o.T && TH == o.TH && K == o.K && L == o.L && P == o.P &&
               std::equal(caps, caps + 6, o.caps);
    }
};

struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
    uint64_t stamp;
};

static std::mutex g_graph_mu;
static std::vector<GraphEntry> g_graphs;
static uint64_t g_graph_clock = 0;
constexpr size_t MAX_GRAPHS = 8;

static lpr_status capture_stream(int device, hipStream_t *out) {
    static std::mutex mu;
    static std::vector<std::pair<int, hipStream_t>> streams;
    std::lock_guard<std::mutex> lk(mu);
    for (auto &p : streams)
        if (p.first == device) {
            *out = p.second;
            return LPR_OK;
        }
    hipStream_t st;
    LPR_TRY_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    streams.emplace_back(device, st);
    *out = st;
    return LPR_OK;
}

// Finds or captures the round graph for `key` and launches it on `s` (under
// the cache lock, so an eviction cannot destroy it in between).
template <int TH>
static lpr_status launch_round_graph(const GraphKey &key, const Dev &D, Layout &Lw,
                                     dim3 grid, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto &e : g_graphs)
        if (e.key == key) {
            e.stamp = ++g_graph_clock;
            LPR_TRY_HIP(hipGraphLaunch(e.exec, s));
            return LPR_OK;
        }
    hipStream_t cs;
    LPR_TRY(capture_stream(key.device, &cs));
    hipGraph_t g;
    LPR_TRY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const lpr_status st = enqueue_round<TH>(cs, D, Lw, grid, key.B, key.K, key.L,
                                            key.P, nullptr, nullptr);
    const hipError_t ce = hipStreamEndCapture(cs, &g);
    if (st != LPR_OK) return st;
    if (ce != hipSuccess) {
        set_error("hipStreamEndCapture failed: %s", hipGetErrorString(ce));
        return LPR_EDEVICE;
    }
    hipGraphExec_t ex;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ie));
        return LPR_EDEVICE;
    }
    if (g_graphs.size() >= MAX_GRAPHS) {
        auto lru = std::min_element(g_graphs.begin(), g_graphs.end(),
                                    [](const GraphEntry &a, const GraphEntry &b) {
                                        return a.stamp < b.stamp;
                                    });
        (void)hipGraphExecDestroy(lru->exec);
        g_graphs.erase(lru);
    }
    g_graphs.push_back(GraphEntry{key, ex, ++g_graph_clock});
    LPR_TRY_HIP(hipGraphLaunch(ex, s));
    return LPR_OK;
}

// Pinned host copy of the scalars, one per calling thread.
static lpr_status host_scalars(Scalars **out) {
    static thread_local Scalars *h = nullptr;
    if (!h) LPR_TRY_HIP(hipHostMalloc(reinterpret_cast<void **>(&h), sizeof(Scalars)));
    *out = h;
    return LPR_OK;
}

template <int TH>
static lpr_status read_scalars(hipStream_t s, Layout &Lw, Scalars **host) {
    LPR_TRY(host_scalars(host));
    LPR_TRY_HIP(hipMemcpyAsync(*host, Lw.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    LPR_TRY_HIP(hipStreamSynchronize(s));
    if ((*host)->err) {
        set_error((*host)->err & 1 ? "negative capacity"
                                   : "capacity exceeds LPR_GRID_MAX_CAP");
        return (*host)->err & 1 ? LPR_EINVAL : LPR_ERANGE;
    }
    return LPR_OK;
}

template <int TH>
static lpr_status solve(const Params &P, int B, const std::vector<Inst> &insts,
                        const std::vector<int32_t> &tile_inst, Dev D,
                        Layout &Lw, const GraphKey &base_key, int64_t *flow_values,
                        uint8_t *side, lpr_grid_stats *stats, hipStream_t s) {
    const int T = int(tile_inst.size());
    const dim3 grid(T);
    EventTimer t_sweep(s), t_bfs(s);
    if (P.timing) {
        t_sweep.enable();
        t_bfs.enable();
    }
    double sweep_ms = 0, bfs_ms = 0;
    int64_t rounds = 0, sweeps = 0, bfs_passes = 0, cut_passes = 0;

    LPR_TRY_HIP(hipMemcpyAsync(Lw.inst, insts.data(), sizeof(Inst) * B,
                               hipMemcpyHostToDevice, s));
    LPR_TRY_HIP(hipMemcpyAsync(Lw.tile_inst, tile_inst.data(),
                               sizeof(int32_t) * T, hipMemcpyHostToDevice, s));
    LPR_TRY(fill_i32(Lw.done, 0, B, s));
    LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(Lw.counters), 0, 8, s));
    LPR_TRY(fill_i32(&Lw.sc->err, 0, 1, s));
    Kern<TH>::init(grid, s, D);
    LPR_TRY_HIP(hipGetLastError());

    // First global relabel: eager, to its fixpoint; its pass count sets the
    // number of BFS passes per later round.
    int dirty_sel = 0;
    Kern<TH>::bfs_seed(grid, s, D, Lw.dirty[0], Lw.dirty[1]);
    LPR_TRY(relax_to_fixpoint<TH>(false, s, D, Lw, &dirty_sel, grid, t_bfs,
                                  &bfs_passes));
    int PB = int(std::min<int64_t>(MAX_PASS_SLOTS, std::max<int64_t>(4, bfs_passes / 2 + 2)));
    PB += PB & 1;
    LPR_TRY(enqueue_count<TH>(s, D, Lw, grid, B, nullptr));
    Scalars *host = nullptr;
    LPR_TRY(read_scalars<TH>(s, Lw, &host));
    const bool use_graph = !P.timing && (P.K % 2 == 0);
    bool converged = false;
    for (;;) {
        if (host->total_active == 0) {
            converged = true;
            break;
        }
        if (rounds >= P.max_rounds) break;
        ++rounds;
        sweeps += P.K;
        bfs_passes += PB;
        if (use_graph) {
            GraphKey key = base_key;
            key.K = P.K;
            key.L = P.L;
            key.P = PB;
            LPR_TRY(launch_round_graph<TH>(key, D, Lw, grid, s));
        } else {
            // odd K alternates the active-flag buffers; keep it on the eager path
            if (P.K % 2) {
                LPR_TRY(enqueue_round<TH>(s, D, Lw, grid, B, P.K + 1, P.L, PB,
                                          &t_sweep, &t_bfs));
                sweeps += 1;
            } else {
                LPR_TRY(enqueue_round<TH>(s, D, Lw, grid, B, P.K, P.L, PB, &t_sweep,
                                          &t_bfs));
            }
        }
        LPR_TRY(read_scalars<TH>(s, Lw, &host));
        if (host->pass_count[PB - 1] != 0) {
            // the BFS needed more than PB passes: finish it, recount, and give
            // the following rounds more passes
            dirty_sel = 0;
            LPR_TRY(relax_to_fixpoint<TH>(false, s, D, Lw, &dirty_sel, grid, t_bfs,
                                          &bfs_passes));
            LPR_TRY(enqueue_count<TH>(s, D, Lw, grid, B, nullptr));
            LPR_TRY(read_scalars<TH>(s, Lw, &host));
            PB = std::min(MAX_PASS_SLOTS, PB + 4);
        }
        LPR_TRY(t_bfs.harvest(&bfs_ms));
        LPR_TRY(t_sweep.harvest(&sweep_ms));
    }
    if (!converged) {
        set_error("grid max-flow: round budget (%d) exhausted", P.max_rounds);
        return LPR_EBUDGET;
    }
    LPR_TRY(fill_i64(flow_values, 0, B, s));
    Kern<TH>::flow(grid, s, D, flow_values);
    LPR_TRY_HIP(hipGetLastError());
    if (side) {
        // every instance takes part in the closure
        dirty_sel = 0;
        Kern<TH>::cut_seed(grid, s, D, Lw.dirty[0], Lw.dirty[1]);
        LPR_TRY_HIP(hipGetLastError());
        EventTimer none(s);
        LPR_TRY(relax_to_fixpoint<TH>(true, s, D, Lw, &dirty_sel, grid, none,
                                      &cut_passes));
        Kern<TH>::cut_write(grid, s, D, side);
        LPR_TRY_HIP(hipGetLastError());
    }
    unsigned long long cnt[8];
    LPR_TRY_HIP(hipMemcpyAsync(cnt, Lw.counters, sizeof(cnt),
                               hipMemcpyDeviceToHost, s));
    LPR_TRY_HIP(hipStreamSynchronize(s));
    LPR_TRY(t_bfs.harvest(&bfs_ms));
    LPR_TRY(t_sweep.harvest(&sweep_ms));
    if (stats) {
        stats->rounds = rounds + 1;
        stats->sweeps = sweeps;
        stats->bfs_passes = bfs_passes;
        stats->cut_passes = cut_passes;
        stats->pushes = int64_t(cnt[0]);
        stats->relabels = int64_t(cnt[1]);
        stats->tiles_swept = int64_t(cnt[2]);
        stats->tiles_relaxed = int64_t(cnt[3]);
        stats->tile_rows = TH;
        stats->local_iters = P.L;
        stats->sweeps_per_relabel = P.K;
        stats->sweep_ms = sweep_ms;
        stats->bfs_ms = bfs_ms;
    }
    return LPR_OK;
}

// ---------------------------------------------------------------------------
// Schedules: (tile rows, local iterations, sweeps per relabel) per size class
// (floor(log2(total pixels))).  Defaults come from a sweep on MI355X;
// lpr_grid_tune replaces them per class for this process and, when the
// environment variable LPR_GRID_TUNE_FILE names a file, persists them there
// (one "class tile_rows local_iters sweeps_per_relabel" line per class).
// ---------------------------------------------------------------------------
struct Sched {
    int TH, L, K;
};

static std::mutex g_sched_mu;
static std::map<int, Sched> g_sched;
static bool g_sched_loaded = false;

static int size_class(int64_t N) {
    int c = 0;
    while ((int64_t(1) << (c + 1)) <= N) ++c;
    return c;
}

static bool valid_sched(const Sched &s) {
    return (s.TH == 8 || s.TH == 16 || s.TH == 32) && s.L >= 1 && s.L <= 4096 &&
           s.K >= 1 && s.K <= 4096;
}

static void load_sched_file_locked() {
    if (g_sched_loaded) return;
    g_sched_loaded = true;
    const char *path = std::getenv("LPR_GRID_TUNE_FILE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    int c;
    Sched sc;
    while (std::fscanf(f, "%d %d %d %d", &c, &sc.TH, &sc.L, &sc.K) == 4)
        if (c >= 0 && c < 64 && valid_sched(sc)) g_sched[c] = sc;
    std::fclose(f);
}

static Sched default_sched(int64_t N) {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    load_sched_file_locked();
    const auto it = g_sched.find(size_class(N));
    if (it != g_sched.end()) return it->second;
    return Sched{8, 16, 4};
}

static void store_sched(int64_t N, const Sched &sc) {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    load_sched_file_locked();
    g_sched[size_class(N)] = sc;
    const char *path = std::getenv("LPR_GRID_TUNE_FILE");
    if (!path) return;
    FILE *f = std::fopen(path, "w");
    if (!f) return;
    for (const auto &e : g_sched)
        std::fprintf(f, "%d %d %d %d\n", e.first, e.second.TH, e.second.L, e.second.K);
    std::fclose(f);
}

static lpr_status run(int32_t B, const int32_t *H, const int32_t *W,
                      const int64_t *node_offset, const int32_t *const caps[6],
                      int64_t *flow_values, uint8_t *side,
                      const lpr_grid_opts *opts, lpr_grid_stats *stats,
                      void *workspace, size_t ws_bytes, void *stream) {
    clear_error();
    if (B < 1 || !H || !W || !node_offset) {
        set_error("invalid batch description");
        return LPR_EINVAL;
    }
    for (int i = 0; i < 6; ++i)
        if (!caps[i]) {
            set_error("NULL capacity array");
            return LPR_EINVAL;
        }
    if (!flow_values || !workspace) {
        set_error("NULL flow_values or workspace");
        return LPR_EINVAL;
    }
    if (node_offset[0] != 0) {
        set_error("node_offset[0] must be 0");
        return LPR_EINVAL;
    }
    for (int b = 0; b < B; ++b) {
        if (H[b] < 1 || W[b] < 1 || int64_t(H[b]) * W[b] >= (int64_t(1) << 30)) {
            set_error("instance %d: bad shape %d x %d", b, H[b], W[b]);
            return LPR_EINVAL;
        }
        if (node_offset[b + 1] != node_offset[b] + int64_t(H[b]) * W[b]) {
            set_error("node_offset is not the prefix sum of H*W at %d", b);
            return LPR_EINVAL;
        }
    }
    if (node_offset[B] >= (int64_t(1) << 30)) {
        // the kernels address a pixel's word by a 32-bit byte offset
        set_error("batch of %lld pixels exceeds 2^30", (long long)node_offset[B]);
        return LPR_EINVAL;
    }
    const Sched ds = default_sched(node_offset[B]);
    Params P;
    P.TH = ds.TH;
    P.L = ds.L;
    P.K = ds.K;
    P.max_rounds = 1 << 16;
    P.timing = false;
    if (opts) {
        if (opts->tile_rows) P.TH = opts->tile_rows;
        if (opts->local_iters) P.L = opts->local_iters;
        if (opts->sweeps_per_relabel) P.K = opts->sweeps_per_relabel;
        if (opts->max_rounds) P.max_rounds = opts->max_rounds;
        P.timing = (opts->flags & LPR_GRID_TIME_KERNELS) != 0;
    }
    if (!(P.TH == 8 || P.TH == 16 || P.TH == 32) || P.L < 1 || P.L > 4096 ||
        P.K < 1 || P.K > 4096 || P.max_rounds < 1) {
        set_error("invalid lpr_grid_opts");
        return LPR_EINVAL;
    }
    const int64_t N = node_offset[B];
    std::vector<Inst> insts(B);
    std::vector<int32_t> tile_inst;
    for (int b = 0; b < B; ++b) {
        Inst &I = insts[b];
        I.off = node_offset[b];
        I.H = H[b];
        I.W = W[b];
        I.tiles_x = ceil_div(W[b], TW);
        I.tiles_y = ceil_div(H[b], P.TH);
        I.tile_base = int32_t(tile_inst.size());
        I.HV = H[b] * W[b] + 2;
        tile_inst.insert(tile_inst.end(), size_t(I.tiles_x) * I.tiles_y, b);
    }
    const int64_t T = int64_t(tile_inst.size());
    if (T >= (int64_t(1) << 31)) {
        set_error("too many tiles");
        return LPR_EINVAL;
    }
    const size_t need = workspace_bytes(B, H, W);
    if (ws_bytes < need) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
        return LPR_ENOMEM;
    }
    Layout Lw;
    Carver cv = carve(Carver(workspace, ws_bytes), N, T, B, &Lw);
    if (!cv.fits()) {
        set_error("workspace layout overflow");
        return LPR_ENOMEM;
    }
    Dev D;
    D.e = Lw.st[0];
    D.h = Lw.st[1];
    D.rr = Lw.st[2];
    D.rl = Lw.st[3];
    D.rd = Lw.st[4];
    D.ru = Lw.st[5];
    D.rs = Lw.st[6];
    D.cap_src = caps[0];
    D.cap_snk = caps[1];
    D.cap_r = caps[2];
    D.cap_l = caps[3];
    D.cap_d = caps[4];
    D.cap_u = caps[5];
    D.inst = Lw.inst;
    D.tile_inst = Lw.tile_inst;
    D.inst_active = Lw.inst_active;
    D.done = Lw.done;
    D.counters = Lw.counters;
    D.sc = Lw.sc;
    D.ntiles = int32_t(T);
    D.ninst = B;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GraphKey key{};
    LPR_TRY_HIP(hipGetDevice(&key.device));
    key.ws = workspace;
    for (int i = 0; i < 6; ++i) key.caps[i] = caps[i];
    key.N = N;
    key.B = B;
    key.T = int(T);
    key.TH = P.TH;
    CallTimer call(s);
    call.start();
    lpr_status st;
    switch (P.TH) {
        case 8:
            st = solve<8>(P, B, insts, tile_inst, D, Lw, key, flow_values, side, stats, s);
            break;
        case 16:
            st = solve<16>(P, B, insts, tile_inst, D, Lw, key, flow_values, side, stats, s);
            break;
        default:
            st = solve<32>(P, B, insts, tile_inst, D, Lw, key, flow_values, side, stats, s);
            break;
    }
    if (st != LPR_OK) {
        (void)hipStreamSynchronize(s);
        return st;
    }
    double ms = 0;
    LPR_TRY(call.stop_ms(&ms));
    if (stats) stats->total_ms = ms;
    return LPR_OK;
}

}  // namespace grid
}  // namespace lpr

using namespace lpr;

extern "C" size_t lpr_grid_maxflow_workspace(int32_t H, int32_t W) {
    if (H < 1 || W < 1) return 0;
    return grid::workspace_bytes(1, &H, &W);
}

extern "C" size_t lpr_grid_maxflow_batched_workspace(int32_t B, const int32_t *H,
                                                      const int32_t *W) {
    if (B < 1 || !H || !W) return 0;
    for (int b = 0; b < B; ++b)
        if (H[b] < 1 || W[b] < 1) return 0;
    return grid::workspace_bytes(B, H, W);
}

extern "C" lpr_status lpr_grid_maxflow(int32_t H, int32_t W,
                                       const int32_t *cap_src,
                                       const int32_t *cap_snk,
                                       const int32_t *cap_right,
                                       const int32_t *cap_left,
                                       const int32_t *cap_down,
                                       const int32_t *cap_up,
                                       int64_t *flow_value,
                                       uint8_t *source_side,
                                       const lpr_grid_opts *opts,
                                       lpr_grid_stats *stats, void *workspace,
                                       size_t workspace_bytes, void *stream) {
    const int32_t *caps[6] = {cap_src, cap_snk, cap_right, cap_left, cap_down, cap_up};
    const int64_t off[2] = {0, int64_t(H) * W};
    if (H < 1 || W < 1) {
        clear_error();
        set_error("bad shape %d x %d", H, W);
        return LPR_EINVAL;
    }
    return grid::run(1, &H, &W, off, caps, flow_value, source_side, opts, stats,
                     workspace, workspace_bytes, stream);
}

extern "C" lpr_status lpr_grid_maxflow_batched(
    int32_t B, const int32_t *H, const int32_t *W, const int64_t *node_offset,
    const int32_t *cap_src, const int32_t *cap_snk, const int32_t *cap_right,
    const int32_t *cap_left, const int32_t *cap_down, const int32_t *cap_up,
    int64_t *flow_values, uint8_t *source_side, const lpr_grid_opts *opts,
    lpr_grid_stats *stats, void *workspace, size_t workspace_bytes,
    void *stream) {
    const int32_t *caps[6] = {cap_src, cap_snk, cap_right, cap_left, cap_down, cap_up};
    return grid::run(B, H, W, node_offset, caps, flow_values, source_side, opts,
                     stats, workspace, workspace_bytes, stream);
}

extern "C" lpr_status lpr_grid_tune(int32_t B, const int32_t *H, const int32_t *W,
                                    const int64_t *node_offset,
                                    const int32_t *cap_src, const int32_t *cap_snk,
                                    const int32_t *cap_right, const int32_t *cap_left,
                                    const int32_t *cap_down, const int32_t *cap_up,
                                    int64_t *flow_values, int32_t reps,
                                    lpr_grid_opts *best, double *best_ms,
                                    void *workspace, size_t workspace_bytes,
                                    void *stream) {
    const int32_t *caps[6] = {cap_src, cap_snk, cap_right, cap_left, cap_down, cap_up};
    if (B < 1 || !node_offset || !flow_values || reps < 1 || reps > 100) {
        clear_error();
        set_error("invalid tuning arguments");
        return LPR_EINVAL;
    }
    static const int THs[3] = {8, 16, 32};
    static const int Ls[4] = {4, 8, 16, 32};
    static const int Ks[3] = {2, 4, 8};
    std::vector<int64_t> ref(B), got(B);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double best_t = 1e300;
    grid::Sched best_s{8, 16, 4};
    bool have_ref = false;
    for (int th : THs)
        for (int l : Ls)
            for (int k : Ks) {
                lpr_grid_opts o{};
                o.tile_rows = th;
                o.local_iters = l;
                o.sweeps_per_relabel = k;
                double t_min = 1e300;
                for (int r = 0; r <= reps; ++r) {  // the first run warms up
                    lpr_grid_stats st{};
                    LPR_TRY(grid::run(B, H, W, node_offset, caps, flow_values, nullptr,
                                      &o, &st, workspace, workspace_bytes, stream));
                    if (r > 0) t_min = std::min(t_min, st.total_ms);
                }
                LPR_TRY_HIP(hipMemcpyAsync(got.data(), flow_values, sizeof(int64_t) * B,
                                           hipMemcpyDeviceToHost, s));
                LPR_TRY_HIP(hipStreamSynchronize(s));
                if (!have_ref) {
                    ref = got;
                    have_ref = true;
                } else if (got != ref) {
                    set_error("schedules disagree on a flow value (tile rows %d, "
                              "local iterations %d, sweeps %d)", th, l, k);
                    return LPR_EDEVICE;
                }
                if (t_min < best_t) {
                    best_t = t_min;
                    best_s = grid::Sched{th, l, k};
                }
            }
    grid::store_sched(node_offset[B], best_s);
    if (best) {
        *best = lpr_grid_opts{};
        best->tile_rows = best_s.TH;
        best->local_iters = best_s.L;
        best->sweeps_per_relabel = best_s.K;
    }
    if (best_ms) *best_ms = best_t;
    return LPR_OK;
}
