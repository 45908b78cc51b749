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
//  * 64 x TH tiles, one wavefront per tile (four tiles per 256-thread
//    workgroup, no barrier): lane c holds column c of the tile in registers
//    and runs `local_iters` lock-free iterations over the rows; horizontal
//    neighbours are read and pushed to by cross-lane shuffles, vertical ones
//    inside the lane's registers.  Flow pushed across the tile edge goes to
//    global memory with device-scope atomics when the visit ends, and the
//    tile's own edge excesses are merged back by atomic deltas.  Every value
//    a pixel reads of another pixel is a lower bound of the true one (excess
//    and residuals are only decreased by their owner, heights only grow
//    between global relabels), which is exactly the staleness Hong's
//    argument admits.
//  * Active-tile flags double-buffered across sweep launches so that quiet
//    tiles cost one flag read.
//  * The BFS (and the cut closure) is a Bellman-Ford style relaxation run to a
//    local fixpoint inside each register-resident tile; tiles whose edge
//    values changed mark their neighbours dirty, and passes repeat until no
//    tile is dirty.  The least fixpoint is exactly the BFS level of every
//    pixel.
//  * Batched solves share every launch: the tile table spans all instances,
//    and an instance whose count reaches zero retires from later rounds.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <chrono>
#include <map>
#include <mutex>
#include <optional>
#include <vector>

#include "lpr_internal.h"

namespace lpr {
namespace grid {

constexpr int TW = 64;        // tile width: one wavefront per tile row
constexpr int NT = 256;       // threads per tile workgroup
constexpr int RPP = NT / TW;  // tile rows covered per thread pass (4)
constexpr int MAX_PASS_SLOTS = 64;
constexpr int RELAX_TH = 32;  // tile height of the relaxation kernels (BFS, cut)

// Element at a 32-bit byte offset from a wave-uniform base: every per-pixel
// array shares the offset, so the compiler keeps one VGPR per pixel instead of
// a 64-bit address per array (the batch holds fewer than 2^30 pixels).
template <class T>
__device__ __forceinline__ T &at(T *base, uint32_t byte_off) {
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off);
}

// Cross-lane moves by DPP (a VALU modifier, no LDS round trip).
// from_left(v, f): lane i gets v of lane i-1, lane 0 gets its own f.
// from_right(v, f): lane i gets v of lane i+1, lane 63 gets its own f.
__device__ __forceinline__ int32_t from_left(int32_t v, int32_t f) {
    return __builtin_amdgcn_update_dpp(f, v, 0x138, 0xF, 0xF, false);  // wave_shr:1
}
__device__ __forceinline__ int32_t from_right(int32_t v, int32_t f) {
    return __builtin_amdgcn_update_dpp(f, v, 0x130, 0xF, 0xF, false);  // wave_shl:1
}

// Segmented min scans across the 64 lanes of a wavefront (Hillis-Steele
// doubling inside each 16-lane row by DPP, then the row carries).
// scan_from_left: v of lane x becomes min v[k] over s(x) <= k <= x, where
// dl = x - s(x) (the lanes s(x)+1 .. x each accept their left neighbour).
__device__ __forceinline__ int32_t scan_from_left(int32_t v, int dl, int lane) {
#define LPR_STEP(o, ctrl)                                                    \
    {                                                                        \
        const int32_t t = __builtin_amdgcn_update_dpp(INT_MAX, v, ctrl, 0xF, \
                                                      0xF, false);           \
        if (dl >= o) v = min(v, t);                                          \
    }
    LPR_STEP(1, 0x111) LPR_STEP(2, 0x112) LPR_STEP(4, 0x114) LPR_STEP(8, 0x118)
#undef LPR_STEP
    // rows 1 and 3 take the inclusive result of lane 15 / 47 (row_bcast:15)
    int32_t t = __builtin_amdgcn_update_dpp(INT_MAX, v, 0x142, 0xA, 0xF, false);
    if (dl > (lane & 15)) v = min(v, t);
    // rows 2 and 3 take the result of lane 31 (row_bcast:31)
    t = __builtin_amdgcn_update_dpp(INT_MAX, v, 0x143, 0xC, 0xF, false);
    if (dl > lane - 32) v = min(v, t);
    return v;
}
// scan_from_right: v of lane x becomes min v[k] over x <= k <= e(x), where
// dr = e(x) - x (the lanes x .. e(x)-1 each accept their right neighbour).
__device__ __forceinline__ int32_t scan_from_right(int32_t v, int dr, int lane) {
#define LPR_STEP(o, ctrl)                                                    \
    {                                                                        \
        const int32_t t = __builtin_amdgcn_update_dpp(INT_MAX, v, ctrl, 0xF, \
                                                      0xF, false);           \
        if (dr >= o) v = min(v, t);                                          \
    }
    LPR_STEP(1, 0x101) LPR_STEP(2, 0x102) LPR_STEP(4, 0x104) LPR_STEP(8, 0x108)
#undef LPR_STEP
    // rows 0 and 2 take the result of lane 16 / 48 (first lane of the next row)
    const int32_t a = __builtin_amdgcn_readlane(v, 16);
    const int32_t b = __builtin_amdgcn_readlane(v, 48);
    if (!(lane & 16) && dr >= 16 - (lane & 15)) v = min(v, lane < 32 ? a : b);
    // rows 0 and 1 take the result of lane 32
    const int32_t c = __builtin_amdgcn_readlane(v, 32);
    if (lane < 32 && dr >= 32 - lane) v = min(v, c);
    return v;
}

// Plain (unsegmented) min scans: prefix_min gives lane x the minimum over
// lanes 0..x, suffix_min the minimum over lanes x..63.  Every step is one DPP
// min with no lane condition.  The relaxation turns its segmented scans into
// these by adding to each lane a multiple of 2^OFF_SHIFT that grows with the
// segment's distance from the scan's end, so no lane of another segment can
// win (exact while the labels and that multiple stay below 2^31).
constexpr int OFF_SHIFT = 25;
constexpr int32_t OFFSET_SCAN_MAX_HV = (1 << OFF_SHIFT) - 64;
__device__ __forceinline__ int32_t prefix_min(int32_t v) {
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x111, 0xF, 0xF, false));  // row_shr:1
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x112, 0xF, 0xF, false));  // row_shr:2
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x114, 0xF, 0xF, false));  // row_shr:4
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x118, 0xF, 0xF, false));  // row_shr:8
    // rows 1 and 3 take lane 15 / 47, then rows 2 and 3 take lane 31
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x142, 0xA, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x143, 0xC, 0xF, false));
    return v;
}
__device__ __forceinline__ int32_t suffix_min(int32_t v, int lane) {
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x101, 0xF, 0xF, false));  // row_shl:1
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x102, 0xF, 0xF, false));  // row_shl:2
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x104, 0xF, 0xF, false));  // row_shl:4
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x108, 0xF, 0xF, false));  // row_shl:8
    // the first lane of each 16-lane row now holds that row's minimum; a row
    // takes the minimum of the rows to its right
    const int32_t a = __builtin_amdgcn_readlane(v, 16);
    const int32_t b = __builtin_amdgcn_readlane(v, 32);
    const int32_t c = __builtin_amdgcn_readlane(v, 48);
    const int32_t bc = min(b, c);
    const int32_t t = lane < 32 ? (lane < 16 ? min(a, bc) : bc) : (lane < 48 ? c : INT_MAX);
    return min(v, t);
}

// Appends the values of the lanes with `take` to a work list: one atomic add
// on the list's count reserves their slots (in lane order), so a wavefront
// that lists several tiles waits for one round trip, not one per tile.
__device__ __forceinline__ void list_append(int32_t *list, int32_t *cnt, bool take, int32_t v,
                                            int lane) {
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int lead = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == lead) base = atomicAdd(cnt, __popcll(m));
    base = __builtin_amdgcn_readlane(base, lead);
    if (take) list[base + __popcll(m & ((1ull << lane) - 1))] = v;
}

struct Inst {
    int64_t off;      // first pixel of the instance in the packed arrays
    int32_t H, W;
    int32_t tiles_x, tiles_y;
    int32_t tile_base;
    int32_t HV;       // |V| = H*W + 2, the gap height
    int32_t tiles_y_r;    // tile rows of the relaxation tiling (RELAX_TH)
    int32_t tile_base_r;  // first relaxation tile of the instance
};

struct Scalars {
    unsigned long long total_active;  // active pixels after the last round
    int32_t err;
    int32_t all_done;   // every instance retired
    int32_t rounds;     // finished rounds that still had an unretired instance
    int32_t open_bfs;   // global relabels that needed more passes than they had
    int32_t max_need;   // most passes a converged global relabel needed
    int32_t seed_count; // entries of the first relaxation list of a relabel
    int32_t act_cnt[3]; // entries of the three active-tile lists of the sweeps
    int32_t pass_count[MAX_PASS_SLOTS];  // entries each relaxation pass listed
};

// Snapshot of the residual network taken at a round boundary, as bit masks:
// for every 64 x 32 relaxation tile and every column c of it, one 32-bit word
// per mask (bit r = row r of the tile): arc to the right, left, down and up
// neighbour with residual capacity, arc to t, and excess.  A global relabel
// reads only these words, so it computes the exact BFS of the state at the
// snapshot even while push sweeps change the live state.
constexpr int NMASK = 6;
constexpr int MK_R = 0, MK_L = 1, MK_D = 2, MK_U = 3, MK_T = 4, MK_E = 5;
// Round-boundary steps (k_boundary)
constexpr unsigned BD_ADOPT = 1, BD_COUNT = 2, BD_SNAPSHOT = 4;

struct Dev {
    int32_t *e, *h, *rr, *rl, *rd, *ru, *rs;
    int32_t *lab;       // labels of the global relabel (and of the cut closure)
    uint32_t *amask;    // snapshot masks: [relaxation tile][NMASK][64 columns]
    const int32_t *cap_src, *cap_snk, *cap_r, *cap_l, *cap_d, *cap_u;
    const Inst *inst;
    const int32_t *tile_inst;    // instance of every sweep tile (64 x TH)
    const int32_t *tile_inst_r;  // instance of every relaxation tile (64 x RELAX_TH)
    unsigned long long *inst_active;  // per-instance active pixels (last count)
    unsigned long long *inst_exact;   // per-instance pixels of the snapshot that
                                      // hold excess and reach t
    int32_t *done;                    // per-instance: no active pixel left
    unsigned long long *counters;     // pushes, relabels, tiles swept,
                                      // tiles relaxed (BFS), tiles relaxed (cut),
                                      // device-scope atomics of the sweeps,
                                      // BFS passes that relaxed a tile
    Scalars *sc;
    // Work lists, three of each (a launch reads one, appends to the next and
    // may clear the third): a flag per tile (listed or not) and the list.
    int32_t *act[3], *alist[3];    // sweep tiles with work
    int32_t *dirty[3], *dlist[3];  // relaxation tiles to relax
    int32_t ntiles, ntiles_r;
    int32_t ninst;
    int32_t seg_scan;  // relax rows with the segmented scans (host's choice)
};

__device__ __forceinline__ int next3(int i) { return i == 2 ? 0 : i + 1; }
__device__ __forceinline__ int prev3(int i) { return i == 0 ? 2 : i - 1; }

struct Geo {
    int inst, H, W, HV, y0, x0, tx, ty, tiles_x, tiles_y;
    int64_t off;
};

// Geometry of tile t of the sweep tiling (RT = false) or of the relaxation
// tiling (RT = true, TH = RELAX_TH).
template <int TH, bool RT = false>
__device__ inline Geo tile_geo(const Dev &D, int t) {
    Geo g;
    g.inst = RT ? D.tile_inst_r[t] : D.tile_inst[t];
    const Inst I = D.inst[g.inst];
    g.H = I.H;
    g.W = I.W;
    g.HV = I.HV;
    g.off = I.off;
    g.tiles_x = I.tiles_x;
    g.tiles_y = RT ? I.tiles_y_r : I.tiles_y;
    int lt = t - (RT ? I.tile_base_r : I.tile_base);
    g.ty = lt / I.tiles_x;
    g.tx = lt - g.ty * I.tiles_x;
    g.y0 = g.ty * TH;
    g.x0 = g.tx * TW;
    return g;
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
    // every row's six loads first, from a clamped valid pixel (the arcs that
    // leave the grid are read and then zeroed), then the checks and stores
    const int c = threadIdx.x & (TW - 1);
    const int x = g.x0 + c;
    const int xc = min(x, g.W - 1);
    int32_t v[TH / RPP][6];
#pragma unroll
    for (int k = 0; k < TH / RPP; ++k) {
        const int y = min(g.y0 + (threadIdx.x >> 6) + RPP * k, g.H - 1);
        const int64_t p = g.off + int64_t(y) * g.W + xc;
        v[k][0] = D.cap_src[p];
        v[k][1] = D.cap_snk[p];
        v[k][2] = D.cap_r[p];
        v[k][3] = D.cap_l[p];
        v[k][4] = D.cap_d[p];
        v[k][5] = D.cap_u[p];
    }
    int bad = 0;
#pragma unroll
    for (int k = 0; k < TH / RPP; ++k) {
        const int y = g.y0 + (threadIdx.x >> 6) + RPP * k;
        if (y >= g.H || x >= g.W) continue;
        const int64_t p = g.off + int64_t(y) * g.W + x;
        const int32_t src = v[k][0], snk = v[k][1];
        const int32_t cr = (x + 1 < g.W) ? v[k][2] : 0;
        const int32_t cl = (x > 0) ? v[k][3] : 0;
        const int32_t cd = (y + 1 < g.H) ? v[k][4] : 0;
        const int32_t cu = (y > 0) ? v[k][5] : 0;
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

constexpr int RW = 8;  // rows per wavefront of the cooperative relaxation
constexpr int RELAX_GRID = 2048;  // most workgroups of a relaxation launch

// The in-tile fixpoint of one relaxation tile: wavefront w holds rows
// RW w .. RW w + RW - 1 (labels d, lane c = column c) with the arcs usable in
// each direction (bit r of mR, mL, mD, mU), the halo above / below the
// wavefront (top, bot) and what the side halo offers lanes 0 / 63 (hs); on
// return every label is at the least fixpoint of the tile given the halo.
// Called by the whole workgroup (barriers inside); `edge` is its LDS.
template <bool SEG, int INC>
__device__ __forceinline__ void tile_fixpoint(int32_t (&d)[RW], uint32_t mR, uint32_t mL,
                                              uint32_t mD, uint32_t mU,
                                              const int32_t (&hs)[RW], int32_t top,
                                              int32_t bot, int lane, int w,
                                              int32_t (&edge)[4][2][64]) {
    // per row: the segment extents (SEG) or the scan offsets, less / plus the
    // column shift of the min-plus form
    int32_t segL[RW], segR[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const uint64_t brkL = __ballot(!((mL >> r) & 1u)) | 1ull;
        const uint64_t brkR = __ballot(!((mR >> r) & 1u)) | (1ull << 63);
        if constexpr (SEG) {
            const uint64_t low = lane == 63 ? ~0ull : (2ull << lane) - 1;
            const int sx = 63 - __clzll((long long)(brkL & low));
            const int ex = lane + __ffsll((unsigned long long)(brkR >> lane)) - 1;
            segL[r] = lane - sx;
            segR[r] = ex - lane;
        } else {
            // breaks at or left of the lane (left scan), strictly left of it
            // (right scan): the lane's segment index in each direction
            const uint32_t bl = __builtin_amdgcn_mbcnt_hi(
                uint32_t(brkL >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(brkL), 0u));
            const uint32_t gl = bl + uint32_t((brkL >> lane) & 1ull);
            const uint32_t gr = __builtin_amdgcn_mbcnt_hi(
                uint32_t(brkR >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(brkR), 0u));
            segL[r] = int32_t((64u - gl) << OFF_SHIFT) - INC * lane;
            segR[r] = int32_t(gr << OFF_SHIFT) + INC * lane;
        }
    }
    edge[w][0][lane] = d[0];
    edge[w][1][lane] = d[RW - 1];
    __syncthreads();
    if (w > 0) top = edge[w - 1][1][lane];
    if (w < 3) bot = edge[w + 1][0][lane];
    uint32_t rows = (1u << RW) - 1;           // wavefront-uniform
    for (;;) {
        __syncthreads();                      // the edges above were read
        while ((rows = __builtin_amdgcn_readfirstlane(rows)) != 0) {
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                if (!((rows >> r) & 1u)) continue;
                int32_t nd = min(d[r], hs[r]);
                if constexpr (SEG) {
                    nd = scan_from_left(nd - INC * lane, segL[r], lane) + INC * lane;
                    nd = scan_from_right(nd + INC * lane, segR[r], lane) - INC * lane;
                } else {
                    nd = prefix_min(nd + segL[r]) - segL[r];
                    nd = suffix_min(nd + segR[r], lane) - segR[r];
                }
                d[r] = nd;
            }
            rows = 0;
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int32_t up = r == 0 ? top : d[r - 1];
                const int32_t nd = (mU >> r) & 1u ? min(d[r], up + INC) : d[r];
                if (__any(nd < d[r])) rows |= 1u << r;
                d[r] = nd;
            }
#pragma unroll
            for (int r = RW - 1; r >= 0; --r) {
                const int32_t dn = r == RW - 1 ? bot : d[r + 1];
                const int32_t nd = (mD >> r) & 1u ? min(d[r], dn + INC) : d[r];
                if (__any(nd < d[r])) rows |= 1u << r;
                d[r] = nd;
            }
        }
        edge[w][0][lane] = d[0];
        edge[w][1][lane] = d[RW - 1];
        __syncthreads();
        if (w > 0) {
            const int32_t v = edge[w - 1][1][lane];
            if (__any(v < top)) rows |= 1u;
            top = min(top, v);
        }
        if (w < 3) {
            const int32_t v = edge[w + 1][0][lane];
            if (__any(v < bot)) rows |= 1u << (RW - 1);
            bot = min(bot, v);
        }
        if (!__syncthreads_or(rows != 0)) break;
    }
}

// After a tile's fixpoint: the sides where a label dropped below the value
// the neighbour across read (right 1, left 2, below 4, above 8) are gathered
// in s_ch (0 beforehand), and lanes 0..3 of wavefront 0 list those
// neighbours on the given list (once each: the flags).  Called by the whole
// workgroup.
__device__ __forceinline__ void tile_list_changed(const Dev &D, const Geo &g, int t,
                                                  bool ch_top, bool ch_bot, bool ch_col,
                                                  int lane, int w, int &s_ch,
                                                  int32_t *dirty, int32_t *list,
                                                  int32_t *cnt) {
    const bool e_top = __any(ch_top), e_bot = __any(ch_bot);
    const bool e_left = __any(lane == 0 && ch_col), e_right = __any(lane == 63 && ch_col);
    if (lane == 0) {
        const int bits = (e_right ? 1 : 0) | (e_left ? 2 : 0) | (e_bot ? 4 : 0) | (e_top ? 8 : 0);
        if (bits) atomicOr(&s_ch, bits);
    }
    __syncthreads();
    if (w == 0) {
        const int bits = s_ch;
        int nb = -1;
        if (lane == 0 && (bits & 1) && g.tx + 1 < g.tiles_x) nb = t + 1;
        if (lane == 1 && (bits & 2) && g.tx > 0) nb = t - 1;
        if (lane == 2 && (bits & 4) && g.ty + 1 < g.tiles_y) nb = t + g.tiles_x;
        if (lane == 3 && (bits & 8) && g.ty > 0) nb = t - g.tiles_x;
        const bool fresh = nb >= 0 && atomicExch(&dirty[nb], 1) == 0;
        list_append(list, cnt, fresh, nb, lane);
    }
}

// ---------------------------------------------------------------------------
// Round boundary, over the relaxation tiling (64 x 32, four wavefronts of
// eight rows).  Per pixel, in this order:
//  ADOPT     h = lab: the heights of the next push sweeps are the levels of
//            the global relabel just finished (Algorithm 4.4, with the gap:
//            unreached pixels keep |V|).
//  COUNT     the exact count of the state the labels belong to: pixels whose
//            snapshot held excess and that reach t (lab < |V|); and the
//            activity the next push sweeps start from: e > 0 and h < |V| with
//            the current excess.  Lists every sweep tile (64 x TH) with an
//            active pixel as the sweeps' first list (buffer 0; the three
//            counts are 0 beforehand) and clears the other flags.
//  SNAPSHOT  the snapshot masks and the next global relabel's first pass:
//            the seeds (1 where u_f(p, t) > 0, |V| elsewhere) relaxed inside
//            the tile to their fixpoint, with the halo at the neighbouring
//            pixels' seeds (upper bounds of their levels, read from the sink
//            residuals, which no kernel changes during this launch); the
//            labels are stored and the neighbours across a side where a label
//            fell below its seed form the relabel's first list (every dirty
//            flag and seed_count are 0 beforehand).  A tile no neighbour
//            lists is at its fixpoint for the halo it will see.
// Retired instances are left untouched: no active or dirty flag.
// ---------------------------------------------------------------------------
// `mode` is a template argument, so that no branch on it separates a row's
// loads from the next row's (the three combinations used are instantiated,
// the two with SNAPSHOT in both row-scan forms).
template <int TH, unsigned mode, bool SEG>
__global__ __launch_bounds__(NT) void k_boundary(Dev D) {
    static_assert(RELAX_TH % TH == 0, "sweep tiles nest in relaxation tiles");
    constexpr int RWB = RELAX_TH / 4;  // rows per wavefront
    static_assert(RWB == RW, "the relaxation's row layout");
    const int rt = blockIdx.x;
    const Geo g = tile_geo<RELAX_TH, true>(D, rt);
    const bool retired = D.done[g.inst] != 0;  // workgroup-uniform
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x = g.x0 + lane;
    __shared__ uint32_t smask[NMASK][TW];
    __shared__ uint32_t s_rows;
    __shared__ int32_t edge[4][2][64];  // the fused first relaxation pass
    __shared__ int s_ch;
    for (int i = threadIdx.x; i < NMASK * TW; i += NT) (&smask[0][0])[i] = 0;
    if (threadIdx.x == 0) s_rows = 0;
    uint32_t *tm = D.amask + size_t(rt) * NMASK * TW;
    // the excess mask of the previous snapshot, read before it is replaced
    const uint32_t oldE = (mode & BD_COUNT) ? tm[MK_E * TW + lane] : 0u;
    __syncthreads();
    unsigned long long n_exact = 0, n_act = 0;
    uint32_t my[NMASK] = {0u, 0u, 0u, 0u, 0u, 0u};
    uint32_t act_rows = 0;
    int32_t d[RWB];  // the seeds of the next relabel (snapshot)
#pragma unroll
    for (int i = 0; i < RWB; ++i) d[i] = g.HV;
    if (!retired && x < g.W) {
        // every load of the wavefront's rows first, then the stores: a store
        // between them would keep the next row's loads behind it (the
        // arrays could alias), one memory latency per row.  Rows past H
        // read row y0 (which exists) and are dropped.
        int32_t ev[RWB], hv[RWB], rsv[RWB], rrv[RWB], rlv[RWB], rdv[RWB], ruv[RWB];
#pragma unroll
        for (int i = 0; i < RWB; ++i) {
            const int y = g.y0 + w * RWB + i;
            const int64_t p = g.off + int64_t(y < g.H ? y : g.y0) * g.W + x;
            ev[i] = D.e[p];
            hv[i] = (mode & BD_ADOPT) ? D.lab[p] : (mode & BD_COUNT) ? D.h[p] : 0;
            rsv[i] = rrv[i] = rlv[i] = rdv[i] = ruv[i] = 0;
            if (mode & BD_SNAPSHOT) {
                rsv[i] = D.rs[p];
                rrv[i] = D.rr[p];
                rlv[i] = D.rl[p];
                rdv[i] = D.rd[p];
                ruv[i] = D.ru[p];
            }
        }
#pragma unroll
        for (int i = 0; i < RWB; ++i) {
            const int r = w * RWB + i, y = g.y0 + r;
            if (y >= g.H) break;
            const int64_t p = g.off + int64_t(y) * g.W + x;
            if (mode & BD_ADOPT) D.h[p] = hv[i];
            if (mode & BD_COUNT) {
                n_exact += (((oldE >> r) & 1u) && hv[i] < g.HV) ? 1 : 0;
                const bool a = ev[i] > 0 && hv[i] < g.HV;
                n_act += a ? 1 : 0;
                act_rows |= uint32_t(a) << r;
            }
            if (mode & BD_SNAPSHOT) {
                my[MK_R] |= uint32_t(rrv[i] > 0) << r;
                my[MK_L] |= uint32_t(rlv[i] > 0) << r;
                my[MK_D] |= uint32_t(rdv[i] > 0) << r;
                my[MK_U] |= uint32_t(ruv[i] > 0) << r;
                my[MK_T] |= uint32_t(rsv[i] > 0) << r;
                my[MK_E] |= uint32_t(ev[i] > 0) << r;
                d[i] = rsv[i] > 0 ? 1 : g.HV;
            }
        }
    }
    if (mode & BD_SNAPSHOT) {
#pragma unroll
        for (int m = 0; m < NMASK; ++m)
            if (my[m]) atomicOr(&smask[m][lane], my[m]);
    }
    if (act_rows) atomicOr(&s_rows, act_rows);
    __syncthreads();
    if constexpr ((mode & BD_SNAPSHOT) != 0) {
        if (!retired) {  // workgroup-uniform
            for (int i = threadIdx.x; i < NMASK * TW; i += NT) tm[i] = (&smask[0][0])[i];
            // the relabel's first pass on this tile: this wavefront's rows of
            // the masks, the halo at the neighbouring pixels' seeds
            if (threadIdx.x == 0) s_ch = 0;
            const int sh = RW * w;
            const uint32_t mR = (my[MK_R] >> sh) & 0xFFu, mL = (my[MK_L] >> sh) & 0xFFu;
            const uint32_t mD = (my[MK_D] >> sh) & 0xFFu, mU = (my[MK_U] >> sh) & 0xFFu;
            const bool colv = x < g.W;
            const int yw = g.y0 + RW * w;
            const int HV = g.HV;
            auto seed = [&](int64_t q) { return D.rs[q] > 0 ? 1 : HV; };
            int32_t top = HV, bot = HV, hs[RW], d0[RW];
            if (w == 0 && colv && g.y0 > 0) top = seed(g.off + int64_t(g.y0 - 1) * g.W + x);
            if (w == 3 && colv && g.y0 + RELAX_TH < g.H)
                bot = seed(g.off + int64_t(g.y0 + RELAX_TH) * g.W + x);
            const int hx = lane == 0 ? g.x0 - 1 : g.x0 + 64;
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int y = yw + r;
                const bool use =
                    (lane == 0 && ((mL >> r) & 1u)) || (lane == 63 && ((mR >> r) & 1u));
                hs[r] = INT_MAX;
                if (use && hx >= 0 && hx < g.W && y < g.H)
                    hs[r] = seed(g.off + int64_t(y) * g.W + hx) + 1;
                d0[r] = d[r];
            }
            tile_fixpoint<SEG, 1>(d, mR, mL, mD, mU, hs, top, bot, lane, w, edge);
            // every label is stored (the array holds the last relabel's)
            bool ch_top = false, ch_bot = false, ch_col = false;
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                if (!colv || yw + r >= g.H) continue;
                D.lab[g.off + int64_t(yw + r) * g.W + x] = d[r];
                if (d[r] == d0[r]) continue;
                ch_col = true;
                if (w == 0 && r == 0) ch_top = true;
                if (w == 3 && r == RW - 1) ch_bot = true;
            }
            tile_list_changed(D, g, rt, ch_top, ch_bot, ch_col, lane, w, s_ch, D.dirty[0],
                              D.dlist[0], &D.sc->seed_count);
        }
    }
    if (mode & BD_COUNT) {
        const unsigned long long se = block_sum_u64(n_exact);
        const unsigned long long sa = block_sum_u64(n_act);
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            if (lane == 0) {
                if (se) atomicAdd(&D.inst_exact[g.inst], se);
                if (sa) atomicAdd(&D.inst_active[g.inst], sa);
            }
            // lane k: the sweep tile of rows k*TH .. k*TH + TH - 1 of this tile
            const uint32_t rows = s_rows;
            constexpr uint32_t TMASK = TH >= 32 ? 0xFFFFFFFFu : ((1u << (TH & 31)) - 1u);
            const int k = lane;
            int st = -1;
            bool a = false;
            if (k < RELAX_TH / TH && g.y0 + k * TH < g.H) {
                st = D.inst[g.inst].tile_base + (g.ty * (RELAX_TH / TH) + k) * g.tiles_x + g.tx;
                a = ((rows >> (k * TH)) & TMASK) != 0;
                D.act[0][st] = a ? 1 : 0;
                D.act[1][st] = 0;
                D.act[2][st] = 0;
            }
            list_append(D.alist[0], &D.sc->act_cnt[0], a, st, lane);
        }
    }
}

// Cut closure, first pass: the seeds (label 0 for pixels holding excess,
// |V| elsewhere) relaxed inside each 64 x 32 tile to their fixpoint over the
// live residual arcs into each pixel (the run has stopped), with the halo at
// the neighbouring pixels' seeds; every label is stored and the neighbours
// across a side where a label fell below its seed form the closure's first
// list (every dirty flag and seed_count are 0 beforehand).  The layout and
// the fixpoint are those of a relaxation pass.
template <bool SEG>
__global__ __launch_bounds__(NT) void k_cut_seed(Dev D) {
    static_assert(RELAX_TH == 4 * RW, "four wavefronts per relaxation tile");
    const int t = blockIdx.x;
    const Geo g = tile_geo<RELAX_TH, true>(D, t);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __shared__ int32_t edge[4][2][64];
    __shared__ int s_ch;
    if (threadIdx.x == 0) s_ch = 0;
    const int HV = g.HV;
    const int x = g.x0 + lane;
    const bool colv = x < g.W;
    const int yw = g.y0 + RW * w;
    auto seed = [&](int64_t q) { return D.e[q] > 0 ? 0 : HV; };
    int32_t d[RW], d0[RW];
    uint32_t mR = 0, mL = 0, mD = 0, mU = 0;  // bit r: an arc into the pixel of row r
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int y = yw + r;
        d[r] = HV;
        if (colv && y < g.H) {
            const int64_t p = g.off + int64_t(y) * g.W + x;
            d[r] = seed(p);
            if (x + 1 < g.W) mR |= uint32_t(D.rl[p + 1] > 0) << r;
            if (x > 0) mL |= uint32_t(D.rr[p - 1] > 0) << r;
            if (y + 1 < g.H) mD |= uint32_t(D.ru[p + g.W] > 0) << r;
            if (y > 0) mU |= uint32_t(D.rd[p - g.W] > 0) << r;
        }
        d0[r] = d[r];
    }
    int32_t top = HV, bot = HV, hs[RW];
    if (w == 0 && colv && g.y0 > 0) top = seed(g.off + int64_t(g.y0 - 1) * g.W + x);
    if (w == 3 && colv && g.y0 + RELAX_TH < g.H)
        bot = seed(g.off + int64_t(g.y0 + RELAX_TH) * g.W + x);
    const int hx = lane == 0 ? g.x0 - 1 : g.x0 + 64;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int y = yw + r;
        const bool use = (lane == 0 && ((mL >> r) & 1u)) || (lane == 63 && ((mR >> r) & 1u));
        hs[r] = INT_MAX;
        if (use && hx >= 0 && hx < g.W && y < g.H) hs[r] = seed(g.off + int64_t(y) * g.W + hx);
    }
    tile_fixpoint<SEG, 0>(d, mR, mL, mD, mU, hs, top, bot, lane, w, edge);
    bool ch_top = false, ch_bot = false, ch_col = false;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        if (!colv || yw + r >= g.H) continue;
        D.lab[g.off + int64_t(yw + r) * g.W + x] = d[r];
        if (d[r] == d0[r]) continue;
        ch_col = true;
        if (w == 0 && r == 0) ch_top = true;
        if (w == 3 && r == RW - 1) ch_bot = true;
    }
    tile_list_changed(D, g, t, ch_top, ch_bot, ch_col, lane, w, s_ch, D.dirty[0], D.dlist[0],
                      &D.sc->seed_count);
}

template <int TH>
__global__ __launch_bounds__(NT) void k_cut_write(Dev D, uint8_t *side) {
    const Geo g = tile_geo<TH>(D, blockIdx.x);
    // every row's load first, from a clamped valid pixel, then the stores
    const int c = threadIdx.x & (TW - 1);
    const int x = g.x0 + c;
    const int xc = min(x, g.W - 1);
    int32_t lv[TH / RPP];
#pragma unroll
    for (int k = 0; k < TH / RPP; ++k) {
        const int y = min(g.y0 + (threadIdx.x >> 6) + RPP * k, g.H - 1);
        lv[k] = D.lab[g.off + int64_t(y) * g.W + xc];
    }
#pragma unroll
    for (int k = 0; k < TH / RPP; ++k) {
        const int y = g.y0 + (threadIdx.x >> 6) + RPP * k;
        if (y < g.H && x < g.W) side[g.off + int64_t(y) * g.W + x] = lv[k] < g.HV ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// Tile relaxation to a local fixpoint.
//   BFS (CUT = false): lab(p) = min(lab(p), lab(q) + 1) over arcs p->q with
//     u_f > 0 in the snapshot -- the backward BFS of Algorithm 4.4 from t;
//     its least fixpoint is the BFS level, |V| where t is unreachable (the
//     gap of Section 4.2).  It reads the snapshot masks, never the live
//     residuals, so push sweeps may run meanwhile.
//   CUT (CUT = true):  lab(p) = min(lab(p), lab(q)) over arcs q->p with
//     u_f > 0 -- forward reachability from the excess pixels (the run has
//     stopped; live residuals).
// Labels only decrease and every value read from a neighbouring tile is an
// upper bound of its final value, so concurrent tiles reach the same least
// fixpoint; tiles whose edge labels changed put their neighbours on the
// next pass's list.
//
// A pass runs on 64 x 32 tiles, four wavefronts per tile (one workgroup):
// wavefront w holds rows 8w .. 8w+7 in registers (lane c owns column c) and
// relaxes them to their local fixpoint: each row by two segmented min-plus
// scans across the lanes (a label crosses the 64 columns in one step), then
// a downward and an upward pass along the columns in registers; only rows a
// column pass lowered are scanned again.  The rows where two wavefronts meet
// are exchanged through LDS and the four relax again until a workgroup vote
// finds no lowered boundary.  A label thus crosses 32 rows in one pass, with
// the latency of an 8-row tile per wavefront.
//
// Row scans (SEG = false): lane x of a row takes the minimum over its segment
// (the lanes joined to it by usable arcs) of the label shifted by its column
// distance.  Adding (segments between the lane and the scan's end) x 2^25 to
// every lane makes each other segment's values larger than any label of the
// lane's own, so a plain prefix / suffix minimum gives the segmented one;
// the multiples are fixed for the pass and kept per row.  This needs every
// label at most 2^25 - 64 (instances of at most 2^25 - 66 pixels); a batch
// with a larger instance uses the segmented scans with a lane test per step
// (SEG = true).
//
// Work list: the pass relaxes the tiles of list `cur` (cnt_cur entries;
// workgroup b takes entries b, b + G, b + 2G, ... of a grid of G <=
// RELAX_GRID workgroups, so the tiles spread over the whole chip however they
// cluster on the grid) and appends the neighbours whose halo changed to the
// next list, once each (the flag), counting them in cnt_next.  A pass whose
// list is empty returns at once (a launch of at most RELAX_GRID workgroups),
// so a round can carry more passes than its global relabel needs at little
// cost.  The first pass of a global relabel (every tile from its seeds) runs
// inside the snapshot launch (k_boundary), that of the cut closure inside
// k_cut_seed; the passes here start from the lists those leave.
// ---------------------------------------------------------------------------
template <bool CUT, bool SEG>
__global__ __launch_bounds__(256) void k_relax4(Dev D, int cur, const int32_t *cnt_cur,
                                               int32_t *cnt_next) {
    static_assert(RELAX_TH == 4 * RW, "four wavefronts per relaxation tile");
    const int n = *cnt_cur;
    if (int(blockIdx.x) >= n) return;         // workgroup-uniform
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // statistics: once per pass
        if (!CUT) atomicAdd(&D.counters[6], 1ull);
        atomicAdd(&D.counters[CUT ? 4 : 3], (unsigned long long)n);
    }
    const int nxt = next3(cur);
    __shared__ int32_t edge[4][2][64];        // row 0 and row 7 of each wavefront
    __shared__ int s_ch;
    // the grid holds at most RELAX_GRID workgroups (a pass whose list is
    // short or empty costs a small launch); each takes every gridDim-th entry
    for (int b = blockIdx.x; b < n; b += gridDim.x) {
        const int t = D.dlist[cur][b];
        // the LDS of the last tile: every read of edge[] ended before the
        // workgroup vote that closed its loop, and s_ch was read by wavefront 0
        // (this thread's own) after the barrier that followed every update
        if (threadIdx.x == 0) {
            s_ch = 0;
            D.dirty[cur][t] = 0;
        }
        __syncthreads();
        const Geo g = tile_geo<RELAX_TH, true>(D, t);
        constexpr int INC = CUT ? 0 : 1;
        const int HV = g.HV;
        const int x = g.x0 + lane;
        const bool colv = x < g.W;
        const int yw = g.y0 + RW * w;             // first row of this wavefront
        int32_t d[RW], d0[RW];
        uint32_t mR = 0, mL = 0, mD = 0, mU = 0;  // bit r: arc usable in row r
        if (!CUT) {
            // this wavefront's eight rows of the column's snapshot masks
            const uint32_t *tm = D.amask + size_t(t) * NMASK * TW + lane;
            const int sh = RW * w;
            mR = (tm[MK_R * TW] >> sh) & 0xFFu;
            mL = (tm[MK_L * TW] >> sh) & 0xFFu;
            mD = (tm[MK_D * TW] >> sh) & 0xFFu;
            mU = (tm[MK_U * TW] >> sh) & 0xFFu;
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int y = yw + r;
            d[r] = HV;
            if (colv && y < g.H) {
                const int64_t p = g.off + int64_t(y) * g.W + x;
                d[r] = D.lab[p];
                if (CUT) {
                    // arcs into p: from the right neighbour (its left arc), etc.
                    if (x + 1 < g.W) mR |= uint32_t(D.rl[p + 1] > 0) << r;
                    if (x > 0) mL |= uint32_t(D.rr[p - 1] > 0) << r;
                    if (y + 1 < g.H) mD |= uint32_t(D.ru[p + g.W] > 0) << r;
                    if (y > 0) mU |= uint32_t(D.rd[p - g.W] > 0) << r;
                }
            }
            d0[r] = d[r];
        }
        // halo: the tile's row above / below (wavefronts 0 / 3), columns left and
        // right (lanes 0 / 63); the rows between wavefronts come from LDS.  hs[r]
        // is what the side halo offers lane 0 / 63 of row r (its label + INC
        // where the arc is usable, else INT_MAX), fixed for the pass.
        int32_t top = HV, bot = HV, hs[RW];
        if (w == 0 && colv && g.y0 > 0) top = D.lab[g.off + int64_t(g.y0 - 1) * g.W + x];
        if (w == 3 && colv && g.y0 + RELAX_TH < g.H)
            bot = D.lab[g.off + int64_t(g.y0 + RELAX_TH) * g.W + x];
        const int hx = lane == 0 ? g.x0 - 1 : g.x0 + 64;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int y = yw + r;
            const bool use = (lane == 0 && ((mL >> r) & 1u)) || (lane == 63 && ((mR >> r) & 1u));
            hs[r] = INT_MAX;
            if (use && hx >= 0 && hx < g.W && y < g.H)
                hs[r] = D.lab[g.off + int64_t(y) * g.W + hx] + INC;
        }
        tile_fixpoint<SEG, INC>(d, mR, mL, mD, mU, hs, top, bot, lane, w, edge);
        bool ch_top = false, ch_bot = false, ch_col = false;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            if (d[r] == d0[r]) continue;
            D.lab[g.off + int64_t(yw + r) * g.W + x] = d[r];
            ch_col = true;
            if (w == 0 && r == 0) ch_top = true;
            if (w == 3 && r == RW - 1) ch_bot = true;
        }
        tile_list_changed(D, g, t, ch_top, ch_bot, ch_col, lane, w, s_ch, D.dirty[nxt],
                          D.dlist[nxt], cnt_next);
    }
}

// ---------------------------------------------------------------------------
// End of a round: retire the instances whose exact count is 0 and publish the
// totals.  The count is exact only when the global relabel reached its
// fixpoint: with `pass_count` given, the last of its P passes must have
// marked no tile; otherwise labels can still lie above the BFS level,
// nothing is retired, and the round is counted as open (the host then gives
// later rounds more passes).  For a converged relabel the number of passes
// it needed (up to the first that marked no tile) is kept in max_need.
// ---------------------------------------------------------------------------
__global__ void k_finish(Dev D, const int32_t *pass_count, int P) {
    const bool exact = pass_count == nullptr || pass_count[P - 1] == 0;
    unsigned long long tot = 0;
    unsigned long long left = 0;
    for (int i = threadIdx.x; i < D.ninst; i += blockDim.x) {
        int dn = D.done[i];
        if (!dn && exact && D.inst_exact[i] == 0) {
            D.done[i] = 1;
            dn = 1;
        }
        if (!dn) {
            tot += D.inst_active[i];
            ++left;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        tot += __shfl_xor(tot, o, 64);
        left += __shfl_xor(left, o, 64);
    }
    __shared__ unsigned long long red[2][4];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = tot;
        red[1][threadIdx.x >> 6] = left;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0, l = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            s += red[0][i];
            l += red[1][i];
        }
        Scalars *sc = D.sc;
        if (!sc->all_done) sc->rounds += 1;
        sc->total_active = s;
        sc->all_done = l == 0 ? 1 : 0;
        if (pass_count) {
            if (!exact) {
                sc->open_bfs += 1;
            } else {
                int need = P;
                for (int i = 0; i < P; ++i)
                    if (pass_count[i] == 0) {
                        need = i + 1;
                        break;
                    }
                sc->max_need = max(sc->max_need, need);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Push sweep: `L` lock-free push/relabel iterations of Algorithm 4.5 per
// active 64 x TH tile, one wavefront per tile, no block barrier.  Lane c owns
// column c of the tile in registers (e, h, the four neighbour residuals and
// the sink residual of each of its TH pixels).  An iteration walks the rows
// top to bottom (rows with no active pixel are skipped as a whole): every
// active pixel reads its horizontal neighbours' current heights by DPP
// (lanes 0 and 63 use the halo heights), picks the lowest residual neighbour
// and pushes or relabels.  The choice is branch-free: each candidate is the
// key (height << 3 | direction) and the minimum key gives the lowest height
// and, on ties, the first direction in the scan order t, right, left, down,
// up.  A push inside the column updates the registers directly, a push to
// the lane on the left or right is handed over by DPP right after the row.
// Flow pushed across the tile edge only lowers the pusher's own residual
// during the visit; the total (that residual's drop) is applied to the
// neighbouring tile with device-scope atomics when the visit ends, which for
// the other tile is a push fulfilled a little later, as Hong's argument
// admits.  The tile's own edge excesses are merged back by atomic deltas, so
// pushes that other tiles make into it meanwhile are kept.  Every value read
// of another pixel is a lower bound of the true one (excess and residuals
// only shrink by their owner's pushes, heights only grow between global
// relabels), the staleness Hong's argument admits.
// ---------------------------------------------------------------------------
// Work list: the launch reads list `cur` (wavefront i takes entry i, so the
// active tiles spread one per SIMD over the chip however they cluster on the
// grid), appends the tiles to visit next to the next list (once each: the
// flag) and clears the count of the third, which the launch before read.
template <int TH>
__global__ __launch_bounds__(256) void k_sweep(Dev D, int cur, int L) {
    const int lane = threadIdx.x & 63;
    const int nxt = next3(cur);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        D.sc->act_cnt[prev3(cur)] = 0;
        // statistics: every listed tile is visited once by this launch
        atomicAdd(&D.counters[2], (unsigned long long)D.sc->act_cnt[cur]);
    }
    const int i = int(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (i >= D.sc->act_cnt[cur]) return;  // wave-uniform
    const int t = D.alist[cur][i];
    if (lane == 0) D.act[cur][t] = 0;
    const Geo g = tile_geo<TH>(D, t);
    const int HV = g.HV;
    const int x = g.x0 + lane;
    const bool colv = x < g.W;
    const uint32_t o0 = 4u * uint32_t(g.off + int64_t(g.y0) * g.W + x);  // row 0
    const uint32_t ow = 4u * uint32_t(g.W);                                // one row
    // Pixels outside the grid hold e = 0, h = |V| and no residual arc, so
    // they never act and are never chosen.
    int32_t e[TH], h[TH], rs[TH], rr[TH], rl[TH], rd[TH], ru[TH];
    uint32_t valid = 0;
#pragma unroll
    for (int r = 0; r < TH; ++r) {
        e[r] = 0; h[r] = HV; rs[r] = 0; rr[r] = 0; rl[r] = 0; rd[r] = 0; ru[r] = 0;
        if (colv && g.y0 + r < g.H) {
            valid |= 1u << r;
            const uint32_t o = o0 + r * ow;
            e[r] = at(D.e, o);
            h[r] = at(D.h, o);
            rs[r] = at(D.rs, o);
            rr[r] = at(D.rr, o);
            rl[r] = at(D.rl, o);
            rd[r] = at(D.rd, o);
            ru[r] = at(D.ru, o);
        }
    }
    // Values at load time: the excess (for the delta merge of edge pixels)
    // and the residuals of the arcs that leave the tile (lane 63 right, lane
    // 0 left, row 0 up, row TH-1 down), whose drop is the flow pushed out.
    int32_t e0[TH], side0[TH];
#pragma unroll
    for (int r = 0; r < TH; ++r) {
        e0[r] = e[r];
        side0[r] = lane == 63 ? rr[r] : rl[r];
    }
    const int32_t top0 = ru[0], bot0 = rd[TH - 1];
    // halo heights (read once; heights only grow, so these are lower bounds)
    int32_t top = HV, bot = HV, hside[TH];
    if (colv && g.y0 > 0) top = at(D.h, o0 - ow);
    if (colv && g.y0 + TH < g.H) bot = at(D.h, o0 + TH * ow);
    const int hx = lane == 0 ? g.x0 - 1 : g.x0 + 64;
#pragma unroll
    for (int r = 0; r < TH; ++r) {
        hside[r] = HV;
        if ((lane == 0 || lane == 63) && hx >= 0 && hx < g.W && g.y0 + r < g.H)
            hside[r] = at(D.h, o0 + r * ow + 4u * uint32_t(hx - x));
    }
    constexpr uint32_t NONE = 0xFFFFFFFFu;
    uint32_t acted = 0;                        // bit r: the pixel pushed or relabelled
    // this lane's pushes and relabels, summed over the wavefront once at
    // the end (a ballot count per row would cost scalar 64-bit adds there)
    uint32_t lane_push = 0, lane_relab = 0;
    for (int it = 0; it < L; ++it) {
        uint32_t act_it = 0;                   // bit r: the pixel acted in this iteration
#pragma unroll
        for (int r = 0; r < TH; ++r) {
            const bool active = e[r] > 0 && h[r] < HV;
            if (!__any(active)) continue;      // wave-uniform skip
            const int32_t hl = from_left(h[r], hside[r]);
            const int32_t hr = from_right(h[r], hside[r]);
            const int32_t hd = r + 1 < TH ? h[r + 1] : bot;
            const int32_t hu = r > 0 ? h[r - 1] : top;
            const uint32_t kS = rs[r] > 0 ? 0u : NONE;
            const uint32_t kR = rr[r] > 0 ? (uint32_t(hr) << 3) | 1u : NONE;
            const uint32_t kL = rl[r] > 0 ? (uint32_t(hl) << 3) | 2u : NONE;
            const uint32_t kD = rd[r] > 0 ? (uint32_t(hd) << 3) | 3u : NONE;
            const uint32_t kU = ru[r] > 0 ? (uint32_t(hu) << 3) | 4u : NONE;
            const uint32_t key = min(min(min(kS, kR), kL), min(kD, kU));
            const uint32_t best = key >> 3;    // NONE >> 3 exceeds every height
            const uint32_t dir = key & 7u;
            const bool push = active && best < uint32_t(h[r]);
            const bool relab = active && !push;
            // PUSH delta = min(e', u_f(x, y~)) towards y~, u_f the chosen
            // arc's residual (selected by constant-indexed registers)
            int32_t cap = rs[r];
            cap = dir == 1 ? rr[r] : cap;
            cap = dir == 2 ? rl[r] : cap;
            cap = dir == 3 ? rd[r] : cap;
            cap = dir == 4 ? ru[r] : cap;
            const int32_t d = push ? min(e[r], cap) : 0;
            const int32_t dS = dir == 0 ? d : 0, dR = dir == 1 ? d : 0;
            const int32_t dL = dir == 2 ? d : 0, dD = dir == 3 ? d : 0;
            const int32_t dU = dir == 4 ? d : 0;
            e[r] -= d;
            rs[r] -= dS;
            rr[r] -= dR;
            rl[r] -= dL;
            rd[r] -= dD;
            ru[r] -= dU;
            if (r + 1 < TH) {
                ru[r + 1] += dD;
                e[r + 1] += dD;
            }
            if (r > 0) {
                rd[r - 1] += dU;
                e[r - 1] += dU;
            }
            // RELABEL h(x) = h~ + 1 (owner only); no residual arc or a height
            // past |V| freezes the pixel (gap height)
            if (relab) h[r] = int32_t(min(best + 1u, uint32_t(HV)));
            // hand the horizontal pushes of this row to the neighbour lanes
            // (lane 63's push right and lane 0's push left leave the wave)
            const int32_t inL = from_left(dR, 0);
            const int32_t inR = from_right(dL, 0);
            rl[r] += inL;
            rr[r] += inR;
            e[r] += inL + inR;
            act_it |= active ? 1u << r : 0u;
            lane_push += push;
            lane_relab += relab;
        }
        acted |= act_it;
        if (!__any(act_it != 0)) break;        // no pixel of the tile acted
    }
    for (int o = 32; o > 0; o >>= 1) {
        lane_push += __shfl_xor(lane_push, o, 64);
        lane_relab += __shfl_xor(lane_relab, o, 64);
    }
    const unsigned long long pushes = lane_push, relabels = lane_relab;
    // Write back the pixels whose state can have changed (they or an in-tile
    // neighbour acted): plain stores where only this tile writes, an atomic
    // delta for the excess of pixels that other tiles can push into, and the
    // flow pushed out of the tile applied to both ends of the crossing arcs.
    const uint32_t touched = acted | (acted << 1) | (acted >> 1) |
                             uint32_t(from_left(int32_t(acted), 0)) |
                             uint32_t(from_right(int32_t(acted), 0));
    bool active_end = false, touch_l = false, touch_r = false;
    bool touch_u = false, touch_d = false;
    uint32_t n_atomic = 0;                     // device-scope atomics of this lane
#pragma unroll
    for (int r = 0; r < TH; ++r) {
        if (!((valid >> r) & 1u)) continue;
        active_end |= e[r] > 0 && h[r] < HV;
        if (!((touched >> r) & 1u)) continue;
        const int y = g.y0 + r;
        const uint32_t o = o0 + r * ow;
        const bool edge = (lane == 63 && x + 1 < g.W) || (lane == 0 && x > 0) ||
                          (r == TH - 1 && y + 1 < g.H) || (r == 0 && y > 0);
        if (edge) {
            if (e[r] != e0[r]) {
                atomicAdd(&at(D.e, o), e[r] - e0[r]);
                ++n_atomic;
            }
        } else {
            at(D.e, o) = e[r];
        }
        at(D.h, o) = h[r];
        at(D.rs, o) = rs[r];
        if (lane < 63) at(D.rr, o) = rr[r];
        if (lane > 0) at(D.rl, o) = rl[r];
        if (r < TH - 1) at(D.rd, o) = rd[r];
        if (r > 0) at(D.ru, o) = ru[r];
        if (lane == 63) {
            const int32_t out = side0[r] - rr[r];
            if (out) {
                atomicSub(&at(D.rr, o), out);
                atomicAdd(&at(D.rl, o + 4), out);
                atomicAdd(&at(D.e, o + 4), out);
                touch_r = true;
                n_atomic += 3;
            }
        }
        if (lane == 0) {
            const int32_t out = side0[r] - rl[r];
            if (out) {
                atomicSub(&at(D.rl, o), out);
                atomicAdd(&at(D.rr, o - 4), out);
                atomicAdd(&at(D.e, o - 4), out);
                touch_l = true;
                n_atomic += 3;
            }
        }
        if (r == 0) {
            const int32_t out = top0 - ru[0];
            if (out) {
                atomicSub(&at(D.ru, o), out);
                atomicAdd(&at(D.rd, o - ow), out);
                atomicAdd(&at(D.e, o - ow), out);
                touch_u = true;
                n_atomic += 3;
            }
        }
        if (r == TH - 1) {
            const int32_t out = bot0 - rd[TH - 1];
            if (out) {
                atomicSub(&at(D.rd, o), out);
                atomicAdd(&at(D.ru, o + ow), out);
                atomicAdd(&at(D.e, o + ow), out);
                touch_d = true;
                n_atomic += 3;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) n_atomic += __shfl_xor(n_atomic, o, 64);
    const bool a_end = __any(active_end);
    const bool a_l = __any(touch_l), a_r = __any(touch_r);
    const bool a_u = __any(touch_u), a_d = __any(touch_d);
    // lanes 0..4 flag the tile itself and its left, right, upper and lower
    // neighbours for the next sweep
    int nb = -1;
    if (lane == 0 && a_end) nb = t;
    if (lane == 1 && a_l) nb = t - 1;
    if (lane == 2 && a_r) nb = t + 1;
    if (lane == 3 && a_u) nb = t - g.tiles_x;
    if (lane == 4 && a_d) nb = t + g.tiles_x;
    const bool fresh = nb >= 0 && atomicExch(&D.act[nxt][nb], 1) == 0;
    list_append(D.alist[nxt], &D.sc->act_cnt[nxt], fresh, nb, lane);
    if (lane == 0) {
        if (pushes) atomicAdd(&D.counters[0], pushes);
        if (relabels) atomicAdd(&D.counters[1], relabels);
        if (n_atomic) atomicAdd(&D.counters[5], (unsigned long long)n_atomic);
    }
}

// Flow value e(t) = sum_p (u(p,t) - u_f(p,t)) per instance (int64).
template <int TH>
__global__ __launch_bounds__(NT) void k_flow_value(Dev D, int64_t *flow) {
    const Geo g = tile_geo<TH>(D, blockIdx.x);
    // every row's loads first, from a clamped valid pixel; rows and columns
    // past the grid add nothing
    const int c = threadIdx.x & (TW - 1);
    const int x = g.x0 + c;
    const int xc = min(x, g.W - 1);
    int32_t cv[TH / RPP], rv[TH / RPP];
#pragma unroll
    for (int k = 0; k < TH / RPP; ++k) {
        const int y = min(g.y0 + (threadIdx.x >> 6) + RPP * k, g.H - 1);
        const int64_t p = g.off + int64_t(y) * g.W + xc;
        cv[k] = D.cap_snk[p];
        rv[k] = D.rs[p];
    }
    unsigned long long s = 0;
#pragma unroll
    for (int k = 0; k < TH / RPP; ++k) {
        const int y = g.y0 + (threadIdx.x >> 6) + RPP * k;
        if (y < g.H && x < g.W) s += (unsigned long long)(int64_t(cv[k]) - rv[k]);
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
    int32_t *lab;
    uint32_t *amask;
    int32_t *tile_inst, *tile_inst_r, *done;
    int32_t *act[3], *alist[3];  // sweep work lists (flags, entries)
    int32_t *dirty_all;          // the three relaxation flag arrays, back to back
    int32_t *dlist[3];
    Inst *inst;
    unsigned long long *inst_cnt;  // active [B], then exact [B]
    unsigned long long *counters;
    Scalars *sc;
};

static Carver carve(Carver cv, int64_t N, int64_t T, int64_t TR, int B, Layout *L) {
    for (int i = 0; i < 7; ++i) L->st[i] = cv.take<int32_t>(size_t(N));
    L->lab = cv.take<int32_t>(size_t(N));
    L->amask = cv.take<uint32_t>(size_t(TR) * NMASK * TW);
    L->tile_inst = cv.take<int32_t>(size_t(T));
    L->tile_inst_r = cv.take<int32_t>(size_t(TR));
    for (int i = 0; i < 3; ++i) {
        L->act[i] = cv.take<int32_t>(size_t(T));
        L->alist[i] = cv.take<int32_t>(size_t(T));
        L->dlist[i] = cv.take<int32_t>(size_t(TR));
    }
    L->dirty_all = cv.take<int32_t>(size_t(3) * TR);
    L->inst = cv.take<Inst>(size_t(B));
    L->inst_cnt = cv.take<unsigned long long>(size_t(2) * B);
    L->done = cv.take<int32_t>(size_t(B));
    L->counters = cv.take<unsigned long long>(8);
    L->sc = cv.take<Scalars>(1);
    return cv;
}

static int64_t tiles_for(int32_t H, int32_t W, int TH) {
    return int64_t(ceil_div(W, TW)) * ceil_div(H, TH);
}

static size_t workspace_bytes(int B, const int32_t *H, const int32_t *W) {
    int64_t N = 0, T = 0, TR = 0;
    for (int b = 0; b < B; ++b) {
        N += int64_t(H[b]) * W[b];
        T += tiles_for(H[b], W[b], 4);  // smallest tile height: most tiles
        TR += tiles_for(H[b], W[b], RELAX_TH);
    }
    Layout L;
    Carver cv = carve(Carver(), N, T, TR, B, &L);
    return cv.used();
}

template <int TH>
struct Kern {
    static void init(hipStream_t s, const Dev &D) {
        hipLaunchKernelGGL(k_init<TH>, dim3(D.ntiles), dim3(NT), 0, s, D);
    }
    static void boundary(hipStream_t s, const Dev &D, unsigned mode) {
        constexpr unsigned AC = BD_ADOPT | BD_COUNT, ACS = BD_ADOPT | BD_COUNT | BD_SNAPSHOT;
        const dim3 gr(D.ntiles_r), bl(NT);
        if (mode == AC)
            hipLaunchKernelGGL((k_boundary<TH, AC, false>), gr, bl, 0, s, D);
        else if (mode == BD_SNAPSHOT && D.seg_scan)
            hipLaunchKernelGGL((k_boundary<TH, BD_SNAPSHOT, true>), gr, bl, 0, s, D);
        else if (mode == BD_SNAPSHOT)
            hipLaunchKernelGGL((k_boundary<TH, BD_SNAPSHOT, false>), gr, bl, 0, s, D);
        else if (D.seg_scan)
            hipLaunchKernelGGL((k_boundary<TH, ACS, true>), gr, bl, 0, s, D);
        else
            hipLaunchKernelGGL((k_boundary<TH, ACS, false>), gr, bl, 0, s, D);
    }
    // the relaxation kernels run on the RELAX_TH tiling, one 4-wavefront
    // workgroup per listed tile
    static void cut_seed(hipStream_t s, const Dev &D) {
        if (D.seg_scan)
            hipLaunchKernelGGL(k_cut_seed<true>, dim3(D.ntiles_r), dim3(NT), 0, s, D);
        else
            hipLaunchKernelGGL(k_cut_seed<false>, dim3(D.ntiles_r), dim3(NT), 0, s, D);
    }
    static void relax(bool cut, hipStream_t s, const Dev &D, int cur, const int32_t *cnt_cur,
                      int32_t *cnt_next) {
        const dim3 gw(std::min(D.ntiles_r, RELAX_GRID));
        if (D.seg_scan) {
            if (cut) hipLaunchKernelGGL((k_relax4<true, true>), gw, dim3(NT), 0, s, D, cur, cnt_cur, cnt_next);
            else hipLaunchKernelGGL((k_relax4<false, true>), gw, dim3(NT), 0, s, D, cur, cnt_cur, cnt_next);
        } else {
            if (cut) hipLaunchKernelGGL((k_relax4<true, false>), gw, dim3(NT), 0, s, D, cur, cnt_cur, cnt_next);
            else hipLaunchKernelGGL((k_relax4<false, false>), gw, dim3(NT), 0, s, D, cur, cnt_cur, cnt_next);
        }
    }
    static void sweep(hipStream_t s, const Dev &D, int cur, int L) {
        hipLaunchKernelGGL(k_sweep<TH>, dim3((D.ntiles + 3) / 4), dim3(NT), 0, s, D, cur, L);
    }
    static void flow(hipStream_t s, const Dev &D, int64_t *f) {
        hipLaunchKernelGGL(k_flow_value<TH>, dim3(D.ntiles), dim3(NT), 0, s, D, f);
    }
    static void cut_write(hipStream_t s, const Dev &D, uint8_t *side) {
        hipLaunchKernelGGL(k_cut_write<TH>, dim3(D.ntiles), dim3(NT), 0, s, D, side);
    }
};

struct Params {
    int TH, L, K, max_rounds;
    int rounds_per_check;  // rounds enqueued between two host reads
    bool timing, no_graph;
    bool arg;      // asynchronous global relabel (BFS on a second stream)
    bool noalloc;  // allocation-free call: no graphs, events, streams or pinned memory
};

// Runs relaxation passes from the seeded list 0 until a pass lists no tile
// (host checks once per batch of passes; a pass after one that listed
// nothing returns at once).  A batch starts from the count the last one
// ended with, carried in seed_count.
__global__ void k_carry(int32_t *dst, const int32_t *src) { *dst = *src; }

template <int TH>
static lpr_status relax_to_fixpoint(bool cut, hipStream_t s, const Dev &D,
                                    Layout &Lw, EventTimer &tm, int64_t *passes) {
    int batch = 8;
    int64_t g = 0;  // passes so far: pass g reads list g mod 3
    const int64_t guard = 16 * int64_t(D.ntiles_r) + 1024;
    int32_t *pc = Lw.sc->pass_count;
    for (;;) {
        if (g > guard) {
            set_error("relaxation did not reach its fixpoint within %lld passes",
                      (long long)guard);
            return LPR_EBUDGET;
        }
        LPR_TRY(fill_i32(pc, 0, batch, s));
        const int ev = tm.begin();
        for (int i = 0; i < batch; ++i, ++g)
            Kern<TH>::relax(cut, s, D, int(g % 3), i ? pc + i - 1 : &Lw.sc->seed_count,
                            pc + i);
        tm.end(ev);
        LPR_TRY_HIP(hipGetLastError());
        *passes += batch;
        int32_t last = 0;
        LPR_TRY_HIP(hipMemcpyAsync(&last, pc + batch - 1, sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s));
        LPR_TRY_HIP(hipStreamSynchronize(s));
        // at the fixpoint every flag is clear again: each listed tile cleared
        // its own and the last pass listed none
        if (last == 0) return LPR_OK;
        hipLaunchKernelGGL(k_carry, dim3(1), dim3(1), 0, s, &Lw.sc->seed_count,
                           pc + batch - 1);
        batch = std::min(batch * 2, MAX_PASS_SLOTS);
    }
}

// Ahead of a boundary kernel: a count clears the counts of the sweep lists
// it rebuilds; a snapshot clears every relaxation flag and the seed count.
template <int TH>
static lpr_status enqueue_boundary(hipStream_t s, const Dev &D, Layout &Lw, unsigned mode) {
    if (mode & BD_SNAPSHOT) {
        LPR_TRY(fill_i32(Lw.dirty_all, 0, 3 * int64_t(D.ntiles_r), s));
        LPR_TRY(fill_i32(&Lw.sc->seed_count, 0, (mode & BD_COUNT) ? 4 : 1, s));
    } else if (mode & BD_COUNT) {
        LPR_TRY(fill_i32(Lw.sc->act_cnt, 0, 3, s));
    }
    Kern<TH>::boundary(s, D, mode);
    LPR_TRY_HIP(hipGetLastError());
    return LPR_OK;
}

// Adopt the labels of the global relabel just finished, count, retire.
template <int TH>
static lpr_status enqueue_adopt(hipStream_t s, const Dev &D, Layout &Lw, int B,
                                unsigned extra, const int32_t *pass_count, int P) {
    LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(Lw.inst_cnt), 0, 2 * int64_t(B), s));
    LPR_TRY(enqueue_boundary<TH>(s, D, Lw, BD_ADOPT | BD_COUNT | extra));
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, D, pass_count, P);
    LPR_TRY_HIP(hipGetLastError());
    return LPR_OK;
}

template <int TH>
static lpr_status enqueue_sweeps(hipStream_t s, const Dev &D, Layout &Lw, int K, int L,
                                 EventTimer *tm) {
    const int ev = tm ? tm->begin() : -1;
    for (int k = 0; k < K; ++k) Kern<TH>::sweep(s, D, k % 3, L);
    if (tm) tm->end(ev);
    LPR_TRY_HIP(hipGetLastError());
    return LPR_OK;
}

// P relaxation passes of the global relabel seeded at the last snapshot
// (its list is list 0).
template <int TH>
static lpr_status enqueue_passes(hipStream_t s, const Dev &D, Layout &Lw, int P,
                                 EventTimer *tm) {
    int32_t *pc = Lw.sc->pass_count;
    const int ev = tm ? tm->begin() : -1;
    for (int i = 0; i < P; ++i)
        Kern<TH>::relax(false, s, D, i % 3, i ? pc + i - 1 : &Lw.sc->seed_count, pc + i);
    if (tm) tm->end(ev);
    LPR_TRY_HIP(hipGetLastError());
    return LPR_OK;
}

// One round of the hybrid scheme (Algorithm 4.8 with the heuristic on the
// device): K push sweeps, the snapshot and seed, P relaxation passes, adopt,
// count and retire.
template <int TH>
static lpr_status enqueue_seq_round(hipStream_t s, const Dev &D, Layout &Lw, int B, int K,
                                    int L, int P, EventTimer *t_sweep, EventTimer *t_bfs) {
    LPR_TRY(enqueue_sweeps<TH>(s, D, Lw, K, L, t_sweep));
    LPR_TRY(enqueue_boundary<TH>(s, D, Lw, BD_SNAPSHOT));
    LPR_TRY(fill_i32(Lw.sc->pass_count, 0, P, s));
    LPR_TRY(enqueue_passes<TH>(s, D, Lw, P, t_bfs));
    return enqueue_adopt<TH>(s, D, Lw, B, 0, Lw.sc->pass_count, P);
}

// End of an asynchronous round (after the join): adopt the labels of the
// global relabel that ran beside the sweeps (the BFS of the previous
// snapshot), count that snapshot exactly and retire, take the next snapshot
// and seed, clear the pass counters of the next relabel.
template <int TH>
static lpr_status enqueue_arg_post(hipStream_t s, const Dev &D, Layout &Lw, int B, int P) {
    LPR_TRY(enqueue_adopt<TH>(s, D, Lw, B, BD_SNAPSHOT, Lw.sc->pass_count, P));
    return fill_i32(Lw.sc->pass_count, 0, P, s);
}

// ---------------------------------------------------------------------------
// Graphs: the kernels of a round (or of one stream's share of it) captured
// once per (buffers, shape, schedule, kind) and replayed with one launch.
// ---------------------------------------------------------------------------
// A captured sequence bakes in every kernel argument (the Dev struct with its
// tile counts, the carved workspace pointers, which follow from the
// workspace base, N, B and both tile counts) and every grid size (T sweep
// tiles, TR relaxation tiles).  The key holds all of them, so two batches
// with the same pixel count but other shapes (e.g. 32 x 64 and 16 x 128:
// the same N and T but TR 1 against 2) never share a graph.  The per-tile
// and per-instance tables are read from the workspace at run time and are
// rewritten by every solve, so their contents need no key.
enum GraphKind { GK_SEQ_ROUND = 0, GK_SWEEPS = 1, GK_PASSES = 2, GK_ARG_POST = 3 };

struct GraphKey {
    int device;
    const void *ws;
    const void *caps[6];
    int64_t N;
    int B, T, TR, TH, K, L, P, kind, seg;
    bool operator==(const GraphKey &o) const {
        return device == o.device && ws == o.ws && N == o.N && B == o.B &&
               T == o.T && TR == o.TR && TH == o.TH && K == o.K && L == o.L &&
               P == o.P && kind == o.kind && seg == o.seg &&
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
constexpr size_t MAX_GRAPHS = 16;

// Library streams per device (default priority, non-blocking): the capture
// stream and the stream the asynchronous global relabel runs on.
static lpr_status library_stream(int device, int which, hipStream_t *out) {
    static std::mutex mu;
    static std::vector<std::pair<int, hipStream_t>> streams;
    std::lock_guard<std::mutex> lk(mu);
    const int id = device * 2 + which;
    for (auto &p : streams)
        if (p.first == id) {
            *out = p.second;
            return LPR_OK;
        }
    hipStream_t st;
    LPR_TRY_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    streams.emplace_back(id, st);
    *out = st;
    return LPR_OK;
}

// Finds or captures the graph of `key` (its kernels enqueued by `fill`) and
// launches it on `s` (under the cache lock, so an eviction cannot destroy it
// in between).
template <class F>
static lpr_status launch_graph(const GraphKey &key, hipStream_t s, F &&fill) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto &e : g_graphs)
        if (e.key == key) {
            e.stamp = ++g_graph_clock;
            LPR_TRY_HIP(hipGraphLaunch(e.exec, s));
            return LPR_OK;
        }
    hipStream_t cs;
    LPR_TRY(library_stream(key.device, 0, &cs));
    hipGraph_t g;
    LPR_TRY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const lpr_status st = fill(cs);
    const hipError_t ce = hipStreamEndCapture(cs, &g);
    if (st != LPR_OK) {
        if (ce == hipSuccess) (void)hipGraphDestroy(g);
        return st;
    }
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

// Fork/join events of the asynchronous rounds, per thread and device (two
// per round of a check interval), created once.
constexpr int MAX_ROUNDS_PER_CHECK = 16;

static lpr_status round_events(int device, hipEvent_t **out) {
    struct Pool {
        int device;
        hipEvent_t ev[2 * MAX_ROUNDS_PER_CHECK];
    };
    static thread_local std::vector<Pool> pools;
    for (auto &p : pools)
        if (p.device == device) {
            *out = p.ev;
            return LPR_OK;
        }
    Pool p;
    p.device = device;
    for (int i = 0; i < 2 * MAX_ROUNDS_PER_CHECK; ++i)
        LPR_TRY_HIP(hipEventCreateWithFlags(&p.ev[i], hipEventDisableTiming));
    pools.push_back(p);
    *out = pools.back().ev;
    return LPR_OK;
}

// Pinned host copy of the scalars, one per calling thread.
static lpr_status host_scalars(Scalars **out) {
    static thread_local Scalars *h = nullptr;
    if (!h) LPR_TRY_HIP(hipHostMalloc(reinterpret_cast<void **>(&h), sizeof(Scalars)));
    *out = h;
    return LPR_OK;
}

// The allocation-free path reads into ordinary (pageable) host memory.
static lpr_status read_scalars(hipStream_t s, Layout &Lw, Scalars **host, bool noalloc) {
    static thread_local Scalars pageable;
    if (noalloc)
        *host = &pageable;
    else
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
                        const std::vector<int32_t> &tile_inst,
                        const std::vector<int32_t> &tile_inst_r, Dev D,
                        Layout &Lw, const GraphKey &base_key, int64_t *flow_values,
                        uint8_t *side, lpr_grid_stats *stats, hipStream_t s) {
    const int T = int(tile_inst.size());
    // the asynchronous global relabel runs its passes on a library stream
    hipStream_t sb = s;
    hipEvent_t *ev = nullptr;
    if (P.arg) {
        LPR_TRY(library_stream(base_key.device, 1, &sb));
        LPR_TRY(round_events(base_key.device, &ev));
    }
    // whatever path leaves this function, nothing the call enqueued on the
    // library stream may still run over the caller's buffers afterwards
    struct SyncOnExit {
        hipStream_t st;
        bool on;
        ~SyncOnExit() {
            if (on) (void)hipStreamSynchronize(st);
        }
    } sync_sb{sb, P.arg};
    EventTimer t_sweep(s), t_bfs(s), t_bfs_b(sb);
    if (P.timing) {
        t_sweep.enable();
        t_bfs.enable();
        t_bfs_b.enable();
    }
    double sweep_ms = 0, bfs_ms = 0;
    // launches enqueued (graph replays included): relaxation passes of the
    // global relabel, push sweeps, cut-closure passes
    int64_t bfs_passes = 0, sweep_launches = 0, cut_passes = 0, rounds_enq = 0;

    LPR_TRY_HIP(hipMemcpyAsync(Lw.inst, insts.data(), sizeof(Inst) * B,
                               hipMemcpyHostToDevice, s));
    LPR_TRY_HIP(hipMemcpyAsync(Lw.tile_inst, tile_inst.data(),
                               sizeof(int32_t) * T, hipMemcpyHostToDevice, s));
    LPR_TRY_HIP(hipMemcpyAsync(Lw.tile_inst_r, tile_inst_r.data(),
                               sizeof(int32_t) * tile_inst_r.size(),
                               hipMemcpyHostToDevice, s));
    LPR_TRY(fill_i32(Lw.done, 0, B, s));
    LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(Lw.counters), 0, 8, s));
    LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(Lw.sc), 0,
                     int64_t(sizeof(Scalars) / sizeof(int32_t)), s));
    Kern<TH>::init(s, D);
    LPR_TRY_HIP(hipGetLastError());

    // An exact global relabel on the current state, to its fixpoint under
    // host control, then adopt, count and retire.
    auto exact_relabel = [&]() -> lpr_status {
        LPR_TRY(enqueue_boundary<TH>(s, D, Lw, BD_SNAPSHOT));
        LPR_TRY(relax_to_fixpoint<TH>(false, s, D, Lw, t_bfs, &bfs_passes));
        LPR_TRY(enqueue_adopt<TH>(s, D, Lw, B, 0, nullptr, 0));
        if (P.arg) {
            // the snapshot the first asynchronous relabel works on
            LPR_TRY(enqueue_boundary<TH>(s, D, Lw, BD_SNAPSHOT));
            LPR_TRY(fill_i32(Lw.sc->pass_count, 0, MAX_PASS_SLOTS, s));
        }
        LPR_TRY_HIP(hipGetLastError());
        return LPR_OK;
    };
    // First global relabel: its pass count sets the passes of later rounds.
    LPR_TRY(exact_relabel());
    int PB = int(std::min<int64_t>(MAX_PASS_SLOTS, std::max<int64_t>(4, bfs_passes / 2 + 4)));
    PB += PB & 1;
    Scalars *host = nullptr;
    LPR_TRY(read_scalars(s, Lw, &host, P.noalloc));
    const bool use_graph = !P.timing && !P.no_graph && !P.noalloc;
    const int R = std::max(1, std::min(P.rounds_per_check, MAX_ROUNDS_PER_CHECK));
    for (;;) {
        if (host->all_done) break;
        if (rounds_enq >= P.max_rounds) break;
        const int nr = int(std::min<int64_t>(R, P.max_rounds - rounds_enq));
        for (int r = 0; r < nr; ++r) {
            ++rounds_enq;
            sweep_launches += P.K;
            bfs_passes += PB;
            if (!P.arg) {
                if (use_graph) {
                    GraphKey key = base_key;
                    key.K = P.K, key.L = P.L, key.P = PB, key.kind = GK_SEQ_ROUND;
                    LPR_TRY(launch_graph(key, s, [&](hipStream_t cs) {
                        return enqueue_seq_round<TH>(cs, D, Lw, B, P.K, P.L, PB, nullptr,
                                                     nullptr);
                    }));
                } else {
                    LPR_TRY(enqueue_seq_round<TH>(s, D, Lw, B, P.K, P.L, PB, &t_sweep,
                                                  &t_bfs));
                }
                continue;
            }
            // asynchronous round: the global relabel of the last snapshot on
            // stream sb beside the K sweeps on s, joined before the post step
            hipEvent_t fork = ev[2 * r], join = ev[2 * r + 1];
            LPR_TRY_HIP(hipEventRecord(fork, s));
            LPR_TRY_HIP(hipStreamWaitEvent(sb, fork, 0));
            if (use_graph) {
                GraphKey kp = base_key;
                kp.K = 0, kp.L = 0, kp.P = PB, kp.kind = GK_PASSES;
                LPR_TRY(launch_graph(kp, sb, [&](hipStream_t cs) {
                    return enqueue_passes<TH>(cs, D, Lw, PB, nullptr);
                }));
            } else {
                LPR_TRY(enqueue_passes<TH>(sb, D, Lw, PB, &t_bfs_b));
            }
            LPR_TRY_HIP(hipEventRecord(join, sb));
            if (use_graph) {
                GraphKey ks = base_key;
                ks.K = P.K, ks.L = P.L, ks.P = 0, ks.kind = GK_SWEEPS;
                LPR_TRY(launch_graph(ks, s, [&](hipStream_t cs) {
                    return enqueue_sweeps<TH>(cs, D, Lw, P.K, P.L, nullptr);
                }));
            } else {
                LPR_TRY(enqueue_sweeps<TH>(s, D, Lw, P.K, P.L, &t_sweep));
            }
            LPR_TRY_HIP(hipStreamWaitEvent(s, join, 0));
            if (use_graph) {
                GraphKey kq = base_key;
                kq.K = 0, kq.L = 0, kq.P = PB, kq.kind = GK_ARG_POST;
                LPR_TRY(launch_graph(kq, s, [&](hipStream_t cs) {
                    return enqueue_arg_post<TH>(cs, D, Lw, B, PB);
                }));
            } else {
                LPR_TRY(enqueue_arg_post<TH>(s, D, Lw, B, PB));
            }
        }
        LPR_TRY(read_scalars(s, Lw, &host, P.noalloc));
        if (host->open_bfs > 0) {
            // some global relabel needed more passes than the round carried:
            // more passes for later rounds; past the slot count, finish an
            // exact relabel under host control instead
            if (PB >= MAX_PASS_SLOTS) {
                LPR_TRY(exact_relabel());
            } else {
                PB = std::min(MAX_PASS_SLOTS, PB + std::max(4, PB / 2));
                PB += PB & 1;
                if (P.arg) LPR_TRY(fill_i32(Lw.sc->pass_count, 0, MAX_PASS_SLOTS, s));
            }
        } else if (host->max_need > 0) {
            // converged relabels: keep a margin of 4 passes over the most
            // needed (lowered in steps of at least 4, so that few graphs are
            // captured)
            int next = std::max(4, host->max_need + 4);
            next += next & 1;
            if (next <= PB - 4) {
                PB = next;
                if (P.arg) LPR_TRY(fill_i32(Lw.sc->pass_count, 0, MAX_PASS_SLOTS, s));
            }
        }
        LPR_TRY(fill_i32(&Lw.sc->open_bfs, 0, 2, s));  // open_bfs, max_need
        LPR_TRY(t_bfs.harvest(&bfs_ms));
        LPR_TRY(t_bfs_b.harvest(&bfs_ms));
        LPR_TRY(t_sweep.harvest(&sweep_ms));
    }
    if (!host->all_done) {
        set_error("grid max-flow: round budget (%d) exhausted", P.max_rounds);
        return LPR_EBUDGET;
    }
    const int64_t rounds = host->rounds;
    LPR_TRY(fill_i64(flow_values, 0, B, s));
    Kern<TH>::flow(s, D, flow_values);
    LPR_TRY_HIP(hipGetLastError());
    if (side) {
        // every instance takes part in the closure
        LPR_TRY(fill_i32(Lw.dirty_all, 0, 3 * int64_t(D.ntiles_r), s));
        LPR_TRY(fill_i32(&Lw.sc->seed_count, 0, 1, s));
        Kern<TH>::cut_seed(s, D);
        LPR_TRY_HIP(hipGetLastError());
        EventTimer none(s);
        LPR_TRY(relax_to_fixpoint<TH>(true, s, D, Lw, none, &cut_passes));
        Kern<TH>::cut_write(s, D, side);
        LPR_TRY_HIP(hipGetLastError());
    }
    unsigned long long cnt[8];
    LPR_TRY_HIP(hipMemcpyAsync(cnt, Lw.counters, sizeof(cnt),
                               hipMemcpyDeviceToHost, s));
    LPR_TRY_HIP(hipStreamSynchronize(s));
    LPR_TRY(t_bfs.harvest(&bfs_ms));
    LPR_TRY(t_bfs_b.harvest(&bfs_ms));
    LPR_TRY(t_sweep.harvest(&sweep_ms));
    if (stats) {
        // rounds counts the exact relabels too (the first one included);
        // sweeps ran K per round after the first relabel
        stats->rounds = rounds;
        stats->sweeps = sweep_launches;
        stats->bfs_passes = bfs_passes;
        stats->bfs_passes_with_work = int64_t(cnt[6]);
        stats->cut_passes = cut_passes;
        stats->pushes = int64_t(cnt[0]);
        stats->relabels = int64_t(cnt[1]);
        stats->tiles_swept = int64_t(cnt[2]);
        stats->tiles_relaxed = int64_t(cnt[3]);
        stats->device_atomics = int64_t(cnt[5]);
        stats->tile_rows = TH;
        stats->local_iters = P.L;
        stats->sweeps_per_relabel = P.K;
        stats->relax_tile_rows = RELAX_TH;
        stats->sweep_ms = sweep_ms;
        stats->bfs_ms = bfs_ms;
        stats->async_relabel = P.arg ? 1 : 0;
        stats->rounds_per_check = R;
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
    int arg;  // asynchronous global relabel
    int R;    // rounds between host checks
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
    return (s.TH == 4 || s.TH == 8 || s.TH == 16 || s.TH == 32) && s.L >= 1 && s.L <= 4096 &&
           s.K >= 1 && s.K <= 4096 && (s.arg == 0 || s.arg == 1) && s.R >= 1 &&
           s.R <= MAX_ROUNDS_PER_CHECK;
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
    while (std::fscanf(f, "%d %d %d %d %d %d", &c, &sc.TH, &sc.L, &sc.K, &sc.arg, &sc.R) == 6)
        if (c >= 0 && c < 64 && valid_sched(sc)) g_sched[c] = sc;
    std::fclose(f);
}

static Sched default_sched(int64_t N) {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    load_sched_file_locked();
    const auto it = g_sched.find(size_class(N));
    if (it != g_sched.end()) return it->second;
    // the schedule search on MI355X: 64 x 8 tiles, 16 local iterations for
    // the 1024 x 1024 graph cut (2.0 ms); 64 x 16 tiles, 16 iterations for the
    // 2048 x 2048 grid alone (8.3 ms) and for the batched workload of 10.5 M
    // pixels (11.3 ms); 4 sweeps per round and the relabel between the
    // sweeps throughout
    if (N >= (int64_t(1) << 22)) return Sched{16, 16, 4, 0, 2};
    return Sched{8, 16, 4, 0, 2};
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
        std::fprintf(f, "%d %d %d %d %d %d\n", e.first, e.second.TH, e.second.L, e.second.K,
                     e.second.arg, e.second.R);
    std::fclose(f);
}

static lpr_status run(int32_t B, const int32_t *H, const int32_t *W,
                      const int64_t *node_offset, const int32_t *const caps[6],
                      int64_t *flow_values, uint8_t *side,
                      const lpr_grid_opts *opts, lpr_grid_stats *stats,
                      void *workspace, size_t ws_bytes, void *stream,
                      bool noalloc = false) {
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
        // heights up to |V| = H*W + 2 are packed with a 3-bit direction into
        // 32 bits by the push sweep
        if (H[b] < 1 || W[b] < 1 || int64_t(H[b]) * W[b] >= (int64_t(1) << 28)) {
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
    P.rounds_per_check = ds.R;
    P.arg = ds.arg != 0;
    P.timing = false;
    P.no_graph = false;
    P.noalloc = noalloc;
    if (opts) {
        if (opts->tile_rows) P.TH = opts->tile_rows;
        if (opts->local_iters) P.L = opts->local_iters;
        if (opts->sweeps_per_relabel) P.K = opts->sweeps_per_relabel;
        if (opts->max_rounds) P.max_rounds = opts->max_rounds;
        if (opts->rounds_per_check) P.rounds_per_check = opts->rounds_per_check;
        P.timing = (opts->flags & LPR_GRID_TIME_KERNELS) != 0;
        P.no_graph = (opts->flags & LPR_GRID_NO_GRAPH) != 0;
        if ((opts->flags & LPR_GRID_ASYNC_RELABEL) && (opts->flags & LPR_GRID_SYNC_RELABEL)) {
            set_error("LPR_GRID_ASYNC_RELABEL and LPR_GRID_SYNC_RELABEL both set");
            return LPR_EINVAL;
        }
        if (opts->flags & LPR_GRID_ASYNC_RELABEL) P.arg = true;
        if (opts->flags & LPR_GRID_SYNC_RELABEL) P.arg = false;
        if (opts->reserved[0] || opts->reserved[1]) {
            set_error("lpr_grid_opts.reserved must be 0");
            return LPR_EINVAL;
        }
    }
    if (!(P.TH == 4 || P.TH == 8 || P.TH == 16 || P.TH == 32) || P.L < 1 || P.L > 4096 ||
        P.K < 1 || P.K > 4096 || P.max_rounds < 1 || P.rounds_per_check < 1 ||
        P.rounds_per_check > MAX_ROUNDS_PER_CHECK) {
        set_error("invalid lpr_grid_opts");
        return LPR_EINVAL;
    }
    if (noalloc && (opts && (opts->flags & LPR_GRID_ASYNC_RELABEL))) {
        set_error("LPR_GRID_ASYNC_RELABEL needs a library stream and events, which the "
                  "allocation-free entry point does not create");
        return LPR_EINVAL;
    }
    if (noalloc) P.arg = false;
    if (noalloc && P.timing) {
        set_error("LPR_GRID_TIME_KERNELS needs HIP events, which the "
                  "allocation-free entry point does not create");
        return LPR_EINVAL;
    }
    const int64_t N = node_offset[B];
    std::vector<Inst> insts(B);
    std::vector<int32_t> tile_inst, tile_inst_r;
    for (int b = 0; b < B; ++b) {
        Inst &I = insts[b];
        I.off = node_offset[b];
        I.H = H[b];
        I.W = W[b];
        I.tiles_x = ceil_div(W[b], TW);
        I.tiles_y = ceil_div(H[b], P.TH);
        I.tile_base = int32_t(tile_inst.size());
        I.HV = H[b] * W[b] + 2;
        I.tiles_y_r = ceil_div(H[b], RELAX_TH);
        I.tile_base_r = int32_t(tile_inst_r.size());
        tile_inst.insert(tile_inst.end(), size_t(I.tiles_x) * I.tiles_y, b);
        tile_inst_r.insert(tile_inst_r.end(), size_t(I.tiles_x) * I.tiles_y_r, b);
    }
    const int64_t T = int64_t(tile_inst.size());
    const int64_t TR = int64_t(tile_inst_r.size());
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
    Carver cv = carve(Carver(workspace, ws_bytes), N, T, TR, B, &Lw);
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
    D.lab = Lw.lab;
    D.amask = Lw.amask;
    for (int i = 0; i < 3; ++i) {
        D.act[i] = Lw.act[i];
        D.alist[i] = Lw.alist[i];
        D.dirty[i] = Lw.dirty_all + int64_t(i) * TR;
        D.dlist[i] = Lw.dlist[i];
    }
    D.cap_src = caps[0];
    D.cap_snk = caps[1];
    D.cap_r = caps[2];
    D.cap_l = caps[3];
    D.cap_d = caps[4];
    D.cap_u = caps[5];
    D.inst = Lw.inst;
    D.tile_inst = Lw.tile_inst;
    D.tile_inst_r = Lw.tile_inst_r;
    D.inst_active = Lw.inst_cnt;
    D.inst_exact = Lw.inst_cnt + B;
    D.done = Lw.done;
    D.counters = Lw.counters;
    D.sc = Lw.sc;
    D.ntiles = int32_t(T);
    D.ntiles_r = int32_t(TR);
    D.ninst = B;
    D.seg_scan = (opts && (opts->flags & LPR_GRID_SEGMENTED_SCAN)) ? 1 : 0;
    for (int b = 0; b < B; ++b)
        if (insts[b].HV > OFFSET_SCAN_MAX_HV) D.seg_scan = 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GraphKey key{};
    LPR_TRY_HIP(hipGetDevice(&key.device));
    key.ws = workspace;
    for (int i = 0; i < 6; ++i) key.caps[i] = caps[i];
    key.N = N;
    key.B = B;
    key.T = int(T);
    key.TR = int(TR);
    key.TH = P.TH;
    key.seg = D.seg_scan;
    // the call's HIP events (not on the allocation-free path, which times the
    // call on the host clock instead)
    std::optional<CallTimer> call;
    if (!noalloc) {
        call.emplace(s);
        call->start();
    }
    const auto t0 = std::chrono::steady_clock::now();
    lpr_status st;
    switch (P.TH) {
        case 4:
            st = solve<4>(P, B, insts, tile_inst, tile_inst_r, D, Lw, key, flow_values, side, stats, s);
            break;
        case 8:
            st = solve<8>(P, B, insts, tile_inst, tile_inst_r, D, Lw, key, flow_values, side, stats, s);
            break;
        case 16:
            st = solve<16>(P, B, insts, tile_inst, tile_inst_r, D, Lw, key, flow_values, side, stats, s);
            break;
        default:
            st = solve<32>(P, B, insts, tile_inst, tile_inst_r, D, Lw, key, flow_values, side, stats, s);
            break;
    }
    if (st != LPR_OK) {
        (void)hipStreamSynchronize(s);
        return st;
    }
    double ms = 0;
    if (call) {
        LPR_TRY(call->stop_ms(&ms));
    } else {
        LPR_TRY_HIP(hipStreamSynchronize(s));
        ms = std::chrono::duration<double, std::milli>(
                 std::chrono::steady_clock::now() - t0).count();
    }
    if (stats) stats->total_ms = ms;
    return LPR_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free entry point: the workspace of one grid lives in `scratch`,
// a device array of the library, so the call needs no caller workspace and
// allocates nothing (no device or pinned memory, no graph, no event).  Every
// GPU the library runs on holds its own copy until the process ends; calls
// that overlap on one GPU share it and race.  Everything a solve reads is
// written by that solve first (state, tables, flags, counters), so the
// previous call's contents do no harm.
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = size_t(40) << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_SCRATCH_DEVICES = 64;

// Device address of the calling device's `scratch` (looked up once per
// device, with that device current; the array's name is a host-side stand-in
// and is never passed to a kernel).
static lpr_status scratch_ptr(void **out) {
    static std::mutex mu;
    static void *ptrs[MAX_SCRATCH_DEVICES] = {};
    int dev = -1;
    LPR_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_SCRATCH_DEVICES) {
        set_error("device %d out of range for the allocation-free entry point", dev);
        return LPR_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!ptrs[dev]) {
        void *p = nullptr;
        LPR_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress returned NULL for the scratch array");
            return LPR_EDEVICE;
        }
        ptrs[dev] = p;
    }
    *out = ptrs[dev];
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

extern "C" size_t lpr_grid_maxflow_noalloc_max_bytes(void) {
    return grid::SCRATCH_BYTES;
}

extern "C" lpr_status lpr_grid_maxflow_noalloc(int32_t H, int32_t W,
                                               const int32_t *cap_src,
                                               const int32_t *cap_snk,
                                               const int32_t *cap_right,
                                               const int32_t *cap_left,
                                               const int32_t *cap_down,
                                               const int32_t *cap_up,
                                               int64_t *flow_value,
                                               uint8_t *source_side,
                                               const lpr_grid_opts *opts,
                                               lpr_grid_stats *stats, void *stream) {
    const int32_t *caps[6] = {cap_src, cap_snk, cap_right, cap_left, cap_down, cap_up};
    const int64_t off[2] = {0, int64_t(H) * W};
    clear_error();
    if (H < 1 || W < 1) {
        set_error("bad shape %d x %d", H, W);
        return LPR_EINVAL;
    }
    const size_t need = grid::workspace_bytes(1, &H, &W);
    if (need > grid::SCRATCH_BYTES) {
        set_error("a %d x %d grid needs %zu bytes of scratch; the allocation-free "
                  "entry point holds %zu (grids of up to about 1.25 M pixels)",
                  H, W, need, grid::SCRATCH_BYTES);
        return LPR_ENOMEM;
    }
    void *ws = nullptr;
    LPR_TRY(grid::scratch_ptr(&ws));
    return grid::run(1, &H, &W, off, caps, flow_value, source_side, opts, stats, ws,
                     grid::SCRATCH_BYTES, stream, /*noalloc=*/true);
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
    static const int THs[4] = {4, 8, 16, 32};
    static const int Ls[4] = {4, 8, 16, 32};
    static const int Ks[3] = {2, 4, 8};
    static const int Rs[4] = {1, 2, 4, 8};
    std::vector<int64_t> ref(B), got(B);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double best_t = 1e300;
    grid::Sched best_s{8, 16, 4, 0, 4};
    bool have_ref = false;
    // one timed schedule: the fastest of `reps` runs after a warm-up, its
    // flow values checked against the first schedule's
    auto trial = [&](const grid::Sched &sc) -> lpr_status {
        lpr_grid_opts o{};
        o.tile_rows = sc.TH;
        o.local_iters = sc.L;
        o.sweeps_per_relabel = sc.K;
        o.rounds_per_check = sc.R;
        o.flags = sc.arg ? LPR_GRID_ASYNC_RELABEL : LPR_GRID_SYNC_RELABEL;
        double t_min = 1e300;
        for (int r = 0; r <= reps; ++r) {  // the first run warms up
            lpr_grid_stats st{};
            LPR_TRY(grid::run(B, H, W, node_offset, caps, flow_values, nullptr, &o, &st,
                              workspace, workspace_bytes, stream));
            if (r > 0) t_min = std::min(t_min, st.total_ms);
        }
        LPR_TRY_HIP(hipMemcpyAsync(got.data(), flow_values, sizeof(int64_t) * B,
                                   hipMemcpyDeviceToHost, s));
        LPR_TRY_HIP(hipStreamSynchronize(s));
        if (!have_ref) {
            ref = got;
            have_ref = true;
        } else if (got != ref) {
            set_error("schedules disagree on a flow value (tile rows %d, local "
                      "iterations %d, sweeps %d, asynchronous relabel %d, rounds "
                      "per check %d)", sc.TH, sc.L, sc.K, sc.arg, sc.R);
            return LPR_EDEVICE;
        }
        if (t_min < best_t) {
            best_t = t_min;
            best_s = sc;
        }
        return LPR_OK;
    };
    // stage 1: every tile height, local iteration count, sweep count and
    // relabel mode at 4 rounds per check; stage 2: the check interval of
    // the winner
    for (int arg = 0; arg <= 1; ++arg)
        for (int th : THs)
            for (int l : Ls)
                for (int k : Ks) LPR_TRY(trial(grid::Sched{th, l, k, arg, 4}));
    const grid::Sched stage1 = best_s;
    for (int r : Rs)
        if (r != stage1.R) LPR_TRY(trial(grid::Sched{stage1.TH, stage1.L, stage1.K, stage1.arg, r}));
    grid::store_sched(node_offset[B], best_s);
    if (best) {
        *best = lpr_grid_opts{};
        best->tile_rows = best_s.TH;
        best->local_iters = best_s.L;
        best->sweeps_per_relabel = best_s.K;
        best->rounds_per_check = best_s.R;
        best->flags = best_s.arg ? LPR_GRID_ASYNC_RELABEL : LPR_GRID_SYNC_RELABEL;
    }
    if (best_ms) *best_ms = best_t;
    return LPR_OK;
}
