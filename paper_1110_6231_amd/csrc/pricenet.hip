// Learned warm start for cost scaling: column features of the cost matrix
// and a small permutation-equivariant price network, forward and backward,
// on gfx950 BF16 matrix cores with FP32 accumulation.
//
// The paper has no learned component.  The network predicts normalised
// column prices q(y); the solver starts from p(y) = rint(q(y) * sc * (2n+1))
// with a small initial epsilon.  Refine recomputes the row prices from p(Y)
// (Algorithm 5.2), so the result of the solve is exact whatever the network
// predicts; only the amount of work depends on it.
//
// Features (16 per column, symmetric over rows): with sc = mean |c| and
// z = c / sc, rr(x,y) = z(x,y) - min_y' z(x,y'):
//   f0..f7  8 smallest z(.,y) ascending   f8, f9  mean, std of z(.,y)
//   f10,f11 2 smallest rr(.,y)             f12     mean rr(.,y)
//   f13     v2(y) - mean v2 with u2(x) = min_y (z - f10(y)),
//           v2(y) = min_x (z - u2(x))
//   f14     g(y) - mean g: the column potential of the entropic (Sinkhorn)
//           dual of the assignment with costs z after SINK_ITERS
//           alternating exact updates at a falling temperature tau,
//             f(x) = -tau log sum_y exp(-(z(x,y) - g(y)) / tau),
//             g(y) = -tau log sum_x exp(-(z(x,y) - f(x)) / tau),
//           from g = 0, tau = SINK_TAU0 times SINK_RATE per step down to
//           SINK_TAU_MIN; as tau falls f + g tends to an optimal dual of
//           the assignment, the quantity the network predicts
//   f15     log(n) / 6
// Network over the columns of each instance (H0 = features):
//   H_l = relu(H_{l-1} W_l + mean_cols(H_{l-1}) U_l + b_l), l = 1..3 (width
//   128), q = H_3 w_o + b_o + f14 (a skip connection: the network predicts
//   the correction to the Sinkhorn potential).  Parameters: one float32 vector, W1 [16,128],
//   U1 [16,128], b1, W2, U2 [128,128], b2, W3, U3, b3, w_o [128], b_o.
// Loss: (1 / sum n) sum ((q - mean q) - t)^2 per instance, t centred.
//
// Layout on the device: columns of all instances are stacked as rows of the
// activation matrices ("rows" below), padded to a multiple of 64.  Every
// activation is kept in bf16 twice, row-major and transposed, so that all
// three GEMMs of a layer (Z = H W, dW = H^T dZ, dH = dZ W^T) read both
// operands contiguously along the reduction dimension (NT GEMM).
#include <algorithm>
#include <cmath>
#include <vector>

#include "lpr_internal.h"

namespace lpr {
namespace net {

constexpr int F_IN = 16;
constexpr int F_PAD = 32;   // features padded to one MFMA K-step
constexpr int WID = 128;
constexpr double SINK_TAU0 = 0.3;
constexpr double SINK_RATE = 0.7;
constexpr double SINK_TAU_MIN = 0.003;
constexpr int SINK_ITERS = 16;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Parameter offsets (floats) inside the flat vector.
constexpr int64_t OFF_W[3] = {0, 4224, 37120};
constexpr int64_t OFF_U[3] = {2048, 20608, 53504};
constexpr int64_t OFF_B[3] = {4096, 36992, 69888};
constexpr int64_t OFF_WO = 70016;
constexpr int64_t OFF_BO = 70144;
constexpr int64_t N_PARAMS = 70145;
constexpr int KIN[3] = {F_IN, WID, WID};    // true input width per layer
constexpr int KPAD[3] = {F_PAD, WID, WID};  // padded input width

struct NInst {
    int64_t cost_off;  // first entry of the instance in the int32 input
    int64_t c16_off;   // first entry in the int16 copy (rows ld entries apart)
    int32_t n;
    int32_t ld;        // row stride of the int16 copy: n rounded up to 8
    int32_t row_off;   // first stacked row (column) of the instance
    int32_t p_off;     // first entry of the instance's padded potentials
};

// Row stride of the int16 copy and of the padded potentials: a multiple of 8
// entries, so that every row starts 16-byte aligned and 8 costs (or 8
// potentials, 32 bytes) are one aligned vector load.
__host__ __device__ inline int ld16(int n) { return (n + 7) & ~7; }
typedef int int4v __attribute__((ext_vector_type(4)));
typedef int int2v __attribute__((ext_vector_type(2)));
typedef float float4v __attribute__((ext_vector_type(4)));

__device__ inline __bf16 to_bf16(float f) { return (__bf16)f; }
__device__ inline float from_bf16(__bf16 b) { return (float)b; }

// ---------------------------------------------------------------------------
// Feature passes
// ---------------------------------------------------------------------------
// Row pass 1: min_y c(x,y), the instance's sum and maximum of |c|, and a
// saturated int16 copy of sign * c that the later passes read instead of the
// int32 input when the instance's costs fit (half the bytes per pass), its
// rows padded with zeros to ld16(n) entries.
// grid = (row blocks, B): block (i, b) takes rows ROWS1 i .. ROWS1 (i+1) - 1
// of instance b, one wavefront per row in turn, and adds its part of the sum
// with one atomic (the instance's rows then meet in few device-scope
// atomics).
constexpr int ROWS1 = 16;
constexpr int C16_MAX = 32767;
__global__ __launch_bounds__(256) void k_feat_rows1(const NInst *inst,
                                                    const int32_t *costs,
                                                    int32_t sign, int32_t *rowmin,
                                                    unsigned long long *abssum,
                                                    int16_t *c16, unsigned *cmax) {
    const NInst I = inst[blockIdx.y];
    const int x0 = blockIdx.x * ROWS1;
    if (x0 >= I.n) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long s = 0;
    unsigned amax = 0;
    for (int x = x0 + wave; x < min(x0 + ROWS1, I.n); x += 4) {
        const int32_t *row = costs + I.cost_off + int64_t(x) * I.n;
        int16_t *crow = c16 + I.c16_off + int64_t(x) * I.ld;
        int mn = INT_MAX;
        // eight columns per lane per step, every load issued first (from a
        // clamped valid column), then the uses
        for (int y0 = 0; y0 < I.n; y0 += 512) {
            int v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = row[min(y0 + lane + 64 * k, I.n - 1)];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int y = y0 + lane + 64 * k;
                if (y >= I.n) break;
                const int c = sign * v[k];
                mn = min(mn, c);
                const unsigned a = unsigned(c < 0 ? -c : c);
                s += a;
                amax = max(amax, a);
                crow[y] = int16_t(max(-C16_MAX, min(C16_MAX, c)));
            }
        }
        if (lane < I.ld - I.n) crow[I.n + lane] = 0;  // padding
        for (int o = 32; o > 0; o >>= 1) mn = min(mn, __shfl_xor(mn, o, 64));
        if (lane == 0) rowmin[I.row_off + x] = mn;
    }
    for (int o = 32; o > 0; o >>= 1) amax = max(amax, unsigned(__shfl_xor(int(amax), o, 64)));
    if (lane == 0 && amax) atomicMax(&cmax[blockIdx.y], amax);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ unsigned long long part[4];
    if (lane == 0) part[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&abssum[blockIdx.y], part[0] + part[1] + part[2] + part[3]);
}

// sign * c(x, y) of an instance: from the int16 copy when the instance's |c|
// fits it, else from the int32 input
struct Costs {
    const int32_t *c32;
    const int16_t *c16;
    const unsigned *cmax;
    int32_t sign;
    __device__ bool small(int b) const { return cmax[b] <= unsigned(C16_MAX); }
    __device__ int at(bool s16, const NInst &I, int x, int y) const {
        return s16 ? int(c16[I.c16_off + int64_t(x) * I.ld + y])
                   : sign * c32[I.cost_off + int64_t(x) * I.n + y];
    }
    // entries y0 .. y0+7 of row x (y0 a multiple of 8); entries at or past n
    // are 0
    __device__ void at8(bool s16, const NInst &I, int x, int y0, int (&c)[8]) const {
        if (s16) {
            const int4v w = *reinterpret_cast<const int4v *>(c16 + I.c16_off +
                                                             int64_t(x) * I.ld + y0);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                c[2 * k] = int(int16_t(w[k] & 0xffff));
                c[2 * k + 1] = w[k] >> 16;
            }
        } else {
            const int32_t *row = c32 + I.cost_off + int64_t(x) * I.n;
#pragma unroll
            for (int k = 0; k < 8; ++k) c[k] = y0 + k < I.n ? sign * row[y0 + k] : 0;
        }
    }
    // entries y0 .. y0+3 of row x (y0 a multiple of 4, y0 < n); entries at
    // or past n are 0 (int16 padding) or not read (int32)
    __device__ void at4(bool s16, const NInst &I, int x, int y0, int (&c)[4]) const {
        if (s16) {
            const int2v w = *reinterpret_cast<const int2v *>(c16 + I.c16_off +
                                                             int64_t(x) * I.ld + y0);
            c[0] = int(int16_t(w[0] & 0xffff));
            c[1] = w[0] >> 16;
            c[2] = int(int16_t(w[1] & 0xffff));
            c[3] = w[1] >> 16;
        } else {
            const int32_t *row = c32 + I.cost_off + int64_t(x) * I.n;
#pragma unroll
            for (int k = 0; k < 4; ++k) c[k] = y0 + k < I.n ? sign * row[y0 + k] : 0;
        }
    }
};

__device__ inline float inst_scale(const NInst &I, const unsigned long long *abssum, int b) {
    const double m = double(abssum[b]) / (double(I.n) * double(I.n));
    return m > 0 ? float(m) : 1.0f;
}

// rows loaded ahead in the column passes (one thread per column leaves
// about one wavefront per SIMD, so the loads in flight set the pace)
constexpr int FEAT_AHEAD = 32;

// Column pass 1: one thread per stacked column.
__global__ __launch_bounds__(256) void k_feat_cols1(const NInst *inst,
                                                    const int32_t *rinst, Costs CV,
                                                    int32_t R, const int32_t *rowmin,
                                                    const unsigned long long *abssum,
                                                    float *F) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= R) return;
    const int b = rinst[r];
    const NInst I = inst[b];
    const int y = r - I.row_off, n = I.n;
    const float inv = 1.0f / inst_scale(I, abssum, b);
    const bool s16 = CV.small(b);
    const int32_t *rm = rowmin + I.row_off;
    float top[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) top[k] = INFINITY;
    float r0 = INFINITY, r1 = INFINITY;
    float sz = 0.f, szz = 0.f, srr = 0.f;
    // the loads of FEAT_AHEAD rows are in flight before the first is used
    int cb[FEAT_AHEAD], mb[FEAT_AHEAD];
    for (int x0 = 0; x0 < n; x0 += FEAT_AHEAD) {
#pragma unroll
        for (int a = 0; a < FEAT_AHEAD; ++a) {
            const int x = x0 + a < n ? x0 + a : n - 1;
            cb[a] = CV.at(s16, I, x, y);
            mb[a] = rm[x];
        }
#pragma unroll
        for (int a = 0; a < FEAT_AHEAD; ++a) {
            if (x0 + a >= n) break;
            const int c = cb[a];
            const float z = float(c) * inv;
            const float rr = float(c - mb[a]) * inv;
            sz += z;
            szz += z * z;
            srr += rr;
            if (z < top[7]) {
                float v = z;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const float lo = fminf(top[k], v);
                    v = fmaxf(top[k], v);
                    top[k] = lo;
                }
            }
            if (rr < r1) {
                if (rr < r0) {
                    r1 = r0;
                    r0 = rr;
                } else {
                    r1 = rr;
                }
            }
        }
    }
    float *f = F + int64_t(r) * F_IN;
    for (int k = 0; k < 8; ++k) f[k] = top[k < n ? k : n - 1];
    const float mean = sz / n;
    f[8] = mean;
    f[9] = sqrtf(fmaxf(szz / n - mean * mean, 0.f));
    f[10] = r0;
    f[11] = n > 1 ? r1 : r0;
    f[12] = srr / n;
}

// Sinkhorn passes of f14: one workgroup per instance runs every iteration
// (instances are independent, so no grid-wide step is needed), with g in
// LDS.  A row x of an iteration, v(y) = z(x,y) - g(y) with the g of the
// iteration before, gives
//   m = min_y v,  e(y) = exp2((m - v(y)) log2(e) / tau),  s = sum_y e,
//   f(x) = m - tau ln s,
// and the same e also give the column update: exp((g(y) + f(x) - z(x,y)) /
// tau) = e(y) / s, so
//   g'(y) = -tau ln sum_x exp(-(z(x,y) - f(x)) / tau) = g(y) - tau ln S(y),
//   S(y) = sum_x e(x,y) / s(x).
// One read of the matrix per iteration, and every term is <= 1 (no
// overflow).  S(y) is the column's mass under the row-normalised plan; if
// it falls below 2^-100 (a column nearly no row wants, where float32 loses
// the sum), that column is recomputed directly from the f of the iteration
// with its own minimum (both log-sum-exps are then taken exactly as the
// definition reads).
constexpr float LOG2E = 1.4426950408889634f;
constexpr int SINK_W = 16;  // wavefronts per workgroup
template <int CTRL>
__device__ inline float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ inline float lane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
// min and sum over the 64 lanes of a fully active wavefront, wave-uniform:
// DPP inside rows of 16 lanes, then the four row results
__device__ inline float wave_minf(float v) {
    v = fminf(v, dpp_f<0xB1>(v));   // quad_perm [1,0,3,2]
    v = fminf(v, dpp_f<0x4E>(v));   // quad_perm [2,3,0,1]
    v = fminf(v, dpp_f<0x141>(v));  // row_half_mirror
    v = fminf(v, dpp_f<0x140>(v));  // row_mirror
    return fminf(fminf(lane_f(v, 0), lane_f(v, 16)), fminf(lane_f(v, 32), lane_f(v, 48)));
}
__device__ inline float wave_sumf(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    return (lane_f(v, 0) + lane_f(v, 16)) + (lane_f(v, 32) + lane_f(v, 48));
}
// The min (or sum) of four rows at once, one value of each per lane: the
// wavefront halves of rows 0 and 1 (2 and 3) are swapped against each other
// (gfx950's permlane32 swap) and combined, so one register holds row 0 in
// lanes 0-31 and row 1 in lanes 32-63; the 16-lane rows of the two
// registers are swapped the same way (permlane16 swap), leaving rows 0, 2,
// 1, 3 in the four 16-lane rows of one register, which the DPP steps above
// reduce together.  About a third of the instructions of four reductions.
template <bool MIN>
__device__ inline float op2(float a, float b) {
    return MIN ? fminf(a, b) : a + b;
}
template <bool MIN>
__device__ inline void wave_reduce4(const float (&v)[4], float (&out)[4]) {
    const auto s01 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[0]),
                                                      __float_as_uint(v[1]), false, false);
    const auto s23 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2]),
                                                      __float_as_uint(v[3]), false, false);
    const float a = op2<MIN>(__uint_as_float(s01[0]), __uint_as_float(s01[1]));
    const float b = op2<MIN>(__uint_as_float(s23[0]), __uint_as_float(s23[1]));
    const auto t = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b),
                                                    false, false);
    float c = op2<MIN>(__uint_as_float(t[0]), __uint_as_float(t[1]));
    c = op2<MIN>(c, dpp_f<0xB1>(c));
    c = op2<MIN>(c, dpp_f<0x4E>(c));
    c = op2<MIN>(c, dpp_f<0x141>(c));
    c = op2<MIN>(c, dpp_f<0x140>(c));
    out[0] = lane_f(c, 0);
    out[2] = lane_f(c, 16);
    out[1] = lane_f(c, 32);
    out[3] = lane_f(c, 48);
}
// Two rows: after the halves swap, one register holds row 0 in lanes 0-31
// and row 1 in lanes 32-63; swapping its 16-lane rows with themselves folds
// each half onto 16 lanes, which the DPP steps then reduce.
template <bool MIN>
__device__ inline void wave_reduce2(const float (&v)[2], float (&out)[2]) {
    const auto s01 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[0]),
                                                      __float_as_uint(v[1]), false, false);
    const float a = op2<MIN>(__uint_as_float(s01[0]), __uint_as_float(s01[1]));
    const auto t = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(a),
                                                    false, false);
    float c = op2<MIN>(__uint_as_float(t[0]), __uint_as_float(t[1]));
    c = op2<MIN>(c, dpp_f<0xB1>(c));
    c = op2<MIN>(c, dpp_f<0x4E>(c));
    c = op2<MIN>(c, dpp_f<0x141>(c));
    c = op2<MIN>(c, dpp_f<0x140>(c));
    out[0] = lane_f(c, 0);
    out[1] = lane_f(c, 32);
}

// V: 8-entry groups per lane per row (rows up to 512 V entries); RW: rows a
// wavefront takes at once (their loads and reductions overlap).  ids[] lists
// the instances of this launch; g is written to gpad[p_off + y].  Dynamic
// LDS: (SINK_W + 2) ld floats (g, SINK_W partial column sums, f).
template <int V, int RW>
__global__ __launch_bounds__(64 * SINK_W) void k_sinkhorn(const NInst *inst,
                                                          const int32_t *ids, Costs CV,
                                                          const unsigned long long *abssum,
                                                          float *gpad) {
    extern __shared__ float sh[];
    const int b = ids[blockIdx.x];
    const NInst I = inst[b];
    const int n = I.n, ld = I.ld;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const float inv = 1.0f / inst_scale(I, abssum, b);
    const bool s16 = CV.small(b);
    float *gs = sh, *part = sh + ld, *fs = sh + (SINK_W + 1) * ld;
    for (int y = threadIdx.x; y < ld; y += 64 * SINK_W) gs[y] = 0.f;
    __syncthreads();
    double t = SINK_TAU0;
    for (int it = 0; it < SINK_ITERS; ++it) {
        const float tau = float(t), kl = LOG2E / tau;
        float acc[V][8];
#pragma unroll
        for (int j = 0; j < V; ++j)
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[j][k] = 0.f;
        // rows x0 .. x0+RW-1 of this wavefront, their costs in c: v, the
        // row minima and sums, f, and the column partial sums
        auto rows = [&](int x0, const int (&c)[RW][V][8]) {
            // -g of the lane's columns, +inf past n (also in a group the
            // clamp repeats), so that v = c / sc - g is one fma, and +inf
            // there; rows past n are computed and dropped
            float ng[V][8];
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const int y0 = 8 * (lane + 64 * j);
                const int yc = min(y0, ld - 8);
                const float4v g0 = *reinterpret_cast<const float4v *>(gs + yc);
                const float4v g1 = *reinterpret_cast<const float4v *>(gs + yc + 4);
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    ng[j][k] = y0 + k < n ? -(k < 4 ? g0[k] : g1[k - 4]) : INFINITY;
            }
            float z[RW][V][8];
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int j = 0; j < V; ++j)
#pragma unroll
                    for (int k = 0; k < 8; ++k) z[r][j][k] = fmaf(float(c[r][j][k]), inv, ng[j][k]);
            float m[RW], sr[RW], part_r[RW];
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                float mm = INFINITY;
#pragma unroll
                for (int j = 0; j < V; ++j)
#pragma unroll
                    for (int k = 0; k < 8; ++k) mm = fminf(mm, z[r][j][k]);
                part_r[r] = mm;
            }
            if constexpr (RW == 4) {
                wave_reduce4<true>(part_r, m);
            } else if constexpr (RW == 2) {
                wave_reduce2<true>(part_r, m);
            } else {
#pragma unroll
                for (int r = 0; r < RW; ++r) m[r] = wave_minf(part_r[r]);
            }
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                // exp2((m - v) kl) with the product m kl taken once
                const float mk = m[r] * kl;
                float ss = 0.f;
#pragma unroll
                for (int j = 0; j < V; ++j)
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        z[r][j][k] = __builtin_amdgcn_exp2f(fmaf(z[r][j][k], -kl, mk));
                        ss += z[r][j][k];
                    }
                part_r[r] = ss;
            }
            if constexpr (RW == 4) {
                wave_reduce4<false>(part_r, sr);
            } else if constexpr (RW == 2) {
                wave_reduce2<false>(part_r, sr);
            } else {
#pragma unroll
                for (int r = 0; r < RW; ++r) sr[r] = wave_sumf(part_r[r]);
            }
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                if (x0 + r >= n) break;
                const float rs = 1.0f / sr[r];
#pragma unroll
                for (int j = 0; j < V; ++j)
#pragma unroll
                    for (int k = 0; k < 8; ++k) acc[j][k] = fmaf(z[r][j][k], rs, acc[j][k]);
                if (lane == 0) fs[x0 + r] = m[r] - tau * __logf(sr[r]);
            }
        };
        // every load is unconditional, from a clamped valid address (a row
        // past n repeats row n-1, a group past ld repeats the last one);
        // the values are masked in rows()
        if (s16) {
            // the int16 rows of the next step are loaded while this step's
            // are processed
            auto load = [&](int x0, int4v (&q)[RW][V]) {
#pragma unroll
                for (int r = 0; r < RW; ++r)
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        const int xr = min(x0 + r, n - 1);
                        const int yc = min(8 * (lane + 64 * j), ld - 8);
                        q[r][j] = *reinterpret_cast<const int4v *>(CV.c16 + I.c16_off +
                                                                   int64_t(xr) * ld + yc);
                    }
            };
            int4v q[RW][V];
            if (RW * w < n) load(RW * w, q);
            for (int x0 = RW * w; x0 < n; x0 += RW * SINK_W) {
                int4v qn[RW][V];
                if (x0 + RW * SINK_W < n) load(x0 + RW * SINK_W, qn);
                int c[RW][V][8];
#pragma unroll
                for (int r = 0; r < RW; ++r)
#pragma unroll
                    for (int j = 0; j < V; ++j)
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            c[r][j][2 * k] = int(int16_t(q[r][j][k] & 0xffff));
                            c[r][j][2 * k + 1] = q[r][j][k] >> 16;
                        }
                rows(x0, c);
#pragma unroll
                for (int r = 0; r < RW; ++r)
#pragma unroll
                    for (int j = 0; j < V; ++j) q[r][j] = qn[r][j];
            }
        } else {
            for (int x0 = RW * w; x0 < n; x0 += RW * SINK_W) {
                int c[RW][V][8];
#pragma unroll
                for (int r = 0; r < RW; ++r)
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        const int32_t *row = CV.c32 + I.cost_off + int64_t(min(x0 + r, n - 1)) * n;
#pragma unroll
                        for (int k = 0; k < 8; ++k)
                            c[r][j][k] = CV.sign * row[min(8 * (lane + 64 * j) + k, n - 1)];
                    }
                rows(x0, c);
            }
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const int y0 = 8 * (lane + 64 * j);
            if (y0 < ld)
#pragma unroll
                for (int k = 0; k < 8; ++k) part[w * ld + y0 + k] = acc[j][k];
        }
        __syncthreads();  // every row read g and wrote its f and partial sums
        for (int y = threadIdx.x; y < n; y += 64 * SINK_W) {
            float S = 0.f;
#pragma unroll
            for (int q = 0; q < SINK_W; ++q) S += part[q * ld + y];
            float gy;
            if (S >= 0x1p-100f) {
                gy = gs[y] - tau * __logf(S);
            } else {
                float mm = INFINITY;
                for (int x = 0; x < n; ++x)
                    mm = fminf(mm, float(CV.at(s16, I, x, y)) * inv - fs[x]);
                float ss = 0.f;
                for (int x = 0; x < n; ++x)
                    ss += __builtin_amdgcn_exp2f(
                        (mm - (float(CV.at(s16, I, x, y)) * inv - fs[x])) * kl);
                gy = mm - tau * __logf(ss);
            }
            gs[y] = gy;  // every read of the old g ended at the barrier above
        }
        __syncthreads();
        t = std::max(SINK_TAU_MIN, t * SINK_RATE);
    }
    for (int y = threadIdx.x; y < n; y += 64 * SINK_W) gpad[I.p_off + y] = gs[y];
}

// Row pass 2: u2(x) = min_y (z(x,y) - f10(y)).
__global__ __launch_bounds__(256) void k_feat_rows2(const NInst *inst,
                                                    const int32_t *rinst, Costs CV,
                                                    int32_t R,
                                                    const unsigned long long *abssum,
                                                    const float *F, float *u2) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= R) return;
    const int b = rinst[r];
    const NInst I = inst[b];
    const int x = r - I.row_off;
    const float inv = 1.0f / inst_scale(I, abssum, b);
    const bool s16 = CV.small(b);
    float mn = INFINITY;
    for (int y = lane; y < I.n; y += 64)
        mn = fminf(mn, float(CV.at(s16, I, x, y)) * inv - F[int64_t(I.row_off + y) * F_IN + 10]);
    for (int o = 32; o > 0; o >>= 1) mn = fminf(mn, __shfl_xor(mn, o, 64));
    if (lane == 0) u2[r] = mn;
}

// Column pass 2: v2(y) = min_x (z(x,y) - u2(x)).
__global__ __launch_bounds__(256) void k_feat_cols2(const NInst *inst,
                                                    const int32_t *rinst, Costs CV,
                                                    int32_t R,
                                                    const unsigned long long *abssum,
                                                    const float *u2, float *v2) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= R) return;
    const int b = rinst[r];
    const NInst I = inst[b];
    const int y = r - I.row_off, n = I.n;
    const float inv = 1.0f / inst_scale(I, abssum, b);
    const bool s16 = CV.small(b);
    float mn = INFINITY;
    for (int x0 = 0; x0 < n; x0 += FEAT_AHEAD) {
        int cb[FEAT_AHEAD];
        float ub[FEAT_AHEAD];
#pragma unroll
        for (int a = 0; a < FEAT_AHEAD; ++a) {
            const int x = x0 + a < n ? x0 + a : n - 1;  // a repeat is harmless for a min
            cb[a] = CV.at(s16, I, x, y);
            ub[a] = u2[I.row_off + x];
        }
#pragma unroll
        for (int a = 0; a < FEAT_AHEAD; ++a)
            mn = fminf(mn, float(cb[a]) * inv - ub[a]);
    }
    v2[r] = mn;
}

// Per instance: centre f13 and f14, set f15, and write the bf16 network
// input (row-major [Rp, 32] and, when XT is not null, transposed [32, Rp];
// zero padded).
__global__ __launch_bounds__(256) void k_feat_finish(const NInst *inst, int32_t Rp,
                                                     float *F, const float *gpad,
                                                     const float *v2, __bf16 *X,
                                                     __bf16 *XT) {
    const NInst I = inst[blockIdx.x];
    __shared__ float red[2][4];
    float a = 0.f, c = 0.f;
    for (int y = threadIdx.x; y < I.n; y += 256) {
        a += v2[I.row_off + y];
        c += gpad[I.p_off + y];
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    const float mv = (red[0][0] + red[0][1] + red[0][2] + red[0][3]) / I.n;
    const float ms = (red[1][0] + red[1][1] + red[1][2] + red[1][3]) / I.n;
    const float ln = logf(float(I.n)) / 6.0f;
    for (int y = threadIdx.x; y < I.n; y += 256) {
        const int r = I.row_off + y;
        float *f = F + int64_t(r) * F_IN;
        f[13] = v2[r] - mv;
        f[14] = gpad[I.p_off + y] - ms;
        f[15] = ln;
        for (int k = 0; k < F_PAD; ++k) {
            const __bf16 v = to_bf16(k < F_IN ? f[k] : 0.f);
            X[int64_t(r) * F_PAD + k] = v;
            if (XT) XT[int64_t(k) * Rp + r] = v;
        }
    }
}

// Prediction without a network (its correction taken as zero): q = f14, the
// centred Sinkhorn potential, with the mean taken as k_feat_finish takes it
// (the same value a network with a zero head adds to f14).
__global__ __launch_bounds__(256) void k_q_sinkhorn(const NInst *inst, const float *gpad,
                                                    float *q) {
    const NInst I = inst[blockIdx.x];
    __shared__ float red[4];
    float c = 0.f;
    for (int y = threadIdx.x; y < I.n; y += 256) c += gpad[I.p_off + y];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    const float ms = (red[0] + red[1] + red[2] + red[3]) / I.n;
    for (int y = threadIdx.x; y < I.n; y += 256) q[I.row_off + y] = gpad[I.p_off + y] - ms;
}

// ---------------------------------------------------------------------------
// NT GEMM on BF16 matrix cores: C[M,N] (=|+=) A[M,K] * Bt[N,K]^T, fp32 out.
// A and Bt row-major bf16 with leading dimensions lda, ldb; M a multiple of
// 16, N of 16 (<= 128), K of 32.  Block = 4 wavefronts, 64 rows; blockIdx.y
// splits K into gridDim.y chunks (ATOMIC accumulates the partial products).
// Fragments of v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)..+7],
// B[8(l/16)..+7][l%16], and D[4(l/16)+v][l%16].
// ---------------------------------------------------------------------------
template <int NT16, bool ATOMIC>
__global__ __launch_bounds__(256) void k_gemm_nt(const __bf16 *A, int lda,
                                                 const __bf16 *Bt, int ldb,
                                                 float *C, int ldc, int M, int K) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 64 + wave * 16;
    if (m0 >= M) return;  // wave-uniform: M is a multiple of 16
    const int kchunk = K / gridDim.y;
    const int kb = blockIdx.y * kchunk;
    const int ke = blockIdx.y + 1 == gridDim.y ? K : kb + kchunk;
    f32x4 acc[NT16];
#pragma unroll
    for (int t = 0; t < NT16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int ar = m0 + (lane & 15);
    const int kl = 8 * (lane >> 4);
    for (int k = kb; k < ke; k += 32) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(A + int64_t(ar) * lda + k + kl);
#pragma unroll
        for (int t = 0; t < NT16; ++t) {
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(
                Bt + int64_t(t * 16 + (lane & 15)) * ldb + k + kl);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT16; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float *dst = C + int64_t(m0 + 4 * (lane >> 4) + v) * ldc + t * 16 + (lane & 15);
            if (ATOMIC) atomicAdd(dst, acc[t][v]);
            else *dst = acc[t][v];
        }
    }
}

// ---------------------------------------------------------------------------
// Forward pieces
// ---------------------------------------------------------------------------
// P[b][j] = sum_k mean_cols(H)[b][k] U[k][j] + bias[j]; also keeps the means.
// 1024 threads = POOL_G groups of WID: group g sums the rows y = g (mod
// POOL_G) of column k = tid % WID (and the terms k = g (mod POOL_G) of the
// product), and the groups' partial sums meet in LDS.
constexpr int POOL_G = 8;
__global__ __launch_bounds__(POOL_G * WID) void k_pool_fwd(const NInst *inst,
                                                           const __bf16 *H, int ldh,
                                                           int Kin, const float *U,
                                                           const float *bias,
                                                           float *Mout, float *P) {
    const NInst I = inst[blockIdx.x];
    const int k = threadIdx.x % WID, g = threadIdx.x / WID;
    __shared__ float part[POOL_G][WID];
    __shared__ float m[WID];
    float s = 0.f;
    if (k < Kin) {
        const __bf16 *h = H + int64_t(I.row_off) * ldh + k;
        int y = g;
        // four rows in flight per thread
        for (; y + 3 * POOL_G < I.n; y += 4 * POOL_G) {
            const float a0 = from_bf16(h[int64_t(y) * ldh]);
            const float a1 = from_bf16(h[int64_t(y + POOL_G) * ldh]);
            const float a2 = from_bf16(h[int64_t(y + 2 * POOL_G) * ldh]);
            const float a3 = from_bf16(h[int64_t(y + 3 * POOL_G) * ldh]);
            s += (a0 + a1) + (a2 + a3);
        }
        for (; y < I.n; y += POOL_G) s += from_bf16(h[int64_t(y) * ldh]);
    }
    part[g][k] = s;
    __syncthreads();
    if (g == 0) {
        float t = 0.f;
        for (int i = 0; i < POOL_G; ++i) t += part[i][k];
        m[k] = k < Kin ? t / I.n : 0.f;
        if (k < Kin) Mout[int64_t(blockIdx.x) * WID + k] = m[k];
    }
    __syncthreads();
    const int j = k;
    float t = 0.f;
    for (int kk = g; kk < Kin; kk += POOL_G) t += m[kk] * U[kk * WID + j];
    part[g][j] = t;
    __syncthreads();
    if (g == 0) {
        float o = bias[j];
        for (int i = 0; i < POOL_G; ++i) o += part[i][j];
        P[int64_t(blockIdx.x) * WID + j] = o;
    }
}

// H = relu(Z + P[inst]) as bf16, row-major; when HT is not null (training)
// also transposed, with Z + P written back for the backward pass.  Padding
// rows are zero.  grid = Rp / 64 blocks of 256 threads: 64 rows x 128
// columns.
__global__ __launch_bounds__(256) void k_act_fwd(const int32_t *rinst, int32_t R,
                                                 int32_t Rp, float *Z, const float *P,
                                                 __bf16 *H, __bf16 *HT) {
    const int r0 = blockIdx.x * 64;
    for (int i = threadIdx.x; i < 64 * WID; i += 256) {
        const int r = r0 + i / WID, j = i % WID;
        float z = 0.f;
        if (r < R) z = Z[int64_t(r) * WID + j] + P[int64_t(rinst[r]) * WID + j];
        if (HT) Z[int64_t(r) * WID + j] = z;  // pre-activations for the backward pass
        const __bf16 h = to_bf16(z > 0.f ? z : 0.f);
        H[int64_t(r) * WID + j] = h;
        if (HT) HT[int64_t(j) * Rp + r] = h;
    }
}

// q = H_3 w_o + b_o + f14: the skip term (float32 feature, no parameter)
// carries the Sinkhorn potential to the prediction at full precision.
__global__ __launch_bounds__(256) void k_head(const __bf16 *H, int32_t R,
                                              const float *params, const float *F,
                                              float *q) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= R) return;
    float s = params[OFF_BO];
    for (int j = 0; j < WID; ++j) s += from_bf16(H[int64_t(r) * WID + j]) * params[OFF_WO + j];
    q[r] = s + F[int64_t(r) * F_IN + 14];
}

// Centred q -> integer scaled prices p = rint(q * sc * (2n+1)), and the
// starting epsilon kappa * sc * (2n+1) (at least 1) when eps0 is given.
__global__ __launch_bounds__(256) void k_prices(const NInst *inst,
                                                const unsigned long long *abssum,
                                                const float *q, int64_t *prices,
                                                float kappa, int64_t *eps0) {
    const int b = blockIdx.x;
    const NInst I = inst[b];
    __shared__ float red[4];
    float s = 0.f;
    for (int y = threadIdx.x; y < I.n; y += 256) s += q[I.row_off + y];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    const float mean = (red[0] + red[1] + red[2] + red[3]) / I.n;
    const double scale = double(inst_scale(I, abssum, b)) * double(2 * I.n + 1);
    if (prices)
        for (int y = threadIdx.x; y < I.n; y += 256)
            prices[I.row_off + y] = llrint(double(q[I.row_off + y] - mean) * scale);
    if (eps0 && threadIdx.x == 0) eps0[b] = max(1ll, llrint(double(kappa) * scale));
}

// ---------------------------------------------------------------------------
// Loss and backward pieces
// ---------------------------------------------------------------------------
// Per instance: t = (p - mean p) / (sc (2n+1)); r = (q - mean q) - t;
// loss += sum r^2 / Ntot; dq = 2 r / Ntot.
__global__ __launch_bounds__(256) void k_loss(const NInst *inst,
                                              const unsigned long long *abssum,
                                              const float *q, const int64_t *tp,
                                              float inv_ntot, float *dq, float *loss) {
    const int b = blockIdx.x;
    const NInst I = inst[b];
    __shared__ double red[2][4];
    double sq = 0, st = 0;
    for (int y = threadIdx.x; y < I.n; y += 256) {
        sq += q[I.row_off + y];
        st += double(tp[I.row_off + y]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        sq += __shfl_xor(sq, o, 64);
        st += __shfl_xor(st, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sq;
        red[1][threadIdx.x >> 6] = st;
    }
    __syncthreads();
    const double mq = (red[0][0] + red[0][1] + red[0][2] + red[0][3]) / I.n;
    const double mt = (red[1][0] + red[1][1] + red[1][2] + red[1][3]) / I.n;
    const double scale = double(inst_scale(I, abssum, b)) * double(2 * I.n + 1);
    float part = 0.f;
    for (int y = threadIdx.x; y < I.n; y += 256) {
        const int r = I.row_off + y;
        const float res = float((double(q[r]) - mq) - (double(tp[r]) - mt) / scale);
        dq[r] = 2.f * res * inv_ntot;
        part += res * res * inv_ntot;
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[0][threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicAdd(loss, float(red[0][0] + red[0][1] + red[0][2] + red[0][3]));
}

// Head backward: dH3 = dq w_o^T (fp32), grad w_o += H3^T dq, grad b_o += sum dq.
__global__ __launch_bounds__(256) void k_head_bwd(const __bf16 *H, int32_t R, int32_t Rp,
                                                  const float *params, const float *dq,
                                                  float *dH, float *grad) {
    const int r0 = blockIdx.x * 64;
    __shared__ float gw[WID];
    __shared__ float gb;
    if (threadIdx.x < WID) gw[threadIdx.x] = 0.f;
    if (threadIdx.x == 0) gb = 0.f;
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * WID; i += 256) {
        const int r = r0 + i / WID, j = i % WID;
        const float d = r < R ? dq[r] : 0.f;
        dH[int64_t(r) * WID + j] = d * params[OFF_WO + j];
        if (d != 0.f) atomicAdd(&gw[j], d * from_bf16(H[int64_t(r) * WID + j]));
        if (j == 0 && d != 0.f) atomicAdd(&gb, d);
    }
    __syncthreads();
    if (threadIdx.x < WID && gw[threadIdx.x] != 0.f)
        atomicAdd(&grad[OFF_WO + threadIdx.x], gw[threadIdx.x]);
    if (threadIdx.x == 0 && gb != 0.f) atomicAdd(&grad[OFF_BO], gb);
}

// dZ = (dH + G[inst]) * (Z > 0), stored as bf16 row-major and transposed,
// with per-instance column sums of dZ (fp32) for the pooled and bias terms.
// G (may be null) is the pooled part of dH coming from the layer above.
// grid = Rp / 64.
__global__ __launch_bounds__(256) void k_act_bwd(const int32_t *rinst, int32_t R,
                                                 int32_t Rp, const float *dH,
                                                 const float *G, const float *Z,
                                                 __bf16 *dZ, __bf16 *dZT, float *dZsum) {
    const int r0 = blockIdx.x * 64;
    for (int i = threadIdx.x; i < 64 * WID; i += 256) {
        const int r = r0 + i / WID, j = i % WID;
        float d = 0.f;
        if (r < R) {
            d = dH[int64_t(r) * WID + j];
            if (G) d += G[int64_t(rinst[r]) * WID + j];
            if (!(Z[int64_t(r) * WID + j] > 0.f)) d = 0.f;
            if (d != 0.f) atomicAdd(&dZsum[int64_t(rinst[r]) * WID + j], d);
        }
        const __bf16 h = to_bf16(d);
        dZ[int64_t(r) * WID + j] = h;
        dZT[int64_t(j) * Rp + r] = h;
    }
}

// grad U[k][j] += sum_b M[b][k] dZsum[b][j]; grad b[j] += sum_b dZsum[b][j];
// G[b][k] = (1/n_b) sum_j dZsum[b][j] U[k][j] (pooled part of dH_{l-1}).
__global__ __launch_bounds__(128) void k_pool_bwd(const NInst *inst, int32_t B, int Kin,
                                                  const float *M, const float *dZsum,
                                                  const float *U, float *gU, float *gb,
                                                  float *G) {
    const int j = threadIdx.x;
    if (blockIdx.x == 0) {
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += dZsum[int64_t(b) * WID + j];
        atomicAdd(&gb[j], s);
    }
    for (int k = blockIdx.x; k < Kin; k += gridDim.x) {
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += M[int64_t(b) * WID + k] * dZsum[int64_t(b) * WID + j];
        atomicAdd(&gU[k * WID + j], s);
    }
    if (G) {
        for (int b = blockIdx.x; b < B; b += gridDim.x) {
            __shared__ float ds[WID];
            __syncthreads();
            ds[j] = dZsum[int64_t(b) * WID + j];
            __syncthreads();
            for (int k = j; k < Kin; k += 128) {
                float s = 0.f;
                for (int jj = 0; jj < WID; ++jj) s += ds[jj] * U[k * WID + jj];
                G[int64_t(b) * WID + k] = s / inst[b].n;
            }
        }
    }
}

// Copies the first Kin rows of an fp32 [Kpad,128] accumulator into grad.
__global__ void k_add_rows(const float *acc, int Kin, float *dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < Kin * WID) dst[i] += acc[i];
}

// Adam (bias-corrected), fp32 master weights.
__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 copies of the weights: WT_l [128][KPAD] (forward operand) and
// Wb_l [KPAD][128] (operand of dH = dZ W^T).
__global__ __launch_bounds__(256) void k_weights(const float *params, __bf16 *WT0,
                                                 __bf16 *WT1, __bf16 *WT2,
                                                 __bf16 *Wb1, __bf16 *Wb2) {
    __bf16 *WT[3] = {WT0, WT1, WT2};
    for (int l = 0; l < 3; ++l) {
        const float *W = params + OFF_W[l];
        for (int i = blockIdx.x * 256 + threadIdx.x; i < WID * KPAD[l]; i += gridDim.x * 256) {
            const int j = i / KPAD[l], k = i % KPAD[l];
            WT[l][i] = to_bf16(k < KIN[l] ? W[k * WID + j] : 0.f);
        }
    }
    for (int i = blockIdx.x * 256 + threadIdx.x; i < WID * WID; i += gridDim.x * 256) {
        Wb1[i] = to_bf16(params[OFF_W[1] + i]);
        Wb2[i] = to_bf16(params[OFF_W[2] + i]);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct Layout {
    NInst *inst;
    int32_t *rinst, *rowmin;
    unsigned long long *abssum;
    unsigned *cmax;   // per instance max |c|
    int16_t *c16;     // saturated int16 copy of sign * c, rows padded to ld16(n)
    int32_t *sids;    // instances of the Sinkhorn launches, grouped by row length
    float *gpad;      // Sinkhorn column potentials, ld16(n) entries per instance
    float *F, *u2, *v2;
    __bf16 *X0, *X0T;
    float *Z[3];
    __bf16 *H[3], *HT[3];
    float *M[3], *P[3];
    float *q, *dq, *dH, *G, *dZsum, *acc, *grad, *loss;
    __bf16 *dZ, *dZT;
    __bf16 *WT[3], *Wb[3];
};

static int64_t pad64(int64_t r) { return (r + 63) / 64 * 64; }

// Sizes of a batch: R stacked columns, P padded potentials (sum of
// ld16(n)), E16 entries of the padded int16 copy.
struct Sizes {
    int64_t R = 0, P = 0, E16 = 0;
};

static Sizes sizes(int B, const int32_t *n) {
    Sizes z;
    for (int b = 0; b < B; ++b) {
        z.R += n[b];
        z.P += ld16(n[b]);
        z.E16 += int64_t(n[b]) * ld16(n[b]);
    }
    return z;
}

static Carver carve(Carver cv, int B, const Sizes &z, Layout *L) {
    const int64_t R = z.R, Rp = pad64(R);
    L->inst = cv.take<NInst>(B);
    L->rinst = cv.take<int32_t>(R);
    L->rowmin = cv.take<int32_t>(R);
    L->abssum = cv.take<unsigned long long>(B);
    L->cmax = cv.take<unsigned>(B);
    L->c16 = cv.take<int16_t>(z.E16);
    L->sids = cv.take<int32_t>(B);
    L->gpad = cv.take<float>(z.P);
    L->F = cv.take<float>(R * F_IN);
    L->u2 = cv.take<float>(R);
    L->v2 = cv.take<float>(R);
    L->X0 = cv.take<__bf16>(Rp * F_PAD);
    L->X0T = cv.take<__bf16>(Rp * F_PAD);
    for (int l = 0; l < 3; ++l) {
        L->Z[l] = cv.take<float>(Rp * WID);
        L->H[l] = cv.take<__bf16>(Rp * WID);
        L->HT[l] = cv.take<__bf16>(Rp * WID);
        L->M[l] = cv.take<float>(int64_t(B) * WID);
        L->P[l] = cv.take<float>(int64_t(B) * WID);
        L->WT[l] = cv.take<__bf16>(WID * KPAD[l]);
        L->Wb[l] = cv.take<__bf16>(WID * WID);
    }
    L->q = cv.take<float>(R);
    L->dq = cv.take<float>(R);
    L->dH = cv.take<float>(Rp * WID);
    L->G = cv.take<float>(int64_t(B) * WID);
    L->dZsum = cv.take<float>(int64_t(B) * WID);
    L->acc = cv.take<float>(WID * WID);
    L->grad = cv.take<float>(N_PARAMS);
    L->loss = cv.take<float>(1);
    L->dZ = cv.take<__bf16>(Rp * WID);
    L->dZT = cv.take<__bf16>(Rp * WID);
    return cv;
}

static size_t workspace_bytes(int B, const int32_t *n) {
    Layout L;
    return carve(Carver(), B, sizes(B, n), &L).used();
}

struct Ctx {
    int B;
    int64_t R, Rp;
    Layout L;
    hipStream_t s;
    std::vector<NInst> insts;
    std::vector<int32_t> rinst, sids;
    int sclass[3] = {0, 0, 0};  // Sinkhorn instances per row-length class
};

// `rows`: also the per-column instance index the feature passes and the
// network read (a prediction without the network needs none of it).
static lpr_status prepare(Ctx &C, int32_t B, const int32_t *n,
                          const int64_t *cost_offset, const int32_t *costs,
                          void *ws, size_t ws_bytes, void *stream, bool rows = true) {
    clear_error();
    if (B < 1 || !n || !cost_offset || !costs || !ws) {
        set_error("invalid arguments (NULL pointer or B < 1)");
        return LPR_EINVAL;
    }
    if (cost_offset[0] != 0) {
        set_error("cost_offset[0] must be 0");
        return LPR_EINVAL;
    }
    C.B = B;
    C.insts.resize(B);
    int64_t R = 0, P = 0, E16 = 0;
    for (int b = 0; b < B; ++b) {
        if (n[b] < 1 || n[b] > LPR_ASSIGN_MAX_N) {
            set_error("instance %d: n = %d outside [1, %d]", b, n[b], LPR_ASSIGN_MAX_N);
            return LPR_EINVAL;
        }
        if (cost_offset[b + 1] != cost_offset[b] + int64_t(n[b]) * n[b]) {
            set_error("cost_offset is not the prefix sum of n^2 at %d", b);
            return LPR_EINVAL;
        }
        C.insts[b] = NInst{cost_offset[b], E16, n[b], ld16(n[b]), int32_t(R), int32_t(P)};
        R += n[b];
        P += ld16(n[b]);
        E16 += int64_t(n[b]) * ld16(n[b]);
    }
    if (R >= (int64_t(1) << 28)) {
        set_error("too many columns");
        return LPR_EINVAL;
    }
    C.R = R;
    C.Rp = pad64(R);
    const size_t need = workspace_bytes(B, n);
    if (ws_bytes < need) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
        return LPR_ENOMEM;
    }
    carve(Carver(ws, ws_bytes), B, sizes(B, n), &C.L);
    C.rinst.resize(rows ? R : 0);
    if (rows)
        for (int b = 0; b < B; ++b)
            std::fill(C.rinst.begin() + C.insts[b].row_off,
                      C.rinst.begin() + C.insts[b].row_off + n[b], b);
    C.s = static_cast<hipStream_t>(stream);
    LPR_TRY_HIP(hipMemcpyAsync(C.L.inst, C.insts.data(), sizeof(NInst) * B,
                               hipMemcpyHostToDevice, C.s));
    if (rows)
        LPR_TRY_HIP(hipMemcpyAsync(C.L.rinst, C.rinst.data(), sizeof(int32_t) * R,
                                   hipMemcpyHostToDevice, C.s));
    // Sinkhorn launches: instances with rows up to 512, 1024, 2048 entries,
    // the largest first in each
    C.sids.clear();
    for (int cls = 0; cls < 3; ++cls) {
        const int lo = cls == 0 ? 0 : 256 << cls, hi = 512 << cls;
        std::vector<int32_t> ids;
        for (int b = 0; b < B; ++b)
            if (n[b] > lo && n[b] <= hi) ids.push_back(b);
        std::stable_sort(ids.begin(), ids.end(),
                         [&](int32_t a, int32_t c) { return n[a] > n[c]; });
        C.sclass[cls] = int(ids.size());
        C.sids.insert(C.sids.end(), ids.begin(), ids.end());
    }
    LPR_TRY_HIP(hipMemcpyAsync(C.L.sids, C.sids.data(), sizeof(int32_t) * B,
                               hipMemcpyHostToDevice, C.s));
    return LPR_OK;
}

// Row pass 1 (row minima, scales, the int16 copy) and the Sinkhorn
// potentials into gpad: what every prediction needs.  `net`: also the
// network's other features and its bf16 input (`train`: transposed too).
static lpr_status run_features(Ctx &C, const int32_t *costs, int32_t sign, bool train,
                               bool net = true) {
    Layout &L = C.L;
    const int R = int(C.R);
    LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(L.abssum), 0, C.B, C.s));
    LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(L.cmax), 0, C.B, C.s));
    const Costs CV{costs, L.c16, L.cmax, sign};
    int nmax = 0;
    for (const NInst &I : C.insts) nmax = std::max(nmax, int(I.n));
    hipLaunchKernelGGL(k_feat_rows1, dim3(ceil_div(nmax, ROWS1), C.B), dim3(256), 0, C.s,
                       L.inst, costs, sign, L.rowmin, L.abssum, L.c16, L.cmax);
    // f14: annealed Sinkhorn potentials, one workgroup per instance
    {
        const int32_t *ids = L.sids;
        for (int cls = 0; cls < 3; ++cls) {
            const int cnt = C.sclass[cls];
            if (!cnt) continue;
            const size_t lds = sizeof(float) * (SINK_W + 2) * (512 << cls);
            const void *fn = cls == 0   ? reinterpret_cast<const void *>(k_sinkhorn<1, 4>)
                             : cls == 1 ? reinterpret_cast<const void *>(k_sinkhorn<2, 2>)
                                        : reinterpret_cast<const void *>(k_sinkhorn<4, 1>);
            LPR_TRY_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            int(lds)));
            if (cls == 0)
                hipLaunchKernelGGL((k_sinkhorn<1, 4>), dim3(cnt), dim3(64 * SINK_W), lds, C.s,
                                   L.inst, ids, CV, L.abssum, L.gpad);
            else if (cls == 1)
                hipLaunchKernelGGL((k_sinkhorn<2, 2>), dim3(cnt), dim3(64 * SINK_W), lds, C.s,
                                   L.inst, ids, CV, L.abssum, L.gpad);
            else
                hipLaunchKernelGGL((k_sinkhorn<4, 1>), dim3(cnt), dim3(64 * SINK_W), lds, C.s,
                                   L.inst, ids, CV, L.abssum, L.gpad);
            ids += cnt;
        }
    }
    if (!net) {
        LPR_TRY_HIP(hipGetLastError());
        return LPR_OK;
    }
    // padding rows of the bf16 input are zero
    LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(L.X0), 0, C.Rp * F_PAD / 2, C.s));
    if (train) LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(L.X0T), 0, C.Rp * F_PAD / 2, C.s));
    hipLaunchKernelGGL(k_feat_cols1, dim3(ceil_div(R, 256)), dim3(256), 0, C.s,
                       L.inst, L.rinst, CV, R, L.rowmin, L.abssum, L.F);
    hipLaunchKernelGGL(k_feat_rows2, dim3(ceil_div(R, 4)), dim3(256), 0, C.s,
                       L.inst, L.rinst, CV, R, L.abssum, L.F, L.u2);
    hipLaunchKernelGGL(k_feat_cols2, dim3(ceil_div(R, 256)), dim3(256), 0, C.s,
                       L.inst, L.rinst, CV, R, L.abssum, L.u2, L.v2);
    hipLaunchKernelGGL(k_feat_finish, dim3(C.B), dim3(256), 0, C.s, L.inst,
                       int32_t(C.Rp), L.F, L.gpad, L.v2, L.X0, train ? L.X0T : nullptr);
    LPR_TRY_HIP(hipGetLastError());
    return LPR_OK;
}

static void gemm(hipStream_t s, const __bf16 *A, int lda, const __bf16 *Bt, int ldb,
                 float *Cm, int ldc, int M, int N, int K, int splits, bool atomic) {
    const dim3 grid((M + 63) / 64, splits);
    if (N == 128) {
        if (atomic) hipLaunchKernelGGL((k_gemm_nt<8, true>), grid, dim3(256), 0, s, A, lda, Bt, ldb, Cm, ldc, M, K);
        else hipLaunchKernelGGL((k_gemm_nt<8, false>), grid, dim3(256), 0, s, A, lda, Bt, ldb, Cm, ldc, M, K);
    } else {  // N == 32
        if (atomic) hipLaunchKernelGGL((k_gemm_nt<2, true>), grid, dim3(256), 0, s, A, lda, Bt, ldb, Cm, ldc, M, K);
        else hipLaunchKernelGGL((k_gemm_nt<2, false>), grid, dim3(256), 0, s, A, lda, Bt, ldb, Cm, ldc, M, K);
    }
}

// train: also keep the transposed activations the backward pass reads
static lpr_status run_forward(Ctx &C, const float *params, bool train) {
    Layout &L = C.L;
    const int R = int(C.R), Rp = int(C.Rp);
    hipLaunchKernelGGL(k_weights, dim3(16), dim3(256), 0, C.s, params, L.WT[0],
                       L.WT[1], L.WT[2], L.Wb[1], L.Wb[2]);
    const __bf16 *Hin = L.X0;
    int ldin = F_PAD;
    for (int l = 0; l < 3; ++l) {
        hipLaunchKernelGGL(k_pool_fwd, dim3(C.B), dim3(POOL_G * WID), 0, C.s, L.inst, Hin, ldin,
                           KIN[l], params + OFF_U[l], params + OFF_B[l], L.M[l], L.P[l]);
        gemm(C.s, Hin, ldin, L.WT[l], KPAD[l], L.Z[l], WID, Rp, WID, KPAD[l], 1, false);
        hipLaunchKernelGGL(k_act_fwd, dim3(Rp / 64), dim3(256), 0, C.s, L.rinst, R, Rp,
                           L.Z[l], L.P[l], L.H[l], train ? L.HT[l] : nullptr);
        Hin = L.H[l];
        ldin = WID;
    }
    hipLaunchKernelGGL(k_head, dim3(ceil_div(R, 256)), dim3(256), 0, C.s, L.H[2], R,
                       params, L.F, L.q);
    LPR_TRY_HIP(hipGetLastError());
    return LPR_OK;
}

static lpr_status run_backward(Ctx &C, const float *params, const int64_t *targets) {
    Layout &L = C.L;
    const int R = int(C.R), Rp = int(C.Rp);
    LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(L.grad), 0, N_PARAMS, C.s));
    LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(L.loss), 0, 1, C.s));
    hipLaunchKernelGGL(k_loss, dim3(C.B), dim3(256), 0, C.s, L.inst, L.abssum, L.q,
                       targets, 1.0f / float(R), L.dq, L.loss);
    hipLaunchKernelGGL(k_head_bwd, dim3(Rp / 64), dim3(256), 0, C.s, L.H[2], R, Rp,
                       params, L.dq, L.dH, L.grad);
    const int splits = std::max(1, std::min(Rp / 512, 128));
    for (int l = 2; l >= 0; --l) {
        LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(L.dZsum), 0, int64_t(C.B) * WID, C.s));
        hipLaunchKernelGGL(k_act_bwd, dim3(Rp / 64), dim3(256), 0, C.s, L.rinst, R, Rp,
                           L.dH, l < 2 ? L.G : nullptr, L.Z[l], L.dZ, L.dZT, L.dZsum);
        // dW_l = H_{l-1}^T dZ (split over rows, accumulated in fp32)
        const __bf16 *HinT = l == 0 ? L.X0T : L.HT[l - 1];
        LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(L.acc), 0, WID * WID, C.s));
        // keep every split a multiple of 32 rows
        int sp = splits;
        while (sp > 1 && (Rp / sp) % 32) --sp;
        gemm(C.s, HinT, Rp, L.dZT, Rp, L.acc, WID, KPAD[l], WID, Rp, sp, true);
        hipLaunchKernelGGL(k_add_rows, dim3(ceil_div(KIN[l] * WID, 256)), dim3(256), 0,
                           C.s, L.acc, KIN[l], L.grad + OFF_W[l]);
        hipLaunchKernelGGL(k_pool_bwd, dim3(std::min(C.B, 64)), dim3(128), 0, C.s,
                           L.inst, C.B, KIN[l], L.M[l], L.dZsum, params + OFF_U[l],
                           L.grad + OFF_U[l], L.grad + OFF_B[l], l > 0 ? L.G : nullptr);
        if (l > 0)  // dH_{l-1} = dZ W_l^T (the pooled part is G)
            gemm(C.s, L.dZ, WID, L.Wb[l], WID, L.dH, WID, Rp, WID, WID, 1, false);
    }
    LPR_TRY_HIP(hipGetLastError());
    return LPR_OK;
}

}  // namespace net
}  // namespace lpr

using namespace lpr;

extern "C" size_t lpr_pricenet_param_count(void) { return size_t(net::N_PARAMS); }

extern "C" size_t lpr_pricenet_workspace(int32_t B, const int32_t *n) {
    if (B < 1 || !n) return 0;
    for (int b = 0; b < B; ++b)
        if (n[b] < 1) return 0;
    return net::workspace_bytes(B, n);
}

extern "C" lpr_status lpr_pricenet_features(int32_t B, const int32_t *n,
                                            const int64_t *cost_offset,
                                            const int32_t *costs, int32_t maximize,
                                            float *feats, float *scales,
                                            void *workspace, size_t workspace_bytes,
                                            void *stream) {
    net::Ctx C;
    LPR_TRY(net::prepare(C, B, n, cost_offset, costs, workspace, workspace_bytes, stream));
    LPR_TRY(net::run_features(C, costs, maximize ? -1 : 1, false));
    if (feats)
        LPR_TRY_HIP(hipMemcpyAsync(feats, C.L.F, sizeof(float) * C.R * net::F_IN,
                                   hipMemcpyDeviceToDevice, C.s));
    std::vector<unsigned long long> as(B);
    LPR_TRY_HIP(hipMemcpyAsync(as.data(), C.L.abssum, sizeof(unsigned long long) * B,
                               hipMemcpyDeviceToHost, C.s));
    LPR_TRY_HIP(hipStreamSynchronize(C.s));
    if (scales) {
        std::vector<float> sc(B);
        for (int b = 0; b < B; ++b) {
            const double m = double(as[b]) / (double(n[b]) * double(n[b]));
            sc[b] = m > 0 ? float(m) : 1.0f;
        }
        LPR_TRY_HIP(hipMemcpy(scales, sc.data(), sizeof(float) * B, hipMemcpyHostToDevice));
    }
    return LPR_OK;
}

extern "C" lpr_status lpr_pricenet_infer(int32_t B, const int32_t *n,
                                         const int64_t *cost_offset,
                                         const int32_t *costs, int32_t maximize,
                                         const float *params, float kappa,
                                         float *q, int64_t *col_prices,
                                         int64_t *eps0, void *workspace,
                                         size_t workspace_bytes, void *stream) {
    if (eps0 && !(kappa > 0.f)) {
        clear_error();
        set_error("eps0 requested with kappa <= 0");
        return LPR_EINVAL;
    }
    net::Ctx C;
    LPR_TRY(net::prepare(C, B, n, cost_offset, costs, workspace, workspace_bytes, stream,
                         params != nullptr));
    LPR_TRY(net::run_features(C, costs, maximize ? -1 : 1, false, params != nullptr));
    if (params) {
        LPR_TRY(net::run_forward(C, params, false));
    } else {
        hipLaunchKernelGGL(net::k_q_sinkhorn, dim3(B), dim3(256), 0, C.s, C.L.inst, C.L.gpad,
                           C.L.q);
        LPR_TRY_HIP(hipGetLastError());
    }
    if (col_prices || eps0) {
        hipLaunchKernelGGL(net::k_prices, dim3(B), dim3(256), 0, C.s, C.L.inst,
                           C.L.abssum, C.L.q, col_prices, kappa, eps0);
        LPR_TRY_HIP(hipGetLastError());
    }
    if (q)
        LPR_TRY_HIP(hipMemcpyAsync(q, C.L.q, sizeof(float) * C.R,
                                   hipMemcpyDeviceToDevice, C.s));
    LPR_TRY_HIP(hipStreamSynchronize(C.s));
    return LPR_OK;
}

// Learned start and solve in one call: the workspace holds the network's
// workspace, the start prices and starting epsilons, and the solve's
// workspace, each 256-B aligned.
static size_t learned_layout(int32_t B, const int32_t *n, void *ws, size_t ws_bytes,
                             void **net_ws, size_t *net_bytes, int64_t **prices,
                             int64_t **eps0, void **solve_ws, size_t *solve_bytes) {
    int64_t R = 0;
    for (int b = 0; b < B; ++b) R += n[b];
    *net_bytes = net::workspace_bytes(B, n);
    *solve_bytes = lpr_assign_batched_workspace(B, n);
    Carver cv(ws, ws_bytes);
    *net_ws = cv.take<uint8_t>(*net_bytes);
    *prices = cv.take<int64_t>(size_t(R));
    *eps0 = cv.take<int64_t>(size_t(B));
    *solve_ws = cv.take<uint8_t>(*solve_bytes);
    return cv.used();
}

extern "C" size_t lpr_assign_learned_workspace(int32_t B, const int32_t *n) {
    if (B < 1 || !n) return 0;
    for (int b = 0; b < B; ++b)
        if (n[b] < 1 || n[b] > LPR_ASSIGN_MAX_N) return 0;
    void *a, *c;
    int64_t *p, *e;
    size_t na, nc;
    return learned_layout(B, n, nullptr, 0, &a, &na, &p, &e, &c, &nc);
}

extern "C" lpr_status lpr_assign_solve_learned(
    int32_t B, const int32_t *n, const int64_t *cost_offset, const int32_t *costs,
    int32_t maximize, const float *params, float kappa, int32_t *row_to_col,
    int64_t *totals, int64_t *col_prices, const lpr_assign_opts *opts,
    lpr_assign_stats *stats, void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (B < 1 || !n || !workspace) {
        set_error("invalid arguments (NULL pointer or B < 1)");
        return LPR_EINVAL;
    }
    if (!(kappa > 0.f)) {
        set_error("kappa must be > 0");
        return LPR_EINVAL;
    }
    if (opts && (opts->init_col_prices || opts->eps0 || opts->eps0_per_instance)) {
        set_error("the start prices and epsilons are the call's own (opts must leave "
                  "init_col_prices, eps0 and eps0_per_instance unset)");
        return LPR_EINVAL;
    }
    const size_t need = lpr_assign_learned_workspace(B, n);
    if (need == 0) {
        set_error("invalid instance sizes");
        return LPR_EINVAL;
    }
    if (workspace_bytes < need) {
        set_error("workspace too small: %zu < %zu bytes", workspace_bytes, need);
        return LPR_ENOMEM;
    }
    void *net_ws, *solve_ws;
    size_t net_bytes, solve_bytes;
    int64_t *prices, *eps0;
    learned_layout(B, n, workspace, workspace_bytes, &net_ws, &net_bytes, &prices, &eps0,
                   &solve_ws, &solve_bytes);
    hipStream_t side;
    hipEvent_t ev_fork, ev_join;
    LPR_TRY(side_stream(&side, &ev_fork, &ev_join));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // everything the caller enqueued before is visible to the side stream
    LPR_TRY_HIP(hipEventRecord(ev_fork, s));
    // the prediction on `s` (C, and the host tables its copies read, stay
    // alive until the solve below has synchronised the stream)
    net::Ctx C;
    LPR_TRY(net::prepare(C, B, n, cost_offset, costs, net_ws, net_bytes, stream,
                         params != nullptr));
    LPR_TRY(net::run_features(C, costs, maximize ? -1 : 1, false, params != nullptr));
    if (params) {
        LPR_TRY(net::run_forward(C, params, false));
    } else {
        hipLaunchKernelGGL(net::k_q_sinkhorn, dim3(B), dim3(256), 0, C.s, C.L.inst, C.L.gpad,
                           C.L.q);
        LPR_TRY_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(net::k_prices, dim3(B), dim3(256), 0, C.s, C.L.inst, C.L.abssum,
                       C.L.q, prices, kappa, eps0);
    LPR_TRY_HIP(hipGetLastError());
    // the solve: its cost copies run on the side stream beside the
    // prediction, the solve kernel after both
    lpr_assign_opts o{};
    if (opts) o = *opts;
    o.init_col_prices = prices;
    o.eps0_per_instance = eps0;
    const lpr_status rc = assign::run_forked(B, n, cost_offset, costs, maximize, row_to_col,
                                             totals, col_prices, &o, stats, solve_ws,
                                             solve_bytes, stream, side, ev_fork, ev_join);
    if (rc != LPR_OK) {
        // a solve that stopped early (options rejected, say) may leave the
        // prediction in flight: it reads C's host tables and writes the
        // caller's workspace, so it has to end before either goes away
        (void)hipStreamSynchronize(s);
        (void)hipStreamSynchronize(side);
    }
    return rc;
}

extern "C" lpr_status lpr_pricenet_train_step(int32_t B, const int32_t *n,
                                              const int64_t *cost_offset,
                                              const int32_t *costs, int32_t maximize,
                                              const int64_t *target_prices,
                                              float *params, float *grad_out,
                                              float *adam_m, float *adam_v,
                                              int32_t step, float lr, float *loss_out,
                                              void *workspace, size_t workspace_bytes,
                                              void *stream) {
    if (!params || !target_prices || step < 0 || (step > 0 && (!adam_m || !adam_v))) {
        clear_error();
        set_error("invalid training arguments");
        return LPR_EINVAL;
    }
    net::Ctx C;
    LPR_TRY(net::prepare(C, B, n, cost_offset, costs, workspace, workspace_bytes, stream));
    LPR_TRY(net::run_features(C, costs, maximize ? -1 : 1, true));
    LPR_TRY(net::run_forward(C, params, true));
    LPR_TRY(net::run_backward(C, params, target_prices));
    if (grad_out)
        LPR_TRY_HIP(hipMemcpyAsync(grad_out, C.L.grad, sizeof(float) * net::N_PARAMS,
                                   hipMemcpyDeviceToDevice, C.s));
    if (loss_out)
        LPR_TRY_HIP(hipMemcpyAsync(loss_out, C.L.loss, sizeof(float),
                                   hipMemcpyDeviceToDevice, C.s));
    if (step > 0) {
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - std::pow(b1, float(step));
        const float c2 = 1.f - std::pow(b2, float(step));
        hipLaunchKernelGGL(net::k_adam, dim3(ceil_div(net::N_PARAMS, 256)), dim3(256), 0,
                           C.s, params, C.L.grad, adam_m, adam_v, net::N_PARAMS, lr, b1,
                           b2, 1e-8f, c1, c2);
        LPR_TRY_HIP(hipGetLastError());
    }
    LPR_TRY_HIP(hipStreamSynchronize(C.s));
    return LPR_OK;
}
