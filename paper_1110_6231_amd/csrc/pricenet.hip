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
    int64_t cost_off;
    int32_t n;
    int32_t row_off;  // first stacked row (column) of the instance
};

__device__ inline __bf16 to_bf16(float f) { return (__bf16)f; }
__device__ inline float from_bf16(__bf16 b) { return (float)b; }

// ---------------------------------------------------------------------------
// Feature passes
// ---------------------------------------------------------------------------
// Row pass 1: min_y c(x,y), the instance's sum and maximum of |c|, and a
// saturated int16 copy of sign * c that the later passes read instead of the
// int32 input when the instance's costs fit (half the bytes per pass).
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
        const int64_t base = I.cost_off + int64_t(x) * I.n;
        const int32_t *row = costs + base;
        int mn = INT_MAX;
        for (int y = lane; y < I.n; y += 64) {
            const int c = sign * row[y];
            mn = min(mn, c);
            const unsigned a = unsigned(c < 0 ? -c : c);
            s += a;
            amax = max(amax, a);
            c16[base + y] = int16_t(max(-C16_MAX, min(C16_MAX, c)));
        }
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

// sign * c at entry idx of the packed costs: from the int16 copy when the
// instance's |c| fits it, else from the int32 input
struct Costs {
    const int32_t *c32;
    const int16_t *c16;
    const unsigned *cmax;
    int32_t sign;
    __device__ bool small(int b) const { return cmax[b] <= unsigned(C16_MAX); }
    __device__ int at(bool s16, int64_t idx) const {
        return s16 ? int(c16[idx]) : sign * c32[idx];
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
    const int64_t col = I.cost_off + y;
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
            cb[a] = CV.at(s16, col + int64_t(x) * n);
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

// Sinkhorn passes of f14.  A log-sum-exp of -v/tau over values v is m -
// tau log s with m = min v and s = sum exp(-(v - m)/tau): every exponent is
// <= 0 and the minimum's term is 1, so nothing overflows however small tau
// is.  The row pass takes the minimum first and then the sum over the same
// entries (a row is short and its second read hits the cache), so neither
// loop carries a dependence beyond its accumulators; the column pass, whose
// second read would come from further away, carries the pair (m, s) along
// instead, rescaled once per group of rows ((inf, 0) is the empty pair).
constexpr float LOG2E = 1.4426950408889634f;

__device__ inline void lse_merge(float &m, float &s, float m2, float s2, float k) {
    if (s2 == 0.f) return;
    if (s == 0.f) {
        m = m2;
        s = s2;
        return;
    }
    const float d = m2 - m;
    const float e = __expf(-fabsf(d) * k);
    if (d < 0.f) {
        s = fmaf(s, e, s2);
        m = m2;
    } else {
        s = fmaf(s2, e, s);
    }
}

// Row update f(x) = -tau log sum_y exp(-(z(x,y) - g(y))/tau): SINK_RL lanes
// per stacked row (64 / SINK_RL rows per wavefront), the row's columns
// strided over them, reduced inside each lane group by butterfly shuffles.
constexpr int SINK_RL = 16;
__global__ __launch_bounds__(256) void k_sink_rows(const NInst *inst, const int32_t *rinst,
                                                   Costs CV, int32_t R,
                                                   const unsigned long long *abssum,
                                                   const float *g, float *f, float tau) {
    const int l = threadIdx.x & (SINK_RL - 1);
    const int r = blockIdx.x * (256 / SINK_RL) + threadIdx.x / SINK_RL;
    const bool live = r < R;
    int n = 0;
    int64_t row = 0;
    float inv = 1.f;
    bool s16 = true;
    const float *gi = g;
    if (live) {
        const int b = rinst[r];
        const NInst I = inst[b];
        n = I.n;
        inv = 1.0f / inst_scale(I, abssum, b);
        s16 = CV.small(b);
        row = I.cost_off + int64_t(r - I.row_off) * n;
        gi = g + I.row_off;
    }
    auto v = [&](int y) { return float(CV.at(s16, row + y)) * inv - gi[y]; };
    constexpr int U = 4 * SINK_RL;
    float m0 = INFINITY, m1 = INFINITY, m2 = INFINITY, m3 = INFINITY;
    int y = l;
    for (; y + 3 * SINK_RL < n; y += U) {
        m0 = fminf(m0, v(y));
        m1 = fminf(m1, v(y + SINK_RL));
        m2 = fminf(m2, v(y + 2 * SINK_RL));
        m3 = fminf(m3, v(y + 3 * SINK_RL));
    }
    for (; y < n; y += SINK_RL) m0 = fminf(m0, v(y));
    float m = fminf(fminf(m0, m1), fminf(m2, m3));
    for (int o = SINK_RL / 2; o > 0; o >>= 1) m = fminf(m, __shfl_xor(m, o, 64));
    const float kl = LOG2E / tau;
    auto e = [&](int yy) { return __builtin_amdgcn_exp2f((m - v(yy)) * kl); };
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    y = l;
    for (; y + 3 * SINK_RL < n; y += U) {
        s0 += e(y);
        s1 += e(y + SINK_RL);
        s2 += e(y + 2 * SINK_RL);
        s3 += e(y + 3 * SINK_RL);
    }
    for (; y < n; y += SINK_RL) s0 += e(y);
    float s = (s0 + s1) + (s2 + s3);
    for (int o = SINK_RL / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (live && l == 0) f[r] = m - tau * __logf(s);
}

// Column update g(y) = -tau log sum_x exp(-(z(x,y) - f(x))/tau).  A
// workgroup takes 64 adjacent stacked columns (the lanes, so a row's loads
// coalesce) and SINK_CW row chunks (the wavefronts: wavefront w takes rows
// w, w + SINK_CW, ...); the chunks' pairs are merged in LDS.  Each group of
// SINK_AHEAD rows is folded into the pair (m, s) at once: its minimum
// first, then one rescale of s and independent exponentials.
constexpr int SINK_CW = 8;
constexpr int SINK_AHEAD = 16;  // rows of a chunk loaded ahead
__global__ __launch_bounds__(64 * SINK_CW) void k_sink_cols(
    const NInst *inst, const int32_t *rinst, Costs CV, int32_t R,
    const unsigned long long *abssum, const float *f, float *g, float tau) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = blockIdx.x * 64 + lane;
    const float k = 1.0f / tau, kl = LOG2E / tau;
    __shared__ float sm[SINK_CW][64], ss[SINK_CW][64];
    float m = INFINITY, s = 0.f;
    if (r < R) {
        const int b = rinst[r];
        const NInst I = inst[b];
        const int y = r - I.row_off, n = I.n;
        const float inv = 1.0f / inst_scale(I, abssum, b);
        const bool s16 = CV.small(b);
        const int64_t col = I.cost_off + y;
        const float *fi = f + I.row_off;
        for (int x0 = w; x0 < n; x0 += SINK_CW * SINK_AHEAD) {
            int cb[SINK_AHEAD];
            float fb[SINK_AHEAD];
#pragma unroll
            for (int a = 0; a < SINK_AHEAD; ++a) {
                const int x = x0 + a * SINK_CW;
                const int xc = x < n ? x : x0;  // a valid row; its value is not used
                cb[a] = CV.at(s16, col + int64_t(xc) * n);
                fb[a] = fi[xc];
            }
            // rows past n count as +inf: their terms are exp2(-inf) = 0
            float vb[SINK_AHEAD];
#pragma unroll
            for (int a = 0; a < SINK_AHEAD; ++a)
                vb[a] = x0 + a * SINK_CW < n ? float(cb[a]) * inv - fb[a] : INFINITY;
            float mq[4] = {vb[0], vb[1], vb[2], vb[3]};
#pragma unroll
            for (int a = 4; a < SINK_AHEAD; ++a) mq[a & 3] = fminf(mq[a & 3], vb[a]);
            // row x0 is below n, so mn is finite; with m = inf the old sum
            // (0) is scaled by exp2(-inf) = 0
            const float mn = fminf(m, fminf(fminf(mq[0], mq[1]), fminf(mq[2], mq[3])));
            float sq[4] = {s * __builtin_amdgcn_exp2f((mn - m) * kl), 0.f, 0.f, 0.f};
#pragma unroll
            for (int a = 0; a < SINK_AHEAD; ++a)
                sq[a & 3] += __builtin_amdgcn_exp2f((mn - vb[a]) * kl);
            s = (sq[0] + sq[1]) + (sq[2] + sq[3]);
            m = mn;
        }
    }
    sm[w][lane] = m;
    ss[w][lane] = s;
    __syncthreads();
    if (w == 0 && r < R) {
        for (int j = 1; j < SINK_CW; ++j) lse_merge(m, s, sm[j][lane], ss[j][lane], k);
        g[r] = m - tau * __logf(s);
    }
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
    const int64_t row = I.cost_off + int64_t(x) * I.n;
    float mn = INFINITY;
    for (int y = lane; y < I.n; y += 64)
        mn = fminf(mn, float(CV.at(s16, row + y)) * inv - F[int64_t(I.row_off + y) * F_IN + 10]);
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
    const int64_t col = I.cost_off + y;
    float mn = INFINITY;
    for (int x0 = 0; x0 < n; x0 += FEAT_AHEAD) {
        int cb[FEAT_AHEAD];
        float ub[FEAT_AHEAD];
#pragma unroll
        for (int a = 0; a < FEAT_AHEAD; ++a) {
            const int x = x0 + a < n ? x0 + a : n - 1;  // a repeat is harmless for a min
            cb[a] = CV.at(s16, col + int64_t(x) * n);
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
                                                     float *F, const float *sval,
                                                     const float *v2, __bf16 *X,
                                                     __bf16 *XT) {
    const NInst I = inst[blockIdx.x];
    __shared__ float red[2][4];
    float a = 0.f, c = 0.f;
    for (int y = threadIdx.x; y < I.n; y += 256) {
        a += v2[I.row_off + y];
        c += sval[I.row_off + y];
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
        f[14] = sval[r] - ms;
        f[15] = ln;
        for (int k = 0; k < F_PAD; ++k) {
            const __bf16 v = to_bf16(k < F_IN ? f[k] : 0.f);
            X[int64_t(r) * F_PAD + k] = v;
            if (XT) XT[int64_t(k) * Rp + r] = v;
        }
    }
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
    int16_t *c16;     // saturated int16 copy of sign * c, packed like the input
    float *F, *sval, *u2, *v2;
    __bf16 *X0, *X0T;
    float *Z[3];
    __bf16 *H[3], *HT[3];
    float *M[3], *P[3];
    float *q, *dq, *dH, *G, *dZsum, *acc, *grad, *loss;
    __bf16 *dZ, *dZT;
    __bf16 *WT[3], *Wb[3];
};

static int64_t pad64(int64_t r) { return (r + 63) / 64 * 64; }

static Carver carve(Carver cv, int B, int64_t R, int64_t E, Layout *L) {
    const int64_t Rp = pad64(R);
    L->inst = cv.take<NInst>(B);
    L->rinst = cv.take<int32_t>(R);
    L->rowmin = cv.take<int32_t>(R);
    L->abssum = cv.take<unsigned long long>(B);
    L->cmax = cv.take<unsigned>(B);
    L->c16 = cv.take<int16_t>(E);
    L->F = cv.take<float>(R * F_IN);
    L->sval = cv.take<float>(R);
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

static int64_t total_rows(int B, const int32_t *n) {
    int64_t R = 0;
    for (int b = 0; b < B; ++b) R += n[b];
    return R;
}

static int64_t total_entries(int B, const int32_t *n) {
    int64_t E = 0;
    for (int b = 0; b < B; ++b) E += int64_t(n[b]) * n[b];
    return E;
}

static size_t workspace_bytes(int B, const int32_t *n) {
    Layout L;
    return carve(Carver(), B, total_rows(B, n), total_entries(B, n), &L).used();
}

struct Ctx {
    int B;
    int64_t R, Rp;
    Layout L;
    hipStream_t s;
    std::vector<NInst> insts;
    std::vector<int32_t> rinst;
};

static lpr_status prepare(Ctx &C, int32_t B, const int32_t *n,
                          const int64_t *cost_offset, const int32_t *costs,
                          void *ws, size_t ws_bytes, void *stream) {
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
    int64_t R = 0;
    for (int b = 0; b < B; ++b) {
        if (n[b] < 1 || n[b] > LPR_ASSIGN_MAX_N) {
            set_error("instance %d: n = %d outside [1, %d]", b, n[b], LPR_ASSIGN_MAX_N);
            return LPR_EINVAL;
        }
        if (cost_offset[b + 1] != cost_offset[b] + int64_t(n[b]) * n[b]) {
            set_error("cost_offset is not the prefix sum of n^2 at %d", b);
            return LPR_EINVAL;
        }
        C.insts[b] = NInst{cost_offset[b], n[b], int32_t(R)};
        R += n[b];
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
    carve(Carver(ws, ws_bytes), B, R, total_entries(B, n), &C.L);
    C.rinst.resize(R);
    for (int b = 0; b < B; ++b)
        std::fill(C.rinst.begin() + C.insts[b].row_off,
                  C.rinst.begin() + C.insts[b].row_off + n[b], b);
    C.s = static_cast<hipStream_t>(stream);
    LPR_TRY_HIP(hipMemcpyAsync(C.L.inst, C.insts.data(), sizeof(NInst) * B,
                               hipMemcpyHostToDevice, C.s));
    LPR_TRY_HIP(hipMemcpyAsync(C.L.rinst, C.rinst.data(), sizeof(int32_t) * R,
                               hipMemcpyHostToDevice, C.s));
    return LPR_OK;
}

static lpr_status run_features(Ctx &C, const int32_t *costs, int32_t sign, bool train) {
    Layout &L = C.L;
    const int R = int(C.R);
    LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(L.abssum), 0, C.B, C.s));
    LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(L.cmax), 0, C.B, C.s));
    const Costs CV{costs, L.c16, L.cmax, sign};
    // padding rows of the bf16 input are zero
    LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(L.X0), 0, C.Rp * F_PAD / 2, C.s));
    if (train) LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(L.X0T), 0, C.Rp * F_PAD / 2, C.s));
    int nmax = 0;
    for (const NInst &I : C.insts) nmax = std::max(nmax, int(I.n));
    hipLaunchKernelGGL(k_feat_rows1, dim3(ceil_div(nmax, ROWS1), C.B), dim3(256), 0, C.s,
                       L.inst, costs, sign, L.rowmin, L.abssum, L.c16, L.cmax);
    hipLaunchKernelGGL(k_feat_cols1, dim3(ceil_div(R, 256)), dim3(256), 0, C.s,
                       L.inst, L.rinst, CV, R, L.rowmin, L.abssum, L.F);
    // f14: annealed Sinkhorn potentials, rows into u2 (scratch until the
    // next pass), columns into sval, from g = 0
    LPR_TRY(fill_i32(reinterpret_cast<int32_t *>(L.sval), 0, R, C.s));
    double tau = SINK_TAU0;
    for (int it = 0; it < SINK_ITERS; ++it) {
        hipLaunchKernelGGL(k_sink_rows, dim3(ceil_div(R, 256 / SINK_RL)), dim3(256), 0, C.s,
                           L.inst, L.rinst, CV, R, L.abssum, L.sval, L.u2, float(tau));
        hipLaunchKernelGGL(k_sink_cols, dim3(ceil_div(R, 64)), dim3(64 * SINK_CW), 0, C.s,
                           L.inst, L.rinst, CV, R, L.abssum, L.u2, L.sval, float(tau));
        tau = std::max(SINK_TAU_MIN, tau * SINK_RATE);
    }
    hipLaunchKernelGGL(k_feat_rows2, dim3(ceil_div(R, 4)), dim3(256), 0, C.s,
                       L.inst, L.rinst, CV, R, L.abssum, L.F, L.u2);
    hipLaunchKernelGGL(k_feat_cols2, dim3(ceil_div(R, 256)), dim3(256), 0, C.s,
                       L.inst, L.rinst, CV, R, L.abssum, L.u2, L.v2);
    hipLaunchKernelGGL(k_feat_finish, dim3(C.B), dim3(256), 0, C.s, L.inst,
                       int32_t(C.Rp), L.F, L.sval, L.v2, L.X0, train ? L.X0T : nullptr);
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
    if (!params || (eps0 && !(kappa > 0.f))) {
        clear_error();
        set_error("NULL params, or eps0 requested with kappa <= 0");
        return LPR_EINVAL;
    }
    net::Ctx C;
    LPR_TRY(net::prepare(C, B, n, cost_offset, costs, workspace, workspace_bytes, stream));
    LPR_TRY(net::run_features(C, costs, maximize ? -1 : 1, false));
    LPR_TRY(net::run_forward(C, params, false));
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
