// Form 1 on an arbitrary directed graph: lock-free push-relabel max-flow on
// an explicit arc list, gfx950.
//
// Method (Section 4).  The network is given as arcs in mate pairs (arc a^1 is
// the reverse of a, as in the node/adjacency design of Section 4.3's
// implementation): u_f(a) = cap(a) - f(a) with a skew-symmetric pseudoflow.
// Init (Algorithm 4.7) saturates every arc leaving s and sets h(s) = |V|.
// The push/relabel operation is Algorithm 4.5 (Hong): an active node u
// (e(u) > 0, h(u) < |V|) finds the lowest neighbour w over its residual arcs;
// if h(u) > h(w) it pushes min(e(u), u_f(u,w)) with atomic updates of the two
// residuals and the two excesses, otherwise it relabels h(u) = h(w) + 1
// (only u's thread writes h(u)).  Between sweeps, the global relabel of
// Algorithm 4.4 recomputes h as the exact BFS distance to t over reverse
// residual arcs; nodes it does not reach get |V| (the gap step).  The solver
// stops when no node is active right after an exact relabel (Algorithm
// 4.8's termination, e(s) + e(t) = total): the preflow is then maximum, e(t)
// is the flow value, and the residual closure of s and of the nodes with
// excess is the minimal source side of a minimum cut.
//
// GPU design.  The arc list is turned into a CSR adjacency by tail on the
// device (degree count, exclusive scan, scatter).  A sweep is one thread per
// node running up to `cycle` operations (the paper's CYCLE); stale reads are
// lower bounds (residuals and excesses shrink only by their owner, heights
// only grow), the staleness Hong's argument admits.  The BFS runs level by
// level over a frontier queue (one launch per level over the whole device,
// frontier sizes kept on the device, the host checking once per batch of
// levels).
#include <algorithm>
#include <climits>

#include "lpr_internal.h"

namespace lpr {
namespace graph {

constexpr int NTB = 256;
constexpr int LEVEL_BATCH = 16;  // BFS levels launched between host checks
constexpr int CHUNK = 64;        // arcs per frontier entry
constexpr int GROUP = 8;         // lanes per frontier entry

struct G {
    int n, m, s, t;
    const int32_t *tail, *head, *cap;
    int32_t *off;    // [n + 1] CSR offsets over arcs grouped by tail
    int32_t *adj;    // [m] arc ids
    int32_t *cur;    // [n] scatter cursors
    int32_t *res;    // [m] residual capacities
    int64_t *e;      // [n] excesses
    int32_t *h;      // [n] heights
    int32_t *lab;    // [n] BFS labels / closure marks
    int64_t *q[2];   // frontier queues: entries (chunk << 32) | node
    int32_t *qn;     // [n + 2] frontier entries per level
    unsigned long long *cnt;  // pushes, relabels, active, error bits
    int32_t *bsum;   // block sums of the scan
};

// Checks the mate-pair structure and ranges (error bits: 1 range or
// structure, 2 capacity) and counts out-degrees into off[tail + 1].
// counter[key] += 1 for every lane with `active`, returning the lane's
// ticket (the old value plus its rank among the lanes of the same key).
// Lanes sharing the key of the first lane still waiting are served by one
// atomic, for two rounds, the rest by one atomic each: s and t can be the
// tail of half of all arcs, and one address taking an atomic per arc
// serialises the whole pass.  Called by every lane of the wavefront that
// runs the loop iteration.
__device__ inline int wave_ticket(int32_t *counter, int key, bool active) {
    const int lane = threadIdx.x & 63;
    bool done = !active;
    int ticket = 0;
    for (int r = 0; r < 2; ++r) {
        const unsigned long long left = __ballot(!done);
        if (!left) break;
        const int leader = __ffsll((long long)left) - 1;
        const int k0 = __shfl(key, leader, 64);
        const bool mine = !done && key == k0;
        const unsigned long long same = __ballot(mine);
        int base = 0;
        if (lane == leader) base = atomicAdd(&counter[k0], __popcll(same));
        base = __shfl(base, leader, 64);
        if (mine) {
            ticket = base + __popcll(same & ((1ull << lane) - 1));
            done = true;
        }
    }
    if (!done) ticket = atomicAdd(&counter[key], 1);
    return ticket;
}

__global__ __launch_bounds__(NTB) void k_validate(G g) {
    // wavefront-uniform trip count (wave_ticket needs every lane)
    for (int a0 = blockIdx.x * NTB; a0 < g.m; a0 += gridDim.x * NTB) {
        const int a = a0 + int(threadIdx.x);
        bool ok = false;
        int u = 0;
        if (a < g.m) {
            u = g.tail[a];
            const int v = g.head[a];
            unsigned bits = 0;
            if (u < 0 || u >= g.n || v < 0 || v >= g.n) {
                bits |= 1;
            } else {
                if (g.tail[a ^ 1] != v || g.head[a ^ 1] != u) bits |= 1;
                const int64_t c = g.cap[a], cr = g.cap[a ^ 1];
                // u_f(a) + u_f(a^1) = cap(a) + cap(a^1) stays below 2^31
                if (c < 0 || c + cr > int64_t(INT_MAX)) bits |= 2;
                ok = true;
            }
            if (bits) atomicOr(&g.cnt[3], (unsigned long long)bits);
        }
        wave_ticket(g.off, u + 1, ok);
    }
}

// Exclusive scan of off[0..n] in place (off[0] = 0 on entry): per-block
// inclusive scans of 1024 entries, then the block sums, then the offsets.
__global__ __launch_bounds__(1024) void k_scan_blocks(int32_t *x, int len, int32_t *bsum) {
    __shared__ int32_t s[1024];
    const int i = blockIdx.x * 1024 + threadIdx.x;
    s[threadIdx.x] = i < len ? x[i] : 0;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int32_t v = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    if (i < len) x[i] = s[threadIdx.x];
    if (threadIdx.x == 1023) bsum[blockIdx.x] = s[1023];
}

__global__ __launch_bounds__(1024) void k_scan_sums(int32_t *bsum, int nb) {
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    __shared__ int32_t s[1024];
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + threadIdx.x;
        s[threadIdx.x] = i < nb ? bsum[i] : 0;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int32_t v = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += v;
            __syncthreads();
        }
        // exclusive prefix of the block sums
        if (i < nb) bsum[i] = carry + s[threadIdx.x] - (i < nb ? bsum[i] : 0);
        __syncthreads();
        if (threadIdx.x == 0) carry += s[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_scan_add(int32_t *x, int len, const int32_t *bsum) {
    const int i = blockIdx.x * 1024 + threadIdx.x;
    if (i < len) x[i] += bsum[blockIdx.x];
}

__global__ __launch_bounds__(NTB) void k_scatter(G g) {
    for (int a0 = blockIdx.x * NTB; a0 < g.m; a0 += gridDim.x * NTB) {
        const int a = a0 + int(threadIdx.x);
        const bool in = a < g.m;
        const int u = in ? g.tail[a] : 0;
        const int k = wave_ticket(g.cur, u, in);
        if (in) g.adj[g.off[u] + k] = a;
    }
}

// Init (Algorithm 4.7) part 1: u_f = cap, e = 0, h = 0 except h(s) = |V|.
__global__ __launch_bounds__(NTB) void k_init(G g) {
    for (int a = blockIdx.x * NTB + threadIdx.x; a < g.m; a += gridDim.x * NTB)
        g.res[a] = g.cap[a];
    for (int v = blockIdx.x * NTB + threadIdx.x; v < g.n; v += gridDim.x * NTB) {
        g.e[v] = 0;
        g.h[v] = v == g.s ? g.n : 0;
        g.cur[v] = 0;
    }
}

// Init part 2: saturate every arc leaving s.
__global__ __launch_bounds__(NTB) void k_saturate(G g) {
    const int b = g.off[g.s], en = g.off[g.s + 1];
    for (int j = b + blockIdx.x * NTB + threadIdx.x; j < en; j += gridDim.x * NTB) {
        const int a = g.adj[j];
        const int32_t d = g.res[a];
        if (d <= 0 || g.head[a] == g.s) continue;
        g.res[a] = 0;
        atomicAdd(&g.res[a ^ 1], d);
        atomicAdd(reinterpret_cast<unsigned long long *>(&g.e[g.head[a]]),
                  (unsigned long long)d);
    }
}

// Algorithm 4.5: every node's thread makes `cycle` attempts (the paper's
// CYCLE loop), each a push or relabel when the node is active at that moment.
// A node with no residual arc at all cannot reach t: it takes |V|.
__global__ __launch_bounds__(NTB) void k_push(G g, int cycle) {
    unsigned long long pushes = 0, relabels = 0;
    for (int u = blockIdx.x * NTB + threadIdx.x; u < g.n; u += gridDim.x * NTB) {
        if (u == g.s || u == g.t) continue;
        const int b = g.off[u], en = g.off[u + 1];
        int hu = g.h[u];
        for (int it = 0; it < cycle; ++it) {
            if (hu >= g.n) break;
            // an idle node keeps polling its excess for the rest of the
            // sweep: flow pushed into it meanwhile moves on in the same sweep
            const int64_t eu = g.e[u];
            if (eu <= 0) continue;
            int hmin = INT_MAX, amin = -1;
            for (int j = b; j < en; ++j) {
                const int a = g.adj[j];
                const int w = g.head[a];
                if (w == u || g.res[a] <= 0) continue;
                const int hw = g.h[w];
                if (hw < hmin) {
                    hmin = hw;
                    amin = a;
                }
            }
            if (amin < 0) {
                hu = g.n;
                g.h[u] = hu;
                ++relabels;
                break;
            }
            if (hu > hmin) {
                const int32_t r = g.res[amin];
                const int32_t d = int32_t(eu < int64_t(r) ? eu : int64_t(r));
                if (d <= 0) continue;
                atomicSub(&g.res[amin], d);
                atomicAdd(&g.res[amin ^ 1], d);
                atomicAdd(reinterpret_cast<unsigned long long *>(&g.e[u]),
                          (unsigned long long)(-int64_t(d)));
                atomicAdd(reinterpret_cast<unsigned long long *>(&g.e[g.head[amin]]),
                          (unsigned long long)d);
                ++pushes;
            } else {
                hu = hmin >= g.n - 1 ? g.n : hmin + 1;
                g.h[u] = hu;
                ++relabels;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        pushes += __shfl_xor(pushes, o, 64);
        relabels += __shfl_xor(relabels, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (pushes) atomicAdd(&g.cnt[0], pushes);
        if (relabels) atomicAdd(&g.cnt[1], relabels);
    }
}

// Frontier entries: a node's arcs in chunks of CHUNK, one entry per chunk
// (at least one), so that a hub's arcs spread over many wavefronts.  A node
// has at most max(1, ceil(d / CHUNK)) entries, and a queue at most
// n + m / CHUNK + 1.
__device__ inline int chunks_of(const G &g, int v) {
    const int d = g.off[v + 1] - g.off[v];
    return d > CHUNK ? (d + CHUNK - 1) / CHUNK : 1;
}

__device__ inline void enqueue(const G &g, int64_t *q, int32_t *count, int v) {
    const int k = chunks_of(g, v);
    const int base = atomicAdd(count, k);
    for (int c = 0; c < k; ++c) q[base + c] = (int64_t(c) << 32) | uint32_t(v);
}

// BFS seeds.  Backward (global relabel): labels |V| except t at 0, frontier
// {t}.  Forward (cut): marks s and every node with excess, frontier = them.
__global__ __launch_bounds__(NTB) void k_bfs_seed(G g, int forward) {
    const int tid = blockIdx.x * NTB + threadIdx.x, nth = gridDim.x * NTB;
    for (int v = tid; v < g.n; v += nth) {
        if (!forward) {
            g.lab[v] = v == g.t ? 0 : g.n;
        } else {
            const bool in = v == g.s || (v != g.t && g.e[v] > 0);
            g.lab[v] = in ? 1 : 0;
            if (in) enqueue(g, g.q[0], &g.qn[0], v);
        }
    }
    if (!forward) {  // t's entries, one per thread
        const int k = chunks_of(g, g.t);
        for (int c = tid; c < k; c += nth) g.q[0][c] = (int64_t(c) << 32) | uint32_t(g.t);
        if (tid == 0) g.qn[0] = k;
    }
}

// Level L of a BFS over the frontier q[L & 1] (`size` entries): GROUP lanes
// per entry over its chunk of the node's arcs, 64 / GROUP entries per
// wavefront at a time.  Backward: w reaches frontier node u over the
// residual arc (w,u) = a^1 of u's arc a = (u,w); w gets L + 1 (s keeps |V|).
// Forward: u reaches w over its residual arc a; w is marked.  The next
// frontier goes to q[(L + 1) & 1].
__device__ inline void bfs_expand(const G &g, int L, int forward, int size, int wid,
                                  int nwaves, int lane) {
    const int64_t *front = g.q[L & 1];
    int64_t *next = g.q[(L + 1) & 1];
    constexpr int PER = 64 / GROUP;
    const int sub = lane % GROUP;
    for (int i = wid * PER + lane / GROUP; i < size; i += nwaves * PER) {
        const int64_t ent = front[i];
        const int u = int(uint32_t(ent));
        const int b = g.off[u] + int(ent >> 32) * CHUNK;
        const int e = min(g.off[u + 1], b + CHUNK);
        for (int j = b + sub; j < e; j += GROUP) {
            const int a = g.adj[j];
            const int w = g.head[a];
            if (!forward) {
                if (w == g.s || g.res[a ^ 1] <= 0 || g.lab[w] != g.n) continue;
                if (atomicCAS(&g.lab[w], g.n, L + 1) == g.n)
                    enqueue(g, next, &g.qn[L + 1], w);
            } else {
                if (g.res[a] <= 0 || g.lab[w] != 0) continue;
                if (atomicCAS(&g.lab[w], 0, 1) == 0) enqueue(g, next, &g.qn[L + 1], w);
            }
        }
    }
}

// One BFS level L over the whole device.
__global__ __launch_bounds__(NTB) void k_bfs_level(G g, int L, int forward) {
    const int size = g.qn[L];
    if (size == 0) return;
    bfs_expand(g, L, forward, size, (blockIdx.x * NTB + threadIdx.x) >> 6,
               (gridDim.x * NTB) >> 6, threadIdx.x & 63);
}

// Heights from the exact labels (unreached: |V|), and the active count.
__global__ __launch_bounds__(NTB) void k_labels_count(G g) {
    unsigned long long act = 0;
    for (int v = blockIdx.x * NTB + threadIdx.x; v < g.n; v += gridDim.x * NTB) {
        if (v == g.s) continue;
        const int hv = g.lab[v];
        g.h[v] = hv;
        if (v != g.t && hv < g.n && g.e[v] > 0) ++act;
    }
    for (int o = 32; o > 0; o >>= 1) act += __shfl_xor(act, o, 64);
    if ((threadIdx.x & 63) == 0 && act) atomicAdd(&g.cnt[2], act);
}

__global__ __launch_bounds__(NTB) void k_side(G g, uint8_t *side) {
    for (int v = blockIdx.x * NTB + threadIdx.x; v < g.n; v += gridDim.x * NTB)
        side[v] = uint8_t(g.lab[v] != 0);
}

static int blocks_for(int64_t k) {
    return int(std::max<int64_t>(1, std::min<int64_t>(4096, (k + NTB - 1) / NTB)));
}

struct Layout {
    int32_t *off, *adj, *cur, *res, *h, *lab, *qn, *bsum;
    int64_t *q0, *q1;
    int64_t *e;
    unsigned long long *cnt;
};

static Carver carve(Carver cv, int n, int m, Layout *L) {
    L->off = cv.take<int32_t>(size_t(n) + 1);
    L->adj = cv.take<int32_t>(size_t(std::max(m, 1)));
    L->cur = cv.take<int32_t>(size_t(n));
    L->res = cv.take<int32_t>(size_t(std::max(m, 1)));
    L->h = cv.take<int32_t>(size_t(n));
    L->lab = cv.take<int32_t>(size_t(n));
    const size_t qcap = size_t(n) + size_t(m) / CHUNK + 1;
    L->q0 = cv.take<int64_t>(qcap);
    L->q1 = cv.take<int64_t>(qcap);
    L->qn = cv.take<int32_t>(size_t(n) + 2);
    L->bsum = cv.take<int32_t>(size_t((n + 1 + 1023) / 1024) + 1);
    L->e = cv.take<int64_t>(size_t(n));
    L->cnt = cv.take<unsigned long long>(4);
    return cv;
}

// A BFS (backward labels or forward closure) to its end: levels launched in
// batches, the host reading the frontier size once per batch.
static lpr_status run_bfs(const G &g, int forward, hipStream_t s, int64_t *levels) {
    LPR_TRY(fill_i32(g.qn, 0, int64_t(g.n) + 2, s));
    hipLaunchKernelGGL(k_bfs_seed, dim3(blocks_for(g.n)), dim3(NTB), 0, s, g, forward);
    LPR_TRY_HIP(hipGetLastError());
    const int grid = blocks_for(g.n);
    for (int L0 = 0; L0 <= g.n; L0 += LEVEL_BATCH) {
        const int L1 = std::min(g.n + 1, L0 + LEVEL_BATCH);
        for (int L = L0; L < L1; ++L)
            hipLaunchKernelGGL(k_bfs_level, dim3(grid), dim3(NTB), 0, s, g, L, forward);
        LPR_TRY_HIP(hipGetLastError());
        int32_t last = 0;
        LPR_TRY_HIP(hipMemcpyAsync(&last, g.qn + L1, sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s));
        LPR_TRY_HIP(hipStreamSynchronize(s));
        *levels += L1 - L0;
        if (last == 0) return LPR_OK;
    }
    return LPR_OK;  // every level up to |V| done: the BFS is complete
}

// The state of a network on its workspace: u_f = cap, e = 0, and the CSR of
// arc ids by tail (degree count with the mate-pair and capacity checks, an
// exclusive scan, the scatter).
static lpr_status build_csr(int n, int m, int s, int t, const int32_t *tail,
                            const int32_t *head, const int32_t *cap, const Layout &L,
                            hipStream_t st, G *out) {
    G g;
    g.n = n;
    g.m = m;
    g.s = s;
    g.t = t;
    g.tail = tail;
    g.head = head;
    g.cap = cap;
    g.off = L.off;
    g.adj = L.adj;
    g.cur = L.cur;
    g.res = L.res;
    g.e = L.e;
    g.h = L.h;
    g.lab = L.lab;
    g.q[0] = L.q0;
    g.q[1] = L.q1;
    g.qn = L.qn;
    g.cnt = L.cnt;
    g.bsum = L.bsum;
    *out = g;
    const int ga = blocks_for(m), gn = blocks_for(n);
    LPR_TRY(fill_i32(L.off, 0, int64_t(n) + 1, st));
    LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(L.cnt), 0, 4, st));
    hipLaunchKernelGGL(k_init, dim3(std::max(ga, gn)), dim3(NTB), 0, st, g);
    if (m > 0) hipLaunchKernelGGL(k_validate, dim3(ga), dim3(NTB), 0, st, g);
    LPR_TRY_HIP(hipGetLastError());
    unsigned long long cnt[4] = {0, 0, 0, 0};
    LPR_TRY_HIP(hipMemcpyAsync(cnt, L.cnt, sizeof(cnt), hipMemcpyDeviceToHost, st));
    LPR_TRY_HIP(hipStreamSynchronize(st));
    if (cnt[3]) {
        if (cnt[3] & 1) {
            set_error("arcs are not mate pairs (a^1 reverses a) over nodes 0..n-1");
            return LPR_EINVAL;
        }
        set_error("a capacity is negative or a mate pair's sum exceeds 2^31 - 1");
        return LPR_ERANGE;
    }
    // CSR by tail: exclusive scan of the degrees, then the scatter
    const int len = n + 1, nb = (len + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(1024), 0, st, L.off, len, L.bsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, L.bsum, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, st, L.off, len, L.bsum);
    if (m > 0) hipLaunchKernelGGL(k_scatter, dim3(ga), dim3(NTB), 0, st, g);
    LPR_TRY_HIP(hipGetLastError());
    return LPR_OK;
}

}  // namespace graph
}  // namespace lpr

using namespace lpr;

extern "C" size_t lpr_graph_maxflow_workspace(int32_t n, int32_t m) {
    if (n < 2 || m < 0 || (m & 1)) return 0;
    graph::Layout L;
    return graph::carve(Carver(), n, m, &L).used();
}

extern "C" lpr_status lpr_graph_maxflow(int32_t n, int32_t m, const int32_t *tail,
                                        const int32_t *head, const int32_t *cap,
                                        int32_t s, int32_t t, int64_t *flow_value,
                                        uint8_t *source_side,
                                        const lpr_graph_opts *opts,
                                        lpr_graph_stats *stats, void *workspace,
                                        size_t workspace_bytes, void *stream) {
    clear_error();
    if (n < 2 || m < 0 || (m & 1) || s < 0 || s >= n || t < 0 || t >= n || s == t ||
        !flow_value || !workspace || (m > 0 && (!tail || !head || !cap)) ||
        n > LPR_GRAPH_MAX_N) {
        set_error("invalid arguments (n, m, s, t or a NULL pointer)");
        return LPR_EINVAL;
    }
    // defaults measured on layered, grid and random networks of 65 k - 262 k
    // nodes (16 x 16 against 1 x 64: 3 - 9 times faster)
    int cycle = 16, max_rounds = 100000, sweeps = 16;
    if (opts) {
        if (opts->cycle) cycle = opts->cycle;
        if (opts->max_rounds) max_rounds = opts->max_rounds;
        if (opts->sweeps_per_relabel) sweeps = opts->sweeps_per_relabel;
    }
    if (cycle < 1 || max_rounds < 1 || sweeps < 1 || sweeps > 1024) {
        set_error("invalid lpr_graph_opts");
        return LPR_EINVAL;
    }
    graph::Layout L;
    const size_t need = graph::carve(Carver(), n, m, &L).used();
    if (workspace_bytes < need) {
        set_error("workspace too small: %zu < %zu bytes", workspace_bytes, need);
        return LPR_ENOMEM;
    }
    graph::carve(Carver(workspace, workspace_bytes), n, m, &L);
    hipStream_t st = static_cast<hipStream_t>(stream);
    CallTimer call(st);
    call.start();
    graph::G g;
    LPR_TRY(graph::build_csr(n, m, s, t, tail, head, cap, L, st, &g));
    const int gn = graph::blocks_for(n);
    unsigned long long cnt[4] = {0, 0, 0, 0};
    hipLaunchKernelGGL(graph::k_saturate, dim3(graph::blocks_for(m)), dim3(graph::NTB), 0,
                       st, g);
    LPR_TRY_HIP(hipGetLastError());

    int64_t rounds = 0, levels = 0;
    for (;;) {
        LPR_TRY(graph::run_bfs(g, 0, st, &levels));
        LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(L.cnt) + 2, 0, 1, st));
        hipLaunchKernelGGL(graph::k_labels_count, dim3(gn), dim3(graph::NTB), 0, st, g);
        LPR_TRY_HIP(hipGetLastError());
        LPR_TRY_HIP(hipMemcpyAsync(cnt, L.cnt, sizeof(cnt), hipMemcpyDeviceToHost, st));
        LPR_TRY_HIP(hipStreamSynchronize(st));
        if (cnt[2] == 0) break;
        if (rounds >= max_rounds) {
            set_error("graph max-flow: round budget (%d) exhausted", max_rounds);
            return LPR_EBUDGET;
        }
        ++rounds;
        for (int k = 0; k < sweeps; ++k)
            hipLaunchKernelGGL(graph::k_push, dim3(gn), dim3(graph::NTB), 0, st, g, cycle);
        LPR_TRY_HIP(hipGetLastError());
    }
    LPR_TRY_HIP(hipMemcpyAsync(flow_value, L.e + t, sizeof(int64_t), hipMemcpyDeviceToHost,
                               st));
    if (source_side) {
        LPR_TRY(graph::run_bfs(g, 1, st, &levels));
        hipLaunchKernelGGL(graph::k_side, dim3(gn), dim3(graph::NTB), 0, st, g, source_side);
        LPR_TRY_HIP(hipGetLastError());
    }
    double ms = 0;
    LPR_TRY(call.stop_ms(&ms));
    if (stats) {
        stats->rounds = rounds;
        stats->pushes = int64_t(cnt[0]);
        stats->relabels = int64_t(cnt[1]);
        stats->bfs_levels = levels;
        stats->total_ms = ms;
    }
    return LPR_OK;
}

// ---------------------------------------------------------------------------
// Minimum-cost flow with supplies by cost scaling (Section 5, Algorithm 5.0:
// Min-Cost, the generic Refine, push, relabel), on the same CSR.  Reduced
// cost c_p(a) = cost(a) S + p(tail) - p(head) with S = n + 1; an arc is
// admissible when residual with c_p < 0.
// ---------------------------------------------------------------------------
namespace lpr {
namespace graph {

struct Mcf {
    const int32_t *cost;    // [m], cost[a ^ 1] = -cost[a]
    const int32_t *supply;  // [n]
    int64_t *p;             // [n] prices of the scaled costs
    int64_t S;              // n + 1
    unsigned long long *w;  // [8]: error bits, max |cost|, supply sum, positive
                            // supply sum, -, eps of the current refine
};

// error bits: 1 costs not antisymmetric, 2 |cost| or |supply| out of range
__global__ __launch_bounds__(NTB) void k_mcf_check(G g, Mcf q) {
    const int tid = blockIdx.x * NTB + threadIdx.x, nth = gridDim.x * NTB;
    unsigned bits = 0, cm = 0;
    long long sum = 0, pos = 0;
    for (int a = tid; a < g.m; a += nth) {
        const int c = q.cost[a];
        if (q.cost[a ^ 1] != -c) bits |= 1;
        const unsigned u = c < 0 ? 0u - unsigned(c) : unsigned(c);
        if (u > unsigned(LPR_MCF_MAX_COST)) bits |= 2;
        cm = max(cm, u);
    }
    for (int v = tid; v < g.n; v += nth) {
        const int d = q.supply[v];
        if (d > LPR_MCF_MAX_SUPPLY || d < -LPR_MCF_MAX_SUPPLY) bits |= 2;
        sum += d;
        pos += d > 0 ? d : 0;
    }
    if (bits) atomicOr(&q.w[0], (unsigned long long)bits);
    if (cm) atomicMax(&q.w[1], (unsigned long long)cm);
    if (sum) atomicAdd(&q.w[2], (unsigned long long)sum);
    if (pos) atomicAdd(&q.w[3], (unsigned long long)pos);
}

// The feasibility network: the arcs as given, then per node v the pairs
// s* -> v (capacity max(d, 0)) and v -> t* (capacity max(-d, 0));
// s* = n, t* = n + 1.
__global__ __launch_bounds__(NTB) void k_mcf_feas_arcs(G g, Mcf q, int32_t *ft, int32_t *fh,
                                                       int32_t *fc) {
    const int tid = blockIdx.x * NTB + threadIdx.x, nth = gridDim.x * NTB;
    for (int a = tid; a < g.m; a += nth) {
        ft[a] = g.tail[a];
        fh[a] = g.head[a];
        fc[a] = g.cap[a];
    }
    for (int v = tid; v < g.n; v += nth) {
        const int d = q.supply[v];
        const int64_t b = int64_t(g.m) + 4 * int64_t(v);
        ft[b] = g.n;
        fh[b] = v;
        fc[b] = d > 0 ? d : 0;
        ft[b + 1] = v;
        fh[b + 1] = g.n;
        fc[b + 1] = 0;
        ft[b + 2] = v;
        fh[b + 2] = g.n + 1;
        fc[b + 2] = d < 0 ? -d : 0;
        ft[b + 3] = g.n + 1;
        fh[b + 3] = v;
        fc[b + 3] = 0;
    }
}

__device__ inline int64_t reduced(const G &g, const Mcf &q, int a, int64_t pu) {
    return int64_t(q.cost[a]) * q.S + pu - q.p[g.head[a]];
}

// Refine's start: every arc of negative reduced cost is saturated (one
// thread per mate pair: c_p(a ^ 1) = -c_p(a), so at most one of the two).
__global__ __launch_bounds__(NTB) void k_mcf_saturate(G g, Mcf q) {
    for (int a = 2 * (blockIdx.x * NTB + threadIdx.x); a < g.m; a += 2 * gridDim.x * NTB) {
        const int64_t cp = reduced(g, q, a, q.p[g.tail[a]]);
        const int r = g.res[a], rr = g.res[a ^ 1];
        if (cp < 0 && r > 0) {
            g.res[a] = 0;
            g.res[a ^ 1] = rr + r;
        } else if (cp > 0 && rr > 0) {
            g.res[a] = r + rr;
            g.res[a ^ 1] = 0;
        }
    }
}

// e(v) = supply(v) - sum of the net flow out of v; nodes with e > 0 counted.
__global__ __launch_bounds__(NTB) void k_mcf_excess(G g, Mcf q) {
    unsigned long long act = 0;
    for (int v = blockIdx.x * NTB + threadIdx.x; v < g.n; v += gridDim.x * NTB) {
        int64_t e = q.supply[v];
        for (int k = g.off[v]; k < g.off[v + 1]; ++k) {
            const int a = g.adj[k];
            e -= int64_t(g.cap[a]) - g.res[a];
        }
        g.e[v] = e;
        act += e > 0;
    }
    for (int o = 32; o > 0; o >>= 1) act += __shfl_xor(act, o, 64);
    if ((threadIdx.x & 63) == 0 && act) atomicAdd(&g.cnt[2], act);
}

__device__ inline int64_t shfl_up64(int64_t v, int d) {
    const int lo = __shfl_up(int(uint32_t(v)), d, 64);
    const int hi = __shfl_up(int(v >> 32), d, 64);
    return int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}

__device__ inline int64_t shfl_xor64(int64_t v, int d) {
    const int lo = __shfl_xor(int(uint32_t(v)), d, 64);
    const int hi = __shfl_xor(int(v >> 32), d, 64);
    return int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}

constexpr int MCF_CYCLE = 8;  // times a push pass visits each node

// Push pass, one wavefront per node, its lanes over 64 arcs at a time:
// prices are fixed; a node with excess sends min(e, u_f) along its
// admissible arcs in CSR order (an inclusive scan of the admissible
// residuals gives every lane its share of what is left).  Only v lowers
// res(a) for its own arcs and only v lowers e(v); others only raise them,
// so every amount read stays available.  Each node is visited MCF_CYCLE
// times per pass, reading its excess from the device-coherent level each
// time, so flow pushed into it meanwhile moves on in the same pass.
__global__ __launch_bounds__(NTB) void k_mcf_push(G g, Mcf q) {
    const int lane = threadIdx.x & 63;
    const int nwaves = (gridDim.x * NTB) >> 6;
    unsigned long long pushes = 0;
    for (int it = 0; it < MCF_CYCLE; ++it)
    for (int v = (blockIdx.x * NTB + threadIdx.x) >> 6; v < g.n; v += nwaves) {
        // others add to e(v) meanwhile: every lane takes lane 0's reading
        int64_t e0 = __hip_atomic_load(&g.e[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        {
            const int lo = __shfl(int(uint32_t(e0)), 0, 64);
            const int hi = __shfl(int(e0 >> 32), 0, 64);
            e0 = int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
        }
        if (e0 <= 0) continue;
        int64_t left = e0;
        const int64_t pv = q.p[v];
        const int end = g.off[v + 1];
        for (int k0 = g.off[v]; k0 < end && left > 0; k0 += 64) {
            const int k = k0 + lane;
            int a = 0;
            int64_t r = 0;
            if (k < end) {
                a = g.adj[k];
                const int rr = g.res[a];
                if (rr > 0 && reduced(g, q, a, pv) < 0) r = rr;
            }
            int64_t incl = r;
            for (int o = 1; o < 64; o <<= 1) {
                const int64_t t = shfl_up64(incl, o);
                if (lane >= o) incl += t;
            }
            const int64_t before = incl - r;
            const int64_t d = min(r, max(int64_t(0), left - before));
            if (d > 0) {
                atomicSub(&g.res[a], int(d));
                atomicAdd(&g.res[a ^ 1], int(d));
                atomicAdd(reinterpret_cast<unsigned long long *>(&g.e[g.head[a]]),
                          (unsigned long long)d);
                ++pushes;
            }
            // the wave sent min(left, sum of the admissible residuals)
            const int lo = __shfl(int(uint32_t(incl)), 63, 64);
            const int hi = __shfl(int(incl >> 32), 63, 64);
            left -= min(left, int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo)));
        }
        if (lane == 0 && left != e0)
            atomicAdd(reinterpret_cast<unsigned long long *>(&g.e[v]),
                      (unsigned long long)(left - e0));
    }
    for (int o = 32; o > 0; o >>= 1) pushes += __shfl_xor(pushes, o, 64);
    if (lane == 0 && pushes) atomicAdd(&g.cnt[0], pushes);
}

// Relabel pass, one wavefront per node: a node with excess and no
// admissible arc takes p(v) = max over residual arcs (v,w) of
// p(w) - cost S - eps.  Neighbours relabelling at the same time only lower
// their prices, and a value read before such a change gives a price that is
// still eps-optimal on both directions of every arc.
__global__ __launch_bounds__(NTB) void k_mcf_relabel(G g, Mcf q) {
    const int64_t eps = int64_t(q.w[5]);
    const int lane = threadIdx.x & 63;
    const int nwaves = (gridDim.x * NTB) >> 6;
    unsigned long long relabels = 0;
    for (int v = (blockIdx.x * NTB + threadIdx.x) >> 6; v < g.n; v += nwaves) {
        if (g.e[v] <= 0) continue;
        const int64_t pv = q.p[v];
        int64_t best = LLONG_MIN;
        bool admissible = false;
        for (int k = g.off[v] + lane; k < g.off[v + 1]; k += 64) {
            const int a = g.adj[k];
            if (g.res[a] <= 0) continue;
            const int64_t val = q.p[g.head[a]] - int64_t(q.cost[a]) * q.S;
            admissible |= val > pv;  // c_p(a) < 0
            best = max(best, val);
        }
        for (int o = 32; o > 0; o >>= 1) best = max(best, shfl_xor64(best, o));
        if (__ballot(admissible) == 0 && best != LLONG_MIN) {
            if (lane == 0) q.p[v] = best - eps;
            ++relabels;
        }
    }
    if (lane == 0 && relabels) atomicAdd(&g.cnt[1], relabels);
}

// Global price update (Algorithm 5.3 on the general network): labels d(v)
// = least sum of lengths floor(c_p(a) / eps) + 1 over residual paths from v
// to a node with a deficit (d = 0 there), capped at LCAP; then
// p(v) -= eps d(v), nodes that reach no deficit taking the largest label
// found.  Any labels with d(v) <= d(w) + length(v,w) on every residual arc
// keep the pseudoflow eps-optimal, and both the cap and a Bellman-Ford
// pass reading labels that are still falling keep that inequality.
// Labels are relaxed to their fixpoint one wavefront per node.
__global__ __launch_bounds__(NTB) void k_mcf_pu_init(G g, int32_t *d, int32_t cap) {
    for (int v = blockIdx.x * NTB + threadIdx.x; v < g.n; v += gridDim.x * NTB)
        d[v] = g.e[v] < 0 ? 0 : cap;
}

__global__ __launch_bounds__(NTB) void k_mcf_pu_relax(G g, Mcf q, int32_t *d, int32_t cap,
                                                      int32_t *changed) {
    const int lane = threadIdx.x & 63;
    const int nwaves = (gridDim.x * NTB) >> 6;
    const int64_t eps = int64_t(q.w[5]);
    for (int v = (blockIdx.x * NTB + threadIdx.x) >> 6; v < g.n; v += nwaves) {
        const int dv = d[v];
        if (dv == 0) continue;
        const int64_t pv = q.p[v];
        int best = cap;
        for (int k = g.off[v] + lane; k < g.off[v + 1]; k += 64) {
            const int a = g.adj[k];
            if (g.res[a] <= 0) continue;
            const int dw = d[g.head[a]];
            if (dw >= cap) continue;
            // c_p >= -eps on residual arcs, so the length is >= 0
            const int64_t cp = reduced(g, q, a, pv);
            const int64_t len = cp < 0 ? 0 : cp / eps + 1;
            best = int(min(int64_t(best), int64_t(dw) + len));
        }
        for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
        if (lane == 0 && best < dv) {
            d[v] = best;
            *changed = 1;
        }
    }
}

__global__ __launch_bounds__(NTB) void k_mcf_pu_max(G g, const int32_t *d, int32_t cap,
                                                    int32_t *dmax) {
    int m = 0;
    for (int v = blockIdx.x * NTB + threadIdx.x; v < g.n; v += gridDim.x * NTB)
        if (d[v] < cap) m = max(m, d[v]);
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0 && m) atomicMax(dmax, m);
}

__global__ __launch_bounds__(NTB) void k_mcf_pu_apply(G g, Mcf q, const int32_t *d,
                                                      int32_t cap, const int32_t *dmax) {
    const int64_t eps = int64_t(q.w[5]);
    for (int v = blockIdx.x * NTB + threadIdx.x; v < g.n; v += gridDim.x * NTB) {
        const int dv = d[v] < cap ? d[v] : *dmax;
        if (dv) q.p[v] -= eps * dv;
    }
}

__global__ __launch_bounds__(NTB) void k_mcf_count(G g) {
    unsigned long long act = 0;
    for (int v = blockIdx.x * NTB + threadIdx.x; v < g.n; v += gridDim.x * NTB)
        act += g.e[v] > 0;
    for (int o = 32; o > 0; o >>= 1) act += __shfl_xor(act, o, 64);
    if ((threadIdx.x & 63) == 0 && act) atomicAdd(&g.cnt[2], act);
}

// sum over pairs of net flow x cost
__global__ __launch_bounds__(NTB) void k_mcf_total(G g, Mcf q, unsigned long long *tot) {
    long long t = 0;
    for (int a = 2 * (blockIdx.x * NTB + threadIdx.x); a < g.m; a += 2 * gridDim.x * NTB)
        t += (long long)(int64_t(g.cap[a]) - g.res[a]) * q.cost[a];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0 && t) atomicAdd(tot, (unsigned long long)t);
}

struct McfLayout {
    Layout L;
    int32_t *d, *flags;  // price-update labels [n]; changed, max label
    int64_t *p;
    unsigned long long *w;
    int32_t *ft, *fh, *fc;
    unsigned char *fws;
    size_t fbytes;
};

static Carver mcf_carve(Carver cv, int n, int m, McfLayout *M) {
    cv = carve(cv, n, m, &M->L);
    const int64_t fm = int64_t(m) + 4 * int64_t(n);
    M->p = cv.take<int64_t>(size_t(n));
    M->d = cv.take<int32_t>(size_t(n));
    M->flags = cv.take<int32_t>(2);
    M->w = cv.take<unsigned long long>(8);
    M->ft = cv.take<int32_t>(size_t(fm));
    M->fh = cv.take<int32_t>(size_t(fm));
    M->fc = cv.take<int32_t>(size_t(fm));
    M->fbytes = lpr_graph_maxflow_workspace(n + 2, int32_t(fm));
    M->fws = cv.take<unsigned char>(M->fbytes);
    return cv;
}

// The passes between two host checks (push and relabel passes, then the
// active count) captured once per call and replayed: the long tail of a
// refine has few active nodes, and each pass there costs little more than
// its launches.  eps is read from the device, so one graph serves every
// refine.
struct McfPasses {
    hipStream_t cs = nullptr;
    hipGraphExec_t ex = nullptr;
    ~McfPasses() {
        if (ex) (void)hipGraphExecDestroy(ex);
        if (cs) (void)hipStreamDestroy(cs);
    }
    lpr_status capture(const G &g, const Mcf &q, int gw, int gn, int passes) {
        LPR_TRY_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        LPR_TRY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < passes; ++k) {
            hipLaunchKernelGGL(k_mcf_push, dim3(gw), dim3(NTB), 0, cs, g, q);
            hipLaunchKernelGGL(k_mcf_relabel, dim3(gw), dim3(NTB), 0, cs, g, q);
        }
        hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, cs,
                           reinterpret_cast<int64_t *>(g.cnt) + 2, int64_t(0), int64_t(1));
        hipLaunchKernelGGL(k_mcf_count, dim3(gn), dim3(NTB), 0, cs, g);
        hipGraph_t gr = nullptr;
        const hipError_t le = hipGetLastError();
        const hipError_t ce = hipStreamEndCapture(cs, &gr);
        if (le != hipSuccess || ce != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            set_error("capturing the min-cost passes failed: %s",
                      hipGetErrorString(le != hipSuccess ? le : ce));
            return LPR_EDEVICE;
        }
        const hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (ie != hipSuccess) {
            ex = nullptr;
            set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ie));
            return LPR_EDEVICE;
        }
        return LPR_OK;
    }
};

static bool mcf_args_ok(int32_t n, int32_t m) {
    return n >= 1 && n <= LPR_MCF_MAX_N && m >= 0 && (m & 1) == 0 &&
           int64_t(m) + 4 * int64_t(n) <= int64_t(INT_MAX) - 1;
}

}  // namespace graph
}  // namespace lpr

extern "C" size_t lpr_mincost_flow_workspace(int32_t n, int32_t m) {
    if (!graph::mcf_args_ok(n, m)) return 0;
    graph::McfLayout M;
    return graph::mcf_carve(Carver(), n, m, &M).used();
}

extern "C" lpr_status lpr_mincost_flow(int32_t n, int32_t m, const int32_t *tail,
                                       const int32_t *head, const int32_t *cap,
                                       const int32_t *cost, const int32_t *supply,
                                       int64_t *total_cost, int32_t *residual,
                                       int64_t *prices, const lpr_mcf_opts *opts,
                                       lpr_mcf_stats *stats, void *workspace,
                                       size_t workspace_bytes, void *stream) {
    using namespace graph;
    clear_error();
    if (!mcf_args_ok(n, m) || !supply || !total_cost || !workspace ||
        (m > 0 && (!tail || !head || !cap || !cost))) {
        set_error("invalid arguments (n = %d, m = %d, or a NULL pointer)", n, m);
        return LPR_EINVAL;
    }
    int32_t alpha = 8, per_check = 32;
    int64_t max_iters = int64_t(1) << 20;
    if (opts) {
        if (opts->alpha) alpha = opts->alpha;
        if (opts->iters_per_check) per_check = opts->iters_per_check;
        if (opts->max_iters) max_iters = opts->max_iters;
    }
    if (alpha < 2 || per_check < 1 || per_check > 1024 || max_iters < 1) {
        set_error("invalid lpr_mcf_opts");
        return LPR_EINVAL;
    }
    const size_t need = lpr_mincost_flow_workspace(n, m);
    if (workspace_bytes < need) {
        set_error("workspace too small: %zu < %zu bytes", workspace_bytes, need);
        return LPR_ENOMEM;
    }
    McfLayout M;
    mcf_carve(Carver(workspace, workspace_bytes), n, m, &M);
    hipStream_t st = static_cast<hipStream_t>(stream);
    CallTimer call(st);
    call.start();
    G g;
    LPR_TRY(build_csr(n, m, 0, 0, tail, head, cap, M.L, st, &g));
    Mcf q;
    q.cost = cost;
    q.supply = supply;
    q.p = M.p;
    q.S = int64_t(n) + 1;
    q.w = M.w;
    const int ga = blocks_for(std::max(m, n)), gn = blocks_for(n);
    const int gp = blocks_for(std::max(m / 2, 1));
    // one wavefront per node: NTB / 64 nodes per block
    const int gw = int(std::min<int64_t>(4096, (int64_t(n) + NTB / 64 - 1) / (NTB / 64)));
    LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(M.w), 0, 8, st));
    hipLaunchKernelGGL(k_mcf_check, dim3(ga), dim3(NTB), 0, st, g, q);
    LPR_TRY_HIP(hipGetLastError());
    unsigned long long w[4];
    LPR_TRY_HIP(hipMemcpyAsync(w, M.w, sizeof(w), hipMemcpyDeviceToHost, st));
    LPR_TRY_HIP(hipStreamSynchronize(st));
    if (w[0] & 1) {
        set_error("cost[a ^ 1] != -cost[a] for some arc");
        return LPR_EINVAL;
    }
    if (w[0] & 2) {
        set_error("a cost above LPR_MCF_MAX_COST or a supply above LPR_MCF_MAX_SUPPLY");
        return LPR_ERANGE;
    }
    if (int64_t(w[2]) != 0) {
        set_error("supplies sum to %lld, not 0", (long long)int64_t(w[2]));
        return LPR_EINVAL;
    }
    // a feasible flow exists iff the supplies can all reach the demands
    if (w[3] > 0) {
        const int64_t fm = int64_t(m) + 4 * int64_t(n);
        hipLaunchKernelGGL(k_mcf_feas_arcs, dim3(blocks_for(std::max<int64_t>(m, n))),
                           dim3(NTB), 0, st, g, q, M.ft, M.fh, M.fc);
        LPR_TRY_HIP(hipGetLastError());
        int64_t routed = 0;
        const lpr_status fs =
            lpr_graph_maxflow(n + 2, int32_t(fm), M.ft, M.fh, M.fc, n, n + 1, &routed,
                              nullptr, nullptr, nullptr, M.fws, M.fbytes, stream);
        if (fs != LPR_OK) return fs;
        if (routed < int64_t(w[3])) {
            set_error("no feasible flow: %lld of %llu supply units can be routed",
                      (long long)routed, w[3]);
            return LPR_EINFEASIBLE;
        }
    }
    // Min-Cost: p = 0, eps = C (scaled), Refine until one at eps = 1 ends
    LPR_TRY(fill_i64(M.p, 0, n, st));
    LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(M.L.cnt), 0, 4, st));
    int64_t eps = int64_t(std::max<unsigned long long>(w[1], 1)) * q.S;
    int64_t refines = 0, iters = 0;
    unsigned long long cnt[4] = {0, 0, 0, 0};
    McfPasses passes;
    LPR_TRY(passes.capture(g, q, gw, gn, per_check));
    // A refine runs at most PU_MAX updates, each lowering a price by at most
    // eps x lcap; lcap (any positive cap keeps the labels valid) is 4n + 4
    // unless eps is so large that the drift could pass 2^50.
    constexpr int PU_MAX = 256, PU_EVERY = 1;  // updates per refine, checks between
    int32_t lcap = 4 * n + 4;
    auto price_update = [&]() -> lpr_status {
        hipLaunchKernelGGL(k_mcf_pu_init, dim3(gn), dim3(NTB), 0, st, g, M.d, lcap);
        int32_t fl[2] = {0, 0};
        bool fixpoint = false;
        // Bellman-Ford reaches its fixpoint within n rounds
        constexpr int ROUNDS = 16;  // relaxation rounds between host checks
        for (int64_t r = 0; r <= int64_t(n) + ROUNDS && !fixpoint; r += ROUNDS) {
            LPR_TRY(fill_i32(M.flags, 0, 2, st));
            for (int k = 0; k < ROUNDS; ++k)
                hipLaunchKernelGGL(k_mcf_pu_relax, dim3(gw), dim3(NTB), 0, st, g, q, M.d,
                                   lcap, M.flags);
            LPR_TRY_HIP(hipGetLastError());
            LPR_TRY_HIP(hipMemcpyAsync(fl, M.flags, sizeof(fl), hipMemcpyDeviceToHost, st));
            LPR_TRY_HIP(hipStreamSynchronize(st));
            fixpoint = fl[0] == 0;
        }
        if (!fixpoint) return LPR_OK;  // labels not final: leave the prices
        hipLaunchKernelGGL(k_mcf_pu_max, dim3(gn), dim3(NTB), 0, st, g, M.d, lcap,
                           M.flags + 1);
        hipLaunchKernelGGL(k_mcf_pu_apply, dim3(gn), dim3(NTB), 0, st, g, q, M.d, lcap,
                           M.flags + 1);
        LPR_TRY_HIP(hipGetLastError());
        return LPR_OK;
    };
    for (;;) {
        eps = std::max<int64_t>(1, eps / alpha);
        lcap = int32_t(std::max<int64_t>(
            1, std::min<int64_t>(4 * int64_t(n) + 4, (int64_t(1) << 50) / (eps * PU_MAX))));
        LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(M.w) + 5, eps, 1, st));
        hipLaunchKernelGGL(k_mcf_saturate, dim3(gp), dim3(NTB), 0, st, g, q);
        LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(M.L.cnt) + 2, 0, 1, st));
        hipLaunchKernelGGL(k_mcf_excess, dim3(gn), dim3(NTB), 0, st, g, q);
        LPR_TRY_HIP(hipGetLastError());
        int pu_done = 0, checks = 0;
        for (;;) {
            LPR_TRY_HIP(hipMemcpyAsync(cnt, M.L.cnt, sizeof(cnt), hipMemcpyDeviceToHost, st));
            LPR_TRY_HIP(hipStreamSynchronize(st));
            if (cnt[2] == 0) break;
            if (iters >= max_iters) {
                set_error("min-cost flow: pass budget (%lld) exhausted", (long long)max_iters);
                return LPR_EBUDGET;
            }
            if (pu_done < PU_MAX && checks % PU_EVERY == 0) {
                LPR_TRY(price_update());
                ++pu_done;
            }
            ++checks;
            LPR_TRY_HIP(hipGraphLaunch(passes.ex, st));
            iters += per_check;
        }
        ++refines;
        if (eps == 1) break;
    }
    LPR_TRY(fill_i64(reinterpret_cast<int64_t *>(M.w), 0, 1, st));
    hipLaunchKernelGGL(k_mcf_total, dim3(gp), dim3(NTB), 0, st, g, q, M.w);
    LPR_TRY_HIP(hipGetLastError());
    unsigned long long tot = 0;
    LPR_TRY_HIP(hipMemcpyAsync(&tot, M.w, sizeof(tot), hipMemcpyDeviceToHost, st));
    if (residual && m > 0)
        LPR_TRY_HIP(hipMemcpyAsync(residual, M.L.res, sizeof(int32_t) * size_t(m),
                                   hipMemcpyDeviceToDevice, st));
    if (prices)
        LPR_TRY_HIP(hipMemcpyAsync(prices, M.p, sizeof(int64_t) * size_t(n),
                                   hipMemcpyDeviceToDevice, st));
    double ms = 0;
    LPR_TRY(call.stop_ms(&ms));
    *total_cost = int64_t(tot);
    if (stats) {
        stats->refines = refines;
        stats->iterations = iters;
        stats->pushes = int64_t(cnt[0]);
        stats->relabels = int64_t(cnt[1]);
        stats->total_ms = ms;
    }
    return LPR_OK;
}
