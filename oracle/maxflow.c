/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded reference implementations of s-t maximum flow on an
 * explicit arc list, used to check the GPU library.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load this code; the
 * product path never does.  Nothing here is shared with the HIP library.
 *
 * Graph representation: nodes 0..n-1, arcs 0..m-1 stored in mate pairs
 * (arc a and arc a^1 are each other's reverse).  cap[a] >= 0 is the capacity
 * u(tail[a], head[a]); the residual capacity is u_f = u - f with the skew
 * symmetric pseudoflow f (flow network and residual definitions, Section 3).
 *
 * Functions:
 *   oracle_maxflow_ek   -- Edmonds-Karp (BFS augmenting paths, Section 4.1);
 *                          returns |f*| and reach(s) in the final residual
 *                          graph, which is the minimal source side of a min cut.
 *   oracle_maxflow_fifo -- generic push-relabel (Algorithms 4.2 and 4.3) with
 *                          the Init of Algorithm 4.7, S kept as a FIFO queue,
 *                          global relabelling (Algorithm 4.4) once every |V|
 *                          relabels and the gap step after each BFS (Section
 *                          4.2).  It stops at a maximum preflow (nodes with
 *                          h >= |V| are never discharged, as in Algorithm 4.8),
 *                          returns e(t) and the minimal source side computed
 *                          as the residual closure of {s} u {v : e(v) > 0}.
 *
 * Parity pins for both live in the tests: brute-force minimum cuts on grids
 * of at most 9 pixels, scipy's maximum_flow, closed forms and metamorphic
 * relations.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n, m;
    int *first;   /* CSR offsets over arcs grouped by tail, size n+1 */
    int *adj;     /* arc ids sorted by tail */
} csr_t;

static int build_csr(int n, int m, const int32_t *tail, csr_t *g) {
    g->n = n;
    g->m = m;
    g->first = (int *)calloc((size_t)n + 1, sizeof(int));
    g->adj = (int *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int));
    if (!g->first || !g->adj) return -1;
    for (int a = 0; a < m; ++a) g->first[tail[a] + 1]++;
    for (int v = 0; v < n; ++v) g->first[v + 1] += g->first[v];
    int *fill = (int *)malloc((size_t)n * sizeof(int));
    if (!fill) return -1;
    memcpy(fill, g->first, (size_t)n * sizeof(int));
    for (int a = 0; a < m; ++a) g->adj[fill[tail[a]]++] = a;
    free(fill);
    return 0;
}

static void free_csr(csr_t *g) {
    free(g->first);
    free(g->adj);
}

static int check_input(int n, int m, const int32_t *tail, const int32_t *head,
                       const int64_t *cap, int s, int t) {
    if (n < 2 || m < 0 || (m & 1) || s < 0 || s >= n || t < 0 || t >= n || s == t)
        return -1;
    for (int a = 0; a < m; ++a) {
        if (tail[a] < 0 || tail[a] >= n || head[a] < 0 || head[a] >= n) return -1;
        if (cap[a] < 0) return -1;
        if (tail[a ^ 1] != head[a] || head[a ^ 1] != tail[a]) return -1;
    }
    return 0;
}

/* Residual closure of the nodes marked in `side` (forward over arcs with
 * r > 0).  Plain BFS. */
static void residual_closure(const csr_t *g, const int32_t *head,
                             const int64_t *r, uint8_t *side) {
    int n = g->n;
    int *queue = (int *)malloc((size_t)n * sizeof(int));
    int qh = 0, qt = 0;
    for (int v = 0; v < n; ++v)
        if (side[v]) queue[qt++] = v;
    while (qh < qt) {
        int x = queue[qh++];
        for (int k = g->first[x]; k < g->first[x + 1]; ++k) {
            int a = g->adj[k];
            int y = head[a];
            if (r[a] > 0 && !side[y]) {
                side[y] = 1;
                queue[qt++] = y;
            }
        }
    }
    free(queue);
}

/* ------------------------------------------------------------------------- */
/* Edmonds-Karp: repeatedly find a shortest s-t path in the residual graph    */
/* by BFS and augment along it by its bottleneck residual capacity.           */
/* ------------------------------------------------------------------------- */
int oracle_maxflow_ek(int n, int m, const int32_t *tail, const int32_t *head,
                      const int64_t *cap, int s, int t, int64_t *flow_value,
                      uint8_t *source_side) {
    if (check_input(n, m, tail, head, cap, s, t)) return -1;
    csr_t g;
    if (build_csr(n, m, tail, &g)) return -2;
    int64_t *r = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int *pred = (int *)malloc((size_t)n * sizeof(int));
    int *queue = (int *)malloc((size_t)n * sizeof(int));
    for (int a = 0; a < m; ++a) r[a] = cap[a];
    int64_t value = 0;
    for (;;) {
        for (int v = 0; v < n; ++v) pred[v] = -2;
        pred[s] = -1;
        int qh = 0, qt = 0;
        queue[qt++] = s;
        while (qh < qt && pred[t] == -2) {
            int x = queue[qh++];
            for (int k = g.first[x]; k < g.first[x + 1]; ++k) {
                int a = g.adj[k];
                int y = head[a];
                if (r[a] > 0 && pred[y] == -2) {
                    pred[y] = a;
                    queue[qt++] = y;
                }
            }
        }
        if (pred[t] == -2) break;
        int64_t delta = INT64_MAX;
        for (int v = t; v != s; v = tail[pred[v]])
            if (r[pred[v]] < delta) delta = r[pred[v]];
        for (int v = t; v != s; v = tail[pred[v]]) {
            r[pred[v]] -= delta;
            r[pred[v] ^ 1] += delta;
        }
        value += delta;
    }
    *flow_value = value;
    if (source_side) {
        memset(source_side, 0, (size_t)n);
        source_side[s] = 1;
        residual_closure(&g, head, r, source_side);
    }
    free(r);
    free(pred);
    free(queue);
    free_csr(&g);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* FIFO push-relabel.                                                          */
/* ------------------------------------------------------------------------- */
typedef struct {
    int n, s, t;
    const csr_t *g;
    const int32_t *tail, *head;
    int64_t *r;     /* residual capacity per arc */
    int64_t *e;     /* excess per node */
    int64_t *h;     /* height per node */
    int *queue;     /* circular FIFO of active nodes (set S) */
    uint8_t *inq;
    int qh, qlen;
    int64_t pushes, relabels, global_relabels;
} pr_t;

static void q_push(pr_t *P, int v) {
    if (P->inq[v]) return;
    P->inq[v] = 1;
    P->queue[(P->qh + P->qlen) % P->n] = v;
    P->qlen++;
}

static int q_pop(pr_t *P) {
    int v = P->queue[P->qh];
    P->qh = (P->qh + 1) % P->n;
    P->qlen--;
    P->inq[v] = 0;
    return v;
}

static int is_active(const pr_t *P, int v) {
    return v != P->s && v != P->t && P->e[v] > 0 && P->h[v] < P->n;
}

/* Algorithm 4.4 followed by the gap step: backward BFS from t over residual
 * arcs assigns h = BFS level; nodes that were not scanned cannot reach t and
 * get h = |V|.  h(s) stays |V|.  Afterwards S is rebuilt from scratch. */
static void global_relabel(pr_t *P) {
    int n = P->n;
    int *bfs = (int *)malloc((size_t)n * sizeof(int));
    uint8_t *scanned = (uint8_t *)calloc((size_t)n, 1);
    int qh = 0, qt = 0;
    for (int v = 0; v < n; ++v) P->h[v] = n;
    P->h[P->t] = 0;
    scanned[P->t] = 1;
    scanned[P->s] = 1; /* the source keeps height |V| */
    bfs[qt++] = P->t;
    while (qh < qt) {
        int x = bfs[qh++];
        int64_t current = P->h[x] + 1;
        /* residual arcs (y, x): the mates of the arcs leaving x */
        for (int k = P->g->first[x]; k < P->g->first[x + 1]; ++k) {
            int a = P->g->adj[k];
            int y = P->head[a];
            if (P->r[a ^ 1] > 0 && !scanned[y]) {
                P->h[y] = current;
                scanned[y] = 1;
                bfs[qt++] = y;
            }
        }
    }
    free(bfs);
    free(scanned);
    P->qh = 0;
    P->qlen = 0;
    memset(P->inq, 0, (size_t)n);
    for (int v = 0; v < n; ++v)
        if (is_active(P, v)) q_push(P, v);
    P->global_relabels++;
}

int oracle_maxflow_fifo(int n, int m, const int32_t *tail, const int32_t *head,
                        const int64_t *cap, int s, int t, int64_t *flow_value,
                        uint8_t *source_side, int64_t *stats /* [3] or NULL */) {
    if (check_input(n, m, tail, head, cap, s, t)) return -1;
    csr_t g;
    if (build_csr(n, m, tail, &g)) return -2;
    pr_t P;
    memset(&P, 0, sizeof(P));
    P.n = n;
    P.s = s;
    P.t = t;
    P.g = &g;
    P.tail = tail;
    P.head = head;
    P.r = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    P.e = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    P.h = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    P.queue = (int *)malloc((size_t)n * sizeof(int));
    P.inq = (uint8_t *)calloc((size_t)n, 1);

    /* Init (Algorithm 4.7): u_f = u on every arc, h(s) = |V|, then saturate
     * every arc leaving s: u_f(s,x) = 0, u_f(x,s) += u_sx, e(x) += u_sx. */
    for (int a = 0; a < m; ++a) P.r[a] = cap[a];
    P.h[s] = n;
    for (int k = g.first[s]; k < g.first[s + 1]; ++k) {
        int a = g.adj[k];
        int64_t d = P.r[a];
        if (d <= 0) continue;
        P.r[a] = 0;
        P.r[a ^ 1] += d;
        P.e[head[a]] += d;
        P.e[s] -= d;
    }
    global_relabel(&P);

    int64_t relabels_since_global = 0;
    while (P.qlen > 0) {
        int x = q_pop(&P);
        if (!is_active(&P, x)) continue;
        /* discharge(x), Algorithm 4.3: push along a residual arc with
         * h(x) = h(y) + 1 if one exists, else relabel. */
        int push_arc = -1;
        int64_t hmin = INT64_MAX;
        for (int k = g.first[x]; k < g.first[x + 1]; ++k) {
            int a = g.adj[k];
            if (P.r[a] <= 0) continue;
            int y = head[a];
            if (P.h[x] == P.h[y] + 1) {
                push_arc = a;
                break;
            }
            if (P.h[y] < hmin) hmin = P.h[y];
        }
        if (push_arc >= 0) {
            int y = head[push_arc];
            int64_t delta = P.r[push_arc] < P.e[x] ? P.r[push_arc] : P.e[x];
            P.e[x] -= delta;
            P.e[y] += delta;
            P.r[push_arc] -= delta;
            P.r[push_arc ^ 1] += delta;
            P.pushes++;
            if (is_active(&P, y)) q_push(&P, y);
        } else {
            /* relabel(x): h(x) = min{h(y) : (x,y) in E_f} + 1.  A node with
             * positive excess always has a residual arc back along the path
             * its excess arrived on. */
            P.h[x] = (hmin == INT64_MAX) ? n : hmin + 1;
            if (P.h[x] > n) P.h[x] = n;
            P.relabels++;
            relabels_since_global++;
        }
        if (relabels_since_global >= n) {
            relabels_since_global = 0;
            global_relabel(&P);
            continue;
        }
        if (is_active(&P, x)) q_push(&P, x);
    }

    *flow_value = P.e[t];
    if (source_side) {
        /* Minimal source side of a minimum cut from a maximum preflow: the
         * residual closure of {s} together with every node holding excess. */
        memset(source_side, 0, (size_t)n);
        source_side[s] = 1;
        for (int v = 0; v < n; ++v)
            if (v != t && P.e[v] > 0) source_side[v] = 1;
        residual_closure(&g, head, P.r, source_side);
    }
    if (stats) {
        stats[0] = P.pushes;
        stats[1] = P.relabels;
        stats[2] = P.global_relabels;
    }
    free(P.r);
    free(P.e);
    free(P.h);
    free(P.queue);
    free(P.inq);
    free_csr(&g);
    return 0;
}
