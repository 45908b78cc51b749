/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain reference implementations for the dense assignment problem (a
 * perfect matching of minimum total cost in the complete bipartite graph
 * X x Y, |X| = |Y| = n; Section 3).  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load this code.  Nothing here is
 * shared with the HIP library.
 *
 *   oracle_hungarian     -- the O(n^3) Hungarian method (shortest augmenting
 *                           paths with row/column potentials).  A textbook
 *                           method, not the paper's; it returns the optimal
 *                           assignment, its cost and integer duals (u, v) with
 *                           u_i + v_j <= c_ij everywhere, equality on the
 *                           assignment and sum(u) + sum(v) = cost.
 *   oracle_cost_scaling  -- the paper's cost-scaling method run sequentially:
 *                           the outer epsilon loop of Algorithm 5.0 around the
 *                           Refine of Algorithm 5.2 (f <- 0, then
 *                           p(x) <- -min_y {c'_p(x,y) + eps} on X), with the
 *                           push / relabel operation of Algorithm 5.4 applied
 *                           to one active node at a time from a FIFO queue.
 *                           Costs are integers scaled by S = 2n+1 and the last
 *                           refine runs at eps = 1, i.e. eps = 1/(2n+1) < 1/n
 *                           in original units.
 *
 * All costs are int32 in memory and handled as int64 arithmetic; prices are
 * int64.  Maximisation (the problem as stated in Section 3) is solved as
 * minimisation of the negated weights by the Python wrapper.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define INF64 (INT64_MAX / 4)

/* Hungarian method.  Rows are inserted one at a time; for the new row a
 * Dijkstra search over reduced costs c_ij - u_i - v_j (all >= 0) finds the
 * cheapest augmenting path, the potentials are shifted by the search
 * distances, and the path is flipped.  Column index n is a virtual column
 * that holds the row being inserted. */
int oracle_hungarian(int n, const int32_t *cost, int32_t *row_to_col,
                     int64_t *total, int64_t *u_out, int64_t *v_out) {
    if (n < 1) return -1;
    int64_t *u = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t *v = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int *col_row = (int *)malloc(((size_t)n + 1) * sizeof(int));
    int *way = (int *)malloc(((size_t)n + 1) * sizeof(int));
    int64_t *minv = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    uint8_t *used = (uint8_t *)malloc((size_t)n + 1);
    for (int j = 0; j <= n; ++j) col_row[j] = -1;

    for (int i = 0; i < n; ++i) {
        int j0 = n; /* virtual column */
        col_row[n] = i;
        for (int j = 0; j <= n; ++j) {
            minv[j] = INF64;
            used[j] = 0;
            way[j] = -1;
        }
        do {
            used[j0] = 1;
            int i0 = col_row[j0];
            int64_t delta = INF64;
            int j1 = -1;
            for (int j = 0; j < n; ++j) {
                if (used[j]) continue;
                int64_t cur = (int64_t)cost[(size_t)i0 * n + j] - u[i0] - v[j];
                if (cur < minv[j]) {
                    minv[j] = cur;
                    way[j] = j0;
                }
                if (minv[j] < delta) {
                    delta = minv[j];
                    j1 = j;
                }
            }
            for (int j = 0; j <= n; ++j) {
                if (used[j]) {
                    u[col_row[j]] += delta;
                    if (j < n) v[j] -= delta;
                } else {
                    minv[j] -= delta;
                }
            }
            j0 = j1;
        } while (col_row[j0] != -1);
        /* flip the augmenting path */
        while (j0 != n) {
            int jp = way[j0];
            col_row[j0] = col_row[jp];
            j0 = jp;
        }
    }
    int64_t sum = 0;
    for (int j = 0; j < n; ++j) {
        row_to_col[col_row[j]] = j;
        sum += cost[(size_t)col_row[j] * n + j];
    }
    *total = sum;
    if (u_out) memcpy(u_out, u, (size_t)n * sizeof(int64_t));
    if (v_out) memcpy(v_out, v, (size_t)n * sizeof(int64_t));
    free(u);
    free(v);
    free(col_row);
    free(way);
    free(minv);
    free(used);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Sequential cost scaling with the refine of Algorithm 5.2.                  */
/*                                                                            */
/* Flow network of the reduction in Section 5: arcs (x,y) with u = 1 and      */
/* cost c(x,y), their reverses (y,x) with u = 0 and cost -c(x,y); excesses    */
/* start at e(x) = 1 on X and e(y) = -1 on Y.  Since unit capacities are used,*/
/* the pseudoflow is the set of matched pairs: each x carries flow on at most */
/* one arc (mate[x], or -1), while a y may hold several x during a refine.   */
/* ------------------------------------------------------------------------- */
typedef struct {
    int n;
    const int64_t *cs;   /* scaled costs, n*n */
    int64_t *p;          /* prices: p[0..n) for X, p[n..2n) for Y */
    int64_t *e;          /* excesses, same indexing */
    int *mate;           /* mate[x] = y or -1 */
    int *queue;          /* FIFO of active nodes */
    uint8_t *inq;
    int qh, qlen;
    int64_t pushes, relabels;
} cs_t;

static void cs_enqueue(cs_t *C, int v) {
    if (C->inq[v]) return;
    C->inq[v] = 1;
    C->queue[(C->qh + C->qlen) % (2 * C->n)] = v;
    C->qlen++;
}

static int cs_dequeue(cs_t *C) {
    int v = C->queue[C->qh];
    C->qh = (C->qh + 1) % (2 * C->n);
    C->qlen--;
    C->inq[v] = 0;
    return v;
}

/* One push or relabel on an active node (Algorithm 5.4 semantics): find the
 * residual arc of least part-reduced cost c'_p(v,w) = c(v,w) - p(w) (ties go
 * to the smallest w); push one unit along it if c'_p + p(v) < 0, otherwise set
 * p(v) <- -(c'_p + eps).  Returns the node that received the unit, or -1. */
static int cs_operate(cs_t *C, int v, int64_t eps) {
    int n = C->n;
    int64_t best = INF64;
    int arg = -1;
    if (v < n) {
        /* x is active iff unmatched, so every arc (x,y) is residual */
        const int64_t *row = C->cs + (size_t)v * n;
        for (int y = 0; y < n; ++y) {
            int64_t cp = row[y] - C->p[n + y];
            if (cp < best) {
                best = cp;
                arg = y;
            }
        }
        if (best + C->p[v] < 0) {
            C->mate[v] = arg;
            C->e[v] -= 1;
            C->e[n + arg] += 1;
            C->pushes++;
            return n + arg;
        }
    } else {
        /* residual arcs of y are the reverses (y,x) of matched pairs */
        int y = v - n;
        for (int x = 0; x < n; ++x) {
            if (C->mate[x] != y) continue;
            int64_t cp = -C->cs[(size_t)x * n + y] - C->p[x];
            if (cp < best) {
                best = cp;
                arg = x;
            }
        }
        if (arg < 0) return -1; /* cannot happen for an active y */
        if (best + C->p[v] < 0) {
            C->mate[arg] = -1;
            C->e[v] -= 1;
            C->e[arg] += 1;
            C->pushes++;
            return arg;
        }
    }
    C->p[v] = -(best + eps);
    C->relabels++;
    return -1;
}

/* Refine(eps) of Algorithm 5.2, eps already divided by alpha by the caller. */
static void cs_refine(cs_t *C, int64_t eps) {
    int n = C->n;
    for (int x = 0; x < n; ++x) {
        C->mate[x] = -1;
        C->e[x] = 1;
        C->e[n + x] = -1;
    }
    for (int x = 0; x < n; ++x) {
        int64_t mn = INF64;
        const int64_t *row = C->cs + (size_t)x * n;
        for (int y = 0; y < n; ++y) {
            int64_t cp = row[y] - C->p[n + y];
            if (cp < mn) mn = cp;
        }
        C->p[x] = -(mn + eps);
    }
    C->qh = 0;
    C->qlen = 0;
    memset(C->inq, 0, (size_t)2 * n);
    for (int x = 0; x < n; ++x) cs_enqueue(C, x);
    while (C->qlen > 0) {
        int v = cs_dequeue(C);
        if (C->e[v] <= 0) continue;
        int w = cs_operate(C, v, eps);
        if (w >= 0 && C->e[w] > 0) cs_enqueue(C, w);
        if (C->e[v] > 0) cs_enqueue(C, v);
    }
}

/* Min-Cost of Algorithm 5.0 with the scaling reading: scaled costs
 * cs = c * (2n+1); eps0 = max|c| * (2n+1) (or 1 if all costs are 0); repeat
 * { eps <- max(1, floor(eps / alpha)); Refine(eps) } until a refine at eps = 1
 * has run.  p starts at 0 unless init_prices (scaled, Y only) is given. */
int oracle_cost_scaling(int n, const int32_t *cost, int alpha,
                        const int64_t *init_col_prices, int64_t eps_start,
                        int32_t *row_to_col, int64_t *total,
                        int64_t *col_prices, int64_t *stats /* [3] */) {
    if (n < 1 || alpha < 2) return -1;
    int64_t S = 2 * (int64_t)n + 1;
    int64_t C = 0;
    size_t nn = (size_t)n * n;
    int64_t *cs = (int64_t *)malloc(nn * sizeof(int64_t));
    for (size_t k = 0; k < nn; ++k) {
        int64_t c = cost[k];
        cs[k] = c * S;
        if (c < 0) c = -c;
        if (c > C) C = c;
    }
    cs_t Cx;
    memset(&Cx, 0, sizeof(Cx));
    Cx.n = n;
    Cx.cs = cs;
    Cx.p = (int64_t *)calloc((size_t)2 * n, sizeof(int64_t));
    Cx.e = (int64_t *)calloc((size_t)2 * n, sizeof(int64_t));
    Cx.mate = (int *)malloc((size_t)n * sizeof(int));
    Cx.queue = (int *)malloc((size_t)2 * n * sizeof(int));
    Cx.inq = (uint8_t *)calloc((size_t)2 * n, 1);
    if (init_col_prices)
        for (int y = 0; y < n; ++y) Cx.p[n + y] = init_col_prices[y];
    int64_t eps = eps_start > 0 ? eps_start : (C > 0 ? C * S : 1);
    int64_t refines = 0;
    for (;;) {
        eps = eps / alpha;
        if (eps < 1) eps = 1;
        cs_refine(&Cx, eps);
        refines++;
        if (eps == 1) break;
    }
    int64_t sum = 0;
    for (int x = 0; x < n; ++x) {
        row_to_col[x] = Cx.mate[x];
        sum += cost[(size_t)x * n + Cx.mate[x]];
    }
    *total = sum;
    if (col_prices) memcpy(col_prices, Cx.p + n, (size_t)n * sizeof(int64_t));
    if (stats) {
        stats[0] = Cx.pushes;
        stats[1] = Cx.relabels;
        stats[2] = refines;
    }
    free(cs);
    free(Cx.p);
    free(Cx.e);
    free(Cx.mate);
    free(Cx.queue);
    free(Cx.inq);
    return 0;
}
