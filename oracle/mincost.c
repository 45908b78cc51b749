/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.  Not part of the GPU library and
 * shares no code with it: only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.
 *
 *   oracle_mincost_flow -- minimum-cost flow with node supplies: the problem
 *       the cost-scaling method of Section 5 (Algorithm 5.0) solves, where
 *       every node v must end with excess 0 after starting from e(v) = d(v)
 *       (the supply d of Section 5's transportation reduction).  Solved by
 *       successive shortest paths: first every residual arc of negative cost
 *       is saturated (so the residual graph has no negative arc, hence no
 *       negative cycle), then, while some node has excess, a Dijkstra search
 *       with node potentials from all excess nodes finds a cheapest residual
 *       path to a node with a deficit and flow is sent along it.  A path of
 *       least reduced cost keeps every reduced cost non-negative, which is
 *       the textbook invariant of the method.
 *
 * Arcs come in mate pairs: arc a ^ 1 is the reverse of arc a, with
 * cost[a ^ 1] = -cost[a]; cap[a] and cap[a ^ 1] bound the flow in each
 * direction.  Outputs: the residual capacities res[a] (the net flow along a
 * is cap[a] - res[a]), the total cost, and the final potentials pi[v], for
 * which every residual arc has cost[a] + pi[tail] - pi[head] >= 0.
 * Returns 0, 1 when no flow meets the supplies, -1 for invalid input.
 */
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int64_t key;
    int v;
} item;

/* binary min-heap with lazy deletion */
static void heap_push(item *h, int *len, int64_t key, int v) {
    int i = (*len)++;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (h[p].key <= key) break;
        h[i] = h[p];
        i = p;
    }
    h[i].key = key;
    h[i].v = v;
}

static item heap_pop(item *h, int *len) {
    item top = h[0];
    item last = h[--(*len)];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, s = i;
        int64_t ks = last.key;
        if (l < *len && h[l].key < ks) {
            s = l;
            ks = h[l].key;
        }
        if (r < *len && h[r].key < ks) s = r;
        if (s == i) break;
        h[i] = h[s];
        i = s;
    }
    if (*len > 0) h[i] = last;
    return top;
}

int oracle_mincost_flow(int n, int m, const int32_t *tail, const int32_t *head,
                        const int64_t *cap, const int64_t *cost,
                        const int64_t *supply, int64_t *res, int64_t *total,
                        int64_t *pi) {
    if (n < 1 || m < 0 || (m & 1)) return -1;
    int64_t sum = 0;
    for (int v = 0; v < n; ++v) sum += supply[v];
    if (sum != 0) return -1;
    for (int a = 0; a < m; ++a) {
        if (tail[a] < 0 || tail[a] >= n || head[a] < 0 || head[a] >= n) return -1;
        if (tail[a ^ 1] != head[a] || head[a ^ 1] != tail[a]) return -1;
        if (cap[a] < 0 || cost[a ^ 1] != -cost[a]) return -1;
    }
    /* adjacency by tail */
    int *deg = (int *)calloc((size_t)n + 1, sizeof(int));
    int *adj = (int *)malloc(((size_t)m + 1) * sizeof(int));
    for (int a = 0; a < m; ++a) deg[tail[a] + 1]++;
    for (int v = 0; v < n; ++v) deg[v + 1] += deg[v];
    int *fill = (int *)malloc(((size_t)n + 1) * sizeof(int));
    for (int v = 0; v <= n; ++v) fill[v] = deg[v];
    for (int a = 0; a < m; ++a) adj[fill[tail[a]]++] = a;
    free(fill);

    int64_t *e = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    for (int v = 0; v < n; ++v) {
        e[v] = supply[v];
        pi[v] = 0;
    }
    for (int a = 0; a < m; ++a) res[a] = cap[a];
    /* saturate the negative arcs */
    for (int a = 0; a < m; ++a)
        if (cost[a] < 0 && res[a] > 0) {
            int64_t r = res[a];
            res[a] = 0;
            res[a ^ 1] += r;
            e[tail[a]] -= r;
            e[head[a]] += r;
        }

    const int64_t INF = INT64_MAX / 4;
    int64_t *dist = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int *via = (int *)malloc((size_t)n * sizeof(int)); /* arc into v, -1 at a source */
    uint8_t *done = (uint8_t *)malloc((size_t)n);
    item *heap = (item *)malloc(((size_t)m + (size_t)n + 1) * sizeof(item));
    int status = 0;
    for (;;) {
        int any = 0;
        for (int v = 0; v < n; ++v) {
            dist[v] = INF;
            via[v] = -1;
            done[v] = 0;
        }
        int len = 0;
        for (int v = 0; v < n; ++v)
            if (e[v] > 0) {
                any = 1;
                dist[v] = 0;
                heap_push(heap, &len, 0, v);
            }
        if (!any) break;
        /* Dijkstra on reduced costs cost + pi[u] - pi[w] >= 0 */
        while (len > 0) {
            item it = heap_pop(heap, &len);
            int u = it.v;
            if (done[u] || it.key != dist[u]) continue;
            done[u] = 1;
            for (int k = deg[u]; k < deg[u + 1]; ++k) {
                int a = adj[k];
                if (res[a] <= 0) continue;
                int w = head[a];
                int64_t d = dist[u] + cost[a] + pi[u] - pi[w];
                if (d < dist[w]) {
                    dist[w] = d;
                    via[w] = a;
                    heap_push(heap, &len, d, w);
                }
            }
        }
        /* the reached deficit node of least distance */
        int t = -1;
        int64_t dmax = 0;
        for (int v = 0; v < n; ++v) {
            if (dist[v] == INF) continue;
            if (dist[v] > dmax) dmax = dist[v];
            if (e[v] < 0 && (t < 0 || dist[v] < dist[t])) t = v;
        }
        if (t < 0) {
            status = 1; /* excess that cannot reach any deficit */
            break;
        }
        /* potentials: + distance (+ the largest distance where unreached) */
        for (int v = 0; v < n; ++v) pi[v] += dist[v] == INF ? dmax : dist[v];
        /* the path back to its excess node, and its bottleneck */
        int64_t delta = -e[t];
        int s = t;
        while (via[s] >= 0) {
            int a = via[s];
            if (res[a] < delta) delta = res[a];
            s = tail[a];
        }
        if (e[s] < delta) delta = e[s];
        for (int v = t; via[v] >= 0; v = tail[via[v]]) {
            int a = via[v];
            res[a] -= delta;
            res[a ^ 1] += delta;
        }
        e[s] -= delta;
        e[t] += delta;
    }
    int64_t tot = 0;
    for (int a = 0; a < m; a += 2) tot += (cap[a] - res[a]) * cost[a];
    *total = tot;
    free(deg);
    free(adj);
    free(e);
    free(dist);
    free(via);
    free(done);
    free(heap);
    return status;
}
