/*
 * CPU oracle for the exact surface max-flow.  TEST INFRASTRUCTURE ONLY:
 * nothing on the product path may link, load or call this file; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg do.
 *
 * It computes, by the plain definitions and in int64 throughout:
 *   - the s-t graph G(c, delta) of a cost volume c[x][y][z] (z fastest),
 *     built explicitly as a CSR arc list (Section 1.2: node weights become
 *     terminal arc capacities; columns are joined by infinite arcs down the
 *     column and to the adjacent columns within the smoothness bound);
 *   - a maximum flow by Dinic's blocking-flow method (Section 2: level graph
 *     from a BFS out of the source, blocking flow along level-increasing
 *     residual arcs, repeated until the sink is unreachable);
 *   - the flow value |f| = sum of flow into the sink (Eq. 5);
 *   - the source side S_min of the inclusion-minimal minimum cut = the set
 *     reachable from s in the residual graph, its capacity (Eq. 6), and
 *     the complement of the set that reaches t (the maximal min cut);
 *   - the surfaces h_min(p) = max{z : (p,z) in S_min}, h_max likewise, and
 *     E* = sum_p c(p, h_min(p)) (Eq. 1, feature term; plus the smoothness
 *     term below when alpha > 0);
 *   - self-checks of the capacity and conservation constraints (Eqs. 2-4)
 *     and of max-flow = min-cut (Theorem 1.1).
 *
 * Graph (the paper describes it only in words, Section 1.2; the concrete
 * form used here):
 *   B = max_p c(p,0) + 1;  w(p,0) = c(p,0) - B;  w(p,z) = c(p,z) - c(p,z-1).
 *   s -> v with capacity -w(v) when w(v) < 0;  v -> t with capacity w(v) when
 *   w(v) > 0;  (p,z) -> (p,z-1) infinite for z >= 1;  (p,z) -> (q, max(0,
 *   z - delta)) infinite for every 4-neighbour q of p inside the grid.
 * Arcs leaving the grid do not exist (Section 3.3: boundary arcs have zero
 * capacity).
 *
 * Soft smoothness (the edge costs of the VCE-weight net surface, Section
 * 1.2, with the convex cost alpha * |h(p) - h(q)| inside the edge
 * interval): with alpha > 0 every 4-neighbour pair also gets the arcs
 * (p,z) -> (q,z) of capacity alpha for z >= 1.  A closed set with column
 * heights h cuts max(0, h(p) - h(q)) of them from p to q, so a cut costs
 * alpha * sum over neighbour pairs of |h(p) - h(q)| more, and the reported
 * energies include that term.
 *
 * Written from the definitions; shares no code with the GPU library.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_INF (INT64_MAX / 4)

typedef struct {
    int64_t n;        /* nodes: voxels + s + t */
    int64_t m;        /* arcs (each with a paired reverse arc) */
    int64_t *first;   /* CSR row starts, size n+1 */
    int64_t *head;    /* arc head node */
    int64_t *res;     /* residual capacity */
    int64_t *rev;     /* index of the paired arc */
    uint8_t *fwd;     /* 1 for an arc of G, 0 for its added reverse */
} or_graph;

typedef struct {
    int64_t flow;          /* |f| */
    int64_t cut;           /* capacity of (S_min, complement) by Eq. 6 */
    int64_t energy;        /* sum_p c(p, h_min(p)) */
    int64_t energy_hmax;   /* sum_p c(p, h_max(p)) */
    int64_t wminus;        /* total source capacity */
    int64_t phases;        /* Dinic BFS phases */
    int32_t conservation_ok;
    int32_t capacity_ok;
    int32_t smin_in_smax;  /* S_min is a subset of S_max */
    int32_t status;        /* 0 ok, <0 allocation or argument failure */
} or_result;

static int64_t node_id(int64_t x, int64_t y, int64_t z, int64_t ny, int64_t K)
{
    return (x * ny + y) * K + z;
}

static void free_graph(or_graph *g)
{
    free(g->first); free(g->head); free(g->res); free(g->rev); free(g->fwd);
    memset(g, 0, sizeof(*g));
}

/* Calls fn(tail, head, cap) for every arc of G(c, delta). */
typedef void (*arc_fn)(void *ctx, int64_t u, int64_t v, int64_t cap);

static void for_each_arc(const int32_t *c, int64_t nx, int64_t ny, int64_t K,
                         int64_t delta, int64_t alpha, arc_fn fn, void *ctx)
{
    const int64_t N = nx * ny * K, s = N, t = N + 1;
    int64_t B = INT64_MIN;
    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y) {
            int64_t c0 = c[node_id(x, y, 0, ny, K)];
            if (c0 > B) B = c0;
        }
    B += 1;
    static const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t z = 0; z < K; ++z) {
                int64_t v = node_id(x, y, z, ny, K);
                int64_t w = (z == 0) ? (int64_t)c[v] - B
                                     : (int64_t)c[v] - (int64_t)c[v - 1];
                if (w < 0) fn(ctx, s, v, -w);
                if (w > 0) fn(ctx, v, t, w);
                if (z >= 1) fn(ctx, v, v - 1, OR_INF);
                int64_t zt = z - delta < 0 ? 0 : z - delta;
                for (int d = 0; d < 4; ++d) {
                    int64_t qx = x + dx[d], qy = y + dy[d];
                    if (qx < 0 || qx >= nx || qy < 0 || qy >= ny) continue;
                    fn(ctx, v, node_id(qx, qy, zt, ny, K), OR_INF);
                    if (alpha > 0 && z >= 1) fn(ctx, v, node_id(qx, qy, z, ny, K), alpha);
                }
            }
}

typedef struct { or_graph *g; int64_t *fill; } build_ctx;

static void count_arc(void *ctx, int64_t u, int64_t v, int64_t cap)
{
    (void)cap;
    or_graph *g = ((build_ctx *)ctx)->g;
    g->first[u + 1] += 1;
    g->first[v + 1] += 1;
}

static void place_arc(void *ctx, int64_t u, int64_t v, int64_t cap)
{
    build_ctx *b = (build_ctx *)ctx;
    or_graph *g = b->g;
    int64_t a = b->fill[u]++, r = b->fill[v]++;
    g->head[a] = v; g->res[a] = cap; g->rev[a] = r; g->fwd[a] = 1;
    g->head[r] = u; g->res[r] = 0;   g->rev[r] = a; g->fwd[r] = 0;
}

static int build_graph(or_graph *g, const int32_t *c, int64_t nx, int64_t ny,
                       int64_t K, int64_t delta, int64_t alpha)
{
    memset(g, 0, sizeof(*g));
    g->n = nx * ny * K + 2;
    g->first = calloc((size_t)g->n + 1, sizeof(int64_t));
    if (!g->first) return -1;
    build_ctx b = {g, NULL};
    for_each_arc(c, nx, ny, K, delta, alpha, count_arc, &b);
    for (int64_t i = 0; i < g->n; ++i) g->first[i + 1] += g->first[i];
    g->m = g->first[g->n];
    g->head = malloc((size_t)g->m * sizeof(int64_t));
    g->res = malloc((size_t)g->m * sizeof(int64_t));
    g->rev = malloc((size_t)g->m * sizeof(int64_t));
    g->fwd = malloc((size_t)g->m);
    b.fill = malloc((size_t)g->n * sizeof(int64_t));
    if (!g->head || !g->res || !g->rev || !g->fwd || !b.fill) {
        free(b.fill); free_graph(g); return -1;
    }
    memcpy(b.fill, g->first, (size_t)g->n * sizeof(int64_t));
    for_each_arc(c, nx, ny, K, delta, alpha, place_arc, &b);
    free(b.fill);
    return 0;
}

/* Breadth-first levels from s over arcs with positive residual capacity. */
static int bfs_levels(const or_graph *g, int64_t s, int64_t t, int64_t *level,
                      int64_t *queue)
{
    for (int64_t i = 0; i < g->n; ++i) level[i] = -1;
    int64_t qh = 0, qt = 0;
    level[s] = 0; queue[qt++] = s;
    while (qh < qt) {
        int64_t u = queue[qh++];
        for (int64_t a = g->first[u]; a < g->first[u + 1]; ++a) {
            int64_t v = g->head[a];
            if (g->res[a] > 0 && level[v] < 0) {
                level[v] = level[u] + 1;
                queue[qt++] = v;
            }
        }
    }
    return level[t] >= 0;
}

/* One blocking flow in the level graph, by repeated depth-first search with
 * current-arc pointers, written iteratively (paths can be as long as n). */
static int64_t blocking_flow(or_graph *g, int64_t s, int64_t t, int64_t *level,
                             int64_t *cur, int64_t *path)
{
    int64_t total = 0, depth = 0, u = s;
    memcpy(cur, g->first, (size_t)g->n * sizeof(int64_t));
    for (;;) {
        if (u == t) {
            int64_t push = OR_INF;
            for (int64_t i = 0; i < depth; ++i)
                if (g->res[path[i]] < push) push = g->res[path[i]];
            int64_t back = -1;
            for (int64_t i = 0; i < depth; ++i) {
                int64_t a = path[i];
                g->res[a] -= push;
                g->res[g->rev[a]] += push;
                if (back < 0 && g->res[a] == 0) back = i;
            }
            total += push;
            depth = back;                   /* retreat to the first saturated arc's tail */
            u = depth == 0 ? s : g->head[path[depth - 1]];
            continue;
        }
        int64_t a = cur[u], end = g->first[u + 1];
        while (a < end && !(g->res[a] > 0 && level[g->head[a]] == level[u] + 1)) ++a;
        cur[u] = a;
        if (a < end) {
            path[depth++] = a;
            u = g->head[a];
        } else {
            level[u] = -1;                  /* dead end: drop u from the level graph */
            if (depth == 0) break;
            --depth;
            u = depth == 0 ? s : g->head[path[depth - 1]];
            cur[u] += 1;
        }
    }
    return total;
}

/* Marks nodes reachable from `src` along residual arcs (forward search). */
static void reach_from(const or_graph *g, int64_t src, uint8_t *mark, int64_t *queue)
{
    memset(mark, 0, (size_t)g->n);
    int64_t qh = 0, qt = 0;
    mark[src] = 1; queue[qt++] = src;
    while (qh < qt) {
        int64_t u = queue[qh++];
        for (int64_t a = g->first[u]; a < g->first[u + 1]; ++a) {
            int64_t v = g->head[a];
            if (g->res[a] > 0 && !mark[v]) { mark[v] = 1; queue[qt++] = v; }
        }
    }
}

/* Marks nodes that can reach `dst` along residual arcs (backward search). */
static void reach_to(const or_graph *g, int64_t dst, uint8_t *mark, int64_t *queue)
{
    memset(mark, 0, (size_t)g->n);
    int64_t qh = 0, qt = 0;
    mark[dst] = 1; queue[qt++] = dst;
    while (qh < qt) {
        int64_t v = queue[qh++];
        for (int64_t a = g->first[v]; a < g->first[v + 1]; ++a) {
            int64_t u = g->head[a];           /* residual arc u -> v is rev[a] */
            if (g->res[g->rev[a]] > 0 && !mark[u]) { mark[u] = 1; queue[qt++] = u; }
        }
    }
}

/* alpha * sum over 4-neighbour column pairs of |h(p) - h(q)|. */
static int64_t smooth_term(const int32_t *h, int64_t nx, int64_t ny, int64_t alpha)
{
    int64_t sum = 0;
    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y) {
            const int64_t a = h[x * ny + y];
            if (x + 1 < nx) sum += llabs(a - h[(x + 1) * ny + y]);
            if (y + 1 < ny) sum += llabs(a - h[x * ny + y + 1]);
        }
    return alpha * sum;
}

/*
 * Max flow of g by Dinic's method (s = N, t = N + 1), the self-checks of
 * the capacity and conservation constraints (Eqs. 2-4) and of max-flow =
 * min-cut (Theorem 1.1), and the residual reach sets: sreach[v] = v is
 * reached from s (S_min), treach[v] = v reaches t (outside S_max).  Fills
 * flow, cut, wminus, phases and the check flags of out; h and energies are
 * left to the caller.  Returns 0, or -2 when memory runs out.
 */
static int max_flow_cuts(or_graph *g, int64_t N, uint8_t *sreach, uint8_t *treach, or_result *out)
{
    const int64_t s = N, t = N + 1;
    int64_t *level = malloc((size_t)g->n * sizeof(int64_t));
    int64_t *cur = malloc((size_t)g->n * sizeof(int64_t));
    int64_t *buf = malloc((size_t)g->n * sizeof(int64_t));
    int64_t *orig = malloc((size_t)g->m * sizeof(int64_t));
    if (!level || !cur || !buf || !orig) {
        free(level); free(cur); free(buf); free(orig);
        return -2;
    }
    memcpy(orig, g->res, (size_t)g->m * sizeof(int64_t));
    for (int64_t a = g->first[s]; a < g->first[s + 1]; ++a)
        if (g->fwd[a]) out->wminus += orig[a];

    while (bfs_levels(g, s, t, level, buf)) {
        out->phases += 1;
        out->flow += blocking_flow(g, s, t, level, cur, buf);
    }

    /* Capacity (Eq. 2) and conservation (Eq. 4) of the final flow; the flow
     * on an arc of G is the residual of its paired reverse arc. */
    out->capacity_ok = 1;
    int64_t *net = cur;    /* reuse: net inflow per node */
    memset(net, 0, (size_t)g->n * sizeof(int64_t));
    for (int64_t u = 0; u < g->n; ++u)
        for (int64_t a = g->first[u]; a < g->first[u + 1]; ++a) {
            if (!g->fwd[a]) continue;
            int64_t f = g->res[g->rev[a]];
            if (f < 0 || f > orig[a] || g->res[a] < 0) out->capacity_ok = 0;
            net[u] -= f;
            net[g->head[a]] += f;
        }
    out->conservation_ok = 1;
    for (int64_t v = 0; v < N; ++v)
        if (net[v] != 0) out->conservation_ok = 0;
    if (net[t] != out->flow || net[s] != -out->flow) out->conservation_ok = 0;

    /* Minimal and maximal minimum cuts. */
    reach_from(g, s, sreach, buf);
    reach_to(g, t, treach, buf);
    out->smin_in_smax = 1;
    for (int64_t v = 0; v < g->n; ++v)
        if (sreach[v] && treach[v]) out->smin_in_smax = 0;

    out->cut = 0;
    for (int64_t u = 0; u < g->n; ++u) {
        if (!sreach[u]) continue;
        for (int64_t a = g->first[u]; a < g->first[u + 1]; ++a)
            if (g->fwd[a] && !sreach[g->head[a]]) {
                out->cut += orig[a] >= OR_INF ? OR_INF : orig[a];
                if (out->cut > OR_INF) out->cut = OR_INF;
            }
    }
    free(level); free(cur); free(buf); free(orig);
    return 0;
}

/*
 * Solve one volume.  cost: nx*ny*K int32, z fastest; alpha >= 0 the soft
 * smoothness weight (0: hard bound only).  Outputs hmin, hmax (nx*ny int32
 * each, may be NULL).  Returns 0 on success, -1 on bad arguments, -2 when
 * memory runs out.
 */
int oracle_solve_soft(const int32_t *cost, int32_t nx, int32_t ny, int32_t K,
                      int32_t delta, int32_t alpha, int32_t *hmin, int32_t *hmax,
                      or_result *out)
{
    memset(out, 0, sizeof(*out));
    if (!cost || nx < 1 || ny < 1 || K < 1 || delta < 0 || alpha < 0) return out->status = -1;
    or_graph g;
    if (build_graph(&g, cost, nx, ny, K, delta, alpha)) return out->status = -2;
    const int64_t N = (int64_t)nx * ny * K;
    uint8_t *sreach = malloc((size_t)g.n), *treach = malloc((size_t)g.n);
    int32_t *hlo = malloc((size_t)nx * ny * sizeof(int32_t));
    int32_t *hhi = malloc((size_t)nx * ny * sizeof(int32_t));
    if (!sreach || !treach || !hlo || !hhi || max_flow_cuts(&g, N, sreach, treach, out)) {
        free(sreach); free(treach); free(hlo); free(hhi);
        free_graph(&g);
        return out->status = -2;
    }

    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y) {
            int32_t lo = -1, hi = -1;
            for (int32_t z = 0; z < K; ++z) {
                int64_t v = node_id(x, y, z, ny, K);
                if (sreach[v]) lo = z;
                if (!treach[v]) hi = z;
            }
            int64_t p = x * ny + y;
            hlo[p] = lo;
            hhi[p] = hi;
            if (hmin) hmin[p] = lo;
            if (hmax) hmax[p] = hi;
            if (lo >= 0) out->energy += cost[node_id(x, y, lo, ny, K)];
            if (hi >= 0) out->energy_hmax += cost[node_id(x, y, hi, ny, K)];
        }
    if (alpha > 0) {
        out->energy += smooth_term(hlo, nx, ny, alpha);
        out->energy_hmax += smooth_term(hhi, nx, ny, alpha);
    }

    free(sreach); free(treach); free(hlo); free(hhi);
    free_graph(&g);
    return 0;
}

/* The hard-bound problem (alpha = 0). */
int oracle_solve(const int32_t *cost, int32_t nx, int32_t ny, int32_t K,
                 int32_t delta, int32_t *hmin, int32_t *hmax, or_result *out)
{
    return oracle_solve_soft(cost, nx, ny, K, delta, 0, hmin, hmax, out);
}

/*
 * Narrow-band graphs (Section 3.4: the graph is built only in a band around
 * the surface that the user's landmark points outline, a stick of heights
 * above and below it per column).  Column p holds the heights off[p] ..
 * off[p] + ext[p] - 1 of the volume; cost[p*K + j] is the cost at height
 * off[p] + j (j < ext[p] <= K; entries beyond ext[p] are not read).  A
 * surface takes one height h(p) in every column's band, with
 * |h(p) - h(q)| <= delta for 4-neighbours.
 *
 * band_effective: the heights that some such surface takes in each column,
 * [lo(p), hi(p)].  Every surface obeys lo(q) >= lo(p) - delta and
 * hi(p) <= hi(q) + delta for neighbours, so the bounds are tightened by these
 * rules until nothing changes; at that fixed point the surfaces h = lo and
 * h = hi are themselves smooth and inside the bands, so each bound is
 * attained.  Returns 0, 1 when some column is left empty (lo > hi: no
 * surface exists), -1 on bad arguments.
 */
static const int band_step[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};   /* +x, -x, +y, -y */

int band_effective(int32_t nx, int32_t ny, int32_t K, int32_t delta, const int32_t *off,
                   const int32_t *ext, int32_t *lo, int32_t *hi)
{
    if (!off || !ext || !lo || !hi || nx < 1 || ny < 1 || K < 1 || delta < 0) return -1;
    const int64_t P = (int64_t)nx * ny;
    for (int64_t p = 0; p < P; ++p) {
        if (off[p] < 0 || ext[p] < 1 || ext[p] > K || (int64_t)off[p] + ext[p] > (1LL << 30)) return -1;
        lo[p] = off[p];
        hi[p] = off[p] + ext[p] - 1;
    }
    for (int changed = 1; changed;) {
        changed = 0;
        for (int64_t x = 0; x < nx; ++x)
            for (int64_t y = 0; y < ny; ++y)
                for (int d = 0; d < 4; ++d) {
                    int64_t qx = x + band_step[d][0], qy = y + band_step[d][1];
                    if (qx < 0 || qx >= nx || qy < 0 || qy >= ny) continue;
                    int64_t p = x * ny + y, q = qx * ny + qy;
                    if (lo[p] - delta > lo[q]) { lo[q] = lo[p] - delta; changed = 1; }
                    if (hi[q] + delta < hi[p]) { hi[p] = hi[q] + delta; changed = 1; }
                }
        for (int64_t p = 0; p < P; ++p)
            if (lo[p] > hi[p]) return 1;
    }
    return 0;
}

typedef struct {
    const int32_t *cost, *off, *lo, *hi;
    const int64_t *base;   /* first node of each column */
    int64_t nx, ny, K, delta;
} band_geom;

/* Calls fn(tail, head, cap) for every arc of the band graph: the graph of
 * Section 1.2 on the heights lo(p)..hi(p) of every column (node (p, z) is
 * base[p] + z - lo(p)), with B = max_p c(p, lo(p)) + 1, w(p, lo(p)) =
 * c(p, lo(p)) - B, w(p, z) = c(p, z) - c(p, z - 1) above, infinite down
 * arcs, and infinite lateral arcs (p, z) -> (q, max(lo(q), z - delta)). */
static void for_each_band_arc(const band_geom *b, arc_fn fn, void *ctx)
{
    const int64_t P = b->nx * b->ny, N = b->base[P], s = N, t = N + 1;
    int64_t B = INT64_MIN;
    for (int64_t p = 0; p < P; ++p) {
        int64_t c0 = b->cost[p * b->K + b->lo[p] - b->off[p]];
        if (c0 > B) B = c0;
    }
    B = B + 1;
    for (int64_t x = 0; x < b->nx; ++x)
        for (int64_t y = 0; y < b->ny; ++y) {
            const int64_t p = x * b->ny + y;
            const int32_t *cp = b->cost + p * b->K - b->off[p];   /* cp[z]: cost at height z */
            for (int64_t z = b->lo[p]; z <= b->hi[p]; ++z) {
                int64_t v = b->base[p] + z - b->lo[p];
                int64_t w = z == b->lo[p] ? (int64_t)cp[z] - B : (int64_t)cp[z] - (int64_t)cp[z - 1];
                if (w < 0) { fn(ctx, s, v, -w); }   /* source arc */
                if (w > 0) { fn(ctx, v, t, w); }    /* sink arc */
                if (z > b->lo[p]) fn(ctx, v, v - 1, OR_INF);
                for (int d = 0; d < 4; ++d) {
                    int64_t qx = x + band_step[d][0], qy = y + band_step[d][1];
                    if (qx < 0 || qx >= b->nx || qy < 0 || qy >= b->ny) continue;
                    int64_t q = qx * b->ny + qy;
                    int64_t zq = z - b->delta < b->lo[q] ? b->lo[q] : z - b->delta;
                    fn(ctx, v, b->base[q] + zq - b->lo[q], OR_INF);
                }
            }
        }
}

static int build_band_graph(or_graph *g, const band_geom *b)
{
    memset(g, 0, sizeof(*g));
    const int64_t P = b->nx * b->ny;
    g->n = b->base[P] + 2;
    g->first = calloc((size_t)g->n + 1, sizeof(int64_t));
    if (!g->first) return -1;
    build_ctx bc = {g, NULL};
    for_each_band_arc(b, count_arc, &bc);
    for (int64_t i = 0; i < g->n; ++i) g->first[i + 1] += g->first[i];
    g->m = g->first[g->n];
    g->head = malloc((size_t)g->m * sizeof(int64_t));
    g->res = malloc((size_t)g->m * sizeof(int64_t));
    g->rev = malloc((size_t)g->m * sizeof(int64_t));
    g->fwd = malloc((size_t)g->m);
    bc.fill = malloc((size_t)g->n * sizeof(int64_t));
    if (!g->head || !g->res || !g->rev || !g->fwd || !bc.fill) {
        free(bc.fill); free_graph(g); return -1;
    }
    memcpy(bc.fill, g->first, (size_t)g->n * sizeof(int64_t));
    for_each_band_arc(b, place_arc, &bc);
    free(bc.fill);
    return 0;
}

/*
 * Solve a narrow-band volume (see band_effective for the layout).  Outputs
 * the effective bands lo, hi and the minimal and maximal minimum-cut
 * surfaces hmin, hmax, all as heights of the volume (nx*ny int32 each; hmin
 * and hmax may be NULL); the energy is sum_p c(p, h_min(p)).  Returns 0,
 * -1 on bad arguments, -2 when memory runs out, -3 when no delta-smooth
 * surface fits the bands.
 */
int oracle_solve_band(const int32_t *cost, int32_t nx, int32_t ny, int32_t K, int32_t delta,
                      const int32_t *off, const int32_t *ext, int32_t *lo, int32_t *hi,
                      int32_t *hmin, int32_t *hmax, or_result *out)
{
    memset(out, 0, sizeof(*out));
    if (!cost) return out->status = -1;
    const int be = band_effective(nx, ny, K, delta, off, ext, lo, hi);
    if (be < 0) return out->status = -1;
    if (be > 0) return out->status = -3;
    const int64_t P = (int64_t)nx * ny;
    int64_t *base = malloc((size_t)(P + 1) * sizeof(int64_t));
    if (!base) return out->status = -2;
    base[0] = 0;
    for (int64_t p = 0; p < P; ++p) base[p + 1] = base[p] + hi[p] - lo[p] + 1;
    band_geom b = {cost, off, lo, hi, base, nx, ny, K, delta};
    or_graph g;
    if (build_band_graph(&g, &b)) { free(base); return out->status = -2; }
    const int64_t N = base[P];
    uint8_t *sreach = malloc((size_t)g.n), *treach = malloc((size_t)g.n);
    if (!sreach || !treach || max_flow_cuts(&g, N, sreach, treach, out)) {
        free(sreach); free(treach); free(base);
        free_graph(&g);
        return out->status = -2;
    }
    for (int64_t p = 0; p < P; ++p) {
        int32_t hl = -1, hh = -1;
        for (int32_t z = lo[p]; z <= hi[p]; ++z) {
            int64_t v = base[p] + z - lo[p];
            if (sreach[v]) hl = z;
            if (!treach[v]) hh = z;
        }
        if (hmin) hmin[p] = hl;
        if (hmax) hmax[p] = hh;
        if (hl >= 0) out->energy += cost[p * K + hl - off[p]];
        if (hh >= 0) out->energy_hmax += cost[p * K + hh - off[p]];
    }
    free(sreach); free(treach); free(base);
    free_graph(&g);
    return 0;
}
