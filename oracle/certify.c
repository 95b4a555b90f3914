/*
 * Max-flow/min-cut certificate checker.  TEST INFRASTRUCTURE ONLY (see
 * oracle.c).  It verifies, at any problem size and in O(n), that a solver's
 * final state is a maximum preflow and that the reported surface is the
 * inclusion-minimal minimum cut:
 *
 *   - capacity and sign bounds of every arc (Eq. 2);
 *   - the excess of every node equals inflow minus outflow (Eq. 8) and is
 *     non-negative, so the state is a preflow;
 *   - the surface is delta-smooth (Section 1.2, proper-ordered columns);
 *   - the set R reachable in the residual graph from every node with
 *     positive excess does not contain the sink and its column heights equal
 *     the surface.  Then no residual arc leaves R, the flow value equals the
 *     capacity of the cut (R, complement) (Theorem 1.1), and R is contained
 *     in every minimum cut, i.e. it is the minimal one.
 *
 * With a soft smoothness weight alpha > 0 the checked graph also has the
 * arcs (p,z) -> (q,z), z >= 1, of capacity alpha (their flows stored per
 * direction at the tail like the lateral ones); they enter the bounds, the
 * conservation, the residual reach, and the cut capacity as alpha *
 * max(0, h(p) - h(q)) per ordered neighbour pair.  The energy then includes
 * alpha * |h(p) - h(q)| per unordered pair.
 *
 * The arc set checked is the one the solver stores: the down arc
 * (p,z)->(p,z-1) for z >= 1, and for each 4-neighbour q of p the lateral arc
 * (p,z)->(q,z-delta) when z > delta, plus (p,0)->(q,0).  The omitted arcs
 * (p,z)->(q,0) for 1 <= z <= delta are implied by (p,z)->(p,0)->(q,0), so
 * the closed sets, the cut capacities and the max-flow value are those of
 * the full graph of oracle.c.  Flows are stored per arc at the arc's tail.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t flow;
    int64_t cut;
    int64_t energy;
    int64_t bad_capacity;
    int64_t bad_conservation;
    int64_t bad_smooth;
    int64_t bad_reach;
    int32_t status;
    int32_t pad;
} cert_result;

static int lat_arc_exists(int64_t z, int64_t delta) { return z == 0 || z > delta; }
static int64_t lat_target(int64_t z, int64_t delta) { return z == 0 ? 0 : z - delta; }

int certify_preflow_soft(const int32_t *cost, int32_t nx_, int32_t ny_, int32_t K_,
                         int32_t delta_, int32_t alpha_, const int32_t *excess,
                         const int32_t *sink_res, const int32_t *flow_down,
                         const int32_t *flow_lat, const int32_t *flow_soft,
                         const int32_t *surface, cert_result *out)
{
    memset(out, 0, sizeof(*out));
    const int64_t nx = nx_, ny = ny_, K = K_, delta = delta_, alpha = alpha_;
    if (nx < 1 || ny < 1 || K < 1 || delta < 0 || alpha < 0 || (alpha > 0 && !flow_soft))
        return out->status = -1;
    const int64_t N = nx * ny * K, P = nx * ny;
    static const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};

    int64_t B = INT64_MIN;
    for (int64_t p = 0; p < P; ++p)
        if (cost[p * K] > B) B = cost[p * K];
    B += 1;

    int64_t *net = calloc((size_t)N, sizeof(int64_t));
    uint8_t *mark = calloc((size_t)N, 1);
    int64_t *queue = malloc((size_t)N * sizeof(int64_t));
    if (!net || !mark || !queue) {
        free(net); free(mark); free(queue);
        return out->status = -2;
    }

    /* Arc flows: bounds, and net inflow per node. */
    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t z = 0; z < K; ++z) {
                int64_t v = (x * ny + y) * K + z;
                int64_t fd = flow_down[v];
                if (fd < 0 || (z == 0 && fd != 0)) out->bad_capacity++;
                if (z > 0) { net[v] -= fd; net[v - 1] += fd; }
                for (int k = 0; k < 4; ++k) {
                    int64_t f = flow_lat[(int64_t)k * N + v];
                    int64_t qx = x + dx[k], qy = y + dy[k];
                    int in = qx >= 0 && qx < nx && qy >= 0 && qy < ny;
                    if (!in || !lat_arc_exists(z, delta)) {
                        if (f != 0) out->bad_capacity++;
                        continue;
                    }
                    if (f < 0) out->bad_capacity++;
                    int64_t u = (qx * ny + qy) * K + lat_target(z, delta);
                    net[v] -= f; net[u] += f;
                }
                if (!flow_soft) continue;
                for (int k = 0; k < 4; ++k) {
                    int64_t f = flow_soft[(int64_t)k * N + v];
                    int64_t qx = x + dx[k], qy = y + dy[k];
                    int in = qx >= 0 && qx < nx && qy >= 0 && qy < ny;
                    if (!in || z == 0 || alpha == 0) {
                        if (f != 0) out->bad_capacity++;
                        continue;
                    }
                    if (f < 0 || f > alpha) out->bad_capacity++;
                    int64_t u = (qx * ny + qy) * K + z;
                    net[v] -= f; net[u] += f;
                }
            }

    /* Terminal arcs: the source arcs are saturated (the solver never returns
     * flow to s), the sink arc keeps residual sink_res. */
    for (int64_t v = 0; v < N; ++v) {
        int64_t z = v % K;
        int64_t w = z == 0 ? (int64_t)cost[v] - B : (int64_t)cost[v] - cost[v - 1];
        int64_t src = w < 0 ? -w : 0, snk = w > 0 ? w : 0;
        int64_t r = sink_res[v];
        if (r < 0 || r > snk) out->bad_capacity++;
        out->flow += snk - r;
        int64_t e = excess[v];
        if (e < 0) out->bad_capacity++;
        if (e != src - (snk - r) + net[v]) out->bad_conservation++;
    }

    /* Smoothness, energy and cut capacity of the surface. */
    for (int64_t x = 0; x < nx; ++x)
        for (int64_t y = 0; y < ny; ++y) {
            int64_t p = x * ny + y, h = surface[p];
            if (h < 0 || h >= K) { out->bad_smooth++; continue; }
            out->energy += cost[p * K + h];
            for (int k = 0; k < 4; ++k) {
                int64_t qx = x + dx[k], qy = y + dy[k];
                if (qx < 0 || qx >= nx || qy < 0 || qy >= ny) continue;
                int64_t hq = surface[qx * ny + qy];
                if (hq - h > delta || h - hq > delta) out->bad_smooth++;
                if (hq >= 0 && hq < K) {
                    if (h > hq) out->cut += alpha * (h - hq);   /* soft arcs (p,z)->(q,z), hq < z <= h */
                    if (k == 0 || k == 2) out->energy += alpha * (h > hq ? h - hq : hq - h);
                }
            }
            for (int64_t z = 0; z < K; ++z) {
                int64_t v = p * K + z;
                int64_t w = z == 0 ? (int64_t)cost[v] - B : (int64_t)cost[v] - cost[v - 1];
                if (z <= h && w > 0) out->cut += w;
                if (z > h && w < 0) out->cut += -w;
            }
        }

    /* Residual reach from all nodes with positive excess. */
    int64_t qh = 0, qt = 0;
    for (int64_t v = 0; v < N; ++v)
        if (excess[v] > 0) { mark[v] = 1; queue[qt++] = v; }
    int reached_sink = 0;
#define VISIT(u) do { if (!mark[u]) { mark[u] = 1; queue[qt++] = (u); } } while (0)
    while (qh < qt) {
        int64_t v = queue[qh++];
        int64_t z = v % K, p = v / K, x = p / ny, y = p % ny;
        if (sink_res[v] > 0) reached_sink = 1;
        if (z > 0) VISIT(v - 1);                               /* down, infinite */
        if (z + 1 < K && flow_down[v + 1] > 0) VISIT(v + 1);  /* reverse of down */
        for (int k = 0; k < 4; ++k) {
            int64_t qx = x + dx[k], qy = y + dy[k];
            if (qx < 0 || qx >= nx || qy < 0 || qy >= ny) continue;
            int64_t q = qx * ny + qy;
            if (lat_arc_exists(z, delta)) VISIT(q * K + lat_target(z, delta));
            /* Reverse residual of q's arc in the opposite direction that
             * lands on v: its tail is (q, z + delta), or (q, 0) when z = 0. */
            int kk = k ^ 1;
            int64_t zt = z == 0 ? 0 : z + delta;
            if (zt < K && lat_arc_exists(zt, delta) && lat_target(zt, delta) == z) {
                int64_t u = q * K + zt;
                if (flow_lat[(int64_t)kk * N + u] > 0) VISIT(u);
            }
            /* soft arc (p,z) -> (q,z): residual alpha - f(p->q) + f(q->p) */
            if (alpha > 0 && z >= 1) {
                int64_t u = q * K + z;
                if (alpha - flow_soft[(int64_t)k * N + v] + flow_soft[(int64_t)kk * N + u] > 0) VISIT(u);
            }
        }
    }
#undef VISIT
    if (reached_sink) out->bad_reach++;
    for (int64_t p = 0; p < P; ++p) {
        int64_t top = -1;
        for (int64_t z = 0; z < K; ++z)
            if (mark[p * K + z]) top = z;
        if (top != surface[p]) out->bad_reach++;
    }

    free(net); free(mark); free(queue);
    return 0;
}

/* The hard-bound certificate (alpha = 0, no soft arcs). */
int certify_preflow(const int32_t *cost, int32_t nx, int32_t ny, int32_t K, int32_t delta,
                    const int32_t *excess, const int32_t *sink_res, const int32_t *flow_down,
                    const int32_t *flow_lat, const int32_t *surface, cert_result *out)
{
    return certify_preflow_soft(cost, nx, ny, K, delta, 0, excess, sink_res, flow_down, flow_lat,
                                NULL, surface, out);
}

/*
 * Certificate of a narrow-band solve (the band graph of oracle.c,
 * oracle_solve_band).  The solver keeps the heights lo(p)..hi(p) that some
 * delta-smooth surface takes in column p (band_effective) and stores node
 * (p, lo(p) + j) at p*K + j; slots j > hi(p) - lo(p) are unused and must hold
 * no excess, sink residual or flow.  Its arcs: the down arc (p,j)->(p,j-1)
 * for j >= 1, and per 4-neighbour q, with sh = delta + lo(q) - lo(p), the
 * lateral arc (p,j)->(q,j-sh) for j > sh plus (p,0)->(q,0); the omitted
 * arcs (p,j)->(q,0), 1 <= j <= sh, are implied by (p,j)->(p,0)->(q,0).
 * The surface is given as heights of the volume.  The checks are those of
 * certify_preflow_soft, on this arc set.  Returns 0, -1 on bad arguments
 * (or bands that admit no smooth surface), -2 when memory runs out.
 */
int band_effective(int32_t nx, int32_t ny, int32_t K, int32_t delta, const int32_t *off,
                   const int32_t *ext, int32_t *lo, int32_t *hi);

int certify_preflow_band(const int32_t *cost, int32_t nx_, int32_t ny_, int32_t K_, int32_t delta_,
                         const int32_t *off, const int32_t *ext, const int32_t *excess,
                         const int32_t *sink_res, const int32_t *flow_down, const int32_t *flow_lat,
                         const int32_t *surface, cert_result *out)
{
    memset(out, 0, sizeof(*out));
    const int64_t nx = nx_, ny = ny_, K = K_, delta = delta_, P = nx * ny, N = P * K;
    if (nx < 1 || ny < 1 || K < 1 || delta < 0) return out->status = -1;
    int32_t *lo = malloc((size_t)P * sizeof(int32_t)), *hi = malloc((size_t)P * sizeof(int32_t));
    int64_t *net = calloc((size_t)N, sizeof(int64_t));
    uint8_t *mark = calloc((size_t)N, 1);
    int64_t *queue = malloc((size_t)N * sizeof(int64_t));
    if (!lo || !hi || !net || !mark || !queue) {
        free(lo); free(hi); free(net); free(mark); free(queue);
        return out->status = -2;
    }
    if (band_effective(nx_, ny_, K_, delta_, off, ext, lo, hi) != 0) {
        free(lo); free(hi); free(net); free(mark); free(queue);
        return out->status = -1;
    }
    static const int stp[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    /* neighbour of column p in direction k, or -1 */
#define NBR(p, k) (((p) / ny + stp[k][0] < 0 || (p) / ny + stp[k][0] >= nx || \
                    (p) % ny + stp[k][1] < 0 || (p) % ny + stp[k][1] >= ny) ? (int64_t)-1 : \
                   ((p) / ny + stp[k][0]) * ny + (p) % ny + stp[k][1])
    /* cost at local slot j of column p */
#define CST(p, j) ((int64_t)cost[(p) * K + lo[p] - off[p] + (j)])
    int64_t Bb = INT64_MIN;
    for (int64_t p = 0; p < P; ++p)
        if (CST(p, 0) > Bb) Bb = CST(p, 0);
    Bb = Bb + 1;

    for (int64_t p = 0; p < P; ++p) {
        const int64_t n = hi[p] - lo[p] + 1;
        for (int64_t j = 0; j < K; ++j) {
            const int64_t v = p * K + j;
            const int64_t fdv = flow_down[v];
            if (j >= n) {   /* unused slot */
                if (excess[v] != 0 || sink_res[v] != 0 || fdv != 0) out->bad_capacity++;
                for (int k = 0; k < 4; ++k)
                    if (flow_lat[(int64_t)k * N + v] != 0) out->bad_capacity++;
                continue;
            }
            if (fdv < 0 || (j == 0 && fdv != 0)) out->bad_capacity++;
            if (j > 0) { net[v - 1] += fdv; net[v] -= fdv; }
            for (int k = 0; k < 4; ++k) {
                const int64_t f = flow_lat[(int64_t)k * N + v];
                const int64_t q = NBR(p, k);
                const int64_t sh = q < 0 ? 0 : delta + lo[q] - lo[p];
                const int64_t jt = j == 0 ? 0 : j - sh;
                if (q < 0 || (j != 0 && j <= sh) || jt > hi[q] - lo[q]) {
                    if (f != 0) out->bad_capacity++;
                    continue;
                }
                if (f < 0) out->bad_capacity++;
                net[v] -= f;
                net[q * K + jt] += f;
            }
        }
    }
    for (int64_t p = 0; p < P; ++p)
        for (int64_t j = 0; j <= hi[p] - lo[p]; ++j) {
            const int64_t v = p * K + j;
            const int64_t w = j == 0 ? CST(p, 0) - Bb : CST(p, j) - CST(p, j - 1);
            const int64_t cap_s = w < 0 ? -w : 0, cap_t = w > 0 ? w : 0, rt = sink_res[v];
            if (rt < 0 || rt > cap_t) out->bad_capacity++;
            out->flow += cap_t - rt;
            if (excess[v] < 0) out->bad_capacity++;
            if (excess[v] != cap_s - (cap_t - rt) + net[v]) out->bad_conservation++;
        }

    /* surface: inside the effective band, smooth; its energy and cut */
    for (int64_t p = 0; p < P; ++p) {
        const int64_t h = surface[p];
        if (h < lo[p] || h > hi[p]) { out->bad_smooth++; continue; }
        out->energy += CST(p, h - lo[p]);
        for (int k = 0; k < 4; ++k) {
            const int64_t q = NBR(p, k);
            if (q >= 0 && (surface[q] - h > delta || h - surface[q] > delta)) out->bad_smooth++;
        }
        for (int64_t j = 0; j <= hi[p] - lo[p]; ++j) {
            const int64_t w = j == 0 ? CST(p, 0) - Bb : CST(p, j) - CST(p, j - 1);
            if (lo[p] + j <= h) { if (w > 0) out->cut += w; }
            else if (w < 0) out->cut -= w;
        }
    }

    /* residual reach from the nodes with excess */
    int64_t head = 0, tail = 0, sink_hit = 0;
    for (int64_t p = 0; p < P; ++p)
        for (int64_t j = 0; j <= hi[p] - lo[p]; ++j)
            if (excess[p * K + j] > 0) { mark[p * K + j] = 1; queue[tail++] = p * K + j; }
#define REACH(u) do { if (!mark[u]) { mark[u] = 1; queue[tail++] = (u); } } while (0)
    while (head < tail) {
        const int64_t v = queue[head++], p = v / K, j = v % K, n = hi[p] - lo[p] + 1;
        if (sink_res[v] > 0) sink_hit = 1;
        if (j > 0) REACH(v - 1);
        if (j + 1 < n && flow_down[v + 1] > 0) REACH(v + 1);
        for (int k = 0; k < 4; ++k) {
            const int64_t q = NBR(p, k);
            if (q < 0) continue;
            const int64_t sh = delta + lo[q] - lo[p];          /* arcs p -> q */
            if (j == 0 || j > sh) REACH(q * K + (j == 0 ? 0 : j - sh));
            /* q's arc towards p (direction k ^ 1) that lands on (p, j) */
            const int64_t shq = delta + lo[p] - lo[q];
            const int64_t jq = j == 0 ? 0 : j + shq;
            if (jq <= hi[q] - lo[q] && flow_lat[(int64_t)(k ^ 1) * N + q * K + jq] > 0) REACH(q * K + jq);
        }
    }
#undef REACH
    if (sink_hit) out->bad_reach++;
    for (int64_t p = 0; p < P; ++p) {
        int64_t top = -1;
        for (int64_t j = 0; j <= hi[p] - lo[p]; ++j)
            if (mark[p * K + j]) top = lo[p] + j;
        if (top != surface[p]) out->bad_reach++;
    }
#undef NBR
#undef CST
    free(lo); free(hi); free(net); free(mark); free(queue);
    return 0;
}

/*
 * The pointwise-highest optimal surface from a maximum preflow of the plain
 * graph (state as for certify_preflow): S_max, the source side of the
 * maximal minimum cut, is the set of nodes that cannot reach t in the
 * residual graph (Theorem 1.1 applied to the maximal cut; returning excess to
 * s changes no residual arc on a path to t, so any maximum preflow gives the
 * same set).  The nodes that reach t are found by a backward search from the
 * sink arcs with residual capacity; hmax[p] = the highest node of column p
 * outside that set (-1 if none).  Returns 0, -1 on bad arguments, -2 when
 * memory runs out.
 */
int certify_hmax(int32_t nx_, int32_t ny_, int32_t K_, int32_t delta_, const int32_t *sink_res,
                 const int32_t *flow_down, const int32_t *flow_lat, int32_t *hmax)
{
    const int64_t nx = nx_, ny = ny_, K = K_, delta = delta_, P = nx * ny, N = P * K;
    if (nx < 1 || ny < 1 || K < 1 || delta < 0 || !hmax) return -1;
    uint8_t *to_t = calloc((size_t)N, 1);
    int64_t *queue = malloc((size_t)N * sizeof(int64_t));
    if (!to_t || !queue) { free(to_t); free(queue); return -2; }
    static const int mx[4] = {1, -1, 0, 0}, my[4] = {0, 0, 1, -1};
    int64_t first = 0, last = 0;
    for (int64_t v = 0; v < N; ++v)
        if (sink_res[v] > 0) { to_t[v] = 1; queue[last++] = v; }
#define BACK(u) do { if (!to_t[u]) { to_t[u] = 1; queue[last++] = (u); } } while (0)
    while (first < last) {
        const int64_t v = queue[first++], z = v % K, p = v / K, x = p / ny, y = p % ny;
        if (z + 1 < K) BACK(v + 1);                    /* (p,z+1) -> (p,z), infinite */
        if (z > 0 && flow_down[v] > 0) BACK(v - 1);    /* reverse of (p,z) -> (p,z-1) */
        for (int k = 0; k < 4; ++k) {
            const int64_t qx = x + mx[k], qy = y + my[k];
            if (qx < 0 || qx >= nx || qy < 0 || qy >= ny) continue;
            const int64_t q = qx * ny + qy;
            /* q's lateral arc towards p landing on (p,z): tail (q,0) or (q,z+delta) */
            const int64_t zq = z == 0 ? 0 : z + delta;
            if (zq < K) BACK(q * K + zq);
            /* reverse of v's own arc (p,z) -> (q, z - delta) carrying flow */
            if ((z == 0 || z > delta) && flow_lat[(int64_t)k * N + v] > 0)
                BACK(q * K + (z == 0 ? 0 : z - delta));
        }
    }
#undef BACK
    for (int64_t p = 0; p < P; ++p) {
        int32_t top = -1;
        for (int64_t z = 0; z < K; ++z)
            if (!to_t[p * K + z]) top = (int32_t)z;
        hmax[p] = top;
    }
    free(to_t); free(queue);
    return 0;
}
