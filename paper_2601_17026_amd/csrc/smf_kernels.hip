// HIP kernels of the exact surface max-flow (gfx950).
//
// Method: push-relabel (Section 2.1) on the implicit column graph of
// Section 1.2, with global relabelling by a reverse breadth-first search
// from the sink (Section 2.1, "global relabeling"; Section 3.2.2) and the
// minimum cut read out as the residual reach set (Section 1.3, Eq. 6,
// Theorem 1.1).  Storage is implicit (Section 3.2.3): no edge lists, only
// per-node excess, label, sink residual and the flows of the five outgoing
// infinite arcs.
//
// Labels.  A valid labelling here satisfies d(u) <= d(w) + len(u, w) for
// every residual arc, with len = 0 for the always-residual down arcs
// (p,z) -> (p,z-1) and len = 1 for every other arc (sink arcs included,
// d(t) = 0).  Down arcs never lie on a cycle of length-0 arcs, so pushes
// along them cannot circulate, and d(v) remains a lower bound of the
// weighted residual distance to t: a node whose label exceeds N cannot reach
// t.  Zero-length down arcs let excess fall down a whole column in one
// sweep and make the breadth-first search count only column changes and
// upward moves.
//
// Concurrency.  A sweep is two launches: a push phase with all labels fixed,
// then a relabel phase with all flows fixed.  In the push phase a thread owns
// one column; an arc and its reverse can never both be admissible under
// fixed labels, so every flow counter has a single writer per phase, and
// only excess counters of other columns are updated with atomics.  In the
// relabel phase labels only grow, so reading a neighbour's old or new label
// both keep the labelling valid.
#include "smf_device.h"
#include <limits.h>

namespace smf {

__device__ __forceinline__ int wave_sum(int v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ long long wave_sum64(long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ void add_excess(int *e, int w, long long a, int &err)
{
    if (a > INT_MAX) { err = 1; a = INT_MAX; }
    int old = atomicAdd(e + w, (int)a);
    if ((long long)old + a > INT_MAX) err = 1;
}

__device__ __forceinline__ int add_flow(int f, long long a, int &err)
{
    long long r = (long long)f + a;
    if (r > INT_MAX) { err = 1; r = INT_MAX; }
    return (int)r;
}

__global__ void k_init_scratch(Scratch *s)
{
    s->bmax = INT_MIN;
    s->err = 0;
    s->changed = 0;
    s->active = 0;
    s->flow = 0;
    s->energy = 0;
    s->bfs_active = 0;
    s->bfs_labelled = 0;
}

__global__ void k_set_int(int *p, int v) { *p = v; }

__global__ void k_fill(int *a, int n, int v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// B - 1 = max_p c(p, 0): the bottom shift that makes every bottom node a
// source node (w(p,0) < 0), so that the empty cut never wins.
__global__ void k_bottom_max(const int *__restrict__ cost, int P, int K, Scratch *s)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    int v = p < P ? cost[(long long)p * K] : INT_MIN;
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) atomicMax(&s->bmax, v);
}

// Graph build: node weights w (Section 1.2), source arcs pre-saturated into
// the excess (Section 2.1 initialisation), sink residuals, zero flows and
// labels 0 (valid lower bounds) until the first breadth-first search.  A 64-column
// x 64-level tile is transposed through LDS from the caller's z-fastest
// layout to the level-major state layout.
__global__ __launch_bounds__(256) void k_build(const int *__restrict__ cost, Geom g, State st,
                                               Scratch *s)
{
    __shared__ int tile[64][65];
    __shared__ int below[64];
    const int p0 = blockIdx.x * 64, z0 = blockIdx.y * 64;
    const int tid = threadIdx.x;
    int bad = 0;
    for (int i = 0; i < 16; ++i) {
        int l = tid + 256 * i, pc = l >> 6, zc = l & 63;
        int p = p0 + pc, z = z0 + zc;
        int c = 0;
        if (p < g.P && z < g.K) {
            c = cost[(long long)p * g.K + z];
            if (c <= -(1 << 30) || c >= (1 << 30)) bad = 1;
        }
        tile[pc][zc] = c;
    }
    if (tid < 64) {
        int p = p0 + tid;
        below[tid] = (z0 > 0 && p < g.P) ? cost[(long long)p * g.K + z0 - 1] : 0;
    }
    __syncthreads();
    const int B = s->bmax + 1;
    long long ts_sum = 0;
    for (int i = 0; i < 16; ++i) {
        int l = tid + 256 * i, zc = l >> 6, pc = l & 63;
        int p = p0 + pc, z = z0 + zc;
        if (p >= g.P || z >= g.K) continue;
        int c = tile[pc][zc];
        int cb = zc > 0 ? tile[pc][zc - 1] : below[pc];
        int w = z == 0 ? c - B : c - cb;
        int v = z * g.P + p;
        st.e[v] = w < 0 ? -w : 0;
        st.ts[v] = w > 0 ? w : 0;
        ts_sum += w > 0 ? w : 0;
        st.d[v] = 0;   // valid lower bound until the first global relabel
        st.fd[v] = 0;
        for (int k = 0; k < 4; ++k) st.fl[(size_t)k * g.N + v] = 0;
    }
    ts_sum = wave_sum64(ts_sum);
    if ((tid & 63) == 0 && ts_sum) atomicAdd((unsigned long long *)&s->flow, (unsigned long long)ts_sum);
    if (bad) atomicOr(&s->err, kErrCostRange);
}

// Loads are issued a chunk of kCh levels at a time so that a thread keeps
// many independent loads in flight instead of one level's worth.
constexpr int kCh = 8;

// ---- global relabel: level-synchronous reverse breadth-first search -------
//
// Exact weighted residual distances to t (Section 2.1 global relabelling;
// the level-by-level order of Section 3.2.2 / Algorithm 3).  Because the
// down arc (p,z) -> (p,z-1) is always residual with length 0, an exact label
// never increases down a column: d(p,z) <= d(p,z-1).  So the set of nodes at
// distance <= L meets column p in a suffix [T_L(p), K), and one BFS level is
// a min-plus update of the per-column thresholds:
//   T_{L+1}(p) = min( T_L(p),
//       lowest z with a lateral arc into q's labelled suffix:
//           0 if T_L(q) = 0, else T_L(q) + delta (when < K);
//       lowest z with a reverse lateral arc into it: the head height of the
//           lowest arc (q,z') -> (p, .) with flow > 0 and z' >= T_L(q);
//       T_L(p) - 1 if the down arc into (p, T_L(p)) carries flow ),
// and the labels d = L+1 are written once, on [T_{L+1}(p), T_L(p)).  Level 1
// is the suffix above the lowest node with a residual sink arc.  The whole
// search reads and writes every node O(1) times; each level touches only
// nx*ny thresholds plus the nodes it labels.
//
// Per-column BFS record, double-buffered by level parity:
//   T[p]      threshold T_L(p) (K when no node of the column is labelled);
//   LF[k][p]  lowest z' >= T_L(p) whose lateral arc in direction k carries
//             flow (K if none) -- the reverse-arc term seen by neighbour k.

__device__ __forceinline__ int lat_head_of(int zp, int dl) { return zp == 0 ? 0 : zp - dl; }

__global__ __launch_bounds__(256) void k_bfs_init(Geom g, State st, int *T, int *LF, int *chg,
                                                  Scratch *s)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) {
        s->lvl_changed[1] = 0;
        s->lvl_lab[1] = 0;
    }
    int act = 0, lab_act = 0;
    if (p < g.P) {
        const int P = g.P, K = g.K, N = g.N;
        int t1 = K;
        int lf[4] = {K, K, K, K};
        for (int z0 = 0; z0 < K; z0 += kCh) {
            int tsv[kCh], ev[kCh], dv[kCh], fv[4][kCh];
#pragma unroll
            for (int j = 0; j < kCh; ++j) {
                const int z = z0 + j;
                tsv[j] = 0;
                ev[j] = 0;
                dv[j] = kInf;
#pragma unroll
                for (int k = 0; k < 4; ++k) fv[k][j] = 0;
                if (z >= K) continue;
                const int u = z * P + p;
                tsv[j] = st.ts[u];
                ev[j] = st.e[u];
                dv[j] = st.d[u];
#pragma unroll
                for (int k = 0; k < 4; ++k) fv[k][j] = st.fl[(size_t)k * N + u];
            }
#pragma unroll
            for (int j = 0; j < kCh; ++j) {
                const int z = z0 + j;
                if (z >= K) break;
                if (t1 == K && tsv[j] > 0) t1 = z;
                const bool lab = t1 < K;
                // a node that could not reach t never can again (new residual
                // arcs only join nodes that reach t), so kInf is kept
                st.d[z * P + p] = lab ? 1 : (dv[j] >= kInf ? kInf : kUnl);
                if (ev[j] > 0 && dv[j] < kInf) {
                    ++act;
                    if (lab) ++lab_act;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (lab && lf[k] == K && fv[k][j] > 0) lf[k] = z;
            }
        }
        T[p] = t1;
        chg[p] = 1;
#pragma unroll
        for (int k = 0; k < 4; ++k) LF[k * P + p] = lf[k];
    }
    act = wave_sum(act);
    lab_act = wave_sum(lab_act);
    if ((threadIdx.x & 63) == 0) {
        if (act) atomicAdd(&s->bfs_active, act);
        if (lab_act) atomicAdd(&s->bfs_labelled, lab_act);
    }
}

// Level L -> L+1 for one column: threshold arithmetic, then the newly
// reached heights [cand, T) are labelled L+1 and scanned (from the top, so
// the last hit is the lowest) for flow-carrying lateral arcs.  Returns the
// number of newly labelled nodes that hold excess.
__device__ __forceinline__ int bfs_column_level(const Geom &g, const State &st, int L, int p,
                                                const int *__restrict__ Tin,
                                                const int *__restrict__ LFin,
                                                const int *__restrict__ chg_in,
                                                int *__restrict__ Tout, int *__restrict__ LFout,
                                                int *__restrict__ chg_out, bool &changed)
{
    const int P = g.P, K = g.K, N = g.N, dl = g.delta;
    const int x = p / g.ny, y = p - x * g.ny;
    int q[4];
    const bool self = chg_in[p] != 0;
    bool near = self;
    for (int k = 0; k < 4; ++k) {
        q[k] = nbr(g, x, y, p, k);
        if (q[k] >= 0 && chg_in[q[k]]) near = true;
    }
    // Frontier: with no change at level L-1 around p, nothing of p's inputs
    // moved.  Both record buffers then already hold p's current record
    // (it did not change at L-1 either), so nothing is written.
    if (!near) {
        chg_out[p] = 0;
        return 0;
    }
    const int T = Tin[p];
    int cand = T;
    for (int k = 0; k < 4; ++k) {
        if (q[k] < 0) continue;
        const int tq = Tin[q[k]];
        if (tq == 0) cand = 0;
        else if (tq + dl < K) cand = min(cand, tq + dl);
        const int lq = LFin[(k ^ 1) * P + q[k]];
        if (lq < K) cand = min(cand, lat_head_of(lq, dl));
    }
    if (T >= 1 && T < K && st.fd[T * P + p] > 0) cand = min(cand, T - 1);
    int lf[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) lf[k] = LFin[k * P + p];
    int lab_act = 0;
    if (cand < T) {
        const int lab = L + 1;
        for (int z0 = T - 1; z0 >= cand; z0 -= kCh) {
            int fv[4][kCh], ev[kCh];
#pragma unroll
            for (int j = 0; j < kCh; ++j) {
                const int z = z0 - j;
                const bool in = z >= cand;
                ev[j] = in ? st.e[z * P + p] : 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) fv[k][j] = in ? st.fl[(size_t)k * N + z * P + p] : 0;
            }
#pragma unroll
            for (int j = 0; j < kCh; ++j) {
                const int z = z0 - j;
                if (z < cand) break;
                st.d[z * P + p] = lab;
                lab_act += ev[j] > 0;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (fv[k][j] > 0) lf[k] = z;
            }
        }
        changed = true;
    }
    // a record that changed at L-1 must also reach the other buffer
    if (cand < T || self) {
        Tout[p] = cand;
#pragma unroll
        for (int k = 0; k < 4; ++k) LFout[k * P + p] = lf[k];
    }
    chg_out[p] = cand < T;
    return lab_act;
}

// One launch per BFS level.
__global__ __launch_bounds__(256) void k_bfs_level(Geom g, State st, int L, const int *__restrict__ Tin,
                                                   const int *__restrict__ LFin,
                                                   const int *__restrict__ chg_in, int *__restrict__ Tout,
                                                   int *__restrict__ LFout, int *__restrict__ chg_out,
                                                   Scratch *s)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    // the slots of the next level are cleared here; stream order puts this
    // before every write of level L+1
    if (p == 0) {
        s->lvl_changed[(L + 1) & 63] = 0;
        s->lvl_lab[(L + 1) & 63] = 0;
    }
    bool changed = false;
    int lab_act = 0;
    if (p < g.P)
        lab_act = bfs_column_level(g, st, L, p, Tin, LFin, chg_in, Tout, LFout, chg_out, changed);
    if (changed) s->lvl_changed[L & 63] = 1;
    lab_act = wave_sum(lab_act);
    if ((threadIdx.x & 63) == 0 && lab_act) atomicAdd(&s->bfs_labelled, lab_act);
}

// End of a global relabel: nodes the search did not reach get `v` (kInf
// when it ran to completion, else the first level it did not finish, which
// is a valid lower bound of their distance).
__global__ void k_bfs_fixup(int *d, int n, int v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && d[i] == kUnl) d[i] = v;
}

// Per-column work ranges.  rlo/rhi bound the heights of the column's nodes
// that may hold excess with a finite label (lo > hi: none).  Every step that
// puts excess on a node records its height in the range of the next phase,
// so a sweep only walks the parts of columns where there is work.

__device__ __forceinline__ void note_range(int *rlo, int *rhi, int p, int z)
{
    atomicMin(rlo + p, z);
    atomicMax(rhi + p, z);
}

// Push phase of one sweep (labels fixed).  The thread owning column p walks
// its work range top-down (kDown) or bottom-up; each node with excess pushes
// along admissible arcs d(u) = d(w) + len(u, w): to t, down the column,
// along reverse lateral arcs (cancelling flow first), along forward lateral
// arcs, and up along reverse down arcs.  Excess moving in the walking
// direction is carried in a register to the next node of the same walk, so
// the walk continues past the range while a carry is alive.
template <bool kDown>
__global__ __launch_bounds__(256) void k_push(Geom g, State st, const int *__restrict__ rlo_in,
                                              const int *__restrict__ rhi_in, int *rlo_out,
                                              int *rhi_out, Scratch *s)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= g.P) return;
    const int lo = rlo_in[p], hi = rhi_in[p];
    if (lo > hi) return;
    const int P = g.P, K = g.K, N = g.N, dl = g.delta;
    int x = p / g.ny, y = p - x * g.ny;
    int q[4];
    for (int k = 0; k < 4; ++k) q[k] = nbr(g, x, y, p, k);
    int err = 0;
    int mylo = K, myhi = -1;   // own nodes left holding excess
    long long carry = 0;
    // walk index i: z = hi - i (down) or lo + i (up)
    const int span = kDown ? hi + 1 : K - lo;
    const int first = kDown ? hi : lo;
    for (int i0 = 0; i0 < span; i0 += kCh) {
        if (i0 > (hi - lo) && carry == 0) break;
        int ev[kCh], dv[kCh];
#pragma unroll
        for (int j = 0; j < kCh; ++j) {
            const int i = i0 + j;
            ev[j] = 0;
            dv[j] = kInf;
            if (i >= span) continue;
            const int u = (kDown ? first - i : first + i) * P + p;
            ev[j] = st.e[u];
            dv[j] = st.d[u];
        }
        for (int j = 0; j < kCh; ++j) {
            const int i = i0 + j;
            if (i >= span || (i > hi - lo && carry == 0)) break;
            const int z = kDown ? first - i : first + i;
            const int u = z * P + p;
            long long ex = carry;
            carry = 0;
            const int eu = ev[j];
            if (eu <= 0 && ex == 0) continue;
            const int du = dv[j];
            if (du >= kInf) {
                if (ex) add_excess(st.e, u, ex, err);   // not reached: carries follow admissible arcs
                continue;
            }
            if (eu > 0) ex += atomicExch(st.e + u, 0);
            if (du == 1) {
                int r = st.ts[u];
                if (r > 0) {
                    int a = (int)min<long long>(ex, r);
                    st.ts[u] = r - a;
                    ex -= a;
                }
            }
            if (ex > 0 && z > 0 && st.d[u - P] == du) {
                st.fd[u] = add_flow(st.fd[u], ex, err);
                if (kDown) {
                    carry = ex;
                } else {
                    add_excess(st.e, u - P, ex, err);
                    mylo = min(mylo, z - 1);
                    myhi = max(myhi, z - 1);
                }
                ex = 0;
            }
            if (ex > 0) {
                int zt = lat_tail(z, dl, K);
                if (zt >= 0) {
                    for (int k = 0; k < 4 && ex > 0; ++k) {
                        if (q[k] < 0) continue;
                        int w = zt * P + q[k];
                        int *fp = st.fl + (size_t)(k ^ 1) * N + w;
                        int f = *fp;
                        if (f > 0 && st.d[w] + 1 == du) {
                            int a = (int)min<long long>(ex, f);
                            *fp = f - a;
                            add_excess(st.e, w, a, err);
                            note_range(rlo_out, rhi_out, q[k], zt);
                            ex -= a;
                        }
                    }
                }
            }
            if (ex > 0 && lat_arc(z, dl)) {
                const int zh = lat_head(z, dl);
                for (int k = 0; k < 4; ++k) {
                    if (q[k] < 0) continue;
                    int w = zh * P + q[k];
                    if (st.d[w] + 1 == du) {
                        st.fl[(size_t)k * N + u] = add_flow(st.fl[(size_t)k * N + u], ex, err);
                        add_excess(st.e, w, ex, err);
                        note_range(rlo_out, rhi_out, q[k], zh);
                        ex = 0;
                        break;
                    }
                }
            }
            if (ex > 0 && z + 1 < K) {
                int w = u + P;
                int f = st.fd[w];
                if (f > 0 && st.d[w] + 1 == du) {
                    int a = (int)min<long long>(ex, f);
                    st.fd[w] = f - a;
                    if (kDown) {
                        add_excess(st.e, w, a, err);
                        mylo = min(mylo, z + 1);
                        myhi = max(myhi, z + 1);
                    } else {
                        carry = a;
                    }
                    ex -= a;
                }
            }
            if (ex > 0) {
                add_excess(st.e, u, ex, err);
                mylo = min(mylo, z);
                myhi = max(myhi, z);
            }
        }
    }
    if (mylo <= myhi) {
        atomicMin(rlo_out + p, mylo);
        atomicMax(rhi_out + p, myhi);
    }
    if (err) atomicOr(&s->err, kErrOverflow);
}

// Relabel phase of one sweep (flows fixed): every node of the work range
// with excess, a finite label and no admissible arc takes d(u) = min over
// residual arcs of d(w) + len(u, w) (kInf when that exceeds every possible
// distance).  The range is then tightened to the nodes that stay active,
// which are counted; the push phase's input range is reset for reuse.
__global__ __launch_bounds__(256) void k_relabel(Geom g, State st, int *rlo, int *rhi,
                                                 int *rlo_reset, int *rhi_reset, Scratch *s)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    int cnt = 0;
    if (p < g.P) {
        const int P = g.P, K = g.K, N = g.N, dl = g.delta;
        rlo_reset[p] = K;
        rhi_reset[p] = -1;
        const int lo = rlo[p], hi = rhi[p];
        int alo = K, ahi = -1;
        if (lo <= hi) {
            int x = p / g.ny, y = p - x * g.ny;
            int q[4];
            for (int k = 0; k < 4; ++k) q[k] = nbr(g, x, y, p, k);
            int prev = lo > 0 ? st.d[(lo - 1) * P + p] : kInf;
            for (int z0 = lo; z0 <= hi; z0 += kCh) {
                int ev[kCh], dv[kCh];
#pragma unroll
                for (int j = 0; j < kCh; ++j) {
                    const int z = z0 + j;
                    ev[j] = 0;
                    dv[j] = kInf;
                    if (z > hi) continue;
                    ev[j] = st.e[z * P + p];
                    dv[j] = st.d[z * P + p];
                }
                for (int j = 0; j < kCh; ++j) {
                    const int z = z0 + j;
                    if (z > hi) break;
                    const int u = z * P + p;
                    int du = dv[j];
                    if (du < kInf && ev[j] > 0) {
                        int b = prev;
                        if (st.ts[u] > 0) b = min(b, 1);
                        if (z + 1 < K && st.fd[u + P] > 0) b = min(b, st.d[u + P] + 1);
                        if (lat_arc(z, dl)) {
                            int zh = lat_head(z, dl) * P;
                            for (int k = 0; k < 4; ++k)
                                if (q[k] >= 0) b = min(b, st.d[zh + q[k]] + 1);
                        }
                        int zt = lat_tail(z, dl, K);
                        if (zt >= 0) {
                            for (int k = 0; k < 4; ++k) {
                                if (q[k] < 0) continue;
                                int w = zt * P + q[k];
                                if (st.fl[(size_t)(k ^ 1) * N + w] > 0) b = min(b, st.d[w] + 1);
                            }
                        }
                        if (b > du) {
                            du = b >= g.lab_cap ? kInf : b;
                            st.d[u] = du;
                        }
                        if (du < kInf) {
                            ++cnt;
                            alo = min(alo, z);
                            ahi = z;
                        }
                    }
                    prev = du;
                }
            }
        }
        rlo[p] = alo;
        rhi[p] = ahi;
    }
    cnt = wave_sum(cnt);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(&s->active, cnt);
}

// Minimum cut: S_min is the set reached in the residual graph from the
// nodes that keep excess (the source arcs are saturated).  Down arcs are
// always residual, so S_min meets every column in a prefix {0..h(p)}; the
// passes below raise h to the fixed point of the residual arcs.
__global__ __launch_bounds__(256) void k_mincut_init(Geom g, State st, int *H)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= g.P) return;
    int h = -1;
    for (int z = 0; z < g.K; ++z)
        if (st.e[z * g.P + p] > 0) h = z;
    H[p] = h;
}

__global__ __launch_bounds__(256) void k_mincut_pass(Geom g, State st, int *H, Scratch *s)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= g.P) return;
    const int P = g.P, K = g.K, N = g.N, dl = g.delta;
    int x = p / g.ny, y = p - x * g.ny;
    const int h0 = H[p];
    int h = h0;
    for (int k = 0; k < 4; ++k) {
        int qq = nbr(g, x, y, p, k);
        if (qq < 0) continue;
        int hq = H[qq];
        if (hq < 0) continue;
        // forward lateral arcs of q's reached prefix land at heights <= hq - delta (or 0)
        h = max(h, hq > dl ? hq - dl : 0);
        // reverse residual of p's own lateral arcs into q's reached prefix
        int top = min(K - 1, hq + dl);
        for (int z = top; z > h; --z) {
            if (lat_arc(z, dl) && st.fl[(size_t)k * N + z * P + p] > 0) { h = z; break; }
        }
    }
    // reverse residual of down arcs with flow: (p,h) -> (p,h+1)
    while (h >= 0 && h + 1 < K && st.fd[(h + 1) * P + p] > 0) ++h;
    if (h != h0) {
        H[p] = h;
        s->changed = 1;
    }
}

// Flow value F = sum_v (w+(v) - ts(v)) and energy E = sum_p c(p, h(p)).
__global__ __launch_bounds__(256) void k_finish(const int *__restrict__ cost, Geom g, State st,
                                                const int *H, Scratch *s)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    long long r = 0, en = 0;
    if (p < g.P) {
        for (int z = 0; z < g.K; ++z) r += st.ts[z * g.P + p];
        int h = H[p];
        if (h >= 0) en = cost[(long long)p * g.K + h];
    }
    r = wave_sum64(r);
    en = wave_sum64(en);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd((unsigned long long *)&s->flow, (unsigned long long)(-r));
        atomicAdd((unsigned long long *)&s->energy, (unsigned long long)en);
    }
}

// Level-major state -> caller's z-fastest layout.
__global__ void k_export(Geom g, State st, int *e, int *ts, int *fd, int *fl)
{
    long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= g.N) return;
    int p = (int)(o / g.K), z = (int)(o - (long long)p * g.K);
    int v = z * g.P + p;
    e[o] = st.e[v];
    ts[o] = st.ts[v];
    fd[o] = st.fd[v];
    for (int k = 0; k < 4; ++k) fl[(long long)k * g.N + o] = st.fl[(long long)k * g.N + v];
}

// ---- launchers --------------------------------------------------------------

static inline unsigned cols_blocks(const Geom &g) { return (unsigned)((g.P + 255) / 256); }

void launch_init_scratch(Scratch *s, hipStream_t st) { hipLaunchKernelGGL(k_init_scratch, 1, 1, 0, st, s); }
void launch_set_int(int *p, int v, hipStream_t st) { hipLaunchKernelGGL(k_set_int, 1, 1, 0, st, p, v); }

void launch_build(const int *cost, const Geom &g, const State &sv, Scratch *s, hipStream_t st)
{
    hipLaunchKernelGGL(k_bottom_max, dim3(cols_blocks(g)), dim3(256), 0, st, cost, g.P, g.K, s);
    dim3 grid((g.P + 63) / 64, (g.K + 63) / 64);
    hipLaunchKernelGGL(k_build, grid, dim3(256), 0, st, cost, g, sv, s);
}

void launch_bfs_init(const Geom &g, const State &sv, int *T, int *LF, int *chg, Scratch *s,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_bfs_init, dim3(cols_blocks(g)), dim3(256), 0, st, g, sv, T, LF, chg, s);
}

void launch_bfs_level(const Geom &g, const State &sv, int L, const int *Tin, const int *LFin,
                      const int *chg_in, int *Tout, int *LFout, int *chg_out, Scratch *s,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_bfs_level, dim3(cols_blocks(g)), dim3(256), 0, st, g, sv, L, Tin, LFin,
                       chg_in, Tout, LFout, chg_out, s);
}

void launch_bfs_fixup(const Geom &g, const State &sv, int v, hipStream_t st)
{
    unsigned blocks = (unsigned)(((long long)g.N + 255) / 256);
    hipLaunchKernelGGL(k_bfs_fixup, dim3(blocks), dim3(256), 0, st, sv.d, g.N, v);
}

void launch_fill(int *a, int n, int v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n, v);
}

void launch_push(const Geom &g, const State &sv, const int *rlo_in, const int *rhi_in,
                 int *rlo_out, int *rhi_out, Scratch *s, bool down, hipStream_t st)
{
    if (down)
        hipLaunchKernelGGL(k_push<true>, dim3(cols_blocks(g)), dim3(256), 0, st, g, sv, rlo_in,
                           rhi_in, rlo_out, rhi_out, s);
    else
        hipLaunchKernelGGL(k_push<false>, dim3(cols_blocks(g)), dim3(256), 0, st, g, sv, rlo_in,
                           rhi_in, rlo_out, rhi_out, s);
}

void launch_relabel(const Geom &g, const State &sv, int *rlo, int *rhi, int *rlo_reset,
                    int *rhi_reset, Scratch *s, hipStream_t st)
{
    hipLaunchKernelGGL(k_relabel, dim3(cols_blocks(g)), dim3(256), 0, st, g, sv, rlo, rhi,
                       rlo_reset, rhi_reset, s);
}

void launch_mincut_init(const Geom &g, const State &sv, int *H, hipStream_t st)
{
    hipLaunchKernelGGL(k_mincut_init, dim3(cols_blocks(g)), dim3(256), 0, st, g, sv, H);
}

void launch_mincut_pass(const Geom &g, const State &sv, int *H, Scratch *s, hipStream_t st)
{
    hipLaunchKernelGGL(k_mincut_pass, dim3(cols_blocks(g)), dim3(256), 0, st, g, sv, H, s);
}

void launch_finish(const int *cost, const Geom &g, const State &sv, const int *H, Scratch *s,
                   hipStream_t st)
{
    hipLaunchKernelGGL(k_finish, dim3(cols_blocks(g)), dim3(256), 0, st, cost, g, sv, H, s);
}

void launch_export(const Geom &g, const State &sv, int *e, int *ts, int *fd, int *fl,
                   hipStream_t st)
{
    unsigned blocks = (unsigned)(((long long)g.N + 255) / 256);
    hipLaunchKernelGGL(k_export, dim3(blocks), dim3(256), 0, st, g, sv, e, ts, fd, fl);
}

}  // namespace smf
