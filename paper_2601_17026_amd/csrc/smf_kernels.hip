// HIP kernels of the exact surface max-flow (gfx950).
//
// Method: push-relabel (Section 2.1) on the implicit column graph of
// Section 1.2, with global relabelling by a reverse breadth-first search
// from the sink (Section 2.1, "global relabeling"; Section 3.2.2 and
// Algorithm 3) and the minimum cut read out as the residual reach set
// (Section 1.3, Eq. 6, Theorem 1.1).  Storage is implicit (Section 3.2.3):
// no edge lists, only per-node excess, label, sink residual and the flows of
// the five outgoing infinite arcs.
//
// Batches.  Every kernel works on all volumes of a batch at once: columns
// are numbered across the batch, each column finds its volume's geometry in
// the volume table, and counters are kept per volume.  No arc joins two
// volumes, so the volumes' solves only share launches.
//
// Labels.  A valid labelling satisfies d(u) <= d(w) + len(u, w) for every
// residual arc, with len = 0 for the always-residual down arcs
// (p,z) -> (p,z-1) and len = 1 for every other arc (sink arcs included,
// d(t) = 0).  Down arcs form no cycle, so pushes along them cannot
// circulate, and d(v) stays a lower bound of the weighted residual distance
// to t: a node whose label exceeds N cannot reach t.  Zero-length down arcs
// let excess fall a whole column per sweep and make exact labels
// non-increasing up every column, which the breadth-first search exploits.
//
// Concurrency.  A sweep is two launches: a push phase with all labels fixed,
// then a relabel phase with all flows fixed.  In the push phase a wave owns a
// column; an arc and its reverse are never both admissible under fixed
// labels, so every flow counter has a single writer per phase, and only the
// excess counters of other columns take atomics.  In the relabel phase labels
// only grow, so a neighbour's old or new label both keep the labelling valid.
#include "smf_device.h"
#include <limits.h>

namespace smf {

// ---- wave utilities ---------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// A value every lane holds alike, moved to a scalar register so that the
// addresses computed from it use scalar loads.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int wave_sum(int v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ long long wave_sum(long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ long long shfl64(long long v, int src)
{
    int lo = __shfl((int)(v & 0xffffffffLL), src, kWave);
    int hi = __shfl((int)(v >> 32), src, kWave);
    return ((long long)hi << 32) | (unsigned int)lo;
}

__device__ __forceinline__ long long shfl64_down(long long v, int off)
{
    int lo = __shfl_down((int)(v & 0xffffffffLL), off, kWave);
    int hi = __shfl_down((int)(v >> 32), off, kWave);
    return ((long long)hi << 32) | (unsigned int)lo;
}

__device__ __forceinline__ long long shfl64_up(long long v, int off)
{
    int lo = __shfl_up((int)(v & 0xffffffffLL), off, kWave);
    int hi = __shfl_up((int)(v >> 32), off, kWave);
    return ((long long)hi << 32) | (unsigned int)lo;
}

// Field `f` of the counters of volume i, given the same field of volume 0.
template <typename T>
__device__ __forceinline__ T *inst_field(T *f0, int i)
{
    return (T *)((char *)f0 + (size_t)i * sizeof(InstScratch));
}

__device__ __forceinline__ void atomic_add(int *p, int v) { atomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(long long *p, long long v)
{
    atomicAdd((unsigned long long *)p, (unsigned long long)v);   // two's complement
}

// Adds `val` of every lane with `has` to field f0 of the lane's volume
// `key`: one atomic per distinct volume among the lanes (the lanes of a
// wave nearly always share one).  Called by all lanes of the wave.
template <typename T>
__device__ __forceinline__ void wave_add_keyed(T *f0, int key, T val, bool has)
{
    const int lane = lane_id();
    bool pending = has && val != 0;
    for (;;) {
        const unsigned long long b = __ballot(pending);
        if (!b) break;
        const int leader = __ffsll((long long)b) - 1;
        const int k = __shfl(key, leader, kWave);
        const bool mine = pending && key == k;
        const T s = wave_sum(mine ? val : (T)0);
        if (lane == leader) atomic_add(inst_field(f0, k), s);
        if (mine) pending = false;
    }
}

// Running per-volume sum of a wave that visits columns in order: the lanes'
// partial sums are flushed with one atomic whenever the volume changes.
template <typename T>
struct VolSum {
    T *f0;
    int cur = -1;
    T acc = 0;
    __device__ explicit VolSum(T *f) : f0(f) {}
    // `ii` is wave-uniform
    __device__ void to(int ii)
    {
        if (ii == cur) return;
        flush();
        cur = ii;
    }
    __device__ void flush()
    {
        if (cur >= 0) {
            const T s = wave_sum(acc);
            if (lane_id() == 0 && s) atomic_add(inst_field(f0, cur), s);
        }
        acc = 0;
    }
};

// Ends a per-volume sum in a kernel of 256-thread blocks that every thread
// reaches: the four waves' last partial sums are combined in LDS and added
// with one atomic per distinct volume of the block, so a counter takes a
// few atomics per block rather than one per wave (atomics on one address
// from many waves serialise).
template <typename T>
__device__ void block_flush(VolSum<T> &vs)
{
    __shared__ int vol[4];
    __shared__ T sum[4];
    const T part = wave_sum(vs.acc);
    const int w = threadIdx.x / kWave;
    __syncthreads();   // an earlier call may still read the arrays
    if (lane_id() == 0) {
        vol[w] = (vs.cur >= 0 && part != 0) ? vs.cur : -1;
        sum[w] = part;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x / kWave;
        for (int i = 0; i < nw; ++i) {
            if (vol[i] < 0) continue;
            T tot = sum[i];
            for (int j = i + 1; j < nw; ++j)
                if (vol[j] == vol[i]) {
                    tot += sum[j];
                    vol[j] = -1;
                }
            atomic_add(inst_field(vs.f0, vol[i]), tot);
        }
    }
    vs.acc = 0;
    vs.cur = -1;
}

// Adds a wave's algorithmic bytes (state words read or written, each access
// counted once) to the solve counter of kernel class `cls`.
__device__ __forceinline__ void count_bytes(const Geom &g, int cls, long long lane_bytes)
{
    const long long b = wave_sum(lane_bytes);
    if ((threadIdx.x & (kWave - 1)) == 0 && b)
        atomicAdd(g.work + ((size_t)cls * kWorkSlots + (blockIdx.x & (kWorkSlots - 1))) * kWorkStride,
                  (unsigned long long)b);
}

__device__ __forceinline__ int add_flow(int f, long long a, int &err)
{
    long long r = (long long)f + a;
    if (r > INT_MAX) { err = 1; r = INT_MAX; }
    return (int)r;
}

// Contiguous share [lo, hi) of the columns [c0, c1) for the wave-per-column
// kernels, so that a wave meets few volume boundaries.
__device__ __forceinline__ void wave_range(int c0, int c1, int &lo, int &hi)
{
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int nwaves = gridDim.x * blockDim.x / kWave;
    const int per = (c1 - c0 + nwaves - 1) / nwaves;
    lo = min(c1, c0 + wave * per);
    hi = min(c1, lo + per);
}

__device__ __forceinline__ void wave_columns(const Geom &g, int &lo, int &hi)
{
    wave_range(0, g.Ptot, lo, hi);
}

// Geometry of the column's volume, with the column's local coordinates.
struct Col {
    Inst I;
    int ii;        // volume
    int pl, x, y;  // local column and its coordinates
    size_t base;   // global node of (p, 0)
};

__device__ __forceinline__ Col column_of(const Geom &g, int p, int ii)
{
    Col c;
    c.ii = ii;
    c.I = g.inst[ii];
    c.pl = p - c.I.col_base;
    c.x = c.pl / c.I.ny;
    c.y = c.pl - c.x * c.I.ny;
    c.base = (size_t)c.I.node_base + (size_t)c.pl * c.I.K;
    return c;
}

__device__ __forceinline__ Col column(const Geom &g, int p) { return column_of(g, p, g.col_inst[p]); }

// Column of the volume `I` (already loaded) of index ii.
__device__ __forceinline__ Col column_in(const Inst &I, int ii, int p)
{
    Col c;
    c.ii = ii;
    c.I = I;
    c.pl = p - I.col_base;
    c.x = c.pl / I.ny;
    c.y = c.pl - c.x * I.ny;
    c.base = (size_t)I.node_base + (size_t)c.pl * I.K;
    return c;
}

// Same for a wave-uniform column: the volume table is read with scalar loads.
__device__ __forceinline__ Col column_uniform(const Geom &g, int p)
{
    return column_of(g, p, uniform(g.col_inst[p]));
}

// Volume of a run of wave-uniform columns: the volume table is read again
// only when a column lies outside the volume of the previous one.
struct VolCache {
    int ii = -1;
    Inst I;
    // true when the volume changed
    __device__ __forceinline__ bool at(const Geom &g, int p)
    {
        if (ii >= 0 && (unsigned)(p - I.col_base) < (unsigned)I.P) return false;
        ii = uniform(g.col_inst[p]);
        I = g.inst[ii];
        return true;
    }
    __device__ __forceinline__ size_t base(int p) const
    {
        return (size_t)I.node_base + (size_t)(p - I.col_base) * I.K;
    }
};

// ---- carries along a column as a scan of clamp functions --------------------
//
// Within one push phase the excess that leaves a node along its column arc
// is a function of the excess that arrives from the previous node of the
// walk: c -> min(U, max(L, c + A)).  Such clamp functions are closed under
// composition, so the carries of 64 consecutive heights follow from one
// wave-wide scan instead of a 64-step dependency chain.
constexpr long long kBig = 1LL << 60;

template <typename V>
struct ClampT {
    V A, L, U;
};
using Clamp = ClampT<long long>;

template <typename V>
__device__ __forceinline__ V clampv(V x, V l, V u)
{
    return x < l ? l : (x > u ? u : x);
}

template <typename V>
__device__ __forceinline__ V apply(const ClampT<V> &f, V c)
{
    return clampv<V>(c + f.A, f.L, f.U);
}

// s o t: apply t first, then s.
template <typename V>
__device__ __forceinline__ ClampT<V> compose(const ClampT<V> &s, const ClampT<V> &t)
{
    ClampT<V> r;
    r.A = t.A + s.A;
    r.L = clampv<V>(t.L + s.A, s.L, s.U);
    r.U = clampv<V>(t.U + s.A, s.L, s.U);
    return r;
}

__device__ __forceinline__ int shflv(int v, int src) { return __shfl(v, src, kWave); }
__device__ __forceinline__ int shflv_down(int v, int off) { return __shfl_down(v, off, kWave); }
__device__ __forceinline__ int shflv_up(int v, int off) { return __shfl_up(v, off, kWave); }
__device__ __forceinline__ long long shflv(long long v, int src) { return shfl64(v, src); }
__device__ __forceinline__ long long shflv_down(long long v, int off) { return shfl64_down(v, off); }
__device__ __forceinline__ long long shflv_up(long long v, int off) { return shfl64_up(v, off); }

// Carry into every lane of a 64-height chunk and out of it, for the clamp
// function f of each lane and the carry c entering the chunk: a suffix scan
// (walking down, the carry enters at lane 63) or a prefix scan (walking up).
template <bool kDown, typename V>
__device__ __forceinline__ void chunk_carry(const ClampT<V> &f, long long c, int lane, long long &cin,
                                            long long &cout)
{
    ClampT<V> sc = f;
    const V cv = (V)c;
    if (kDown) {
        for (int off = 1; off < kWave; off <<= 1) {
            const ClampT<V> o = {shflv_down(sc.A, off), shflv_down(sc.L, off), shflv_down(sc.U, off)};
            if (lane + off < kWave) sc = compose(sc, o);
        }
        const ClampT<V> prev = {shflv_down(sc.A, 1), shflv_down(sc.L, 1), shflv_down(sc.U, 1)};
        cin = lane + 1 < kWave ? (long long)apply(prev, cv) : c;
        const ClampT<V> all = {shflv(sc.A, 0), shflv(sc.L, 0), shflv(sc.U, 0)};
        cout = (long long)apply(all, cv);
    } else {
        for (int off = 1; off < kWave; off <<= 1) {
            const ClampT<V> o = {shflv_up(sc.A, off), shflv_up(sc.L, off), shflv_up(sc.U, off)};
            if (lane >= off) sc = compose(sc, o);
        }
        const ClampT<V> prev = {shflv_up(sc.A, 1), shflv_up(sc.L, 1), shflv_up(sc.U, 1)};
        cin = lane > 0 ? (long long)apply(prev, cv) : c;
        const ClampT<V> all = {shflv(sc.A, kWave - 1), shflv(sc.L, kWave - 1), shflv(sc.U, kWave - 1)};
        cout = (long long)apply(all, cv);
    }
}

// The scan runs in 32-bit arithmetic when every lane's |A| is at most
// kSmallA and the entering carry at most kSmallCarry: then every partial
// composition and every carry stays below 2^27, so capping U at kCapU
// (> 2^27) changes no result and nothing overflows.
constexpr long long kSmallA = 1LL << 20, kSmallCarry = 1LL << 26, kCapU = 1LL << 29;

// ---- label histogram (gap heuristic) ---------------------------------------------
//
// With labels that drop by at most one along a residual arc (len <= 1), a
// label g held by no node cuts every node labelled above g off from t
// (Section 2.1, gap relabelling).  The histogram of each volume's finite
// labels below hist_len is rebuilt from all its nodes whenever a gap search
// runs.

// Per-block histogram in LDS, flushed to the volume's global one; blockIdx.y
// is the volume.
__global__ __launch_bounds__(256) void k_hist_build(Geom g, const int *__restrict__ d)
{
    extern __shared__ int bins[];
    const int ii = blockIdx.y;
    const Inst I = g.inst[ii];
    const int len = g.hist_len;
    for (int i = threadIdx.x; i < len; i += blockDim.x) bins[i] = 0;
    __syncthreads();
    const long long stride = (long long)gridDim.x * blockDim.x;
    const int *dv = d + I.node_base;
    for (long long v = blockIdx.x * blockDim.x + threadIdx.x; v < I.N; v += stride) {
        const int l = dv[v];
        if (l >= 1 && l < len) atomicAdd(&bins[l], 1);
    }
    __syncthreads();
    int *h = g.hist + (size_t)ii * len;
    for (int i = threadIdx.x; i < len; i += blockDim.x)
        if (bins[i]) atomicAdd(h + i, bins[i]);
}

// First label >= 1 held by no node while some node holds a larger label
// (kInf if none): one block per volume scans its histogram.
__global__ __launch_bounds__(1024) void k_gap_find(Geom g)
{
    __shared__ int first_zero, last_used;
    const int ii = blockIdx.x;
    if (threadIdx.x == 0) {
        first_zero = INT_MAX;
        last_used = 0;
    }
    __syncthreads();
    const int len = g.hist_len;
    const int *h = g.hist + (size_t)ii * len;
    const int per = (len + blockDim.x - 1) / blockDim.x;
    const int lo = max(1, (int)threadIdx.x * per), hi = min(len, ((int)threadIdx.x + 1) * per);
    int fz = INT_MAX, lu = 0;
    for (int l = lo; l < hi; ++l) {
        const int c = h[l];
        if (c == 0 && fz == INT_MAX) fz = l;
        if (c > 0) lu = l;
    }
    if (fz != INT_MAX) atomicMin(&first_zero, fz);
    if (lu) atomicMax(&last_used, lu);
    __syncthreads();
    if (threadIdx.x == 0) g.is[ii].gap = first_zero < last_used ? first_zero : kInf;
}

// ---- small kernels ------------------------------------------------------------

__global__ void k_init_scratch(Geom g, Scratch *s)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < g.n) {
        InstScratch &r = g.is[i];
        r.flow = 0;
        r.energy = 0;
        r.bmax = INT_MIN;
        r.active = 0;
        r.bfs_active = 0;
        r.bfs_unsat[0] = r.bfs_unsat[1] = 0;
        r.gap = kInf;
        r.gap_frozen = 0;
    }
    if (i == 0) {
        s->err = 0;
        s->changed = 0;
        s->block_levels = 0;
        s->block_done = 0;
        s->count[0] = 0;
        s->count[1] = 0;
    }
}

__global__ void k_set_int(int *p, int v) { *p = v; }

__global__ void k_fill(int *a, long long n, int v)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = v;
}

// Work lists before the first sweep: every column, every chunk group.
__global__ void k_work_init(Geom g, Work a, Work b)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < g.Ptot) {
        const Inst I = g.inst[g.col_inst[p]];
        const int bits = (I.nch + I.cpb - 1) / I.cpb;
        a.mask[p] = bits >= 64 ? ~0ULL : ((1ULL << bits) - 1);
        a.list[p] = p;
        b.mask[p] = 0;
    }
    if (p == 0) *a.count = g.Ptot;
}

// B - 1 = max_p c(p, 0) per volume: the bottom shift that makes every
// bottom node a source node (w(p,0) < 0), so that the empty cut never wins.
__global__ void k_bottom_max(const int *__restrict__ cost, Geom g)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = lane_id();
    int ii = -1, v = INT_MIN;
    if (p < g.Ptot) {
        const Col c = column(g, p);
        ii = c.ii;
        v = cost[(size_t)c.I.cost_base + (size_t)c.pl * c.I.K + (g.band ? g.bcs[p] : 0)];
    }
    bool pending = ii >= 0;
    for (;;) {
        const unsigned long long b = __ballot(pending);
        if (!b) break;
        const int leader = __ffsll((long long)b) - 1;
        const int k = __shfl(ii, leader, kWave);
        const bool mine = pending && ii == k;
        const int m = wave_max(mine ? v : INT_MIN);
        if (lane == leader) atomicMax(&g.is[k].bmax, m);
        if (mine) pending = false;
    }
}

// Graph build, one wave per column: node weights w (Section 1.2), source
// arcs pre-saturated into the excess (Section 2.1 initialisation), sink
// residuals, zero flows and labels 0 (valid lower bounds) until the first
// breadth-first search.  The state has the cost volume's own layout.
__global__ __launch_bounds__(256) void k_build(const int *__restrict__ cost, Geom g, State st,
                                               Scratch *s)
{
    const int lane = lane_id();
    int lo, hi;
    wave_columns(g, lo, hi);
    int bad = 0;
    VolSum<long long> ts_sum(&g.is[0].flow);
    for (int p = lo; p < hi; ++p) {
        const Col c = column_uniform(g, p);
        ts_sum.to(c.ii);
        const int K = c.I.K;
        const int B = g.is[c.ii].bmax + 1;
        const int ext = g.band ? g.bext[p] : K;   // node slots the column uses
        const size_t cb0 = (size_t)c.I.cost_base + (size_t)c.pl * K + (g.band ? g.bcs[p] : 0);
        for (int ch = 0; ch < c.I.nch; ++ch) {
            const int z = ch * kWave + lane;
            const bool in = z < K;
            const bool live = z < ext;
            const int cv = live ? cost[cb0 + z] : 0;
            const int up = __shfl_up(cv, 1, kWave);
            const int cbelow = z == 0 ? B : (lane == 0 ? (live ? cost[cb0 + z - 1] : 0) : up);
            if (!in) continue;
            const size_t v = c.base + z;
            if (!live) {
                // an unused slot above the column's band: no excess, no arcs
                st.e[v] = 0;
                st.ts[v] = 0;
                st.d[v] = kInf;
                st.fd[v] = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) st.fl[(size_t)k * g.Ntot + v] = 0;
                continue;
            }
            if (cv <= -(1 << 30) || cv >= (1 << 30)) bad = 1;
            const int w = cv - cbelow;
            st.e[v] = w < 0 ? -w : 0;
            st.ts[v] = w > 0 ? w : 0;
            ts_sum.acc += w > 0 ? w : 0;
            st.d[v] = 0;
            st.fd[v] = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) st.fl[(size_t)k * g.Ntot + v] = 0;
        }
    }
    block_flush(ts_sum);
    if (bad) atomicOr(&s->err, kErrCostRange);
}

// ---- push phase -----------------------------------------------------------

// Appends `value` for every lane with `want` to a device list with one
// counter atomic per wave (a single counter shared by all waves would
// otherwise serialise every append).  Called by all lanes of the wave.
__device__ __forceinline__ void wave_append(int *list, int *count, bool want, int value)
{
    const unsigned long long b = __ballot(want);
    if (!b) return;
    const int lane = lane_id();
    const int leader = __ffsll((long long)b) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(b));
    base = __shfl(base, leader, kWave);
    if (want) list[base + __popcll(b & ((1ULL << lane) - 1ULL))] = value;
}

// Records that column q may hold work in the chunk groups `bits` after the
// push phase.  No value is returned, so the wave does not wait for it; the
// phase's column list is built afterwards from the masks (k_compact).
__device__ __forceinline__ void mark_mask(const Work &w, int q, unsigned long long bits)
{
    atomicOr(w.mask + q, bits);
}

// Column list of every column with a non-empty work mask.  Also clears the
// counters that the relabel phase after it fills: the size of its output
// list and the per-volume active counts.  A block of 1024 columns takes its
// share of the list with one atomic (one per wave serialised on the single
// counter when the columns number millions).
__global__ __launch_bounds__(1024) void k_compact(Geom g, Work w, int *next_count)
{
    __shared__ int wave_n[16], block_base;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    if (p == 0) *next_count = 0;
    if (p < g.n) g.is[p].active = 0;
    const bool want = p < g.Ptot && w.mask[p] != 0;
    const unsigned long long b = __ballot(want);
    if (lane == 0) wave_n[wid] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        int total = 0;
        for (int i = 0; i < (int)blockDim.x / kWave; ++i) total += wave_n[i];
        block_base = total ? atomicAdd(w.count, total) : 0;
    }
    __syncthreads();
    int off = block_base;
    for (int i = 0; i < wid; ++i) off += wave_n[i];
    if (want) w.list[off + __popcll(b & ((1ULL << lane) - 1ULL))] = p;
}

// Loads of one 64-height chunk of a column: the node words of every lane,
// plus the label below lane 0 and the label and down flow above lane 63.
struct ChunkIn {
    int e, d, ts, fd;      // this lane's node
    int d_below;           // label of (p, z-1) (kInf at z = 0 or outside)
    int d_above, fd_above; // label and down flow of (p, z+1) (kInf / 0 at the top)
};

__device__ __forceinline__ ChunkIn load_chunk(const State &st, size_t v, int z, int K, int lane)
{
    ChunkIn r;
    const bool in = z < K;
    r.e = in ? st.e[v] : 0;
    r.d = in ? st.d[v] : kInf;
    r.ts = in ? st.ts[v] : 0;
    r.fd = in ? st.fd[v] : 0;
    const int edge_below = (lane == 0 && in && z > 0) ? st.d[v - 1] : kInf;
    const bool top_lane = lane == kWave - 1 && z + 1 < K;
    const int edge_d_above = top_lane ? st.d[v + 1] : kInf;
    const int edge_fd_above = top_lane ? st.fd[v + 1] : 0;
    const int sd_below = __shfl_up(r.d, 1, kWave);
    const int sd_above = __shfl_down(r.d, 1, kWave);
    const int sfd_above = __shfl_down(r.fd, 1, kWave);
    r.d_below = lane == 0 ? edge_below : (in ? sd_below : kInf);
    if (lane == kWave - 1) {
        r.d_above = edge_d_above;
        r.fd_above = edge_fd_above;
    } else {
        r.d_above = z + 1 < K ? sd_above : kInf;
        r.fd_above = z + 1 < K ? sfd_above : 0;
    }
    return r;
}

// Lateral neighbourhood of one node: labels of the heads of its forward
// lateral arcs, and flow and tail label of the lateral arcs that end at it
// (its reverse residual arcs).  Loaded only for lanes that need them; the
// words of a chunk are 64 consecutive heights of the neighbour column.
// Node (q, 0) of neighbour k lies dq[k] words from the column's node (p, 0)
// at `base` (has[k] false: no neighbour); the arcs' heights follow the
// column's band geometry bc.
struct Lateral {
    int d_fwd[4];   // label of (q, zh) (kInf: no arc)
    int f_rev[4];   // flow on (q, zt) -> (p, z) (0: no arc)
    int d_rev[4];   // label of (q, zt)
};

__device__ __forceinline__ void load_lateral(Lateral &l, const State &st, size_t base,
                                             const int dq[4], const bool has[4], const BandCol &bc,
                                             int z, size_t Ntot, bool need)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool fwd = need && has[k] && lat_arc(z, bc.sh[k]);
        const int zh = lat_head(z, bc.sh[k]);
        const int zt = lat_tail(z, bc.shr[k], bc.qext[k]);
        l.d_fwd[k] = fwd ? st.d[base + (ptrdiff_t)(dq[k] + zh)] : kInf;
        const bool rev = need && has[k] && zt >= 0;
        const size_t w = base + (ptrdiff_t)(rev ? dq[k] + zt : 0);
        l.f_rev[k] = rev ? st.fl[(size_t)(k ^ 1) * Ntot + w] : 0;
        l.d_rev[k] = rev ? st.d[w] : kInf;
    }
}

// Soft smoothness arcs (p,z) -> (q,z), z >= 1, of capacity alpha in every
// direction k: residual capacity alpha - sf[k](p,z) + sf[k^1](q,z) (flow on
// the arc, and flow on its reverse that can be cancelled), and the label of
// the head.  Loaded only for lanes that need them.
struct SoftLat {
    int d[4];      // label of (q, z) (kInf: no arc)
    int own[4];    // flow on (p,z) -> (q,z)
    int back[4];   // flow on (q,z) -> (p,z)
    int r[4];      // residual capacity of (p,z) -> (q,z)
};

__device__ __forceinline__ void load_soft(SoftLat &l, const State &st, size_t base, const int dq[4],
                                          const bool has[4], int z, size_t Ntot, int alpha, bool need)
{
    const size_t v = base + z;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool on = need && alpha > 0 && has[k] && z >= 1;
        const size_t w = base + (ptrdiff_t)(on ? dq[k] + z : 0);
        l.d[k] = on ? st.d[w] : kInf;
        l.own[k] = on ? st.sf[(size_t)k * Ntot + v] : 0;
        l.back[k] = on ? st.sf[(size_t)(k ^ 1) * Ntot + w] : 0;
        l.r[k] = on ? alpha - l.own[k] + l.back[k] : 0;
    }
}

// Global neighbour columns of a column, and the word offsets of their
// nodes (q, 0) from the column's node (p, 0).
__device__ __forceinline__ void neighbours(const Col &c, int p, int q[4], int dq[4], bool has[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        q[k] = nbr(c.I.nx, c.I.ny, c.x, c.y, p, k);
        has[k] = q[k] >= 0;
        dq[k] = (q[k] - p) * c.I.K;
    }
}

// Push phase of one sweep (labels fixed).  A wave takes a column from the
// work list and walks the chunks of its work mask top-down (kDown) or
// bottom-up.  Every node with excess pushes along admissible arcs
// d(u) = d(w) + len(u, w): to t, then along its column arc in the walking
// direction (all of it down a length-0 down arc; up a reverse down arc as
// far as its flow allows), the rest along the column arc against the walking
// direction, reverse lateral arcs (cancelling flow first) and a forward
// lateral arc.  The carries along the column come from one clamp-function
// scan per chunk and continue into the next chunk, so the walk extends past
// the mask while a carry is alive.  A node's excess word is read once and
// corrected by one atomic add of the net change; other columns only add to
// it, so the value read is a valid lower bound of what the node holds.
template <bool kDown, bool kSoft>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_push(Geom g, State st, Work win, Work wout, Scratch *s)
{
    const int lane = lane_id();
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int nwaves = gridDim.x * blockDim.x / kWave;
    const size_t Ntot = (size_t)g.Ntot;
    const int count = *win.count;
    // the list of wout is built by the compaction after this phase
    if (blockIdx.x == 0 && threadIdx.x == 0) *wout.count = 0;
    long long worst = 0;   // largest excess word produced by an atomic add
    long long bytes = 0;   // algorithmic bytes moved by this lane
    int err = 0;
    Inst cur;              // volume of the previous column (reloaded on a change)
    int cur_ii = -1;
    // batches of up to 64 list entries per wave, sized so that every wave of
    // the grid gets one: lane i fetches entry i, then the wave works through
    // the batch one column at a time
    const int bs = min(kWave, max(1, (count + nwaves - 1) / nwaves));
    for (int b0 = wave * bs; b0 < count; b0 += nwaves * bs) {
      const int myp = (lane < bs && b0 + lane < count) ? win.list[b0 + lane] : -1;
      const unsigned long long mym = myp >= 0 ? win.mask[myp] : 0ULL;
      const int myii = myp >= 0 ? g.col_inst[myp] : 0;
      if (myp >= 0) win.mask[myp] = 0;
      unsigned long long myown = 0;
      unsigned long long todo = __ballot(mym != 0);
      while (todo) {
        const int src = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        const int p = uniform(__shfl(myp, src, kWave));
        const unsigned long long m = (unsigned long long)shfl64((long long)mym, src);
        const int ii = uniform(__shfl(myii, src, kWave));
        if (ii != cur_ii) {
            cur = g.inst[ii];
            cur_ii = ii;
        }
        const Col col = column_in(cur, ii, p);
        const int nch = col.I.nch, cpb = col.I.cpb;
        int q[4], dq[4];
        bool has[4];
        neighbours(col, p, q, dq, has);
        BandCol bc;
        band_col(g, p, q, col.I.K, col.I.delta, bc);
        const int K = bc.ext;   // node slots of the column
        const size_t base = col.base;
        const int gtop = 63 - __clzll(m), glow = __ffsll((long long)m) - 1;
        const int ctop = min(nch - 1, gtop * cpb + cpb - 1), clow = glow * cpb;
        unsigned long long own = 0;      // own chunk groups left holding excess
        long long carry = 0;             // wave-uniform carry into the next chunk
        for (int step = 0; step < nch; ++step) {
            const int c = kDown ? ctop - step : clow + step;
            if (c < 0 || c >= nch) break;
            const bool set = (m >> (c / cpb)) & 1ULL;
            if (!set && carry == 0) {
                if (kDown ? c < clow : c > ctop) break;
                continue;
            }
            const int z = c * kWave + lane;
            const bool in = z < K;
            const size_t v = base + z;
            const ChunkIn ci = load_chunk(st, v, z, K, lane);
            bytes += in ? 16 : 0;
            const int dv = ci.d;
            const bool live = in && dv < kInf;
            const long long taken = (live && ci.e > 0) ? ci.e : 0;
            const long long sink_cap = (live && dv == 1) ? ci.ts : 0;
            const bool adm_down = live && z > 0 && ci.d_below == dv;
            const bool adm_up = live && !adm_down && ci.fd_above > 0 && ci.d_above + 1 == dv;
            // the carry function of this node in the walking direction
            Clamp f = {0, 0, 0};
            if (kDown && adm_down) f = {taken - sink_cap, 0, kBig};
            if (!kDown && adm_up) f = {taken - sink_cap, 0, (long long)ci.fd_above};
            // carries into the lanes and out of the chunk: nothing moves when
            // no carry enters and no lane has excess to pass on
            long long cin = 0;
            if (carry != 0 || __ballot(f.A > 0)) {
                long long cout;
                if (carry <= kSmallCarry && !__ballot(f.A < -kSmallA || f.A > kSmallA)) {
                    const ClampT<int> f32 = {(int)f.A, (int)f.L, (int)min(f.U, kCapU)};
                    chunk_carry<kDown, int>(f32, carry, lane, cin, cout);
                } else {
                    chunk_carry<kDown, long long>(f, carry, lane, cin, cout);
                }
                carry = cout;
            }
            long long rem = live ? taken + cin : 0;
            if (rem > 0 && sink_cap > 0) {
                const long long a = min(rem, sink_cap);
                st.ts[v] = ci.ts - (int)a;
                rem -= a;
                bytes += 4;
            }
            // results of excess atomics are only inspected at the end of the
            // chunk, so the wave does not wait for each of them in turn
            int o_col = 0, o_rev[4] = {0, 0, 0, 0}, o_fwd = 0, o_own = 0;
            // amounts those atomics added (an amount beyond int32 has set err)
            int a_col = 0, a_rev[4] = {0, 0, 0, 0}, a_fwd = 0, a_own = 0;
            if (rem > 0 && adm_down) {
                st.fd[v] = add_flow(ci.fd, rem, err);
                bytes += kDown ? 4 : 12;
                if (!kDown) {
                    a_col = (int)min(rem, (long long)INT_MAX);
                    o_col = atomicAdd(st.e + v - 1, a_col);
                    own |= 1ULL << ((z - 1) / kWave / cpb);
                }
                rem = 0;   // walking down: the carry scan already moved it
            }
            if (rem > 0 && adm_up) {
                const long long a = min(rem, (long long)ci.fd_above);
                st.fd[v + 1] = ci.fd_above - (int)a;
                bytes += kDown ? 12 : 4;
                if (kDown) {
                    a_col = (int)a;
                    o_col = atomicAdd(st.e + v + 1, a_col);
                    own |= 1ULL << ((z + 1) / kWave / cpb);
                }
                rem -= a;  // walking up: the carry scan already moved it
            }
            const bool need = rem > 0;
            if (__ballot(need)) {
                Lateral lt;
                load_lateral(lt, st, base, dq, has, bc, z, Ntot, need);
                bytes += need ? 64 : 0;
                SoftLat sl;
                if constexpr (kSoft) {
                    load_soft(sl, st, base, dq, has, z, Ntot, col.I.alpha, need);
                    bytes += need && col.I.alpha > 0 ? 48 : 0;
                }
                int fown[4];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    fown[k] = (need && has[k] && lat_arc(z, bc.sh[k])) ? st.fl[(size_t)k * Ntot + v] : 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const bool go = rem > 0 && lt.f_rev[k] > 0 && lt.d_rev[k] + 1 == dv;
                    const int zt = lat_tail(z, bc.shr[k], bc.qext[k]);
                    if (go) {
                        const long long a = min(rem, (long long)lt.f_rev[k]);
                        const size_t w = base + (ptrdiff_t)(dq[k] + zt);
                        st.fl[(size_t)(k ^ 1) * Ntot + w] = lt.f_rev[k] - (int)a;
                        a_rev[k] = (int)a;
                        o_rev[k] = atomicAdd(st.e + w, a_rev[k]);
                        rem -= a;
                        bytes += 8;
                    }
                    if (go) mark_mask(wout, q[k], 1ULL << (zt / kWave / cpb));
                }
                if constexpr (kSoft) {
                    // soft arcs: cancel flow on the reverse arc first
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const bool go = rem > 0 && sl.r[k] > 0 && sl.d[k] + 1 == dv;
                        if (go) {
                            const long long a = min(rem, (long long)sl.r[k]);
                            const int back = (int)min(a, (long long)sl.back[k]);
                            const size_t w = base + (ptrdiff_t)(dq[k] + z);
                            if (back > 0) st.sf[(size_t)(k ^ 1) * Ntot + w] = sl.back[k] - back;
                            if (a > back) st.sf[(size_t)k * Ntot + v] = sl.own[k] + (int)(a - back);
                            const int o = atomicAdd(st.e + w, (int)a);
                            worst = max(worst, (long long)o + a);
                            rem -= a;
                            bytes += 12;
                        }
                        if (go) mark_mask(wout, q[k], 1ULL << (z / kWave / cpb));
                    }
                }
                int fwd_k = -1;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (fwd_k < 0 && rem > 0 && lt.d_fwd[k] + 1 == dv) fwd_k = k;
                const int zh = fwd_k >= 0 ? lat_head(z, bc.sh[fwd_k]) : 0;
                if (fwd_k >= 0) {
                    const size_t w = base + (ptrdiff_t)(dq[fwd_k] + zh);
                    st.fl[(size_t)fwd_k * Ntot + v] = add_flow(fown[fwd_k], rem, err);
                    a_fwd = (int)min(rem, (long long)INT_MAX);
                    o_fwd = atomicAdd(st.e + w, a_fwd);
                    rem = 0;
                    bytes += 8;
                }
                if (fwd_k >= 0) mark_mask(wout, q[fwd_k], 1ULL << (zh / kWave / cpb));
            }
            // net change of this node's excess word
            const long long delta = rem - taken;
            if (delta != 0) {
                if (rem > INT_MAX) err = 1;
                a_own = (int)delta;
                o_own = atomicAdd(st.e + v, a_own);
                bytes += 4;
            }
            if (rem > 0) own |= 1ULL << (c / cpb);
            worst = max(worst, a_col ? (long long)o_col + a_col : 0LL);
            worst = max(worst, a_fwd ? (long long)o_fwd + a_fwd : 0LL);
            worst = max(worst, a_own ? (long long)o_own + a_own : 0LL);
#pragma unroll
            for (int k = 0; k < 4; ++k) worst = max(worst, a_rev[k] ? (long long)o_rev[k] + a_rev[k] : 0LL);
        }
        // combine the lanes' own-column marks; the batch lane of this column
        // keeps them until the batch is done
        unsigned lo32 = (unsigned)own, hi32 = (unsigned)(own >> 32);
        for (int off = 32; off > 0; off >>= 1) {
            lo32 |= (unsigned)__shfl_xor((int)lo32, off, kWave);
            hi32 |= (unsigned)__shfl_xor((int)hi32, off, kWave);
        }
        if (lane == src) myown = ((unsigned long long)hi32 << 32) | lo32;
      }
      if (myown) mark_mask(wout, myp, myown);
    }
    if (g.count_work) count_bytes(g, 1, bytes);
    if (err || worst > INT_MAX) atomicOr(&s->err, kErrOverflow);
}

// Relabel phase of one sweep (flows fixed).  A wave takes a column of the
// push phase's output list: every node of its marked chunks with excess, a
// finite label and no admissible arc takes d(u) = min over residual arcs of
// d(w) + len(u, w) (kInf when that exceeds every possible distance).  The
// column's mask is rebuilt from the nodes that stay active, which are
// counted per volume, and the column goes on the next push phase's list.
// With use_gap (only in the relabel phase right after a gap search: the
// pushes in between change no label) a node labelled above its volume's gap
// was cut off from t when the gap was found and is frozen; a later phase
// must not use that gap, since a node relabelled across it since then may
// still reach t.
// Eight waves per SIMD (64 VGPRs, a few spilled): with the sweep grid of
// 8192 waves every wave is resident at once, and the phase is bound by
// memory latency, which more waves in flight hide.
template <bool kSoft>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_relabel(Geom g, State st, Work win, Work wout, int use_gap)
{
    const int lane = lane_id();
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int nwaves = gridDim.x * blockDim.x / kWave;
    const size_t Ntot = (size_t)g.Ntot;
    const int count = *win.count;
    VolSum<int> cnt(&g.is[0].active);
    VolSum<int> frozen(&g.is[0].gap_frozen);
    long long bytes = 0;
    Inst cur;              // volume of the previous column (reloaded on a change)
    int cur_ii = -1, gap = kInf;
    const int bs = min(kWave, max(1, (count + nwaves - 1) / nwaves));
    for (int b0 = wave * bs; b0 < count; b0 += nwaves * bs) {
      const int myp = (lane < bs && b0 + lane < count) ? win.list[b0 + lane] : -1;
      const unsigned long long mym = myp >= 0 ? win.mask[myp] : 0ULL;
      const int myii = myp >= 0 ? g.col_inst[myp] : 0;
      if (myp >= 0) win.mask[myp] = 0;
      unsigned long long mynm = 0;
      unsigned long long todo = __ballot(mym != 0);
      while (todo) {
        const int src = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        const int p = uniform(__shfl(myp, src, kWave));
        const unsigned long long m = (unsigned long long)shfl64((long long)mym, src);
        const int ii = uniform(__shfl(myii, src, kWave));
        if (ii != cur_ii) {
            cur = g.inst[ii];
            gap = use_gap ? g.is[ii].gap : kInf;
            cur_ii = ii;
        }
        const Col col = column_in(cur, ii, p);
        const int nch = col.I.nch, cpb = col.I.cpb;
        cnt.to(col.ii);
        frozen.to(col.ii);
        int q[4], dq[4];
        bool has[4];
        neighbours(col, p, q, dq, has);
        BandCol bc;
        band_col(g, p, q, col.I.K, col.I.delta, bc);
        const int K = bc.ext;   // node slots of the column
        const size_t base = col.base;
        unsigned long long nm = 0;
        for (int c = 0; c < nch; ++c) {
            if (!((m >> (c / cpb)) & 1ULL)) continue;
            const int z = c * kWave + lane;
            const bool in = z < K;
            const size_t v = base + z;
            const ChunkIn ci = load_chunk(st, v, z, K, lane);
            bytes += in ? 16 : 0;
            int dv = ci.d;
            bool act = in && ci.e > 0 && dv < kInf;
            if (act && dv > gap) {
                // cut off from t by a label gap: frozen for good
                dv = kInf;
                st.d[v] = kInf;
                act = false;
                ++frozen.acc;
            }
            if (!__ballot(act)) continue;
            Lateral lt;
            load_lateral(lt, st, base, dq, has, bc, z, Ntot, act);
            bytes += act ? 48 : 0;
            SoftLat sl;
            if constexpr (kSoft) {
                load_soft(sl, st, base, dq, has, z, Ntot, col.I.alpha, act);
                bytes += act && col.I.alpha > 0 ? 48 : 0;
            }
            if (act) {
                int b = ci.d_below;   // length-0 down arc
                if (ci.ts > 0) b = min(b, 1);
                if (ci.fd_above > 0) b = min(b, ci.d_above + 1);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    b = min(b, lt.d_fwd[k] + 1);
                    if (lt.f_rev[k] > 0) b = min(b, lt.d_rev[k] + 1);
                    if constexpr (kSoft) {
                        if (sl.r[k] > 0) b = min(b, sl.d[k] + 1);
                    }
                }
                if (b > dv) {
                    dv = b >= col.I.lab_cap ? kInf : b;
                    st.d[v] = dv;
                    bytes += 4;
                }
                act = dv < kInf;
            }
            if (__ballot(act)) nm |= 1ULL << (c / cpb);
            cnt.acc += act ? 1 : 0;
        }
        if (lane == src) mynm = nm;
      }
      if (mynm) wout.mask[myp] = mynm;
      wave_append(wout.list, wout.count, mynm != 0, myp);
    }
    if (g.count_work) count_bytes(g, 2, bytes);
    block_flush(cnt);
    block_flush(frozen);
}

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
// the thresholds of columns next to a change plus the nodes it labels.
//
// Per-column BFS record, double-buffered by level parity (global columns):
//   T[p]      threshold T_L(p) (the column's extent when no node of it is
//             labelled) in bits 0-29, in bit 30 whether the down arc into
//             (p, T_L(p)) carries flow (the one per-node fact the next level
//             needs at the threshold), and in bit 31 whether the record
//             changed when level L was produced (so one load gives all three);
//   LF[k][p]  lowest z' >= T_L(p) whose lateral arc in direction k carries
//             flow (K if none) -- the reverse-arc term seen by neighbour k;
// Volumes that do not take part in a search keep CH = 0 on all their
// columns, so every level skips them.

__device__ __forceinline__ int lat_head_of(int zp, int dl) { return zp == 0 ? 0 : zp - dl; }

constexpr int kChanged = (int)0x80000000u;   // change flag of a threshold word
constexpr int kFdAtT = 0x40000000;           // flow on the down arc into (p, T)
constexpr int kTMask = 0x3fffffff;           // the threshold bits

// Word w of bit mask m of column p.
// Where a level reads the bit masks: word w of mask m of global column p is
// bits[(m * nch + w) * P + p - off] (the global masks, off 0, or a volume's
// copy in LDS, off its first column).
struct MaskSrc {
    const unsigned long long *bits;
    int nch, P, off;
    __device__ unsigned long long word(int m, int w, int p) const
    {
        return bits[((size_t)m * nch + w) * P + (p - off)];
    }
};

__device__ __forceinline__ MaskSrc global_masks(const Geom &g) { return MaskSrc{g.bits, g.max_nch, g.Ptot, 0}; }

// Bits [lo, hi) of the heights 64w..64w+63 (lo < 64(w+1), hi > 64w).
__device__ __forceinline__ unsigned long long range_bits(int w, int lo, int hi)
{
    const int a = max(lo - kWave * w, 0), b = min(hi - kWave * w, kWave);
    const unsigned long long upto = b >= kWave ? ~0ULL : ((1ULL << b) - 1ULL);
    return upto & ~((1ULL << a) - 1ULL);
}

// Before level 1: clears the level flags and early-stop counters of the
// volumes that take part, and forgets their known gap.
__global__ void k_bfs_begin(Geom g)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < g.n && g.part[i]) {
        for (int l = 0; l < kLvlSlots; ++l) g.is[i].lvl_changed[l] = 0;
        g.is[i].bfs_active = 0;
        g.is[i].bfs_unsat[0] = g.is[i].bfs_unsat[1] = 0;
        g.is[i].gap = kInf;
    }
}

// Node words of one 64-height chunk that level 1 reads.
struct InitWords {
    int ts, e, d, fd, f[4];
};

__device__ __forceinline__ void load_init_words(const State &st, size_t Ntot, size_t v, bool in,
                                                InitWords &w)
{
    w.ts = 0;
    w.e = 0;
    w.d = kInf;
    w.fd = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) w.f[k] = 0;
    if (in) {
        w.ts = st.ts[v];
        w.e = st.e[v];
        w.d = st.d[v];
        w.fd = st.fd[v];
#pragma unroll
        for (int k = 0; k < 4; ++k) w.f[k] = st.fl[(size_t)k * Ntot + v];
    }
}

// chunks of a column whose words level 1 requests together
constexpr int kInitGroup = 2;

// Level 1, one wave per column.  Nodes that could not reach t before keep
// kInf: new residual arcs only ever join nodes that reach t, so a node cut
// off from t stays cut off.  Counts per volume the nodes with excess and a
// finite label, and those of them labelled 1, for the early stop, and
// writes the column's bit masks (flows and excess do not change during the
// search).  The words of kInitGroup chunks are loaded before any of them
// is used, so that a wave keeps that many chunks' loads in flight; at eight
// waves per SIMD.
template <bool kSoft>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_bfs_init(Geom g, State st, int *T, int *LF, int c0, int c1)
{
    const int lane = lane_id();
    const size_t Ntot = (size_t)g.Ntot;
    const int Ptot = g.Ptot;
    int lo, hi;
    wave_range(c0, c1, lo, hi);
    VolSum<int> act(&g.is[0].bfs_active);
    // short columns of up to 64 consecutive columns, appended to the list
    // with one counter atomic
    unsigned long long shortm = 0;
    int sbase = lo;
    auto flush_short = [&]() {
        const int cnt = __popcll(shortm);
        if (cnt) {
            int base = 0;
            if (lane == 0) base = atomicAdd(g.short_count, cnt);
            base = __shfl(base, 0, kWave);
            if ((shortm >> lane) & 1ULL)
                g.short_list[base + __popcll(shortm & ((1ULL << lane) - 1ULL))] = sbase + lane;
        }
        shortm = 0;
    };
    VolCache vc;
    bool vpart = false;
    for (int p = lo; p < hi; ++p) {
        if (p - sbase == kWave) {
            flush_short();
            sbase = p;
        }
        if (vc.at(g, p)) vpart = g.part[vc.ii] != 0;
        if (!vpart) {
            if (lane == 0) T[p] = 0;   // no change flag: every level skips it
            continue;
        }
        act.to(vc.ii);
        // slots used (Kc) and the volume's K, which also marks "no arc" in lf
        const int K = vc.I.K, nch = vc.I.nch, Kc = g.band ? g.bext[p] : K;
        const size_t base = vc.base(p);
        int t1 = Kc, la = Kc;
        unsigned long long fd1 = 0;   // flow on the down arc into (p, t1)
        int lf[4] = {K, K, K, K};
        for (int cg = 0; cg < nch; cg += kInitGroup) {
            InitWords w[kInitGroup];
#pragma unroll
            for (int j = 0; j < kInitGroup; ++j) {
                const int z = (cg + j) * kWave + lane;
                load_init_words(st, Ntot, base + z, z < Kc, w[j]);
            }
#pragma unroll
            for (int j = 0; j < kInitGroup; ++j) {
                const int c = cg + j;
                if (c >= nch) break;
                const int z = c * kWave + lane;
                const bool in = z < Kc;
                // the chunk's words of the bit masks, one mask per lane 0..5
                unsigned long long wm[kMasks];
#pragma unroll
                for (int k = 0; k < 4; ++k) wm[kMaskFl + k] = __ballot(in && w[j].f[k] > 0);
                wm[kMaskFd] = __ballot(in && w[j].fd > 0);
                unsigned long long mine = 0;
#pragma unroll
                for (int m = 0; m < kMasks; ++m)
                    if (lane == m) mine = wm[m];
                if (lane < kMasks) g.bits[((size_t)lane * g.max_nch + c) * Ptot + p] = mine;
                if (t1 == Kc) {
                    const unsigned long long sm = __ballot(in && w[j].ts > 0);
                    if (sm) {
                        t1 = c * kWave + __ffsll((long long)sm) - 1;
                        fd1 = (wm[kMaskFd] >> (t1 - c * kWave)) & 1ULL;
                    }
                }
                const bool lab = in && z >= t1;
                const int dv = w[j].d;
                // labels that keep their value (kInf stays kInf) are not rewritten
                const int dn = lab ? 1 : (dv >= kInf ? kInf : kUnl);
                if (in && dn != dv) st.d[base + z] = dn;
                const bool isact = in && w[j].e > 0 && dv < kInf;
                if (isact) ++act.acc;
                if (la == Kc) {
                    const unsigned long long am = __ballot(isact);
                    if (am) la = c * kWave + __ffsll((long long)am) - 1;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (lf[k] < K) continue;
                    const unsigned long long fm = __ballot(lab && w[j].f[k] > 0);
                    if (fm) lf[k] = c * kWave + __ffsll((long long)fm) - 1;
                }
            }
        }
        if constexpr (kSoft) {
            // residual soft arcs (p,z) -> (q_k,z), one mask per direction
            const int alpha = vc.I.alpha;
            if (alpha > 0) {
                const int pl = p - vc.I.col_base, x = pl / vc.I.ny, y = pl - x * vc.I.ny;
                for (int c = 0; c < nch; ++c) {
                    const int z = c * kWave + lane;
                    unsigned long long mine = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int q = nbr(vc.I.nx, vc.I.ny, x, y, p, k);
                        const bool on = q >= 0 && z >= 1 && z < K;
                        const size_t v = base + z;
                        const size_t w = base + (ptrdiff_t)(on ? (q - p) * K + z : 0);
                        const int r = on ? alpha - st.sf[(size_t)k * Ntot + v] + st.sf[(size_t)(k ^ 1) * Ntot + w] : 0;
                        const unsigned long long b = __ballot(r > 0);
                        if (lane == k) mine = b;
                    }
                    if (lane < 4) g.sbits[((size_t)lane * g.max_nch + c) * Ptot + p] = mine;
                }
            }
        }
        // a column whose lowest active node lies below the level-1 suffix
        // keeps the search from stopping early until a level reaches it
        if (la < t1) shortm |= 1ULL << (p - sbase);
        if (lane == 0) {
            T[p] = t1 | (fd1 ? kFdAtT : 0) | kChanged;
            g.low_act[p] = la;
#pragma unroll
            for (int k = 0; k < 4; ++k) LF[(size_t)k * Ptot + p] = lf[k];
        }
    }
    flush_short();
    block_flush(act);
}

// Early-stop count at a host poll: the columns of the short list whose
// threshold has not yet reached their lowest active node, per volume, into
// bfs_unsat[slot] (cleared by the previous call, which clears the other slot
// for the next one).
__global__ __launch_bounds__(256) void k_bfs_count(Geom g, const int *__restrict__ T, int slot)
{
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < g.n; i += blockDim.x) g.is[i].bfs_unsat[slot ^ 1] = 0;
    const int n = *g.short_count;
    VolSum<int> cnt(&g.is[0].bfs_unsat[slot]);
    const int stride = gridDim.x * blockDim.x;
    for (int i0 = blockIdx.x * blockDim.x; i0 < n; i0 += stride) {
        const int i = i0 + threadIdx.x;
        int ii = -1;
        bool unsat = false;
        if (i < n) {
            const int p = g.short_list[i];
            ii = g.col_inst[p];
            unsat = (T[p] & kTMask) > g.low_act[p];
        }
        // list entries come in wave-sized runs of one volume's columns
        const int first = uniform(ii);
        if (__ballot(ii >= 0 && ii != first) == 0) {
            if (first >= 0) {
                cnt.to(first);
                cnt.acc += unsat ? 1 : 0;
            }
        } else {
            wave_add_keyed(&g.is[0].bfs_unsat[slot], ii, 1, unsat);
        }
    }
    block_flush(cnt);
}

// One level for one column: the new threshold cand from the column's
// threshold T and its neighbours' thresholds tq[k] (-1: no neighbour in
// direction k) and lowest flow-carrying arcs into the column lq[k] (K: none;
// arc heights and the column's extent from bc); lf[]
// (the column's lowest flow-carrying lateral arc per direction at or above
// its threshold) is lowered over the newly reached heights [cand, T) from
// the bit masks.  fdT: the down arc into (p, T) carries flow; fd_new gets
// the same fact for the new threshold.  Returns the mask words read.
template <bool kSoft>
__device__ __forceinline__ int level_update(const Geom &g, const MaskSrc &ms, int p, int K, const BandCol &bc, int alpha,
                                           int T, bool fdT, const int tq[4], const int lq[4], int lf[4],
                                           int &cand, bool &fd_new)
{
    cand = T;
    int words = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (tq[k] < 0) continue;
        if (tq[k] == 0) cand = 0;
        else if (tq[k] + bc.sh[k] < bc.ext) cand = min(cand, tq[k] + bc.sh[k]);
        if (lq[k] < K) cand = min(cand, lat_head_of(lq[k], bc.shr[k]));
    }
    if constexpr (kSoft) {
        // soft arcs (p,z) -> (q,z): the lowest z >= T(q) (z >= 1) whose arc
        // is residual, when below the candidate so far
        if (alpha > 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int lo = max(tq[k], 1);
                if (tq[k] < 0 || lo >= cand) continue;
                for (int w = lo >> 6; w <= (cand - 1) >> 6; ++w) {
                    const unsigned long long b =
                        g.sbits[((size_t)k * g.max_nch + w) * g.Ptot + p] & range_bits(w, lo, cand);
                    ++words;
                    if (b) {
                        cand = w * kWave + __ffsll((long long)b) - 1;
                        break;
                    }
                }
            }
        }
    }
    if (fdT && T >= 1 && T < bc.ext) cand = min(cand, T - 1);
    fd_new = fdT;
    if (cand < T) {
        // the word the scan below starts in holds the new threshold's bit
        ++words;
        fd_new = (ms.word(kMaskFd, cand >> 6, p) >> (cand & 63)) & 1ULL;
    }
    // an lf below T was found in an earlier word
    for (int w = cand >> 6; cand < T && w <= (T - 1) >> 6; ++w) {
        if (lf[0] < T && lf[1] < T && lf[2] < T && lf[3] < T) break;
        const unsigned long long r = range_bits(w, cand, T);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (lf[k] < T) continue;
            const unsigned long long fm = ms.word(kMaskFl + k, w, p) & r;
            if (fm) lf[k] = w * kWave + __ffsll((long long)fm) - 1;
        }
        words += 4;
    }
    return words;
}

// Writes d = lab on the heights [lo, hi) of every lane's column (node (p, 0)
// at base): ranges of 64 or more heights one column at a time by the whole
// wave (coalesced stores), the others as one flattened list of (column,
// height) items, 64 stores per step, so a wave's time follows the number of
// nodes it labels rather than its longest range.  Called by all lanes;
// returns the lane's bytes written.
__device__ __forceinline__ long long label_ranges(int *d, int lab, int lo, int hi, long long base)
{
    const int lane = lane_id();
    long long bytes = 0;
    const bool whole = hi - lo >= kWave;
    for (unsigned long long lm = __ballot(whole); lm; lm &= lm - 1) {
        const int src = __ffsll((long long)lm) - 1;
        const int a = __shfl(lo, src, kWave), b = __shfl(hi, src, kWave);
        const long long pbase = shfl64(base, src);
        for (int z = a + lane; z < b; z += kWave) d[(size_t)pbase + z] = lab;
        bytes += lane == 0 ? 4LL * (b - a) : 0;
    }
    const int len = !whole && hi > lo ? hi - lo : 0;
    int incl = len;
    for (int off = 1; off < kWave; off <<= 1) {
        const int t = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += t;
    }
    const int excl = incl - len;
    const int total = __shfl(incl, kWave - 1, kWave);
    for (int i0 = 0; i0 < total; i0 += kWave) {
        const int item = i0 + lane;
        // owner: the last lane whose exclusive prefix is <= item
        int o = 0;
        for (int step = 32; step > 0; step >>= 1) {
            const int c = o + step;
            const int ex = __shfl(excl, c < kWave ? c : kWave - 1, kWave);
            if (c < kWave && ex <= item) o = c;
        }
        const int top = __shfl(hi, o, kWave);
        const long long pbase = shfl64(base, o);
        const int z = top - 1 - (item - __shfl(excl, o, kWave));
        if (item < total) {
            d[(size_t)pbase + z] = lab;
            bytes += 4;
        }
    }
    return bytes;
}

// Sets the level flag `slot` of the volumes of the lanes with `flag`.
__device__ __forceinline__ void set_level_flag(const Geom &g, int ii, bool flag, int slot)
{
    const int lane = lane_id();
    bool pending = flag;
    for (;;) {
        const unsigned long long b = __ballot(pending);
        if (!b) break;
        const int leader = __ffsll((long long)b) - 1;
        const int k = __shfl(ii, leader, kWave);
        if (lane == leader) g.is[k].lvl_changed[slot] = 1;
        if (pending && ii == k) pending = false;
    }
}

// One column's step of level L -> L+1: reads the threshold words of column
// p and of its neighbours from Tin (P columns per array), sets T (the old
// threshold), cand (the new one when the column moved), `self` (the column
// changed at level L-1) and tword (the column's threshold word for Tout),
// and returns whether the threshold moved.  The change flags in the
// threshold words give the frontier: with no change at level L-1 around p
// none of p's inputs moved, and both record buffers already hold p's
// record.  The lowest-flow records lf[] of the column and lq[] of its
// neighbours (LFin) are loaded in the same round as the threshold words, so
// that a column next to a change waits for one round of loads before its
// mask scan; `bytes` counts the column's algorithmic bytes: its threshold
// word read and rewritten, and when near a change its 16-byte record and the
// mask words scanned (a quiet column does not need its record; neighbours'
// words are their own records, counted with their own column).
template <bool kSoft>
__device__ __forceinline__ bool column_step(const Geom &g, const MaskSrc &ms, const Col &col, int p, const int *Tin,
                                            const int *LFin, int P, int &T, int &cand, int lf[4],
                                            bool &self, int &tword, long long &bytes)
{
    const int K = col.I.K;
    int q[4], tq[4], lq[4];
    const int tw = Tin[p];
    bool near = tw < 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        q[k] = nbr(col.I.nx, col.I.ny, col.x, col.y, p, k);
        const int w = q[k] >= 0 ? Tin[q[k]] : -1;
        lq[k] = q[k] >= 0 ? LFin[(size_t)(k ^ 1) * P + q[k]] : K;
        lf[k] = LFin[(size_t)k * P + p];
        near = near || (q[k] >= 0 && w < 0);
        tq[k] = q[k] >= 0 ? (w & kTMask) : -1;
    }
    self = tw < 0;
    T = tw & kTMask;
    tword = tw & ~kChanged;
    bytes = 8;
    cand = T;
    if (!near) return false;
    BandCol bc;
    band_col(g, p, q, K, col.I.delta, bc);
    bool fd_new = false;
    bytes += 16 + 8 * level_update<kSoft>(g, ms, p, K, bc, col.I.alpha, T, (tw & kFdAtT) != 0, tq, lq, lf,
                                          cand, fd_new);
    if (cand < T) tword = cand | (fd_new ? kFdAtT : 0) | kChanged;
    return cand < T;
}

// Level L -> L+1, one lane per column of the ranges R.  The threshold
// arithmetic reads the records of the column and its neighbours; the lowest
// flow-carrying lateral arcs among the newly reached heights [cand, T) come
// from the column's bit masks, so no per-node word is read.
template <bool kSoft>
__global__ __launch_bounds__(1024) void k_bfs_level(Geom g, int *__restrict__ d, int L,
                                                   const int *__restrict__ Tin,
                                                   const int *__restrict__ LFin, int *__restrict__ Tout,
                                                   int *__restrict__ LFout, LevelRanges R, Inst I0, int single)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    // the flags of the next level are cleared here; stream order puts this
    // before every write of level L+1
    if (t < g.n) g.is[t].lvl_changed[(L + 1) % kLvlSlots] = 0;
    const int P = g.Ptot;
    int r = 0;
    for (int j = 1; j < R.n; ++j) r += t >= R.pre[j];
    const bool valid = t < R.pre[R.n];
    const int p = valid ? R.lo[r] + (t - R.pre[r]) : 0;
    bool self = false, need = false;
    int T = 0, cand = 0, ii = 0, tword = 0;
    long long base = 0;
    int lf[4] = {0, 0, 0, 0};
    long long bytes = 0;
    if (valid) {
        // a single volume's geometry comes with the launch (no table loads
        // ahead of the column's own)
        const Col col = single ? column_in(I0, 0, p) : column(g, p);
        ii = col.ii;
        base = (long long)col.base;
        need = column_step<kSoft>(g, global_masks(g), col, p, Tin, LFin, P, T, cand, lf, self, tword, bytes);
    }
    if (valid) {
        Tout[p] = tword;
        if (need || self) {
#pragma unroll
            for (int k = 0; k < 4; ++k) LFout[(size_t)k * P + p] = lf[k];
            bytes += 16;
        }
    }
    // level L labelled something in the volumes of the lanes with `need`:
    // for a single volume one store per block (thousands of waves storing to
    // one word serialise in the memory system), else per volume and wave
    if (single) {
        if (__syncthreads_or(need) && threadIdx.x == 0) g.is[0].lvl_changed[L % kLvlSlots] = 1;
    } else {
        set_level_flag(g, ii, need, L % kLvlSlots);
    }
    bytes += label_ranges(d, L + 1, need ? cand : 0, need ? T : 0, base);
    if (g.count_work) count_bytes(g, 0, bytes);
}

// A whole search of small volumes, one block per volume (block i takes
// volume i when it takes part; every volume of at most kBlockSearchCols
// columns): the records live in LDS, double-buffered as in global memory,
// and block barriers separate the levels instead of launches and host
// polls.  Level 1 comes from k_bfs_init (records T1,
// LF1).  The search ends when a level labels nothing (unreached nodes get
// kInf) or, with early_stop, once no column's threshold lies above its
// lowest active node (unreached nodes get the first level not run).  The
// block then writes those fill labels itself and adds its level count to
// s->block_levels.  Every column step is the one of k_bfs_level, so the
// labels are the same.
constexpr int kBlockSearchCols = 2048;

constexpr int kBlockSearchSlots = 2;   // columns per thread
static_assert(kBlockSearchCols <= kBlockSearchSlots * 1024, "a one-block search takes 2 columns a thread");

template <bool kSoft, bool kStage>
__global__ __launch_bounds__(1024) void k_bfs_block(Geom g, int *__restrict__ d, const int *__restrict__ T1,
                                                   const int *__restrict__ LF1, int early_stop,
                                                   int max_level, int quorum, Scratch *s)
{
    extern __shared__ unsigned long long sml[];
    int *const sm = reinterpret_cast<int *>(sml);
    const int ii = blockIdx.x;
    if (!g.part[ii]) return;
    const Inst I = g.inst[ii];
    // local columns p of the volume are global columns c0 + p
    const int P = I.P, c0 = I.col_base, Ptot = g.Ptot;
    // records of level L in buffer L & 1: thresholds at sm + (L & 1) P,
    // lowest-flow records at sm + 2P + 4P (L & 1); the buffers are picked by
    // arithmetic on the LDS base, so the compiler keeps LDS accesses
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        sm[P + i] = T1[c0 + i];
#pragma unroll
        for (int k = 0; k < 4; ++k) sm[6 * P + k * P + i] = LF1[(size_t)k * Ptot + c0 + i];
    }
    // kStage: the level-1 bit masks are copied into LDS after the records
    // (40 bytes per column and chunk), so that a level reads no global
    // memory and only writes its labels there
    unsigned long long *const sb = sml + 5 * (size_t)P;
    if constexpr (kStage) {
        const int per = I.nch * P;
        for (int i = threadIdx.x; i < kMasks * per; i += blockDim.x) {
            const int m = i / per, r = i - m * per, w = r / P, p = r - w * P;
            sb[i] = g.bits[((size_t)m * g.max_nch + w) * Ptot + c0 + p];
        }
    }
    const MaskSrc ms = kStage ? MaskSrc{sb, I.nch, P, c0} : global_masks(g);
    // each thread's lowest active heights, for the early stop
    int la[kBlockSearchSlots];
#pragma unroll
    for (int j = 0; j < kBlockSearchSlots; ++j) {
        const int p = j * (int)blockDim.x + (int)threadIdx.x;
        la[j] = p < P ? g.low_act[c0 + p] : 0;
    }
    __syncthreads();
    const int slots = (P + (int)blockDim.x - 1) / (int)blockDim.x;
    // per level L, red[L % 3] gathers bit 0: a column moved, bit 1: a column
    // is still short of its lowest active node, bit 2: `quorum` volumes'
    // searches have ended (s->block_done, read once per level by thread 0),
    // which ends this one too
    __shared__ int red[3];
    if (threadIdx.x < 3) red[threadIdx.x] = 0;
    __syncthreads();
    // the geometry of the thread's columns, fixed for the whole search:
    // node (p, 0), the neighbours (local columns, -1: none) and the band
    // shifts
    long long cbase[kBlockSearchSlots];
    int cq[kBlockSearchSlots][4];
    BandCol cbc[kBlockSearchSlots];
#pragma unroll
    for (int j = 0; j < kBlockSearchSlots; ++j) {
        // a slot past the last column takes column 0's geometry, unused
        const int pj = j * (int)blockDim.x + (int)threadIdx.x;
        const int p = c0 + (pj < P ? pj : 0);
        const Col col = column_in(I, ii, p);
        cbase[j] = (long long)col.base;
        int qg[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            qg[k] = nbr(I.nx, I.ny, col.x, col.y, p, k);
            cq[j][k] = qg[k] >= 0 ? qg[k] - c0 : -1;
        }
        band_col(g, p, qg, I.K, I.delta, cbc[j]);
    }
    long long bytes = 0;
    int L = 1, cur = 1, run = 0;
    bool complete = false;
    for (;; ++L, cur ^= 1) {
        if (L > max_level) {
            if (threadIdx.x == 0) atomicOr(&s->err, kErrSearch);
            break;
        }
        const int *Tin = sm + cur * P, *LFin = sm + 2 * P + 4 * P * cur;
        int *Tout = sm + (cur ^ 1) * P, *LFout = sm + 2 * P + 4 * P * (cur ^ 1);
        bool moved = false, shortc = false;
#pragma unroll
        for (int j = 0; j < kBlockSearchSlots; ++j) {
            if (j >= slots) break;
            const int p = j * (int)blockDim.x + (int)threadIdx.x;
            const bool valid = p < P;
            bool need = false;
            int T = 0, cand = 0, tout = 0;
            long long b = 0;
            if (valid) {
                // the step of column_step, on the hoisted geometry
                int tq[4], lq[4], lf[4];
                const int tw = Tin[p];
                bool near = tw < 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int q = cq[j][k];
                    const int w = q >= 0 ? Tin[q] : -1;
                    lq[k] = q >= 0 ? LFin[(k ^ 1) * P + q] : I.K;
                    lf[k] = LFin[k * P + p];
                    near = near || (q >= 0 && w < 0);
                    tq[k] = q >= 0 ? (w & kTMask) : -1;
                }
                const bool self = tw < 0;
                T = tw & kTMask;
                cand = T;
                int tword = tw & ~kChanged;
                b = 8;
                if (near) {
                    bool fd_new = false;
                    b += 16 + 8 * level_update<kSoft>(g, ms, c0 + p, I.K, cbc[j], I.alpha, T, (tw & kFdAtT) != 0,
                                                      tq, lq, lf, cand, fd_new);
                    need = cand < T;
                    if (need) tword = cand | (fd_new ? kFdAtT : 0) | kChanged;
                }
                Tout[p] = tword;
                tout = tword;
                if (need || self)
#pragma unroll
                    for (int k = 0; k < 4; ++k) LFout[k * P + p] = lf[k];
            }
            // labels: short ranges (at most 8 heights in every lane) one
            // store per height, longer ones spread over the wave
            const int len = need ? T - cand : 0;
            if (__ballot(len > 8)) {
                bytes += b + label_ranges(d, L + 1, need ? cand : 0, need ? T : 0, cbase[j]);
            } else {
                for (int i = 0; __ballot(i < len); ++i)
                    if (i < len) d[(size_t)cbase[j] + cand + i] = L + 1;
                bytes += b + 4LL * len;
            }
            moved = moved || need;
            shortc = shortc || (valid && (tout & kTMask) > la[j]);
        }
        ++run;
        // early stop: a column of this thread still short of its lowest
        // active node (shortc, from the records just written)
        const bool short_col = early_stop && shortc;
        // each wave ORs its two flags into red[L % 3], and one barrier both
        // publishes them and puts every record of level L+1 before any read
        // of the next level.  red[(L + 1) % 3] is cleared for the next level
        // before this barrier: it was last read between the barriers of
        // levels L - 2 and L - 1
        const int wf = (__ballot(moved) ? 1 : 0) | (__ballot(short_col) ? 2 : 0);
        if (lane_id() == 0 && wf) atomicOr(&red[L % 3], wf);
        if (threadIdx.x == 0) {
            red[(L + 1) % 3] = 0;
            if (__hip_atomic_load(&s->block_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= quorum)
                atomicOr(&red[L % 3], 4);
        }
        __syncthreads();
        const int f = red[L % 3];
        const bool any_m = f & 1, any_s = f & 2;
        if (!any_m) {
            complete = true;   // level L labelled nothing
            break;
        }
        if ((early_stop && !any_s) || (f & 4)) {
            ++L;   // levels <= L are done: unreached nodes lie beyond L + 1
            break;
        }
    }
    if (threadIdx.x == 0) atomicAdd(&s->block_done, 1);
    // fix-up: L is the first level whose labels were not all written
    const int fill = complete ? kInf : L + 1;
    for (long long v = threadIdx.x; v < (long long)I.N; v += blockDim.x)
        if (d[I.node_base + v] == kUnl) d[I.node_base + v] = fill;
    if (threadIdx.x == 0) atomicAdd(&s->block_levels, run);
    if (g.count_work) count_bytes(g, 0, bytes);
}

// End of a global relabel: nodes the search did not reach get the volume's
// fill label (kInf when its search ran to completion, else the first level
// it did not finish, which is a valid lower bound of their distance).
__global__ __launch_bounds__(256) void k_bfs_fixup(Geom g, int *d, int c0, int c1)
{
    constexpr int kGroup = 4;   // chunks whose labels are loaded together
    const int lane = lane_id();
    int lo, hi;
    wave_range(c0, c1, lo, hi);
    VolCache vc;
    int fill = -1;
    for (int p = lo; p < hi; ++p) {
        if (vc.at(g, p)) fill = g.fill[vc.ii];
        if (fill < 0) continue;
        const int K = vc.I.K;
        int *dc = d + vc.base(p);
        for (int z0 = 0; z0 < K; z0 += kGroup * kWave) {
            int dv[kGroup];
#pragma unroll
            for (int j = 0; j < kGroup; ++j) {
                const int z = z0 + j * kWave + lane;
                dv[j] = z < K ? dc[z] : 0;
            }
#pragma unroll
            for (int j = 0; j < kGroup; ++j) {
                const int z = z0 + j * kWave + lane;
                if (z < K && dv[j] == kUnl) dc[z] = fill;
            }
        }
    }
}

// ---- minimum cut ---------------------------------------------------------------
//
// S_min is the set reached in the residual graph from the nodes that keep
// excess (the source arcs are saturated).  Down arcs are always residual,
// so S_min meets every column in a prefix {0..h(p)}; the passes below raise
// h to the fixed point of the residual arcs.

// h(p) = highest node of the column with excess (-1 if none); one wave per column.
__global__ __launch_bounds__(256) void k_mincut_init(Geom g, State st, int *H)
{
    const int lane = lane_id();
    int lo, hi;
    wave_columns(g, lo, hi);
    for (int p = lo; p < hi; ++p) {
        const Col col = column_uniform(g, p);
        int h = -1;
        for (int c = col.I.nch - 1; c >= 0 && h < 0; --c) {
            const int z = c * kWave + lane;
            const bool hit = z < col.I.K && st.e[col.base + z] > 0;
            const unsigned long long b = __ballot(hit);
            if (b) h = c * kWave + 63 - __clzll(b);
        }
        if (lane == 0) H[p] = h;
    }
}

// h_max(p) = the highest node of the column that cannot reach t, after a
// complete search has left exactly those nodes at kInf (a prefix of the
// column): one below the lowest node with a finite label, or the column's
// top if there is none.  Heights of the volume with a band.  One wave per
// column.
__global__ __launch_bounds__(256) void k_hmax(Geom g, State st, int *Hmax)
{
    const int lane = lane_id();
    int lo, hi;
    wave_columns(g, lo, hi);
    for (int p = lo; p < hi; ++p) {
        const Col col = column_uniform(g, p);
        const int ext = g.band ? g.bext[p] : col.I.K;
        int hm = ext - 1;
        for (int c = 0; c < col.I.nch; ++c) {
            const int z = c * kWave + lane;
            const unsigned long long b = __ballot(z < ext && st.d[col.base + z] < kInf);
            if (b) {
                hm = c * kWave + __ffsll((long long)b) - 2;
                break;
            }
        }
        if (lane == 0) Hmax[p] = hm + (g.band ? g.blo[p] : 0);
    }
}

template <bool kSoft>
__global__ __launch_bounds__(256) void k_mincut_pass(Geom g, State st, int *H, Scratch *s)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= g.Ptot) return;
    const Col col = column(g, p);
    const int K = col.I.K;
    const size_t Ntot = (size_t)g.Ntot;
    const size_t base = col.base;
    const int h0 = H[p];
    int h = h0;
    int qn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) qn[k] = nbr(col.I.nx, col.I.ny, col.x, col.y, p, k);
    BandCol bc;
    band_col(g, p, qn, K, col.I.delta, bc);
    for (int k = 0; k < 4; ++k) {
        const int qq = qn[k];
        if (qq < 0) continue;
        const int hq = H[qq];
        if (hq < 0) continue;
        // forward lateral arcs of q's reached prefix land at heights <= hq - shr (or 0)
        h = max(h, hq > bc.shr[k] ? hq - bc.shr[k] : 0);
        // reverse residual of p's own lateral arcs into q's reached prefix
        const int top = min(bc.ext - 1, hq + bc.sh[k]);
        for (int z = top; z > h; --z) {
            if (lat_arc(z, bc.sh[k]) && st.fl[(size_t)k * Ntot + base + z] > 0) {
                h = z;
                break;
            }
        }
        if constexpr (kSoft) {
            // residual soft arcs (q,z) -> (p,z) out of q's reached prefix:
            // alpha - flow(q -> p) + flow(p -> q) > 0
            const int alpha = col.I.alpha;
            if (alpha > 0) {
                const size_t qbase = base + (ptrdiff_t)(qq - p) * K;
                for (int z = min(hq, K - 1); z > h && z >= 1; --z) {
                    if (alpha - st.sf[(size_t)(k ^ 1) * Ntot + qbase + z] + st.sf[(size_t)k * Ntot + base + z] > 0) {
                        h = z;
                        break;
                    }
                }
            }
        }
    }
    // reverse residual of down arcs with flow: (p,h) -> (p,h+1)
    while (h >= 0 && h + 1 < bc.ext && st.fd[base + h + 1] > 0) ++h;
    if (h != h0) {
        H[p] = h;
        s->changed = 1;
    }
}

// Flow value F = sum_v (w+(v) - ts(v)) per volume: the build accumulated
// sum w+; here the residual sink capacities are subtracted and
// E = sum_p c(p, h(p)) is added (with soft smoothness also alpha times
// |h(p) - h(q)| for the +x and +y neighbour of every column), one wave per
// column.
template <bool kSoft>
__global__ __launch_bounds__(256) void k_finish(const int *__restrict__ cost, Geom g, State st,
                                                int *H)
{
    const int lane = lane_id();
    int lo, hi;
    wave_columns(g, lo, hi);
    VolSum<long long> flow(&g.is[0].flow), energy(&g.is[0].energy);
    for (int p = lo; p < hi; ++p) {
        const Col col = column_uniform(g, p);
        flow.to(col.ii);
        energy.to(col.ii);
        for (int c = 0; c < col.I.nch; ++c) {
            const int z = c * kWave + lane;
            if (z < col.I.K) flow.acc -= st.ts[col.base + z];
        }
        if (lane == 0) {
            const int h = H[p];
            const int cs = g.band ? g.bcs[p] : 0;   // cost index of the column's slot 0
            if (h >= 0) energy.acc += cost[(size_t)col.I.cost_base + (size_t)col.pl * col.I.K + cs + h];
            // a band column's surface is reported as a height of the volume
            // (no later pass reads H; soft smoothness never runs with a band)
            if (g.band && h >= 0) H[p] = h + g.blo[p];
            if constexpr (kSoft) {
                if (col.I.alpha > 0)
                    for (int k = 0; k < 4; k += 2) {   // +x, +y
                        const int q = nbr(col.I.nx, col.I.ny, col.x, col.y, p, k);
                        if (q >= 0) energy.acc += (long long)col.I.alpha * abs(h - H[q]);
                    }
            }
        }
    }
    block_flush(flow);
    block_flush(energy);
}

// ---- launchers --------------------------------------------------------------

static inline unsigned blocks_for(long long n)
{
    const long long b = (n + 255) / 256;
    return (unsigned)(b > 0 ? b : 1);
}

// Grid of the wave-per-column kernels: enough waves to fill the chip, each
// working through its share of the columns.
static inline unsigned wave_blocks(const Geom &g)
{
    long long want = (g.Ptot + 3) / 4;     // 4 waves per 256-thread block
    return (unsigned)(want < 2048 ? (want > 0 ? want : 1) : 2048);
}

// Grid of the push and relabel phases: sweep_waves waves (at most one per
// column), 4 per block.
static inline unsigned sweep_blocks(const Geom &g)
{
    long long want = (g.Ptot + 3) / 4, cap = g.sweep_waves / 4;
    if (want > cap) want = cap;
    return (unsigned)(want > 0 ? want : 1);
}

void launch_init_scratch(const Geom &g, Scratch *s, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_scratch, dim3(blocks_for(g.n)), dim3(256), 0, st, g, s);
}

void launch_set_int(int *p, int v, hipStream_t st) { hipLaunchKernelGGL(k_set_int, 1, 1, 0, st, p, v); }

void launch_fill(int *a, long long n, int v, hipStream_t st)
{
    unsigned b = blocks_for(n);
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_fill, dim3(b), dim3(256), 0, st, a, n, v);
}

void launch_work_init(const Geom &g, const Work &a, const Work &b, hipStream_t st)
{
    hipLaunchKernelGGL(k_work_init, dim3(blocks_for(g.Ptot)), dim3(256), 0, st, g, a, b);
}

void launch_build(const int *cost, const Geom &g, const State &sv, Scratch *s, hipStream_t st)
{
    hipLaunchKernelGGL(k_bottom_max, dim3(blocks_for(g.Ptot)), dim3(256), 0, st, cost, g);
    hipLaunchKernelGGL(k_build, dim3(wave_blocks(g)), dim3(256), 0, st, cost, g, sv, s);
}

void launch_bfs_begin(const Geom &g, hipStream_t st)
{
    hipLaunchKernelGGL(k_bfs_begin, dim3(blocks_for(g.n)), dim3(256), 0, st, g);
}

// Grid of the wave-per-column kernels over the columns [c0, c1).
static inline unsigned range_wave_blocks(int c0, int c1, unsigned cap = 2048)
{
    long long want = ((long long)c1 - c0 + 3) / 4;
    if (want > (long long)cap) want = cap;
    return (unsigned)(want > 0 ? want : 1);
}

// Blocks of `block` threads of kernel f that the chip holds at once (2048
// if the runtime cannot tell).  A wave-per-column kernel whose waves each
// take a fixed share of the columns runs in one round on such a grid, with
// no second round of a few waves at the end.
static unsigned resident_blocks(const void *f, int block)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, block, 0) != hipSuccess || per < 1 ||
        cus < 1)
        return 2048;
    return (unsigned)per * (unsigned)cus;
}

void launch_bfs_init(const Geom &g, const State &sv, int *T, int *LF, int c0, int c1, hipStream_t st)
{
    if (g.soft) {
        static const unsigned cap = resident_blocks(reinterpret_cast<const void *>(k_bfs_init<true>), 256);
        hipLaunchKernelGGL(k_bfs_init<true>, dim3(range_wave_blocks(c0, c1, cap)), dim3(256), 0, st, g,
                           sv, T, LF, c0, c1);
    } else {
        static const unsigned cap = resident_blocks(reinterpret_cast<const void *>(k_bfs_init<false>), 256);
        hipLaunchKernelGGL(k_bfs_init<false>, dim3(range_wave_blocks(c0, c1, cap)), dim3(256), 0, st, g,
                           sv, T, LF, c0, c1);
    }
}

void launch_bfs_count(const Geom &g, const int *T, int slot, hipStream_t st)
{
    hipLaunchKernelGGL(k_bfs_count, dim3(256), dim3(256), 0, st, g, T, slot);
}

void launch_bfs_level(const Geom &g, const State &sv, int L, const int *Tin, const int *LFin,
                      int *Tout, int *LFout, const LevelRanges &R, const Inst *single, hipStream_t st)
{
    const long long cols = R.pre[R.n];
    const long long n = cols > g.n ? cols : g.n;
    const int b = g.level_block;
    const Inst I0 = single ? *single : Inst{};
    const int one = single ? 1 : 0;
    if (g.soft)
        hipLaunchKernelGGL(k_bfs_level<true>, dim3((unsigned)((n + b - 1) / b)), dim3(b), 0, st, g, sv.d,
                           L, Tin, LFin, Tout, LFout, R, I0, one);
    else
        hipLaunchKernelGGL(k_bfs_level<false>, dim3((unsigned)((n + b - 1) / b)), dim3(b), 0, st, g, sv.d,
                           L, Tin, LFin, Tout, LFout, R, I0, one);
}

// LDS of a one-block search (gfx950: 160 KB per workgroup).
constexpr size_t kBlockSearchLds = 160 * 1024;

// Chunks a one-block search takes (its masks then stay in global memory;
// measured: 32x48x500 with 12288 chunks 0.51 s against 0.70 s for launched
// levels).  Beyond 2048 columns a thread walks more than two columns per
// level and the launched levels win (measured: even at 3072 columns, 10%
// slower at 4032).
constexpr long long kBlockSearchChunks = 16384;

bool bfs_block_fits(const Geom &g)
{
    return g.max_cols <= kBlockSearchCols && g.max_chunks <= kBlockSearchChunks;
}

void launch_bfs_block(const Geom &g, const State &sv, const int *T1, const int *LF1, int early_stop,
                      int max_level, int quorum, Scratch *s, hipStream_t st)
{
    // records, and the masks when they fit beside them
    // LDS for the largest volume; one block per volume
    const size_t rec = sizeof(int) * 10 * (size_t)g.max_cols;
    const size_t masks = sizeof(unsigned long long) * kMasks * (size_t)g.max_chunks;
    // (1 KB of the 160 KB stays free for the kernel's static LDS)
    const int stage = rec + masks + 1024 <= kBlockSearchLds ? 1 : 0;
    const size_t lds = rec + (stage ? masks : 0);
    // gfx950 gives a workgroup up to 160 KB of LDS; the limit is raised once
    // per kernel (a runtime that refuses reports it at the launch)
    static const bool raised = [] {
        for (const void *f : {reinterpret_cast<const void *>(k_bfs_block<true, true>),
                              reinterpret_cast<const void *>(k_bfs_block<false, true>)})
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBlockSearchLds) !=
                hipSuccess)
                (void)hipGetLastError();
        return true;
    }();
    (void)raised;
    if (stage) {
        if (g.soft)
            hipLaunchKernelGGL((k_bfs_block<true, true>), dim3(g.n), dim3(1024), lds, st, g, sv.d, T1, LF1,
                               early_stop, max_level, quorum, s);
        else
            hipLaunchKernelGGL((k_bfs_block<false, true>), dim3(g.n), dim3(1024), lds, st, g, sv.d, T1, LF1,
                               early_stop, max_level, quorum, s);
        return;
    }
    if (g.soft)
        hipLaunchKernelGGL((k_bfs_block<true, false>), dim3(g.n), dim3(1024), rec, st, g, sv.d, T1, LF1, early_stop,
                           max_level, quorum, s);
    else
        hipLaunchKernelGGL((k_bfs_block<false, false>), dim3(g.n), dim3(1024), rec, st, g, sv.d, T1, LF1,
                           early_stop, max_level, quorum, s);
}

void launch_bfs_fixup(const Geom &g, const State &sv, int c0, int c1, hipStream_t st)
{
    static const unsigned cap = resident_blocks(reinterpret_cast<const void *>(k_bfs_fixup), 256);
    hipLaunchKernelGGL(k_bfs_fixup, dim3(range_wave_blocks(c0, c1, cap)), dim3(256), 0, st, g, sv.d,
                       c0, c1);
}

void launch_gap_find(const Geom &g, const State &sv, long long max_inst_nodes, hipStream_t st)
{
    launch_fill(g.hist, (long long)g.n * g.hist_len, 0, st);
    unsigned bx = blocks_for(max_inst_nodes);
    if (bx > 512) bx = 512;
    hipLaunchKernelGGL(k_hist_build, dim3(bx, g.n), dim3(256), sizeof(int) * g.hist_len, st, g, sv.d);
    hipLaunchKernelGGL(k_gap_find, dim3(g.n), dim3(1024), 0, st, g);
}

void launch_push(const Geom &g, const State &sv, const Work &win, const Work &wout, Scratch *s,
                 bool down, hipStream_t st)
{
    const dim3 grid(sweep_blocks(g)), block(256);
    if (g.soft) {
        if (down) hipLaunchKernelGGL((k_push<true, true>), grid, block, 0, st, g, sv, win, wout, s);
        else hipLaunchKernelGGL((k_push<false, true>), grid, block, 0, st, g, sv, win, wout, s);
    } else {
        if (down) hipLaunchKernelGGL((k_push<true, false>), grid, block, 0, st, g, sv, win, wout, s);
        else hipLaunchKernelGGL((k_push<false, false>), grid, block, 0, st, g, sv, win, wout, s);
    }
}

void launch_compact(const Geom &g, const Work &w, int *next_count, hipStream_t st)
{
    const long long n = g.Ptot > g.n ? g.Ptot : g.n;
    hipLaunchKernelGGL(k_compact, dim3((unsigned)((n + 1023) / 1024)), dim3(1024), 0, st, g, w, next_count);
}

void launch_relabel(const Geom &g, const State &sv, const Work &win, const Work &wout, bool use_gap,
                    hipStream_t st)
{
    const int ug = use_gap ? 1 : 0;
    if (g.soft) hipLaunchKernelGGL(k_relabel<true>, dim3(sweep_blocks(g)), dim3(256), 0, st, g, sv, win, wout, ug);
    else hipLaunchKernelGGL(k_relabel<false>, dim3(sweep_blocks(g)), dim3(256), 0, st, g, sv, win, wout, ug);
}

void launch_mincut_init(const Geom &g, const State &sv, int *H, hipStream_t st)
{
    hipLaunchKernelGGL(k_mincut_init, dim3(wave_blocks(g)), dim3(256), 0, st, g, sv, H);
}

void launch_hmax(const Geom &g, const State &sv, int *Hmax, hipStream_t st)
{
    hipLaunchKernelGGL(k_hmax, dim3(wave_blocks(g)), dim3(256), 0, st, g, sv, Hmax);
}

void launch_mincut_pass(const Geom &g, const State &sv, int *H, Scratch *s, hipStream_t st)
{
    if (g.soft) hipLaunchKernelGGL(k_mincut_pass<true>, dim3(blocks_for(g.Ptot)), dim3(256), 0, st, g, sv, H, s);
    else hipLaunchKernelGGL(k_mincut_pass<false>, dim3(blocks_for(g.Ptot)), dim3(256), 0, st, g, sv, H, s);
}

void launch_finish(const int *cost, const Geom &g, const State &sv, int *H, hipStream_t st)
{
    if (g.soft) hipLaunchKernelGGL(k_finish<true>, dim3(wave_blocks(g)), dim3(256), 0, st, cost, g, sv, H);
    else hipLaunchKernelGGL(k_finish<false>, dim3(wave_blocks(g)), dim3(256), 0, st, cost, g, sv, H);
}

}  // namespace smf
