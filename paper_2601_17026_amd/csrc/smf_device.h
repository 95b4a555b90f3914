// Device-side layout and helpers shared by the solver kernels.
//
// A solve handles a batch of n independent volumes (n = 1 for a plain
// solve).  Their columns are numbered globally, volume after volume, and
// their node state is packed the same way: node (p, z) of local column
// p = x*ny + y of volume i lives at index node_base(i) + p*K(i) + z (z
// fastest, the layout of the caller's cost volume).  A wave owns one column
// at a time and processes it in chunks of 64 consecutive heights, one lane
// per height, so every load and store of the column is a coalesced 256-byte
// access; the lateral neighbours (q, z -+ delta) of a chunk are again 64
// consecutive words of column q, and the neighbours up and down the column
// are one lane away.  A kernel finds a column's volume in `col_inst` and
// its geometry in the volume table.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smf {

constexpr int kInf = 0x40000000;       // label of a node that cannot reach t
constexpr int kUnl = kInf - 1;         // not (yet) reached by the running BFS
constexpr int kErrCostRange = 1;       // a cost outside (-2^30, 2^30)
constexpr int kErrOverflow = 2;        // an int32 excess or flow would overflow
constexpr int kErrSearch = 4;          // a one-block search ran past its level bound
constexpr int kWave = 64;              // CDNA wavefront width = heights per chunk
constexpr int kLvlSlots = 64;          // BFS level flags kept per volume
constexpr int kMaxRanges = 16;         // column ranges a BFS level launch covers

// Geometry of one volume of the batch (64 bytes, read with scalar loads).
struct Inst {
    int nx, ny, K, delta;
    int P;          // columns
    int nch;        // 64-height chunks per column
    int cpb;        // chunks per work-mask bit (nch <= 64 * cpb)
    int lab_cap;    // labels >= lab_cap are unreachable (N + 1, at most kInf)
    int col_base;   // first global column
    int alpha;      // soft smoothness weight: arcs (p,z) -> (q,z), z >= 1, capacity alpha
    long long node_base;   // first global node
    long long cost_base;   // first cost word in the caller's packed cost array
    long long N;           // nodes
};

// Per-volume device counters.
struct InstScratch {
    long long flow;      // sum of flow into t
    long long energy;    // sum_p c(p, h(p))
    int bmax;            // max_p c(p, 0)
    int active;          // active nodes after the last relabel phase
    int bfs_active;      // nodes with excess and a finite label when the BFS starts
    int bfs_unsat[2];    // columns holding such a node that the running BFS has not
                         // labelled yet (the early stop waits for 0), counted at
                         // alternate host polls into alternate slots
    int gap;             // labels above `gap` cannot reach t (kInf: no gap known)
    int gap_frozen;      // active nodes cut off by the gap heuristic
    int pad[5];
    int lvl_changed[kLvlSlots];   // BFS level L labelled something: slot L % 64
};

struct Geom {
    int n;                  // volumes
    int Ptot;               // columns of all volumes
    long long Ntot;         // nodes of all volumes
    const Inst *inst;       // n entries
    const int *col_inst;    // Ptot entries: the volume of each global column
    InstScratch *is;        // n entries
    const int *part;        // n: 1 if the volume takes part in the running global relabel
    const int *fill;        // n: label of the nodes that relabel left unreached (-1: none)
    int count_work;         // 1: kernels add their algorithmic bytes to `work`
    // [3 classes][64 slots][16] counters: a wave adds to slot blockIdx % 64 of
    // its class (entry 0 of the slot), so the adds spread over 64 cache lines
    unsigned long long *work;
    int *hist;              // n x hist_len: nodes per finite label, labels < hist_len
    int hist_len;
    // Per-column bit masks of the running global relabel, one bit per node,
    // word-major: word w (heights 64w..64w+63) of mask m of column p is
    // bits[(m * max_nch + w) * Ptot + p], so that the columns of a wave read
    // adjacent words.  Masks: kMaskFl + k (lateral arc in direction k carries
    // flow), kMaskFd (down arc carries flow).
    unsigned long long *bits;
    int max_nch;
    // the largest volume's columns and 64-height column chunks (whether every
    // volume's search fits one block)
    int max_cols;
    long long max_chunks;
    // With soft smoothness (some volume has alpha > 0): four more masks,
    // bit set where the soft arc (p,z) -> (q_k,z) is residual, stored like
    // `bits` (sbits[(k * max_nch + w) * Ptot + p]); soft is 0 otherwise and
    // the kernels without soft arcs run.
    unsigned long long *sbits;
    int soft;
    // Per column, the lowest height of a node with excess and a finite label
    // when the running global relabel started (K if none), and the list of
    // the columns whose lowest such node lies below the level-1 suffix.
    int *low_act;
    int *short_list;
    int *short_count;
    // launch geometry: threads per block of a BFS level, waves of a push or
    // relabel phase
    int level_block;
    int sweep_waves;
    // Narrow band (a single volume): column p holds the heights blo[p] ..
    // blo[p] + bext[p] - 1 of the volume (the range that smooth surfaces
    // inside the caller's bands take there) in its node slots 0 .. bext[p]-1;
    // the slots above are unused (no excess, no arcs, label kInf).  Slot j's
    // cost is the caller's cost bcs[p] + j of the column.  band = 0: every
    // column holds the heights 0 .. K-1.
    int band;
    const int *blo;
    const int *bext;
    const int *bcs;
};
constexpr int kMaskFl = 0, kMaskFd = 4, kMasks = 5;
constexpr int kWorkSlots = 64, kWorkStride = 16;

// Per-node solver state; each array holds Ntot int32, packed as above.
struct State {
    int *e;    // excess
    int *d;    // distance label (lower bound of the residual distance to t)
    int *ts;   // residual capacity of v -> t
    int *fd;   // flow on (p,z) -> (p,z-1)
    int *fl;   // 4 x Ntot: flow on (p,z) -> (q, zt(z)), q = p + (+x, -x, +y, -y)
    int *sf;   // 4 x Ntot with soft smoothness: flow on (p,z) -> (q,z) (else NULL)
};

// Work tracking of the push/relabel sweeps: per global column a 64-bit mask
// of the chunk groups that may hold a node with excess and a finite label,
// and a list of the columns whose mask is not empty.
struct Work {
    unsigned long long *mask;   // Ptot masks
    int *list;                  // up to Ptot column ids
    int *count;                 // device counter of `list`
};

// Batch-wide device counters and flags.  The per-volume counters follow
// them in the same allocation, kScratchHead bytes after the start, so one
// copy snapshots both.
// Columns that a BFS level launch covers: thread t with pre[r] <= t <
// pre[r + 1] (r < n) takes column lo[r] + t - pre[r].
struct LevelRanges {
    int n;
    int lo[kMaxRanges];
    int pre[kMaxRanges + 1];
};

struct Scratch {
    int err;             // kErr* bits
    int changed;         // a min-cut pass changed something
    int count[2];        // sizes of the two column work lists
    int short_count;     // size of the running global relabel's short-column list
    int block_levels;    // levels run by one-block searches since the solve began
    int block_done;      // volumes whose one-block search has ended (the running search)
};
constexpr int kScratchHead = 64;
static_assert(sizeof(Scratch) <= kScratchHead, "Scratch must fit its header");
static_assert(sizeof(InstScratch) % 8 == 0, "InstScratch keeps 8-byte alignment");

// Lateral arcs kept by the solver: (p,z) -> (q, z - delta) for z > delta,
// and (p,0) -> (q,0).  The arcs (p,z) -> (q,0), 1 <= z <= delta, are implied
// by (p,z) -> (p,0) -> (q,0) and change no closed set, hence no cut.
__device__ __forceinline__ bool lat_arc(int z, int delta) { return z == 0 || z > delta; }
__device__ __forceinline__ int lat_head(int z, int delta) { return z == 0 ? 0 : z - delta; }
// Height of the tail of the lateral arc that ends at height z (or -1 when
// no kept arc ends there within a column of K nodes).
__device__ __forceinline__ int lat_tail(int z, int delta, int K)
{
    int zt = z == 0 ? 0 : z + delta;
    return zt < K ? zt : -1;
}

// Band geometry of column p: its extent, and per neighbour direction k the
// height shift sh[k] of its lateral arcs (p, z) -> (q_k, z - sh[k]) (z > sh[k],
// plus (p,0) -> (q_k,0)), the shift shr[k] of the arcs (q_k, z) -> (p, z -
// shr[k]) and q_k's extent.  Without a band every shift is delta and every
// extent K.  q[k] < 0: no neighbour (the values are then unused).
struct BandCol {
    int ext;
    int sh[4], shr[4], qext[4];
};

__device__ __forceinline__ void band_col(const Geom &g, int p, const int q[4], int K, int delta, BandCol &b)
{
    if (!g.band) {
        b.ext = K;
#pragma unroll
        for (int k = 0; k < 4; ++k) { b.sh[k] = delta; b.shr[k] = delta; b.qext[k] = K; }
        return;
    }
    const int lo = g.blo[p];
    b.ext = g.bext[p];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int lq = q[k] >= 0 ? g.blo[q[k]] : lo;
        b.sh[k] = delta + lq - lo;
        b.shr[k] = delta + lo - lq;
        b.qext[k] = q[k] >= 0 ? g.bext[q[k]] : K;
    }
}

// Global neighbour column in direction k (0:+x, 1:-x, 2:+y, 3:-y) of global
// column p at local position (x, y) of a volume with nx x ny columns, or -1.
__device__ __forceinline__ int nbr(int nx, int ny, int x, int y, int p, int k)
{
    switch (k) {
    case 0: return x + 1 < nx ? p + ny : -1;
    case 1: return x > 0 ? p - ny : -1;
    case 2: return y + 1 < ny ? p + 1 : -1;
    default: return y > 0 ? p - 1 : -1;
    }
}

}  // namespace smf
