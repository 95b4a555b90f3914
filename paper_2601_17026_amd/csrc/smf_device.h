// Device-side layout and helpers shared by the solver kernels.
//
// Node state is stored column-major exactly like the caller's cost volume:
// node (p, z) of column p = x*ny + y lives at index p*K + z (z fastest).  A
// wave owns one column at a time and processes it in chunks of 64
// consecutive heights, one lane per height, so every load and store of the
// column is a coalesced 256-byte access; the lateral neighbours (q, z -+
// delta) of a chunk are again 64 consecutive words of column q, and the
// neighbours up and down the column are one lane away.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smf {

constexpr int kInf = 0x40000000;       // label of a node that cannot reach t
constexpr int kUnl = kInf - 1;         // not (yet) reached by the running BFS
constexpr int kErrCostRange = 1;       // a cost outside (-2^30, 2^30)
constexpr int kErrOverflow = 2;        // an int32 excess or flow would overflow
constexpr int kWave = 64;              // CDNA wavefront width = heights per chunk

struct Geom {
    int nx, ny, K, delta;
    int P;        // columns
    int N;        // nodes (< 2^31)
    int lab_cap;  // labels >= lab_cap are unreachable (N + 1, at most kInf)
    int nch;      // 64-height chunks per column
    int cpb;      // chunks per work-mask bit (nch <= 64 * cpb)
    int count_work;  // 1: kernels add their algorithmic bytes to `work`
    // [3 classes][64 slots][16] counters: a wave adds to slot blockIdx % 64 of
    // its class (entry 0 of the slot), so the adds spread over 64 cache lines
    unsigned long long *work;
    int *hist;       // number of nodes per finite label, labels < hist_len
    int hist_len;
};
constexpr int kWorkSlots = 64, kWorkStride = 16;

// Per-node solver state; each array holds N int32, column-major.
struct State {
    int *e;    // excess
    int *d;    // distance label (lower bound of the residual distance to t)
    int *ts;   // residual capacity of v -> t
    int *fd;   // flow on (p,z) -> (p,z-1)
    int *fl;   // 4 x N: flow on (p,z) -> (q, zt(z)), q = p + (+x, -x, +y, -y)
};

// Work tracking of the push/relabel sweeps: per column a 64-bit mask of the
// chunk groups that may hold a node with excess and a finite label, and a
// list of the columns whose mask is not empty.
struct Work {
    unsigned long long *mask;   // P masks
    int *list;                  // up to P column ids
    int *count;                 // device counter of `list`
};

// Device-resident counters and flags of one solve.
struct Scratch {
    int bmax;            // max_p c(p, 0)
    int err;             // kErr* bits
    int changed;         // a min-cut pass changed something
    int active;          // active nodes after the last relabel phase
    long long flow;      // sum of flow into t
    long long energy;    // sum_p c(p, h(p))
    int bfs_active;      // nodes with excess and a finite label when the BFS starts
    int bfs_labelled;    // ... of which the running BFS has labelled so far
    int count[2];        // sizes of the two column work lists
    int gap;             // labels above `gap` cannot reach t (kInf: no gap known)
    int gap_frozen;      // active nodes cut off by the gap heuristic
    int lvl_changed[64]; // BFS level L labelled something: slot L % 64
};

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

// Neighbour column in direction k (0:+x, 1:-x, 2:+y, 3:-y), or -1.
__device__ __forceinline__ int nbr(const Geom &g, int x, int y, int p, int k)
{
    switch (k) {
    case 0: return x + 1 < g.nx ? p + g.ny : -1;
    case 1: return x > 0 ? p - g.ny : -1;
    case 2: return y + 1 < g.ny ? p + 1 : -1;
    default: return y > 0 ? p - 1 : -1;
    }
}

}  // namespace smf
