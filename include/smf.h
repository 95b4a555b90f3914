/*
 * smf -- exact surface max-flow on MI355X (gfx950).
 *
 * Solves the optimal delta-smooth net surface of an int32 cost volume as an
 * exact s-t minimum cut (Section 1.2: multi-column proper-ordered graph whose
 * node weights become terminal arc capacities; Section 1.3: max-flow / min-cut,
 * Eqs. 2-7, Theorem 1.1) with a push-relabel method (Section 2.1) run as
 * hand-written HIP kernels.
 *
 * The graph G(c, delta) of a cost volume c[x][y][z] (nx * ny columns of K
 * nodes, z fastest in memory):
 *   B = max_p c(p,0) + 1;  w(p,0) = c(p,0) - B;  w(p,z) = c(p,z) - c(p,z-1);
 *   s -> v with capacity -w(v) if w(v) < 0;  v -> t with capacity w(v) if
 *   w(v) > 0;  (p,z) -> (p,z-1) infinite (z >= 1);  (p,z) -> (q, max(0,
 *   z - delta)) infinite for each 4-neighbour column q inside the grid.
 * Results:
 *   - the max-flow value F (Eq. 5), as int64;
 *   - the surface h(p) = max{z : (p,z) in S_min}, where S_min is the source
 *     side of the inclusion-minimal minimum cut.  h is the pointwise-lowest
 *     surface minimising E(h) = sum_p c(p, h(p)) subject to
 *     |h(p) - h(q)| <= delta for 4-neighbours (Eq. 1 with a hard prior);
 *   - E* = E(h).
 *
 * Conventions for every entry point:
 *   - "device pointer" means memory the caller allocated on the current HIP
 *     device; the caller keeps ownership.  Volumes are contiguous
 *     [nx][ny][K] int32 (z fastest), surfaces contiguous [nx][ny] int32.
 *   - A handle belongs to the HIP device that was current when it was
 *     created: every device pointer and stream passed with it must belong
 *     to that device (the library cannot check this; memory of another
 *     device is a fault, not an error code).
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *   - Every int-returning call returns SMF_OK (0) or a negative SMF_ERR_*
 *     code; smf_last_error() then describes the failure (thread-local).
 *   - A handle is not thread-safe; use one handle per host thread.
 */
#ifndef SMF_H
#define SMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SMF_OK = 0,
    SMF_ERR_ARG = -1,           /* bad argument (NULL, size, shape mismatch) */
    SMF_ERR_NOMEM = -2,         /* device or host allocation failed */
    SMF_ERR_RANGE = -3,         /* |cost| >= 2^30, nx*ny*K > 2^30 - 2 for a volume,
                                   2^31 or more columns in a batch, or an int32
                                   excess/flow counter would overflow */
    SMF_ERR_NOT_CONVERGED = -4, /* sweep cap reached before termination */
    SMF_ERR_HIP = -5,           /* a HIP runtime call failed */
    SMF_ERR_NOT_SOLVED = -6     /* result requested before a successful solve */
};

typedef struct smf_handle smf_handle;

/* Allocates all solver state for one nx x ny x K volume with smoothness
 * bound delta (Section 1.2, the "edge interval") on the current device:
 * 32 bytes per node, 5 bits per node (rounded up to 64 heights) of
 * breadth-first-search bit masks, plus O(nx*ny).  Returns NULL on failure (see
 * smf_last_error).  Requires nx, ny, K >= 1, delta >= 0,
 * nx*ny*K <= 2^30 - 2 (every finite distance label then stays below the
 * solver's reserved label values).  The handle is a batch of one volume:
 * the smf_batch_* calls accept it too.  If the environment variable
 * SMF_DEVICE_MEM_LIMIT holds a byte count, a handle that would need more
 * device memory than that is refused with SMF_ERR_NOMEM before anything is
 * allocated (also for smf_batch_create). */
smf_handle *smf_create(int32_t nx, int32_t ny, int32_t K, int32_t delta);

/* Allocates one handle for a batch of n independent volumes of uneven
 * shapes (nx[i], ny[i], K[i], delta[i]; host arrays of n entries, read
 * during the call only), each meeting the limits of smf_create; the batch
 * holds fewer than 2^31 columns in total.  The volumes are solved together:
 * every kernel launch of a solve covers all of them, each with its own
 * work lists, global-relabel schedule and termination (the paper solves
 * one volume at a time; batching serves many small volumes, which alone
 * would leave most of the GPU idle).  Node state is packed volume after
 * volume in the order given, 32 bytes per node. */
smf_handle *smf_batch_create(int32_t n, const int32_t *nx, const int32_t *ny,
                             const int32_t *K, const int32_t *delta);

/* Releases the handle and its device memory.  NULL is allowed. */
void smf_destroy(smf_handle *h);

/* Solves the volume `cost_dev` (device pointer, [nx][ny][K] int32, every
 * value in (-2^30, 2^30)): builds the graph of Section 1.2 from the costs,
 * runs push-relabel with global relabelling (Section 2.1) to a maximum
 * preflow, and reads the minimum cut off it (Section 1.3, Eqs. 5-7,
 * Theorem 1.1).  Work is enqueued on `stream`; the call drives
 * the iteration from the host and returns when the result is complete, so
 * on SMF_OK the flow value, energy and surface are ready.  The cost buffer
 * is only read.  SMF_ERR_ARG for a batch handle of more than one volume. */
int smf_solve(smf_handle *h, const int32_t *cost_dev, void *stream);

/* Solves every volume of a batch handle.  Volume i's [nx][ny][K] int32
 * costs start at packed_cost_dev + offsets_host[i] (device pointer plus a
 * host array of n non-negative int64 element offsets, read during the call;
 * NULL offsets mean densely packed in order).  Same value range, stream and
 * completion rules as smf_solve; one failing volume fails the call. */
int smf_batch_solve(smf_handle *h, const int32_t *packed_cost_dev, const int64_t *offsets_host,
                    void *stream);

/* Max-flow value F of the last successful solve (host int64 out): the
 * flow into t of Eq. 5, equal to the capacity of the minimum cut
 * (Theorem 1.1).
 * SMF_ERR_ARG for a batch of more than one volume. */
int smf_flow_value(const smf_handle *h, int64_t *out);

/* Optimal energy E* = sum_p c(p, h(p)) of the last successful solve (the
 * surface cost of Eq. 1 at the minimal-cut surface), plus
 * alpha * sum |h(p) - h(q)| over 4-neighbour column pairs when the soft
 * smoothness weight alpha ("smooth_weight") is positive.
 * SMF_ERR_ARG for a batch of more than one volume. */
int smf_energy(const smf_handle *h, int64_t *out);

/* Max-flow values of every volume of the last successful batch solve
 * (host array of n int64, Eq. 5 per volume). */
int smf_batch_flow_values(const smf_handle *h, int64_t *out);

/* Optimal energies E* of every volume of the last successful batch solve
 * (host array of n int64). */
int smf_batch_energies(const smf_handle *h, int64_t *out);

/* Copies the minimal-cut surface h (values in [0, K-1]) of the last
 * successful solve into `out_dev`: h(p) is the highest node of column p on
 * the source side of the inclusion-minimal minimum cut (Eqs. 6-7,
 * Theorem 1.1), the pointwise-lowest minimiser of Eq. 1 under the smoothness
 * bound (device pointer, [nx][ny] int32),
 * enqueued on `stream`. */
int smf_surface(const smf_handle *h, int32_t *out_dev, void *stream);

/* Copies the pointwise-highest optimal surface h_max of the last successful
 * solve into `out_dev` (device pointer, [nx][ny] int32; for a batch the
 * packed surfaces as smf_batch_surfaces): h_max(p) is the highest node of
 * column p on the source side of the maximal minimum cut, the set of nodes
 * that cannot reach t in the residual graph (Eq. 6, Theorem 1.1).  Where
 * h_max(p) = h(p) the column's optimal height is unique, which is where the
 * energy is differentiable in that column's costs (Eq. 1).  Needs param
 * "hmax" = 1 during the solve (one more complete global relabel after
 * termination); SMF_ERR_NOT_SOLVED otherwise.  Enqueued on `stream`. */
int smf_surface_max(const smf_handle *h, int32_t *out_dev, void *stream);

/* Copies the surfaces of every volume of the last successful batch solve
 * into `packed_out_dev` (device pointer, sum_i nx[i]*ny[i] int32): volume
 * i's [nx][ny] heights follow those of volumes 0..i-1.  Enqueued on
 * `stream`. */
int smf_batch_surfaces(const smf_handle *h, int32_t *packed_out_dev, void *stream);

/* Copies the final preflow of the last successful solve into caller device
 * buffers, each [nx][ny][K] int32 (z fastest) except `flow_lat_dev`, which
 * is [4][nx][ny][K] in neighbour order +x, -x, +y, -y:
 *   excess_dev   -- excess e(v) >= 0 left at each node;
 *   sink_res_dev -- residual capacity of v -> t;
 *   flow_down_dev-- flow on (p,z) -> (p,z-1) (0 at z = 0);
 *   flow_lat_dev -- flow on (p,z) -> (q, z - delta), stored for z > delta,
 *                   and on (p,0) -> (q,0); 0 for absent arcs.  The solver
 *                   omits the arcs (p,z) -> (q,0) for 1 <= z <= delta, which
 *                   are implied by (p,z) -> (p,0) -> (q,0) and change no cut.
 * Source arcs are saturated and never carry flow back.  For a batch, each
 * buffer holds the volumes' nodes packed in order (total T nodes; flow_lat
 * [4][T]).  The flows on the soft smoothness arcs (smooth_weight > 0) come
 * from smf_export_soft_flows.  For certificates and debugging; enqueued on
 * `stream`. */
int smf_export_state(const smf_handle *h, int32_t *excess_dev, int32_t *sink_res_dev,
                     int32_t *flow_down_dev, int32_t *flow_lat_dev, void *stream);

/* Copies the flows on the soft smoothness arcs (p,z) -> (q,z) of the last
 * successful solve into `flow_soft_dev` (device pointer, [4][nx][ny][K]
 * int32 in neighbour order +x, -x, +y, -y; for a batch [4][T] over the
 * packed nodes): the arc's flow is stored at its tail, 0 at z = 0 and for
 * absent neighbours (the soft arcs of Section 1.2's edge costs, see
 * "smooth_weight").  SMF_ERR_ARG if no positive smooth_weight is set.
 * Enqueued on `stream`. */
int smf_export_soft_flows(const smf_handle *h, int32_t *flow_soft_dev, void *stream);

/* Narrow band (Section 3.4: the graph is built only in a band of heights
 * around the surface that the user's landmarks outline, a stick of heights
 * above and below it).  For a handle of one volume: column p = x*ny + y
 * holds only the heights offset_host[p] .. offset_host[p] + extent_host[p]
 * - 1 of the volume (host arrays of nx*ny int32, read during the call;
 * offset >= 0, 1 <= extent <= K, offset + extent <= 2^30), and the cost
 * volume passed to smf_solve then holds, at [x][y][j], the cost at height
 * offset[p] + j (j < extent[p]; entries beyond are not read).  A surface takes
 * one height in every column's band with |h(p) - h(q)| <= delta.  The call
 * finds the heights such surfaces actually take per column, [lo(p), hi(p)]
 * (the pairwise bounds lo(q) >= lo(p) - delta, hi(p) <= hi(q) + delta at
 * their fixed point; each bound is attained), and the graph is Section 1.2's
 * on those heights: B = max_p c(p, lo(p)) + 1, w(p, lo(p)) = c(p, lo(p)) - B,
 * lateral arcs (p, z) -> (q, max(lo(q), z - delta)).  smf_surface then
 * returns heights of the volume, smf_energy sum_p c(p, h(p)) and
 * smf_flow_value the max-flow of that graph; smf_export_state stores node
 * (p, lo(p) + j) at [x][y][j] (slots above hi(p) - lo(p) unused, all zero).
 * SMF_ERR_ARG when no delta-smooth surface fits the bands, for a batch of more
 * than one volume, with a positive smooth_weight, or for bad values;
 * SMF_ERR_NOMEM if the 12-byte-per-column table cannot be allocated (once
 * per handle).  NULL for both arrays removes the band. */
int smf_set_band(smf_handle *h, const int32_t *offset_host, const int32_t *extent_host);

/* Tuning and limits.  Keys:
 *   "relabel_period"  -- sweeps between global relabels (>= 1, default 2;
 *                        for a batch: of every volume, replacing any per-volume
 *                        periods)
 *   "push_phases"     -- push phases per sweep, each followed by a list of the
 *                        columns it left with excess; one relabel phase ends
 *                        the sweep (1..8, default 3; for the whole handle)
 *   "max_sweeps"      -- sweep cap before SMF_ERR_NOT_CONVERGED (>= 1)
 *   "poll_every"      -- sweeps between host termination checks (>= 1)
 *   "bfs_poll_every"  -- BFS levels between host convergence checks (1..62)
 *   "gap_every"       -- sweeps between searches for an empty label (gap
 *                        heuristic, Section 2.1; labels below 4096 are
 *                        tracked); 0 turns it off (default 0)
 *   "level_block"     -- threads per block of a breadth-first-search level
 *                        launch (power of two in [64, 1024], default 256)
 *   "sweep_waves"     -- waves of a push or relabel launch (default 8192;
 *                        at most one per column)
 *   "bfs_early_stop"  -- 1 (default): end a global relabel once every node
 *                        with excess is labelled; 0: always run it to the end
 *   "search_quorum"   -- for a batch: a global relabel ends for all of its
 *                        volumes once this percentage of them has ended (1..100,
 *                        default 90); the nodes of the others that no level
 *                        reached get the first level not run as their label,
 *                        a valid lower bound of their distance to t (the
 *                        complete global relabel of "hmax" always runs to its
 *                        end)
 *   "block_search"    -- 1 (default): when every volume of the handle has at
 *                        most 2048 columns and 16384 64-height column chunks,
 *                        each global relabel runs as one block per volume
 *                        with its records (and, when both fit in 160 KB, its
 *                        bit masks) in LDS (no launch or host poll per level;
 *                        in a batch the blocks also stop once search_quorum of
 *                        the volumes have ended); 0: always one launch per level
 *   "hmax"            -- 1: every solve also reads out the highest optimal
 *                        surface (smf_surface_max) with one complete global
 *                        relabel after termination; the first 1 allocates
 *                        4 bytes per column (SMF_ERR_NOMEM if that fails)
 *   "verbose"         -- 1: one progress line per poll and global relabel on stderr
 *   "count_work"      -- 1: kernels count their algorithmic bytes ("bytes.<class>"
 *                        statistics of bfs, push, relabel; one atomic per wave
 *                        into 64 spread counters)
 *   "kernel_timing"   -- bit mask of kernel classes (bit 0 build, 1 bfs_reset,
 *                        2 bfs, 3 push, 4 relabel, 5 mincut, 6 finish): every
 *                        launch of a selected class is bracketed by HIP events
 *                        on the solve stream (for benchmarks); 0: off
 *   "smooth_weight"   -- soft smoothness weight alpha in [0, 2^29] (default 0;
 *                        for a batch: of every volume).  The energy becomes
 *                        sum_p c(p, h(p)) + alpha * sum |h(p) - h(q)| over
 *                        4-neighbour column pairs, still with |h(p) - h(q)|
 *                        <= delta (the edge costs of the VCE-weight net
 *                        surface, Section 1.2, with the convex cost alpha|d|):
 *                        arcs (p,z) -> (q,z) of capacity alpha for z >= 1.
 *                        The first positive weight allocates 16 bytes and 4
 *                        bits (rounded up to 64 heights) more per node, kept
 *                        until smf_destroy; SMF_ERR_NOMEM if that fails.
 *                        With every weight 0 the solver runs its kernels
 *                        without soft arcs.
 * Returns SMF_ERR_ARG for an unknown key or an out-of-range value. */
int smf_set_param(smf_handle *h, const char *key, int64_t value);

/* Per-volume tuning of a batch: `values` is a host array of n int64.
 * Key "relabel_period": sweeps between global relabels of each volume
 * (0: the handle's relabel_period).  A search starts once some volume's
 * period has come round, and every volume at least halfway through its own
 * period joins it, so volumes of different periods share searches.
 * Key "smooth_weight": the soft smoothness weight of each volume (as for
 * smf_set_param; volumes may differ, 0 for none).
 * SMF_ERR_ARG for other keys or out-of-range values. */
int smf_batch_set_param(smf_handle *h, const char *key, const int64_t *values);

/* Counters of the last solve.  Keys: "sweeps", "global_relabels",
 * "bfs_passes", "mincut_passes", "gap_relabels" (active nodes frozen by the
 * gap heuristic), "gap_searches", and with kernel_timing on,
 * "time_ns.<class>" (summed event time) and "launches.<class>" for the
 * kernel classes build, bfs_reset, bfs, push, relabel, mincut, finish, and
 * "band" (1 with a narrow band set), the settings "push_phases" and
 * "relabel_period" (the handle's), "bytes.<class>": algorithmic bytes of the
 * class over the solve (state words
 * read or written, each access counted once; counted on the device for the
 * data-dependent classes bfs, push and relabel), and the sizes "volumes",
 * "columns" and "nodes".  For a batch the counters cover the whole batch
 * ("sweeps" and "global_relabels" count batch-wide steps). */
int smf_get_stat(const smf_handle *h, const char *key, int64_t *out);

/* Per-volume values into a host array of n int64.  Counters of the last
 * batch solve: "sweeps" (sweeps while the volume still had active nodes),
 * "global_relabels" (searches the volume took part in), "gap_relabels";
 * settings: "relabel_period" (the period in use), "smooth_weight" and the
 * shape keys "nx", "ny", "K", "delta". */
int smf_batch_get_stat(const smf_handle *h, const char *key, int64_t *out);

/* Autotuner of the schedule: the relabel period and the push phases per
 * sweep (the paper tunes its relabel factor empirically, Section 3.4).
 * Volumes fall into classes keyed by (ceil log2 K, min(delta, 4), floor log2
 * (nx*ny), smooth_weight > 0).  For every class of the handle's volumes that
 * the process-wide tuning cache does not hold yet, the largest volume of that
 * class is solved (with its smooth_weight) on a temporary handle with each
 * candidate (period, push phases) pair -- (4,1), (2,2), (1,3), (2,3), (3,3),
 * (1,4), (2,4) -- timed on the host clock (the fastest of three runs when a
 * solve takes under 0.25 s, of two under 2 s), and the fastest pair is
 * cached; then every volume of `h` gets its class's period
 * (smf_batch_set_param) and `h` the push phases of its cached class holding
 * the most nodes (push phases are one value per handle).  For a batch of
 * more than one volume the tuner then times whole solves of `h` (the faster
 * of two each) with every volume's period scaled by 1, 1.5, 2 and 3 (with the
 * class push phases) and with the uniform schedules (2,4), (3,3) and (1,6),
 * and keeps the fastest (the volumes of a batch share their searches, which
 * can favour other schedules than solving each volume alone); the cache
 * keeps the unscaled class periods.  `packed_cost_dev` and `offsets_host` are as for smf_batch_solve
 * (a plain handle: the volume, NULL offsets).  Allocates and frees the
 * temporary handles; work runs on `stream`.  If the environment variable
 * SMF_TUNE_CACHE names a file, the cache is loaded from it on first use and
 * saved to it after new timings.  The cache is shared by all host threads
 * (calls serialise on a lock).  SMF_ERR_ARG for a handle with a narrow band. */
int smf_autotune(smf_handle *h, const int32_t *packed_cost_dev, const int64_t *offsets_host,
                 void *stream);

/* Gives every volume of `h` the cached period of its class, and `h` the
 * cached push phases of its largest class, without timing (volumes of
 * unknown classes keep the handle's relabel_period). */
int smf_tune_apply(smf_handle *h);

/* Adds the entries of a tuning-cache text file (lines "kbits delta pbits
 * soft period phases best_ns"; lines "kbits delta pbits soft period
 * best_ns" are entries with one push phase, lines "kbits delta pbits period
 * best_ns" classes with soft = 0) to the cache, or writes the cache to one.
 * SMF_ERR_ARG if the file cannot be opened. */
int smf_tune_cache_load(const char *path);
int smf_tune_cache_save(const char *path);

/* Empties the tuning cache (and stops it reading SMF_TUNE_CACHE). */
int smf_tune_cache_clear(void);

/* Cached period for a volume shape without the soft smoothness term (0 if
 * its class is not cached). */
int smf_tune_lookup(int32_t nx, int32_t ny, int32_t K, int32_t delta, int64_t *period);

/* Backward of the optimal energy with respect to the costs (Section 1.1,
 * Eq. 1): grad_cost[b][x][y][z] = grad_energy[b] if z == surface[b][x][y],
 * else 0, for a batch of n surfaces.  All pointers are device pointers:
 * surface [n][nx][ny] int32 (heights in [0, K-1]), grad_energy [n] float,
 * grad_cost [n][nx][ny][K] float (fully overwritten; 16-byte aligned when
 * K % 4 == 0).  The indicator is the derivative wherever a column's optimal
 * height is unique and a supergradient otherwise.  Enqueued on `stream`;
 * returns SMF_ERR_ARG for bad sizes (n > 65535 or nx*ny > 2^31 - 1
 * included) or NULL pointers. */
int smf_onehot_backward(const int32_t *surface_dev, const float *grad_energy_dev,
                        float *grad_cost_dev, int32_t n, int32_t nx, int32_t ny, int32_t K,
                        void *stream);

/* Allocation-free solve of one volume, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Computes what smf_create + smf_solve +
 * smf_flow_value + smf_energy + smf_surface + smf_destroy give for the same
 * volume (no soft smoothness term, default schedule) and calls no hipMalloc,
 * hipFree, pinned-memory or other allocating routine.  Inputs and outputs are
 * the caller's: cost_dev [nx][ny][K] int32 device pointer (values in
 * (-2^30, 2^30)), surface_dev [nx][ny] int32 device pointer (written),
 * flow_out and energy_out host int64 (written on SMF_OK).  All solver state
 * lives in one static device array of SMF_NOALLOC_MAX_BYTES bytes that every
 * GPU the library runs on holds until the process ends; a volume needs
 * about 33 bytes per node plus 120 bytes per column, and a larger one is
 * refused with SMF_ERR_NOMEM before any device work.  Calls on one GPU share
 * that array: calls that overlap on one GPU (other host threads, or streams
 * not ordered with the previous call's) race and give wrong results.
 * Blocks the host until the result is complete (counters are read with
 * blocking copies); work runs on `stream`. */
#define SMF_NOALLOC_MAX_BYTES (64ULL << 20)
int smf_solve_noalloc(const int32_t *cost_dev, int32_t nx, int32_t ny, int32_t K, int32_t delta,
                      int32_t *surface_dev, int64_t *flow_out, int64_t *energy_out, void *stream);

/* Static text for a status code. */
const char *smf_status_string(int status);

/* Description of the last failure on this host thread ("" if none). */
const char *smf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SMF_H */
