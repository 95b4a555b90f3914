// Host driver and C-ABI of the exact surface max-flow (include/smf.h).
//
// One handle owns the node state of one volume (32 bytes per node, in the
// caller's [nx][ny][K] layout) plus per-column work lists and BFS records,
// a small device scratch block and a pinned host mirror of it.
// smf_solve enqueues the build, the initial global relabel and then sweeps
// of push and relabel phases on the caller's stream; the host polls the
// device's active-node counter every `poll_every` sweeps (the only
// device-to-host traffic of the loop) and runs a global relabel every
// `relabel_period` sweeps.  Termination: no node with excess and a finite
// label remains (Section 3.2.4 decides this with flags and locks across
// threads; here it is one counter written by the relabel phase).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/smf.h"
#include "smf_device.h"

namespace smf {
void launch_init_scratch(Scratch *s, hipStream_t st);
void launch_set_int(int *p, int v, hipStream_t st);
void launch_fill(int *a, int n, int v, hipStream_t st);
void launch_work_init(const Geom &g, const Work &a, const Work &b, hipStream_t st);
void launch_build(const int *cost, const Geom &g, const State &sv, Scratch *s, hipStream_t st);
void launch_bfs_init(const Geom &g, const State &sv, int *T, int *LF, int *CH, Scratch *s,
                     hipStream_t st);
void launch_bfs_level(const Geom &g, const State &sv, int L, const int *Tin, const int *LFin,
                      const int *CHin, int *Tout, int *LFout, int *CHout, Scratch *s,
                      hipStream_t st);
void launch_bfs_fixup(const Geom &g, const State &sv, int v, hipStream_t st);
void launch_push(const Geom &g, const State &sv, const Work &win, const Work &wout, Scratch *s,
                 bool down, hipStream_t st);
void launch_relabel(const Geom &g, const State &sv, const Work &win, const Work &wout, Scratch *s,
                    hipStream_t st);
void launch_compact(const Geom &g, const Work &w, hipStream_t st);
void launch_gap_find(const Geom &g, const State &sv, Scratch *s, hipStream_t st);
void launch_mincut_init(const Geom &g, const State &sv, int *H, hipStream_t st);
void launch_mincut_pass(const Geom &g, const State &sv, int *H, Scratch *s, hipStream_t st);
void launch_finish(const int *cost, const Geom &g, const State &sv, const int *H, Scratch *s,
                   hipStream_t st);
}  // namespace smf

using namespace smf;

static thread_local std::string g_last_error;

static int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

#define HIP_TRY(call)                                                                     \
    do {                                                                                  \
        hipError_t err_ = (call);                                                         \
        if (err_ != hipSuccess)                                                           \
            return fail(SMF_ERR_HIP, std::string(#call ": ") + hipGetErrorString(err_)); \
    } while (0)

// Optional per-kernel timing with HIP events recorded on the solve stream
// around every launch of a kernel class; read back at the host sync points.
enum KClass { KC_BUILD, KC_BFS_RESET, KC_BFS, KC_PUSH, KC_RELABEL, KC_MINCUT, KC_FINISH, KC_COUNT };
static const char *const kKClassName[KC_COUNT] = {"build", "bfs_reset", "bfs", "push", "relabel",
                                                  "mincut", "finish"};

struct KernelTimer {
    unsigned on = 0;   // bit i: time kernel class i
    struct Pending { int kc; int n; hipEvent_t a, b; };
    std::vector<hipEvent_t> pool;
    std::vector<Pending> pending;
    double ns[KC_COUNT] = {};
    int64_t launches[KC_COUNT] = {};

    hipEvent_t take()
    {
        if (pool.empty()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            return e;
        }
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    void reset()
    {
        for (int i = 0; i < KC_COUNT; ++i) { ns[i] = 0; launches[i] = 0; }
    }
    // Called after the stream has been synchronised.
    void collect()
    {
        for (auto &p : pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                ns[p.kc] += 1e6 * (double)ms;
                launches[p.kc] += p.n;
            }
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
    ~KernelTimer()
    {
        for (auto &p : pending) { pool.push_back(p.a); pool.push_back(p.b); }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// RAII bracket: records a start event before and an end event after the
// `n` back-to-back launches of one class made in its scope (events around
// every launch of a microsecond-scale kernel would distort its duration).
struct TimedScope {
    KernelTimer &t;
    int kc;
    hipStream_t s;
    int n;
    hipEvent_t a = nullptr;
    TimedScope(KernelTimer &t_, int kc_, hipStream_t s_, int n_ = 1) : t(t_), kc(kc_), s(s_), n(n_)
    {
        if (((t.on >> kc) & 1u) && (a = t.take())) (void)hipEventRecord(a, s);
    }
    ~TimedScope()
    {
        if (!a) return;
        hipEvent_t b = t.take();
        if (!b) { t.pool.push_back(a); return; }
        (void)hipEventRecord(b, s);
        t.pending.push_back({kc, n, a, b});
    }
};

constexpr int kHistLen = 4096;      // labels tracked by the gap heuristic (LDS bins)

struct smf_handle {
    Geom g{};
    int device = 0;
    int *state = nullptr;      // 8 * N int32
    int *H = nullptr;          // P int32 surface
    int *bfs = nullptr;        // 12 * P int32: two per-column BFS records (T, LF[4], changed)
    unsigned long long *wcount = nullptr; // algorithmic byte counters (Geom::work)
    int *hist = nullptr;                  // label histogram (Geom::hist)
    unsigned long long work_bytes[3] = {};  // their sums after the last solve
    unsigned long long *wmask = nullptr;  // 2 * P work masks
    int *wlist = nullptr;                 // 2 * P work-list entries
    Work work[2]{};            // push reads work[0] and writes work[1]; relabel the reverse
    Scratch *scr = nullptr;    // device scratch
    Scratch *host = nullptr;   // pinned mirror
    State st{};
    // parameters
    int64_t relabel_period = 6;
    int64_t max_sweeps = 2000000;
    int64_t poll_every = 1;
    int64_t bfs_poll_every = 16;
    int64_t bfs_early_stop = 1;
    int64_t verbose = 0;           // 1: progress lines on stderr
    int64_t gap_every = 0;         // sweeps between gap searches (0: off)

    // results and counters of the last solve
    bool solved = false;
    int64_t flow = 0, energy = 0;
    int64_t sweeps = 0, global_relabels = 0, bfs_passes = 0, mincut_passes = 0, gap_relabels = 0;
    int64_t gap_searches = 0;
    KernelTimer timer;
};

static void release(smf_handle *h)
{
    if (!h) return;
    if (h->state) (void)hipFree(h->state);
    if (h->H) (void)hipFree(h->H);
    if (h->bfs) (void)hipFree(h->bfs);
    if (h->wcount) (void)hipFree(h->wcount);
    if (h->hist) (void)hipFree(h->hist);
    if (h->wmask) (void)hipFree(h->wmask);
    if (h->wlist) (void)hipFree(h->wlist);
    if (h->scr) (void)hipFree(h->scr);
    if (h->host) (void)hipHostFree(h->host);
    delete h;
}

extern "C" smf_handle *smf_create(int32_t nx, int32_t ny, int32_t K, int32_t delta)
{
    g_last_error.clear();
    if (nx < 1 || ny < 1 || K < 1 || delta < 0) {
        fail(SMF_ERR_ARG, "smf_create: need nx, ny, K >= 1 and delta >= 0");
        return nullptr;
    }
    long long N = (long long)nx * ny * K;
    if (N >= (1LL << 31) || 4 * N >= (1LL << 62)) {
        fail(SMF_ERR_RANGE, "smf_create: nx*ny*K must be below 2^31");
        return nullptr;
    }
    smf_handle *h = new (std::nothrow) smf_handle;
    if (!h) {
        fail(SMF_ERR_NOMEM, "smf_create: host allocation failed");
        return nullptr;
    }
    h->g.nx = nx; h->g.ny = ny; h->g.K = K; h->g.delta = delta;
    h->g.P = nx * ny;
    h->g.N = (int)N;
    h->g.lab_cap = N + 1 < kInf ? (int)(N + 1) : kInf;
    h->g.nch = (K + kWave - 1) / kWave;
    h->g.cpb = (h->g.nch + 63) / 64;
    if (hipGetDevice(&h->device) != hipSuccess ||
        hipMalloc((void **)&h->state, sizeof(int) * 8 * (size_t)N) != hipSuccess ||
        hipMalloc((void **)&h->H, sizeof(int) * (size_t)h->g.P) != hipSuccess ||
        hipMalloc((void **)&h->bfs, sizeof(int) * 12 * (size_t)h->g.P) != hipSuccess ||
        hipMalloc((void **)&h->wcount, sizeof(unsigned long long) * 3 * kWorkSlots * kWorkStride) != hipSuccess ||
        hipMalloc((void **)&h->hist, sizeof(int) * kHistLen) != hipSuccess ||
        hipMalloc((void **)&h->wmask, sizeof(unsigned long long) * 2 * (size_t)h->g.P) != hipSuccess ||
        hipMalloc((void **)&h->wlist, sizeof(int) * 2 * (size_t)h->g.P) != hipSuccess ||
        hipMalloc((void **)&h->scr, sizeof(Scratch)) != hipSuccess ||
        hipHostMalloc((void **)&h->host, sizeof(Scratch), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        release(h);
        fail(SMF_ERR_NOMEM, "smf_create: device allocation of " +
                                std::to_string(32.0 * N / (1 << 20)) + " MiB failed");
        return nullptr;
    }
    h->g.work = h->wcount;
    h->g.hist = h->hist;
    h->g.hist_len = kHistLen;
    int *b = h->state;
    size_t n = (size_t)N;
    h->st.e = b;
    h->st.d = b + n;
    h->st.ts = b + 2 * n;
    h->st.fd = b + 3 * n;
    h->st.fl = b + 4 * n;
    for (int i = 0; i < 2; ++i) {
        h->work[i].mask = h->wmask + (size_t)i * h->g.P;
        h->work[i].list = h->wlist + (size_t)i * h->g.P;
        h->work[i].count = &h->scr->count[i];
    }
    return h;
}

extern "C" void smf_destroy(smf_handle *h) { release(h); }

// Copies the scratch block to the pinned mirror and waits for the stream.
static int sync_scratch(smf_handle *h, hipStream_t s)
{
    HIP_TRY(hipMemcpyAsync(h->host, h->scr, sizeof(Scratch), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    h->timer.collect();
    if (h->host->err & kErrCostRange)
        return fail(SMF_ERR_RANGE, "smf_solve: a cost lies outside (-2^30, 2^30)");
    if (h->host->err & kErrOverflow)
        return fail(SMF_ERR_RANGE, "smf_solve: an int32 excess or flow counter overflowed");
    return SMF_OK;
}

// Global relabel: level 1 from the sink arcs, then one launch per BFS level
// until a level labels nothing (exact distances; unreached nodes get kInf)
// or, with bfs_early_stop, until every node that holds excess is labelled
// (unreached nodes then get the first unfinished level, a valid lower
// bound).  The host checks every bfs_poll_every levels; levels launched
// after the last productive one are no-ops.
static int global_relabel(smf_handle *h, hipStream_t s)
{
    const int P = h->g.P;
    int *T[2] = {h->bfs, h->bfs + 5 * (size_t)P};
    int *LF[2] = {h->bfs + P, h->bfs + 6 * (size_t)P};
    int *CH[2] = {h->bfs + 10 * (size_t)P, h->bfs + 11 * (size_t)P};
    launch_set_int(&h->scr->bfs_active, 0, s);
    launch_set_int(&h->scr->bfs_labelled, 0, s);
    launch_set_int(&h->scr->gap, kInf, s);
    {
        TimedScope ts(h->timer, KC_BFS_RESET, s);
        launch_bfs_init(h->g, h->st, T[1], LF[1], CH[1], h->scr, s);   // level 1 lives in buffer 1
    }
    int L = 1;
    int fill = kInf;
    for (;;) {
        {
            TimedScope ts(h->timer, KC_BFS, s, (int)h->bfs_poll_every);
            for (int64_t i = 0; i < h->bfs_poll_every; ++i, ++L) {
                launch_bfs_level(h->g, h->st, L, T[L & 1], LF[L & 1], CH[L & 1], T[(L + 1) & 1],
                                 LF[(L + 1) & 1], CH[(L + 1) & 1], h->scr, s);
                h->bfs_passes++;
            }
        }
        HIP_TRY(hipGetLastError());
        int rc = sync_scratch(h, s);
        if (rc) return rc;
        if (!h->host->lvl_changed[(L - 1) & 63]) break;   // the last level launched
        if (h->bfs_early_stop && h->host->bfs_labelled >= h->host->bfs_active) {
            fill = L + 1;   // levels <= L are complete
            break;
        }
        // every productive level lowers at least one threshold by >= 1
        if ((int64_t)L > (int64_t)h->g.N + 2 + h->bfs_poll_every)
            return fail(SMF_ERR_NOT_CONVERGED, "smf_solve: breadth-first search did not settle");
    }
    {
        TimedScope ts(h->timer, KC_BFS_RESET, s);
        launch_bfs_fixup(h->g, h->st, fill, s);
    }
    if (h->verbose)
        fprintf(stderr, "smf: global relabel %lld at sweep %lld: %d levels, active %d, labelled %d, %s\n",
                (long long)h->global_relabels, (long long)h->sweeps, L - 1, h->host->bfs_active,
                h->host->bfs_labelled, fill == kInf ? "complete" : "early stop");
    h->global_relabels++;
    return SMF_OK;
}

extern "C" int smf_solve(smf_handle *h, const int32_t *cost_dev, void *stream)
{
    g_last_error.clear();
    if (!h || !cost_dev) return fail(SMF_ERR_ARG, "smf_solve: NULL handle or cost");
    hipStream_t s = (hipStream_t)stream;
    h->solved = false;
    h->sweeps = h->global_relabels = h->bfs_passes = h->mincut_passes = h->gap_relabels = 0;
    h->gap_searches = 0;
    HIP_TRY(hipSetDevice(h->device));

    h->timer.reset();
    if (h->g.count_work)
        launch_fill((int *)h->wcount, 2 * 3 * kWorkSlots * kWorkStride, 0, s);
    launch_init_scratch(h->scr, s);
    {
        TimedScope ts(h->timer, KC_BUILD, s);
        launch_build(cost_dev, h->g, h->st, h->scr, s);
    }
    HIP_TRY(hipGetLastError());
    int rc = sync_scratch(h, s);
    if (rc) return rc;
    rc = global_relabel(h, s);
    if (rc) return rc;

    // work lists: every column may hold excess anywhere before the first sweep
    launch_work_init(h->g, h->work[0], h->work[1], s);
    bool done = false;
    while (!done) {
        if (h->sweeps >= h->max_sweeps)
            return fail(SMF_ERR_NOT_CONVERGED, "smf_solve: sweep cap reached");
        for (int64_t i = 0; i < h->poll_every; ++i) {
            if (h->sweeps > 0 && h->sweeps % h->relabel_period == 0) {
                rc = global_relabel(h, s);
                if (rc) return rc;
            }
            launch_set_int(h->work[1].count, 0, s);
            {
                TimedScope ts(h->timer, KC_PUSH, s);
                launch_push(h->g, h->st, h->work[0], h->work[1], h->scr, (h->sweeps & 1) == 0, s);
            }
            launch_compact(h->g, h->work[1], s);
            launch_set_int(h->work[0].count, 0, s);
            launch_set_int(&h->scr->active, 0, s);
            {
                TimedScope ts(h->timer, KC_RELABEL, s);
                launch_relabel(h->g, h->st, h->work[1], h->work[0], h->scr, s);
            }
            h->sweeps++;
            if (h->gap_every > 0 && h->sweeps % h->gap_every == 0) {
                launch_gap_find(h->g, h->st, h->scr, s);
                h->gap_searches++;
            }
        }
        HIP_TRY(hipGetLastError());
        rc = sync_scratch(h, s);
        if (rc) return rc;
        done = h->host->active == 0;
        if (h->verbose) fprintf(stderr, "smf: sweep %lld active %d columns %d\n", (long long)h->sweeps,
                                h->host->active, h->host->count[0]);
    }

    {
        TimedScope ts(h->timer, KC_MINCUT, s);
        launch_mincut_init(h->g, h->st, h->H, s);
    }
    for (;;) {
        launch_set_int(&h->scr->changed, 0, s);
        {
            TimedScope ts(h->timer, KC_MINCUT, s);
            launch_mincut_pass(h->g, h->st, h->H, h->scr, s);
        }
        h->mincut_passes++;
        rc = sync_scratch(h, s);
        if (rc) return rc;
        if (!h->host->changed) break;
        if (h->mincut_passes > (int64_t)h->g.N + 2)
            return fail(SMF_ERR_NOT_CONVERGED, "smf_solve: minimum-cut search did not settle");
    }
    {
        TimedScope ts(h->timer, KC_FINISH, s);
        launch_finish(cost_dev, h->g, h->st, h->H, h->scr, s);
    }
    HIP_TRY(hipGetLastError());
    rc = sync_scratch(h, s);
    if (rc) return rc;
    h->flow = h->host->flow;
    h->energy = h->host->energy;
    h->gap_relabels = h->host->gap_frozen;
    if (h->g.count_work) {
        unsigned long long w[3 * kWorkSlots * kWorkStride];
        HIP_TRY(hipMemcpyAsync(w, h->wcount, sizeof(w), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int c = 0; c < 3; ++c) {
            h->work_bytes[c] = 0;
            for (int i = 0; i < kWorkSlots; ++i) h->work_bytes[c] += w[(c * kWorkSlots + i) * kWorkStride];
        }
    } else {
        h->work_bytes[0] = h->work_bytes[1] = h->work_bytes[2] = 0;
    }
    h->solved = true;
    return SMF_OK;
}

extern "C" int smf_flow_value(const smf_handle *h, int64_t *out)
{
    if (!h || !out) return fail(SMF_ERR_ARG, "smf_flow_value: NULL argument");
    if (!h->solved) return fail(SMF_ERR_NOT_SOLVED, "smf_flow_value: no successful solve");
    *out = h->flow;
    return SMF_OK;
}

extern "C" int smf_energy(const smf_handle *h, int64_t *out)
{
    if (!h || !out) return fail(SMF_ERR_ARG, "smf_energy: NULL argument");
    if (!h->solved) return fail(SMF_ERR_NOT_SOLVED, "smf_energy: no successful solve");
    *out = h->energy;
    return SMF_OK;
}

extern "C" int smf_surface(const smf_handle *h, int32_t *out_dev, void *stream)
{
    if (!h || !out_dev) return fail(SMF_ERR_ARG, "smf_surface: NULL argument");
    if (!h->solved) return fail(SMF_ERR_NOT_SOLVED, "smf_surface: no successful solve");
    HIP_TRY(hipMemcpyAsync(out_dev, h->H, sizeof(int) * (size_t)h->g.P, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return SMF_OK;
}

extern "C" int smf_export_state(const smf_handle *h, int32_t *excess_dev, int32_t *sink_res_dev,
                                int32_t *flow_down_dev, int32_t *flow_lat_dev, void *stream)
{
    if (!h || !excess_dev || !sink_res_dev || !flow_down_dev || !flow_lat_dev)
        return fail(SMF_ERR_ARG, "smf_export_state: NULL argument");
    if (!h->solved) return fail(SMF_ERR_NOT_SOLVED, "smf_export_state: no successful solve");
    // the state already has the caller's [nx][ny][K] layout
    const size_t n = sizeof(int) * (size_t)h->g.N;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(excess_dev, h->st.e, n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(sink_res_dev, h->st.ts, n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(flow_down_dev, h->st.fd, n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(flow_lat_dev, h->st.fl, 4 * n, hipMemcpyDeviceToDevice, s));
    return SMF_OK;
}

extern "C" int smf_set_param(smf_handle *h, const char *key, int64_t value)
{
    if (!h || !key) return fail(SMF_ERR_ARG, "smf_set_param: NULL argument");
    int64_t *slot = nullptr;
    if (!strcmp(key, "relabel_period")) slot = &h->relabel_period;
    else if (!strcmp(key, "max_sweeps")) slot = &h->max_sweeps;
    else if (!strcmp(key, "poll_every")) slot = &h->poll_every;
    else if (!strcmp(key, "bfs_poll_every")) slot = &h->bfs_poll_every;
    else if (!strcmp(key, "gap_every")) {
        if (value < 0) return fail(SMF_ERR_ARG, "smf_set_param: gap_every must be >= 0");
        h->gap_every = value;
        return SMF_OK;
    }
    else if (!strcmp(key, "count_work")) {
        if (value != 0 && value != 1) return fail(SMF_ERR_ARG, "smf_set_param: count_work is 0 or 1");
        h->g.count_work = (int)value;
        return SMF_OK;
    }
    else if (!strcmp(key, "verbose")) {
        if (value != 0 && value != 1) return fail(SMF_ERR_ARG, "smf_set_param: verbose is 0 or 1");
        h->verbose = value;
        return SMF_OK;
    }
    else if (!strcmp(key, "bfs_early_stop")) {
        if (value != 0 && value != 1) return fail(SMF_ERR_ARG, "smf_set_param: bfs_early_stop is 0 or 1");
        h->bfs_early_stop = value;
        return SMF_OK;
    }
    else if (!strcmp(key, "kernel_timing")) {
        if (value < 0 || value >= (1 << KC_COUNT))
            return fail(SMF_ERR_ARG, "smf_set_param: kernel_timing is a mask of the kernel classes");
        h->timer.on = (unsigned)value;
        return SMF_OK;
    }
    if (!slot) return fail(SMF_ERR_ARG, std::string("smf_set_param: unknown key ") + key);
    if (value < 1) return fail(SMF_ERR_ARG, std::string("smf_set_param: ") + key + " must be >= 1");
    *slot = value;
    return SMF_OK;
}

extern "C" int smf_get_stat(const smf_handle *h, const char *key, int64_t *out)
{
    if (!h || !key || !out) return fail(SMF_ERR_ARG, "smf_get_stat: NULL argument");
    if (!strcmp(key, "sweeps")) *out = h->sweeps;
    else if (!strcmp(key, "global_relabels")) *out = h->global_relabels;
    else if (!strcmp(key, "bfs_passes")) *out = h->bfs_passes;
    else if (!strcmp(key, "mincut_passes")) *out = h->mincut_passes;
    else if (!strcmp(key, "gap_relabels")) *out = h->gap_relabels;
    else if (!strcmp(key, "gap_searches")) *out = h->gap_searches;
    else if (!strncmp(key, "bytes.", 6)) {
        // algorithmic bytes of the last solve per kernel class: counted on the
        // device for the data-dependent kernels, by formula for the others
        const char *name = key + 6;
        const int64_t N = h->g.N, P = h->g.P;
        if (!strcmp(name, "bfs")) *out = (int64_t)h->work_bytes[0];
        else if (!strcmp(name, "push")) *out = (int64_t)h->work_bytes[1];
        else if (!strcmp(name, "relabel")) *out = (int64_t)h->work_bytes[2];
        else if (!strcmp(name, "build")) *out = 36 * N + 4 * P;
        else if (!strcmp(name, "bfs_reset")) *out = h->global_relabels * (32 * N + 4 * N);
        else if (!strcmp(name, "finish")) *out = 4 * N + 8 * P;
        else if (!strcmp(name, "mincut")) *out = 4 * N + h->mincut_passes * 24 * P;
        else return fail(SMF_ERR_ARG, std::string("smf_get_stat: unknown kernel class in ") + key);
    }
    else if (!strncmp(key, "time_ns.", 8) || !strncmp(key, "launches.", 9)) {
        bool t = key[0] == 't';
        const char *name = key + (t ? 8 : 9);
        int kc = -1;
        for (int i = 0; i < KC_COUNT; ++i)
            if (!strcmp(name, kKClassName[i])) kc = i;
        if (kc < 0) return fail(SMF_ERR_ARG, std::string("smf_get_stat: unknown kernel class in ") + key);
        *out = t ? (int64_t)h->timer.ns[kc] : h->timer.launches[kc];
    }
    else return fail(SMF_ERR_ARG, std::string("smf_get_stat: unknown key ") + key);
    return SMF_OK;
}

extern "C" const char *smf_status_string(int status)
{
    switch (status) {
    case SMF_OK: return "ok";
    case SMF_ERR_ARG: return "invalid argument";
    case SMF_ERR_NOMEM: return "out of memory";
    case SMF_ERR_RANGE: return "value out of int32 range";
    case SMF_ERR_NOT_CONVERGED: return "not converged within the sweep cap";
    case SMF_ERR_HIP: return "HIP runtime error";
    case SMF_ERR_NOT_SOLVED: return "no successful solve";
    default: return "unknown status";
    }
}

extern "C" const char *smf_last_error(void) { return g_last_error.c_str(); }
