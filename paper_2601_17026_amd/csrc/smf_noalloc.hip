// Allocation-free solve of one volume: smf_solve_noalloc (include/smf.h).
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).  All
// solver state lives in one file-scope device array, `scratch`, of
// kNoAllocBytes bytes, which every GPU the library runs on holds until the
// process ends.  Host code never uses the array's name as an address: at the
// first call on a device the array's address on that device is looked up
// with hipGetSymbolAddress and kept per device, and only that address is
// handed to kernels.
//
// The kernels are those of smf_solve.  The host driver here runs the same
// method with the default schedule (sweeps of three push phases and one
// relabel phase, a global relabel every 2 sweeps, search levels polled every
// 16, early-stopping searches, one-block searches for small volumes) and no soft smoothness term; it reads the device counters
// with blocking copies into a stack buffer instead of pinned snapshots, so
// it uses no events and no pinned memory.  Every call on a GPU shares that
// GPU's array and leaves its contents behind; every word a solve reads is
// written by the solve first.  Calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <climits>

#include <atomic>
#include <cstdio>
#include <string>

#include "../../include/smf.h"
#include "smf_device.h"

namespace smf {
void launch_init_scratch(const Geom &g, Scratch *s, hipStream_t st);
void launch_set_int(int *p, int v, hipStream_t st);
void launch_fill(int *a, long long n, int v, hipStream_t st);
void launch_work_init(const Geom &g, const Work &a, const Work &b, hipStream_t st);
void launch_build(const int *cost, const Geom &g, const State &sv, Scratch *s, hipStream_t st);
void launch_bfs_begin(const Geom &g, hipStream_t st);
void launch_bfs_init(const Geom &g, const State &sv, int *T, int *LF, int c0, int c1, hipStream_t st);
void launch_bfs_level(const Geom &g, const State &sv, int L, const int *Tin, const int *LFin,
                      int *Tout, int *LFout, const LevelRanges &R, const Inst *single, hipStream_t st);
void launch_bfs_fixup(const Geom &g, const State &sv, int c0, int c1, hipStream_t st);
bool bfs_block_fits(const Geom &g);
void launch_bfs_block(const Geom &g, const State &sv, const int *T1, const int *LF1, int early_stop,
                      int max_level, int quorum, Scratch *s, hipStream_t st);
void launch_bfs_count(const Geom &g, const int *T, int slot, hipStream_t st);
void launch_push(const Geom &g, const State &sv, const Work &win, const Work &wout, Scratch *s,
                 bool down, hipStream_t st);
void launch_relabel(const Geom &g, const State &sv, const Work &win, const Work &wout, bool use_gap,
                    hipStream_t st);
void launch_compact(const Geom &g, const Work &w, int *next_count, hipStream_t st);
void launch_mincut_init(const Geom &g, const State &sv, int *H, hipStream_t st);
void launch_mincut_pass(const Geom &g, const State &sv, int *H, Scratch *s, hipStream_t st);
void launch_finish(const int *cost, const Geom &g, const State &sv, int *H, hipStream_t st);
int set_error_text(int code, const char *msg);
}  // namespace smf

using namespace smf;

constexpr size_t kNoAllocBytes = size_t(SMF_NOALLOC_MAX_BYTES);   // the workspace on every GPU used

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
constexpr int kPeriod = 2;             // sweeps between global relabels
constexpr int kPushPhases = 3;         // push phases per sweep
constexpr int kLevelsPerPoll = 16;     // search levels between host checks
constexpr long long kMaxSweeps = 2000000;
constexpr long long kMaxInstNodes = (1LL << 30) - 2;

// Address of `scratch` on each device, looked up at the first call there.
std::atomic<void *> g_scratch_ptr[kMaxDevices];

__global__ void k_store_inst(Inst *dst, Inst v) { *dst = v; }

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of the solver's arrays in the workspace for a volume of P
// columns, N nodes and nch 64-height chunks per column.
struct Layout {
    size_t cnt, inst, part, fill, col_inst, state, bfs, bits, work, wmask, wlist, end;
};

Layout layout_for(size_t P, size_t N, size_t nch)
{
    Layout l;
    size_t o = 0;
    auto take = [&o](size_t bytes) { const size_t at = o; o += up256(bytes ? bytes : 1); return at; };
    l.cnt = take(kScratchHead + sizeof(InstScratch));
    l.inst = take(sizeof(Inst));
    l.part = take(sizeof(int));
    l.fill = take(sizeof(int));
    l.col_inst = take(sizeof(int) * P);
    l.state = take(sizeof(int) * 8 * N);
    l.bfs = take(sizeof(int) * 12 * P);
    l.bits = take(sizeof(unsigned long long) * kMasks * nch * P);
    l.work = take(sizeof(unsigned long long) * 3 * kWorkSlots * kWorkStride);
    l.wmask = take(sizeof(unsigned long long) * 2 * P);
    l.wlist = take(sizeof(int) * 2 * P);
    l.end = o;
    return l;
}

int fail_hip(const char *what, hipError_t e)
{
    char msg[256];
    snprintf(msg, sizeof msg, "smf_solve_noalloc: %s: %s", what, hipGetErrorString(e));
    return set_error_text(SMF_ERR_HIP, msg);
}

#define NA_TRY(call)                                   \
    do {                                               \
        const hipError_t e_ = (call);                  \
        if (e_ != hipSuccess) return fail_hip(#call, e_); \
    } while (0)

// One solve's device arrays (all inside the workspace) and stream.
struct Run {
    Geom g{};
    State st{};
    Work work[2]{};
    Scratch *scr = nullptr;
    char *cnt = nullptr;
    int *fill = nullptr;
    int *T[2] = {};
    int *LF[2] = {};
    hipStream_t s = nullptr;
    long long N = 0;
    Inst I{};   // the volume (also handed to every level launch)
    // counters read by the last poll
    alignas(8) unsigned char snap[kScratchHead + sizeof(InstScratch)];
    const Scratch &host() const { return *reinterpret_cast<const Scratch *>(snap); }
    const InstScratch &inst() const { return *reinterpret_cast<const InstScratch *>(snap + kScratchHead); }
};

// Blocking read of the counters after all work enqueued so far; reports
// the error flags they carry.
int poll(Run &r)
{
    NA_TRY(hipGetLastError());
    NA_TRY(hipMemcpyAsync(r.snap, r.cnt, sizeof r.snap, hipMemcpyDeviceToHost, r.s));
    NA_TRY(hipStreamSynchronize(r.s));
    const int err = r.host().err;
    if (err & kErrCostRange) return set_error_text(SMF_ERR_RANGE, "smf_solve_noalloc: a cost lies outside (-2^30, 2^30)");
    if (err & kErrOverflow)
        return set_error_text(SMF_ERR_RANGE, "smf_solve_noalloc: an int32 excess or flow counter overflowed");
    if (err & kErrSearch)
        return set_error_text(SMF_ERR_NOT_CONVERGED, "smf_solve_noalloc: breadth-first search did not settle");
    return SMF_OK;
}

// Global relabel (reverse breadth-first search from t, Section 2.1 and
// Section 3.2.2): level 1 from the sink arcs, then levels until one labels
// nothing (unreached nodes get kInf) or every node with excess is labelled
// (unreached nodes get the first level not run, a valid lower bound).
int search(Run &r)
{
    const Geom &g = r.g;
    const int P = g.Ptot;
    launch_bfs_begin(g, r.s);
    launch_set_int(g.short_count, 0, r.s);
    launch_bfs_init(g, r.st, r.T[1], r.LF[1], 0, P, r.s);   // level 1 lives in buffer 1
    if (bfs_block_fits(g)) {
        launch_bfs_block(g, r.st, r.T[1], r.LF[1], 1, (int)(r.N + 2), INT_MAX, r.scr, r.s);   // one volume: no quorum
        NA_TRY(hipGetLastError());
        return SMF_OK;
    }
    LevelRanges R{};
    R.n = 1;
    R.lo[0] = 0;
    R.pre[0] = 0;
    R.pre[1] = P;
    int L = 1, cur = 1, fill = kInf;
    for (int npoll = 0;; ++npoll) {
        for (int i = 0; i < kLevelsPerPoll; ++i, ++L, cur ^= 1)
            launch_bfs_level(g, r.st, L, r.T[cur], r.LF[cur], r.T[cur ^ 1], r.LF[cur ^ 1], R, &r.I, r.s);
        launch_bfs_count(g, r.T[cur], npoll & 1, r.s);
        const int rc = poll(r);
        if (rc) return rc;
        // levels 1 .. L-1 have run: labels up to L are written
        const bool complete = !r.inst().lvl_changed[(L - 1) % kLvlSlots];
        const bool labelled = r.inst().bfs_unsat[npoll & 1] == 0;
        if (complete || labelled) {
            fill = complete ? kInf : L + 1;
            break;
        }
        if ((long long)L > r.N + 2 + 2 * kLevelsPerPoll)
            return set_error_text(SMF_ERR_NOT_CONVERGED, "smf_solve_noalloc: breadth-first search did not settle");
    }
    launch_set_int(r.fill, fill, r.s);
    launch_bfs_fixup(g, r.st, 0, P, r.s);
    NA_TRY(hipGetLastError());
    return SMF_OK;
}

int solve(Run &r, const int32_t *cost, int32_t *surface, int64_t *flow_out, int64_t *energy_out)
{
    const Geom &g = r.g;
    launch_init_scratch(g, r.scr, r.s);
    launch_build(cost, g, r.st, r.scr, r.s);
    int rc = search(r);
    if (rc) return rc;
    launch_work_init(g, r.work[0], r.work[1], r.s);
    int since = 0, cur = 0;
    long long pushes = 0;
    for (long long sweeps = 0;; ++sweeps) {
        if (sweeps >= kMaxSweeps) return set_error_text(SMF_ERR_NOT_CONVERGED, "smf_solve_noalloc: sweep cap reached");
        if (since >= kPeriod) {
            rc = search(r);
            if (rc) return rc;
            since = 0;
        }
        // push phases (labels fixed), each followed by the list of the
        // columns it marked, then relabel (flows fixed); the lists alternate
        int a = cur;
        for (int j = 0; j < kPushPhases; ++j, a ^= 1) {
            launch_push(g, r.st, r.work[a], r.work[a ^ 1], r.scr, (pushes++ & 1) == 0, r.s);
            launch_compact(g, r.work[a ^ 1], r.work[a].count, r.s);
        }
        launch_relabel(g, r.st, r.work[a], r.work[a ^ 1], false, r.s);
        cur = a ^ 1;
        ++since;
        rc = poll(r);
        if (rc) return rc;
        if (r.inst().active == 0) break;   // a maximum preflow
    }
    // minimum cut: residual reach of the nodes that keep excess
    launch_mincut_init(g, r.st, surface, r.s);
    for (long long pass = 0;; ++pass) {
        launch_set_int(&r.scr->changed, 0, r.s);
        launch_mincut_pass(g, r.st, surface, r.scr, r.s);
        rc = poll(r);
        if (rc) return rc;
        if (!r.host().changed) break;
        if (pass > r.N + 2)
            return set_error_text(SMF_ERR_NOT_CONVERGED, "smf_solve_noalloc: minimum-cut search did not settle");
    }
    launch_finish(cost, g, r.st, surface, r.s);
    rc = poll(r);
    if (rc) return rc;
    *flow_out = r.inst().flow;
    *energy_out = r.inst().energy;
    return SMF_OK;
}

}  // namespace

extern "C" int smf_solve_noalloc(const int32_t *cost_dev, int32_t nx, int32_t ny, int32_t K, int32_t delta,
                                 int32_t *surface_dev, int64_t *flow_out, int64_t *energy_out, void *stream)
{
    if (!cost_dev || !surface_dev || !flow_out || !energy_out)
        return set_error_text(SMF_ERR_ARG, "smf_solve_noalloc: NULL argument");
    if (nx < 1 || ny < 1 || K < 1 || delta < 0)
        return set_error_text(SMF_ERR_ARG, "smf_solve_noalloc: need nx, ny, K >= 1 and delta >= 0");
    const long long P = (long long)nx * ny, N = P * K;
    if (N > kMaxInstNodes) return set_error_text(SMF_ERR_RANGE, "smf_solve_noalloc: nx*ny*K above 2^30 - 2");
    const int nch = (K + kWave - 1) / kWave;
    const Layout l = layout_for((size_t)P, (size_t)N, (size_t)nch);
    if (l.end > kNoAllocBytes) {
        char msg[200];
        snprintf(msg, sizeof msg,
                 "smf_solve_noalloc: the volume needs %zu bytes of solver state, more than the "
                 "%zu-byte static workspace", l.end, kNoAllocBytes);
        return set_error_text(SMF_ERR_NOMEM, msg);
    }
    int dev = 0;
    NA_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return set_error_text(SMF_ERR_ARG, "smf_solve_noalloc: device index above 63");
    void *ws = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!ws) {
        // set-up on this device: the array's address here, looked up once
        NA_TRY(hipGetSymbolAddress(&ws, HIP_SYMBOL(scratch)));
        if (!ws) return set_error_text(SMF_ERR_HIP, "smf_solve_noalloc: no address for the static workspace");
        g_scratch_ptr[dev].store(ws, std::memory_order_release);
    }
    char *base = static_cast<char *>(ws);

    Run r;
    r.s = (hipStream_t)stream;
    r.N = N;
    Inst &I = r.I;
    I.nx = nx; I.ny = ny; I.K = K; I.delta = delta;
    I.P = (int)P;
    I.nch = nch;
    I.cpb = (nch + 63) / 64;
    I.lab_cap = (int)(N + 1);
    I.col_base = 0;
    I.alpha = 0;
    I.node_base = 0;
    I.cost_base = 0;
    I.N = N;
    r.cnt = base + l.cnt;
    r.scr = reinterpret_cast<Scratch *>(r.cnt);
    r.fill = reinterpret_cast<int *>(base + l.fill);
    int *part = reinterpret_cast<int *>(base + l.part);
    int *col_inst = reinterpret_cast<int *>(base + l.col_inst);
    int *bfs = reinterpret_cast<int *>(base + l.bfs);
    Geom &g = r.g;
    g.n = 1;
    g.Ptot = (int)P;
    g.Ntot = N;
    g.inst = reinterpret_cast<Inst *>(base + l.inst);
    g.col_inst = col_inst;
    g.is = reinterpret_cast<InstScratch *>(r.cnt + kScratchHead);
    g.part = part;
    g.fill = r.fill;
    g.count_work = 0;
    g.work = reinterpret_cast<unsigned long long *>(base + l.work);
    g.hist = nullptr;
    g.hist_len = 0;
    g.bits = reinterpret_cast<unsigned long long *>(base + l.bits);
    g.max_nch = nch;
    g.max_cols = (int)P;
    g.max_chunks = (long long)P * nch;
    g.sbits = nullptr;
    g.soft = 0;
    g.low_act = bfs + 10 * P;
    g.short_list = bfs + 11 * P;
    g.short_count = &r.scr->short_count;
    g.level_block = 256;
    g.sweep_waves = 8192;
    int *sv = reinterpret_cast<int *>(base + l.state);
    r.st.e = sv;
    r.st.d = sv + N;
    r.st.ts = sv + 2 * N;
    r.st.fd = sv + 3 * N;
    r.st.fl = sv + 4 * N;
    r.st.sf = nullptr;
    auto *wmask = reinterpret_cast<unsigned long long *>(base + l.wmask);
    int *wlist = reinterpret_cast<int *>(base + l.wlist);
    for (int i = 0; i < 2; ++i) {
        r.work[i].mask = wmask + (size_t)i * P;
        r.work[i].list = wlist + (size_t)i * P;
        r.work[i].count = &r.scr->count[i];
    }
    r.T[0] = bfs;
    r.LF[0] = bfs + P;
    r.T[1] = bfs + 5 * P;
    r.LF[1] = bfs + 6 * P;

    // the volume table, the column -> volume map and the search flags are
    // written by kernels (no host buffer has to outlive an asynchronous copy)
    hipLaunchKernelGGL(k_store_inst, dim3(1), dim3(1), 0, r.s, const_cast<Inst *>(g.inst), I);
    launch_fill(col_inst, P, 0, r.s);
    launch_set_int(part, 1, r.s);
    const int rc = solve(r, cost_dev, surface_dev, flow_out, energy_out);
    if (rc != SMF_OK) (void)hipStreamSynchronize(r.s);   // nothing left in flight on failure
    return rc;
}
