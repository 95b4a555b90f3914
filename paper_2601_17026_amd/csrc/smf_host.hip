// Host driver and C-ABI of the exact surface max-flow (include/smf.h).
//
// A handle owns the node state of a batch of n volumes (n = 1 for the plain
// entry points): 32 bytes per node, packed volume after volume in each
// volume's own [nx][ny][K] layout, plus per-column work lists and BFS
// records, the volume table, per-volume counters and their pinned host
// mirror.  A solve enqueues the build, the initial global relabel and then
// sweeps of push and relabel phases on the caller's stream, every launch
// covering all volumes.  The host polls the per-volume active-node counters
// every `poll_every` sweeps (the only device-to-host traffic of the loop)
// and runs a global relabel for the volumes whose relabel period has come
// round.  Termination: no node with excess and a finite label remains in
// any volume (Section 3.2.4 decides this with flags and locks across
// threads; here it is one counter per volume written by the relabel phase).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/smf.h"
#include "level_cover.h"
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
void launch_gap_find(const Geom &g, const State &sv, long long max_inst_nodes, hipStream_t st);
void launch_mincut_init(const Geom &g, const State &sv, int *H, hipStream_t st);
void launch_hmax(const Geom &g, const State &sv, int *Hmax, hipStream_t st);
void launch_mincut_pass(const Geom &g, const State &sv, int *H, Scratch *s, hipStream_t st);
void launch_finish(const int *cost, const Geom &g, const State &sv, int *H, hipStream_t st);
}  // namespace smf

using namespace smf;

// Text of the last failure on this host thread, kept in a fixed buffer so
// that recording a failure allocates nothing (longer texts are cut).
constexpr size_t kErrLen = 512;
static thread_local char g_last_error[kErrLen];

static int fail_text(int code, const char *msg)
{
    size_t i = 0;
    for (; msg && msg[i] && i + 1 < kErrLen; ++i) g_last_error[i] = msg[i];
    g_last_error[i] = 0;
    return code;
}

static int fail(int code, const std::string &msg) { return fail_text(code, msg.c_str()); }

namespace smf {
// Records the failure of an entry point defined in another source file.
int set_error(int code, const std::string &msg) { return fail(code, msg); }
int set_error_text(int code, const char *msg) { return fail_text(code, msg); }
void clear_error() { g_last_error[0] = 0; }
}  // namespace smf

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
    // Adds the brackets whose end event has completed; the others stay
    // pending (work may still be in flight behind a host poll).
    void collect()
    {
        size_t keep = 0;
        for (auto &p : pending) {
            if (hipEventQuery(p.b) != hipSuccess) {
                pending[keep++] = p;
                continue;
            }
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                ns[p.kc] += 1e6 * (double)ms;
                launches[p.kc] += p.n;
            }
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.resize(keep);
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

constexpr int kHistLen = 4096;            // labels tracked by the gap heuristic (LDS bins)
constexpr int kSlotSweep = 0, kSlotBfs = 2, kSlotSync = 4, kSnapSlots = 5;
constexpr long long kMaxInstNodes = (1LL << 30) - 2;   // finite labels stay below kUnl
constexpr int64_t kMaxAlpha = 1LL << 29;   // soft residuals alpha - f + f' stay below 2^31

struct smf_handle {
    Geom g{};
    int device = 0;
    int cus = 0;                  // compute units of the device
    int n = 0;
    std::vector<Inst> inst;       // host copy of the volume table
    long long max_inst_nodes = 0;
    // device memory
    Inst *inst_dev = nullptr;
    int *col_inst = nullptr;      // Ptot
    char *cnt_dev = nullptr;      // Scratch, then n InstScratch (kScratchHead offset)
    InstScratch *is_dev = nullptr;
    int *part_dev = nullptr;      // n: volume takes part in the running global relabel
    int *fill_dev = nullptr;      // n: fixup label of the running global relabel (-1: none)
    int *state = nullptr;         // 8 * Ntot int32
    int *H = nullptr;             // Ptot int32 surfaces
    int *Hmax = nullptr;          // Ptot int32 highest optimal surfaces (param hmax)
    int *bfs = nullptr;           // 12 * Ptot int32: two per-column BFS records (threshold word,
                                  // LF[4]), the lowest active heights and the short-column list
    unsigned long long *bits = nullptr;   // kMasks * max_nch * Ptot BFS bit-mask words
    int *soft_flow = nullptr;             // 4 * Ntot soft-arc flows, once some alpha > 0
    unsigned long long *sbits = nullptr;  // 4 * max_nch * Ptot soft-arc masks, likewise
    int *band_dev = nullptr;              // 3 * Ptot: lowest height, extent, cost shift per column
    unsigned long long *wcount = nullptr; // algorithmic byte counters (Geom::work)
    int *hist = nullptr;                  // n x kHistLen label histograms (Geom::hist)
    unsigned long long *wmask = nullptr;  // 2 * Ptot work masks
    int *wlist = nullptr;                 // 2 * Ptot work-list entries
    Scratch *scr = nullptr;
    // pinned host memory; each upload area is rewritten only after a stream
    // synchronisation that follows its previous upload.  Counter snapshots
    // go to five slots: the sweep loop and the BFS loop each alternate
    // between two (kSlotSweep, kSlotBfs) while the host polls one batch of
    // work behind the device, and kSlotSync serves blocking reads; `host`
    // and `is_host` point at the slot read last.
    Scratch *host_buf[kSnapSlots] = {};
    InstScratch *is_buf[kSnapSlots] = {};
    hipEvent_t snap_ev[kSnapSlots] = {};
    Scratch *host = nullptr;
    InstScratch *is_host = nullptr;
    Inst *inst_up = nullptr;      // volume table upload
    int *part_up = nullptr;       // n
    int *fill_up = nullptr;       // n
    State st{};
    Work work[2]{};               // each phase reads one and fills the other (cur_work)
    unsigned long long work_bytes[3] = {};  // device byte counters after the last solve
    // parameters
    int64_t relabel_period = 2;
    std::vector<int64_t> inst_period;       // per volume; 0: relabel_period
    int64_t max_sweeps = 2000000;
    int64_t poll_every = 1;
    int64_t bfs_poll_every = 16;
    int64_t bfs_early_stop = 1;
    int64_t block_search = 1;      // small volumes: each whole search in one block per volume
    int64_t verbose = 0;           // 1: progress lines on stderr
    int64_t gap_every = 0;         // sweeps between gap searches (0: off)
    int64_t want_hmax = 0;         // 1: also read out the highest optimal surface
    int64_t push_phases = 3;       // push phases per sweep (one relabel phase)
    int64_t search_quorum = 90;    // a batch search ends once this percentage of its volumes ended
    int cur_work = 0;              // work[cur_work] holds the columns of the next push phase
    bool hmax_ready = false;       // the last solve computed Hmax

    // results and counters of the last solve
    bool solved = false;
    std::vector<int64_t> flow, energy, inst_sweeps, inst_relabels, inst_gap;
    int64_t pushes = 0;            // push phases of the running solve
    int64_t sweeps = 0, global_relabels = 0, bfs_passes = 0, mincut_passes = 0, gap_relabels = 0;
    int64_t gap_searches = 0;
    int64_t reset_nodes = 0;       // nodes swept by level-1 passes and fixups
    int64_t reset_chunks = 0;      // their 64-height chunks (five mask words, one low-active word per column)
    KernelTimer timer;
};

static void release(smf_handle *h)
{
    if (!h) return;
    void *dev[] = {h->inst_dev, h->col_inst, h->cnt_dev, h->part_dev, h->fill_dev, h->state, h->H,
                   h->bfs, h->bits, h->wcount, h->hist, h->wmask, h->wlist, h->soft_flow, h->sbits,
                   h->band_dev, h->Hmax};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    for (int i = 0; i < kSnapSlots; ++i)
        if (h->snap_ev[i]) (void)hipEventSynchronize(h->snap_ev[i]);
    for (int i = 0; i < kSnapSlots; ++i) {
        if (h->host_buf[i]) (void)hipHostFree(h->host_buf[i]);
        if (h->snap_ev[i]) (void)hipEventDestroy(h->snap_ev[i]);
    }
    void *pinned[] = {h->inst_up, h->part_up, h->fill_up};
    for (void *p : pinned)
        if (p) (void)hipHostFree(p);
    delete h;
}

template <typename T>
static bool dev_alloc(T *&p, size_t count)
{
    return hipMalloc((void **)&p, sizeof(T) * (count ? count : 1)) == hipSuccess;
}

template <typename T>
static bool host_alloc(T *&p, size_t count)
{
    return hipHostMalloc((void **)&p, sizeof(T) * (count ? count : 1), hipHostMallocDefault) == hipSuccess;
}

// Bytes of the counter block: Scratch, then the per-volume counters.
static size_t counter_bytes(int n) { return kScratchHead + sizeof(InstScratch) * (size_t)n; }

static bool alloc_snapshots(smf_handle *h)
{
    for (int i = 0; i < kSnapSlots; ++i) {
        char *b = nullptr;
        if (!host_alloc(b, counter_bytes(h->n)) ||
            hipEventCreateWithFlags(&h->snap_ev[i], hipEventDisableTiming) != hipSuccess) {
            if (b) h->host_buf[i] = (Scratch *)b;
            return false;
        }
        h->host_buf[i] = (Scratch *)b;
        h->is_buf[i] = (InstScratch *)(b + kScratchHead);
    }
    return true;
}

extern "C" smf_handle *smf_batch_create(int32_t n, const int32_t *nx, const int32_t *ny,
                                        const int32_t *K, const int32_t *delta)
{
    g_last_error[0] = 0;
    if (n < 1 || !nx || !ny || !K || !delta) {
        fail(SMF_ERR_ARG, "smf_batch_create: need n >= 1 and non-NULL shape arrays");
        return nullptr;
    }
    std::vector<Inst> inst((size_t)n);
    long long Ptot = 0, Ntot = 0, max_nodes = 0;
    int max_nch = 1;
    for (int i = 0; i < n; ++i) {
        if (nx[i] < 1 || ny[i] < 1 || K[i] < 1 || delta[i] < 0) {
            fail(SMF_ERR_ARG, "smf_batch_create: volume " + std::to_string(i) +
                                  " needs nx, ny, K >= 1 and delta >= 0");
            return nullptr;
        }
        const long long P = (long long)nx[i] * ny[i];
        const long long N = P * K[i];
        if (N > kMaxInstNodes) {
            fail(SMF_ERR_RANGE, "smf_batch_create: volume " + std::to_string(i) +
                                    " has nx*ny*K above 2^30 - 2");
            return nullptr;
        }
        Inst &I = inst[i];
        I.nx = nx[i]; I.ny = ny[i]; I.K = K[i]; I.delta = delta[i];
        I.P = (int)P;
        I.nch = (K[i] + kWave - 1) / kWave;
        I.cpb = (I.nch + 63) / 64;
        I.lab_cap = (int)(N + 1);
        I.col_base = (int)Ptot;
        I.alpha = 0;
        I.node_base = Ntot;
        I.cost_base = Ntot;
        I.N = N;
        Ptot += P;
        Ntot += N;
        max_nodes = std::max(max_nodes, N);
        max_nch = std::max(max_nch, I.nch);
        if (Ptot >= (1LL << 31)) {
            fail(SMF_ERR_RANGE, "smf_batch_create: more than 2^31 - 1 columns in the batch");
            return nullptr;
        }
    }
    // device memory of the handle (the allocations below), checked against
    // the caller's budget before anything is allocated
    const size_t need = sizeof(Inst) * (size_t)n + sizeof(int) * (size_t)Ptot + counter_bytes(n) +
                        2 * sizeof(int) * (size_t)n + sizeof(int) * 8 * (size_t)Ntot +
                        sizeof(int) * (size_t)Ptot + sizeof(int) * 12 * (size_t)Ptot +
                        sizeof(unsigned long long) * kMasks * (size_t)max_nch * (size_t)Ptot +
                        sizeof(unsigned long long) * 3 * kWorkSlots * kWorkStride +
                        sizeof(int) * (size_t)n * kHistLen + sizeof(unsigned long long) * 2 * (size_t)Ptot +
                        sizeof(int) * 2 * (size_t)Ptot;
    if (const char *lim = getenv("SMF_DEVICE_MEM_LIMIT")) {
        char *end = nullptr;
        const unsigned long long cap = strtoull(lim, &end, 10);
        if (end != lim && need > cap) {
            fail(SMF_ERR_NOMEM, "smf_batch_create: the handle needs " + std::to_string(need) +
                                    " bytes of device memory, more than SMF_DEVICE_MEM_LIMIT = " +
                                    std::to_string(cap));
            return nullptr;
        }
    }
    smf_handle *h = new (std::nothrow) smf_handle;
    if (!h) {
        fail(SMF_ERR_NOMEM, "smf_batch_create: host allocation failed");
        return nullptr;
    }
    h->n = n;
    h->inst = inst;
    h->max_inst_nodes = max_nodes;
    h->inst_period.assign((size_t)n, 0);
    const size_t P = (size_t)Ptot, N = (size_t)Ntot;
    const hipError_t dev_err = hipGetDevice(&h->device);
    if (dev_err != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        fail(SMF_ERR_HIP, std::string("smf_batch_create: no usable HIP device: ") + hipGetErrorString(dev_err));
        return nullptr;
    }
    if (hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) {
        (void)hipGetLastError();
        h->cus = 0;   // no quorum in block searches
    }
    if (!dev_alloc(h->inst_dev, n) ||
        !dev_alloc(h->col_inst, P) || !dev_alloc(h->cnt_dev, counter_bytes(n)) || !dev_alloc(h->part_dev, n) ||
        !dev_alloc(h->fill_dev, n) || !dev_alloc(h->state, 8 * N) || !dev_alloc(h->H, P) ||
        !dev_alloc(h->bfs, 12 * P) || !dev_alloc(h->bits, (size_t)kMasks * max_nch * P) ||
        !dev_alloc(h->wcount, 3 * kWorkSlots * kWorkStride) ||
        !dev_alloc(h->hist, (size_t)n * kHistLen) || !dev_alloc(h->wmask, 2 * P) ||
        !dev_alloc(h->wlist, 2 * P) || !host_alloc(h->inst_up, n) ||
        !host_alloc(h->part_up, n) || !host_alloc(h->fill_up, n) || !alloc_snapshots(h)) {
        (void)hipGetLastError();
        release(h);
        fail(SMF_ERR_NOMEM, "smf_batch_create: device allocation of " +
                                std::to_string(32.0 * (double)Ntot / (1 << 20)) + " MiB failed");
        return nullptr;
    }
    // the volume table and the column -> volume map are uploaded once
    std::vector<int> ci(P);
    for (int i = 0; i < n; ++i)
        std::fill(ci.begin() + inst[i].col_base, ci.begin() + inst[i].col_base + inst[i].P, i);
    if (hipMemcpy(h->inst_dev, inst.data(), sizeof(Inst) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->col_inst, ci.data(), sizeof(int) * P, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        release(h);
        fail(SMF_ERR_HIP, "smf_batch_create: upload of the volume table failed");
        return nullptr;
    }
    h->scr = (Scratch *)h->cnt_dev;
    h->is_dev = (InstScratch *)(h->cnt_dev + kScratchHead);
    Geom &g = h->g;
    g.n = n;
    g.Ptot = (int)Ptot;
    g.Ntot = Ntot;
    g.inst = h->inst_dev;
    g.col_inst = h->col_inst;
    g.is = h->is_dev;
    g.part = h->part_dev;
    g.fill = h->fill_dev;
    g.count_work = 0;
    g.work = h->wcount;
    g.hist = h->hist;
    g.hist_len = kHistLen;
    g.bits = h->bits;
    g.max_nch = max_nch;
    g.max_cols = 0;
    g.max_chunks = 0;
    for (int i = 0; i < n; ++i) {
        g.max_cols = std::max(g.max_cols, inst[i].P);
        g.max_chunks = std::max(g.max_chunks, (long long)inst[i].P * inst[i].nch);
    }
    g.level_block = 256;
    g.sweep_waves = 8192;
    g.soft = 0;
    g.sbits = nullptr;
    g.band = 0;
    g.blo = g.bext = g.bcs = nullptr;
    h->st.sf = nullptr;
    g.low_act = h->bfs + 10 * P;
    g.short_list = h->bfs + 11 * P;
    g.short_count = &h->scr->short_count;
    int *b = h->state;
    h->st.e = b;
    h->st.d = b + N;
    h->st.ts = b + 2 * N;
    h->st.fd = b + 3 * N;
    h->st.fl = b + 4 * N;
    for (int i = 0; i < 2; ++i) {
        h->work[i].mask = h->wmask + (size_t)i * P;
        h->work[i].list = h->wlist + (size_t)i * P;
        h->work[i].count = &h->scr->count[i];
    }
    return h;
}

extern "C" smf_handle *smf_create(int32_t nx, int32_t ny, int32_t K, int32_t delta)
{
    return smf_batch_create(1, &nx, &ny, &K, &delta);
}

extern "C" void smf_destroy(smf_handle *h) { release(h); }

// Enqueues a snapshot of the batch-wide and per-volume counters into pinned
// slot `slot`, taken in stream order after the work enqueued so far.
static int post_snapshot(smf_handle *h, hipStream_t s, int slot)
{
    HIP_TRY(hipMemcpyAsync(h->host_buf[slot], h->cnt_dev, counter_bytes(h->n), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(h->snap_ev[slot], s));
    return SMF_OK;
}

// Waits for the snapshot in `slot` and makes it the one `host` / `is_host`
// show; reports the error flags it carries.
static int wait_snapshot(smf_handle *h, int slot)
{
    HIP_TRY(hipEventSynchronize(h->snap_ev[slot]));
    h->host = h->host_buf[slot];
    h->is_host = h->is_buf[slot];
    h->timer.collect();
    if (h->host->err & kErrCostRange)
        return fail(SMF_ERR_RANGE, "smf_solve: a cost lies outside (-2^30, 2^30)");
    if (h->host->err & kErrOverflow)
        return fail(SMF_ERR_RANGE, "smf_solve: an int32 excess or flow counter overflowed");
    if (h->host->err & kErrSearch)
        return fail(SMF_ERR_NOT_CONVERGED, "smf_solve: breadth-first search did not settle");
    return SMF_OK;
}

// Blocking read of the counters after all work enqueued so far.
static int sync_scratch(smf_handle *h, hipStream_t s)
{
    int rc = post_snapshot(h, s, kSlotSync);
    return rc ? rc : wait_snapshot(h, kSlotSync);
}

// Global relabel of the volumes with part[i]: level 1 from the sink arcs,
// then one launch per BFS level (covering every taking-part volume) until
// each of them has either run to completion -- a level labelled nothing:
// exact distances, unreached nodes get kInf -- or, with bfs_early_stop, has
// labelled every node that holds excess (unreached nodes then get the first
// unfinished level, a valid lower bound).  The host checks every
// bfs_poll_every levels; levels launched after a volume's last productive
// one are no-ops for it.
// Chooses the volumes, and so the column ranges, that the next levels of a
// search cover (every live volume, `cover` only shrinking; level_cover.h).
// False if more than kMaxRanges ranges would be needed, which the rules of
// the choice exclude.
static bool shrink_cover(const smf_handle *h, const std::vector<char> &live, std::vector<char> &cover,
                         LevelRanges &R)
{
    const int nr = cover_ranges(
        h->n, [h](int i) { return h->inst[i].col_base; }, [h](int i) { return h->inst[i].P; }, live,
        cover, kMaxRanges, R.lo, R.pre);
    if (nr < 0) return false;
    R.n = nr;
    return true;
}

// One global relabel (reverse breadth-first search from t) of the volumes
// with part[i], as a resumable state on one stream: begin() enqueues level 1
// (or, for small volumes, each whole search in one block), step() the
// next batch of bfs_poll_every levels with the early-stop count and a
// counter snapshot, examine() reads the oldest snapshot in flight and
// decides which volumes' searches have ended, and finish() enqueues the
// fix-up.  A volume's search ends when a level labelled nothing in it (exact
// distances: unreached nodes get kInf) or, with early stop, when every node
// holding excess is labelled (unreached nodes get the first level not run, a
// valid lower bound).  The host reads the counters one batch of levels
// behind the device, so the device never waits for the host; levels after a
// volume's search ended are no-ops for it, or label more nodes exactly.
struct Search {
    smf_handle *h = nullptr;
    hipStream_t s = nullptr;
    int64_t early_stop = 0;
    std::vector<char> part, live, cover;
    std::vector<int> fill_out;
    LevelRanges R{};
    int c0 = 0, c1 = 0;
    int L = 1, cur = 1, slot = 0, npoll = 0, inflight = 0;
    int Lsnap[2] = {0, 0}, Csnap[2] = {0, 0};
    bool whole = false;   // nothing to do, or the one-block search already ran
    bool exact = false;   // a complete search: no early stop and no quorum
    int *T[2] = {}, *LF[2] = {};

    int begin(smf_handle *hh, hipStream_t ss, const std::vector<char> &p, bool complete)
    {
        h = hh;
        s = ss;
        const int n = h->n;
        // a complete search runs until a level labels nothing, whatever
        // bfs_early_stop says
        early_stop = complete ? 0 : h->bfs_early_stop;
        exact = complete;
        const size_t P = (size_t)h->g.Ptot;
        T[0] = h->bfs;
        T[1] = h->bfs + 5 * P;
        LF[0] = h->bfs + P;
        LF[1] = h->bfs + 6 * P;
        part = p;
        L = 1;
        cur = 1;
        slot = 0;
        npoll = 0;
        inflight = 0;
        whole = false;
        // the launches cover the columns [c0, c1) spanned by the volumes that
        // take part (volumes are packed in order)
        c0 = h->g.Ptot;
        c1 = 0;
        for (int i = 0; i < n; ++i) {
            h->part_up[i] = part[i] ? 1 : 0;
            if (part[i]) {
                h->reset_nodes += h->inst[i].N;
                h->reset_chunks += (int64_t)h->inst[i].P * h->inst[i].nch;
                c0 = std::min(c0, h->inst[i].col_base);
                c1 = std::max(c1, h->inst[i].col_base + h->inst[i].P);
            }
        }
        if (c0 >= c1) {
            whole = true;
            return SMF_OK;
        }
        // The levels cover the volumes of [c0, c1) that take part (others
        // only where more than kMaxRanges column ranges would be needed); a
        // volume whose search has ended drops out of the later levels, with
        // its fill label fixed when it leaves (fill_out).
        live.assign(part.begin(), part.end());
        cover.assign((size_t)n, 0);
        fill_out.assign((size_t)n, -1);
        for (int i = 0; i < n; ++i)
            cover[i] = h->inst[i].col_base >= c0 && h->inst[i].col_base < c1;
        if (!shrink_cover(h, live, cover, R))
            return fail(SMF_ERR_HIP, "smf_solve: internal error in the level ranges");
        HIP_TRY(hipMemcpyAsync(h->part_dev, h->part_up, sizeof(int) * n, hipMemcpyHostToDevice, s));
        launch_bfs_begin(h->g, s);
        launch_set_int(&h->scr->short_count, 0, s);
        {
            TimedScope ts(h->timer, KC_BFS_RESET, s);
            launch_bfs_init(h->g, h->st, T[1], LF[1], c0, c1, s);   // level 1 lives in buffer 1
        }
        if (h->block_search && bfs_block_fits(h->g)) {
            // small volumes: each volume's whole search in one block, no polls
            {
                TimedScope ts(h->timer, KC_BFS, s);
                // the quorum rule of batch searches: the blocks stop once
                // that many volumes' searches have ended
                int npart = 0;
                for (int i = 0; i < n; ++i) npart += part[i] ? 1 : 0;
                // (only while every volume's block can be resident at once:
                // a block that starts after the quorum would stop at once)
                const int quorum = !exact && npart > 1 && npart <= h->cus
                                       ? std::max<int>(1, (int)((h->search_quorum * npart + 99) / 100))
                                       : INT_MAX;
                launch_set_int(&h->scr->block_done, 0, s);
                launch_bfs_block(h->g, h->st, T[1], LF[1], (int)early_stop,
                                 (int)std::min<int64_t>(h->max_inst_nodes + 2, INT32_MAX), quorum, h->scr, s);
            }
            HIP_TRY(hipGetLastError());
            whole = true;
        }
        return SMF_OK;
    }

    // Enqueues the next batch of levels, the early-stop count and a snapshot.
    int step()
    {
        const int n = h->n;
        {
            // cur: the record buffer that holds every column's record of level L
            TimedScope ts(h->timer, KC_BFS, s, (int)h->bfs_poll_every);
            for (int64_t i = 0; i < h->bfs_poll_every; ++i, ++L, cur ^= 1) {
                launch_bfs_level(h->g, h->st, L, T[cur], LF[cur], T[cur ^ 1], LF[cur ^ 1], R,
                                 n == 1 ? &h->inst[0] : nullptr, s);
                h->bfs_passes++;
            }
        }
        // this poll's count goes to bfs_unsat[npoll & 1]
        if (early_stop) launch_bfs_count(h->g, T[cur], npoll & 1, s);
        HIP_TRY(hipGetLastError());
        const int sl = (slot + inflight) & 1;
        const int rc = post_snapshot(h, s, kSlotBfs + sl);
        if (rc) return rc;
        Lsnap[sl] = L;
        Csnap[sl] = npoll++ & 1;
        ++inflight;
        // every productive level lowers at least one threshold by >= 1
        if ((int64_t)L > h->max_inst_nodes + 2 + 2 * h->bfs_poll_every)
            return fail(SMF_ERR_NOT_CONVERGED, "smf_solve: breadth-first search did not settle");
        return SMF_OK;
    }

    // The oldest snapshot in flight is complete (hipEventQuery).
    bool ready() const { return inflight > 0 && hipEventQuery(h->snap_ev[kSlotBfs + slot]) == hipSuccess; }

    // Waits for the oldest snapshot in flight and decides which volumes'
    // searches have ended; all: every volume's search has ended (the fill
    // labels are then set in fill_up).
    int examine(bool &all)
    {
        const int n = h->n;
        all = false;
        const int rc = wait_snapshot(h, kSlotBfs + slot);
        if (rc) return rc;
        // at that snapshot the last level launched had produced level Lp
        const int Lp = Lsnap[slot], cslot = Csnap[slot];
        slot ^= 1;
        --inflight;
        bool ended = false;
        all = true;
        int nlive = 0, npart = 0;
        for (int i = 0; i < n; ++i) {
            npart += part[i] ? 1 : 0;
            if (!live[i]) continue;
            const InstScratch &r = h->is_host[i];
            const bool complete = !r.lvl_changed[(Lp - 1) % kLvlSlots];
            const bool labelled = early_stop && r.bfs_unsat[cslot] == 0;
            if (complete || labelled) {
                live[i] = 0;
                ended = true;
                // levels < L have run over it: unreached nodes are > L away
                fill_out[i] = complete ? kInf : L + 1;
            } else {
                all = false;
                ++nlive;
            }
        }
        // the volumes still searching when the quorum has ended take the
        // first level not run as their fill label, a valid lower bound (not
        // in a complete search, whose unreached nodes must be exactly those
        // that cannot reach t)
        if (!exact && !all && 100 * (int64_t)(npart - nlive) >= h->search_quorum * npart) all = true;
        if (all) {
            // levels < L are complete now (the batches after the snapshot
            // included); a volume still covered takes the latest fill
            for (int i = 0; i < n; ++i) {
                const bool complete = !h->is_host[i].lvl_changed[(Lp - 1) % kLvlSlots];
                h->fill_up[i] = !part[i] ? -1 : !cover[i] ? fill_out[i] : (complete ? kInf : L + 1);
            }
            return SMF_OK;
        }
        if (ended && !shrink_cover(h, live, cover, R))
            return fail(SMF_ERR_HIP, "smf_solve: internal error in the level ranges");
        return SMF_OK;
    }

    // Enqueues the fix-up (nothing for a one-block search, which fixes its
    // own labels) and books the search.
    int finish()
    {
        const int n = h->n;
        if (c0 < c1 && !(h->block_search && bfs_block_fits(h->g))) {
            HIP_TRY(hipMemcpyAsync(h->fill_dev, h->fill_up, sizeof(int) * n, hipMemcpyHostToDevice, s));
            TimedScope ts(h->timer, KC_BFS_RESET, s);
            launch_bfs_fixup(h->g, h->st, c0, c1, s);
        }
        if (c0 >= c1) return SMF_OK;
        if (h->verbose) {
            int npart = 0, act = 0, lab = 0;
            for (int i = 0; i < n; ++i)
                if (part[i]) {
                    ++npart;
                    act += h->is_host[i].bfs_active;
                    lab += std::min(h->is_host[i].bfs_unsat[0], h->is_host[i].bfs_unsat[1]);
                }
            fprintf(stderr, "smf: global relabel %lld at sweep %lld: %d volumes, %d levels, active %d, columns short %d\n",
                    (long long)h->global_relabels, (long long)h->sweeps, npart, L - 1, act, lab);
        }
        for (int i = 0; i < n; ++i)
            if (part[i]) h->inst_relabels[i]++;
        h->global_relabels++;
        return SMF_OK;
    }
};

// A whole global relabel on one stream: levels are enqueued one batch ahead
// of the host's reading of the counters.
static int global_relabel(smf_handle *h, hipStream_t s, const std::vector<char> &part, bool complete = false)
{
    Search S;
    int rc = S.begin(h, s, part, complete);
    if (rc) return rc;
    if (!S.whole) {
        rc = S.step();
        for (bool all = false; !rc && !all;) {
            rc = S.step();
            if (!rc) rc = S.examine(all);
        }
        if (rc) return rc;
    }
    return S.finish();
}

// One sweep: push phases, each reading the list of work[a] and marking
// work[a^1], whose list the compaction then builds (clearing the size of the
// list filled next, and the active counts); then the relabel phase, which
// reads the last list and fills the other one.
static void enqueue_sweep(smf_handle *h, hipStream_t s, bool use_gap)
{
    int a = h->cur_work;
    for (int64_t j = 0; j < h->push_phases; ++j, a ^= 1) {
        {
            TimedScope ts(h->timer, KC_PUSH, s);
            launch_push(h->g, h->st, h->work[a], h->work[a ^ 1], h->scr, (h->pushes++ & 1) == 0, s);
        }
        launch_compact(h->g, h->work[a ^ 1], h->work[a].count, s);
    }
    {
        TimedScope ts(h->timer, KC_RELABEL, s);
        // a gap holds only for the labels it was found on: the relabel
        // phase right after its search uses it, no later one
        launch_relabel(h->g, h->st, h->work[a], h->work[a ^ 1], use_gap, s);
    }
    h->cur_work = a ^ 1;
    h->sweeps++;
}

// Solve of every volume of the batch; costs of volume i start at
// cost_dev + off[i].
static int solve_batch(smf_handle *h, const int32_t *cost_dev, const int64_t *off, hipStream_t s)
{
    const int n = h->n;
    h->solved = false;
    h->hmax_ready = false;
    h->sweeps = h->global_relabels = h->bfs_passes = h->mincut_passes = h->gap_relabels = 0;
    h->gap_searches = h->reset_nodes = h->reset_chunks = 0;
    h->flow.assign(n, 0);
    h->energy.assign(n, 0);
    h->inst_sweeps.assign(n, 0);
    h->inst_relabels.assign(n, 0);
    h->inst_gap.assign(n, 0);
    HIP_TRY(hipSetDevice(h->device));

    // volume table with this call's cost offsets
    for (int i = 0; i < n; ++i) {
        h->inst_up[i] = h->inst[i];
        h->inst_up[i].cost_base = off ? off[i] : h->inst[i].node_base;
    }
    HIP_TRY(hipMemcpyAsync(h->inst_dev, h->inst_up, sizeof(Inst) * n, hipMemcpyHostToDevice, s));

    h->timer.reset();
    if (h->g.count_work)
        launch_fill((int *)h->wcount, 2LL * 3 * kWorkSlots * kWorkStride, 0, s);
    launch_init_scratch(h->g, h->scr, s);
    if (h->g.soft) launch_fill(h->soft_flow, 4LL * h->g.Ntot, 0, s);   // no soft-arc flow yet
    {
        TimedScope ts(h->timer, KC_BUILD, s);
        launch_build(cost_dev, h->g, h->st, h->scr, s);
    }
    HIP_TRY(hipGetLastError());
    std::vector<char> all((size_t)n, 1), part((size_t)n, 0), done((size_t)n, 0);
    std::vector<int64_t> since((size_t)n, 0), period((size_t)n);
    for (int i = 0; i < n; ++i) period[i] = h->inst_period[i] > 0 ? h->inst_period[i] : h->relabel_period;
    int rc = SMF_OK;
    rc = global_relabel(h, s, all);
    if (rc) return rc;
    // work lists: every column may hold excess anywhere before the first sweep
    launch_work_init(h->g, h->work[0], h->work[1], s);
    h->cur_work = 0;
    h->pushes = 0;
    // Sweeps are polled one batch behind, like the BFS levels: a batch
    // enqueued after the volumes have finished finds empty work lists.
    int slot = 0;
    bool inflight = false;
    bool gap_fresh = false;   // a gap search ran after the last relabel phase
    for (;;) {
        if (h->sweeps >= h->max_sweeps)
            return fail(SMF_ERR_NOT_CONVERGED, "smf_solve: sweep cap reached");
        for (int64_t it = 0; it < h->poll_every; ++it) {
            // a search runs once some volume's period has come round; volumes
            // at least halfway through their own period join it, so that
            // volumes of different periods share searches (a level costs
            // one launch however many volumes take part)
            bool any = false;
            for (int i = 0; i < n; ++i) any = any || (!done[i] && since[i] >= period[i]);
            for (int i = 0; i < n; ++i) part[i] = any && !done[i] && 2 * since[i] >= period[i];
            if (any) {
                rc = global_relabel(h, s, part);
                if (rc) return rc;
                for (int i = 0; i < n; ++i)
                    if (part[i]) since[i] = 0;
            }
            enqueue_sweep(h, s, gap_fresh);
            gap_fresh = false;
            for (int i = 0; i < n; ++i)
                if (!done[i]) { since[i]++; h->inst_sweeps[i]++; }
            if (h->gap_every > 0 && h->sweeps % h->gap_every == 0) {
                launch_gap_find(h->g, h->st, h->max_inst_nodes, s);
                h->gap_searches++;
                gap_fresh = true;
            }
        }
        HIP_TRY(hipGetLastError());
        rc = post_snapshot(h, s, kSlotSweep + slot);
        if (rc) return rc;
        if (inflight) {
            rc = wait_snapshot(h, kSlotSweep + (slot ^ 1));
            if (rc) return rc;
            bool finished = true;
            int left = 0;
            for (int i = 0; i < n; ++i) {
                done[i] = h->is_host[i].active == 0;
                finished = finished && done[i];
                left += h->is_host[i].active;
            }
            if (h->verbose)
                fprintf(stderr, "smf: sweep %lld active %d columns %d\n", (long long)h->sweeps, left,
                        h->host->count[0]);
            if (finished) break;
        }
        inflight = true;
        slot ^= 1;
    }

    if (h->want_hmax) {
        // S_max, the source side of the maximal minimum cut, is the set of
        // nodes that cannot reach t in the residual graph of any maximum
        // preflow; a complete search leaves exactly those at kInf, and they
        // form a prefix of each column
        rc = global_relabel(h, s, all, true);
        if (rc) return rc;
        launch_hmax(h->g, h->st, h->Hmax, s);
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
        if (h->mincut_passes > h->max_inst_nodes + 2)
            return fail(SMF_ERR_NOT_CONVERGED, "smf_solve: minimum-cut search did not settle");
    }
    {
        TimedScope ts(h->timer, KC_FINISH, s);
        launch_finish(cost_dev, h->g, h->st, h->H, s);
    }
    HIP_TRY(hipGetLastError());
    rc = sync_scratch(h, s);
    if (rc) return rc;
    h->bfs_passes += h->host->block_levels;
    for (int i = 0; i < n; ++i) {
        h->flow[i] = h->is_host[i].flow;
        h->energy[i] = h->is_host[i].energy;
        h->inst_gap[i] = h->is_host[i].gap_frozen;
        h->gap_relabels += h->is_host[i].gap_frozen;
    }
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
    h->hmax_ready = h->want_hmax != 0;
    h->solved = true;
    return SMF_OK;
}

// A failed solve may leave work and counter copies in flight; they are
// drained before the call returns, so the handle can be reused or freed.
static int solve_checked(smf_handle *h, const int32_t *cost_dev, const int64_t *off, hipStream_t s)
{
    const int rc = solve_batch(h, cost_dev, off, s);
    if (rc != SMF_OK) {
        (void)hipStreamSynchronize(s);
    }
    return rc;
}

extern "C" int smf_solve(smf_handle *h, const int32_t *cost_dev, void *stream)
{
    g_last_error[0] = 0;
    if (!h || !cost_dev) return fail(SMF_ERR_ARG, "smf_solve: NULL handle or cost");
    if (h->n != 1) return fail(SMF_ERR_ARG, "smf_solve: the handle holds a batch; use smf_batch_solve");
    return solve_checked(h, cost_dev, nullptr, (hipStream_t)stream);
}

extern "C" int smf_batch_solve(smf_handle *h, const int32_t *packed_cost_dev,
                               const int64_t *offsets_host, void *stream)
{
    g_last_error[0] = 0;
    if (!h || !packed_cost_dev) return fail(SMF_ERR_ARG, "smf_batch_solve: NULL handle or cost");
    if (offsets_host)
        for (int i = 0; i < h->n; ++i)
            if (offsets_host[i] < 0)
                return fail(SMF_ERR_ARG, "smf_batch_solve: negative cost offset");
    return solve_checked(h, packed_cost_dev, offsets_host, (hipStream_t)stream);
}

extern "C" int smf_flow_value(const smf_handle *h, int64_t *out)
{
    if (!h || !out) return fail(SMF_ERR_ARG, "smf_flow_value: NULL argument");
    if (h->n != 1) return fail(SMF_ERR_ARG, "smf_flow_value: the handle holds a batch");
    if (!h->solved) return fail(SMF_ERR_NOT_SOLVED, "smf_flow_value: no successful solve");
    *out = h->flow[0];
    return SMF_OK;
}

extern "C" int smf_energy(const smf_handle *h, int64_t *out)
{
    if (!h || !out) return fail(SMF_ERR_ARG, "smf_energy: NULL argument");
    if (h->n != 1) return fail(SMF_ERR_ARG, "smf_energy: the handle holds a batch");
    if (!h->solved) return fail(SMF_ERR_NOT_SOLVED, "smf_energy: no successful solve");
    *out = h->energy[0];
    return SMF_OK;
}

extern "C" int smf_batch_flow_values(const smf_handle *h, int64_t *out)
{
    if (!h || !out) return fail(SMF_ERR_ARG, "smf_batch_flow_values: NULL argument");
    if (!h->solved) return fail(SMF_ERR_NOT_SOLVED, "smf_batch_flow_values: no successful solve");
    std::copy(h->flow.begin(), h->flow.end(), out);
    return SMF_OK;
}

extern "C" int smf_batch_energies(const smf_handle *h, int64_t *out)
{
    if (!h || !out) return fail(SMF_ERR_ARG, "smf_batch_energies: NULL argument");
    if (!h->solved) return fail(SMF_ERR_NOT_SOLVED, "smf_batch_energies: no successful solve");
    std::copy(h->energy.begin(), h->energy.end(), out);
    return SMF_OK;
}

static int copy_surfaces(const smf_handle *h, int32_t *out_dev, void *stream, const char *who)
{
    if (!h || !out_dev) return fail(SMF_ERR_ARG, std::string(who) + ": NULL argument");
    if (!h->solved) return fail(SMF_ERR_NOT_SOLVED, std::string(who) + ": no successful solve");
    HIP_TRY(hipMemcpyAsync(out_dev, h->H, sizeof(int) * (size_t)h->g.Ptot, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return SMF_OK;
}

extern "C" int smf_surface(const smf_handle *h, int32_t *out_dev, void *stream)
{
    if (h && h->n != 1) return fail(SMF_ERR_ARG, "smf_surface: the handle holds a batch");
    return copy_surfaces(h, out_dev, stream, "smf_surface");
}

extern "C" int smf_batch_surfaces(const smf_handle *h, int32_t *packed_out_dev, void *stream)
{
    return copy_surfaces(h, packed_out_dev, stream, "smf_batch_surfaces");
}

extern "C" int smf_surface_max(const smf_handle *h, int32_t *out_dev, void *stream)
{
    if (!h || !out_dev) return fail(SMF_ERR_ARG, "smf_surface_max: NULL argument");
    if (!h->solved || !h->hmax_ready)
        return fail(SMF_ERR_NOT_SOLVED, "smf_surface_max: the last solve did not read out h_max (param hmax)");
    HIP_TRY(hipMemcpyAsync(out_dev, h->Hmax, sizeof(int) * (size_t)h->g.Ptot, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return SMF_OK;
}

extern "C" int smf_export_state(const smf_handle *h, int32_t *excess_dev, int32_t *sink_res_dev,
                                int32_t *flow_down_dev, int32_t *flow_lat_dev, void *stream)
{
    if (!h || !excess_dev || !sink_res_dev || !flow_down_dev || !flow_lat_dev)
        return fail(SMF_ERR_ARG, "smf_export_state: NULL argument");
    if (!h->solved) return fail(SMF_ERR_NOT_SOLVED, "smf_export_state: no successful solve");
    // the state already has the caller's packed [nx][ny][K] layout
    const size_t n = sizeof(int) * (size_t)h->g.Ntot;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(excess_dev, h->st.e, n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(sink_res_dev, h->st.ts, n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(flow_down_dev, h->st.fd, n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(flow_lat_dev, h->st.fl, 4 * n, hipMemcpyDeviceToDevice, s));
    return SMF_OK;
}

// Soft smoothness weights of the volumes (Inst::alpha): the soft-arc flows
// and masks are allocated the first time some weight is positive, and kept.
static int set_alpha(smf_handle *h, const int64_t *alpha, const char *who)
{
    for (int i = 0; i < h->n; ++i)
        if (alpha[i] < 0 || alpha[i] > kMaxAlpha)
            return fail(SMF_ERR_ARG, std::string(who) + ": smooth_weight must lie in [0, 2^29]");
    bool any = false;
    for (int i = 0; i < h->n; ++i) any = any || alpha[i] > 0;
    if (any && h->g.band)
        return fail(SMF_ERR_ARG, std::string(who) + ": the soft smoothness term is not available with a narrow band");
    if (any && !h->soft_flow) {
        int *sf = nullptr;
        unsigned long long *sb = nullptr;
        if (!dev_alloc(sf, 4 * (size_t)h->g.Ntot) ||
            !dev_alloc(sb, (size_t)4 * h->g.max_nch * (size_t)h->g.Ptot)) {
            if (sf) (void)hipFree(sf);
            return fail(SMF_ERR_NOMEM, std::string(who) + ": allocation of the soft-arc state failed");
        }
        h->soft_flow = sf;
        h->sbits = sb;
    }
    for (int i = 0; i < h->n; ++i) h->inst[i].alpha = (int)alpha[i];
    h->g.soft = any ? 1 : 0;
    h->g.sbits = h->sbits;
    h->st.sf = h->soft_flow;
    return SMF_OK;
}

// Narrow band (Section 3.4): the heights each column can take on a smooth
// surface inside the caller's bands, from the pairwise bounds lo(q) >=
// lo(p) - delta and hi(p) <= hi(q) + delta, propagated from a queue of
// columns until they hold everywhere.  False when some column's range empties.
static bool band_ranges(const Inst &I, const int32_t *off, const int32_t *ext, std::vector<int> &lo,
                        std::vector<int> &hi)
{
    const int nx = I.nx, ny = I.ny, P = I.P, dl = I.delta;
    lo.resize((size_t)P);
    hi.resize((size_t)P);
    std::vector<int> queue((size_t)P);
    std::vector<char> queued((size_t)P, 1);
    for (int p = 0; p < P; ++p) {
        lo[p] = off[p];
        hi[p] = off[p] + ext[p] - 1;
        queue[p] = p;
    }
    size_t head = 0, count = (size_t)P;   // ring buffer of queued columns
    while (count) {
        const int p = queue[head];
        head = (head + 1) % (size_t)P;
        --count;
        queued[p] = 0;
        const int x = p / ny, y = p % ny;
        const int nb[4] = {x + 1 < nx ? p + ny : -1, x > 0 ? p - ny : -1, y + 1 < ny ? p + 1 : -1,
                           y > 0 ? p - 1 : -1};
        for (int q : nb) {
            if (q < 0) continue;
            bool moved = false;
            if (lo[p] - dl > lo[q]) { lo[q] = lo[p] - dl; moved = true; }
            if (hi[p] + dl < hi[q]) { hi[q] = hi[p] + dl; moved = true; }
            if (!moved) continue;
            if (lo[q] > hi[q]) return false;
            if (!queued[q]) {
                queue[(head + count) % (size_t)P] = q;
                ++count;
                queued[q] = 1;
            }
        }
    }
    return true;
}

extern "C" int smf_set_band(smf_handle *h, const int32_t *offset_host, const int32_t *extent_host)
{
    if (!h) return fail(SMF_ERR_ARG, "smf_set_band: NULL handle");
    if (!offset_host && !extent_host) {
        h->g.band = 0;
        return SMF_OK;
    }
    if (!offset_host || !extent_host) return fail(SMF_ERR_ARG, "smf_set_band: NULL offsets or extents");
    if (h->n != 1) return fail(SMF_ERR_ARG, "smf_set_band: a band needs a handle of one volume");
    if (h->inst[0].alpha > 0)
        return fail(SMF_ERR_ARG, "smf_set_band: the soft smoothness term is not available with a narrow band");
    const Inst &I = h->inst[0];
    for (int p = 0; p < I.P; ++p)
        if (offset_host[p] < 0 || extent_host[p] < 1 || extent_host[p] > I.K ||
            (long long)offset_host[p] + extent_host[p] > (1LL << 30))
            return fail(SMF_ERR_ARG, "smf_set_band: need offset >= 0, 1 <= extent <= K and offset + extent "
                                     "<= 2^30 in every column");
    std::vector<int> lo, hi;
    if (!band_ranges(I, offset_host, extent_host, lo, hi))
        return fail(SMF_ERR_ARG, "smf_set_band: no delta-smooth surface fits the bands");
    const size_t P = (size_t)I.P;
    std::vector<int> up(3 * P);
    for (size_t p = 0; p < P; ++p) {
        up[p] = lo[p];
        up[P + p] = hi[p] - lo[p] + 1;
        up[2 * P + p] = lo[p] - offset_host[p];
    }
    HIP_TRY(hipSetDevice(h->device));
    if (!h->band_dev && !dev_alloc(h->band_dev, 3 * P))
        return fail(SMF_ERR_NOMEM, "smf_set_band: allocation of the band table failed");
    HIP_TRY(hipMemcpy(h->band_dev, up.data(), sizeof(int) * 3 * P, hipMemcpyHostToDevice));
    h->g.band = 1;
    h->g.blo = h->band_dev;
    h->g.bext = h->band_dev + P;
    h->g.bcs = h->band_dev + 2 * P;
    h->solved = false;
    return SMF_OK;
}

extern "C" int smf_export_soft_flows(const smf_handle *h, int32_t *flow_soft_dev, void *stream)
{
    if (!h || !flow_soft_dev) return fail(SMF_ERR_ARG, "smf_export_soft_flows: NULL argument");
    if (!h->soft_flow || !h->g.soft)
        return fail(SMF_ERR_ARG, "smf_export_soft_flows: no positive smooth_weight is set");
    if (!h->solved) return fail(SMF_ERR_NOT_SOLVED, "smf_export_soft_flows: no successful solve");
    HIP_TRY(hipMemcpyAsync(flow_soft_dev, h->soft_flow, 4 * sizeof(int) * (size_t)h->g.Ntot,
                           hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return SMF_OK;
}

extern "C" int smf_set_param(smf_handle *h, const char *key, int64_t value)
{
    if (!h || !key) return fail(SMF_ERR_ARG, "smf_set_param: NULL argument");
    int64_t *slot = nullptr;
    if (!strcmp(key, "smooth_weight")) {
        std::vector<int64_t> all((size_t)h->n, value);
        return set_alpha(h, all.data(), "smf_set_param");
    }
    if (!strcmp(key, "relabel_period")) {
        if (value < 1) return fail(SMF_ERR_ARG, "smf_set_param: relabel_period must be >= 1");
        h->relabel_period = value;
        std::fill(h->inst_period.begin(), h->inst_period.end(), 0);
        return SMF_OK;
    }
    else if (!strcmp(key, "max_sweeps")) slot = &h->max_sweeps;
    else if (!strcmp(key, "poll_every")) slot = &h->poll_every;
    else if (!strcmp(key, "bfs_poll_every")) {
        if (value < 1 || value > kLvlSlots - 2)
            return fail(SMF_ERR_ARG, "smf_set_param: bfs_poll_every must lie in [1, 62]");
        h->bfs_poll_every = value;
        return SMF_OK;
    }
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
    else if (!strcmp(key, "search_quorum")) {
        if (value < 1 || value > 100) return fail(SMF_ERR_ARG, "smf_set_param: search_quorum lies in [1, 100]");
        h->search_quorum = value;
        return SMF_OK;
    }
    else if (!strcmp(key, "push_phases")) {
        if (value < 1 || value > 8) return fail(SMF_ERR_ARG, "smf_set_param: push_phases lies in [1, 8]");
        h->push_phases = value;
        return SMF_OK;
    }
    else if (!strcmp(key, "hmax")) {
        if (value != 0 && value != 1) return fail(SMF_ERR_ARG, "smf_set_param: hmax is 0 or 1");
        if (value && !h->Hmax) {
            HIP_TRY(hipSetDevice(h->device));
            if (!dev_alloc(h->Hmax, (size_t)h->g.Ptot))
                return fail(SMF_ERR_NOMEM, "smf_set_param: allocation of the h_max surface failed");
        }
        h->want_hmax = value;
        return SMF_OK;
    }
    else if (!strcmp(key, "verbose")) {
        if (value != 0 && value != 1) return fail(SMF_ERR_ARG, "smf_set_param: verbose is 0 or 1");
        h->verbose = value;
        return SMF_OK;
    }
    else if (!strcmp(key, "level_block")) {
        if (value < 64 || value > 1024 || (value & (value - 1)))
            return fail(SMF_ERR_ARG, "smf_set_param: level_block is a power of two in [64, 1024]");
        h->g.level_block = (int)value;
        return SMF_OK;
    }
    else if (!strcmp(key, "sweep_waves")) {
        if (value < 4 || value > (1 << 20))
            return fail(SMF_ERR_ARG, "smf_set_param: sweep_waves must lie in [4, 2^20]");
        h->g.sweep_waves = (int)value;
        return SMF_OK;
    }
    else if (!strcmp(key, "block_search")) {
        if (value != 0 && value != 1) return fail(SMF_ERR_ARG, "smf_set_param: block_search is 0 or 1");
        h->block_search = value;
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

extern "C" int smf_batch_set_param(smf_handle *h, const char *key, const int64_t *values)
{
    if (!h || !key || !values) return fail(SMF_ERR_ARG, "smf_batch_set_param: NULL argument");
    if (!strcmp(key, "smooth_weight")) return set_alpha(h, values, "smf_batch_set_param");
    if (strcmp(key, "relabel_period"))
        return fail(SMF_ERR_ARG, std::string("smf_batch_set_param: unknown key ") + key);
    for (int i = 0; i < h->n; ++i)
        if (values[i] < 0)
            return fail(SMF_ERR_ARG, "smf_batch_set_param: relabel_period must be >= 0");
    std::copy(values, values + h->n, h->inst_period.begin());
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
    else if (!strcmp(key, "volumes")) *out = h->n;
    else if (!strcmp(key, "columns")) *out = h->g.Ptot;
    else if (!strcmp(key, "nodes")) *out = h->g.Ntot;
    else if (!strcmp(key, "band")) *out = h->g.band;
    else if (!strcmp(key, "push_phases")) *out = h->push_phases;
    else if (!strcmp(key, "relabel_period")) *out = h->relabel_period;
    else if (!strncmp(key, "bytes.", 6)) {
        // algorithmic bytes of the last solve per kernel class: counted on the
        // device for the data-dependent kernels, by formula for the others
        const char *name = key + 6;
        const int64_t N = h->g.Ntot, P = h->g.Ptot;
        if (!strcmp(name, "bfs")) *out = (int64_t)h->work_bytes[0];
        else if (!strcmp(name, "push")) *out = (int64_t)h->work_bytes[1];
        else if (!strcmp(name, "relabel")) *out = (int64_t)h->work_bytes[2];
        else if (!strcmp(name, "build")) *out = 36 * N + 4 * P;
        else if (!strcmp(name, "bfs_reset")) *out = 40 * h->reset_nodes + 44 * h->reset_chunks;
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

extern "C" int smf_batch_get_stat(const smf_handle *h, const char *key, int64_t *out)
{
    if (!h || !key || !out) return fail(SMF_ERR_ARG, "smf_batch_get_stat: NULL argument");
    const std::vector<int64_t> *src = nullptr;
    if (!strcmp(key, "relabel_period")) {
        for (int i = 0; i < h->n; ++i) out[i] = h->inst_period[i] > 0 ? h->inst_period[i] : h->relabel_period;
        return SMF_OK;
    }
    if (!strcmp(key, "smooth_weight")) {
        for (int i = 0; i < h->n; ++i) out[i] = h->inst[i].alpha;
        return SMF_OK;
    }
    if (!strcmp(key, "nx") || !strcmp(key, "ny") || !strcmp(key, "K") || !strcmp(key, "delta")) {
        for (int i = 0; i < h->n; ++i) {
            const Inst &I = h->inst[i];
            out[i] = key[0] == 'n' ? (key[1] == 'x' ? I.nx : I.ny) : (key[0] == 'K' ? I.K : I.delta);
        }
        return SMF_OK;
    }
    if (!strcmp(key, "sweeps")) src = &h->inst_sweeps;
    else if (!strcmp(key, "global_relabels")) src = &h->inst_relabels;
    else if (!strcmp(key, "gap_relabels")) src = &h->inst_gap;
    else return fail(SMF_ERR_ARG, std::string("smf_batch_get_stat: unknown key ") + key);
    if (src->size() != (size_t)h->n) return fail(SMF_ERR_NOT_SOLVED, "smf_batch_get_stat: no solve yet");
    std::copy(src->begin(), src->end(), out);
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

extern "C" const char *smf_last_error(void) { return g_last_error; }
