// Autotuner of the solver's schedule (include/smf.h, smf_autotune): the
// relabel period and the push phases per sweep.
//
// The frequency of global relabelling trades the cost of one search against
// the sweeps it saves; the paper settles it empirically (Section 3.4, the
// relabel factor of the global-relabel sweep).  Push phases between relabel
// phases move excess more hops per sweep.  Here the pair is chosen per class
// of volume -- key (ceil log2 K, min(delta, 4), floor log2 of the column
// count, whether the soft smoothness weight is positive) -- by timing
// complete solves of the largest volume of each class with every candidate
// pair (the fastest of three runs for short solves), and remembered in a
// process-wide cache that can be saved to and loaded from a text file (one
// line per class: "kbits delta pbits soft period phases best_ns"; lines of
// six fields are entries with one push phase, lines of five fields entries
// without the soft flag).
//
// The tuner is a client of the C-ABI: it solves the representative volume
// on a temporary handle of its own and writes the chosen periods into the
// caller's handle with smf_batch_set_param.  For a batch it then times whole
// solves of the caller's batch with the periods scaled by a common factor.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/smf.h"

namespace smf {
int set_error(int code, const std::string &msg);
void clear_error();
}  // namespace smf

namespace {

using Key = std::tuple<int, int, int, int>;

struct Choice {
    int64_t period;
    int64_t phases;
    int64_t best_ns;
};

std::mutex g_mu;
std::map<Key, Choice> g_cache;
bool g_env_loaded = false;

// (relabel period, push phases) pairs: the measured optima of the 32x32x64,
// 256^3 and 512x512x384 workloads lie among them
const int64_t kCandidates[][2] = {{4, 1}, {2, 2}, {1, 3}, {2, 3}, {3, 3}, {1, 4}, {2, 4}};
// scale factors 1, 1.5, 2 and 3 (doubled) of the whole-batch step
const int kBatchScale2[] = {2, 3, 4, 6};
// Uniform (period, push phases) schedules a batch also tries.
const int64_t kBatchUniform[][2] = {{2, 4}, {3, 3}, {1, 6}};
// Repeats per candidate: the run-to-run spread of a solve is a few
// percent, as large as the differences between neighbouring periods, so
// the fastest of three runs counts for solves under 0.25 s and the faster
// of two under 2 s.
constexpr int64_t kShortSolveNs = 250000000, kLongSolveNs = 2000000000;

int ceil_log2(int64_t v)
{
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

int floor_log2(int64_t v)
{
    int b = 0;
    while ((int64_t(2) << b) <= v) ++b;
    return b;
}

Key key_of(int32_t nx, int32_t ny, int32_t K, int32_t delta, int64_t alpha)
{
    return Key(ceil_log2(K), std::min<int32_t>(delta, 4), floor_log2((int64_t)nx * ny), alpha > 0 ? 1 : 0);
}

int load_locked(const char *path)
{
    FILE *f = fopen(path, "r");
    if (!f) return smf::set_error(SMF_ERR_ARG, std::string("smf_tune_cache_load: cannot open ") + path);
    char line[256];
    while (fgets(line, sizeof line, f)) {
        int a, b, c, d;
        long long v[3];
        const int got = sscanf(line, "%d %d %d %d %lld %lld %lld", &a, &b, &c, &d, &v[0], &v[1], &v[2]);
        if (got == 7 && v[0] >= 1 && v[1] >= 1 && v[1] <= 8) g_cache[Key(a, b, c, d)] = Choice{v[0], v[1], v[2]};
        else if (got == 6 && v[0] >= 1) g_cache[Key(a, b, c, d)] = Choice{v[0], 1, v[1]};
        else if (got == 5 && (long long)d >= 1) g_cache[Key(a, b, c, 0)] = Choice{d, 1, v[0]};
    }
    fclose(f);
    return SMF_OK;
}

int save_locked(const char *path)
{
    FILE *f = fopen(path, "w");
    if (!f) return smf::set_error(SMF_ERR_ARG, std::string("smf_tune_cache_save: cannot open ") + path);
    for (const auto &kv : g_cache)
        fprintf(f, "%d %d %d %d %lld %lld %lld\n", std::get<0>(kv.first), std::get<1>(kv.first),
                std::get<2>(kv.first), std::get<3>(kv.first), (long long)kv.second.period,
                (long long)kv.second.phases, (long long)kv.second.best_ns);
    if (fclose(f) != 0)
        return smf::set_error(SMF_ERR_ARG, std::string("smf_tune_cache_save: cannot write ") + path);
    return SMF_OK;
}

void load_env_locked()
{
    if (g_env_loaded) return;
    g_env_loaded = true;
    const char *path = getenv("SMF_TUNE_CACHE");
    if (path && *path) (void)load_locked(path);
}

// Shapes and soft smoothness weights of the handle's volumes via the C-ABI.
int shapes_of(smf_handle *h, std::vector<int64_t> s[5])
{
    int64_t n = 0;
    int rc = smf_get_stat(h, "volumes", &n);
    if (rc) return rc;
    const char *keys[5] = {"nx", "ny", "K", "delta", "smooth_weight"};
    for (int j = 0; j < 5; ++j) {
        s[j].assign((size_t)n, 0);
        rc = smf_batch_get_stat(h, keys[j], s[j].data());
        if (rc) return rc;
    }
    return SMF_OK;
}

// Periods for the handle's volumes from the cache (0 where no entry), and
// the push phases of the cached class holding the most nodes (0 if none).
std::vector<int64_t> periods_locked(const std::vector<int64_t> s[5], int64_t *phases)
{
    std::vector<int64_t> out(s[0].size(), 0);
    std::map<Key, int64_t> nodes;
    for (size_t i = 0; i < out.size(); ++i) {
        const Key k = key_of((int32_t)s[0][i], (int32_t)s[1][i], (int32_t)s[2][i], (int32_t)s[3][i], s[4][i]);
        auto it = g_cache.find(k);
        if (it == g_cache.end()) continue;
        out[i] = it->second.period;
        nodes[k] += s[0][i] * s[1][i] * s[2][i];
    }
    *phases = 0;
    int64_t most = -1;
    for (const auto &kv : nodes)
        if (kv.second > most) {
            most = kv.second;
            *phases = g_cache[kv.first].phases;
        }
    return out;
}

// The cached choices into the handle: per-volume periods, and the push
// phases (one value for the whole handle) of its largest cached class.
int apply_locked(smf_handle *h, const std::vector<int64_t> s[5])
{
    int64_t phases = 0;
    const std::vector<int64_t> per = periods_locked(s, &phases);
    const int rc = smf_batch_set_param(h, "relabel_period", per.data());
    if (rc || phases < 1) return rc;
    return smf_set_param(h, "push_phases", phases);
}

}  // namespace

extern "C" int smf_autotune(smf_handle *h, const int32_t *packed_cost_dev,
                            const int64_t *offsets_host, void *stream)
{
    smf::clear_error();
    if (!h || !packed_cost_dev) return smf::set_error(SMF_ERR_ARG, "smf_autotune: NULL handle or cost");
    int64_t band = 0;
    if (smf_get_stat(h, "band", &band) == SMF_OK && band)
        return smf::set_error(SMF_ERR_ARG, "smf_autotune: the tuner times full-height volumes; a handle "
                                           "with a narrow band keeps its relabel period");
    std::vector<int64_t> s[5];
    int rc = shapes_of(h, s);
    if (rc) return rc;
    const size_t n = s[0].size();
    std::vector<int64_t> off(n);
    for (size_t i = 0, acc = 0; i < n; ++i) {
        off[i] = offsets_host ? offsets_host[i] : (int64_t)acc;
        acc += (size_t)(s[0][i] * s[1][i] * s[2][i]);
    }
    std::lock_guard<std::mutex> lock(g_mu);
    load_env_locked();
    // the largest volume of every class that the cache does not know yet
    std::map<Key, size_t> todo;
    for (size_t i = 0; i < n; ++i) {
        const Key k = key_of((int32_t)s[0][i], (int32_t)s[1][i], (int32_t)s[2][i], (int32_t)s[3][i], s[4][i]);
        if (g_cache.count(k)) continue;
        auto it = todo.find(k);
        const int64_t size = s[0][i] * s[1][i] * s[2][i];
        if (it == todo.end() || size > s[0][it->second] * s[1][it->second] * s[2][it->second])
            todo[k] = i;
    }
    for (const auto &kv : todo) {
        const size_t i = kv.second;
        smf_handle *t = smf_create((int32_t)s[0][i], (int32_t)s[1][i], (int32_t)s[2][i], (int32_t)s[3][i]);
        if (!t) return SMF_ERR_NOMEM;   // smf_create described the failure
        const int32_t *cost = packed_cost_dev + off[i];
        rc = smf_set_param(t, "smooth_weight", s[4][i]);
        if (!rc) rc = smf_solve(t, cost, stream);   // warm-up
        Choice best{0, 0, 0};
        for (const auto &cand : kCandidates) {
            if (rc) break;
            const int64_t p = cand[0], m = cand[1];
            rc = smf_set_param(t, "relabel_period", p);
            if (!rc) rc = smf_set_param(t, "push_phases", m);
            if (rc) break;
            int64_t ns = -1;
            for (int rep = 0; rep < 3 && !rc; ++rep) {
                const auto t0 = std::chrono::steady_clock::now();
                rc = smf_solve(t, cost, stream);   // returns once the result is complete
                const auto t1 = std::chrono::steady_clock::now();
                const int64_t d = std::chrono::duration_cast<std::chrono::nanoseconds>(t1 - t0).count();
                ns = ns < 0 ? d : std::min(ns, d);
                if (d >= kLongSolveNs || (rep == 1 && d >= kShortSolveNs)) break;
            }
            if (!rc && (best.period == 0 || ns < best.best_ns)) best = Choice{p, m, ns};
        }
        smf_destroy(t);
        if (rc) return rc;
        g_cache[kv.first] = best;
    }
    const char *path = getenv("SMF_TUNE_CACHE");
    if (path && *path && !todo.empty()) (void)save_locked(path);
    rc = apply_locked(h, s);
    if (rc || n == 1) return rc;
    // The volumes of a batch share their searches (a level costs one launch
    // however many volumes take part), which can favour other schedules than
    // solving each volume alone: whole-batch solves are timed with every
    // class period scaled by each factor (the class push phases), and with a
    // few uniform schedules; each is timed twice and the fastest kept.
    std::vector<int64_t> eff(n), scaled(n);
    rc = smf_batch_get_stat(h, "relabel_period", eff.data());
    if (rc) return rc;
    int64_t phases0 = 0;
    rc = smf_get_stat(h, "push_phases", &phases0);
    if (rc) return rc;
    struct Sched {
        std::vector<int64_t> per;
        int64_t phases;
    };
    std::vector<Sched> cands;
    for (int f2 : kBatchScale2) {   // twice the scale factor
        for (size_t i = 0; i < n; ++i) scaled[i] = std::max<int64_t>(1, (eff[i] * f2 + 1) / 2);
        cands.push_back({scaled, phases0});
    }
    for (const auto &u : kBatchUniform) cands.push_back({std::vector<int64_t>(n, u[0]), u[1]});
    int64_t best_ns = -1;
    size_t best = 0;
    for (size_t c = 0; c < cands.size(); ++c) {
        rc = smf_batch_set_param(h, "relabel_period", cands[c].per.data());
        if (!rc) rc = smf_set_param(h, "push_phases", cands[c].phases);
        if (!rc && c == 0) rc = smf_batch_solve(h, packed_cost_dev, off.data(), stream);   // warm-up
        int64_t ns = -1;
        for (int rep = 0; rep < 2 && !rc; ++rep) {
            const auto t0 = std::chrono::steady_clock::now();
            rc = smf_batch_solve(h, packed_cost_dev, off.data(), stream);
            const auto t1 = std::chrono::steady_clock::now();
            const int64_t d = std::chrono::duration_cast<std::chrono::nanoseconds>(t1 - t0).count();
            ns = ns < 0 ? d : std::min(ns, d);
        }
        if (rc) return rc;
        if (best_ns < 0 || ns < best_ns) {
            best_ns = ns;
            best = c;
        }
    }
    rc = smf_batch_set_param(h, "relabel_period", cands[best].per.data());
    return rc ? rc : smf_set_param(h, "push_phases", cands[best].phases);
}

extern "C" int smf_tune_apply(smf_handle *h)
{
    smf::clear_error();
    if (!h) return smf::set_error(SMF_ERR_ARG, "smf_tune_apply: NULL handle");
    std::vector<int64_t> s[5];
    int rc = shapes_of(h, s);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    load_env_locked();
    return apply_locked(h, s);
}

extern "C" int smf_tune_cache_load(const char *path)
{
    smf::clear_error();
    if (!path) return smf::set_error(SMF_ERR_ARG, "smf_tune_cache_load: NULL path");
    std::lock_guard<std::mutex> lock(g_mu);
    return load_locked(path);
}

extern "C" int smf_tune_cache_save(const char *path)
{
    smf::clear_error();
    if (!path) return smf::set_error(SMF_ERR_ARG, "smf_tune_cache_save: NULL path");
    std::lock_guard<std::mutex> lock(g_mu);
    return save_locked(path);
}

extern "C" int smf_tune_cache_clear(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache.clear();
    g_env_loaded = true;   // an explicit clear also forgets the environment's file
    return SMF_OK;
}

extern "C" int smf_tune_lookup(int32_t nx, int32_t ny, int32_t K, int32_t delta, int64_t *period)
{
    smf::clear_error();
    if (!period || nx < 1 || ny < 1 || K < 1 || delta < 0)
        return smf::set_error(SMF_ERR_ARG, "smf_tune_lookup: bad shape or NULL output");
    std::lock_guard<std::mutex> lock(g_mu);
    load_env_locked();
    auto it = g_cache.find(key_of(nx, ny, K, delta, 0));
    *period = it == g_cache.end() ? 0 : it->second.period;
    return SMF_OK;
}
