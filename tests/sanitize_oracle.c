/*
 * Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * oracle and certificate sources (tests/test_sanitizers.py).  It runs every
 * exported function on many small seeded inputs, the certificates also on
 * arbitrary (invalid) solver states, and checks only the return codes: the
 * sanitizers report any out-of-bounds access, overflow or leak.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int64_t flow, cut, energy, energy_hmax, wminus, phases;
    int32_t conservation_ok, capacity_ok, smin_in_smax, status;
} or_result;

typedef struct {
    int64_t flow, cut, energy, bad_capacity, bad_conservation, bad_smooth, bad_reach;
    int32_t status, pad;
} cert_result;

int oracle_solve_soft(const int32_t *, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t *,
                      int32_t *, or_result *);
int oracle_solve_band(const int32_t *, int32_t, int32_t, int32_t, int32_t, const int32_t *,
                      const int32_t *, int32_t *, int32_t *, int32_t *, int32_t *, or_result *);
int band_effective(int32_t, int32_t, int32_t, int32_t, const int32_t *, const int32_t *, int32_t *,
                   int32_t *);
int certify_preflow_soft(const int32_t *, int32_t, int32_t, int32_t, int32_t, int32_t, const int32_t *,
                         const int32_t *, const int32_t *, const int32_t *, const int32_t *,
                         const int32_t *, cert_result *);
int certify_preflow_band(const int32_t *, int32_t, int32_t, int32_t, int32_t, const int32_t *,
                         const int32_t *, const int32_t *, const int32_t *, const int32_t *,
                         const int32_t *, const int32_t *, cert_result *);
int certify_hmax(int32_t, int32_t, int32_t, int32_t, const int32_t *, const int32_t *, const int32_t *,
                 int32_t *);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static int32_t draw(int32_t lo, int32_t hi)   /* uniform in [lo, hi], xorshift64* */
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    const uint64_t r = rng_state * 0x2545F4914F6CDD1Dull;
    return lo + (int32_t)(r % (uint64_t)(hi - lo + 1));
}

static int32_t *fill(size_t n, int32_t lo, int32_t hi)
{
    int32_t *a = malloc((n ? n : 1) * sizeof(int32_t));
    for (size_t i = 0; i < n; ++i) a[i] = draw(lo, hi);
    return a;
}

int main(void)
{
    int failures = 0;
    for (int it = 0; it < 400; ++it) {
        const int32_t nx = draw(1, 5), ny = draw(1, 5), K = draw(1, 9), delta = draw(0, 3);
        const int32_t alpha = it % 3 == 0 ? draw(1, 7) : 0;
        const size_t P = (size_t)nx * ny, N = P * K;
        int32_t *cost = fill(N, -40, 90);
        int32_t *hmin = malloc(P * sizeof(int32_t)), *hmax = malloc(P * sizeof(int32_t));
        int32_t *lo = malloc(P * sizeof(int32_t)), *hi = malloc(P * sizeof(int32_t));
        or_result r;
        if (oracle_solve_soft(cost, nx, ny, K, delta, alpha, hmin, hmax, &r) != 0 || r.flow != r.cut) ++failures;

        /* bands: random offsets and extents, feasible or not */
        int32_t *off = fill(P, 0, 4), *ext = fill(P, 1, K);
        const int be = band_effective(nx, ny, K, delta, off, ext, lo, hi);
        const int rc = oracle_solve_band(cost, nx, ny, K, delta, off, ext, lo, hi, hmin, hmax, &r);
        if ((be == 0) != (rc == 0)) ++failures;

        /* certificates on arbitrary states: any verdict, never a fault */
        int32_t *e = fill(N, -3, 50), *ts = fill(N, -3, 50), *fd = fill(N, -3, 50);
        int32_t *fl = fill(4 * N, -3, 50), *fs = fill(4 * N, -3, 50), *surf = fill(P, -2, K + 1);
        cert_result c;
        if (certify_preflow_soft(cost, nx, ny, K, delta, alpha, e, ts, fd, fl, alpha ? fs : NULL, surf, &c))
            ++failures;
        if (be == 0 && certify_preflow_band(cost, nx, ny, K, delta, off, ext, e, ts, fd, fl, surf, &c))
            ++failures;
        if (certify_hmax(nx, ny, K, delta, ts, fd, fl, hmax)) ++failures;
        free(cost); free(hmin); free(hmax); free(lo); free(hi); free(off); free(ext);
        free(e); free(ts); free(fd); free(fl); free(fs); free(surf);
    }
    printf("sanitized oracle runs: %d failures\n", failures);
    return failures != 0;
}
