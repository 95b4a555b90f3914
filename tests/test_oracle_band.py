"""Pins of the oracle's narrow-band solver (CPU only).

The band graph (Section 3.4: the graph is built only in a band of heights
around the surface that the user's landmarks outline) gives each column its
own range of heights.  oracle.solve_band and oracle.certify_band are pinned
here against what the definition fixes, with code that shares nothing with
them: brute force over every smooth surface inside the bands (the optimum,
both extreme optimal surfaces, and each column's feasible range), a
single-row dynamic program with per-pair windows, the closed form of the
flow value, scipy's max-flow on the explicit band graph, the reductions to
the plain problem (equal offsets and full extents, a constant shift of all
offsets, a smoothness bound wider than every band), and a textbook
push-relabel preflow that the certificate must accept and, with planted
mistakes, reject.
"""
import numpy as np
import pytest

import oracle
import pins


def _random_band(rng, nx, ny, K, max_off, min_ext=1):
    off = rng.integers(0, max_off + 1, (nx, ny)).astype(np.int32)
    ext = rng.integers(min_ext, K + 1, (nx, ny)).astype(np.int32)
    cost = rng.integers(-20, 60, (nx, ny, K)).astype(np.int32)
    return cost, off, ext


def _tiny_cases(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        nx, ny = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        K = int(rng.integers(1, 5))
        delta = int(rng.integers(0, 3))
        cost, off, ext = _random_band(rng, nx, ny, K, max_off=4)
        yield cost, delta, off, ext


def test_effective_band_is_the_feasible_range():
    feasible = infeasible = 0
    for cost, delta, off, ext in _tiny_cases(300, 11):
        bf = pins.brute_force_band(cost, delta, off, ext)
        eff = oracle.band_effective(off, ext, delta, cost.shape[2])
        alt = pins.band_bounds(off, ext, delta)
        if bf is None:
            infeasible += 1
            assert eff is None and alt is None
            continue
        feasible += 1
        np.testing.assert_array_equal(eff[0], bf[3])
        np.testing.assert_array_equal(eff[1], bf[4])
        np.testing.assert_array_equal(alt[0], bf[3])
        np.testing.assert_array_equal(alt[1], bf[4])
    assert feasible > 100 and infeasible > 10


def test_band_optimum_matches_brute_force():
    n = 0
    for cost, delta, off, ext in _tiny_cases(300, 12):
        bf = pins.brute_force_band(cost, delta, off, ext)
        if bf is None:
            with pytest.raises(oracle.NoFeasibleSurface):
                oracle.solve_band(cost, delta, off, ext)
            continue
        r = oracle.solve_band(cost, delta, off, ext)
        assert r.energy == bf[0] and r.energy_hmax == bf[0]
        np.testing.assert_array_equal(r.hmin, bf[1])
        np.testing.assert_array_equal(r.hmax, bf[2])
        assert r.flow == r.cut
        assert r.conservation_ok and r.capacity_ok and r.smin_in_smax
        n += 1
    assert n > 100


@pytest.mark.parametrize("seed", range(6))
def test_band_row_matches_dp(seed):
    rng = np.random.default_rng(100 + seed)
    n, K = 14, 9
    delta = int(rng.integers(0, 3))
    # offsets of a smooth reference row so that most instances are feasible
    ref = np.cumsum(rng.integers(-delta - 1, delta + 2, n)).clip(0, None)
    off = ref.astype(np.int32).reshape(1, n)
    ext = rng.integers(1, K + 1, (1, n)).astype(np.int32)
    cost = rng.integers(0, 40, (1, n, K)).astype(np.int32)
    dp = pins.row_dp_band(cost[0], delta, off[0], ext[0])
    if dp is None:
        with pytest.raises(oracle.NoFeasibleSurface):
            oracle.solve_band(cost, delta, off, ext)
        return
    r = oracle.solve_band(cost, delta, off, ext)
    assert r.energy == dp[0]
    np.testing.assert_array_equal(r.hmin[0], dp[1])
    np.testing.assert_array_equal(r.hmax[0], dp[2])


@pytest.mark.parametrize("seed", range(8))
def test_band_flow_closed_form_and_scipy(seed):
    rng = np.random.default_rng(200 + seed)
    nx, ny, K = 4, 5, 7
    delta = int(rng.integers(1, 3))
    eff = None
    while eff is None:   # a sloping band with ragged extents that admits a surface
        base = rng.integers(0, 3, (nx, ny))
        off = (base + np.arange(nx)[:, None] // 2).astype(np.int32)
        ext = rng.integers(1, K + 1, (nx, ny)).astype(np.int32)
        eff = oracle.band_effective(off, ext, delta, K)
    cost = rng.integers(0, 50, (nx, ny, K)).astype(np.int32)
    r = oracle.solve_band(cost, delta, off, ext)
    lo, hi = eff
    assert r.flow == pins.band_flow_closed_form(cost, off, lo, hi, r.energy)
    assert r.flow == pins.scipy_band_flow(cost, delta, off, lo, hi)
    assert r.flow == r.cut
    assert r.energy == int(pins.band_cost_at(cost, off, r.hmin).sum())


def test_equal_offsets_and_full_extents_reduce_to_the_plain_problem():
    rng = np.random.default_rng(7)
    for _ in range(20):
        nx, ny, K = int(rng.integers(1, 5)), int(rng.integers(1, 5)), int(rng.integers(1, 8))
        delta = int(rng.integers(0, 3))
        cost = rng.integers(-10, 40, (nx, ny, K)).astype(np.int32)
        o = int(rng.integers(0, 6))
        off = np.full((nx, ny), o, np.int32)
        ext = np.full((nx, ny), K, np.int32)
        r = oracle.solve_band(cost, delta, off, ext)
        p = oracle.solve(cost, delta)
        assert (r.flow, r.energy) == (p.flow, p.energy)
        np.testing.assert_array_equal(r.hmin, p.hmin + o)
        np.testing.assert_array_equal(r.hmax, p.hmax + o)


def test_shifting_every_band_shifts_the_surface():
    rng = np.random.default_rng(8)
    for _ in range(20):
        cost, off, ext = _random_band(rng, 3, 4, 6, max_off=2)
        delta = int(rng.integers(1, 3))
        if oracle.band_effective(off, ext, delta, 6) is None:
            continue
        a = oracle.solve_band(cost, delta, off, ext)
        b = oracle.solve_band(cost, delta, off + 5, ext)
        assert (a.flow, a.energy) == (b.flow, b.energy)
        np.testing.assert_array_equal(b.hmin, a.hmin + 5)
        np.testing.assert_array_equal(b.lo, a.lo + 5)


def test_wide_bound_gives_independent_columns():
    # delta at least the spread of all bands: every column takes its own
    # lowest minimum
    rng = np.random.default_rng(9)
    for _ in range(20):
        cost, off, ext = _random_band(rng, 3, 3, 6, max_off=3)
        delta = int((off + ext).max())
        r = oracle.solve_band(cost, delta, off, ext)
        for x in range(3):
            for y in range(3):
                col = cost[x, y, :ext[x, y]]
                assert r.hmin[x, y] == off[x, y] + int(np.argmin(col))


def test_single_node_columns_pin_their_neighbours():
    # a column of one node fixes its height; its neighbours must stay within
    # delta of it, so their feasible range shrinks to that window
    cost = np.random.default_rng(10).integers(0, 30, (3, 3, 8)).astype(np.int32)
    off = np.zeros((3, 3), np.int32)
    ext = np.full((3, 3), 8, np.int32)
    off[1, 1], ext[1, 1] = 5, 1
    lo, hi = oracle.band_effective(off, ext, 1, 8)
    assert (lo[1, 1], hi[1, 1]) == (5, 5)
    assert (lo[0, 1], hi[0, 1]) == (4, 6) and (lo[1, 0], hi[1, 0]) == (4, 6)
    assert (lo[0, 0], hi[0, 0]) == (3, 7)
    bf = pins.brute_force_band(cost, 1, off, ext)
    r = oracle.solve_band(cost, 1, off, ext)
    assert r.energy == bf[0]
    np.testing.assert_array_equal(r.hmin, bf[1])


def _band_preflow_case(seed):
    rng = np.random.default_rng(300 + seed)
    nx, ny, K, delta = 3, 4, 6, 1
    off = (rng.integers(0, 2, (nx, ny)) + np.arange(ny)[None, :] // 2).astype(np.int32)
    ext = rng.integers(2, K + 1, (nx, ny)).astype(np.int32)
    cost = rng.integers(0, 40, (nx, ny, K)).astype(np.int32)
    lo, hi = oracle.band_effective(off, ext, delta, K)
    return cost, delta, off, ext, lo, hi


@pytest.mark.parametrize("seed", range(4))
def test_band_certificate_accepts_a_textbook_preflow(seed):
    cost, delta, off, ext, lo, hi = _band_preflow_case(seed)
    e, ts, fd, fl, flow = pins.reduced_preflow_band(cost, delta, off, lo, hi)
    r = oracle.solve_band(cost, delta, off, ext)
    cert = oracle.certify_band(cost, delta, off, ext, e, ts, fd, fl, r.hmin)
    assert cert.ok, cert
    assert cert.flow == flow == r.flow
    assert cert.energy == r.energy


def test_band_certificate_rejects_planted_mistakes():
    cost, delta, off, ext, lo, hi = _band_preflow_case(0)
    e, ts, fd, fl, flow = pins.reduced_preflow_band(cost, delta, off, lo, hi)
    r = oracle.solve_band(cost, delta, off, ext)
    args = lambda **kw: dict(dict(excess=e, sink_res=ts, flow_down=fd, flow_lat=fl,
                                  surface=r.hmin), **kw)
    cert = lambda **kw: oracle.certify_band(cost, delta, off, ext, **args(**kw))
    assert cert().ok
    # the surface one height higher in one column that can rise
    bump = r.hmin.copy()
    x, y = np.argwhere(bump < hi)[0]
    bump[x, y] += 1
    assert not cert(surface=bump).ok
    # an unused slot above a column's feasible range holding excess
    tall = np.argwhere(hi - lo + 1 < cost.shape[2])[0]
    e2 = e.copy()
    e2[tall[0], tall[1], cost.shape[2] - 1] = 1
    assert not cert(excess=e2).ok
    # one unit taken back from a saturated sink arc inside the minimal cut
    ts2 = ts.copy()
    sat = [(x, y, j) for x in range(ts.shape[0]) for y in range(ts.shape[1])
           for j in range(hi[x, y] - lo[x, y] + 1)
           if ts[x, y, j] == 0 and lo[x, y] + j <= r.hmin[x, y]
           and (j == 0 or cost[x, y, lo[x, y] - off[x, y] + j] > cost[x, y, lo[x, y] - off[x, y] + j - 1])]
    if sat:
        x, y, j = sat[0]
        ts2[x, y, j] = 1
        e3 = e.copy()
        e3[x, y, j] += 1
        c = cert(sink_res=ts2, excess=e3)
        assert not c.ok
    # a lateral flow moved to the arc of the other direction
    nz = np.argwhere(fl[0] > 0)
    if len(nz):
        fl2 = fl.copy()
        x, y, j = nz[0]
        fl2[1, x, y, j], fl2[0, x, y, j] = fl2[0, x, y, j], 0
        assert not cert(flow_lat=fl2).ok
