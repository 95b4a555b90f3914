"""Pins of the CPU oracle (no GPU): the oracle against brute force, an exact
row DP, closed forms, library max-flow routines and its own invariants."""
import json
import os

import numpy as np
import pytest

import oracle
import pins
from paper_2601_17026_amd import synth


def _check_invariants(cost, delta, r):
    nx, ny, K = cost.shape
    assert r.conservation_ok and r.capacity_ok          # Eq. 2-4 on the final flow
    assert r.smin_in_smax                                # minimal cut inside maximal cut
    assert r.flow == r.cut                               # Theorem 1.1
    assert r.flow == pins.flow_closed_form(cost, r.energy)
    assert r.energy == r.energy_hmax                     # both extreme cuts are optimal
    for h in (r.hmin, r.hmax):
        assert h.min() >= 0 and h.max() < K
        assert np.abs(np.diff(h.astype(np.int64), axis=0)).max(initial=0) <= delta
        assert np.abs(np.diff(h.astype(np.int64), axis=1)).max(initial=0) <= delta
    assert (r.hmin <= r.hmax).all()
    E = np.take_along_axis(cost.astype(np.int64), r.hmin[:, :, None].astype(np.int64), 2).sum()
    assert E == r.energy


TINY = [(1, 1, 5), (1, 3, 4), (3, 1, 4), (2, 2, 4), (2, 3, 3), (3, 2, 4), (1, 6, 3), (2, 3, 4)]


@pytest.mark.parametrize("shape", TINY)
@pytest.mark.parametrize("delta", [0, 1, 2, 4])
@pytest.mark.parametrize("lohi", [(-20, 20), (0, 3), (0, 1000)])
def test_brute_force(shape, delta, lohi):
    for seed in range(3):
        c = synth.random_cost(*shape, *lohi, seed=hash((shape, delta, lohi, seed)) % 2**31)
        r = oracle.solve(c, delta)
        E, hmin, hmax = pins.brute_force(c, delta)
        assert r.energy == E
        np.testing.assert_array_equal(r.hmin, hmin)
        np.testing.assert_array_equal(r.hmax, hmax)
        _check_invariants(c, delta, r)


@pytest.mark.parametrize("n,K,delta", [(64, 32, 1), (48, 20, 0), (40, 16, 3), (33, 7, 2), (5, 64, 5)])
@pytest.mark.parametrize("axis", [0, 1])
def test_row_dp(n, K, delta, axis):
    for seed in range(2):
        row = synth.random_cost(n, 1, K, 0, 50, seed=1000 * n + 7 * K + seed)[:, 0, :]
        c = row[:, None, :] if axis == 0 else row[None, :, :]
        r = oracle.solve(np.ascontiguousarray(c), delta)
        E, hmin, hmax = pins.row_dp(row, delta)
        assert r.energy == E
        np.testing.assert_array_equal(r.hmin.reshape(-1), hmin)
        np.testing.assert_array_equal(r.hmax.reshape(-1), hmax)
        _check_invariants(np.ascontiguousarray(c), delta, r)


def test_row_dp_agrees_with_brute_force():
    # the DP pin is itself pinned to brute force
    for seed in range(20):
        row = synth.random_cost(6, 1, 4, -5, 5, seed=seed)[:, 0, :]
        for delta in (0, 1, 2):
            a = pins.row_dp(row, delta)
            b = pins.brute_force(row[:, None, :], delta)
            assert a[0] == b[0]
            np.testing.assert_array_equal(a[1], b[1].reshape(-1))
            np.testing.assert_array_equal(a[2], b[2].reshape(-1))


def test_unconstrained_columns():
    # delta >= K-1: every column independently takes its lowest/highest argmin
    c = synth.random_cost(7, 5, 9, 0, 6, seed=11)
    r = oracle.solve(c, 8)
    np.testing.assert_array_equal(r.hmin, np.argmin(c, axis=2))
    np.testing.assert_array_equal(r.hmax, 8 - np.argmin(c[:, :, ::-1], axis=2))
    assert r.energy == c.min(axis=2).sum()


def test_flat_surface_delta0():
    # delta = 0: the surface is flat at the argmin of the summed column costs
    c = synth.random_cost(4, 6, 11, -9, 9, seed=12)
    r = oracle.solve(c, 0)
    tot = c.astype(np.int64).sum(axis=(0, 1))
    assert (r.hmin == np.argmin(tot)).all()
    assert (r.hmax == 10 - np.argmin(tot[::-1])).all()
    assert r.energy == tot.min()


def test_non_decreasing_columns():
    # costs non-decreasing up every column: h = 0 is optimal and no flow moves
    c = np.sort(synth.random_cost(5, 4, 8, 0, 40, seed=13), axis=2)
    c[:, :, 0] -= 1   # make the bottom the strict unique minimum
    r = oracle.solve(np.ascontiguousarray(c), 1)
    assert (r.hmin == 0).all() and (r.hmax == 0).all()
    assert r.flow == 0


def test_planted_surface():
    # noise-free planted surface with slope <= delta is recovered exactly
    rng = np.random.default_rng(14)
    nx, ny, K, delta = 9, 7, 20, 2
    h = np.zeros((nx, ny), dtype=np.int64)
    h[0, 0] = 10
    for x in range(nx):
        for y in range(ny):
            if x == 0 and y == 0:
                continue
            ref = h[x - 1, y] if x > 0 else h[x, y - 1]
            lo, hi = ref - 2, ref + 2
            if x > 0 and y > 0:
                lo, hi = max(lo, h[x, y - 1] - 2), min(hi, h[x, y - 1] + 2)
            h[x, y] = np.clip(rng.integers(lo, hi + 1), 0, K - 1)
    c = rng.integers(1, 100, size=(nx, ny, K)).astype(np.int32)
    np.put_along_axis(c, h[:, :, None], 0, axis=2)
    r = oracle.solve(c, delta)
    np.testing.assert_array_equal(r.hmin, h)
    np.testing.assert_array_equal(r.hmax, h)
    assert r.energy == 0
    _check_invariants(c, delta, r)


@pytest.mark.parametrize("shape,delta", [((3, 4, 6), 1), ((4, 3, 5), 0), ((2, 5, 7), 2), ((3, 3, 8), 3)])
def test_library_maxflow(shape, delta):
    for seed in range(2):
        c = synth.random_cost(*shape, -30, 60, seed=77 + seed)
        r = oracle.solve(c, delta)
        assert r.flow == pins.scipy_flow(c, delta)
        assert r.flow == pins.networkx_flow(c, delta)


def test_small_workload_invariants():
    c, delta = synth.config_small()
    r = oracle.solve(c, delta)
    _check_invariants(c, delta, r)


@pytest.mark.parametrize("shape,delta", [((2, 3, 5), 1), ((3, 3, 6), 2), ((1, 4, 7), 0), ((4, 2, 6), 3)])
def test_certificate_accepts_reduced_preflow(shape, delta):
    # An independent push-relabel on the reduced arc set yields the same flow
    # value as the oracle on the full graph, and the certificate checker
    # accepts its final state together with the oracle's minimal surface.
    for seed in range(3):
        c = synth.random_cost(*shape, -25, 25, seed=500 + seed)
        r = oracle.solve(c, delta)
        e, ts, fd, fl, flow = pins.reduced_preflow(c, delta)
        assert flow == r.flow
        cert = oracle.certify(c, delta, e, ts, fd, fl, r.hmin)
        assert cert.ok, cert
        assert cert.flow == r.flow and cert.energy == r.energy


def test_certificate_rejects_mistakes():
    c = synth.random_cost(3, 3, 6, -25, 25, seed=600)
    delta = 1
    r = oracle.solve(c, delta)
    e, ts, fd, fl, flow = pins.reduced_preflow(c, delta)
    assert oracle.certify(c, delta, e, ts, fd, fl, r.hmin).ok
    # a different surface
    h2 = r.hmin.copy(); h2[1, 1] += 1
    assert not oracle.certify(c, delta, e, ts, fd, fl, h2).ok
    # a flow that breaks conservation
    fd2 = fd.copy(); fd2[0, 0, 3] += 1
    assert oracle.certify(c, delta, e, ts, fd2, fl, r.hmin).bad_conservation > 0
    # the zero flow is a preflow but not a maximum one
    N0 = np.zeros_like(e)
    B = int(c[:, :, 0].max()) + 1
    w = np.concatenate([c[:, :, :1].astype(np.int64) - B, np.diff(c.astype(np.int64), axis=2)], axis=2)
    e0 = np.maximum(0, -w).astype(np.int32)
    ts0 = np.maximum(0, w).astype(np.int32)
    z = oracle.certify(c, delta, e0, ts0, N0, np.zeros_like(fl), r.hmin)
    assert z.bad_conservation == 0 and not z.ok
    # one unit taken back from a sink arc inside the minimal cut: the state
    # is still a preflow whose reach set has the same column tops, but it is
    # one unit short of maximum and the sink is reachable from the excess
    inside = (np.arange(c.shape[2])[None, None, :] <= r.hmin[:, :, None]) & (w > 0) & (ts < w)
    assert inside.any()
    v = tuple(np.argwhere(inside)[0])
    e1, ts1 = e.copy(), ts.copy()
    e1[v] += 1
    ts1[v] += 1
    short = oracle.certify(c, delta, e1, ts1, fd, fl, r.hmin)
    assert short.bad_capacity == 0 and short.bad_conservation == 0
    assert short.bad_reach > 0 and short.flow == r.flow - 1 and not short.ok


# ---- soft smoothness: alpha * sum |h(p) - h(q)| over neighbour pairs ----------

def _soft_energy(cost, h, alpha):
    E = int(np.take_along_axis(cost.astype(np.int64), h[:, :, None].astype(np.int64), 2).sum())
    hh = h.astype(np.int64)
    return E + alpha * int(np.abs(np.diff(hh, axis=0)).sum() + np.abs(np.diff(hh, axis=1)).sum())


def _check_soft_invariants(cost, delta, alpha, r):
    assert r.conservation_ok and r.capacity_ok and r.smin_in_smax
    assert r.flow == r.cut                                   # Theorem 1.1
    assert r.flow == pins.flow_closed_form(cost, r.energy)   # same closed form
    assert r.energy == r.energy_hmax
    assert r.energy == _soft_energy(cost, r.hmin, alpha)
    for h in (r.hmin, r.hmax):
        assert np.abs(np.diff(h.astype(np.int64), axis=0)).max(initial=0) <= delta
        assert np.abs(np.diff(h.astype(np.int64), axis=1)).max(initial=0) <= delta


@pytest.mark.parametrize("shape", [(1, 3, 4), (2, 2, 4), (2, 3, 3), (3, 2, 4), (1, 6, 3)])
@pytest.mark.parametrize("delta", [0, 1, 2])
@pytest.mark.parametrize("alpha", [1, 3, 25])
def test_soft_brute_force(shape, delta, alpha):
    for seed in range(3):
        c = synth.random_cost(*shape, -20, 20, seed=hash((shape, delta, alpha, seed)) % 2**31)
        r = oracle.solve(c, delta, alpha)
        E, hmin, hmax = pins.brute_force(c, delta, alpha)
        assert r.energy == E
        np.testing.assert_array_equal(r.hmin, hmin)
        np.testing.assert_array_equal(r.hmax, hmax)
        _check_soft_invariants(c, delta, alpha, r)


@pytest.mark.parametrize("n,K,delta,alpha", [(40, 24, 2, 3), (33, 16, 4, 7), (25, 30, 1, 1), (20, 12, 6, 20)])
def test_soft_row_dp(n, K, delta, alpha):
    for seed in range(2):
        row = synth.random_cost(n, 1, K, 0, 60, seed=3000 + 11 * n + K + seed)[:, 0, :]
        r = oracle.solve(np.ascontiguousarray(row[:, None, :]), delta, alpha)
        E, hmin, hmax = pins.row_dp(row, delta, alpha)
        assert r.energy == E
        np.testing.assert_array_equal(r.hmin.reshape(-1), hmin)
        np.testing.assert_array_equal(r.hmax.reshape(-1), hmax)


def test_soft_row_dp_agrees_with_brute_force():
    for seed in range(15):
        row = synth.random_cost(5, 1, 5, -6, 6, seed=4000 + seed)[:, 0, :]
        for delta in (0, 1, 3):
            for alpha in (1, 4):
                a = pins.row_dp(row, delta, alpha)
                b = pins.brute_force(row[:, None, :], delta, alpha)
                assert a[0] == b[0]
                np.testing.assert_array_equal(a[1], b[1].reshape(-1))
                np.testing.assert_array_equal(a[2], b[2].reshape(-1))


def test_soft_alpha_zero_is_hard():
    c = synth.layered_cost(12, 10, 30, 2, 0.4, 255, 0.05, 41)
    a, b = oracle.solve(c, 2), oracle.solve(c, 2, 0)
    assert (a.flow, a.energy) == (b.flow, b.energy)
    np.testing.assert_array_equal(a.hmin, b.hmin)


def test_soft_large_alpha_is_flat():
    # alpha above columns * cost range: any step costs more than the feature
    # term can gain, so the surface is flat at the lowest argmin of the summed
    # column costs
    c = synth.random_cost(5, 4, 9, 0, 30, seed=42)
    alpha = 5 * 4 * 31
    r = oracle.solve(c, 3, alpha)
    tot = c.astype(np.int64).sum(axis=(0, 1))
    assert (r.hmin == np.argmin(tot)).all()
    assert r.energy == tot.min()


@pytest.mark.parametrize("shape,delta,alpha", [((3, 4, 6), 1, 2), ((4, 3, 5), 0, 5), ((2, 5, 7), 2, 1), ((3, 3, 8), 3, 9)])
def test_soft_library_maxflow(shape, delta, alpha):
    for seed in range(2):
        c = synth.random_cost(*shape, -30, 60, seed=5077 + seed)
        r = oracle.solve(c, delta, alpha)
        assert r.flow == pins.scipy_flow(c, delta, alpha)
        assert r.flow == pins.networkx_flow(c, delta, alpha)
        _check_soft_invariants(c, delta, alpha, r)


def test_soft_planted_surface():
    # a planted surface with steps of at most 1 whose columns have a deep
    # minimum on it survives a small alpha exactly
    rng = np.random.default_rng(43)
    nx, ny, K = 8, 6, 16
    h = np.clip(7 + np.cumsum(rng.integers(-1, 2, size=nx))[:, None] + np.zeros((1, ny), np.int64), 0, K - 1)
    c = rng.integers(200, 300, size=(nx, ny, K)).astype(np.int32)
    np.put_along_axis(c, h[:, :, None], 0, axis=2)
    r = oracle.solve(c, 1, 2)
    np.testing.assert_array_equal(r.hmin, h)
    _check_soft_invariants(c, 1, 2, r)


@pytest.mark.parametrize("shape,delta,alpha", [((2, 3, 5), 1, 2), ((3, 3, 6), 2, 5), ((1, 4, 7), 0, 3), ((4, 2, 6), 3, 1)])
def test_certificate_accepts_soft_preflow(shape, delta, alpha):
    # an independent push-relabel with the soft arcs reaches the oracle's
    # flow value, and the certificate accepts its state with the oracle's
    # minimal surface and soft energy
    for seed in range(3):
        c = synth.random_cost(*shape, -25, 25, seed=700 + seed)
        r = oracle.solve(c, delta, alpha)
        e, ts, fd, fl, fs, flow = pins.reduced_preflow_soft(c, delta, alpha)
        assert flow == r.flow
        cert = oracle.certify(c, delta, e, ts, fd, fl, r.hmin, alpha=alpha, flow_soft=fs)
        assert cert.ok, cert
        assert cert.flow == r.flow and cert.energy == r.energy


def test_certificate_rejects_soft_mistakes():
    c = synth.random_cost(3, 3, 6, -25, 25, seed=701)
    delta, alpha = 1, 3
    r = oracle.solve(c, delta, alpha)
    e, ts, fd, fl, fs, flow = pins.reduced_preflow_soft(c, delta, alpha)
    assert oracle.certify(c, delta, e, ts, fd, fl, r.hmin, alpha=alpha, flow_soft=fs).ok
    # the soft flows left out: conservation fails where they moved excess
    if fs.any():
        assert not oracle.certify(c, delta, e, ts, fd, fl, r.hmin, alpha=alpha,
                                  flow_soft=np.zeros_like(fs)).ok
    # a soft flow above its capacity
    fs2 = fs.copy(); fs2[0, 0, 0, 2] = alpha + 1
    assert oracle.certify(c, delta, e, ts, fd, fl, r.hmin, alpha=alpha, flow_soft=fs2).bad_capacity > 0
    # the hard-bound surface is not the soft optimum here, or the checker
    # must still accept it only if it is the soft minimal cut
    hard = oracle.solve(c, delta)
    cert_h = oracle.certify(c, delta, e, ts, fd, fl, hard.hmin, alpha=alpha, flow_soft=fs)
    assert cert_h.ok == bool((hard.hmin == r.hmin).all())
    # a soft preflow checked as if there were no soft arcs fails
    if fs.any():
        assert not oracle.certify(c, delta, e, ts, fd, fl, r.hmin).ok


# ---- stored expected values (tests/golden, written by make_golden.py) -------

def _stored(name):
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("name,maker", [("small", synth.config_small), ("mid", synth.config_mid)])
def test_generators_reproduce_stored_inputs(name, maker):
    # the seeded inputs are the bytes the stored values were computed on
    cost, delta = maker()
    ref = _stored(name)
    assert list(cost.shape) == ref["shape"] and delta == ref["delta"]
    assert synth.sha256(cost) == ref["cost_sha256"], "input generator drifted"


def test_oracle_reproduces_stored_small_workload():
    # regression check of the oracle itself on the 32x32x64 workload
    cost, delta = synth.config_small()
    ref = _stored("small")
    r = oracle.solve(cost, delta)
    assert (r.flow, r.energy) == (ref["flow"], ref["energy"])
    assert synth.sha256(r.hmin.astype(np.int32)) == ref["surface_sha256"]
    assert synth.sha256(r.hmax.astype(np.int32)) == ref["surface_max_sha256"]


# ---- a second oracle: scipy's max-flow with cuts read off its residual ------

def test_second_oracle_small_workload():
    # the 32x32x64 workload: flow value and both extreme minimum cuts agree
    # bit for bit (the two cuts differ in some columns, so h_max is checked
    # on its own)
    cost, delta = synth.config_small()
    r = oracle.solve(cost, delta)
    F, hmin, hmax = pins.scipy_cuts(cost, delta)
    assert F == r.flow
    np.testing.assert_array_equal(hmin, r.hmin)
    np.testing.assert_array_equal(hmax, r.hmax)
    assert (r.hmin != r.hmax).any()


@pytest.mark.parametrize("shape,delta,alpha", [
    ((1, 9, 7), 1, 0), ((6, 1, 5), 0, 0), ((5, 6, 1), 2, 0), ((4, 5, 6), 9, 0),
    ((12, 10, 20), 2, 0), ((9, 8, 33), 1, 0), ((7, 9, 12), 1, 2), ((10, 6, 15), 3, 5),
])
def test_second_oracle_random_shapes(shape, delta, alpha):
    # degenerate shapes (one row, one column line, K = 1, delta >= K),
    # random and layered costs, with and without the soft term
    for seed in range(2):
        if seed == 0:
            c = synth.random_cost(*shape, 0, 3, seed=800 + sum(shape))    # many ties
        else:
            c = synth.layered_cost(*shape, 1, 0.4, 255, 0.05, 810 + sum(shape))
        r = oracle.solve(c, delta, alpha)
        F, hmin, hmax = pins.scipy_cuts(c, delta, alpha)
        assert F == r.flow
        np.testing.assert_array_equal(hmin, r.hmin)
        np.testing.assert_array_equal(hmax, r.hmax)


@pytest.mark.parametrize("seed", range(6))
def test_hmax_from_a_textbook_preflow(seed):
    # the highest optimal surface read off an independent maximum preflow
    # equals the oracle's h_max (and brute force on the tiny volumes)
    rng = np.random.default_rng(900 + seed)
    nx, ny, K = int(rng.integers(1, 4)), int(rng.integers(1, 4)), int(rng.integers(2, 6))
    delta = int(rng.integers(0, 3))
    cost = rng.integers(0, 6, (nx, ny, K)).astype(np.int32)   # small range: many ties
    e, ts, fd, fl, flow = pins.reduced_preflow(cost, delta)
    hm = oracle.hmax_from_preflow(delta, ts, fd, fl)
    r = oracle.solve(cost, delta)
    np.testing.assert_array_equal(hm, r.hmax)
    _, _, bf_hmax = pins.brute_force(cost, delta)
    np.testing.assert_array_equal(hm, bf_hmax)
