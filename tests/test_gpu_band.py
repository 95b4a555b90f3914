"""GPU parity of narrow-band solves (Section 3.4) against the band oracle.

Every column holds its own range of heights; flow value, energy and the
minimal-cut surface (heights of the volume) must equal oracle.solve_band's
bit for bit, and the final preflow must pass the band certificate.  Cases:
random ragged bands (single-node columns, bands whose pairwise bounds cut
the feasible range), layered volumes banded around a landmark surface, and
the seismic volume's band at full size (certificate and closed form).
"""
import numpy as np
import pytest

import oracle
import pins
from paper_2601_17026_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_17026_amd import smf as mod
    return mod


def _gpu_band(smf, cost, delta, off, ext, params=None):
    c = torch.from_numpy(np.ascontiguousarray(cost, dtype=np.int32)).cuda()
    with smf.Solver(*cost.shape, delta) as s:
        s.set_band(off, ext)
        for k, v in (params or {}).items():
            s.set_param(k, v)
        s.solve(c)
        surf = s.surface().cpu().numpy()
        e, ts, fd, fl = (t.cpu().numpy() for t in s.export_state())
        torch.cuda.synchronize()
        cert = oracle.certify_band(cost, delta, off, ext, e, ts, fd, fl, surf)
        return dict(flow=s.flow_value(), energy=s.energy(), surface=surf, cert=cert)


def _check(cost, delta, off, ext, g):
    r = oracle.solve_band(cost, delta, off, ext)
    assert (g["flow"], g["energy"]) == (r.flow, r.energy)
    np.testing.assert_array_equal(g["surface"], r.hmin)
    assert g["cert"].ok, g["cert"]


def _random_feasible_band(rng, nx, ny, K, delta, max_off, min_ext=1):
    while True:
        off = rng.integers(0, max_off + 1, (nx, ny)).astype(np.int32)
        ext = rng.integers(min_ext, K + 1, (nx, ny)).astype(np.int32)
        if oracle.band_effective(off, ext, delta, K) is not None:
            return off, ext


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 7, 5), (3, 4, 9), (6, 5, 70), (9, 2, 130)])
@pytest.mark.parametrize("delta", [0, 1, 3])
def test_random_ragged_bands(smf, shape, delta):
    rng = np.random.default_rng(hash((shape, delta)) % (1 << 32))
    nx, ny, K = shape
    off, ext = _random_feasible_band(rng, nx, ny, K, delta, max_off=max(1, K // 3))
    cost = rng.integers(-50, 200, shape).astype(np.int32)
    print(f"case: random band {shape} delta {delta}", flush=True)
    _check(cost, delta, off, ext, _gpu_band(smf, cost, delta, off, ext))


def test_bands_that_force_the_bound(smf):
    # one-node columns and steep offsets: the effective ranges are much
    # smaller than the bands the caller gave
    rng = np.random.default_rng(5)
    nx, ny, K, delta = 12, 10, 40, 1
    off = (np.arange(nx)[:, None] + np.zeros((1, ny), np.int64)).astype(np.int32)
    ext = np.full((nx, ny), K, np.int32)
    off[6, 4], ext[6, 4] = 20, 1
    off[2, 7], ext[2, 7] = 14, 1
    lo, hi = oracle.band_effective(off, ext, delta, K)
    assert (hi - lo + 1 < ext).sum() > 20
    cost = rng.integers(0, 100, (nx, ny, K)).astype(np.int32)
    print("case: forced bounds 12x10x40 delta 1", flush=True)
    _check(cost, delta, off, ext, _gpu_band(smf, cost, delta, off, ext))


@pytest.mark.parametrize("shape,delta,stick", [((48, 40, 160), 2, 20), ((70, 33, 96), 1, 12)])
def test_layered_band_around_landmarks(smf, shape, delta, stick):
    cost, hs = synth.layered_cost(*shape, 3, 0.4, 255, 0.05, 61, heights=True)
    ref = synth.landmark_reference(hs[1], 8)
    band, off, ext = synth.band_from_reference(cost, ref, stick)
    print(f"case: layered band {shape} delta {delta} stick {stick}", flush=True)
    for params in ({}, {"block_search": 0}):
        _check(band, delta, off, ext, _gpu_band(smf, band, delta, off, ext, params))


def test_band_errors_and_removal(smf):
    cost = synth.layered_cost(16, 16, 40, 1, 0.3, 255, 0.0, 62)
    with smf.Solver(16, 16, 40, 1) as s:
        off = np.zeros((16, 16), np.int32)
        ext = np.full((16, 16), 40, np.int32)
        off[3, 3], ext[3, 3] = 30, 1
        off[3, 4], ext[3, 4] = 0, 1          # |30 - 0| > delta: no smooth surface
        with pytest.raises(smf.SmfError) as ei:
            s.set_band(off, ext)
        assert ei.value.status == smf.ERR_ARG
        ext[3, 4] = 0
        with pytest.raises(smf.SmfError):
            s.set_band(off, ext)
        s.set_band(np.zeros((16, 16), np.int32), np.full((16, 16), 40, np.int32))
        with pytest.raises(smf.SmfError):
            s.set_param("smooth_weight", 3)
        s.set_band(None, None)
        c = torch.from_numpy(cost).cuda()
        s.solve(c)
        r = oracle.solve(cost, 1)
        assert (s.flow_value(), s.energy()) == (r.flow, r.energy)


def test_full_size_seismic_band(smf):
    # 512 x 512 columns, 97 heights around the landmark surface of the
    # middle horizon (25.4 M nodes): certificate, closed form and the
    # surface inside the feasible range
    band, off, ext, delta = synth.config_seismic_band()
    print(f"case: seismic band {band.shape} delta {delta}", flush=True)
    g = _gpu_band(smf, band, delta, off, ext)
    assert g["cert"].ok, g["cert"]
    lo, hi = oracle.band_effective(off, ext, delta, band.shape[2])
    assert ((g["surface"] >= lo) & (g["surface"] <= hi)).all()
    assert g["energy"] == g["cert"].energy
    assert g["flow"] == pins.band_flow_closed_form(band, off, lo, hi, g["energy"])
    # a crop solved by the oracle: same volume, same bands
    sub = (slice(200, 236), slice(300, 330))
    bc, oc, ec = band[sub], off[sub], ext[sub]
    _check(np.ascontiguousarray(bc), delta, np.ascontiguousarray(oc), np.ascontiguousarray(ec),
           _gpu_band(smf, np.ascontiguousarray(bc), delta, np.ascontiguousarray(oc),
                     np.ascontiguousarray(ec)))


def test_band_hmax_matches_oracle(smf):
    rng = np.random.default_rng(91)
    nx, ny, K, delta = 14, 11, 50, 1
    off, ext = _random_feasible_band(rng, nx, ny, K, delta, max_off=10, min_ext=5)
    cost = rng.integers(0, 4, (nx, ny, K)).astype(np.int32)
    c = torch.from_numpy(cost).cuda()
    print("case: band hmax 14x11x50", flush=True)
    with smf.Solver(nx, ny, K, delta) as s:
        s.set_band(off, ext)
        s.set_param("hmax", 1)
        s.solve(c)
        r = oracle.solve_band(cost, delta, off, ext)
        np.testing.assert_array_equal(s.surface().cpu().numpy(), r.hmin)
        np.testing.assert_array_equal(s.surface_max().cpu().numpy(), r.hmax)
        assert (r.hmax > r.hmin).any()
