"""GPU parity of the soft smoothness term (set_param "smooth_weight"):
the energy alpha * sum |h(p) - h(q)| over neighbour columns on top of the
hard bound delta, as finite arcs (p,z) -> (q,z) of capacity alpha.  Flow
value, energy (with the smoothness term) and minimal-cut surface must match
the CPU oracle bit for bit."""
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


def _solve(smf, cost, delta, alpha, params=None, certify=False):
    c = torch.from_numpy(np.ascontiguousarray(cost, dtype=np.int32)).cuda()
    with smf.Solver(*cost.shape, delta) as s:
        s.set_param("smooth_weight", alpha)
        for k, v in (params or {}).items():
            s.set_param(k, v)
        s.solve(c)
        out = dict(flow=s.flow_value(), energy=s.energy(), surface=s.surface().cpu().numpy())
        if certify:
            e, ts, fd, fl = (t.cpu().numpy() for t in s.export_state())
            fs = s.export_soft_flows().cpu().numpy()
            torch.cuda.synchronize()
            out["cert"] = oracle.certify(cost, delta, e, ts, fd, fl, out["surface"], alpha=alpha,
                                         flow_soft=fs)
        return out


def _check(cost, delta, alpha, g):
    r = oracle.solve(cost, delta, alpha)
    assert g["flow"] == r.flow
    assert g["energy"] == r.energy
    np.testing.assert_array_equal(g["surface"], r.hmin)
    assert g["flow"] == pins.flow_closed_form(cost, g["energy"])


@pytest.mark.parametrize("shape", [(1, 1, 5), (1, 6, 4), (3, 4, 5), (5, 3, 9), (2, 7, 3), (4, 4, 70)])
@pytest.mark.parametrize("delta", [0, 1, 3])
@pytest.mark.parametrize("alpha", [1, 4, 50])
def test_soft_tiny(smf, shape, delta, alpha):
    for seed, (lo, hi) in enumerate([(-20, 20), (0, 1000)]):
        cost = synth.random_cost(*shape, lo, hi, seed=9100 + seed)
        print(f"case: soft tiny {shape} delta {delta} alpha {alpha} seed {seed}", flush=True)
        g = _solve(smf, cost, delta, alpha)
        _check(cost, delta, alpha, g)
        if np.prod(shape[:2]) <= 6 and shape[2] <= 5:
            E, hmin, _ = pins.brute_force(cost, delta, alpha)
            assert g["energy"] == E
            np.testing.assert_array_equal(g["surface"], hmin)


@pytest.mark.parametrize("case", ["small", "layered", "ragged"])
@pytest.mark.parametrize("alpha", [1, 3, 16])
def test_soft_workloads(smf, case, alpha):
    # several tiles of columns and chunks, K not a multiple of 64; the final
    # preflow with its soft-arc flows also passes the certificate
    cost, delta = {"small": synth.config_small(),
                   "layered": (synth.layered_cost(37, 29, 70, 2, 0.4, 255, 0.05, 23), 1),
                   "ragged": (synth.layered_cost(50, 21, 130, 2, 0.5, 255, 0.1, 29), 2)}[case]
    print(f"case: soft {case} {cost.shape} delta {delta} alpha {alpha}", flush=True)
    g = _solve(smf, cost, delta, alpha, certify=True)
    _check(cost, delta, alpha, g)
    assert g["cert"].ok, g["cert"]
    assert g["cert"].flow == g["flow"] and g["cert"].energy == g["energy"]


def test_soft_full_size_seismic(smf):
    # 512 x 512 x 384 with alpha 16, the soft leg of the benchmark: too large
    # for the oracle, so the max-flow/min-cut certificate of the final
    # preflow (soft flows included) proves F and the minimal surface, and F
    # equals the closed form of the energy
    cost, delta = synth.config_seismic()
    print("case: soft full-size seismic 512x512x384 delta 2 alpha 16", flush=True)
    g = _solve(smf, cost, delta, 16, certify=True)
    assert g["cert"].ok, g["cert"]
    assert g["cert"].flow == g["flow"] and g["cert"].energy == g["energy"]
    assert g["flow"] == pins.flow_closed_form(cost, g["energy"])


def test_soft_export_errors(smf):
    cost, delta = synth.config_small()
    with smf.Solver(*cost.shape, delta) as s:
        s.solve(torch.from_numpy(cost).cuda())
        with pytest.raises(smf.SmfError):
            s.export_soft_flows()       # no soft term set


@pytest.mark.parametrize("params", [{"relabel_period": 1}, {"gap_every": 1}, {"bfs_early_stop": 0},
                                    {"relabel_period": 1000, "gap_every": 1}, {"block_search": 0}])
def test_soft_parameter_variants(smf, params):
    cost = synth.layered_cost(24, 31, 45, 2, 0.4, 255, 0.05, 31)
    print(f"case: soft variants {params}", flush=True)
    _check(cost, 2, 5, _solve(smf, cost, 2, 5, params))


def test_soft_weight_back_to_zero(smf):
    # one handle: soft, then alpha 0 again (the kernels without soft arcs)
    cost, delta = synth.config_small()
    c = torch.from_numpy(cost).cuda()
    with smf.Solver(*cost.shape, delta) as s:
        for alpha in (4, 0, 2):
            s.set_param("smooth_weight", alpha)
            s.solve(c)
            r = oracle.solve(cost, delta, alpha)
            assert (s.flow_value(), s.energy()) == (r.flow, r.energy), alpha
            np.testing.assert_array_equal(s.surface().cpu().numpy(), r.hmin)


def test_soft_batch_mixed_weights(smf):
    shapes = [(32, 32, 64, 2), (37, 29, 70, 1), (5, 3, 9, 3), (16, 16, 130, 4), (1, 300, 40, 3)]
    alphas = [3, 0, 7, 1, 2]
    vols = [synth.layered_cost(nx, ny, K, 2, 0.4, 255, 0.05, 60 + i) for i, (nx, ny, K, _) in enumerate(shapes)]
    with smf.BatchSolver(shapes) as b:
        b.set_param_per_volume("smooth_weight", alphas)
        assert b.stat_per_volume("smooth_weight") == alphas
        print("case: soft batch with mixed weights", flush=True)
        b.solve(b.pack([torch.from_numpy(v).cuda() for v in vols]))
        flows, energies = b.flow_values(), b.energies()
        surfs = [s.cpu().numpy() for s in b.unpack_surfaces(b.surfaces())]
    for (nx, ny, K, dl), a, v, f, e, h in zip(shapes, alphas, vols, flows, energies, surfs):
        r = oracle.solve(v, dl, a)
        assert (f, e) == (r.flow, r.energy)
        np.testing.assert_array_equal(h, r.hmin)


def test_soft_weight_errors(smf):
    with smf.Solver(4, 4, 4, 1) as s:
        with pytest.raises(smf.SmfError):
            s.set_param("smooth_weight", -1)
        with pytest.raises(smf.SmfError):
            s.set_param("smooth_weight", 1 << 30)


def test_soft_mid_volume(smf):
    # 80 x 72 x 66 (5760 columns, two chunks each, a ragged top chunk):
    # large enough for many waves per launch, small enough for the oracle
    cost = synth.layered_cost(80, 72, 66, 3, 0.4, 255, 0.05, 71)
    print("case: soft 80x72x66 delta 2 alpha 2", flush=True)
    _check(cost, 2, 2, _solve(smf, cost, 2, 2))


def test_soft_weight_at_its_limit(smf):
    # alpha = 2^29 is the largest weight accepted (the soft residuals
    # alpha - f + f' then stay below 2^31); 2^29 + 1 is refused
    amax = 1 << 29
    with smf.Solver(4, 4, 4, 1) as s:
        with pytest.raises(smf.SmfError):
            s.set_param("smooth_weight", amax + 1)
    for shape, delta in [((5, 4, 9), 2), ((3, 6, 70), 1)]:
        cost = synth.random_cost(*shape, 0, 1000, seed=9300)
        print(f"case: soft weight 2^29 {shape} delta {delta}", flush=True)
        g = _solve(smf, cost, delta, amax, certify=True)
        _check(cost, delta, amax, g)
        assert g["cert"].ok, g["cert"]
        # any step costs more than the whole feature term could gain
        assert (g["surface"] == g["surface"][0, 0]).all()
    # the largest weight with costs over the whole accepted range: the exact
    # result or ERR_RANGE, never a wrong answer
    M = (1 << 30) - 1
    for seed in range(3):
        cost = synth.random_cost(4, 4, 6, -M, M, seed=9310 + seed)
        print(f"case: soft weight 2^29 extreme costs seed {seed}", flush=True)
        try:
            g = _solve(smf, cost, 1, amax, certify=True)
        except smf.SmfError as e:
            assert e.status == smf.ERR_RANGE, e
            continue
        _check(cost, 1, amax, g)
        assert g["cert"].ok, g["cert"]
