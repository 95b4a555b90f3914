"""GPU checks of the schedule autotuner (smf_autotune): it picks a candidate
(relabel period, push phases) pair per volume class, applies the period
to every volume of the class and the push phases of the largest class to
the handle (for a batch, the class periods scaled by one common factor or
a uniform schedule, whichever whole-batch solve was fastest), the cache
round-trips through a file (old entries without push phases load with one),
and tuned solves stay exact."""
import numpy as np
import pytest

import oracle
from paper_2601_17026_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CANDIDATES = {1, 2, 3, 4}            # periods of the candidate pairs
PHASES = {1, 2, 3, 4}


@pytest.fixture(scope="module")
def smf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_17026_amd import smf as mod
    return mod


def test_autotune_batch(smf, tmp_path):
    # two volumes share a class (same K bucket, delta, column bucket), one differs
    shapes = [(40, 40, 100, 2), (36, 44, 120, 2), (20, 30, 60, 1)]
    vols = [synth.layered_cost(nx, ny, K, 2, 0.4, 255, 0.05, 1500 + i)
            for i, (nx, ny, K, _) in enumerate(shapes)]
    smf.tune_cache_clear()
    with smf.BatchSolver(shapes) as b:
        packed = b.pack([torch.from_numpy(v).cuda() for v in vols])
        print("case: autotune of a 3-volume batch", flush=True)
        smf.autotune(b, packed)
        periods = b.stat_per_volume("relabel_period")
        classes = [smf.tune_lookup(*sh) for sh in shapes]
        assert set(classes) <= CANDIDATES
        assert periods[0] == periods[1]
        # the batch step scales every class period by one common factor
        # (1, 1.5, 2 or 3, rounded half up) or takes a uniform schedule
        scaled = any(periods == [max(1, (c * f2 + 1) // 2) for c in classes] for f2 in (2, 3, 4, 6))
        uniform = (periods, b.stat("push_phases")) in [([p] * 3, m) for p, m in ((2, 4), (3, 3), (1, 6))]
        assert scaled or uniform, (periods, classes, b.stat("push_phases"))
        b.solve(packed)
        flows, energies = b.flow_values(), b.energies()
        surfs = [s.cpu().numpy() for s in b.unpack_surfaces(b.surfaces())]
    for (nx, ny, K, dl), v, f, e, s in zip(shapes, vols, flows, energies, surfs):
        r = oracle.solve(v, dl)
        assert (f, e) == (r.flow, r.energy)
        np.testing.assert_array_equal(s, r.hmin)
    # the cache survives a save / clear / load round trip and is applied
    # to a new handle without timing
    path = str(tmp_path / "tune.txt")
    smf.tune_cache_save(path)
    smf.tune_cache_clear()
    assert smf.tune_lookup(*shapes[0]) == 0
    smf.tune_cache_load(path)
    with smf.Solver(*shapes[2]) as s:
        smf.tune_apply(s)
        assert s.stat_per_volume("relabel_period") == [classes[2]]
    with smf.BatchSolver(shapes[:1]) as b1:
        smf.tune_apply(b1)
        assert b1.stat_per_volume("relabel_period") == [classes[0]]
        assert b1.stat("push_phases") in PHASES
    lines = [line.split() for line in open(path).read().splitlines()]
    assert all(len(f) == 7 and int(f[5]) in PHASES for f in lines)
    # an entry written without push phases loads with one push phase
    legacy = tmp_path / "legacy.txt"
    legacy.write_text(" ".join(lines[0][:5] + lines[0][6:]) + "\n")
    smf.tune_cache_clear()
    smf.tune_cache_load(str(legacy))
    smf.tune_cache_save(path)
    assert open(path).read().split()[5] == "1"


def test_autotune_plain_handle(smf):
    cost, delta = synth.config_small()
    smf.tune_cache_clear()
    c = torch.from_numpy(cost).cuda()
    with smf.Solver(*cost.shape, delta) as s:
        print("case: autotune of a plain handle", flush=True)
        smf.autotune(s, c)
        assert smf.tune_lookup(*cost.shape, delta) in CANDIDATES
        assert s.stat("push_phases") in PHASES
        s.solve(c)
        r = oracle.solve(cost, delta)
        assert s.flow_value() == r.flow and s.energy() == r.energy
        np.testing.assert_array_equal(s.surface().cpu().numpy(), r.hmin)


def test_autotune_soft_class(smf, tmp_path):
    # one shape with and without the soft smoothness term: two classes,
    # each timed with its own weight; tuned solves stay exact
    shapes = [(40, 40, 100, 2), (40, 40, 100, 2)]
    alphas = [0, 6]
    vols = [synth.layered_cost(40, 40, 100, 2, 0.4, 255, 0.05, 1600 + i) for i in range(2)]
    smf.tune_cache_clear()
    with smf.BatchSolver(shapes) as b:
        b.set_param_per_volume("smooth_weight", alphas)
        packed = b.pack([torch.from_numpy(v).cuda() for v in vols])
        print("case: autotune with a soft class", flush=True)
        smf.autotune(b, packed)
        assert all(p >= 1 for p in b.stat_per_volume("relabel_period"))
        b.solve(packed)
        flows, energies = b.flow_values(), b.energies()
        surfs = [s.cpu().numpy() for s in b.unpack_surfaces(b.surfaces())]
    for v, a, f, e, s in zip(vols, alphas, flows, energies, surfs):
        r = oracle.solve(v, 2, a)
        assert (f, e) == (r.flow, r.energy)
        np.testing.assert_array_equal(s, r.hmin)
    path = tmp_path / "tune.txt"
    smf.tune_cache_save(str(path))
    keys = sorted(tuple(line.split()[:4]) for line in path.read_text().splitlines())
    assert keys == [("7", "2", "10", "0"), ("7", "2", "10", "1")]
    smf.tune_cache_clear()
