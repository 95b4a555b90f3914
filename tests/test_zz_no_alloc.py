"""The allocation-free entry point against the handle-based solve.

smf_solve_noalloc keeps all solver state in the library's static device
workspace; its flow value, energy and surface must equal those of
smf_create + smf_solve bit for bit.  Two calls in a row, the second on a
smaller volume, check that a call does not depend on what the previous one
left in the shared workspace.
"""
import numpy as np
import pytest

from paper_2601_17026_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_17026_amd import smf as mod
    return mod


def _handle_solve(smf, c, delta):
    with smf.Solver(*c.shape, delta) as s:
        s.solve(c)
        return s.flow_value(), s.energy(), s.surface().cpu().numpy()


def test_noalloc_matches_solve_on_two_calls(smf):
    # 48 x 40 columns (searches launched level by level), then 20 x 24
    # columns (whole searches in one block), ragged K
    cases = [((48, 40, 100), 2, 31), ((20, 24, 40), 1, 32)]
    for shape, delta, seed in cases:
        cost = synth.layered_cost(*shape, 2, 0.4, 255, 0.05, seed)
        print(f"case: noalloc {shape} delta {delta} seed {seed}", flush=True)
        c = torch.from_numpy(cost).cuda()
        flow, energy, surf = smf.solve_noalloc(c, delta)
        torch.cuda.synchronize()
        ref = _handle_solve(smf, c, delta)
        assert (flow, energy) == ref[:2]
        np.testing.assert_array_equal(surf.cpu().numpy(), ref[2])


def test_noalloc_refuses_a_volume_beyond_its_workspace(smf):
    # 33 bytes per node: 256 x 256 x 64 nodes need more than 64 MiB
    c = torch.zeros((256, 256, 64), dtype=torch.int32, device="cuda")
    with pytest.raises(smf.SmfError) as ei:
        smf.solve_noalloc(c, 1)
    assert ei.value.status == smf.ERR_NOMEM
    assert "static workspace" in str(ei.value)
