"""GPU tests of the differentiable surface energy: the one-hot backward kernel
against a plain torch indicator, the forward against the oracle, and the
gradient against integer +-1 finite differences of the exact energy."""
import numpy as np
import pytest

import oracle
from paper_2601_17026_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_17026_amd import autograd, smf
    return smf, autograd


@pytest.mark.parametrize("n,nx,ny,K", [(1, 1, 1, 1), (2, 3, 5, 7), (3, 16, 9, 64), (2, 40, 33, 130),
                                       (1, 7, 6, 1029), (4, 33, 2, 256), (3, 5, 3, 2)])
def test_onehot_backward_kernel(mods, n, nx, ny, K):
    smf, _ = mods
    g = torch.Generator(device="cpu").manual_seed(7)
    h = torch.randint(0, K, (n, nx, ny), generator=g, dtype=torch.int32)
    gE = torch.randn(n, generator=g, dtype=torch.float32)
    out = smf.onehot_backward(h.cuda(), gE.cuda(), K).cpu()
    ref = torch.zeros(n, nx, ny, K)
    ref.scatter_(3, h.long()[..., None], gE[:, None, None, None].expand(n, nx, ny, 1))
    assert torch.equal(out, ref)


def _energy_oracle(ci, delta):
    return oracle.solve(ci, delta).energy


def test_forward_matches_oracle(mods):
    _, ag = mods
    cost, _, _ = synth.diff_costs(batch=2, n=24, K=40, device="cuda")
    E, h = ag.surface_energy(cost, 2)
    ci = ag.quantize(cost).cpu().numpy()
    for b in range(2):
        r = oracle.solve(ci[b], 2)
        assert E[b].item() == pytest.approx(r.energy / 16.0, abs=0)
        np.testing.assert_array_equal(h[b].cpu().numpy(), r.hmin)


def test_gradient_finite_differences_oracle(mods):
    """On columns whose optimal height is unique (h_min = h_max, from the
    oracle), integer +-1 perturbations of one cost change the exact energy by
    exactly the one-hot gradient."""
    _, ag = mods
    cost, _, _ = synth.diff_costs(batch=1, n=12, K=24, seed0=5101, device="cuda")
    cost = cost.clone().requires_grad_(True)
    E, h = ag.surface_energy(cost, 2)
    E.sum().backward()
    grad = cost.grad[0].cpu().numpy()
    ci = ag.quantize(cost.detach())[0].cpu().numpy()
    ref = oracle.solve(ci, 2)
    np.testing.assert_array_equal(h[0].cpu().numpy(), ref.hmin)
    rng = np.random.default_rng(3)
    uniq = np.argwhere(ref.hmin == ref.hmax)
    assert len(uniq) > 20
    checked = 0
    for (x, y) in uniq[rng.permutation(len(uniq))[:20]]:
        for z in {int(ref.hmin[x, y]), int(rng.integers(0, 24))}:
            up = ci.copy(); up[x, y, z] += 1
            dn = ci.copy(); dn[x, y, z] -= 1
            d_up = _energy_oracle(up, 2) - ref.energy
            d_dn = ref.energy - _energy_oracle(dn, 2)
            assert d_up == d_dn == int(grad[x, y, z]), (x, y, z, d_up, d_dn, grad[x, y, z])
            checked += 1
    assert checked >= 20


def test_soft_forward_and_gradient(mods):
    """With the soft smoothness term (alpha = 0.5 in cost units, weight 8
    after the x16 quantisation): the forward against the oracle, and the
    gradient, still the one-hot of the surface, against +-1 finite
    differences of the exact soft energy on columns of unique height."""
    _, ag = mods
    cost, _, _ = synth.diff_costs(batch=2, n=12, K=24, seed0=5201, device="cuda")
    cost = cost.clone().requires_grad_(True)
    a = ag.soft_weight(0.5)
    assert a == 8
    E, h = ag.surface_energy(cost, 2, alpha=0.5)
    E.sum().backward()
    ci = ag.quantize(cost.detach()).cpu().numpy()
    rng = np.random.default_rng(4)
    checked = 0
    for b in range(2):
        ref = oracle.solve(ci[b], 2, a)
        assert E[b].item() == pytest.approx(ref.energy / 16.0, abs=0)
        np.testing.assert_array_equal(h[b].cpu().numpy(), ref.hmin)
        grad = cost.grad[b].cpu().numpy()
        uniq = np.argwhere(ref.hmin == ref.hmax)
        for (x, y) in uniq[rng.permutation(len(uniq))[:8]]:
            for z in {int(ref.hmin[x, y]), int(rng.integers(0, 24))}:
                up = ci[b].copy(); up[x, y, z] += 1
                dn = ci[b].copy(); dn[x, y, z] -= 1
                d_up = oracle.solve(up, 2, a).energy - ref.energy
                d_dn = ref.energy - oracle.solve(dn, 2, a).energy
                assert d_up == d_dn == int(grad[x, y, z]), (b, x, y, z, d_up, d_dn)
                checked += 1
    assert checked >= 16
    # the cached solver goes back to the hard bound with alpha = 0
    E0, h0 = ag.surface_energy(cost.detach(), 2)
    r0 = oracle.solve(ci[0], 2)
    assert E0[0].item() == pytest.approx(r0.energy / 16.0, abs=0)
    np.testing.assert_array_equal(h0[0].cpu().numpy(), r0.hmin)


def test_gradient_reaches_the_network(mods):
    _, ag = mods
    _, net, x = synth.diff_costs(batch=2, n=16, K=32, device="cuda")
    y = net(x)[:, 0]
    c = (y - y.mean(dim=(1, 2, 3), keepdim=True)) / y.std(dim=(1, 2, 3), keepdim=True) * 4.0
    E, h = ag.surface_energy(c, 2)
    E.sum().backward()
    grads = [p.grad for p in net.parameters()]
    assert all(g is not None and torch.isfinite(g).all() for g in grads)
    assert any(g.abs().sum() > 0 for g in grads)


def test_differentiable_workload_full_size(mods):
    """8 volumes of 128x128x128, delta 2.  Every solve, perturbed ones
    included, is certified optimal; h_max is read out on the GPU and must
    equal the one read off the certified preflow; the backward must be the
    indicator of the certified surface; and 200 integer +-1 finite
    differences (100 voxels on the surface, 50 one height off it, 50
    anywhere in the column), all in columns whose optimal height is unique
    (h_min = h_max), must equal the gradient exactly: d_up == d_dn ==
    [z == h(p)]."""
    smf, ag = mods
    cost, _, _ = synth.diff_costs(batch=8, n=128, K=128, device="cuda")
    cost = cost.clone().requires_grad_(True)
    print("case: differentiable 8x128^3 delta 2", flush=True)
    E, h = ag.surface_energy(cost, 2)
    gE = torch.linspace(0.5, 2.0, 8, device="cuda")
    (E * gE).sum().backward()
    ci = ag.quantize(cost.detach())
    hs = h.cpu().numpy()
    grad = cost.grad
    ref = torch.zeros_like(grad)
    ref.scatter_(3, h.long()[..., None], gE[:, None, None, None].expand(8, 128, 128, 1))
    assert torch.equal(grad, ref)
    kinds = ["on", "near", "on", "any"] * 50
    rng = np.random.default_rng(11)
    checked = 0
    with smf.Solver(128, 128, 128, 2) as s:
        s.set_param("hmax", 1)

        def certified(c):
            s.solve(c)
            surf = s.surface().cpu().numpy()
            e, ts, fd, fl = (t.cpu().numpy() for t in s.export_state())
            cert = oracle.certify(c.cpu().numpy(), 2, e, ts, fd, fl, surf)
            assert cert.ok, cert
            assert cert.energy == s.energy()
            return s.energy(), surf, ts, fd, fl

        for b in range(8):
            base, surf, ts, fd, fl = certified(ci[b])
            np.testing.assert_array_equal(surf, hs[b])
            assert base / 16.0 == E[b].item()
            hmax = s.surface_max().cpu().numpy()
            np.testing.assert_array_equal(hmax, oracle.hmax_from_preflow(2, ts, fd, fl))
            unique = np.argwhere(hmax == surf)
            assert len(unique) > 1000, len(unique)
            c0 = ci[b].clone()
            for i, j in enumerate(rng.choice(len(unique), 25, replace=False)):
                x, y = (int(v) for v in unique[j])
                hz = int(surf[x, y])
                kind = kinds[25 * b + i]
                if kind == "on":
                    z = hz
                elif kind == "near":
                    z = hz + 1 if (hz + 1 < 128 and rng.integers(2)) or hz == 0 else hz - 1
                else:
                    z = int(rng.integers(0, 128))
                c0[x, y, z] += 1
                d_up = certified(c0)[0] - base
                c0[x, y, z] -= 2
                d_dn = base - certified(c0)[0]
                c0[x, y, z] += 1
                want = int(z == hz)
                assert d_up == d_dn == want, (b, x, y, z, hz, d_up, d_dn)
                assert grad[b, x, y, z].item() == want * gE[b].item()
                checked += 1
    assert checked == 200
