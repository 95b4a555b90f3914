"""Seeded synthetic cost volumes for the multi-column surface problem.

The paper measures on two seismic volumes (Section 3.4, Table 1) that are not
available; these generators stand in for them with the same structure: a
column-major int32 cost volume c[x, y, z] (z fastest) that is low along a few
smooth nested horizons and high elsewhere (Section 1.1, Eq. 1: the feature
term is a per-voxel cost summed along the surface).

This module is shared by the HIP path's tests and benchmarks and by the CPU
oracle's golden-value scripts.  It holds no arithmetic of the max-flow method
itself: it only draws random numbers and shapes them into costs.

Determinism: every value is produced from numpy's PCG64 streams and plain IEEE
add/multiply/abs/rint; the only transcendental calls go through Python's
`math.sin`/`math.cos` on 1-D axes (never numpy's vectorised sin, whose SIMD
dispatch can differ between host CPUs), so the same seed gives the same bytes
on every x86-64 host with this image.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

__all__ = [
    "layered_intensity",
    "layered_cost",
    "random_cost",
    "config_small",
    "config_mid",
    "config_seismic",
    "batch_shapes",
    "batch_instance",
    "diff_costs",
    "sha256",
]

TWO_PI = 2.0 * math.pi


def _axis_trig(n: int, f: float, phase: float):
    a = [TWO_PI * f * i / n + phase for i in range(n)]
    return (np.array([math.sin(t) for t in a], dtype=np.float64),
            np.array([math.cos(t) for t in a], dtype=np.float64))


def _surfaces(nx: int, ny: int, K: int, nsurf: int, rng) -> list:
    """Nested integer height maps h_i(x, y), i = 0..nsurf-1, lowest first."""
    out = []
    span = 0.75 * K
    for i in range(nsurf):
        s = np.zeros((nx, ny), dtype=np.float64)
        for _ in range(3):
            fx = rng.uniform(0.5, 2.0)
            fy = rng.uniform(0.5, 2.0)
            phi = rng.uniform(0.0, TWO_PI)
            # sin(Ax + By) = sin(Ax)cos(By) + cos(Ax)sin(By), Ax carrying the phase.
            sa, ca = _axis_trig(nx, fx, phi)
            sb, cb = _axis_trig(ny, fy, 0.0)
            s = s + (np.multiply.outer(sa, cb) + np.multiply.outer(ca, sb))
        lo, hi = float(s.min()), float(s.max())
        s = (s - lo) / (hi - lo) * 2.0 - 1.0 if hi > lo else np.zeros_like(s)
        if nsurf == 1:
            off, amp = K / 2.0, 3.0 * K / 8.0
        else:
            off = K / 8.0 + (i + 0.5) * span / nsurf
            amp = 0.4 * span / nsurf
        out.append(np.rint(off + amp * s).astype(np.int64))
    return out


def layered_intensity(nx, ny, K, nsurf, sigma, seed):
    """Noisy layered intensity I[x, y, z] (float64) and the planted heights.

    I = sum_i a_i [z < h_i] + N(0, sigma^2), a_0 = 1, a_i ~ U[0.5, 0.9].
    Returns (I, heights) with heights a list of (nx, ny) int64 arrays.
    """
    rng = np.random.default_rng(seed)
    hs = _surfaces(nx, ny, K, nsurf, rng)
    amps = [1.0] + [float(v) for v in rng.uniform(0.5, 0.9, size=max(0, nsurf - 1))]
    z = np.arange(K, dtype=np.int64)
    I = np.empty((nx, ny, K), dtype=np.float64)
    for x in range(nx):
        slab = np.zeros((ny, K), dtype=np.float64)
        for h, a in zip(hs, amps):
            slab += a * (z[None, :] < h[x][:, None])
        if sigma > 0:
            nrng = np.random.default_rng([seed, 1, x])
            slab += sigma * nrng.standard_normal((ny, K))
        I[x] = slab
    return I, hs


def layered_cost(nx, ny, K, nsurf, sigma, cmax, fault, seed, heights=False):
    """int32 cost c[x, y, z] in [0, cmax], low where the intensity jumps.

    D(z) = |I(z) - I(z-1)| (D(0) = 0); c = rint(cmax (1 - D / max D)).
    A fraction `fault` of the columns is replaced by iid U{0..cmax} costs.
    heights=True also returns the planted heights (lowest first).
    """
    I, hs = layered_intensity(nx, ny, K, nsurf, sigma, seed)
    D = np.zeros_like(I)
    np.abs(I[:, :, 1:] - I[:, :, :-1], out=D[:, :, 1:])
    del I
    m = float(D.max())
    if m > 0:
        D /= m
    np.subtract(1.0, D, out=D)
    D *= float(cmax)
    c = np.rint(D).astype(np.int32)
    del D
    if fault > 0:
        frng = np.random.default_rng([seed, 2])
        mask = frng.uniform(size=(nx, ny)) < fault
        cols = int(mask.sum())
        if cols:
            c[mask] = frng.integers(0, cmax + 1, size=(cols, K), dtype=np.int32)
    c = np.ascontiguousarray(c)
    return (c, hs) if heights else c


def random_cost(nx, ny, K, lo, hi, seed):
    """iid uniform integer costs in [lo, hi] (may be negative)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(nx, ny, K), dtype=np.int64).astype(np.int32)


# ---- the named workloads -------------------------------------------------

def config_small(seed=1):
    """32x32 columns x K=64, delta=2, one planted surface in [8, 56], sigma 0.3."""
    return layered_cost(32, 32, 64, 1, 0.3, 255, 0.0, seed), 2


def config_mid(seed=2):
    """256x256 columns x K=256, delta=1, two planted surfaces, sigma 0.5."""
    return layered_cost(256, 256, 256, 2, 0.5, 255, 0.0, seed), 1


def config_seismic(seed=3, heights=False):
    """512x512 columns x K=384, delta=2, five nested surfaces, sigma 0.4,
    costs in [0, 1023], 10% of columns uniformly random (faults).
    heights=True: (cost, delta, planted heights)."""
    if heights:
        c, hs = layered_cost(512, 512, 384, 5, 0.4, 1023, 0.10, seed, heights=True)
        return c, 2, hs
    return layered_cost(512, 512, 384, 5, 0.4, 1023, 0.10, seed), 2


def batch_shapes(n=64, seed=4000):
    """Shapes (nx, ny, K) ~ U{64..256} and delta ~ U{1,2,3} for a batch."""
    rng = np.random.default_rng(seed)
    shp = rng.integers(64, 257, size=(n, 3))
    dl = rng.integers(1, 4, size=n)
    return [(int(a), int(b), int(c), int(d)) for (a, b, c), d in zip(shp, dl)]


def batch_instance(i, shape):
    nx, ny, K, delta = shape
    return layered_cost(nx, ny, K, 2, 0.4, 255, 0.0, 4001 + i), delta


def diff_costs(batch=8, n=128, K=128, seed0=5001, net_seed=5000, device="cuda"):
    """Float costs of the differentiable workload: a batch of noisy layered
    intensities (two horizons, sigma 0.3) through a seeded 3-layer 3x3x3
    convolution net (1 -> 16 -> 16 -> 1 channels, ReLU between, fp32),
    standardised per volume to mean 0 and std 4.  Returns the (B, n, n, K)
    costs (no autograd history), the net and its (B, 1, n, n, K) input."""
    import torch

    torch.manual_seed(net_seed)
    net = torch.nn.Sequential(
        torch.nn.Conv3d(1, 16, 3, padding=1), torch.nn.ReLU(),
        torch.nn.Conv3d(16, 16, 3, padding=1), torch.nn.ReLU(),
        torch.nn.Conv3d(16, 1, 3, padding=1)).to(device)
    vols = [layered_intensity(n, n, K, 2, 0.3, seed0 + b)[0] for b in range(batch)]
    x = torch.from_numpy(np.stack(vols).astype(np.float32))[:, None].to(device)
    with torch.no_grad():
        y = net(x)[:, 0]
    mu = y.mean(dim=(1, 2, 3), keepdim=True)
    sd = y.std(dim=(1, 2, 3), keepdim=True).clamp_min(1e-6)
    return ((y - mu) / sd * 4.0).contiguous(), net, x


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ---- narrow bands around landmarks (Section 3.4) ------------------------------
#
# The user marks landmark points on the horizon; the graph covers a stick of
# heights above and below the surface they outline.  Here the landmarks are
# the planted horizon's heights on a coarse grid of columns, the outlined
# surface is their bilinear interpolation, and every column holds
# 2 * stick + 1 heights centred on it (fewer where the volume ends).


def landmark_reference(h: np.ndarray, step: int) -> np.ndarray:
    """Bilinear interpolation of h sampled every `step` columns in x and y
    (the last row and column always sampled), rounded to heights."""
    nx, ny = h.shape
    xs = sorted(set(list(range(0, nx, step)) + [nx - 1]))
    ys = sorted(set(list(range(0, ny, step)) + [ny - 1]))
    marks = h[np.ix_(xs, ys)].astype(np.float64)
    out = np.empty((nx, ny), dtype=np.float64)
    for x in range(nx):
        i = max(0, min(len(xs) - 2, int(np.searchsorted(xs, x, side="right")) - 1)) if len(xs) > 1 else 0
        tx = 0.0 if len(xs) == 1 else (x - xs[i]) / (xs[i + 1] - xs[i])
        row = marks[i] if len(xs) == 1 else (1 - tx) * marks[i] + tx * marks[i + 1]
        out[x] = np.interp(np.arange(ny), ys, row)
    return np.rint(out).astype(np.int64)


def band_from_reference(cost: np.ndarray, ref: np.ndarray, stick: int):
    """(band costs [nx][ny][2 stick + 1], offsets, extents): column (x, y)
    holds the heights off .. off + ext - 1 around ref(x, y), clipped to the
    volume; band[x, y, j] = cost[x, y, off + j] (padding beyond ext: 0)."""
    nx, ny, K = cost.shape
    width = 2 * stick + 1
    off = np.clip(ref - stick, 0, K - 1).astype(np.int32)
    ext = np.minimum(ref + stick + 1, K).astype(np.int64) - off
    ext = np.clip(ext, 1, width).astype(np.int32)
    band = np.zeros((nx, ny, width), dtype=np.int32)
    for x in range(nx):
        for y in range(ny):
            band[x, y, :ext[x, y]] = cost[x, y, off[x, y]:off[x, y] + ext[x, y]]
    return band, off, ext


def config_seismic_band(seed=3, stick=48, step=32, horizon=2, seismic=None):
    """The seismic volume (512 x 512 x 384, delta = 2) restricted to a band of
    2 * stick + 1 heights around the landmark surface of planted horizon
    `horizon` (landmarks every `step` columns).  `seismic`: the (cost,
    delta, heights) of config_seismic(heights=True) if already made."""
    cost, delta, hs = seismic if seismic is not None else config_seismic(seed, heights=True)
    band, off, ext = band_from_reference(cost, landmark_reference(hs[horizon], step), stick)
    return band, off, ext, delta
