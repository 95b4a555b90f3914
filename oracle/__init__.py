"""CPU oracle for the exact surface max-flow -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never calls it.

`solve(cost, delta, alpha=0)` returns the max-flow value, the minimal and
maximal minimum-cut surfaces and the optimal energy of an int32 cost volume
c[x, y, z] (z fastest), computed by Dinic's method on the explicit s-t graph
(oracle.c); alpha > 0 adds the soft smoothness term.  `certify(...)` checks a solver's final preflow against the
max-flow/min-cut certificate (certify.c).  Both are plain C built with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_SOURCES = ["oracle.c", "certify.c"]
_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle's C sources into _liboracle.so with gcc."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", _LIB_PATH + ".tmp", *srcs]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Result(ctypes.Structure):
    _fields_ = [
        ("flow", ctypes.c_int64),
        ("cut", ctypes.c_int64),
        ("energy", ctypes.c_int64),
        ("energy_hmax", ctypes.c_int64),
        ("wminus", ctypes.c_int64),
        ("phases", ctypes.c_int64),
        ("conservation_ok", ctypes.c_int32),
        ("capacity_ok", ctypes.c_int32),
        ("smin_in_smax", ctypes.c_int32),
        ("status", ctypes.c_int32),
    ]


class _Cert(ctypes.Structure):
    _fields_ = [
        ("flow", ctypes.c_int64),
        ("cut", ctypes.c_int64),
        ("energy", ctypes.c_int64),
        ("bad_capacity", ctypes.c_int64),
        ("bad_conservation", ctypes.c_int64),
        ("bad_smooth", ctypes.c_int64),
        ("bad_reach", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_solve.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, P, P, ctypes.POINTER(_Result)]
        lib.oracle_solve.restype = ctypes.c_int
        lib.oracle_solve_soft.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, P, P,
                                          ctypes.POINTER(_Result)]
        lib.oracle_solve_soft.restype = ctypes.c_int
        lib.certify_preflow.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, P, P, P, P, P,
                                        ctypes.POINTER(_Cert)]
        lib.certify_preflow.restype = ctypes.c_int
        lib.certify_preflow_soft.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P,
                                             ctypes.POINTER(_Cert)]
        lib.certify_preflow_soft.restype = ctypes.c_int
        lib.certify_hmax.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, P, P, P, P]
        lib.certify_hmax.restype = ctypes.c_int
        lib.band_effective.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, P, P, P, P]
        lib.band_effective.restype = ctypes.c_int
        lib.oracle_solve_band.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, P, P, P, P, P, P,
                                          ctypes.POINTER(_Result)]
        lib.oracle_solve_band.restype = ctypes.c_int
        lib.certify_preflow_band.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, P, P, P, P, P, P, P,
                                             ctypes.POINTER(_Cert)]
        lib.certify_preflow_band.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class OracleResult:
    flow: int          # max-flow value |f| (Eq. 5)
    cut: int           # capacity of the minimal min cut (Eq. 6)
    energy: int        # E* = sum_p c(p, h_min(p)) (+ alpha * sum |h(p) - h(q)|)
    energy_hmax: int   # sum_p c(p, h_max(p)) (equal to E* when correct)
    wminus: int        # total source-arc capacity
    phases: int        # Dinic phases
    hmin: np.ndarray   # (nx, ny) int32, pointwise-lowest optimal surface
    hmax: np.ndarray   # (nx, ny) int32, pointwise-highest optimal surface
    conservation_ok: bool
    capacity_ok: bool
    smin_in_smax: bool


def solve(cost: np.ndarray, delta: int, alpha: int = 0) -> OracleResult:
    """alpha > 0 adds the soft smoothness term alpha * sum |h(p) - h(q)| over
    4-neighbour column pairs (finite arcs (p,z) -> (q,z), z >= 1)."""
    c = np.ascontiguousarray(cost, dtype=np.int32)
    if c.ndim != 3:
        raise ValueError("cost must be (nx, ny, K)")
    nx, ny, K = c.shape
    hmin = np.empty((nx, ny), dtype=np.int32)
    hmax = np.empty((nx, ny), dtype=np.int32)
    r = _Result()
    rc = _load().oracle_solve_soft(c.ctypes.data, nx, ny, K, int(delta), int(alpha),
                                   hmin.ctypes.data, hmax.ctypes.data, ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"oracle_solve failed with status {rc}")
    return OracleResult(r.flow, r.cut, r.energy, r.energy_hmax, r.wminus, r.phases,
                        hmin, hmax, bool(r.conservation_ok), bool(r.capacity_ok),
                        bool(r.smin_in_smax))


@dataclass
class Certificate:
    flow: int              # sum of flow into the sink
    cut: int               # capacity of the cut given by the surface
    energy: int            # sum_p c(p, h(p))
    bad_capacity: int      # arcs/nodes violating a capacity or sign bound
    bad_conservation: int  # nodes whose excess does not balance
    bad_smooth: int        # neighbour pairs with |h(p) - h(q)| > delta
    bad_reach: int         # columns where h differs from the residual reach set

    @property
    def ok(self) -> bool:
        return (self.bad_capacity == 0 and self.bad_conservation == 0
                and self.bad_smooth == 0 and self.bad_reach == 0
                and self.flow == self.cut)


def certify(cost, delta, excess, sink_res, flow_down, flow_lat, surface, alpha=0,
            flow_soft=None) -> Certificate:
    """Check a final preflow of the implicit column graph and a surface.
    With alpha > 0, flow_soft (4, nx, ny, K) holds the flows on the soft
    arcs (p,z) -> (q,z) of capacity alpha, neighbour order +x, -x, +y, -y,
    and the energy includes alpha * |h(p) - h(q)|.

    excess, sink_res, flow_down: (nx, ny, K) int32; flow_lat: (4, nx, ny, K)
    int32 in the neighbour order +x, -x, +y, -y; surface: (nx, ny) int32.
    The arc set is the one the GPU solver stores (documented in
    include/smf.h): (p,z)->(p,z-1) for z>=1 and (p,z)->(q,z-delta) for
    z>delta (plus (p,0)->(q,0)); it has the same closed sets as G(c, delta).
    """
    c = np.ascontiguousarray(cost, dtype=np.int32)
    nx, ny, K = c.shape
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in
            (excess, sink_res, flow_down, flow_lat, surface)]
    r = _Cert()
    if alpha:
        fs = np.ascontiguousarray(flow_soft, dtype=np.int32)
        if fs.shape != (4, nx, ny, K):
            raise ValueError("flow_soft must be (4, nx, ny, K)")
        rc = _load().certify_preflow_soft(c.ctypes.data, nx, ny, K, int(delta), int(alpha),
                                          *[a.ctypes.data for a in arrs[:4]], fs.ctypes.data,
                                          arrs[4].ctypes.data, ctypes.byref(r))
    else:
        rc = _load().certify_preflow(c.ctypes.data, nx, ny, K, int(delta),
                                     *[a.ctypes.data for a in arrs], ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"certify_preflow failed with status {rc}")
    return Certificate(r.flow, r.cut, r.energy, r.bad_capacity, r.bad_conservation,
                       r.bad_smooth, r.bad_reach)


def hmax_from_preflow(delta, sink_res, flow_down, flow_lat) -> np.ndarray:
    """The pointwise-highest optimal surface read off a maximum preflow of the
    plain graph (certify.c, certify_hmax): per column the highest node that
    cannot reach t in the residual graph.  Arrays as for certify()."""
    ts = np.ascontiguousarray(sink_res, dtype=np.int32)
    nx, ny, K = ts.shape
    fd = np.ascontiguousarray(flow_down, dtype=np.int32)
    fl = np.ascontiguousarray(flow_lat, dtype=np.int32)
    out = np.empty((nx, ny), dtype=np.int32)
    rc = _load().certify_hmax(nx, ny, K, int(delta), ts.ctypes.data, fd.ctypes.data,
                              fl.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"certify_hmax failed with status {rc}")
    return out


# ---- narrow-band volumes (Section 3.4) ---------------------------------------
#
# Column p holds the heights off[p] .. off[p] + ext[p] - 1 of the volume; the
# band costs are cost[x, y, j] = cost at height off[x, y] + j for j < ext[x, y]
# (the array is padded to K >= max ext; padding is not read).  A surface takes
# one height per column inside its band, |h(p) - h(q)| <= delta for
# 4-neighbours.  Heights are reported as heights of the volume.


def _band_arrays(off, ext, nx, ny):
    o = np.ascontiguousarray(off, dtype=np.int32)
    e = np.ascontiguousarray(ext, dtype=np.int32)
    if o.shape != (nx, ny) or e.shape != (nx, ny):
        raise ValueError("off and ext must be (nx, ny)")
    return o, e


def band_effective(off, ext, delta: int, K: int | None = None):
    """(lo, hi): the heights that some delta-smooth surface inside the bands
    takes in each column, or None when no such surface exists."""
    o = np.ascontiguousarray(off, dtype=np.int32)
    nx, ny = o.shape
    o, e = _band_arrays(off, ext, nx, ny)
    lo = np.empty((nx, ny), dtype=np.int32)
    hi = np.empty((nx, ny), dtype=np.int32)
    rc = _load().band_effective(nx, ny, int(K if K is not None else e.max()), int(delta),
                                o.ctypes.data, e.ctypes.data, lo.ctypes.data, hi.ctypes.data)
    if rc < 0:
        raise ValueError("bad band arguments")
    return None if rc else (lo, hi)


@dataclass
class BandResult:
    flow: int          # max-flow value of the band graph (Eq. 5)
    cut: int           # capacity of its minimal min cut (Eq. 6)
    energy: int        # E* = sum_p c(p, h_min(p))
    energy_hmax: int   # sum_p c(p, h_max(p))
    hmin: np.ndarray   # (nx, ny) heights of the volume, pointwise-lowest optimum
    hmax: np.ndarray   # (nx, ny) pointwise-highest optimum
    lo: np.ndarray     # (nx, ny) lowest feasible height per column
    hi: np.ndarray     # (nx, ny) highest feasible height per column
    conservation_ok: bool
    capacity_ok: bool
    smin_in_smax: bool


class NoFeasibleSurface(ValueError):
    """No delta-smooth surface fits the bands."""


def solve_band(cost: np.ndarray, delta: int, off, ext) -> BandResult:
    c = np.ascontiguousarray(cost, dtype=np.int32)
    nx, ny, K = c.shape
    o, e = _band_arrays(off, ext, nx, ny)
    outs = [np.empty((nx, ny), dtype=np.int32) for _ in range(4)]
    r = _Result()
    rc = _load().oracle_solve_band(c.ctypes.data, nx, ny, K, int(delta), o.ctypes.data,
                                   e.ctypes.data, *[a.ctypes.data for a in outs], ctypes.byref(r))
    if rc == -3:
        raise NoFeasibleSurface("no delta-smooth surface fits the bands")
    if rc != 0:
        raise RuntimeError(f"oracle_solve_band failed with status {rc}")
    lo, hi, hmin, hmax = outs
    return BandResult(r.flow, r.cut, r.energy, r.energy_hmax, hmin, hmax, lo, hi,
                      bool(r.conservation_ok), bool(r.capacity_ok), bool(r.smin_in_smax))


def certify_band(cost, delta, off, ext, excess, sink_res, flow_down, flow_lat,
                 surface) -> Certificate:
    """Check a final preflow of a band solve.  The state arrays hold node
    (p, lo(p) + j) at [x, y, j] (lo from band_effective; slots above hi(p) -
    lo(p) unused), flow_lat is (4, nx, ny, K) in the order +x, -x, +y, -y;
    the surface holds heights of the volume."""
    c = np.ascontiguousarray(cost, dtype=np.int32)
    nx, ny, K = c.shape
    o, e = _band_arrays(off, ext, nx, ny)
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in
            (excess, sink_res, flow_down, flow_lat, surface)]
    r = _Cert()
    rc = _load().certify_preflow_band(c.ctypes.data, nx, ny, K, int(delta), o.ctypes.data,
                                      e.ctypes.data, *[a.ctypes.data for a in arrs],
                                      ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"certify_preflow_band failed with status {rc}")
    return Certificate(r.flow, r.cut, r.energy, r.bad_capacity, r.bad_conservation,
                       r.bad_smooth, r.bad_reach)
