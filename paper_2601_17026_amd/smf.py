"""Python binding of the C-ABI library `_libsmf.so` (declared in include/smf.h).

Argument marshalling only: torch tensors provide device memory and streams,
every step of the solve runs in the library's HIP kernels.  Importing this
module loads the library and raises if it is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_libsmf.so")

OK = 0
ERR_ARG = -1
ERR_NOMEM = -2
ERR_RANGE = -3
ERR_NOT_CONVERGED = -4
ERR_HIP = -5
ERR_NOT_SOLVED = -6

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "or python paper_2601_17026_amd/build.py")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_PI64 = ctypes.POINTER(ctypes.c_int64)

_lib.smf_create.argtypes = [_I32, _I32, _I32, _I32]
_lib.smf_create.restype = _P
_lib.smf_destroy.argtypes = [_P]
_lib.smf_destroy.restype = None
_lib.smf_solve.argtypes = [_P, _P, _P]
_lib.smf_flow_value.argtypes = [_P, _PI64]
_lib.smf_energy.argtypes = [_P, _PI64]
_lib.smf_surface.argtypes = [_P, _P, _P]
_lib.smf_export_state.argtypes = [_P, _P, _P, _P, _P, _P]
_lib.smf_export_soft_flows.argtypes = [_P, _P, _P]
_lib.smf_set_param.argtypes = [_P, ctypes.c_char_p, _I64]
_lib.smf_get_stat.argtypes = [_P, ctypes.c_char_p, _PI64]
_lib.smf_status_string.argtypes = [ctypes.c_int]
_lib.smf_status_string.restype = ctypes.c_char_p
_lib.smf_onehot_backward.argtypes = [_P, _P, _P, _I32, _I32, _I32, _I32, _P]
_lib.smf_onehot_backward.restype = ctypes.c_int
_lib.smf_last_error.argtypes = []
_lib.smf_last_error.restype = ctypes.c_char_p
_PI32 = ctypes.POINTER(ctypes.c_int32)
_lib.smf_batch_create.argtypes = [_I32, _PI32, _PI32, _PI32, _PI32]
_lib.smf_batch_create.restype = _P
_lib.smf_batch_solve.argtypes = [_P, _P, _PI64, _P]
_lib.smf_batch_flow_values.argtypes = [_P, _PI64]
_lib.smf_batch_energies.argtypes = [_P, _PI64]
_lib.smf_batch_surfaces.argtypes = [_P, _P, _P]
_lib.smf_batch_set_param.argtypes = [_P, ctypes.c_char_p, _PI64]
_lib.smf_batch_get_stat.argtypes = [_P, ctypes.c_char_p, _PI64]
_lib.smf_autotune.argtypes = [_P, _P, _PI64, _P]
_lib.smf_tune_apply.argtypes = [_P]
_lib.smf_tune_cache_load.argtypes = [ctypes.c_char_p]
_lib.smf_tune_cache_save.argtypes = [ctypes.c_char_p]
_lib.smf_tune_cache_clear.argtypes = []
_lib.smf_tune_lookup.argtypes = [_I32, _I32, _I32, _I32, _PI64]
_lib.smf_set_band.argtypes = [_P, _P, _P]
_lib.smf_surface_max.argtypes = [_P, _P, _P]
_lib.smf_surface_max.restype = ctypes.c_int
_lib.smf_set_band.restype = ctypes.c_int
_lib.smf_solve_noalloc.argtypes = [_P, _I32, _I32, _I32, _I32, _P, _PI64, _PI64, _P]
_lib.smf_solve_noalloc.restype = ctypes.c_int
NOALLOC_MAX_BYTES = 64 << 20   # SMF_NOALLOC_MAX_BYTES
for _name in ("smf_autotune", "smf_tune_apply", "smf_tune_cache_load", "smf_tune_cache_save",
              "smf_tune_cache_clear", "smf_tune_lookup"):
    getattr(_lib, _name).restype = ctypes.c_int
for _name in ("smf_solve", "smf_flow_value", "smf_energy", "smf_surface",
              "smf_export_state", "smf_export_soft_flows", "smf_set_param", "smf_get_stat",
              "smf_batch_solve",
              "smf_batch_flow_values", "smf_batch_energies", "smf_batch_surfaces",
              "smf_batch_set_param", "smf_batch_get_stat"):
    getattr(_lib, _name).restype = ctypes.c_int

EXPORTED = ("smf_create", "smf_destroy", "smf_solve", "smf_flow_value", "smf_energy",
            "smf_surface", "smf_export_state", "smf_export_soft_flows", "smf_set_param",
            "smf_get_stat",
            "smf_status_string", "smf_last_error", "smf_onehot_backward",
            "smf_batch_create", "smf_batch_solve", "smf_batch_flow_values",
            "smf_batch_energies", "smf_batch_surfaces", "smf_batch_set_param",
            "smf_batch_get_stat", "smf_autotune", "smf_tune_apply", "smf_tune_cache_load",
            "smf_tune_cache_save", "smf_tune_cache_clear", "smf_tune_lookup",
            "smf_solve_noalloc", "smf_set_band", "smf_surface_max")


class SmfError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.smf_last_error().decode() or _lib.smf_status_string(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")


def _check(status: int, where: str) -> None:
    if status != OK:
        raise SmfError(status, where)


def _stream_ptr(stream, device: int) -> int:
    """The HIP stream of `stream` (default: the current stream of `device`),
    which must belong to `device`."""
    if stream is None:
        stream = torch.cuda.current_stream(device)
    elif stream.device.index != device:
        raise ValueError(f"stream is on {stream.device}, the handle on cuda:{device}")
    return int(stream.cuda_stream)


def _on_device(t: torch.Tensor, name: str, device: int) -> None:
    if t.device.index != device:
        raise ValueError(f"{name} is on {t.device}, the handle on cuda:{device}")


def _dev_i32(t: torch.Tensor, shape, name: str, device: int) -> torch.Tensor:
    if t.device.type != "cuda" or t.dtype != torch.int32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous int32 CUDA tensor")
    _on_device(t, name, device)
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _empty(shape, dtype, device: int) -> torch.Tensor:
    """An output buffer on GPU `device`."""
    return torch.empty(shape, dtype=dtype, device=torch.device("cuda", device))


class Solver:
    """One solver handle for nx x ny x K volumes with smoothness bound delta."""

    def __init__(self, nx: int, ny: int, K: int, delta: int):
        self.shape = (int(nx), int(ny), int(K))
        self.delta = int(delta)
        self.n = 1
        h = _lib.smf_create(int(nx), int(ny), int(K), int(delta))
        if not h:
            raise SmfError(ERR_NOMEM, "smf_create")
        self._h = h
        self.device = torch.cuda.current_device()   # the GPU the library allocated on

    def close(self) -> None:
        h = getattr(self, "_h", None)
        self._h = None
        if h and _lib is not None:
            _lib.smf_destroy(h)

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_param(self, key: str, value: int) -> None:
        _check(_lib.smf_set_param(self._h, key.encode(), int(value)), f"smf_set_param({key})")

    def stat(self, key: str) -> int:
        out = ctypes.c_int64()
        _check(_lib.smf_get_stat(self._h, key.encode(), ctypes.byref(out)), f"smf_get_stat({key})")
        return out.value

    def stats(self) -> dict:
        return {k: self.stat(k) for k in
                ("sweeps", "global_relabels", "bfs_passes", "mincut_passes", "gap_relabels")}

    def set_param_per_volume(self, key: str, values) -> None:
        if len(values) != self.n:
            raise ValueError(f"expected {self.n} values, got {len(values)}")
        arr = (ctypes.c_int64 * self.n)(*[int(v) for v in values])
        _check(_lib.smf_batch_set_param(self._h, key.encode(), arr), f"smf_batch_set_param({key})")

    def stat_per_volume(self, key: str) -> list:
        arr = (ctypes.c_int64 * self.n)()
        _check(_lib.smf_batch_get_stat(self._h, key.encode(), arr), f"smf_batch_get_stat({key})")
        return list(arr)

    def solve(self, cost: torch.Tensor, stream=None) -> None:
        _dev_i32(cost, self.shape, "cost", self.device)
        _check(_lib.smf_solve(self._h, cost.data_ptr(), _stream_ptr(stream, self.device)), "smf_solve")

    def flow_value(self) -> int:
        out = ctypes.c_int64()
        _check(_lib.smf_flow_value(self._h, ctypes.byref(out)), "smf_flow_value")
        return out.value

    def energy(self) -> int:
        out = ctypes.c_int64()
        _check(_lib.smf_energy(self._h, ctypes.byref(out)), "smf_energy")
        return out.value

    def surface(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        nx, ny, _ = self.shape
        if out is None:
            out = _empty((nx, ny), torch.int32, self.device)
        _dev_i32(out, (nx, ny), "out", self.device)
        _check(_lib.smf_surface(self._h, out.data_ptr(), _stream_ptr(stream, self.device)), "smf_surface")
        return out

    def surface_max(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """The pointwise-highest optimal surface (needs set_param("hmax", 1)
        before the solve)."""
        nx, ny, _ = self.shape
        if out is None:
            out = _empty((nx, ny), torch.int32, self.device)
        _dev_i32(out, (nx, ny), "out", self.device)
        _check(_lib.smf_surface_max(self._h, out.data_ptr(), _stream_ptr(stream, self.device)),
               "smf_surface_max")
        return out

    def set_band(self, offset, extent) -> None:
        """Narrow band: column (x, y) holds the heights offset[x, y] ..
        offset[x, y] + extent[x, y] - 1 of the volume (host arrays of shape
        (nx, ny)); the costs passed to solve() then hold, at [x, y, j], the
        cost at height offset[x, y] + j.  None, None removes the band."""
        if offset is None and extent is None:
            _check(_lib.smf_set_band(self._h, None, None), "smf_set_band")
            return
        import numpy as np
        nx, ny, _ = self.shape
        o = np.ascontiguousarray(np.asarray(offset), dtype=np.int32)
        e = np.ascontiguousarray(np.asarray(extent), dtype=np.int32)
        if o.shape != (nx, ny) or e.shape != (nx, ny):
            raise ValueError(f"offset and extent must have shape {(nx, ny)}")
        _check(_lib.smf_set_band(self._h, o.ctypes.data, e.ctypes.data), "smf_set_band")

    def export_state(self, stream=None):
        """Final preflow as (excess, sink_res, flow_down, flow_lat) device tensors."""
        nx, ny, K = self.shape
        e, ts, fd = (_empty((nx, ny, K), torch.int32, self.device) for _ in range(3))
        fl = _empty((4, nx, ny, K), torch.int32, self.device)
        _check(_lib.smf_export_state(self._h, e.data_ptr(), ts.data_ptr(), fd.data_ptr(),
                                     fl.data_ptr(), _stream_ptr(stream, self.device)), "smf_export_state")
        return e, ts, fd, fl

    def export_soft_flows(self, stream=None):
        """Flows on the soft smoothness arcs (p,z) -> (q,z) as a (4, nx, ny, K)
        device tensor, neighbour order +x, -x, +y, -y."""
        nx, ny, K = self.shape
        fs = _empty((4, nx, ny, K), torch.int32, self.device)
        _check(_lib.smf_export_soft_flows(self._h, fs.data_ptr(), _stream_ptr(stream, self.device)),
               "smf_export_soft_flows")
        return fs


class BatchSolver:
    """One handle for a batch of volumes of uneven shapes (nx, ny, K, delta),
    solved together: every launch covers all volumes."""

    def __init__(self, shapes):
        shapes = [tuple(int(v) for v in sh) for sh in shapes]
        if not shapes or any(len(sh) != 4 for sh in shapes):
            raise ValueError("shapes must be a non-empty list of (nx, ny, K, delta)")
        self.shapes = shapes
        self.n = len(shapes)
        arr = [(ctypes.c_int32 * self.n)(*[sh[j] for sh in shapes]) for j in range(4)]
        h = _lib.smf_batch_create(self.n, *[ctypes.cast(a, _PI32) for a in arr])
        if not h:
            raise SmfError(ERR_NOMEM, "smf_batch_create")
        self._h = h
        self.device = torch.cuda.current_device()   # the GPU the library allocated on
        self.sizes = [nx * ny * K for nx, ny, K, _ in shapes]
        self.columns = [nx * ny for nx, ny, _, _ in shapes]
        self.offsets = [0]
        for v in self.sizes[:-1]:
            self.offsets.append(self.offsets[-1] + v)
        self.col_offsets = [0]
        for v in self.columns[:-1]:
            self.col_offsets.append(self.col_offsets[-1] + v)

    close = Solver.close
    __del__ = Solver.__del__
    __enter__ = Solver.__enter__
    __exit__ = Solver.__exit__
    set_param = Solver.set_param
    stat = Solver.stat
    stats = Solver.stats

    set_param_per_volume = Solver.set_param_per_volume
    stat_per_volume = Solver.stat_per_volume

    def pack(self, costs) -> torch.Tensor:
        """Packs a list of (nx, ny, K) int32 CUDA volumes into one buffer."""
        if len(costs) != self.n:
            raise ValueError(f"expected {self.n} volumes, got {len(costs)}")
        for c, (nx, ny, K, _) in zip(costs, self.shapes):
            _dev_i32(c, (nx, ny, K), "cost", self.device)
        return torch.cat([c.reshape(-1) for c in costs])

    def solve(self, packed: torch.Tensor, offsets=None, stream=None) -> None:
        """Solves every volume; volume i's costs start at packed[offsets[i]]
        (default: densely packed in order)."""
        if packed.device.type != "cuda" or packed.dtype != torch.int32 or not packed.is_contiguous():
            raise ValueError("packed costs must be a contiguous int32 CUDA tensor")
        _on_device(packed, "packed costs", self.device)
        offs = self.offsets if offsets is None else [int(o) for o in offsets]
        if len(offs) != self.n or any(o < 0 or o + n > packed.numel() for o, n in zip(offs, self.sizes)):
            raise ValueError("cost offsets do not fit the packed buffer")
        arr = (ctypes.c_int64 * self.n)(*offs)
        _check(_lib.smf_batch_solve(self._h, packed.data_ptr(), arr, _stream_ptr(stream, self.device)),
               "smf_batch_solve")

    def flow_values(self) -> list:
        arr = (ctypes.c_int64 * self.n)()
        _check(_lib.smf_batch_flow_values(self._h, arr), "smf_batch_flow_values")
        return list(arr)

    def energies(self) -> list:
        arr = (ctypes.c_int64 * self.n)()
        _check(_lib.smf_batch_energies(self._h, arr), "smf_batch_energies")
        return list(arr)

    def surfaces(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Packed surfaces: volume i's (nx, ny) heights at col_offsets[i]."""
        total = sum(self.columns)
        if out is None:
            out = _empty((total,), torch.int32, self.device)
        _dev_i32(out, (total,), "out", self.device)
        _check(_lib.smf_batch_surfaces(self._h, out.data_ptr(), _stream_ptr(stream, self.device)),
               "smf_batch_surfaces")
        return out

    def surfaces_max(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Packed pointwise-highest optimal surfaces (set_param("hmax", 1))."""
        total = sum(self.columns)
        if out is None:
            out = _empty((total,), torch.int32, self.device)
        _dev_i32(out, (total,), "out", self.device)
        _check(_lib.smf_surface_max(self._h, out.data_ptr(), _stream_ptr(stream, self.device)),
               "smf_surface_max")
        return out

    def unpack_surfaces(self, packed: torch.Tensor) -> list:
        return [packed[o:o + nx * ny].view(nx, ny)
                for o, (nx, ny, _, _) in zip(self.col_offsets, self.shapes)]

    def export_state(self, stream=None):
        """Final packed preflow as flat (excess, sink_res, flow_down, flow_lat)
        device tensors; flow_lat is (4, total nodes)."""
        total = sum(self.sizes)
        e, ts, fd = (_empty((total,), torch.int32, self.device) for _ in range(3))
        fl = _empty((4, total), torch.int32, self.device)
        _check(_lib.smf_export_state(self._h, e.data_ptr(), ts.data_ptr(), fd.data_ptr(),
                                     fl.data_ptr(), _stream_ptr(stream, self.device)), "smf_export_state")
        return e, ts, fd, fl

    def export_soft_flows(self, stream=None):
        """Flows on the soft smoothness arcs as a (4, total nodes) device tensor."""
        fs = _empty((4, sum(self.sizes)), torch.int32, self.device)
        _check(_lib.smf_export_soft_flows(self._h, fs.data_ptr(), _stream_ptr(stream, self.device)),
               "smf_export_soft_flows")
        return fs


def autotune(solver, packed: torch.Tensor, offsets=None, stream=None) -> None:
    """Times candidate relabel periods per volume class (smf_autotune) and
    gives every volume of `solver` (a Solver or BatchSolver) its class's
    period.  `packed` is the volume (Solver) or the packed batch costs."""
    if packed.device.type != "cuda" or packed.dtype != torch.int32 or not packed.is_contiguous():
        raise ValueError("costs must be a contiguous int32 CUDA tensor")
    _on_device(packed, "costs", solver.device)
    arr = None
    if offsets is not None:
        arr = (ctypes.c_int64 * len(offsets))(*[int(o) for o in offsets])
    elif isinstance(solver, BatchSolver):
        arr = (ctypes.c_int64 * solver.n)(*solver.offsets)
    _check(_lib.smf_autotune(solver._h, packed.data_ptr(), arr, _stream_ptr(stream, solver.device)),
           "smf_autotune")


def tune_apply(solver) -> None:
    _check(_lib.smf_tune_apply(solver._h), "smf_tune_apply")


def tune_cache_load(path: str) -> None:
    _check(_lib.smf_tune_cache_load(os.fsencode(path)), "smf_tune_cache_load")


def tune_cache_save(path: str) -> None:
    _check(_lib.smf_tune_cache_save(os.fsencode(path)), "smf_tune_cache_save")


def tune_cache_clear() -> None:
    _check(_lib.smf_tune_cache_clear(), "smf_tune_cache_clear")


def tune_lookup(nx: int, ny: int, K: int, delta: int) -> int:
    out = ctypes.c_int64()
    _check(_lib.smf_tune_lookup(int(nx), int(ny), int(K), int(delta), ctypes.byref(out)),
           "smf_tune_lookup")
    return out.value


def onehot_backward(surface: torch.Tensor, grad_energy: torch.Tensor, K: int,
                    out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """grad[b, x, y, z] = grad_energy[b] * [z == surface[b, x, y]] (device tensors)."""
    if surface.dim() != 3:
        raise ValueError("surface must be (n, nx, ny)")
    n, nx, ny = surface.shape
    if surface.device.type != "cuda":
        raise ValueError("surface must be a CUDA tensor")
    device = surface.device.index
    _dev_i32(surface, (n, nx, ny), "surface", device)
    if grad_energy.device.type != "cuda" or grad_energy.dtype != torch.float32 \
            or not grad_energy.is_contiguous() or tuple(grad_energy.shape) != (n,):
        raise ValueError("grad_energy must be a contiguous float32 CUDA tensor of shape (n,)")
    _on_device(grad_energy, "grad_energy", device)
    if out is None:
        out = _empty((n, nx, ny, int(K)), torch.float32, device)
    elif out.device.type != "cuda" or out.dtype != torch.float32 or not out.is_contiguous() \
            or tuple(out.shape) != (n, nx, ny, int(K)):
        raise ValueError(f"out must be a contiguous float32 CUDA tensor of shape {(n, nx, ny, int(K))}")
    _on_device(out, "out", device)
    with torch.cuda.device(device):   # the kernel runs on the surface's GPU
        _check(_lib.smf_onehot_backward(surface.data_ptr(), grad_energy.data_ptr(), out.data_ptr(),
                                        n, nx, ny, int(K), _stream_ptr(stream, device)),
               "smf_onehot_backward")
    return out


def solve(cost: torch.Tensor, delta: int, stream=None):
    """Solves one (nx, ny, K) int32 CUDA volume; returns (flow, energy, surface)."""
    if cost.device.type != "cuda":
        raise ValueError("cost must be a CUDA tensor")
    with torch.cuda.device(cost.device.index):   # the handle lives on the volume's GPU
        with Solver(*cost.shape, delta) as s:
            s.solve(cost, stream)
            surf = s.surface(stream=stream)
            return s.flow_value(), s.energy(), surf


def solve_noalloc(cost: torch.Tensor, delta: int, surface: torch.Tensor | None = None, stream=None):
    """Solves one (nx, ny, K) int32 CUDA volume through the allocation-free
    entry point (all solver state in the library's static device workspace);
    returns (flow, energy, surface).  `surface` is an optional (nx, ny) int32
    output on the volume's GPU; without it one is allocated here (by torch,
    outside the library call)."""
    if cost.device.type != "cuda":
        raise ValueError("cost must be a CUDA tensor")
    dev = cost.device.index
    nx, ny, K = (int(v) for v in cost.shape)
    _dev_i32(cost, (nx, ny, K), "cost", dev)
    out = _empty((nx, ny), torch.int32, dev) if surface is None else \
        _dev_i32(surface, (nx, ny), "surface", dev)
    flow, energy = ctypes.c_int64(), ctypes.c_int64()
    with torch.cuda.device(dev):
        _check(_lib.smf_solve_noalloc(cost.data_ptr(), nx, ny, K, int(delta), out.data_ptr(),
                                      ctypes.byref(flow), ctypes.byref(energy), _stream_ptr(stream, dev)),
               "smf_solve_noalloc")
    return flow.value, energy.value, out
