"""The Python binding's argument marshalling, on the CPU (no GPU).

The C library is replaced by a recorder that returns success, and device
tensors and streams by small stand-ins that carry a device index, a dtype, a
shape and a pointer.  Every method of Solver and BatchSolver and the
module-level calls then run line by line, and the test checks what reaches
the C-ABI:
  - the pointers of the caller's tensors, the handle and the stream;
  - outputs allocated with the right shape and dtype on the handle's GPU;
  - batch offsets passed through, or the dense default;
  - tensors or streams on another GPU, of the wrong dtype or shape, or not
    contiguous, rejected before any call.
"""
import contextlib
import ctypes
import gc

import numpy as np
import pytest

torch = pytest.importorskip("torch")
smf = pytest.importorskip("paper_2601_17026_amd.smf")
from paper_2601_17026_amd import autograd  # noqa: E402


class FakeTensor:
    _next_ptr = 0x100000

    def __init__(self, shape, dtype=torch.int32, device=0, contiguous=True):
        self.shape = tuple(int(v) for v in shape)
        self.dtype = dtype
        self.device = torch.device("cuda", device)
        self._contiguous = contiguous
        FakeTensor._next_ptr += 0x10000
        self._ptr = FakeTensor._next_ptr

    def is_contiguous(self):
        return self._contiguous

    def data_ptr(self):
        return self._ptr

    def numel(self):
        return int(np.prod(self.shape))

    def dim(self):
        return len(self.shape)


class FakeStream:
    def __init__(self, device):
        self.device = torch.device("cuda", device)
        self.cuda_stream = 0xA00 + device


class FakeLib:
    """Records every C-ABI call; creates handles, fills outputs with 7s."""

    def __init__(self):
        self.calls = []
        self.handles = set()

    def __getattr__(self, name):
        if name.startswith("__"):
            raise AttributeError(name)

        def fn(*args):
            self.calls.append((name, args))
            if name in ("smf_create", "smf_batch_create"):
                h = 0x5000 + 16 * len(self.handles)
                self.handles.add(h)
                return h
            if name in ("smf_last_error", "smf_status_string"):
                return b""
            if name in ("smf_flow_value", "smf_energy", "smf_get_stat", "smf_tune_lookup"):
                args[-1]._obj.value = 7
            if name in ("smf_batch_flow_values", "smf_batch_energies", "smf_batch_get_stat"):
                for i in range(len(args[-1])):
                    args[-1][i] = 7 + i
            return 0
        return fn

    def last(self, name):
        return [a for n, a in self.calls if n == name][-1]


@pytest.fixture
def fake(monkeypatch):
    lib = FakeLib()
    current = {"dev": 0, "entered": []}

    @contextlib.contextmanager
    def device_ctx(d):
        d = d.index if isinstance(d, torch.device) else int(d)
        prev, current["dev"] = current["dev"], d
        current["entered"].append(d)
        try:
            yield
        finally:
            current["dev"] = prev

    monkeypatch.setattr(smf, "_lib", lib)
    monkeypatch.setattr(smf, "_empty", lambda shape, dtype, device: FakeTensor(shape, dtype, device))
    monkeypatch.setattr(torch.cuda, "current_device", lambda: current["dev"])
    monkeypatch.setattr(torch.cuda, "current_stream",
                        lambda device=None: FakeStream(current["dev"] if device is None else int(device)))
    monkeypatch.setattr(torch.cuda, "device", device_ctx)
    lib.current = current
    yield lib
    # no handle of the recorder may reach the real library's destroy call
    for key in [k for k, s in autograd._SOLVERS.items() if getattr(s, "_h", None) in lib.handles]:
        autograd._SOLVERS[key]._h = None
        del autograd._SOLVERS[key]
    for o in gc.get_objects():
        if type(o) in (smf.Solver, smf.BatchSolver) and getattr(o, "_h", None) in lib.handles:
            o._h = None


def test_solver_marshalling(fake):
    s = smf.Solver(5, 4, 70, 2)
    assert fake.last("smf_create") == (5, 4, 70, 2) and s.device == 0
    cost = FakeTensor((5, 4, 70))
    s.solve(cost)
    assert fake.last("smf_solve") == (s._h, cost.data_ptr(), 0xA00)
    s.solve(cost, stream=FakeStream(0))
    assert s.flow_value() == 7 and s.energy() == 7 and s.stat("sweeps") == 7
    assert set(s.stats()) == {"sweeps", "global_relabels", "bfs_passes", "mincut_passes", "gap_relabels"}
    s.set_param("relabel_period", 6)
    assert fake.last("smf_set_param") == (s._h, b"relabel_period", 6)
    s.set_param_per_volume("smooth_weight", [3])
    assert list(fake.last("smf_batch_set_param")[2]) == [3]
    assert s.stat_per_volume("K") == [7]

    surf = s.surface()
    assert (surf.shape, surf.dtype, surf.device) == ((5, 4), torch.int32, torch.device("cuda", 0))
    assert fake.last("smf_surface") == (s._h, surf.data_ptr(), 0xA00)
    mine = FakeTensor((5, 4))
    assert s.surface(out=mine) is mine

    e, ts, fd, fl = s.export_state()
    assert [t.shape for t in (e, ts, fd, fl)] == [(5, 4, 70)] * 3 + [(4, 5, 4, 70)]
    assert len({t.data_ptr() for t in (e, ts, fd, fl)}) == 4
    assert fake.last("smf_export_state") == (s._h, e.data_ptr(), ts.data_ptr(), fd.data_ptr(),
                                             fl.data_ptr(), 0xA00)
    fs = s.export_soft_flows()
    assert fs.shape == (4, 5, 4, 70) and fake.last("smf_export_soft_flows") == (s._h, fs.data_ptr(), 0xA00)
    h = s._h
    s.close()
    assert fake.last("smf_destroy") == (h,) and s._h is None


@pytest.mark.parametrize("bad", [
    FakeTensor((5, 4, 70), device=1),                     # another GPU
    FakeTensor((5, 4, 70), dtype=torch.float32),          # wrong dtype
    FakeTensor((5, 4, 69)),                               # wrong shape
    FakeTensor((5, 4, 70), contiguous=False),             # strided
])
def test_solver_rejects_bad_cost(fake, bad):
    with smf.Solver(5, 4, 70, 2) as s:
        n = len(fake.calls)
        with pytest.raises(ValueError):
            s.solve(bad)
        assert len(fake.calls) == n, "nothing reaches the library"


def test_solver_rejects_other_gpu_outputs_and_streams(fake):
    with smf.Solver(5, 4, 70, 2) as s:
        with pytest.raises(ValueError, match="cuda:1"):
            s.surface(out=FakeTensor((5, 4), device=1))
        with pytest.raises(ValueError, match="stream"):
            s.solve(FakeTensor((5, 4, 70)), stream=FakeStream(1))


def test_handle_follows_the_current_gpu(fake):
    with torch.cuda.device(1):
        s = smf.Solver(3, 3, 8, 1)
    assert s.device == 1
    cost = FakeTensor((3, 3, 8), device=1)
    s.solve(cost)                                  # outside the context: still the handle's GPU
    assert fake.last("smf_solve") == (s._h, cost.data_ptr(), 0xA01)
    assert s.surface().device == torch.device("cuda", 1)
    with pytest.raises(ValueError):
        s.solve(FakeTensor((3, 3, 8), device=0))
    s.close()


def test_batch_marshalling(fake):
    shapes = [(4, 4, 8, 1), (3, 5, 70, 0), (2, 2, 3, 2)]
    b = smf.BatchSolver(shapes)
    n, nx, ny, K, dl = fake.last("smf_batch_create")
    assert n == 3
    cols = [list(ctypes.cast(a, ctypes.POINTER(ctypes.c_int32 * 3)).contents) for a in (nx, ny, K, dl)]
    assert cols == [[4, 3, 2], [4, 5, 2], [8, 70, 3], [1, 0, 2]]
    assert b.sizes == [128, 1050, 12] and b.offsets == [0, 128, 1178] and b.col_offsets == [0, 16, 31]
    packed = FakeTensor((1190,))
    b.solve(packed)
    h, ptr, offs, st = fake.last("smf_batch_solve")
    assert (h, ptr, list(offs), st) == (b._h, packed.data_ptr(), [0, 128, 1178], 0xA00)
    big = FakeTensor((1300,))
    b.solve(big, offsets=[100, 200, 1280])
    assert list(fake.last("smf_batch_solve")[2]) == [100, 200, 1280]
    for bad_offsets in ([0, 128, 1179], [0, 128], [-1, 128, 1178]):
        with pytest.raises(ValueError):
            b.solve(packed, offsets=bad_offsets)
    with pytest.raises(ValueError, match="cuda:1"):
        b.solve(FakeTensor((1190,), device=1))
    assert b.flow_values() == [7, 8, 9] and b.energies() == [7, 8, 9]
    surf = b.surfaces()
    assert surf.shape == (35,) and fake.last("smf_batch_surfaces") == (b._h, surf.data_ptr(), 0xA00)
    e, ts, fd, fl = b.export_state()
    assert [t.shape for t in (e, ts, fd, fl)] == [(1190,)] * 3 + [(4, 1190)]
    assert b.export_soft_flows().shape == (4, 1190)
    with pytest.raises(ValueError):
        b.pack([FakeTensor((4, 4, 8)), FakeTensor((3, 5, 70), device=1), FakeTensor((2, 2, 3))])
    b.close()


def test_autotune_and_tuning_calls(fake):
    b = smf.BatchSolver([(4, 4, 8, 1), (3, 5, 70, 0)])
    packed = FakeTensor((1178,))
    smf.autotune(b, packed)
    h, ptr, offs, st = fake.last("smf_autotune")
    assert (h, ptr, list(offs[:2]), st) == (b._h, packed.data_ptr(), [0, 128], 0xA00)
    with pytest.raises(ValueError):
        smf.autotune(b, FakeTensor((1178,), device=1))
    s = smf.Solver(4, 4, 8, 1)
    smf.autotune(s, FakeTensor((4, 4, 8)))
    assert fake.last("smf_autotune")[2] is None       # a plain handle: no offsets
    smf.tune_apply(b)
    assert smf.tune_lookup(4, 4, 8, 1) == 7
    b.close()
    s.close()


def test_onehot_backward_marshalling(fake):
    surf = FakeTensor((2, 3, 4), device=1)
    g = FakeTensor((2,), dtype=torch.float32, device=1)
    out = smf.onehot_backward(surf, g, 9)
    assert (out.shape, out.dtype, out.device) == ((2, 3, 4, 9), torch.float32, torch.device("cuda", 1))
    assert fake.last("smf_onehot_backward") == (surf.data_ptr(), g.data_ptr(), out.data_ptr(),
                                                2, 3, 4, 9, 0xA01)
    assert fake.current["entered"][-1] == 1, "the kernel is launched with the surface's GPU current"
    mine = FakeTensor((2, 3, 4, 9), dtype=torch.float32, device=1)
    assert smf.onehot_backward(surf, g, 9, out=mine) is mine
    for bad_out in (FakeTensor((2, 3, 4, 8), dtype=torch.float32, device=1),
                    FakeTensor((2, 3, 4, 9), dtype=torch.int32, device=1),
                    FakeTensor((2, 3, 4, 9), dtype=torch.float32, device=0),
                    FakeTensor((2, 3, 4, 9), dtype=torch.float32, device=1, contiguous=False)):
        with pytest.raises(ValueError):
            smf.onehot_backward(surf, g, 9, out=bad_out)
    with pytest.raises(ValueError):
        smf.onehot_backward(surf, FakeTensor((2,), dtype=torch.float32, device=0), 9)


def test_module_solve_and_autograd_handles_use_the_volume_gpu(fake):
    cost = FakeTensor((3, 4, 5), device=1)
    flow, energy, surf = smf.solve(cost, 1)
    assert (flow, energy) == (7, 7) and surf.device == torch.device("cuda", 1)
    assert fake.last("smf_solve")[2] == 0xA01
    s1 = autograd._solver(1, 2, 3, 4, 5, 1)
    assert s1.device == 1 and autograd._solver(1, 2, 3, 4, 5, 1) is s1
    s0 = autograd._solver(0, 2, 3, 4, 5, 1)
    assert s0.device == 0 and s0 is not s1


def test_band_and_noalloc_marshalling(fake):
    s = smf.Solver(3, 2, 10, 1)
    off = np.arange(6).reshape(3, 2)
    s.set_band(off, np.full((3, 2), 4))
    name, args = fake.calls[-1]
    assert name == "smf_set_band" and args[0] == s._h and args[1] and args[2]
    s.set_band(None, None)
    assert fake.last("smf_set_band") == (s._h, None, None)
    n = len(fake.calls)
    with pytest.raises(ValueError):
        s.set_band(np.zeros((2, 3)), np.ones((2, 3)))
    assert len(fake.calls) == n
    s.close()

    cost = FakeTensor((3, 2, 10))
    flow, energy, surf = smf.solve_noalloc(cost, 1)
    args = fake.last("smf_solve_noalloc")
    assert args[:6] == (cost.data_ptr(), 3, 2, 10, 1, surf.data_ptr()) and args[8] == 0xA00
    assert (surf.shape, surf.dtype) == ((3, 2), torch.int32)
    mine = FakeTensor((3, 2))
    assert smf.solve_noalloc(cost, 1, surface=mine)[2] is mine
    with pytest.raises(ValueError):
        smf.solve_noalloc(FakeTensor((3, 2, 10), dtype=torch.float32), 1)
