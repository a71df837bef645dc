"""ctypes binding of libhacc_sr.so (declared in include/hacc_sr.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides device memory (the output tensors and the
workspace) and the stream (the current torch stream of the tensors'
device).  The library must be built (``__graft_entry__.build()``); there is
no fallback, a missing library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhacc_sr.so")

EXPORTS = (
    "hacc_sr_version", "hacc_sr_source_hash", "hacc_sr_strerror", "hacc_sr_set_stream",
    "hacc_sr_grid_dim", "hacc_sr_workspace_bytes", "hacc_sr_set_workspace",
    "hacc_sr_bin", "hacc_sr_force", "hacc_sr_force_vjp", "hacc_sr_kick",
    "hacc_sr_stream", "hacc_sr_kick_adjoint", "hacc_sr_count_pairs",
    "hacc_sr_timing_enable", "hacc_sr_timing_read", "hacc_sr_force_plain",
    "hacc_sr_force_vjp_plain", "hacc_sr_valu_probe", "hacc_sr_workspace_bytes_rcb",
    "hacc_sr_rcb_bin", "hacc_sr_force_rcb", "hacc_sr_force_vjp_rcb",
    "hacc_sr_force_noalloc", "hacc_sr_pm_workspace_bytes", "hacc_sr_pm_accel",
    "hacc_sr_full_step", "hacc_sr_binning_token", "hacc_sr_force_vjp_binned",
)

OK, EINVAL, EDOMAIN, ENOSPACE, EHIP, ESTALE = 0, -1, -2, -3, -4, -5
TIMER_FORCE, TIMER_VJP, TIMER_BIN, TIMER_WORKLIST = 0, 1, 2, 3
TIMER_FORCE_PLAIN, TIMER_VJP_PLAIN, TIMER_RCB, TIMER_PM = 4, 5, 6, 7


class HaccSrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hacc_sr error {code}: {msg}")
        self.code = code


_lib = None


class StaleLibraryError(RuntimeError):
    pass


def load():
    """Load the library.  Raises if it has not been built, or if it was built
    from other sources than those in the tree (its embedded source hash
    differs): a stale binary never runs."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    lib.hacc_sr_source_hash.argtypes = []
    lib.hacc_sr_source_hash.restype = ctypes.c_char_p
    from . import build as _build
    built = lib.hacc_sr_source_hash().decode()
    want = _build.source_hash()
    if built != want:
        raise StaleLibraryError(
            f"{LIB_PATH} was built from other sources (sha256 {built[:16]}..., "
            f"tree {want[:16]}...); rebuild with __graft_entry__.build()")
    P, I64, D, F, I = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                       ctypes.c_float, ctypes.c_int)
    sig = {
        "hacc_sr_version": ([], I),
        "hacc_sr_source_hash": ([], ctypes.c_char_p),
        "hacc_sr_strerror": ([I], ctypes.c_char_p),
        "hacc_sr_set_stream": ([P], I),
        "hacc_sr_grid_dim": ([D, F, P], I),
        "hacc_sr_workspace_bytes": ([I64, D, F, P], I),
        "hacc_sr_set_workspace": ([P, ctypes.c_size_t], I),
        "hacc_sr_bin": ([P, P, I64, D, F, P, P, P], I),
        "hacc_sr_force": ([P, P, I64, D, F, F, P, P], I),
        "hacc_sr_force_vjp": ([P, P, I64, D, F, F, P, P, P], I),
        "hacc_sr_force_plain": ([P, P, I64, D, F, F, P, P], I),
        "hacc_sr_force_vjp_plain": ([P, P, I64, D, F, F, P, P, P], I),
        "hacc_sr_kick": ([P, P, I64, D], I),
        "hacc_sr_stream": ([P, P, I64, D, D], I),
        "hacc_sr_kick_adjoint": ([P, P, I64, D], I),
        "hacc_sr_count_pairs": ([P, I64, D, F, F, P], I),
        "hacc_sr_timing_enable": ([I], I),
        "hacc_sr_timing_read": ([I, P, P], I),
        "hacc_sr_valu_probe": ([I, I, P], I),
        "hacc_sr_workspace_bytes_rcb": ([I64, D, F, P], I),
        "hacc_sr_rcb_bin": ([P, P, I64, D, F, I, P, P, P, P, P, P, P, P], I),
        "hacc_sr_force_rcb": ([P, P, I64, D, F, F, P, I, P], I),
        "hacc_sr_force_vjp_rcb": ([P, P, I64, D, F, F, P, I, P, P], I),
        "hacc_sr_force_noalloc": ([P, P, I64, D, F, F, P, P], I),
        "hacc_sr_pm_workspace_bytes": ([I, I64, P], I),
        "hacc_sr_pm_accel": ([P, P, I64, D, I, F, I, P], I),
        "hacc_sr_full_step": ([P, P, P, I64, D, I, F, I, F, F, P, D, I, P], I),
        "hacc_sr_binning_token": ([P], I),
        "hacc_sr_force_vjp_binned": ([ctypes.c_uint64, I64, D, F, F, P, P, P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != OK:
        raise HaccSrError(rc, load().hacc_sr_strerror(rc).decode())


def strerror(rc: int) -> str:
    return load().hacc_sr_strerror(rc).decode()


def poly_array(poly: Sequence[float]):
    """Host float[6] for the polynomial coefficients c_0..c_5."""
    arr = np.ascontiguousarray(np.asarray(poly, dtype=np.float32).reshape(6))
    return (ctypes.c_float * 6)(*arr.tolist())


def grid_dim(box: float, r_cut: float) -> int:
    out = ctypes.c_int32(0)
    check(load().hacc_sr_grid_dim(float(box), float(r_cut), ctypes.byref(out)))
    return out.value


def workspace_bytes(n: int, box: float, r_cut: float, rcb: bool = False) -> int:
    out = ctypes.c_size_t(0)
    fn = load().hacc_sr_workspace_bytes_rcb if rcb else load().hacc_sr_workspace_bytes
    check(fn(int(n), float(box), float(r_cut), ctypes.byref(out)))
    return out.value


# ------------------------------------------------------------------ torch side

def _torch():
    import torch
    return torch


_workspaces: dict = {}


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _require(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _bind(device, n: int, box: float, r_cut: float, rcb: bool = False,
          need: int | None = None) -> None:
    """Register torch's current stream and that stream's own workspace, large
    enough for n.  One workspace per (device, stream): work queued on two
    streams never shares scratch memory.  A workspace is allocated while its
    stream is current, so torch's stream-ordered allocator reuses the memory
    of a replaced one only after the work queued on that stream."""
    torch = _torch()
    lib = load()
    dev = torch.device(device)
    stream = torch.cuda.current_stream(dev)
    check(lib.hacc_sr_set_stream(ctypes.c_void_p(stream.cuda_stream)))
    if need is None:
        need = workspace_bytes(n, box, r_cut, rcb)
    index = dev.index if dev.index is not None else torch.cuda.current_device()
    key = (index, stream.cuda_stream)
    ws = _workspaces.get(key)
    if ws is None or ws.numel() < need:
        _workspaces.pop(key, None)
        ws = torch.empty(int(need * 1.125) + 4096, dtype=torch.uint8, device=dev)
        _workspaces[key] = ws
    check(lib.hacc_sr_set_workspace(_ptr(ws), ws.numel()))


def release_workspace() -> None:
    _workspaces.clear()
    if _lib is not None:
        _lib.hacc_sr_set_workspace(None, 0)


def bin(pos, mass, box: float, r_cut: float):
    """Chaining-mesh binning: returns (cell_start int32 (N^3+1),
    perm int32 (n), sorted_rec float32 (n, 4))."""
    torch = _torch()
    n = pos.shape[0]
    _require(pos, torch.float64, (n, 3), "pos")
    _require(mass, torch.float32, (n,), "mass")
    N = grid_dim(box, r_cut)
    cs = torch.empty(N ** 3 + 1, dtype=torch.int32, device=pos.device)
    perm = torch.empty(n, dtype=torch.int32, device=pos.device)
    rec = torch.empty((n, 4), dtype=torch.float32, device=pos.device)
    with torch.cuda.device(pos.device):
        _bind(pos.device, n, box, r_cut)
        check(load().hacc_sr_bin(_ptr(pos), _ptr(mass), n, float(box),
                                 float(r_cut), _ptr(cs), _ptr(perm), _ptr(rec)))
    return cs, perm, rec


def force(pos, mass, box: float, r_cut: float, eps: float, poly, out=None):
    """Short-range accelerations (n, 3) float32 in input order."""
    torch = _torch()
    n = pos.shape[0]
    _require(pos, torch.float64, (n, 3), "pos")
    _require(mass, torch.float32, (n,), "mass")
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
    _require(out, torch.float32, (n, 3), "out")
    with torch.cuda.device(pos.device):
        _bind(pos.device, n, box, r_cut)
        check(load().hacc_sr_force(_ptr(pos), _ptr(mass), n, float(box),
                                   float(r_cut), float(eps), poly_array(poly),
                                   _ptr(out)))
    return out


def binning_token() -> int:
    """Token of the binning that the last force or force_vjp call left in the
    workspace (0: none); see force_vjp's `binned`."""
    out = ctypes.c_uint64(0)
    check(load().hacc_sr_binning_token(ctypes.byref(out)))
    return out.value


def force_vjp(pos, mass, box: float, r_cut: float, eps: float, poly, grad_acc,
              out=None, binned: int | None = None):
    """dL/dx (n, 3) float64 for L = sum(grad_acc * acc).

    binned: a binning_token() taken right after the force call at these
    positions and masses.  While that binning is still in the workspace (no
    other binning, PM, probe or workspace change since) the VJP reuses it
    and does not bin again; otherwise it bins from pos as usual."""
    torch = _torch()
    n = pos.shape[0]
    _require(pos, torch.float64, (n, 3), "pos")
    _require(mass, torch.float32, (n,), "mass")
    _require(grad_acc, torch.float32, (n, 3), "grad_acc")
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    _require(out, torch.float64, (n, 3), "out")
    with torch.cuda.device(pos.device):
        _bind(pos.device, n, box, r_cut)
        if binned:
            rc = load().hacc_sr_force_vjp_binned(int(binned), n, float(box), float(r_cut),
                                                 float(eps), poly_array(poly),
                                                 _ptr(grad_acc), _ptr(out))
            if rc != ESTALE:
                check(rc)
                return out
        check(load().hacc_sr_force_vjp(_ptr(pos), _ptr(mass), n, float(box),
                                       float(r_cut), float(eps),
                                       poly_array(poly), _ptr(grad_acc),
                                       _ptr(out)))
    return out


def rcb_bin(pos, mass, box: float, r_cut: float, leaf_max: int = 64,
            with_nodes: bool = False):
    """Chaining-mesh binning with RCB fat leaves inside the cells: returns
    (cell_start, perm, sorted_rec, leaf_start[:n_leaves + 1]) and, with
    with_nodes, also (nodes (m, 4) int32, node_split (m,) float32) for the m
    internal nodes."""
    torch = _torch()
    n = pos.shape[0]
    _require(pos, torch.float64, (n, 3), "pos")
    _require(mass, torch.float32, (n,), "mass")
    N = grid_dim(box, r_cut)
    dev = pos.device
    cs = torch.empty(N ** 3 + 1, dtype=torch.int32, device=dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    rec = torch.empty((n, 4), dtype=torch.float32, device=dev)
    ls = torch.empty(n + 1, dtype=torch.int32, device=dev)
    nl = torch.zeros(1, dtype=torch.int32, device=dev)
    if with_nodes:
        nodes = torch.empty((max(n, 1), 4), dtype=torch.int32, device=dev)
        split = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
        nn = torch.zeros(1, dtype=torch.int32, device=dev)
        extra = (_ptr(nodes), _ptr(split), _ptr(nn))
    else:
        extra = (None, None, None)
    with torch.cuda.device(dev):
        _bind(dev, n, box, r_cut, rcb=True)
        check(load().hacc_sr_rcb_bin(_ptr(pos), _ptr(mass), n, float(box), float(r_cut),
                                     int(leaf_max), _ptr(cs), _ptr(perm), _ptr(rec),
                                     _ptr(ls), _ptr(nl), *extra))
    k = int(nl.item())
    out = (cs, perm, rec, ls[:k + 1])
    if with_nodes:
        m = int(nn.item())
        out = out + (nodes[:m], split[:m])
    return out


def force_rcb(pos, mass, box: float, r_cut: float, eps: float, poly,
              leaf_max: int = 64, out=None):
    """Short-range accelerations with the RCB fat leaves as work items."""
    torch = _torch()
    n = pos.shape[0]
    _require(pos, torch.float64, (n, 3), "pos")
    _require(mass, torch.float32, (n,), "mass")
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
    _require(out, torch.float32, (n, 3), "out")
    with torch.cuda.device(pos.device):
        _bind(pos.device, n, box, r_cut, rcb=True)
        check(load().hacc_sr_force_rcb(_ptr(pos), _ptr(mass), n, float(box),
                                       float(r_cut), float(eps), poly_array(poly),
                                       int(leaf_max), _ptr(out)))
    return out


def force_vjp_rcb(pos, mass, box: float, r_cut: float, eps: float, poly, grad_acc,
                  leaf_max: int = 64, out=None):
    """VJP with the RCB fat leaves as work items."""
    torch = _torch()
    n = pos.shape[0]
    _require(pos, torch.float64, (n, 3), "pos")
    _require(mass, torch.float32, (n,), "mass")
    _require(grad_acc, torch.float32, (n, 3), "grad_acc")
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    _require(out, torch.float64, (n, 3), "out")
    with torch.cuda.device(pos.device):
        _bind(pos.device, n, box, r_cut, rcb=True)
        check(load().hacc_sr_force_vjp_rcb(_ptr(pos), _ptr(mass), n, float(box),
                                           float(r_cut), float(eps), poly_array(poly),
                                           int(leaf_max), _ptr(grad_acc), _ptr(out)))
    return out


def pm_workspace_bytes(ng: int, n: int) -> int:
    out = ctypes.c_size_t(0)
    check(load().hacc_sr_pm_workspace_bytes(int(ng), int(n), ctypes.byref(out)))
    return out.value


def pm_accel(pos, mass, box: float, ng: int, sigma: float = 0.8, n_s: int = 3, out=None):
    """Long-range accelerations (n, 3) float32 from the spectral PM solver."""
    torch = _torch()
    n = pos.shape[0]
    _require(pos, torch.float64, (n, 3), "pos")
    _require(mass, torch.float32, (n,), "mass")
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
    _require(out, torch.float32, (n, 3), "out")
    with torch.cuda.device(pos.device):
        _bind(pos.device, n, box, 0.0, need=pm_workspace_bytes(ng, n))
        check(load().hacc_sr_pm_accel(_ptr(pos), _ptr(mass), n, float(box), int(ng),
                                      float(sigma), int(n_s), _ptr(out)))
    return out


def full_step(pos, vel, mass, box: float, ng: int, r_cut: float, eps: float, poly,
              dt: float, n_c: int, sigma: float = 0.8, n_s: int = 3, scratch=None):
    """One split-operator step M_lr(dt/2) (M_sr(dt/n_c))^n_c M_lr(dt/2), in
    place on pos and vel."""
    torch = _torch()
    n = pos.shape[0]
    _require(pos, torch.float64, (n, 3), "pos")
    _require(vel, torch.float64, (n, 3), "vel")
    _require(mass, torch.float32, (n,), "mass")
    if scratch is None:
        scratch = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
    _require(scratch, torch.float32, (n, 3), "scratch")
    with torch.cuda.device(pos.device):
        need = max(workspace_bytes(n, box, r_cut), pm_workspace_bytes(ng, n))
        _bind(pos.device, n, box, r_cut, need=need)
        check(load().hacc_sr_full_step(_ptr(pos), _ptr(vel), _ptr(mass), n, float(box),
                                       int(ng), float(sigma), int(n_s), float(r_cut),
                                       float(eps), poly_array(poly), float(dt), int(n_c),
                                       _ptr(scratch)))


def force_plain(pos, mass, box: float, r_cut: float, eps: float, poly, out=None):
    """The plain float32 reference kernel (comparison only)."""
    torch = _torch()
    n = pos.shape[0]
    _require(pos, torch.float64, (n, 3), "pos")
    _require(mass, torch.float32, (n,), "mass")
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
    _require(out, torch.float32, (n, 3), "out")
    with torch.cuda.device(pos.device):
        _bind(pos.device, n, box, r_cut)
        check(load().hacc_sr_force_plain(_ptr(pos), _ptr(mass), n, float(box),
                                         float(r_cut), float(eps),
                                         poly_array(poly), _ptr(out)))
    return out


def force_vjp_plain(pos, mass, box: float, r_cut: float, eps: float, poly,
                    grad_acc, out=None):
    """The plain float32 reference VJP kernel (comparison only)."""
    torch = _torch()
    n = pos.shape[0]
    _require(pos, torch.float64, (n, 3), "pos")
    _require(mass, torch.float32, (n,), "mass")
    _require(grad_acc, torch.float32, (n, 3), "grad_acc")
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    _require(out, torch.float64, (n, 3), "out")
    with torch.cuda.device(pos.device):
        _bind(pos.device, n, box, r_cut)
        check(load().hacc_sr_force_vjp_plain(_ptr(pos), _ptr(mass), n, float(box),
                                             float(r_cut), float(eps),
                                             poly_array(poly), _ptr(grad_acc),
                                             _ptr(out)))
    return out


def kick(vel, acc, dt: float) -> None:
    """vel += dt * acc in place (float64 += float32)."""
    torch = _torch()
    n = vel.shape[0]
    _require(vel, torch.float64, (n, 3), "vel")
    _require(acc, torch.float32, (n, 3), "acc")
    with torch.cuda.device(vel.device):
        check(load().hacc_sr_set_stream(
            ctypes.c_void_p(torch.cuda.current_stream(vel.device).cuda_stream)))
        check(load().hacc_sr_kick(_ptr(vel), _ptr(acc), n, float(dt)))


def stream(pos, vel, dt: float, box: float) -> None:
    """pos += dt * vel in place, wrapped into [0, box) when box > 0."""
    torch = _torch()
    n = pos.shape[0]
    _require(pos, torch.float64, (n, 3), "pos")
    _require(vel, torch.float64, (n, 3), "vel")
    with torch.cuda.device(pos.device):
        check(load().hacc_sr_set_stream(
            ctypes.c_void_p(torch.cuda.current_stream(pos.device).cuda_stream)))
        check(load().hacc_sr_stream(_ptr(pos), _ptr(vel), n, float(dt), float(box)))


def kick_adjoint(grad_vel, dt: float, out=None):
    """float32(dt * grad_vel)."""
    torch = _torch()
    n = grad_vel.shape[0]
    _require(grad_vel, torch.float64, (n, 3), "grad_vel")
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=grad_vel.device)
    _require(out, torch.float32, (n, 3), "out")
    with torch.cuda.device(grad_vel.device):
        check(load().hacc_sr_set_stream(
            ctypes.c_void_p(torch.cuda.current_stream(grad_vel.device).cuda_stream)))
        check(load().hacc_sr_kick_adjoint(_ptr(grad_vel), _ptr(out), n, float(dt)))
    return out


def count_pairs(pos, box: float, r_cut: float, eps: float):
    """(candidate pairs, pairs inside r_cut) the pair kernel evaluates."""
    torch = _torch()
    n = pos.shape[0]
    _require(pos, torch.float64, (n, 3), "pos")
    out = torch.zeros(2, dtype=torch.int64, device=pos.device)
    with torch.cuda.device(pos.device):
        _bind(pos.device, n, box, r_cut)
        check(load().hacc_sr_count_pairs(_ptr(pos), n, float(box), float(r_cut),
                                         float(eps), _ptr(out)))
    c = out.cpu().tolist()
    return int(c[0]), int(c[1])


def timing_enable(on: bool = True) -> None:
    check(load().hacc_sr_timing_enable(1 if on else 0))


def timing_read(which: int):
    """(launches, total milliseconds) recorded for a timer since enabling."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    check(load().hacc_sr_timing_read(int(which), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


PROBE_FMA, PROBE_RSQ, PROBE_PAIR_MIX, PROBE_FMAC = 0, 1, 2, 3


def valu_probe(kind: int, waves_per_simd: int = 8, device=None):
    """Float32 VALU rate probe on the current torch stream: dict with lane
    operations per second, the mean shader clock (GHz), the shader cycles
    between two instructions of one wave, and milliseconds per launch."""
    torch = _torch()
    dev = torch.device(device if device is not None else "cuda:0")
    out = (ctypes.c_double * 4)()
    with torch.cuda.device(dev):
        _bind(dev, 1 << 20, 1.0, 0.25)
        check(load().hacc_sr_valu_probe(int(kind), int(waves_per_simd), out))
    return {"lane_ops_per_s": out[0], "clock_ghz": out[1],
            "wave_cycles_per_instr": out[2], "ms_per_launch": out[3]}
