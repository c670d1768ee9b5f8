"""Python binding of the solver: argument marshalling only.

Device memory (phase grid, workspace, outputs) comes from torch on the HIP
device and the library works on torch's current stream of that device; every
step of the method runs in the library's kernels.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import ADIABATIC, F32, F64, PERIODIC, TOL_KEFF, TOL_MAXDT, Launch, Result, check, load

_SIDES = {"periodic": PERIODIC, "adiabatic": ADIABATIC, PERIODIC: PERIODIC, ADIABATIC: ADIABATIC}
_KINDS = {"maxdt": TOL_MAXDT, "keff": TOL_KEFF, TOL_MAXDT: TOL_MAXDT, TOL_KEFF: TOL_KEFF}
_STORAGE = {"populations": 0, "moments": 1, 0: 0, 1: 1}
_PREC = {"f32": F32, "float32": F32, torch.float32: F32, F32: F32,
         "f64": F64, "float64": F64, torch.float64: F64, F64: F64}


def _aligned_bytes(nbytes: int, device) -> tuple[torch.Tensor, int]:
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    ptr = buf.data_ptr()
    off = (-ptr) % 256
    return buf, ptr + off


class Medium:
    """One voxel medium on one GPU.

    phase: uint8 array/tensor (nz, ny, nx); k: (nphase, 6) float64 tensors
    (kxx, kyy, kzz, kxy, kxz, kyz) in physical units.  storage=None sizes
    the workspace for either state storage (starting with populations);
    "moments" allocates only what moment storage needs (4 of 7 values per
    node) and the medium cannot switch to populations.
    """

    def __init__(self, phase, k, precision="f32", device="cuda:0", storage=None):
        L = load()
        self.device = torch.device(device)
        if isinstance(phase, np.ndarray):
            phase = torch.from_numpy(np.ascontiguousarray(phase, dtype=np.uint8))
        self.phase = phase.to(self.device, dtype=torch.uint8).contiguous()
        nz, ny, nx = self.phase.shape
        self.shape = (nz, ny, nx)
        self.k = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(-1, 6))
        self.nphase = self.k.shape[0]
        self.prec = _PREC[precision]
        self.dtype = torch.float64 if self.prec == F64 else torch.float32
        if storage is None:
            nbytes = L.mrtlbm_workspace_bytes(nx, ny, nz, self.nphase, self.prec)
        else:
            nbytes = L.mrtlbm_workspace_bytes_storage(nx, ny, nz, self.nphase, self.prec, _STORAGE[storage])
        if nbytes == 0:
            raise ValueError(f"invalid medium sizes {self.shape} / nphase {self.nphase}")
        with torch.cuda.device(self.device):
            self._ws, wptr = _aligned_bytes(nbytes, self.device)
            self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        kp = self.k.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        check(L.mrtlbm_create(nx, ny, nz, self.phase.data_ptr(), kp, self.nphase, self.prec, wptr, nbytes,
                              self.stream.cuda_stream, ctypes.byref(h)))
        self._h = h
        self.grad_axis, self.t_hot, self.t_cold = 0, 1.0, 0.0
        if storage is not None:
            self.set_storage(storage)

    # -- lifetime ---------------------------------------------------------
    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            load().mrtlbm_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- configuration ----------------------------------------------------
    def set_bc(self, grad_axis: int, t_hot: float = 1.0, t_cold: float = 0.0, sides=("periodic",) * 3):
        arr = (ctypes.c_int * 3)(*[_SIDES[s] for s in sides])
        check(load().mrtlbm_set_bc(self._h, int(grad_axis), float(t_hot), float(t_cold), arr))
        self.grad_axis, self.t_hot, self.t_cold = int(grad_axis), float(t_hot), float(t_cold)
        return self

    def set_storage(self, storage):
        """"populations" (7 values per node) or "moments" (4 values per node)."""
        check(load().mrtlbm_set_storage(self._h, _STORAGE[storage]))
        return self

    def set_scale(self, dmax: float):
        check(load().mrtlbm_set_scale(self._h, float(dmax)))
        return self

    def set_side_flux(self, axis: int, q_lo: float, q_hi: float):
        """Heat flux into the cell through the two Neumann faces of an
        adiabatic side axis (Eq. 24), in the units of flux()."""
        check(load().mrtlbm_set_side_flux(self._h, int(axis), float(q_lo), float(q_hi)))
        return self

    def set_relaxation(self, tau4: float = 1.0, tau5: float = 1.0, tau6: float = 1.0):
        """tau_4..6 of Eq. 12 (population storage only when not all 1)."""
        check(load().mrtlbm_set_relaxation(self._h, float(tau4), float(tau5), float(tau6)))
        return self

    def set_launch(self, vec=None, bx=None, by=None, nt=0, map=0):
        if vec is None:
            check(load().mrtlbm_set_launch(self._h, None))
        else:
            check(load().mrtlbm_set_launch(self._h, ctypes.byref(Launch(vec, bx, by, nt, map))))
        return self

    def info(self) -> dict:
        s = ctypes.c_double()
        n = ctypes.c_longlong()
        L = Launch()
        check(load().mrtlbm_info(self._h, ctypes.byref(s), ctypes.byref(n), ctypes.byref(L)))
        return dict(scale=s.value, steps=n.value, launch=(L.vec, L.bx, L.by, L.nt, L.map))

    def autotune(self, cache_path: str | None = None):
        L = Launch()
        check(load().mrtlbm_autotune(self._h, cache_path.encode() if cache_path else None, ctypes.byref(L)))
        return (L.vec, L.bx, L.by, L.nt, L.map)

    def load_tuned(self, cache_path: str) -> bool:
        st = check(load().mrtlbm_load_tuned(self._h, cache_path.encode()), allow=(0, 1))
        return st == 0

    # -- state --------------------------------------------------------------
    def init(self, T0=None, flux: bool = False):
        ptr = None
        if T0 is not None:
            if isinstance(T0, np.ndarray):
                T0 = torch.from_numpy(T0)
            T0 = T0.to(self.device, dtype=self.dtype).contiguous()
            assert tuple(T0.shape) == self.shape
            self._t0 = T0
            ptr = T0.data_ptr()
        check(load().mrtlbm_init(self._h, ptr, 1 if flux else 0))
        return self

    def step(self, n: int = 1):
        check(load().mrtlbm_step(self._h, int(n)))
        return self

    def solve(self, tol: float = 1e-4, kind="keff", max_steps: int = 10**7, check_every: int = 1000) -> dict:
        r = Result()
        st = check(load().mrtlbm_solve(self._h, float(tol), _KINDS[kind], int(max_steps), int(check_every),
                                       ctypes.byref(r)), allow=(0, 1))
        d = r.to_dict()
        d["status"] = _lib.STATUS[st]
        return d

    def keff(self) -> dict:
        r = Result()
        check(load().mrtlbm_keff(self._h, ctypes.byref(r)))
        return r.to_dict()

    def temperature(self) -> torch.Tensor:
        out = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        check(load().mrtlbm_temperature(self._h, out.data_ptr()))
        return out

    def flux(self) -> torch.Tensor:
        out = torch.empty((3,) + self.shape, dtype=self.dtype, device=self.device)
        check(load().mrtlbm_flux(self._h, out.data_ptr()))
        return out

    def state_get(self) -> torch.Tensor:
        nv = load().mrtlbm_state_values(self._h)
        out = torch.empty((nv,) + self.shape, dtype=self.dtype, device=self.device)
        check(load().mrtlbm_state_get(self._h, out.data_ptr()))
        return out

    def state_set(self, f: torch.Tensor, steps: int = 0):
        f = f.to(self.device, dtype=self.dtype).contiguous()
        assert tuple(f.shape) == (load().mrtlbm_state_values(self._h),) + self.shape
        self._fset = f
        check(load().mrtlbm_state_set(self._h, f.data_ptr(), int(steps)))
        return self

    def time_steps(self, n: int) -> float:
        ms = ctypes.c_double()
        check(load().mrtlbm_time_steps(self._h, int(n), ctypes.byref(ms)))
        return ms.value


def batch_solve(media, tol: float = 1e-4, kind="keff", max_steps: int = 10**7, check_every: int = 1000):
    """Solve several initialised media together (one launch per step for all
    active cells, graph-replayed between checks)."""
    L = load()
    n = len(media)
    arr = (ctypes.c_void_p * n)(*[m.handle.value for m in media])
    nbytes = L.mrtlbm_batch_workspace_bytes(arr, n)
    if nbytes == 0:
        raise ValueError("batch workspace size is zero (bad media list)")
    dev = media[0].device
    with torch.cuda.device(dev):
        ws, wptr = _aligned_bytes(nbytes, dev)
    res = (Result * n)()
    st = check(L.mrtlbm_batch_solve(arr, n, float(tol), _KINDS[kind], int(max_steps), int(check_every), wptr, nbytes,
                                    res), allow=(0, 1))
    del ws
    out = [r.to_dict() for r in res]
    return out, _lib.STATUS[st]


def batch_autotune(media) -> dict:
    """Choose the batched step's shape for these media (mrtlbm_batch_autotune).
    Overwrites their states: call init() on every medium afterwards."""
    L = load()
    n = len(media)
    arr = (ctypes.c_void_p * n)(*[m.handle.value for m in media])
    nbytes = L.mrtlbm_batch_workspace_bytes(arr, n)
    if nbytes == 0:
        raise ValueError("batch workspace size is zero (bad media list)")
    dev = media[0].device
    with torch.cuda.device(dev):
        ws, wptr = _aligned_bytes(nbytes, dev)
    best = Launch()
    check(L.mrtlbm_batch_autotune(arr, n, wptr, nbytes, ctypes.byref(best)))
    del ws
    return dict(vec=best.vec, bx=best.bx, by=best.by, nt=best.nt, map=best.map)
