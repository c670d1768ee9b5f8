"""CPU oracle for the anisotropic-conduction MRT lattice Boltzmann solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product (the HIP
library under ``paper_1503_08718_amd`` and its binding) never imports, loads or
calls it, and the two share no code.

``lbm_oracle.c`` is a plain FP64 implementation that follows the paper's
Sec. 2 literally (7x7 collision matrix M^-1 S M per phase, push streaming,
Eqs. 14-16 and 22 for the observables); ``matrix_form`` builds the same
one-step map as explicit dense matrices for tiny grids; ``conv`` is the FP64
reference of the warm-start network's layers.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblbm_oracle.so")

PERIODIC, ADIABATIC = 0, 1
TOL_MAXDT, TOL_KEFF = 0, 1


def build(force: bool = True) -> str:
    """Compile the C oracle (plain gcc, FP64, no fused multiply-add)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


#: flags of the timing copy (the CPU baseline): the same source, built on the
#: host that runs it, with its full instruction set
TIMING_FLAGS = ["-O3", "-march=native", "-ffp-contract=off", "-fopenmp"]

_lib = None
_timing_lib = None


def build_timing_copy(directory: str | None = None) -> str:
    """Compile lbm_oracle.c with TIMING_FLAGS into ``directory`` (default: a
    fresh temporary directory) on this host, for timing only.  The checker
    build (build()) is left alone."""
    import tempfile

    d = directory or tempfile.mkdtemp(prefix="lbm_oracle_timing_")
    path = os.path.join(d, "liblbm_oracle_timing.so")
    subprocess.run(["gcc", *TIMING_FLAGS, "-shared", "-fPIC", "-o", path, _SRC, "-lm"], check=True)
    return path


def timing_lib():
    """The oracle built with TIMING_FLAGS on this host (compiled on first use)."""
    global _timing_lib
    if _timing_lib is None:
        _timing_lib = _bind(ctypes.CDLL(build_timing_copy()))
    return _timing_lib


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _bind(L):
    P, D, I, LL = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_longlong
    dp = ctypes.POINTER(ctypes.c_double)
    L.oracle_create.restype = P
    L.oracle_create.argtypes = [I, I, I, P, dp, I, D, dp]
    L.oracle_destroy.argtypes = [P]
    L.oracle_scale.restype = D
    L.oracle_scale.argtypes = [P]
    L.oracle_omega.argtypes = [P, I, dp]
    L.oracle_tau.argtypes = [P, I, dp]
    L.oracle_steps.restype = LL
    L.oracle_steps.argtypes = [P]
    L.oracle_set_threads.argtypes = [P, I]
    L.oracle_set_bc.restype = I
    L.oracle_set_bc.argtypes = [P, I, D, D, ctypes.POINTER(ctypes.c_int)]
    L.oracle_set_side_flux.restype = I
    L.oracle_set_side_flux.argtypes = [P, I, D, D]
    L.oracle_init.argtypes = [P, dp]
    L.oracle_init_flux.argtypes = [P, dp]
    L.oracle_collide_node.argtypes = [P, I, dp, dp]
    L.oracle_step.argtypes = [P, LL]
    L.oracle_temperature.argtypes = [P, dp]
    L.oracle_flux.argtypes = [P, dp, dp]
    L.oracle_keff.argtypes = [P, dp]
    L.oracle_solve.restype = I
    L.oracle_solve.argtypes = [P, D, I, LL, I, dp]
    L.oracle_get_f.argtypes = [P, dp]
    L.oracle_set_f.argtypes = [P, dp]
    L.oracle_last_fluxes.argtypes = [P, dp]
    return L


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """One medium on the CPU.  Arrays are numpy, (nz, ny, nx) order."""

    def __init__(self, phase: np.ndarray, k: np.ndarray, dmax: float = 1.0, tau_rest=None, threads: int = 0,
                 timing: bool = False):
        """timing=True runs on the copy built with TIMING_FLAGS (CPU baseline)."""
        L = timing_lib() if timing else lib()
        self._L = L
        self.phase = np.ascontiguousarray(phase, dtype=np.uint8)
        self.k = np.ascontiguousarray(k, dtype=np.float64)
        nz, ny, nx = self.phase.shape
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        tr = None if tau_rest is None else np.ascontiguousarray(tau_rest, dtype=np.float64)
        h = L.oracle_create(nx, ny, nz, self.phase.ctypes.data, _dp(self.k), self.k.shape[0], float(dmax),
                            _dp(tr) if tr is not None else None)
        if not h:
            raise ValueError("oracle_create rejected the medium (bad dims, phase id or non-SPD tensor)")
        self._h = ctypes.c_void_p(h)
        self._tr = tr
        if threads:
            L.oracle_set_threads(self._h, int(threads))
        self.grad_axis = 0
        self.t_hot, self.t_cold = 1.0, 0.0

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(self, "_L", None)
        if h is not None and L is not None:
            L.oracle_destroy(h)
            self._h = None

    @property
    def scale(self) -> float:
        return self._L.oracle_scale(self._h)

    @property
    def steps(self) -> int:
        return self._L.oracle_steps(self._h)

    def set_threads(self, n: int):
        self._L.oracle_set_threads(self._h, int(n))

    def omega(self, p: int) -> np.ndarray:
        out = np.zeros(49)
        self._L.oracle_omega(self._h, p, _dp(out))
        return out.reshape(7, 7)

    def tau(self, p: int) -> np.ndarray:
        out = np.zeros(9)
        self._L.oracle_tau(self._h, p, _dp(out))
        return out.reshape(3, 3)

    def set_bc(self, grad_axis: int, t_hot: float = 1.0, t_cold: float = 0.0, sides=(PERIODIC, PERIODIC, PERIODIC)):
        arr = (ctypes.c_int * 3)(*[int(s) for s in sides])
        if self._L.oracle_set_bc(self._h, int(grad_axis), float(t_hot), float(t_cold), arr):
            raise ValueError("bad boundary specification")
        self.grad_axis, self.t_hot, self.t_cold = int(grad_axis), float(t_hot), float(t_cold)

    def set_side_flux(self, axis: int, q_lo: float, q_hi: float):
        """Heat flux into the cell through the two faces of an adiabatic axis
        (Eq. 24; physical units of k times temperature per voxel)."""
        if self._L.oracle_set_side_flux(self._h, int(axis), float(q_lo), float(q_hi)):
            raise ValueError("side flux needs an adiabatic axis")

    def init(self, T0=None, flux: bool = False):
        """Equilibrium start at T0 (zero field if None); with flux=True the
        pre-collision flux -eps tau grad T0 of Eq. 15 is added, grad T0 by
        central differences (see oracle_init_flux)."""
        if T0 is None:
            assert not flux, "a flux start needs a field"
            self._L.oracle_init(self._h, None)
        else:
            t = np.ascontiguousarray(T0, dtype=np.float64).reshape(-1)
            assert t.size == self.n
            if flux:
                self._L.oracle_init_flux(self._h, _dp(t))
            else:
                self._L.oracle_init(self._h, _dp(t))

    def collide_node(self, p: int, f7) -> np.ndarray:
        fin = np.ascontiguousarray(f7, dtype=np.float64)
        out = np.zeros(7)
        self._L.oracle_collide_node(self._h, int(p), _dp(fin), _dp(out))
        return out

    def step(self, n: int = 1):
        self._L.oracle_step(self._h, int(n))

    def temperature(self) -> np.ndarray:
        out = np.zeros(self.n)
        self._L.oracle_temperature(self._h, _dp(out))
        return out.reshape(self.shape)

    def flux(self):
        q = np.zeros(3 * self.n)
        g = np.zeros(3 * self.n)
        self._L.oracle_flux(self._h, _dp(q), _dp(g))
        return q.reshape((3,) + self.shape), g.reshape((3,) + self.shape)

    @staticmethod
    def _kdict(out, steps=None, converged=None):
        d = dict(keff=out[0], keff_vol=out[0], keff_hot=out[1], keff_cold=out[2],
                 keff_col=np.array(out[3:6]), resid=out[6])
        d["keff_mid"] = 0.5 * (out[1] + out[2])
        if steps is not None:
            d["steps"] = steps
        if converged is not None:
            d["converged"] = converged
        return d

    def keff(self) -> dict:
        out = np.zeros(7)
        self._L.oracle_keff(self._h, _dp(out))
        return self._kdict(out, self.steps)

    def solve(self, tol: float, kind: int = TOL_MAXDT, max_steps: int = 10**7, check_every: int = 1) -> dict:
        out = np.zeros(7)
        rc = self._L.oracle_solve(self._h, float(tol), int(kind), int(max_steps), int(check_every), _dp(out))
        if rc < 0:
            raise FloatingPointError("oracle state became non-finite")
        return self._kdict(out, self.steps, bool(rc))

    def get_f(self) -> np.ndarray:
        out = np.zeros(7 * self.n)
        self._L.oracle_get_f(self._h, _dp(out))
        return out.reshape((7,) + self.shape)

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        assert f.size == 7 * self.n
        self._L.oracle_set_f(self._h, _dp(f))

    def last_fluxes(self):
        out = np.zeros(3)
        self._L.oracle_last_fluxes(self._h, _dp(out))
        return dict(phi_hot=out[0], phi_cold=out[1], resid=out[2])


def from_medium(m, dmax: float = 1.0, **kw) -> Oracle:
    return Oracle(m.phase, m.k, dmax=dmax, **kw)
