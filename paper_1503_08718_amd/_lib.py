"""ctypes loader for libmrtlbm.so (the C ABI of include/mrtlbm.h)."""

from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrtlbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mrtlbm.h")

OK, NOT_CONVERGED = 0, 1
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "E_ARG", -2: "E_TENSOR", -3: "E_BC", -4: "E_HIP",
          -5: "E_NONFINITE", -6: "E_DIVERGED", -7: "E_WORKSPACE"}
F32, F64 = 0, 1
PERIODIC, ADIABATIC = 0, 1
TOL_MAXDT, TOL_KEFF = 0, 1


class MrtlbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Result(ctypes.Structure):
    _fields_ = [
        ("keff", ctypes.c_double),
        ("keff_hot", ctypes.c_double),
        ("keff_cold", ctypes.c_double),
        ("keff_vol", ctypes.c_double),
        ("keff_col", ctypes.c_double * 3),
        ("resid", ctypes.c_double),
        ("temp_mean", ctypes.c_double),
        ("keff_leak", ctypes.c_double),
        ("keff_side", ctypes.c_double),
        ("steps", ctypes.c_longlong),
        ("converged", ctypes.c_int),
        ("nonfinite", ctypes.c_int),
    ]

    def to_dict(self) -> dict:
        return dict(keff=self.keff, keff_hot=self.keff_hot, keff_cold=self.keff_cold, keff_vol=self.keff_vol,
                    keff_col=list(self.keff_col), resid=self.resid, temp_mean=self.temp_mean,
                    keff_leak=self.keff_leak, keff_side=self.keff_side, steps=self.steps,
                    converged=bool(self.converged), nonfinite=self.nonfinite)


class Launch(ctypes.Structure):
    _fields_ = [("vec", ctypes.c_int), ("bx", ctypes.c_int), ("by", ctypes.c_int), ("nt", ctypes.c_int),
                ("map", ctypes.c_int)]


_lib = None
PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_char_p, ctypes.c_void_p)
_progress_keep = None


def set_progress(fn=None, interval_s: float = 30.0):
    """Report long solves: fn(message: str) is called at check points, at
    most every interval_s seconds (None switches reports off)."""
    global _progress_keep
    L = load()
    if fn is None:
        _progress_keep = None
        L.mrtlbm_set_progress(PROGRESS_FN(), None, 0.0)
        return
    _progress_keep = PROGRESS_FN(lambda msg, user: fn(msg.decode()))
    L.mrtlbm_set_progress(_progress_keep, None, float(interval_s))


def declared_symbols() -> list[str]:
    """Function names declared in include/*.h (for export checks)."""
    inc = os.path.dirname(HEADER)
    names = []
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(mrtlbm_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def load():
    """Load the HIP library.  There is no fallback: a missing library is an error."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    # torch carries its own HIP runtime under the same soname; loading torch
    # first makes the library bind to that runtime, so the process holds one
    # HIP runtime (two would each try to own the device)
    import torch  # noqa: F401

    L = ctypes.CDLL(LIB_PATH)
    P, I, D, LL, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong, ctypes.c_size_t
    PP = ctypes.POINTER(ctypes.c_void_p)
    RP = ctypes.POINTER(Result)
    LP = ctypes.POINTER(Launch)
    sig = {
        "mrtlbm_workspace_bytes": (SZ, [I, I, I, I, I]),
        "mrtlbm_workspace_bytes_storage": (SZ, [I, I, I, I, I, I]),
        "mrtlbm_create": (I, [I, I, I, P, ctypes.POINTER(ctypes.c_double), I, I, P, SZ, P, PP]),
        "mrtlbm_set_bc": (I, [P, I, D, D, ctypes.POINTER(ctypes.c_int)]),
        "mrtlbm_set_scale": (I, [P, D]),
        "mrtlbm_set_side_flux": (I, [P, I, D, D]),
        "mrtlbm_set_relaxation": (I, [P, D, D, D]),
        "mrtlbm_init": (I, [P, P, I]),
        "mrtlbm_step": (I, [P, LL]),
        "mrtlbm_solve": (I, [P, D, I, LL, I, RP]),
        "mrtlbm_solve_noalloc": (I, [P, D, I, LL, I, RP]),
        "mrtlbm_stream_copy": (I, [P, P, LL, I, I, P]),
        "mrtlbm_keff": (I, [P, RP]),
        "mrtlbm_temperature": (I, [P, P]),
        "mrtlbm_flux": (I, [P, P]),
        "mrtlbm_state_get": (I, [P, P]),
        "mrtlbm_state_set": (I, [P, P, LL]),
        "mrtlbm_set_storage": (I, [P, I]),
        "mrtlbm_state_values": (I, [P]),
        "mrtlbm_info": (I, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong), LP]),
        "mrtlbm_set_launch": (I, [P, LP]),
        "mrtlbm_autotune": (I, [P, ctypes.c_char_p, LP]),
        "mrtlbm_load_tuned": (I, [P, ctypes.c_char_p]),
        "mrtlbm_time_steps": (I, [P, LL, ctypes.POINTER(ctypes.c_double)]),
        "mrtlbm_destroy": (None, [P]),
        "mrtlbm_last_error": (ctypes.c_char_p, []),
        "mrtlbm_batch_workspace_bytes": (SZ, [PP, I]),
        "mrtlbm_batch_solve": (I, [PP, I, D, I, LL, I, P, SZ, RP]),
        "mrtlbm_batch_autotune": (I, [PP, I, P, SZ, ctypes.POINTER(Launch)]),
    }
    F = ctypes.c_float
    FP = ctypes.POINTER(ctypes.c_float)
    sig.update({
        "mrtlbm_nn_kpad": (I, [I]),
        "mrtlbm_nn_conv3d_fwd": (I, [P, I, I, I, I, I, P, P, I, I, I, P, P, P]),
        "mrtlbm_nn_conv3d_dgrad": (I, [P, I, I, I, I, I, P, I, I, P, P, P]),
        "mrtlbm_nn_wgrad_scratch_bytes": (SZ, [I, I, I, I, I, I]),
        "mrtlbm_nn_conv3d_wgrad": (I, [P, P, I, I, I, I, I, I, I, P, P, P, P]),
        "mrtlbm_nn_relu_bwd": (I, [P, P, P, LL, P]),
        "mrtlbm_nn_add": (I, [P, P, P, LL, P]),
        "mrtlbm_nn_pool2": (I, [I, P, I, I, I, I, I, P, P]),
        "mrtlbm_nn_up2": (I, [I, P, I, I, I, I, I, P, P]),
        "mrtlbm_nn_mse": (I, [P, I, P, LL, P, P, P, P]),
        "mrtlbm_nn_adam": (I, [P, P, P, P, LL, F, F, F, F, I, P, P]),
        "mrtlbm_nn_to_bf16": (I, [P, LL, P, P]),
        "mrtlbm_nn_features": (I, [P, I, I, I, P, P, P]),
        "mrtlbm_nn_target": (I, [P, I, I, I, F, P, P]),
        "mrtlbm_nn_to_temperature": (I, [P, I, I, I, I, I, I, I, F, F, P, P, ctypes.POINTER(ctypes.c_longlong), P]),
        "mrtlbm_nn_feature_table": (I, [ctypes.POINTER(ctypes.c_double), I, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_float)]),
        "mrtlbm_nn_features_resampled": (I, [P, I, I, I, P, I, I, I, P, P]),
    })
    del FP
    sig["mrtlbm_set_progress"] = (None, [PROGRESS_FN, P, D])
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return _lib


def check(status: int, allow=(OK,)) -> int:
    if status in allow:
        return status
    msg = load().mrtlbm_last_error()
    raise MrtlbmError(status, msg.decode() if msg else "")
