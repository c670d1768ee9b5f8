"""The HIP library loads and exports the C ABI (no GPU compute here)."""

import ctypes
import os
import subprocess

import pytest

import paper_1503_08718_amd as pkg
from paper_1503_08718_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmrtlbm.so is not built (run __graft_entry__.build())")
    return pkg.load()


def test_every_declared_symbol_is_exported(lib):
    names = pkg.declared_symbols()
    assert "mrtlbm_create" in names and "mrtlbm_batch_solve" in names
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True, check=True)
    exported = {l.split()[-1] for l in out.stdout.splitlines() if " T " in l}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert getattr(lib, n) is not None


def test_library_carries_only_gfx950_code():
    blob = open(_lib.LIB_PATH, "rb").read()
    import re

    targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx[0-9a-z]+)", blob))
    assert targets == {b"gfx950"}, targets


def test_workspace_bytes(lib):
    f32 = lib.mrtlbm_workspace_bytes(128, 128, 128, 5, _lib.F32)
    f64 = lib.mrtlbm_workspace_bytes(128, 128, 128, 5, _lib.F64)
    n = 128 ** 3
    assert f32 >= 2 * 7 * n * 4 and f64 >= 2 * 7 * n * 8
    assert f32 < 2 * 7 * n * 4 * 1.02
    assert lib.mrtlbm_workspace_bytes(0, 4, 4, 2, _lib.F32) == 0
    assert lib.mrtlbm_workspace_bytes(4, 4, 4, 0, _lib.F32) == 0
    assert lib.mrtlbm_workspace_bytes(4, 4, 4, 300, _lib.F32) == 0
    assert lib.mrtlbm_workspace_bytes(4, 4, 4, 2, 7) == 0
    # moment storage: two buffers of 4 values per node
    m32 = lib.mrtlbm_workspace_bytes_storage(128, 128, 128, 5, _lib.F32, 1)
    assert 2 * 4 * n * 4 <= m32 < 2 * 4 * n * 4 * 1.03
    assert lib.mrtlbm_workspace_bytes_storage(128, 128, 128, 5, _lib.F32, 0) == f32
    assert lib.mrtlbm_workspace_bytes_storage(4, 4, 4, 2, _lib.F32, 2) == 0


def test_errors_before_any_device_work(lib):
    # argument checks that return before the library touches the device
    out = ctypes.c_void_p()
    k = (ctypes.c_double * 6)(1, 1, 1, 0, 0, 0)
    st = lib.mrtlbm_create(4, 4, 4, None, k, 1, _lib.F32, None, 0, None, ctypes.byref(out))
    assert st == -1 and b"NULL" in lib.mrtlbm_last_error()
    bad = (ctypes.c_double * 6)(1, 1, 1, 2, 0, 0)  # not positive definite
    fake = ctypes.c_void_p(256)
    ws = lib.mrtlbm_workspace_bytes(4, 4, 4, 1, _lib.F32)
    st = lib.mrtlbm_create(4, 4, 4, fake, bad, 1, _lib.F32, fake, ws, None, ctypes.byref(out))
    assert st == -2
    wsm = lib.mrtlbm_workspace_bytes_storage(4, 4, 4, 1, _lib.F32, 1)
    st = lib.mrtlbm_create(4, 4, 4, fake, k, 1, _lib.F32, fake, wsm - 1, None, ctypes.byref(out))
    assert st == -7
    assert lib.mrtlbm_set_bc(None, 0, 1.0, 0.0, None) == -1
    assert lib.mrtlbm_step(None, 1) == -1


def test_product_does_not_touch_the_oracle():
    src = os.path.join(ROOT, "paper_1503_08718_amd")
    for dirpath, _, files in os.walk(src):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "oracle" not in txt.lower(), fn


def _c_kind(decl: str) -> str:
    """Argument class of one C parameter (type and name) or return type."""
    words = decl.replace("*", " * ").replace("[", " [ ").replace("const", " ").split()
    if "*" in words or "[" in words or words[0] == "mrtlbm_progress_fn":
        return "ptr"
    kinds = {("long", "long"): "ll", ("double",): "double", ("float",): "float", ("size_t",): "size",
             ("int",): "int", ("mrtlbm_precision",): "int", ("mrtlbm_tol_kind",): "int",
             ("mrtlbm_status",): "int", ("void",): "void"}
    for n in (2, 1):
        if tuple(words[:n]) in kinds:
            return kinds[tuple(words[:n])]
    raise AssertionError(f"unknown C type in {decl!r}")


def _py_kind(t) -> str:
    if t is None:
        return "void"
    if t in (ctypes.c_void_p, ctypes.c_char_p) or hasattr(t, "_type_") and isinstance(t._type_, type) \
            or getattr(t, "_flags_", 0) & 1:  # POINTER(...) or CFUNCTYPE(...)
        return "ptr"
    return {ctypes.c_double: "double", ctypes.c_float: "float", ctypes.c_int: "int", ctypes.c_longlong: "ll",
            ctypes.c_size_t: "size"}[t]


def test_binding_signatures_match_the_headers(lib):
    # every declared function: same arity and argument classes in the ctypes binding
    import re

    decls = {}
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(inc, fn)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", "", txt)
        txt = "\n".join(l for l in txt.splitlines() if not l.lstrip().startswith("#"))
        for m in re.finditer(r"([A-Za-z_][\w\s\*]*?)\b(mrtlbm_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", txt, flags=re.S):
            ret, name, params = m.group(1), m.group(2), " ".join(m.group(3).split())
            ret = ret.split("\n")[-1].strip() or ret.strip()
            if "typedef" in ret:
                continue
            args = [] if params in ("", "void") else [_c_kind(p) for p in params.split(",")]
            decls[name] = (_c_kind(ret.replace("extern", "").replace('"C"', "").strip()), args)
    assert len(decls) == len(pkg.declared_symbols()), sorted(set(pkg.declared_symbols()) - set(decls))
    for name, (ret, args) in decls.items():
        f = getattr(lib, name)
        got = [_py_kind(a) for a in (f.argtypes or [])]
        assert got == args, (name, got, args)
        assert _py_kind(f.restype) == ret, (name, f.restype, ret)
