"""The allocation-free solve (mrtlbm_solve_noalloc) against mrtlbm_solve.

Both run the same kernels with the same block shapes and reduction order;
only where the check partials live (a fixed device array vs the medium's
workspace) and how the steps are launched (one by one vs graph replays)
differ.  Two calls in a row, the second on a smaller medium, each checked
against mrtlbm_solve on an identical medium: results and final states bit
for bit (FP64 and FP32)."""

import ctypes

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    from paper_1503_08718_amd import _lib, solver

    return solver, _lib


def _noalloc(lib_mod, g, tol, kind, max_steps, check_every):
    L = lib_mod.load()
    r = lib_mod.Result()
    st = L.mrtlbm_solve_noalloc(g.handle, float(tol), {"maxdt": 0, "keff": 1}[kind], int(max_steps),
                                int(check_every), ctypes.byref(r))
    return st, r.to_dict()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_solve_equals_solve(env, prec):
    import torch

    solver, lib_mod = env
    cases = [(w.braid(40, 32, 48, 30.0, 0.5), 0, ("periodic", "adiabatic", "periodic"), 1e-5, 600_000),
             (w.random_medium(9, 12, 10, 8, 3), 2, ("adiabatic", "periodic", "periodic"), 1e-6, 400_000)]
    for m, grad, sides, tol, max_steps in cases:  # the second call runs on a smaller medium
        a = solver.Medium(m.phase, m.k, precision=prec).set_bc(grad, 1.0, 0.0, sides).init()
        b = solver.Medium(m.phase, m.k, precision=prec).set_bc(grad, 1.0, 0.0, sides).init()
        ra = a.solve(tol, "keff", max_steps, check_every=200)
        st, rb = _noalloc(lib_mod, b, tol, "keff", max_steps, 200)
        assert st == 0 and ra["status"] == "OK", (st, ra)
        for key in ("keff", "keff_hot", "keff_cold", "keff_vol", "resid", "keff_leak", "steps", "converged"):
            assert rb[key] == ra[key], (key, rb[key], ra[key])
        assert rb["keff_col"] == ra["keff_col"]
        assert torch.equal(a.state_get(), b.state_get())
        # a run that ends on max_steps (a partial last block) as well
        c = solver.Medium(m.phase, m.k, precision=prec).set_bc(grad, 1.0, 0.0, sides).init()
        d = solver.Medium(m.phase, m.k, precision=prec).set_bc(grad, 1.0, 0.0, sides).init()
        rc = c.solve(1e-30, "keff", 1234, check_every=100)
        st, rd = _noalloc(lib_mod, d, 1e-30, "keff", 1234, 100)
        assert st == 1 and rc["status"] == "NOT_CONVERGED"
        assert rd["steps"] == rc["steps"] == 1234 and rd["keff"] == rc["keff"]
        assert torch.equal(c.state_get(), d.state_get())


def test_noalloc_rejects_a_check_step_beyond_its_scratch(env):
    solver, lib_mod = env
    # 1025 x 65 row blocks of 64 threads: more check partials than the fixed
    # array holds; refused before any device work
    m = w.Medium(np.zeros((1, 65, 65600), np.uint8), np.array([[1.0, 1.0, 1.0, 0.0, 0.0, 0.0]]))
    g = solver.Medium(m.phase, m.k, precision="f32").set_bc(0).set_launch(1, 64, 1, 0, 0).init()
    st, _ = _noalloc(lib_mod, g, 1e-4, "keff", 100, 10)
    assert st == -7  # MRTLBM_E_WORKSPACE
    assert b"scratch" in lib_mod.load().mrtlbm_last_error()
