"""Parity at the benchmark's own configuration: the 256^3 braided cell
(braiding angle 30 deg, yarn fraction 0.5) in FP32 and in FP64, both state
storages, each with the launch shape the benchmark loads from the autotune
cache, against the FP64 oracle.  The FP64 GPU path at this size is the
reference that FP32 k_eff errors at 256^3 are measured against.

Collected last: with the FP64 oracle on the whole cell it is the longest
of the GPU tests."""

import os

import numpy as np
import pytest

import workloads as w
from oracle import PERIODIC, Oracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE = os.path.join(ROOT, "paper_1503_08718_amd", "tuned_launch.txt")
N = 256
STEPS = 12


@pytest.fixture(scope="module")
def Medium():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    from paper_1503_08718_amd.solver import Medium

    return Medium


@pytest.fixture(scope="module")
def cell():
    m = w.braid(N, N, N, 30.0, 0.5)
    rng = np.random.default_rng(N)
    # smooth random start so that every node moves from the first step
    z, y, x = np.meshgrid(*(np.linspace(0, 2 * np.pi, N, endpoint=False),) * 3, indexing="ij")
    T0 = 0.5 + 0.3 * np.sin(x + rng.uniform(0, 6)) * np.cos(2 * y) + 0.1 * np.sin(3 * z)
    del x, y, z
    o = Oracle(m.phase, m.k)
    o.set_threads(0)
    o.set_bc(0, 1.0, 0.0, (PERIODIC, PERIODIC, PERIODIC))
    o.init(T0)
    o.step(STEPS)
    t_ref = o.temperature()
    o.step(1)
    k_ref = o.keff()
    del o
    return m, T0, t_ref, k_ref


def _tuned_launch(storage, prec):
    key = f"{N} {N} {N} {prec}{'m' if storage == 'moments' else 'd'}"
    for line in open(TUNE):
        parts = line.split()
        if len(parts) >= 10 and " ".join(parts[1:5]) == key:
            return tuple(int(v) for v in parts[5:10])
    raise AssertionError(f"no tuned launch for {key}")


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("storage", ["moments", "populations"])
def test_bench_configuration_256(Medium, cell, storage, prec):
    m, T0, t_ref, k_ref = cell
    g = Medium(m.phase, m.k, precision=prec, storage=storage)
    assert g.load_tuned(TUNE)
    assert g.info()["launch"] == _tuned_launch(storage, prec)
    g.set_bc(0, 1.0, 0.0, ("periodic", "periodic", "periodic")).init(T0)
    g.step(STEPS)
    tg = g.temperature().double().cpu().numpy()
    # FP64: rounding-order differences only; FP32 state: a few ulp of T per
    # step over 12 steps
    tol, ktol = (1e-12, 1e-9) if prec == "f64" else (2e-6, 2e-3)
    assert np.abs(tg - t_ref).max() < tol * np.abs(t_ref).max()
    kg = g.keff()
    assert abs(kg["keff_vol"] - k_ref["keff_vol"]) < ktol * abs(k_ref["keff_vol"])
    if prec == "f64":
        for key in ("keff_hot", "keff_cold"):
            assert abs(kg[key] - k_ref[key]) < 1e-9 * max(1.0, abs(k_ref[key])), key
    g.close()
