"""Batched many-cell solver: on the FP64 oracle cell by cell, and identical
to stepping each cell alone."""

import numpy as np
import pytest

import workloads as w
from oracle import ADIABATIC, PERIODIC, Oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    from paper_1503_08718_amd import solver

    return solver


def _cells(api, prec):
    specs = [
        # (medium, grad axis, sides)
        (w.braid(16, 16, 24, 25.0, 0.45), 2, ("periodic", "periodic", "periodic")),
        (w.braid(24, 16, 16, 40.0, 0.55), 0, ("periodic", "adiabatic", "periodic")),
        (w.random_medium(3, 20, 12, 10, 3), 1, ("adiabatic", "periodic", "periodic")),
        (w.random_medium(4, 13, 9, 7, 2), 0, ("periodic", "adiabatic", "adiabatic")),  # odd nx
    ]
    out = []
    for m, g, sides in specs:
        c = api.Medium(m.phase, m.k, precision=prec)
        c.set_bc(g, 1.0, 0.0, sides)
        c.init()
        out.append(c)
    return out


ORACLE_SIDES = {"periodic": PERIODIC, "adiabatic": ADIABATIC}


@pytest.mark.parametrize("storage", ["populations", "moments"])
def test_batch_matches_oracle(api, storage):
    """Every cell of an FP64 batch (uneven sizes, braids and random media,
    all wall mixes, odd nx) against the oracle stepped beside it: 600 steps
    from a random start, field within 1e-12, the last check's wall and
    volume fluxes within 1e-10."""
    specs = [
        (w.braid(16, 16, 24, 25.0, 0.45), 2, ("periodic", "periodic", "periodic")),
        (w.braid(24, 16, 16, 40.0, 0.55), 0, ("periodic", "adiabatic", "periodic")),
        (w.random_medium(3, 20, 12, 10, 3), 1, ("adiabatic", "periodic", "periodic")),
        (w.random_medium(4, 13, 9, 7, 2), 0, ("periodic", "adiabatic", "adiabatic")),
        (w.random_medium(5, 7, 5, 11, 4), 2, ("adiabatic", "adiabatic", "periodic")),
        (w.random_medium(6, 40, 3, 2, 2), 0, ("periodic", "periodic", "adiabatic")),
    ]
    cells, oracles = [], []
    for i, (m, g, sides) in enumerate(specs):
        T0 = np.random.default_rng(80 + i).uniform(-0.5, 1.5, m.phase.shape)
        c = api.Medium(m.phase, m.k, precision="f64", storage=storage)
        c.set_bc(g, 0.8, -0.4, sides).init(T0)
        cells.append(c)
        o = Oracle(m.phase, m.k)
        o.set_bc(g, 0.8, -0.4, [ORACLE_SIDES[s] for s in sides])
        o.init(T0)
        oracles.append(o)
    res, st = api.batch_solve(cells, tol=1e-30, kind="keff", max_steps=600, check_every=200)
    assert st == "NOT_CONVERGED"
    for c, o, r in zip(cells, oracles, res):
        assert r["steps"] == 600
        o.step(600)
        to = o.temperature()
        tg = c.temperature().double().cpu().numpy()
        assert np.abs(tg - to).max() < 1e-12 * np.abs(to).max()
        # the check ran on the 600th step: wall fluxes of that step, volume
        # flux of the state it produced
        ko = o.keff()
        for key in ("keff_hot", "keff_cold", "keff_vol"):
            assert abs(r[key] - ko[key]) < 1e-10 * max(1.0, abs(ko[key])), key
        assert np.allclose(r["keff_col"], ko["keff_col"], rtol=1e-10, atol=1e-10)
        assert abs(r["resid"] - ko["resid"]) < 1e-13


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_equals_individual_steps(api, prec):
    import torch

    batch = _cells(api, prec)
    alone = _cells(api, prec)
    res, st = api.batch_solve(batch, tol=1e-30, kind="keff", max_steps=600, check_every=100)
    assert st == "NOT_CONVERGED"
    for b, a, r in zip(batch, alone, res):
        ra = a.solve(1e-30, "keff", 600, check_every=100)
        assert r["steps"] == ra["steps"] == 600
        assert torch.equal(b.state_get(), a.state_get())
        for key in ("keff_hot", "keff_cold", "keff_vol"):
            assert abs(r[key] - ra[key]) <= 1e-12 * max(1.0, abs(ra[key])), key
        assert r["resid"] == ra["resid"]


def test_batch_converges_each_cell_on_its_own_rule(api):
    batch = _cells(api, "f64")
    alone = _cells(api, "f64")
    res, st = api.batch_solve(batch, tol=1e-6, kind="keff", max_steps=400000, check_every=200)
    assert st == "OK"
    steps = set()
    for a, r in zip(alone, res):
        ra = a.solve(1e-6, "keff", 400000, check_every=200)
        assert r["converged"] and ra["converged"]
        assert r["steps"] == ra["steps"]
        assert abs(r["keff"] - ra["keff"]) <= 1e-12 * abs(ra["keff"])
        steps.add(r["steps"])
    assert len(steps) > 1  # cells left the batch at different times


def test_batch_sweep_cells_fp32(api):
    # a small stand-in of the parametric sweep: uneven sizes, angles, fractions
    cells = [dict(nx=24, ny=32, nz=16, gamma=22.0, v=0.4), dict(nx=32, ny=16, nz=24, gamma=44.0, v=0.58),
             dict(nx=16, ny=24, nz=32, gamma=31.0, v=0.36)]
    media = []
    for c in cells:
        m = w.braid(c["nx"], c["ny"], c["nz"], c["gamma"], c["v"])
        g = api.Medium(m.phase, m.k, precision="f32").set_bc(0).init()
        media.append(g)
    res, st = api.batch_solve(media, tol=1e-4, kind="keff", max_steps=500000, check_every=500)
    assert st == "OK"
    for r in res:
        assert r["converged"] and r["keff"] > 0.2


@pytest.mark.parametrize("storage", ["populations", "moments"])
def test_xcd_tile_order_and_batch_autotune(api, storage):
    """The XCD-aware tile order (map) and every shape the batch autotuner
    may pick leave the arithmetic alone: states stay bit-identical to
    stepping each cell alone."""
    import torch

    def cells():
        out = _cells(api, "f32")
        for c in out:
            c.set_storage(storage).init()
        return out

    alone = cells()
    for c in alone:
        c.step(600)
    for mp in (0, 1):
        batch = cells()
        batch[0].set_launch(1, 64, 2, 0, mp)  # vec 1: the odd-nx cell allows no more
        api.batch_solve(batch, tol=1e-30, kind="keff", max_steps=600, check_every=100)
        for b, a in zip(batch, alone):
            assert torch.equal(b.state_get(), a.state_get())
    batch = cells()
    best = api.batch_autotune(batch)
    assert best["vec"] == 1 and best["bx"] * best["by"] in (64, 128, 256) and best["map"] in (0, 1)
    assert batch[0].info()["launch"] == (best["vec"], best["bx"], best["by"], best["nt"], best["map"])
    for c in batch:
        c.init()
    res, st = api.batch_solve(batch, tol=1e-30, kind="keff", max_steps=600, check_every=100)
    assert all(r["steps"] == 600 for r in res)
    for b, a in zip(batch, alone):
        assert torch.equal(b.state_get(), a.state_get())


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_of_degenerate_cells(api, prec):
    # extents of 1 and 2 in one batch (one row per thread for nx = 1)
    import torch

    specs = [((1, 5, 4), 0, ("periodic", "periodic", "adiabatic")),
             ((5, 1, 3), 1, ("adiabatic", "periodic", "periodic")),
             ((4, 3, 1), 2, ("periodic", "adiabatic", "periodic")),
             ((2, 2, 2), 0, ("periodic", "adiabatic", "adiabatic")),
             ((1, 1, 1), 0, ("periodic", "periodic", "periodic")),
             ((8, 1, 1), 0, ("periodic", "periodic", "adiabatic"))]

    def make():
        out = []
        for i, (shape, g, sides) in enumerate(specs):
            m = w.random_medium(20 + i, *shape, 2)
            out.append(api.Medium(m.phase, m.k, precision=prec).set_bc(g, 1.0, 0.0, sides).init())
        return out

    batch, alone = make(), make()
    res, st = api.batch_solve(batch, tol=1e-30, kind="keff", max_steps=300, check_every=100)
    assert st == "NOT_CONVERGED"
    for b, a, r in zip(batch, alone, res):
        ra = a.solve(1e-30, "keff", 300, check_every=100)
        assert r["steps"] == ra["steps"] == 300
        assert torch.equal(b.state_get(), a.state_get())
        for key in ("keff_hot", "keff_cold", "keff_vol"):
            assert abs(r[key] - ra[key]) <= 1e-12 * max(1.0, abs(ra[key])), key


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_rows_longer_than_a_block(api, prec):
    """Rows of more nodes than a tile has threads are cut into x-chunks, one
    tile each; such a cell batched with short-row cells evolves bit for bit
    like the same cell stepped alone, and (FP64) like the oracle."""
    import torch

    specs = [((300, 3, 2), 0, ("periodic", "periodic", "adiabatic")),   # 300 > 256 threads at vec 1
             ((1030, 2, 2), 1, ("periodic", "periodic", "periodic")),   # periodic x across 5 chunks
             ((13, 6, 5), 2, ("adiabatic", "periodic", "periodic"))]

    def make():
        out = []
        for i, (shape, g, sides) in enumerate(specs):
            m = w.random_medium(90 + i, *shape, 3)
            T0 = np.random.default_rng(90 + i).uniform(0, 1, m.phase.shape)
            out.append((m, g, sides, T0, api.Medium(m.phase, m.k, precision=prec).set_bc(g, 1.0, 0.0, sides).init(T0)))
        return out

    batch, alone = make(), make()
    batch[0][4].set_launch(1, 64, 1, 0, 1)  # 64 threads per tile: 300 nodes = 5 chunks
    res, st = api.batch_solve([b[4] for b in batch], tol=1e-30, kind="keff", max_steps=200, check_every=100)
    assert st == "NOT_CONVERGED"
    for (m, g, sides, T0, b), (_, _, _, _, a), r in zip(batch, alone, res):
        ra = a.solve(1e-30, "keff", 200, check_every=100)
        assert r["steps"] == ra["steps"] == 200
        assert torch.equal(b.state_get(), a.state_get())
        if prec == "f64":
            o = Oracle(m.phase, m.k)
            o.set_bc(g, 1.0, 0.0, [ORACLE_SIDES[s] for s in sides])
            o.init(T0)
            o.step(200)
            to = o.temperature()
            assert np.abs(b.temperature().cpu().numpy() - to).max() < 1e-12 * np.abs(to).max()
