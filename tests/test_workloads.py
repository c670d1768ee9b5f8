"""Input generators and the unit-cell calculators (Eqs. 26, 32-37)."""

import math

import numpy as np
import pytest

import workloads as w
from conftest import golden


def test_table2_yarn_conductivities():
    g = golden("table2_yarn_conductivity.json")
    for phi_f, lam_l, lam_t in g["rows"]:
        L, T = w.yarn_conductivities(phi_f)
        assert abs(L - lam_l) <= 1.5 * g["printed_precision"]
        assert abs(T - lam_t) <= 1.5 * g["printed_precision"]


def test_eq37_printed_numerator_does_not_reproduce_table2():
    # the reading phi_fy (not 1 - phi_fy) in the numerator is forced by Table II
    lam_m, lam_ft = 0.178, 0.675
    for phi_f, _, lam_t in golden("table2_yarn_conductivity.json")["rows"]:
        phi_fy = phi_f / 0.68
        printed = lam_m + (1 - phi_fy) / (1 / (lam_ft - lam_m) + (1 - phi_fy) / (2 * lam_m))
        assert abs(printed - lam_t) > 0.05


def test_sec5_unit_cell_geometry():
    g = golden("sec5_unit_cell.json")
    geo = w.unit_cell_geometry(g["phi_f"], g["gamma_deg"])
    for key in ("a", "h", "c", "d"):
        assert abs(geo[key] - g[key]) <= 1.5 * g["printed_precision"], key
    # grid 56 x 56 x 120: the voxel is a/56 and h / (a/56) ~ 120
    assert abs(geo["h"] / (geo["a"] / 56) - 120) < 0.5
    # Eq. 35: yarn fraction pi sqrt(3)/8 ~ 0.68
    assert abs(w.PHI_Y_EXACT - 0.68) < 5e-4
    # c = sqrt(3) d cos gamma (Eq. 33) and a = 8 d (Eq. 32)
    assert math.isclose(geo["c"], math.sqrt(3) * geo["d"] * math.cos(math.radians(25)))
    assert math.isclose(geo["a"], 8 * geo["d"])


def test_eq26_rotation_entries():
    t = w.slab_tensor_eq26(2.0, 1.0, 75.0)
    b = math.radians(75.0)
    assert math.isclose(t[1, 1], 2 * math.sin(b) ** 2 + math.cos(b) ** 2)
    assert math.isclose(t[0, 0], 2 * math.cos(b) ** 2 + math.sin(b) ** 2)
    assert np.allclose(t, t.T)
    assert np.allclose(np.linalg.eigvalsh(t[:2, :2]), [1.0, 2.0])


def test_c1_tensor():
    m = w.c1_layered()
    assert m.shape == (16, 16, 16)
    assert np.allclose(m.k[0], [0.875, 0.625, 0.5, 0.21650635, 0, 0])
    assert np.allclose(m.k[1], [0.2, 0.2, 0.2, 0, 0, 0])
    assert (m.phase[:, :, :8] == 0).all() and (m.phase[:, :, 8:] == 1).all()


def test_braid_tensor_and_fraction():
    m = w.braid(32, 32, 32, 30.0, 0.5)
    assert m.phase.dtype == np.uint8 and m.phase.shape == (32, 32, 32)
    assert abs((m.phase > 0).mean() - 0.5) <= 0.002
    assert set(np.unique(m.phase)) <= {0, 1, 2, 3, 4}
    assert np.allclose(m.k[1], [2.125, 2.125, 7.75, 1.125, 2.7557, 2.7557], atol=1e-4)
    for r in m.k:
        assert np.all(np.linalg.eigvalsh(w.full3(r)) > 0)
    # family axes: eigenvalues (10, 1, 1)
    assert np.allclose(sorted(np.linalg.eigvalsh(w.full3(m.k[2]))), [1, 1, 10])


def test_braid_deterministic_and_symmetric_under_quarter_turn_counts():
    a = w.braid(24, 24, 16, 35.0, 0.45)
    b = w.braid(24, 24, 16, 35.0, 0.45)
    assert np.array_equal(a.phase, b.phase)


def test_sweep_cells_seeded():
    c1 = w.sweep_cells(1503)
    c2 = w.sweep_cells(1503)
    assert c1 == c2 and len(c1) == 64
    for c in c1:
        assert c["nx"] in (64, 96, 128) and 20 <= c["gamma"] <= 45 and 0.35 <= c["v"] <= 0.6


def test_permuted_medium_roundtrip():
    m = w.random_medium(3, 5, 4, 3, 3)
    p = m.permuted((1, 2, 0))
    assert p.phase.shape == (m.nx, m.nz, m.ny)  # (z', y', x') = (x, z, y)
    # voxel (x', y', z') of p is voxel (x=z', y=x', z=y') of m
    assert p.phase[2, 1, 3] == m.phase[1, 3, 2]
    K = w.full3(m.k[1])
    Kp = w.full3(p.k[1])
    assert math.isclose(Kp[0, 0], K[1, 1]) and math.isclose(Kp[0, 2], K[1, 0])


def test_braid_voxelisation_independent_of_threads_and_slabs():
    from workloads.media import _braid_radius

    r1, f1 = _braid_radius(20, 12, 18, 33.0, z_chunk=18, workers=1)
    for chunk, workers in ((1, 4), (5, 3), (7, 16)):
        r, f = _braid_radius(20, 12, 18, 33.0, z_chunk=chunk, workers=workers)
        assert np.array_equal(r, r1) and np.array_equal(f, f1), (chunk, workers)
