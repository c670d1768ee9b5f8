"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself:
closed-form solutions (series and parallel laminates, homogeneous rotated
tensors, Table I), algebraic identities of the collision operator derived from
the orthogonality of M (Eq. 11), library routines (numpy.roll for periodic
streaming, numpy.linalg.solve for the steady state of the affine one-step
map), conservation laws, exact lattice symmetries and the values the paper
prints.
"""

import math

import numpy as np
import pytest

import workloads as w
from conftest import golden
from oracle import ADIABATIC, PERIODIC, TOL_KEFF, TOL_MAXDT, Oracle
from oracle import matrix_form as mf

EPS = 0.25


def make(m, grad=0, sides=(PERIODIC, PERIODIC, PERIODIC), dmax=1.0, t_hot=1.0, t_cold=0.0, T0=None, **kw):
    o = Oracle(m.phase, m.k, dmax=dmax, **kw)
    o.set_bc(grad, t_hot, t_cold, sides)
    o.init(T0)
    return o


def closed_form_collision(f, tau):
    """Post-collision state from the moment algebra: with tau_4 = tau_5 =
    tau_6 = 1, M's orthogonal rows give f_hat_0 = T/4 and
    f_hat_{2a+1,2a+2} = T/8 +- jhat_a / 2 with jhat = (I - tau^-1) j."""
    T = f.sum()
    j = np.array([f[1] - f[2], f[3] - f[4], f[5] - f[6]])
    jh = (np.eye(3) - np.linalg.inv(tau)) @ j
    out = np.empty(7)
    out[0] = T / 4
    for a in range(3):
        out[1 + 2 * a] = T / 8 + jh[a] / 2
        out[2 + 2 * a] = T / 8 - jh[a] / 2
    return out


# ---------------------------------------------------------------------------
# collision operator
# ---------------------------------------------------------------------------


def test_collision_equals_moment_closed_form():
    m = w.random_medium(11, 3, 3, 3, nphase=4)
    o = make(m)
    rng = np.random.default_rng(5)
    for p in range(4):
        tau = o.tau(p)
        for _ in range(20):
            f = rng.standard_normal(7)
            assert np.allclose(o.collide_node(p, f), closed_form_collision(f, tau), rtol=0, atol=1e-14)


def test_tau_from_eq13_and_scale():
    m = w.random_medium(12, 2, 2, 2, nphase=3)
    o = make(m, dmax=0.8)
    lmax = max(np.linalg.eigvalsh(w.full3(r)).max() for r in m.k)
    assert math.isclose(o.scale, 0.8 * EPS / lmax, rel_tol=1e-14)
    for p in range(3):
        expect = 0.5 * np.eye(3) + o.scale * w.full3(m.k[p]) / EPS
        assert np.allclose(o.tau(p), expect, atol=1e-15)
    # the largest eigenvalue of tau - I/2 over all phases is dmax
    top = max(np.linalg.eigvalsh(o.tau(p) - 0.5 * np.eye(3)).max() for p in range(3))
    assert math.isclose(top, 0.8, rel_tol=1e-13)


def test_omega_independent_of_c_placement():
    # Eq. 11 carries a factor c; it cancels in M^-1 S M whether it scales all
    # of M or only the flux rows.
    m = w.random_medium(13, 2, 2, 2, nphase=2)
    o = make(m)
    for p in range(2):
        tau = o.tau(p)
        base = o.omega(p)
        for c, rows in ((1.0, False), (3.7, False), (0.01, True), (250.0, True)):
            assert np.allclose(base, mf.omega(tau, c=c, rows_123_only=rows), atol=1e-12)


@pytest.mark.parametrize("tau_rest", [(1, 1, 1, 1), (0.8, 1.3, 0.7, 1.9)])
def test_collision_conserves_T_and_keeps_equilibrium(tau_rest):
    m = w.random_medium(14, 2, 2, 2, nphase=2)
    o = make(m, tau_rest=np.array(tau_rest, float))
    wv = np.array([0.25] + [0.125] * 6)
    rng = np.random.default_rng(0)
    for p in range(2):
        P = np.stack([o.collide_node(p, e) for e in np.eye(7)], axis=1)
        assert np.allclose(P.sum(axis=0), 1.0, atol=1e-14)  # 1^T P = 1^T
        assert np.allclose(P @ wv, wv, atol=1e-14)  # P w = w
        f = rng.standard_normal(7)
        assert math.isclose(o.collide_node(p, f).sum(), f.sum(), rel_tol=0, abs_tol=1e-13)


# ---------------------------------------------------------------------------
# streaming and walls
# ---------------------------------------------------------------------------


def _post_collision(o, m, f):
    out = np.empty_like(f)
    nz, ny, nx = m.phase.shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                out[:, z, y, x] = closed_form_collision(f[:, z, y, x], o.tau(m.phase[z, y, x]))
    return out


@pytest.mark.parametrize("side_y", [PERIODIC, ADIABATIC])
def test_streaming_matches_numpy_roll(side_y):
    m = w.random_medium(21, 5, 4, 3, nphase=3)
    o = make(m, grad=0, sides=(0, side_y, PERIODIC), t_hot=0.7, t_cold=-0.3)
    rng = np.random.default_rng(1)
    f = rng.standard_normal((7,) + m.phase.shape)
    o.set_f(f)
    o.step(1)
    fh = _post_collision(o, m, f)
    exp = np.empty_like(fh)
    exp[0] = fh[0]
    # array axes are (z, y, x); population 2a+1 moves +a, 2a+2 moves -a
    for i, (ax, sh) in enumerate([(2, 1), (2, -1), (1, 1), (1, -1), (0, 1), (0, -1)], start=1):
        exp[i] = np.roll(fh[i], sh, axis=ax)
    # x walls: Dirichlet, Eq. 23
    exp[1][:, :, 0] = -fh[2][:, :, 0] + EPS * 0.7
    exp[2][:, :, -1] = -fh[1][:, :, -1] + EPS * (-0.3)
    if side_y == ADIABATIC:  # Eq. 24 with zero flux
        exp[3][:, 0, :] = fh[4][:, 0, :]
        exp[4][:, -1, :] = fh[3][:, -1, :]
    assert np.allclose(o.get_f(), exp, rtol=0, atol=1e-14)


def test_energy_identity_per_step():
    m = w.random_medium(22, 6, 5, 4, nphase=3)
    o = make(m, grad=1, sides=(ADIABATIC, 0, PERIODIC), t_hot=0.9, t_cold=0.1)
    rng = np.random.default_rng(2)
    f = rng.uniform(0, 0.2, (7,) + m.phase.shape)
    o.set_f(f)
    fh = _post_collision(o, m, f)
    before = f.sum()
    o.step(1)
    after = o.get_f().sum()
    # gradient along y: hot face at y = 0 loses population 4 (moving -y)
    phi_hot = (EPS * 0.9 - 2 * fh[4][:, 0, :]).sum()
    phi_cold = (2 * fh[3][:, -1, :] - EPS * 0.1).sum()
    assert math.isclose(after - before, phi_hot - phi_cold, rel_tol=1e-12, abs_tol=1e-13)
    lf = o.last_fluxes()
    assert math.isclose(lf["phi_hot"], phi_hot, rel_tol=1e-12)
    assert math.isclose(lf["phi_cold"], phi_cold, rel_tol=1e-12)


def test_energy_identity_with_side_flux():
    # Eq. 24 with phi_n != 0: each Neumann link adds s q per step
    m = w.random_medium(23, 6, 5, 4, nphase=3)
    o = make(m, grad=2, sides=(ADIABATIC, ADIABATIC, 0), t_hot=0.6, t_cold=-0.2)
    qs = {0: (0.3, -0.7), 1: (-0.2, 0.45)}
    for a, (lo, hi) in qs.items():
        o.set_side_flux(a, lo, hi)
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 0.2, (7,) + m.phase.shape)
    o.set_f(f)
    fh = _post_collision(o, m, f)
    before = f.sum()
    o.step(1)
    after = o.get_f().sum()
    phi_hot = (EPS * 0.6 - 2 * fh[6][0, :, :]).sum()
    phi_cold = (2 * fh[5][-1, :, :] - EPS * (-0.2)).sum()
    nz, ny, nx = m.phase.shape
    side = o.scale * ((qs[0][0] + qs[0][1]) * ny * nz + (qs[1][0] + qs[1][1]) * nx * nz)
    assert math.isclose(after - before, phi_hot - phi_cold + side, rel_tol=1e-12, abs_tol=1e-13)
    # the reflected link itself: population 1 re-enters at x = 0 as f_hat_2 + s q_lo
    assert np.allclose(o.get_f()[1][:, :, 0], fh[2][:, :, 0] + o.scale * qs[0][0], atol=1e-14)
    assert np.allclose(o.get_f()[4][:, -1, :], fh[3][:, -1, :] + o.scale * qs[1][1], atol=1e-14)


# ---------------------------------------------------------------------------
# closed-form steady states
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("tau_rest", [(1, 1, 1, 1), (1, 0.7, 1.6, 1.2)])
def test_side_flux_of_the_linear_solution_makes_it_exact(tau_rest):
    """A homogeneous anisotropic cell with a z gradient: with periodic sides
    the steady field is T_lin(z) and the flux q = -K grad T has side
    components q_x = K_xz dT/L, q_y = K_yz dT/L.  Imposing exactly those
    fluxes on Neumann x and y faces (in through the low face, out through the
    high one) keeps T_lin(z) exact, so k = K_zz; zero flux (adiabatic) does
    not.  Holds for any tau_4..6."""
    rng = np.random.default_rng(33)
    K = w.random_spd(rng, 0.3, 1.5)
    K[0, 2] = K[2, 0] = 0.3
    K[1, 2] = K[2, 1] = -0.25
    assert np.all(np.linalg.eigvalsh(K) > 0)
    nx, ny, nz = 5, 4, 9
    m = w.Medium(np.zeros((nz, ny, nx), np.uint8), w.sym6(K)[None, :])
    dT = 1.0
    o = make(m, grad=2, sides=(ADIABATIC, ADIABATIC, 0), tau_rest=np.array(tau_rest, float))
    qx, qy = K[0, 2] * dT / nz, K[1, 2] * dT / nz
    o.set_side_flux(0, qx, -qx)
    o.set_side_flux(1, qy, -qy)
    r = o.solve(1e-15, TOL_MAXDT, 2_000_000)
    tlin = 1.0 - (np.arange(nz) + 0.5) / nz
    assert np.allclose(o.temperature(), tlin[:, None, None], rtol=0, atol=1e-11)
    assert math.isclose(r["keff_hot"], K[2, 2], rel_tol=1e-9)
    assert math.isclose(r["keff_cold"], K[2, 2], rel_tol=1e-9)
    # the energy-balance stop rule sees the side inflow (here zero net)
    o2 = make(m, grad=2, sides=(ADIABATIC, ADIABATIC, 0), tau_rest=np.array(tau_rest, float))
    o2.set_side_flux(0, qx, -qx)
    o2.set_side_flux(1, qy, -qy)
    assert o2.solve(1e-9, TOL_KEFF, 2_000_000, check_every=20)["converged"]
    a = make(m, grad=2, sides=(ADIABATIC, ADIABATIC, 0), tau_rest=np.array(tau_rest, float))
    ra = a.solve(1e-15, TOL_MAXDT, 2_000_000)
    assert ra["keff_hot"] < K[2, 2] * (1 - 1e-3)


def test_side_inflow_balances_at_steady_state():
    # net heat put in through the sides leaves through the walls:
    # Phi_cold - Phi_hot = s * sum of q * face area
    m = w.random_medium(24, 5, 6, 4, nphase=2)
    o = make(m, grad=0, sides=(0, ADIABATIC, ADIABATIC))
    o.set_side_flux(1, 0.05, 0.02)
    o.set_side_flux(2, -0.01, 0.04)
    o.solve(1e-15, TOL_MAXDT, 2_000_000)
    o.step(1)
    lf = o.last_fluxes()
    nz, ny, nx = m.phase.shape
    side = o.scale * ((0.05 + 0.02) * nx * nz + (-0.01 + 0.04) * nx * ny)
    assert math.isclose(lf["phi_cold"] - lf["phi_hot"], side, rel_tol=1e-9)


def test_c1_layered_series_mean():
    m = w.c1_layered(16)
    o = make(m, grad=0)
    r = o.solve(1e-10, TOL_MAXDT, 200000)
    exact = 14.0 / 43.0  # 2 * 0.875 * 0.2 / (0.875 + 0.2)
    assert r["converged"]
    for key in ("keff_vol", "keff_hot", "keff_cold"):
        assert abs(r[key] - exact) / exact < 1e-6, key


def test_table1_series_slabs():
    g = golden("table1_series_slabs.json")
    for ratio, a75, _, a15, _ in g["rows"]:
        for beta, printed in ((75.0, a75), (15.0, a15)):
            m = w.table1_slabs(ratio, beta, n_per_slab=5, nx=1)
            ly = [w.full3(r)[1, 1] for r in m.k]
            exact = 2 * ly[0] * ly[1] / (ly[0] + ly[1])
            assert abs(exact - printed) <= 1.5e-4
            o = make(m, grad=1, dmax=1.0)
            r = o.solve(1e-15, TOL_MAXDT, 2_000_000)
            assert r["converged"]
            assert abs(r["keff_vol"] - exact) / exact < 1e-9, (ratio, beta, r)
            assert abs(r["keff_hot"] - exact) / exact < 1e-9


def _series_profile(m, keff, axis):
    """Exact steady temperature of a series laminate (T = 1 -> 0)."""
    kk = [w.full3(r)[axis, axis] for r in m.k]
    n = m.phase.shape[2 - axis]
    sl = [0, 0, 0]
    idx = []
    for i in range(n):
        sl[2 - axis] = i
        idx.append(m.phase[tuple(sl)])
    q = keff / n  # flux for dT = 1 over n voxels
    T = np.empty(n)
    t = 1.0
    for i in range(n):
        t -= 0.5 * q / kk[idx[i]]
        T[i] = t
        t -= 0.5 * q / kk[idx[i]]
    shape = [1, 1, 1]
    shape[2 - axis] = n
    return np.broadcast_to(T.reshape(shape), m.phase.shape).copy()


def test_homogeneous_rotated_tensor_gives_its_column():
    rng = np.random.default_rng(31)
    k = w.random_spd(rng, 0.3, 1.5)
    m = w.Medium(np.zeros((2, 2, 10), np.uint8), w.sym6(k)[None, :])
    o = make(m, grad=0)
    r = o.solve(1e-15, TOL_MAXDT, 1_000_000)
    assert np.allclose(r["keff_col"], k[:, 0], rtol=1e-9, atol=1e-12)
    assert math.isclose(r["keff_hot"], k[0, 0], rel_tol=1e-9)


def test_parallel_laminate_arithmetic_mean():
    # layers normal to y, tensors rotated about y: no x-y coupling
    tA = w.rotate_tensor([1.0, 0.5, 0.3], w.rot_y(25.0))
    tB = w.rotate_tensor([0.2, 0.4, 0.9], w.rot_y(-40.0))
    m = w.layered((8, 6, 2), 1, [2, 4], [tA, tB])
    o = make(m, grad=0)
    r = o.solve(1e-15, TOL_MAXDT, 2_000_000)
    exact = (2 * tA[0, 0] + 4 * tB[0, 0]) / 6
    assert abs(r["keff_vol"] - exact) / exact < 1e-9


def test_refinement_and_scale_leave_laminates_unchanged():
    tA = w.rotate_tensor([1.0, 0.5, 0.5], w.rot_z(30.0))
    tB = 0.2 * np.eye(3)
    res = []
    for n, dmax in ((8, 1.0), (16, 1.0), (8, 0.4)):
        m = w.layered((n, 1, 1), 0, [n // 2, n // 2], [tA, tB])
        T0 = _series_profile(m, 14 / 43, axis=0)
        o = make(m, grad=0, dmax=dmax, T0=T0)
        res.append(o.solve(1e-12, TOL_KEFF, 2_000_000, check_every=50)["keff_vol"])
    assert np.allclose(res, 14 / 43, rtol=1e-9)


# ---------------------------------------------------------------------------
# whole fixed point, inequalities and symmetries
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("sides", [(0, ADIABATIC, PERIODIC), (0, PERIODIC, ADIABATIC)])
def test_dense_fixed_point(sides):
    m = w.random_medium(41, 3, 3, 3, nphase=3, lo=0.3, hi=1.5)
    fstar, s = mf.fixed_point(m.phase, m.k, 1.0, 0, 1.0, 0.0, sides)
    o = make(m, grad=0, sides=sides)
    assert math.isclose(o.scale, s, rel_tol=1e-14)
    o.solve(1e-16, TOL_MAXDT, 200000)
    assert np.allclose(o.get_f(), fstar, rtol=0, atol=1e-12)
    # one more step leaves the fixed point where it is
    L, b, _ = mf.affine_step(m.phase, m.k, 1.0, 0, 1.0, 0.0, sides)
    fs = fstar.reshape(-1)
    assert np.allclose(L @ fs + b, fs, atol=1e-13)


def test_adiabatic_bounds_homogeneous_layer_a():
    kA = w.rotate_tensor([1.0, 0.5, 0.5], w.rot_z(30.0))
    m = w.Medium(np.zeros((1, 8, 8), np.uint8), w.sym6(kA)[None, :])
    per = make(m, grad=0).solve(1e-14, TOL_MAXDT, 1_000_000)["keff_vol"]
    adi = make(m, grad=0, sides=(0, ADIABATIC, PERIODIC)).solve(1e-14, TOL_MAXDT, 1_000_000)["keff_vol"]
    assert math.isclose(per, 0.875, rel_tol=1e-8)
    lower = 1.0 / np.linalg.inv(kA)[0, 0]  # 0.8
    assert lower - 1e-9 <= adi < per - 1e-3


def test_periodic_at_least_adiabatic_random():
    m = w.random_medium(42, 6, 6, 2, nphase=3, lo=0.2, hi=2.0)
    per = make(m, grad=0).solve(1e-14, TOL_MAXDT, 1_000_000)["keff_vol"]
    adi = make(m, grad=0, sides=(0, ADIABATIC, PERIODIC)).solve(1e-14, TOL_MAXDT, 1_000_000)["keff_vol"]
    assert per >= adi - 1e-10


def test_mirror_symmetric_periodic_equals_adiabatic():
    rng = np.random.default_rng(43)
    half = rng.integers(0, 3, size=(2, 3, 7), dtype=np.uint8)
    phase = np.concatenate([half, half[:, ::-1, :]], axis=1)  # symmetric in y
    tensors = []
    for _ in range(3):
        t = w.random_spd(rng, 0.2, 1.5)
        t[0, 1] = t[1, 0] = t[1, 2] = t[2, 1] = 0.0  # mirror-invariant in y
        t += 0.5 * np.eye(3)
        tensors.append(t)
    m = w.Medium(np.ascontiguousarray(phase), np.stack([w.sym6(t) for t in tensors]))
    a = make(m, grad=0)
    b = make(m, grad=0, sides=(0, ADIABATIC, PERIODIC))
    a.step(300)
    b.step(300)
    assert np.allclose(a.temperature(), b.temperature(), rtol=0, atol=1e-12)
    assert math.isclose(a.keff()["keff_vol"], b.keff()["keff_vol"], rel_tol=1e-11)


def test_axis_permutation_equivariance():
    m = w.random_medium(44, 5, 4, 3, nphase=3)
    a = make(m, grad=0, sides=(0, ADIABATIC, PERIODIC))
    mp = m.permuted((1, 0, 2))  # swap x and y
    b = make(mp, grad=1, sides=(ADIABATIC, 0, PERIODIC))
    a.step(150)
    b.step(150)
    Ta = a.temperature()
    Tb = b.temperature()
    assert np.allclose(Tb, Ta.transpose(0, 2, 1), rtol=0, atol=1e-12)
    ka, kb = a.keff(), b.keff()
    assert math.isclose(ka["keff_hot"], kb["keff_hot"], rel_tol=1e-11)
    assert np.allclose(ka["keff_col"][[1, 0, 2]], kb["keff_col"], rtol=1e-10, atol=1e-13)


def test_reflection_equivariance():
    m = w.random_medium(45, 4, 5, 3, nphase=2)
    R = np.diag([1.0, -1.0, 1.0])
    mr = w.Medium(np.ascontiguousarray(m.phase[:, ::-1, :]),
                  np.stack([w.sym6(R @ w.full3(r) @ R) for r in m.k]))
    a = make(m, grad=0, sides=(0, ADIABATIC, PERIODIC))
    b = make(mr, grad=0, sides=(0, ADIABATIC, PERIODIC))
    a.step(120)
    b.step(120)
    assert np.allclose(b.temperature(), a.temperature()[:, ::-1, :], rtol=0, atol=1e-12)


def test_keff_tensor_symmetric_for_homogeneous_medium():
    rng = np.random.default_rng(46)
    k = w.random_spd(rng, 0.4, 1.2)
    m = w.Medium(np.zeros((2, 6, 6), np.uint8), w.sym6(k)[None, :])
    rx = make(m, grad=0).solve(1e-15, TOL_MAXDT, 1_000_000)
    ry = make(m, grad=1).solve(1e-15, TOL_MAXDT, 1_000_000)
    assert math.isclose(rx["keff_col"][1], ry["keff_col"][0], rel_tol=1e-8)
    assert math.isclose(rx["keff_col"][1], k[0, 1], rel_tol=1e-8)


def test_steady_state_plane_flux_is_constant():
    m = w.random_medium(47, 6, 4, 3, nphase=3, lo=0.3, hi=1.5)
    o = make(m, grad=0, sides=(0, ADIABATIC, PERIODIC))
    r = o.solve(1e-15, TOL_MAXDT, 1_000_000)
    f = o.get_f()
    fh = _post_collision(o, m, f)
    # link flux across the plane between x and x + 1
    planes = [(fh[1][:, :, x] - fh[2][:, :, x + 1]).sum() for x in range(m.nx - 1)]
    lf = o.last_fluxes()
    assert np.allclose(planes, lf["phi_hot"], rtol=1e-9)
    assert math.isclose(lf["phi_hot"], lf["phi_cold"], rel_tol=1e-9)
    assert math.isclose(r["keff_vol"], r["keff_hot"], rel_tol=1e-9)


def test_interface_normal_flux_continuity():
    # Sec. 3.3 checks that the normal flux across the interface is
    # continuous; in a laminate the node flux (Eq. 16) is the same on both
    # sides of every interface
    m = w.dual_component_cube(6)
    m = w.Medium(np.ascontiguousarray(m.phase[:, :1, :1]), m.k)  # 1 x 1 x 6 column
    o = make(m, grad=2)
    o.solve(1e-15, TOL_MAXDT, 1_000_000)
    q, _ = o.flux()
    qz = q[2].reshape(-1)
    assert np.allclose(qz, qz.mean(), rtol=1e-9)


def test_sec33_dual_component_cube():
    g = golden("sec33_dual_component.json")
    m = w.dual_component_cube(g["n"])
    lmax = max(np.linalg.eigvalsh(w.full3(r)).max() for r in m.k)
    dmax = g["lattice_tau_minus_half_over_lambda"] * lmax
    kz1, kz2 = m.k[0][2], m.k[1][2]
    series = 2 * kz1 * kz2 / (kz1 + kz2)
    # periodic sides: exact series mean (10.909)
    mp = w.Medium(np.ascontiguousarray(m.phase[:, :1, :1]), m.k)
    rp = make(mp, grad=2, dmax=dmax).solve(1e-15, TOL_MAXDT, 1_000_000)
    assert math.isclose(rp["keff_vol"], series, rel_tol=1e-9)
    # adiabatic sides: the paper's configuration, 10.40 by its LBM, 10.34 by FEM
    o = make(m, grad=2, dmax=dmax, sides=(ADIABATIC, ADIABATIC, 0))
    r = o.solve(1e-6, TOL_KEFF, 400000, check_every=100)
    assert r["converged"]
    assert abs(r["keff_mid"] - g["k_lbm"]) / g["k_lbm"] < 0.012
    assert abs(r["keff_mid"] - g["k_fluent"]) / g["k_fluent"] < 0.005
    assert r["keff_mid"] < series


# ---------------------------------------------------------------------------
# failure handling
# ---------------------------------------------------------------------------


def test_rejects_bad_media():
    m = w.random_medium(51, 2, 2, 2, nphase=2)
    bad = m.k.copy()
    bad[1] = [1.0, 1.0, 1.0, 2.0, 0.0, 0.0]  # not positive definite
    with pytest.raises(ValueError):
        Oracle(m.phase, bad)
    ph = m.phase.copy()
    ph[0, 0, 0] = 7
    with pytest.raises(ValueError):
        Oracle(ph, m.k)


def test_nonfinite_state_is_reported():
    m = w.random_medium(52, 3, 3, 3, nphase=2)
    o = make(m)
    f = o.get_f()
    f[3, 1, 1, 1] = np.nan
    o.set_f(f)
    with pytest.raises(FloatingPointError):
        o.solve(1e-12, TOL_MAXDT, 100)


# ---------------------------------------------------------------------------
# relaxation times tau_4..6 (Eq. 12) act on their own moments of Eq. 11
# ---------------------------------------------------------------------------

# rows of Eq. 11 that tau_4, tau_5, tau_6 relax, and their equilibria per
# unit temperature (6 f_0 - sum f_i at f_eq = 6 T/4 - 6 T/8 = 3 T/4; the
# other two vanish at equilibrium)
HIGHER_ROWS = {4: ([6, -1, -1, -1, -1, -1, -1], 0.75), 5: ([0, 2, 2, -1, -1, -1, -1], 0.0),
               6: ([0, 0, 0, 1, 1, -1, -1], 0.0)}


@pytest.mark.parametrize("tau_rest", [(0.8, 0.7, 1.6, 1.2), (1.0, 1.9, 0.6, 1.0)])
def test_each_relaxation_time_acts_on_its_own_moment(tau_rest):
    """With S block diagonal in the moment basis (Eq. 12), a state that is
    off equilibrium only in moment k of Eq. 11 keeps that direction, and one
    collision scales the deviation by 1 - 1/tau_k, the other moments
    untouched.  tau_4, tau_5, tau_6 differ, so assigning any of them to the
    wrong row fails."""
    m = w.random_medium(15, 2, 2, 2, nphase=2)
    o = make(m, tau_rest=np.array(tau_rest, float))
    taus = {4: tau_rest[1], 5: tau_rest[2], 6: tau_rest[3]}
    rng = np.random.default_rng(7)
    for p in range(2):
        for k, (row, _) in HIGHER_ROWS.items():
            phi = np.array(row, float)
            T = rng.uniform(-1, 1)
            feq = np.array([T / 4] + [T / 8] * 6)
            d = 0.37 * phi / (phi @ phi)  # moment k of d is 0.37, every other moment 0
            out = o.collide_node(p, feq + d)
            assert np.allclose(out, feq + (1.0 - 1.0 / taus[k]) * d, rtol=0, atol=1e-15), (p, k)
        # and the equilibria: moment k of f_eq(T) is its row's value
        for k, (row, per_t) in HIGHER_ROWS.items():
            assert math.isclose(np.dot(row, [0.25] + [0.125] * 6), per_t, abs_tol=1e-15)


@pytest.mark.parametrize("sides", [(0, ADIABATIC, PERIODIC), (0, PERIODIC, ADIABATIC)])
def test_dense_fixed_point_general_relaxation(sides):
    """Fixed point with tau_0, tau_4..6 other than 1: the iterated oracle
    against numpy.linalg.solve of (I - L) f* = b."""
    tau_rest = (0.9, 0.7, 1.6, 1.2)
    m = w.random_medium(48, 3, 3, 2, nphase=2, lo=0.3, hi=1.5)
    fstar, s = mf.fixed_point(m.phase, m.k, 1.0, 0, 1.0, 0.0, sides, tau_rest)
    o = make(m, grad=0, sides=sides, tau_rest=np.array(tau_rest, float))
    o.solve(1e-16, TOL_MAXDT, 400000)
    assert np.allclose(o.get_f(), fstar, rtol=0, atol=1e-12)
    # a different tau_4..6 gives a different pre-collision fixed point (the
    # higher moments are not at equilibrium near walls and interfaces)
    f1, _ = mf.fixed_point(m.phase, m.k, 1.0, 0, 1.0, 0.0, sides)
    assert np.abs(f1 - fstar).max() > 1e-6


# ---------------------------------------------------------------------------
# start with a flux part: j = -eps tau grad T0 (Eq. 15 read backwards)
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("grad", [0, 1, 2])
def test_flux_start_of_the_linear_solution_is_steady(grad):
    """A homogeneous anisotropic cell with periodic sides has the steady
    field T_lin along the gradient axis with the constant flux j = -eps tau
    grad T (Eq. 15).  Starting from T_lin with that flux part is the steady
    state itself: a step changes nothing.  The equilibrium start from the
    same field is not steady."""
    rng = np.random.default_rng(61 + grad)
    K = w.random_spd(rng, 0.3, 1.5)
    shape = [3, 4, 5]  # (nz, ny, nx)
    shape[2 - grad] = 7
    m = w.Medium(np.zeros(shape, np.uint8), w.sym6(K)[None, :])
    n = shape[2 - grad]
    view = [1, 1, 1]
    view[2 - grad] = n
    tlin = np.broadcast_to((0.9 - 1.3 * (np.arange(n) + 0.5) / n).reshape(view), shape).copy()
    o = Oracle(m.phase, m.k, dmax=0.8)
    o.set_bc(grad, 0.9, -0.4)
    o.init(tlin, flux=True)
    f0 = o.get_f()
    o.step(1)
    assert np.allclose(o.get_f(), f0, rtol=0, atol=1e-15)
    assert o.last_fluxes()["resid"] < 1e-15
    r = o.keff()
    assert np.allclose(r["keff_col"], K[:, grad], rtol=1e-12, atol=1e-14)
    o.init(tlin)
    fe = o.get_f()
    o.step(1)
    assert np.abs(o.get_f() - fe).max() > 1e-3


@pytest.mark.parametrize("tau_rest", [(1, 1, 1, 1), (1, 0.7, 1.6, 1.2)])
def test_flux_start_with_neumann_faces_is_steady(tau_rest):
    """The side-flux case above (T_lin exact under the linear solution's own
    side fluxes): the flux start from T_lin is already that steady state; the
    mirror rule at the Neumann faces sees a field that is uniform across
    them."""
    rng = np.random.default_rng(33)
    K = w.random_spd(rng, 0.3, 1.5)
    K[0, 2] = K[2, 0] = 0.3
    K[1, 2] = K[2, 1] = -0.25
    nx, ny, nz = 5, 4, 9
    m = w.Medium(np.zeros((nz, ny, nx), np.uint8), w.sym6(K)[None, :])
    o = make(m, grad=2, sides=(ADIABATIC, ADIABATIC, 0), tau_rest=np.array(tau_rest, float))
    qx, qy = K[0, 2] / nz, K[1, 2] / nz
    o.set_side_flux(0, qx, -qx)
    o.set_side_flux(1, qy, -qy)
    tlin = np.broadcast_to((1.0 - (np.arange(nz) + 0.5) / nz)[:, None, None], (nz, ny, nx)).copy()
    o.init(tlin, flux=True)
    f0 = o.get_f()
    o.step(3)
    assert np.allclose(o.get_f(), f0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("sides", [(0, PERIODIC, ADIABATIC), (ADIABATIC, 0, PERIODIC), (PERIODIC, ADIABATIC, 0)])
def test_flux_start_gradient_matches_numpy(sides):
    """Eq. 15 applied to the flux start returns grad T0 by central
    differences: at every node off the isothermal walls it equals
    numpy.gradient of T0 padded by wrapping (periodic axis) or by mirroring
    the edge node (adiabatic face)."""
    grad_axis = [a for a in range(3) if sides[a] == 0 and a not in
                 [b for b in range(3) if sides[b] == ADIABATIC]][0]
    m = w.random_medium(62, 6, 5, 4, nphase=3)
    rng = np.random.default_rng(9)
    T0 = rng.uniform(-1, 1, m.phase.shape)
    side_arg = [PERIODIC if (a == grad_axis) else sides[a] for a in range(3)]
    o = Oracle(m.phase, m.k)
    o.set_bc(grad_axis, 1.0, 0.0, side_arg)
    o.init(T0, flux=True)
    _, g = o.flux()
    assert np.allclose(o.temperature(), T0, rtol=0, atol=1e-15)
    for a in range(3):
        ax = 2 - a  # array axis of lattice axis a
        if a == grad_axis:
            pad = np.pad(T0, [(1, 1) if d == ax else (0, 0) for d in range(3)], mode="edge")  # unused at walls
        else:
            mode = "wrap" if side_arg[a] == PERIODIC else "symmetric"
            pad = np.pad(T0, [(1, 1) if d == ax else (0, 0) for d in range(3)], mode=mode)
        ref = np.gradient(pad, axis=ax)
        ref = np.take(ref, range(1, T0.shape[ax] + 1), axis=ax)
        got = g[a]
        if a == grad_axis:  # interior nodes only; the wall nodes are pinned by the linear-solution tests
            sl = [slice(None)] * 3
            sl[ax] = slice(1, -1)
            ref, got = ref[tuple(sl)], got[tuple(sl)]
        assert np.allclose(got, ref, rtol=0, atol=1e-12), a


def test_flux_start_translation_equivariance():
    """Shifting the medium and the start field along the periodic axes
    shifts the flux start with them (the wrap of Eq. 25)."""
    m = w.random_medium(63, 5, 6, 4, nphase=3)
    rng = np.random.default_rng(10)
    T0 = rng.uniform(-1, 1, m.phase.shape)
    a = Oracle(m.phase, m.k)
    a.set_bc(0, 1.0, 0.0)
    a.init(T0, flux=True)
    sh = (1, -2)  # (z, y)
    ms = w.Medium(np.ascontiguousarray(np.roll(m.phase, sh, axis=(0, 1))), m.k)
    b = Oracle(ms.phase, ms.k)
    b.set_bc(0, 1.0, 0.0)
    b.init(np.roll(T0, sh, axis=(0, 1)), flux=True)
    assert np.allclose(b.get_f(), np.roll(a.get_f(), sh, axis=(1, 2)), rtol=0, atol=1e-15)
