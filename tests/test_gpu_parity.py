"""GPU (HIP, gfx950) path vs the FP64 CPU oracle, through the C ABI.

Bar: FP64 fields within 1e-12 of the oracle relative to max |T| at identical
step counts; FP64 observables within 1e-10 relative (they are sums of
differences of O(1) numbers); FP32 within the tolerances stated per test.
"""

import numpy as np
import pytest

import workloads as w
from oracle import ADIABATIC, PERIODIC, TOL_KEFF, TOL_MAXDT, Oracle

pytestmark = pytest.mark.gpu

SIDE_NAMES = {PERIODIC: "periodic", ADIABATIC: "adiabatic"}


@pytest.fixture(scope="module")
def Medium():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    from paper_1503_08718_amd.solver import Medium

    return Medium


def pair(Medium, m, grad, sides, prec="f64", dmax=1.0, T0=None, launch=None, t_hot=1.0, t_cold=0.0):
    g = Medium(m.phase, m.k, precision=prec)
    g.set_bc(grad, t_hot, t_cold, [SIDE_NAMES[s] for s in sides])
    if dmax != 1.0:
        g.set_scale(dmax)
    if launch:
        g.set_launch(*launch)
    g.init(T0)
    o = Oracle(m.phase, m.k, dmax=dmax)
    o.set_bc(grad, t_hot, t_cold, sides)
    o.init(T0)
    return g, o


def field_err(g, o):
    tg = g.temperature().double().cpu().numpy()
    to = o.temperature()
    return float(np.abs(tg - to).max() / max(np.abs(to).max(), 1e-300))


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# ---------------------------------------------------------------------------


@pytest.mark.parametrize("steps", [1, 10, 1000])
def test_c1_field_fp64(Medium, steps):
    m = w.c1_layered(16)
    g, o = pair(Medium, m, 0, (0, PERIODIC, PERIODIC))
    g.step(steps)
    o.step(steps)
    assert field_err(g, o) < 1e-12


def test_c1_solve_series_mean(Medium):
    m = w.c1_layered(16)
    g, o = pair(Medium, m, 0, (0, PERIODIC, PERIODIC))
    r = g.solve(1e-10, "maxdt", 200000, check_every=2)
    assert r["converged"], r
    exact = 14.0 / 43.0
    for key in ("keff", "keff_hot", "keff_cold", "keff_vol"):
        assert rel(r[key], exact) < 1e-6, (key, r)
    # same step count on the oracle: identical field and observables
    o.step(r["steps"])
    assert field_err(g, o) < 1e-12
    ko = o.keff()
    assert rel(r["keff_hot"], ko["keff_hot"]) < 1e-10
    assert rel(r["keff_cold"], ko["keff_cold"]) < 1e-10
    assert rel(r["keff_vol"], ko["keff_vol"]) < 1e-10
    assert abs(r["resid"] - ko["resid"]) < 1e-14


CASES = [
    # (nx, ny, nz, nphase, grad, sides, seed)
    (12, 7, 5, 3, 0, (0, PERIODIC, ADIABATIC), 1),
    (10, 9, 6, 4, 1, (ADIABATIC, 0, PERIODIC), 2),
    (8, 6, 11, 3, 2, (PERIODIC, ADIABATIC, 0), 3),
    (13, 5, 4, 2, 0, (0, ADIABATIC, ADIABATIC), 4),  # odd nx: scalar path
    (6, 8, 7, 5, 2, (ADIABATIC, ADIABATIC, 0), 5),  # nx % 4 != 0
    (68, 3, 3, 3, 0, (0, PERIODIC, PERIODIC), 6),  # rows longer than a wave chunk
    (40, 4, 9, 3, 1, (PERIODIC, 0, ADIABATIC), 7),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:3])) + f"_g{c[4]}")
def test_random_media_fp64(Medium, case):
    nx, ny, nz, nph, grad, sides, seed = case
    m = w.random_medium(seed, nx, ny, nz, nph)
    rng = np.random.default_rng(seed)
    T0 = rng.uniform(-0.5, 1.5, m.phase.shape)
    g, o = pair(Medium, m, grad, sides, T0=T0, t_hot=0.8, t_cold=-0.4)
    for n in (1, 7, 60):
        g.step(n)
        o.step(n)
        assert field_err(g, o) < 1e-12, n
    # observables of the next transition: GPU probe at t vs oracle at t+1
    kg = g.keff()
    o.step(1)
    ko = o.keff()
    for key in ("keff_hot", "keff_cold", "keff_vol"):
        assert abs(kg[key] - ko[key]) < 1e-10 * max(1.0, abs(ko[key])), key
    assert np.allclose(kg["keff_col"], ko["keff_col"], rtol=1e-10, atol=1e-10)
    assert abs(kg["resid"] - ko["resid"]) < 1e-13


def test_flux_field_fp64(Medium):
    m = w.random_medium(8, 12, 6, 5, 3)
    rng = np.random.default_rng(8)
    T0 = rng.uniform(0, 1, m.phase.shape)
    g, o = pair(Medium, m, 0, (0, ADIABATIC, PERIODIC), T0=T0)
    g.step(25)
    o.step(26)
    qg = g.flux().cpu().numpy()
    qo, _ = o.flux()
    qo = qo / o.scale  # oracle flux is in lattice units
    assert np.abs(qg - qo).max() < 1e-11 * np.abs(qo).max()


@pytest.mark.parametrize("launch", [(1, 16, 4), (2, 8, 8), (2, 32, 2), (4, 8, 16), (4, 64, 1), (1, 64, 4),
                                    (4, 64, 4, 1), (4, 32, 8, 2), (2, 16, 16, 3), (4, 8, 8, 0, 1), (2, 16, 4, 3, 1)])
def test_launch_shapes_bitwise_identical(Medium, launch):
    # 64 rows: with by = 4 or 8 the number of row blocks is a multiple of 8, as the XCD remap needs
    m = w.random_medium(9, 32, 64, 6, 3)
    ref, _ = pair(Medium, m, 1, (ADIABATIC, 0, PERIODIC))
    ref.step(40)
    g, _ = pair(Medium, m, 1, (ADIABATIC, 0, PERIODIC), launch=launch)
    g.step(40)
    import torch

    assert torch.equal(ref.state_get(), g.state_get())
    # the FP64 observables are sums in a launch-shape-dependent order
    ka, kb = ref.keff(), g.keff()
    for key in ("keff_hot", "keff_cold", "keff_vol", "resid"):
        assert abs(ka[key] - kb[key]) <= 1e-13 * max(1.0, abs(ka[key])), key


def test_checkpoint_resume_bitwise(Medium):
    import torch

    m = w.braid(16, 16, 24, 30.0, 0.5)
    for prec in ("f32", "f64"):
        a = Medium(m.phase, m.k, precision=prec).set_bc(2).init()
        a.step(50)
        snap = a.state_get().clone()
        a.step(70)
        b = Medium(m.phase, m.k, precision=prec).set_bc(2)
        b.state_set(snap, steps=50)
        b.step(70)
        assert torch.equal(a.state_get(), b.state_get())
        assert a.info()["steps"] == b.info()["steps"] == 120


def test_determinism_of_solve(Medium):
    m = w.braid(24, 24, 24, 35.0, 0.45)
    out = []
    for _ in range(2):
        g = Medium(m.phase, m.k, precision="f32").set_bc(0).init()
        out.append(g.solve(1e-3, "keff", 40000, check_every=200))
    assert out[0] == out[1]


def test_warm_start_init_matches_oracle(Medium):
    m = w.random_medium(10, 9, 8, 7, 3)
    rng = np.random.default_rng(10)
    T0 = rng.uniform(0, 1, m.phase.shape)
    g, o = pair(Medium, m, 2, (PERIODIC, ADIABATIC, 0), T0=T0)
    assert field_err(g, o) < 1e-14
    g.step(33)
    o.step(33)
    assert field_err(g, o) < 1e-12


# every wall mix, both storages: the start with a flux part (Eq. 15 read
# backwards, grad T0 by central differences) against the oracle's own
FLUX_START_CASES = CASES + [(9, 8, 7, 3, 2, (PERIODIC, ADIABATIC, 0), 10), (5, 1, 3, 2, 1, (ADIABATIC, 0, PERIODIC), 11),
                            (2, 2, 2, 2, 0, (0, ADIABATIC, ADIABATIC), 12)]


@pytest.mark.parametrize("storage", ["populations", "moments"])
@pytest.mark.parametrize("case", FLUX_START_CASES, ids=lambda c: "x".join(map(str, c[:3])) + f"_g{c[4]}")
def test_flux_start_matches_oracle(Medium, case, storage):
    nx, ny, nz, nph, grad, sides, seed = case
    m = w.random_medium(70 + seed, nx, ny, nz, nph)
    rng = np.random.default_rng(70 + seed)
    T0 = rng.uniform(-0.5, 1.5, m.phase.shape)
    g = Medium(m.phase, m.k, precision="f64", storage=storage)
    g.set_bc(grad, 0.8, -0.4, [SIDE_NAMES[s] for s in sides]).init(T0, flux=True)
    o = Oracle(m.phase, m.k)
    o.set_bc(grad, 0.8, -0.4, sides)
    o.init(T0, flux=True)
    assert field_err(g, o) < 1e-14
    # the flux part matters: one step from the equilibrium start at the same
    # field lands elsewhere
    e = Oracle(m.phase, m.k)
    e.set_bc(grad, 0.8, -0.4, sides)
    e.init(T0)
    e.step(1)
    for n in (1, 9, 50):
        g.step(n)
        o.step(n)
        assert field_err(g, o) < 1e-12, n
        if n == 1:
            assert field_err(g, e) > 1e-9
    kg = g.keff()
    o.step(1)
    ko = o.keff()
    for key in ("keff_hot", "keff_cold", "keff_vol"):
        assert abs(kg[key] - ko[key]) < 1e-10 * max(1.0, abs(ko[key])), key


def test_flux_start_fp32_matches_oracle(Medium):
    m = w.braid(24, 20, 16, 35.0, 0.5)
    rng = np.random.default_rng(75)
    T0 = 0.5 + 0.3 * rng.standard_normal(m.phase.shape) * 0.1
    for storage in ("populations", "moments"):
        g = Medium(m.phase, m.k, precision="f32", storage=storage)
        g.set_bc(2, 1.0, 0.0, ["periodic", "adiabatic", "periodic"]).init(T0, flux=True)
        o = Oracle(m.phase, m.k)
        o.set_bc(2, 1.0, 0.0, (PERIODIC, ADIABATIC, 0))
        o.init(T0, flux=True)
        g.step(40)
        o.step(40)
        assert field_err(g, o) < 2e-6, storage


def test_fp32_close_to_fp64(Medium):
    # FP32 at the production tolerance (wall-flux gap 1e-4) against an FP64
    # solve converged far tighter
    m = w.braid(32, 32, 32, 30.0, 0.5)
    g64 = Medium(m.phase, m.k, precision="f64").set_bc(0).init()
    r64 = g64.solve(1e-9, "keff", 2_000_000, check_every=500)
    assert r64["converged"], r64
    g32 = Medium(m.phase, m.k, precision="f32").set_bc(0).init()
    r32 = g32.solve(1e-4, "keff", 2_000_000, check_every=500)
    assert r32["converged"], r32
    assert rel(r32["keff"], r64["keff"]) < 1e-4


def test_fp32_converges_past_its_rounding_floor(Medium):
    # the plain wall-flux gap of an FP32 run stalls at a rounding floor that
    # grows like N_g^2; with the rounding energy accounted for exactly the
    # stop rule still closes, and k stays within 1e-5 of FP64
    m = w.braid(64, 64, 64, 30.0, 0.5)
    g64 = Medium(m.phase, m.k, precision="f64").set_bc(0).init()
    r64 = g64.solve(1e-9, "keff", 3_000_000, check_every=1000)
    g32 = Medium(m.phase, m.k, precision="f32").set_bc(0).init()
    r32 = g32.solve(1e-5, "keff", 3_000_000, check_every=1000)
    assert r64["converged"] and r32["converged"], (r64, r32)
    assert rel(r32["keff"], r64["keff"]) < 1e-5
    assert rel(r32["keff_vol"], r64["keff_vol"]) < 1e-5
    assert abs(r64["keff_leak"]) < 1e-10 * r64["keff"]


@pytest.mark.parametrize("storage", ["moments", "populations"])
def test_fp32_has_no_rounding_floor(Medium, storage):
    """Adiabatic sides, where round-to-nearest FP32 lost energy coherently
    (T/8 absorbed by jhat/2 in the populations) and stalled at a fixed point:
    with exact population rebuild (moments) or dithered populations, and a
    dithered T, the FP32 solve lands on the FP64 answer far inside the
    tolerance and its rounding energy is noise."""
    m = w.braid(64, 64, 64, 30.0, 0.5)
    sides = ("periodic", "adiabatic", "adiabatic")
    g64 = Medium(m.phase, m.k, precision="f64").set_bc(0, 1.0, 0.0, sides).init()
    r64 = g64.solve(1e-9, "keff", 4_000_000, check_every=1000)
    g32 = Medium(m.phase, m.k, precision="f32", storage=storage).set_bc(0, 1.0, 0.0, sides).init()
    r32 = g32.solve(1e-6, "keff", 4_000_000, check_every=1000)
    assert r64["converged"] and r32["converged"], (r64, r32)
    assert rel(r32["keff"], r64["keff"]) < 2e-6, (r32, r64)
    assert rel(r32["keff_vol"], r64["keff_vol"]) < 2e-6
    # one step's rounding energy: random, ~sqrt(N) dithered roundings
    # (round-to-nearest left a coherent 5e-5 here)
    assert abs(r32["keff_leak"]) < 1e-5 * r32["keff"]


# extents of 1 and 2: a node is its own periodic neighbour, or sits on both
# walls of an axis at once
DEGENERATE = [
    (1, 5, 4, 0, (0, PERIODIC, ADIABATIC)),
    (5, 1, 3, 1, (ADIABATIC, 0, PERIODIC)),
    (4, 3, 1, 2, (PERIODIC, ADIABATIC, 0)),
    (2, 2, 2, 0, (0, ADIABATIC, ADIABATIC)),
    (1, 1, 1, 0, (0, PERIODIC, PERIODIC)),
    (8, 1, 1, 0, (0, PERIODIC, ADIABATIC)),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("storage", ["populations", "moments"])
@pytest.mark.parametrize("case", DEGENERATE, ids=lambda c: "x".join(map(str, c[:3])) + f"_g{c[3]}")
def test_degenerate_extents(Medium, case, storage, prec):
    nx, ny, nz, grad, sides = case
    m = w.random_medium(11, nx, ny, nz, 2)
    T0 = np.random.default_rng(11).uniform(-0.5, 1.5, m.phase.shape)
    g = Medium(m.phase, m.k, precision=prec, storage=storage)
    g.set_bc(grad, 0.8, -0.4, [SIDE_NAMES[s] for s in sides]).init(T0)
    o = Oracle(m.phase, m.k)
    o.set_bc(grad, 0.8, -0.4, sides)
    o.init(T0)
    tol = 1e-12 if prec == "f64" else 1e-5
    for n in (1, 40):
        g.step(n)
        o.step(n)
        assert field_err(g, o) < tol, n
    kg = g.keff()
    o.step(1)
    ko = o.keff()
    for key in ("keff_hot", "keff_cold", "keff_vol"):
        assert abs(kg[key] - ko[key]) < (1e-10 if prec == "f64" else 2e-3) * max(1.0, abs(ko[key])), key


# ---------------------------------------------------------------------------
# full-size windows: the configurations the benchmark times
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("n,prec,tol", [(128, "f64", 1e-12), (128, "f32", 2e-6)])
def test_braid_window_full_size(Medium, n, prec, tol):
    m = w.braid(n, n, n, 30.0, 0.5)
    rng = np.random.default_rng(128)
    # smooth random start so that every node is active from the first step
    z, y, x = np.meshgrid(*(np.linspace(0, 2 * np.pi, n, endpoint=False),) * 3, indexing="ij")
    T0 = 0.5 + 0.3 * np.sin(x + rng.uniform(0, 6)) * np.cos(2 * y) + 0.1 * np.sin(3 * z)
    g, o = pair(Medium, m, 0, (0, PERIODIC, PERIODIC), prec=prec, T0=T0)
    o.set_threads(0)
    steps = 12
    g.step(steps)
    o.step(steps)
    assert field_err(g, o) < tol
    kg = g.keff()
    o.step(1)
    ko = o.keff()
    ktol = 1e-9 if prec == "f64" else 2e-3
    assert abs(kg["keff_vol"] - ko["keff_vol"]) < ktol * abs(ko["keff_vol"])


def test_energy_identity_full_size(Medium):
    # sum T(t+1) - sum T(t) = Phi_hot - Phi_cold (collision conserves T,
    # interior / periodic / adiabatic links conserve the sum)
    n = 128
    m = w.braid(n, n, n, 30.0, 0.5)
    g = Medium(m.phase, m.k, precision="f64").set_bc(2, sides=("periodic", "adiabatic", "periodic")).init()
    g.step(200)
    t0 = g.temperature().sum().item()
    k = g.keff()
    g.step(1)
    t1 = g.temperature().sum().item()
    info = g.info()
    area = n * n
    ng = n
    s = info["scale"]
    phi_hot = k["keff_hot"] * area * s / ng
    phi_cold = k["keff_cold"] * area * s / ng
    assert abs((t1 - t0) - (phi_hot - phi_cold)) < 1e-9 * max(1.0, abs(phi_hot))


# ---------------------------------------------------------------------------
# error paths
# ---------------------------------------------------------------------------


def test_rejects_bad_phase_and_tensor(Medium):
    from paper_1503_08718_amd import MrtlbmError

    m = w.random_medium(11, 4, 4, 4, 2)
    ph = m.phase.copy()
    ph[1, 2, 3] = 5
    with pytest.raises(MrtlbmError, match="E_ARG"):
        Medium(ph, m.k)
    bad = m.k.copy()
    bad[0] = [1, 1, 1, 2, 0, 0]
    with pytest.raises(MrtlbmError, match="E_TENSOR"):
        Medium(m.phase, bad)
    g = Medium(m.phase, m.k)
    with pytest.raises(MrtlbmError, match="E_BC"):
        g.set_bc(3)
    with pytest.raises(MrtlbmError, match="E_ARG"):
        g.step(1)  # not initialised


def test_nonfinite_start_is_reported(Medium):
    from paper_1503_08718_amd import MrtlbmError

    m = w.random_medium(12, 8, 8, 8, 2)
    T0 = np.zeros(m.phase.shape)
    T0[3, 3, 3] = np.nan
    g = Medium(m.phase, m.k, precision="f32").set_bc(0).init(T0)
    with pytest.raises(MrtlbmError, match="E_NONFINITE"):
        g.solve(1e-6, "keff", 1000, check_every=10)


def test_max_steps_gives_partial_result(Medium):
    m = w.braid(16, 16, 16, 30.0, 0.5)
    g = Medium(m.phase, m.k).set_bc(0).init()
    r = g.solve(1e-9, "keff", 300, check_every=100)
    assert r["status"] == "NOT_CONVERGED" and not r["converged"] and r["steps"] == 300
    assert r["keff_hot"] > r["keff_cold"]


# ---------------------------------------------------------------------------
# moment storage: 4 values per node, bit-identical evolution
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", CASES[:5] + [(32, 16, 12, 5, 2, (PERIODIC, ADIABATIC, 0), 9)],
                         ids=lambda c: "x".join(map(str, c[:3])) + f"_g{c[4]}")
def test_moment_storage_equals_populations(Medium, case, prec):
    """FP64: bit for bit.  FP32: the moment path keeps the populations exact
    and the population path must round them (dithered), so the two agree to
    the FP32 noise of the fields."""
    import torch

    nx, ny, nz, nph, grad, sides, seed = case
    m = w.random_medium(seed, nx, ny, nz, nph)
    rng = np.random.default_rng(seed)
    T0 = rng.uniform(-0.5, 1.5, m.phase.shape)
    runs = []
    for storage in ("populations", "moments"):
        g = Medium(m.phase, m.k, precision=prec)
        g.set_storage(storage)
        g.set_bc(grad, 0.8, -0.4, [SIDE_NAMES[s] for s in sides])
        g.init(T0, flux=True)
        g.step(37)
        runs.append((g.temperature(), g.flux(), g.keff(), g.solve(1e-30, "keff", 137, check_every=50)))
    (ta, qa, ka, ra), (tb, qb, kb, rb) = runs
    if prec == "f64":
        assert torch.equal(ta, tb)
        assert torch.equal(qa, qb)
        assert ka == kb and ra == rb
        return
    assert (ta - tb).abs().max().item() <= 1e-5 * max(1.0, ta.abs().max().item())
    assert (qa - qb).abs().max().item() <= 1e-5 * max(1e-3, qa.abs().max().item())
    for a, b in ((ka, kb), (ra, rb)):
        for key in ("keff_hot", "keff_cold", "keff_vol"):
            assert abs(a[key] - b[key]) <= 1e-4 * max(1.0, abs(b[key])), key


def test_moment_storage_matches_oracle_and_resumes(Medium):
    import torch

    m = w.c1_layered(16)
    g, o = pair(Medium, m, 0, (0, PERIODIC, PERIODIC))
    g.set_storage("moments")
    g.init()
    g.step(250)
    o.step(250)
    assert field_err(g, o) < 1e-12
    snap = g.state_get()
    assert snap.shape[0] == 4
    g.step(40)
    h = Medium(m.phase, m.k, precision="f64").set_storage("moments").set_bc(0)
    h.state_set(snap, steps=250)
    h.step(40)
    assert torch.equal(g.state_get(), h.state_get())


def test_moment_storage_batch(Medium):
    import torch

    from paper_1503_08718_amd.solver import batch_solve

    media = [w.braid(16, 16, 24, 25.0, 0.45), w.braid(24, 16, 16, 40.0, 0.55)]
    a = [Medium(mm.phase, mm.k, precision="f32").set_storage("moments").set_bc(ax).init()
         for mm, ax in zip(media, (2, 0))]
    b = [Medium(mm.phase, mm.k, precision="f32").set_bc(ax).init() for mm, ax in zip(media, (2, 0))]
    ra, _ = batch_solve(a, tol=1e-30, kind="keff", max_steps=400, check_every=100)
    rb, _ = batch_solve(b, tol=1e-30, kind="keff", max_steps=400, check_every=100)
    for x, y, p, q in zip(a, b, ra, rb):
        # FP32: exact populations (moments) vs dithered ones (populations)
        assert (x.temperature() - y.temperature()).abs().max().item() < 1e-5
        for key in ("keff_hot", "keff_cold", "keff_vol"):  # early transient: k_cold is still ~1e-3
            assert abs(p[key] - q[key]) <= 1e-4 * abs(q[key]) + 1e-6, key


# ---------------------------------------------------------------------------
# general tau_4..6 (Eq. 12) and Neumann faces with a given flux (Eq. 24)
# ---------------------------------------------------------------------------

TAU_REST = (0.7, 1.6, 1.2)


@pytest.mark.parametrize("case", [(12, 7, 5, 3, 0, (0, ADIABATIC, PERIODIC)), (9, 10, 8, 4, 2, (ADIABATIC, PERIODIC, 0)),
                                  (16, 6, 6, 2, 1, (PERIODIC, 0, ADIABATIC))],
                         ids=lambda c: "x".join(map(str, c[:3])) + f"_g{c[4]}")
def test_general_relaxation_matches_oracle(Medium, case):
    nx, ny, nz, nph, grad, sides = case
    m = w.random_medium(40 + nph, nx, ny, nz, nph)
    g = Medium(m.phase, m.k, precision="f64").set_bc(grad, 1.0, 0.0, [SIDE_NAMES[s] for s in sides])
    g.set_relaxation(*TAU_REST).init()
    o = Oracle(m.phase, m.k, tau_rest=np.array((1.0,) + TAU_REST))
    o.set_bc(grad, 1.0, 0.0, sides)
    o.init()
    g.step(400)
    o.step(400)
    assert field_err(g, o) < 1e-12
    # the GPU's observables belong to the step after the state it holds
    kg = g.keff()
    o.step(1)
    lf = o.last_fluxes()
    ng = (nx, ny, nz)[grad]
    area = nx * ny * nz / ng
    assert rel(kg["keff_hot"], ng * lf["phi_hot"] / (area * o.scale)) < 1e-10
    assert rel(kg["keff_cold"], ng * lf["phi_cold"] / (area * o.scale)) < 1e-10
    # and the relaxation does change the transient: tau_4..6 = 1 differs
    h = Medium(m.phase, m.k, precision="f64").set_bc(grad, 1.0, 0.0, [SIDE_NAMES[s] for s in sides]).init()
    h.step(400)
    assert field_err(h, o) > 1e-9


def test_fp32_general_relaxation_matches_oracle(Medium):
    """FP32 population storage with tau_4..6 other than 1: the seven outputs
    of the general relaxation are formed in FP64 and dithered like the
    others; a 300-step window stays on the oracle to FP32 noise."""
    m = w.random_medium(44, 16, 12, 10, 4)
    rng = np.random.default_rng(44)
    T0 = rng.uniform(0.0, 1.0, m.phase.shape)
    g = Medium(m.phase, m.k, precision="f32").set_bc(0, 1.0, 0.0, ["periodic", "adiabatic", "periodic"])
    g.set_relaxation(*TAU_REST).init(T0)
    o = Oracle(m.phase, m.k, tau_rest=np.array((1.0,) + TAU_REST))
    o.set_bc(0, 1.0, 0.0, (0, ADIABATIC, PERIODIC))
    o.init(T0)
    g.step(300)
    o.step(300)
    assert field_err(g, o) < 2e-6


def test_fp32_general_relaxation_close_to_fp64(Medium):
    """64^3 braided cell, adiabatic sides, tau_4..6 = (0.7, 1.6, 1.2): the
    FP32 solve lands within 2e-6 of the FP64 answer, with no rounding
    floor."""
    m = w.braid(64, 64, 64, 30.0, 0.5)
    sides = ("periodic", "adiabatic", "adiabatic")
    g64 = Medium(m.phase, m.k, precision="f64").set_bc(0, 1.0, 0.0, sides).set_relaxation(*TAU_REST).init()
    r64 = g64.solve(1e-9, "keff", 4_000_000, check_every=1000)
    g32 = Medium(m.phase, m.k, precision="f32").set_bc(0, 1.0, 0.0, sides).set_relaxation(*TAU_REST).init()
    r32 = g32.solve(1e-6, "keff", 4_000_000, check_every=1000)
    assert r64["converged"] and r32["converged"], (r64, r32)
    assert rel(r32["keff"], r64["keff"]) < 2e-6, (r32, r64)
    assert rel(r32["keff_vol"], r64["keff_vol"]) < 2e-6
    assert abs(r32["keff_leak"]) < 1e-5 * r32["keff"]


@pytest.mark.parametrize("storage", ["populations", "moments"])
def test_side_flux_matches_oracle(Medium, storage):
    m = w.random_medium(51, 11, 9, 7, 3)
    sides = (0, ADIABATIC, ADIABATIC)
    g = Medium(m.phase, m.k, precision="f64").set_storage(storage)
    g.set_bc(0, 0.8, -0.2, [SIDE_NAMES[s] for s in sides])
    g.set_side_flux(1, 0.04, -0.01).set_side_flux(2, -0.03, 0.05).init()
    o = Oracle(m.phase, m.k)
    o.set_bc(0, 0.8, -0.2, sides)
    o.set_side_flux(1, 0.04, -0.01)
    o.set_side_flux(2, -0.03, 0.05)
    o.init()
    g.step(500)
    o.step(500)
    assert field_err(g, o) < 1e-12
    r = g.keff()
    area = 9 * 7
    exp_side = 11 * ((0.04 - 0.01) * 11 * 7 + (-0.03 + 0.05) * 11 * 9) / (1.0 * area)
    assert rel(r["keff_side"], exp_side) < 1e-14


@pytest.mark.parametrize("prec,tau", [("f64", (1.0, 1.0, 1.0)), ("f64", TAU_REST), ("f32", (1.0, 1.0, 1.0))])
def test_side_flux_of_the_linear_solution_is_exact(Medium, prec, tau):
    """Homogeneous anisotropic cell, z gradient, x and y Neumann faces carrying
    the flux of the linear profile: T_lin(z) is the steady state and k = K_zz
    (any tau_4..6); zero side flux (adiabatic) gives less."""
    rng = np.random.default_rng(33)
    K = w.random_spd(rng, 0.3, 1.5)
    K[0, 2] = K[2, 0] = 0.3
    K[1, 2] = K[2, 1] = -0.25
    nx, ny, nz = 16, 12, 24
    m = w.Medium(np.zeros((nz, ny, nx), np.uint8), w.sym6(K)[None, :])
    qx, qy = K[0, 2] / nz, K[1, 2] / nz
    g = Medium(m.phase, m.k, precision=prec).set_bc(2, 1.0, 0.0, ["adiabatic", "adiabatic", "periodic"])
    g.set_relaxation(*tau).set_side_flux(0, qx, -qx).set_side_flux(1, qy, -qy).init()
    tol = 1e-9 if prec == "f64" else 1e-5
    r = g.solve(tol, "keff", 2_000_000, check_every=200)
    assert r["converged"], r
    assert abs(r["keff_side"]) < 1e-15
    assert rel(r["keff"], K[2, 2]) < 10 * tol
    tlin = 1.0 - (np.arange(nz) + 0.5) / nz
    assert np.abs(g.temperature().double().cpu().numpy() - tlin[:, None, None]).max() < (1e-7 if prec == "f64" else 1e-4)
    a = Medium(m.phase, m.k, precision=prec).set_bc(2, 1.0, 0.0, ["adiabatic", "adiabatic", "periodic"]).init()
    ra = a.solve(tol, "keff", 2_000_000, check_every=200)
    assert ra["keff"] < K[2, 2] * (1 - 1e-3)


def test_side_flux_and_relaxation_errors(Medium):
    from paper_1503_08718_amd import MrtlbmError
    from paper_1503_08718_amd.solver import batch_solve

    m = w.random_medium(52, 8, 8, 8, 2)
    g = Medium(m.phase, m.k, precision="f32").set_bc(0, 1.0, 0.0, ["periodic", "adiabatic", "periodic"])
    with pytest.raises(MrtlbmError, match="E_BC"):
        g.set_side_flux(0, 0.1, 0.1)  # gradient axis
    with pytest.raises(MrtlbmError, match="E_BC"):
        g.set_side_flux(2, 0.1, 0.1)  # periodic axis
    with pytest.raises(MrtlbmError, match="E_ARG"):
        g.set_relaxation(0.5, 1.0, 1.0)  # tau must exceed 1/2
    g.set_relaxation(1.2, 1.0, 1.0)
    with pytest.raises(MrtlbmError, match="E_ARG"):
        g.set_storage("moments")
    h = Medium(m.phase, m.k, precision="f32").set_storage("moments")
    with pytest.raises(MrtlbmError, match="E_ARG"):
        h.set_relaxation(1.2, 1.0, 1.0)
    g.init()
    with pytest.raises(MrtlbmError, match="E_ARG"):
        batch_solve([g], tol=1e-3, kind="keff", max_steps=100, check_every=10)
    # set_bc clears the side flux
    g.set_side_flux(1, 0.2, 0.0)
    g.set_bc(0, 1.0, 0.0, ["periodic", "adiabatic", "periodic"]).init()
    assert g.keff()["keff_side"] == 0.0


def test_moment_sized_workspace(Medium):
    import torch

    from paper_1503_08718_amd import MrtlbmError

    m = w.random_medium(61, 12, 8, 6, 3)
    big = Medium(m.phase, m.k, precision="f64").set_storage("moments").set_bc(0).init()
    small = Medium(m.phase, m.k, precision="f64", storage="moments").set_bc(0).init()
    assert small._ws.numel() < big._ws.numel()
    big.step(123)
    small.step(123)
    assert torch.equal(big.state_get(), small.state_get())
    with pytest.raises(MrtlbmError, match="E_WORKSPACE"):
        small.set_storage("populations")
