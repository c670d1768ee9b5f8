"""Voxel media: phase grids plus per-phase conductivity tensors.

Conventions shared by every generator here:

* ``phase`` is a C-contiguous ``uint8`` array of shape ``(nz, ny, nx)``; the
  voxel with indices ``(k, j, i)`` has its centre at ``(i + 1/2, j + 1/2,
  k + 1/2)`` in voxel units.  Each node of the lattice is one voxel and is
  wholly one phase (the "half lattice division": interfaces and outer walls
  sit on voxel faces, half-way between nodes -- paper Sec. 2.3).
* ``k`` is a float64 array of shape ``(nphase, 6)`` with rows
  ``(kxx, kyy, kzz, kxy, kxz, kyz)`` of a symmetric positive-definite tensor in
  physical units.
"""

from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

# ---------------------------------------------------------------------------
# tensor helpers
# ---------------------------------------------------------------------------


def sym6(t) -> np.ndarray:
    """Pack a symmetric 3x3 tensor as (xx, yy, zz, xy, xz, yz)."""
    t = np.asarray(t, dtype=np.float64)
    return np.array([t[0, 0], t[1, 1], t[2, 2], t[0, 1], t[0, 2], t[1, 2]])


def full3(k6) -> np.ndarray:
    """Unpack (xx, yy, zz, xy, xz, yz) into a symmetric 3x3 tensor."""
    xx, yy, zz, xy, xz, yz = (float(v) for v in k6)
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def rot_z(deg: float) -> np.ndarray:
    """Active rotation by ``deg`` degrees about +z."""
    a = math.radians(deg)
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rot_y(deg: float) -> np.ndarray:
    a = math.radians(deg)
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def rot_x(deg: float) -> np.ndarray:
    a = math.radians(deg)
    c, s = math.cos(a), math.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def rotate_tensor(diag, R) -> np.ndarray:
    """Principal values ``diag`` carried into Cartesian axes: R diag(d) R^T."""
    R = np.asarray(R, dtype=np.float64)
    return R @ np.diag(np.asarray(diag, dtype=np.float64)) @ R.T


def slab_tensor_eq26(l_eta: float, l_zeta: float, beta_deg: float, l_z: float | None = None) -> np.ndarray:
    """In-plane tensor of a slab whose principal axes are tilted by beta
    (paper Sec. 3.1, Eq. 26), embedded in 3-D with an uncoupled z entry.

    Eq. 26 multiplies diag(l_eta, l_zeta) on the left by [[c, s], [-s, c]] and
    on the right by its transpose, which gives
    l_xx = c^2 l_eta + s^2 l_zeta,  l_yy = s^2 l_eta + c^2 l_zeta,
    l_xy = c s (l_zeta - l_eta).
    """
    b = math.radians(beta_deg)
    c, s = math.cos(b), math.sin(b)
    P = np.array([[c, s], [-s, c]])
    lam2 = P @ np.diag([l_eta, l_zeta]) @ P.T
    t = np.zeros((3, 3))
    t[:2, :2] = lam2
    t[2, 2] = l_zeta if l_z is None else l_z
    return t


def transversely_isotropic(k_axial: float, k_trans: float, u) -> np.ndarray:
    """k_T I + (k_A - k_T) u u^T for a unit fibre/yarn axis u."""
    u = np.asarray(u, dtype=np.float64)
    u = u / np.linalg.norm(u)
    return k_trans * np.eye(3) + (k_axial - k_trans) * np.outer(u, u)


def random_spd(rng: np.random.Generator, lo: float = 0.1, hi: float = 2.0) -> np.ndarray:
    """Random SPD tensor: a random orthogonal frame times eigenvalues in [lo, hi]."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    return rotate_tensor(rng.uniform(lo, hi, 3), q)


# ---------------------------------------------------------------------------
# the medium record
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Medium:
    phase: np.ndarray  # uint8 (nz, ny, nx)
    k: np.ndarray  # float64 (nphase, 6)
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def shape(self):
        return self.phase.shape

    @property
    def nx(self):
        return self.phase.shape[2]

    @property
    def ny(self):
        return self.phase.shape[1]

    @property
    def nz(self):
        return self.phase.shape[0]

    @property
    def nphase(self):
        return self.k.shape[0]

    def permuted(self, order) -> "Medium":
        """Relabel the Cartesian axes.  ``order`` lists, for new axes
        (x', y', z'), which old axis (0=x, 1=y, 2=z) each one is.  The phase
        grid is transposed and every tensor is conjugated by the permutation."""
        order = tuple(order)
        P = np.zeros((3, 3))
        for new, old in enumerate(order):
            P[new, old] = 1.0
        # array axes are (z, y, x): array axis of Cartesian axis a is 2 - a
        arr_axes = tuple(2 - order[2 - ax] for ax in range(3))
        phase = np.ascontiguousarray(np.transpose(self.phase, arr_axes))
        k = np.stack([sym6(P @ full3(r) @ P.T) for r in self.k])
        return Medium(phase, k, self.name + f"[perm{order}]", dict(self.meta))


def _finish(phase, tensors, name, **meta) -> Medium:
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    k = np.stack([sym6(t) for t in tensors]).astype(np.float64)
    return Medium(phase, k, name, meta)


# ---------------------------------------------------------------------------
# laminates and the paper's validation media
# ---------------------------------------------------------------------------


def layered(shape, axis: int, thicknesses, tensors, name: str = "layered") -> Medium:
    """Layers stacked along Cartesian ``axis`` (0=x, 1=y, 2=z).  Layer ``i``
    has ``thicknesses[i]`` voxels and phase id ``i``.  ``shape`` is (nx, ny, nz)."""
    nx, ny, nz = shape
    n_along = (nx, ny, nz)[axis]
    if sum(thicknesses) != n_along:
        raise ValueError("layer thicknesses must add up to the grid extent")
    ids = np.concatenate([np.full(t, i, dtype=np.uint8) for i, t in enumerate(thicknesses)])
    phase = np.empty((nz, ny, nx), dtype=np.uint8)
    if axis == 0:
        phase[:] = ids[None, None, :]
    elif axis == 1:
        phase[:] = ids[None, :, None]
    else:
        phase[:] = ids[:, None, None]
    return _finish(phase, tensors, name, axis=axis, thicknesses=list(thicknesses))


def c1_layered(n: int = 16) -> Medium:
    """Two-phase laminate: layers of n/2 voxels normal to x.  Layer A is
    diag(1, 0.5, 0.5) rotated 30 degrees about z; layer B is isotropic 0.2."""
    kA = rotate_tensor([1.0, 0.5, 0.5], rot_z(30.0))
    kB = 0.2 * np.eye(3)
    return layered((n, n, n), 0, [n // 2, n - n // 2], [kA, kB], name=f"c1_layered_{n}")


def table1_slabs(ratio: float, beta_deg: float, n_per_slab: int = 10, nx: int = 2) -> Medium:
    """Paper Sec. 3.1 / Table I: two equally thick slabs in series along y
    (gradient along y), each with l_eta = 2 l_zeta and principal axes tilted
    by beta (Eq. 26); slab 1 has l_eta = 2, slab 2 has l_eta = 2 * ratio.
    The grid is (nx, 2 n_per_slab, 1); the slabs are infinite in x and z."""
    t1 = slab_tensor_eq26(2.0, 1.0, beta_deg)
    t2 = slab_tensor_eq26(2.0 * ratio, 1.0 * ratio, beta_deg)
    return layered((nx, 2 * n_per_slab, 1), 1, [n_per_slab, n_per_slab], [t1, t2],
                   name=f"table1_{ratio}_{beta_deg}")


def dual_component_cube(n: int = 30) -> Medium:
    """Paper Sec. 3.3: two layers (n/2 voxels each) stacked along z with the
    tensors of Eq. 31."""
    l1 = np.array([[4.0, 1.0, 2.0], [1.0, 8.0, 1.0], [2.0, 1.0, 10.0]])
    l2 = np.array([[10.0, 1.0, 4.0], [1.0, 8.0, 1.0], [4.0, 1.0, 12.0]])
    return layered((n, n, n), 2, [n // 2, n - n // 2], [l1, l2], name=f"dual_component_{n}")


def random_medium(seed: int, nx: int, ny: int, nz: int, nphase: int = 3,
                  lo: float = 0.1, hi: float = 2.0) -> Medium:
    """Random phase ids (uniform) with random SPD tensors -- parity fodder."""
    rng = np.random.default_rng(seed)
    phase = rng.integers(0, nphase, size=(nz, ny, nx), dtype=np.uint8)
    tensors = [random_spd(rng, lo, hi) for _ in range(nphase)]
    return _finish(phase, tensors, f"random_{seed}_{nx}x{ny}x{nz}")


# ---------------------------------------------------------------------------
# synthetic four-directional braid
# ---------------------------------------------------------------------------

_FAMILY_SIGNS = ((1, 1), (-1, 1), (1, -1), (-1, -1))


def braid_family_axes(gamma_deg: float) -> np.ndarray:
    """Unit axes of the four yarn families: tilted by the interior braiding
    angle gamma from z inside the two diagonal planes x = +-y."""
    g = math.radians(gamma_deg)
    sg, cg = math.sin(g), math.cos(g)
    return np.array([[sx * sg / math.sqrt(2.0), sy * sg / math.sqrt(2.0), cg] for sx, sy in _FAMILY_SIGNS])


def _braid_radius(nx, ny, nz, gamma_deg, z_chunk=None, workers=None):
    """Per voxel: the smallest normalised elliptical radius over all yarn
    centrelines (and their periodic images), and the family of that line.
    Slabs of z-planes are evaluated on a thread pool (NumPy releases the GIL
    in its array loops); every voxel's arithmetic is the same whatever the
    slab size or thread count, so the result is too."""
    g = math.radians(gamma_deg)
    aspect = math.sqrt(3.0) * math.cos(g)  # c/d of the paper's cross-section (Eq. 33)
    axes = braid_family_axes(gamma_deg)
    lines = []
    for fam in range(4):
        u = axes[fam]
        nvec = np.cross([0.0, 0.0, 1.0], u)
        nvec /= np.linalg.norm(nvec)
        mvec = np.cross(u, nvec)
        for l in range(2):
            anchor = np.array([(l / 2 + fam / 8 + 0.25) * nx, (l / 2 + 0.25) * ny, nz / 2.0])
            lines.append((fam, mvec, nvec, anchor))
    shifts = np.array([[sx * nx, sy * ny, sz * nz] for sx in (-1, 0, 1) for sy in (-1, 0, 1) for sz in (-1, 0, 1)],
                      dtype=np.float64)
    xs = np.arange(nx) + 0.5
    ys = np.arange(ny) + 0.5
    best = np.full((nz, ny, nx), np.inf, dtype=np.float64)
    fam_of = np.zeros((nz, ny, nx), dtype=np.uint8)
    if z_chunk is None:
        z_chunk = max(1, (1 << 18) // (nx * ny))

    def slab(z0):
        z1 = min(nz, z0 + z_chunk)
        zs = np.arange(z0, z1) + 0.5
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        cb = best[z0:z1]
        cf = fam_of[z0:z1]
        for fam, m, nv, anc in lines:
            a_base = (X - anc[0]) * m[0] + (Y - anc[1]) * m[1] + (Z - anc[2]) * m[2]
            b_base = (X - anc[0]) * nv[0] + (Y - anc[1]) * nv[1] + (Z - anc[2]) * nv[2]
            rho2 = np.full(a_base.shape, np.inf)
            for s in shifts:
                a = (a_base + s @ m) / aspect
                b = b_base + s @ nv
                np.minimum(rho2, a * a + b * b, out=rho2)
            upd = rho2 < cb
            cb[upd] = rho2[upd]
            cf[upd] = fam + 1

    starts = list(range(0, nz, z_chunk))
    if workers is None:
        workers = min(16, os.cpu_count() or 1, len(starts))
    if workers <= 1:
        for z0 in starts:
            slab(z0)
    else:
        from concurrent.futures import ThreadPoolExecutor

        with ThreadPoolExecutor(max_workers=workers) as pool:
            list(pool.map(slab, starts))
    return np.sqrt(best), fam_of


def braid(nx: int, ny: int, nz: int, gamma_deg: float = 30.0, v: float = 0.5,
          k_axial: float = 10.0, k_trans: float = 1.0, k_matrix: float = 0.2, workers: int | None = None) -> Medium:
    """Synthetic four-directional braided unit cell (a stand-in for the
    paper's unit cell, whose yarn coordinates are not given in the paper).

    * phase 0 is the isotropic matrix; phases 1..4 are the yarn families with
      in-plane signs (+,+), (-,+), (+,-), (-,-); family axis
      u = (sx sin g / sqrt2, sy sin g / sqrt2, cos g).
    * yarn tensors are transversely isotropic, k_T I + (k_A - k_T) u u^T.
    * two straight centrelines per family run through the mid-plane z = nz/2
      at x = (l/2 + f/8 + 1/4) nx, y = (l/2 + 1/4) ny (line l = 0, 1; family
      f = 0..3), with periodic images in every direction.
    * cross-sections are ellipses, semi-major axis in the braiding plane (the
      plane of u and z) and semi-minor axis normal to it, with the paper's
      aspect c/d = sqrt(3) cos g (Eq. 33); one common scale is chosen so that
      the yarn voxel fraction equals v to within one voxel.
    * a voxel covered by several yarns takes the nearest one (smallest
      normalised radius), ties going to the lower phase id.

    Deterministic: no random numbers are drawn; ``workers`` (threads for the
    voxelisation, default up to 16) does not change the result.
    """
    rad, fam = _braid_radius(nx, ny, nz, gamma_deg, workers=workers)
    n = rad.size
    target = int(round(v * n))
    phase = np.zeros((nz, ny, nx), dtype=np.uint8)
    if target > 0:
        flat = rad.ravel()
        sigma = np.partition(flat, target - 1)[target - 1]
        sel = rad <= sigma
        phase[sel] = fam[sel]
    axes = braid_family_axes(gamma_deg)
    tensors = [k_matrix * np.eye(3)] + [transversely_isotropic(k_axial, k_trans, axes[f]) for f in range(4)]
    return _finish(phase, tensors, f"braid_{nx}x{ny}x{nz}_g{gamma_deg:g}_v{v:g}",
                   gamma=gamma_deg, v=v, yarn_fraction=float((phase > 0).mean()))


def sweep_cells(seed: int = 1503, n: int = 64, sizes=(64, 96, 128)):
    """Parametric sweep of braided cells: per cell, each axis extent drawn
    uniformly from ``sizes``, braiding angle ~ U[20, 45] deg, yarn volume
    fraction ~ U[0.35, 0.6].  Returns a list of dicts (no voxelisation)."""
    rng = np.random.default_rng(seed)
    dims = rng.choice(np.asarray(sizes), size=(n, 3))
    gam = rng.uniform(20.0, 45.0, n)
    vf = rng.uniform(0.35, 0.6, n)
    return [dict(nx=int(d[0]), ny=int(d[1]), nz=int(d[2]), gamma=float(g), v=float(v))
            for d, g, v in zip(dims, gam, vf)]


def warmstart_cells(seed: int, n: int, size: int):
    """Random cubic braided cells for the learned warm start's data: braiding
    angle ~ U[20, 45] deg and yarn fraction ~ U[0.35, 0.6]."""
    rng = np.random.default_rng(seed)
    gam = rng.uniform(20.0, 45.0, n)
    vf = rng.uniform(0.35, 0.6, n)
    return [dict(nx=size, ny=size, nz=size, gamma=float(g), v=float(v)) for g, v in zip(gam, vf)]


def warmstart_cells_mixed(seed: int, n: int, sizes=(32, 40, 48, 64)):
    """Braided cells of uneven extent for the learned warm start's data: each
    axis extent drawn uniformly from ``sizes`` (the grids that cells of the
    parametric sweep are coarsened to for inference), braiding angle ~
    U[20, 45] deg, yarn fraction ~ U[0.35, 0.6]."""
    rng = np.random.default_rng(seed)
    dims = rng.choice(np.asarray(sizes), size=(n, 3))
    gam = rng.uniform(20.0, 45.0, n)
    vf = rng.uniform(0.35, 0.6, n)
    return [dict(nx=int(d[0]), ny=int(d[1]), nz=int(d[2]), gamma=float(g), v=float(v))
            for d, g, v in zip(dims, gam, vf)]
