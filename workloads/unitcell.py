"""Geometry and yarn properties of the paper's braided unit cell.

Sec. 4.1 (Eqs. 32-35) ties the cell's side a, pitch h and the elliptical yarn
cross-section (semi-axes c, d) to the fibre count n_f, the fibre diameter d_f,
the fibre volume fraction phi_f and the interior braiding angle gamma.
Sec. 4.2 (Eqs. 36-37) gives the yarn's longitudinal and transverse
conductivities from those of fibre and matrix.
"""

from __future__ import annotations

import math

#: yarn volume fraction of the cell, pi*sqrt(3)/8 (Eq. 35)
PHI_Y_EXACT = math.pi * math.sqrt(3.0) / 8.0
#: the two-digit value the paper carries into its numbers (Eq. 35, Table II)
PHI_Y_ROUNDED = 0.68


def unit_cell_geometry(phi_f: float, gamma_deg: float, n_f: int = 9000, d_f: float = 6.9e-3,
                       phi_y: float = PHI_Y_ROUNDED) -> dict:
    """Eqs. 32-35.  Lengths in the unit of ``d_f`` (default mm).

    The fibre fraction inside a yarn is phi_fy = phi_f / phi_y; the yarn
    cross-section area A = n_f pi d_f^2 / 4 / phi_fy equals pi d c with
    c = sqrt(3) d cos(gamma) (Eqs. 33-34), which fixes d; then a = 8 d
    (Eq. 32).  The pitch h is not stated in the paper; h = a / tan(gamma)
    reproduces the worked example of Sec. 5 (a = 2.724 mm, h = 5.843 mm at
    gamma = 25 deg, phi_f = 0.4).
    """
    g = math.radians(gamma_deg)
    phi_fy = phi_f / phi_y
    area = n_f * math.pi * d_f * d_f / 4.0 / phi_fy
    d = math.sqrt(area / (math.pi * math.sqrt(3.0) * math.cos(g)))
    c = math.sqrt(3.0) * d * math.cos(g)
    a = 8.0 * d
    h = a / math.tan(g)
    return dict(a=a, h=h, c=c, d=d, area=area, phi_fy=phi_fy)


def yarn_conductivities(phi_f: float, lam_f_long: float = 7.81, lam_f_trans: float = 0.675,
                        lam_m: float = 0.178, phi_y: float = PHI_Y_ROUNDED):
    """Eqs. 36-37: (longitudinal, transverse) conductivity of a yarn.

    The transverse rule is read with phi_fy (not 1 - phi_fy) in the
    numerator of the fraction: only that reading reproduces Table II
    (0.363 / 0.445 / 0.530 W/(m K)); the printed form gives values that fall
    with phi_f.
    """
    phi_fy = phi_f / phi_y
    lam_l = lam_f_long * phi_fy + lam_m * (1.0 - phi_fy)
    lam_t = lam_m + phi_fy / (1.0 / (lam_f_trans - lam_m) + (1.0 - phi_fy) / (2.0 * lam_m))
    return lam_l, lam_t


def paper_unit_cell(gamma_deg: float, phi_f: float, nxy: int = 56, lam_f_long: float = 7.81,
                    lam_f_trans: float = 0.675, lam_m: float = 0.178):
    """The paper's unit cell on the synthetic braid: an a x a x h box of
    Eqs. 32-35 with ``nxy`` voxels across (nz = nxy h / a rounded to an even
    count), yarn fraction phi_y = pi sqrt(3) / 8 (Eq. 35), yarn tensors from
    Eqs. 36-37 and an isotropic epoxy matrix.  Sec. 5's example grid is
    56 x 56 x 120 at gamma = 25 deg.  Returns (medium, geometry dict)."""
    from .media import braid

    geo = unit_cell_geometry(phi_f, gamma_deg)
    nz = int(round(nxy * geo["h"] / geo["a"]))
    nz += nz % 2
    lam_l, lam_t = yarn_conductivities(phi_f, lam_f_long, lam_f_trans, lam_m)
    m = braid(nxy, nxy, nz, gamma_deg, PHI_Y_EXACT, lam_l, lam_t, lam_m)
    return m, dict(geo, nx=nxy, ny=nxy, nz=nz, lam_l=lam_l, lam_t=lam_t, gamma=gamma_deg, phi_f=phi_f)
