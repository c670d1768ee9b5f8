"""Dense matrix form of one lattice Boltzmann step, for tiny grids.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The scheme of Sec. 2 is affine in the distributions: one step maps the
pre-collision state f (7 N values, population-major) to

    f(t+1) = L f(t) + b,   L = S_stream C,

where C is block diagonal with one 7x7 block P = I - Omega (I - w 1^T) per
node (collision, Eq. 5 with f_eq = w T of Eq. 6 and Omega = M^-1 S M of
Eq. 8), S_stream moves each post-collision population along its link
(Eq. 21) or reflects it at a wall (Eqs. 23-25), and b carries the wall
temperatures of the Dirichlet faces.  The steady state is the solution of
(I - L) f* = b.  Everything here is written independently of the C oracle.
"""

from __future__ import annotations

import numpy as np

GAMMA = 1.0 / 8.0
EPS = 2.0 * GAMMA
E = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
OPP = np.array([0, 2, 1, 4, 3, 6, 5])
W = np.array([1 - 6 * GAMMA] + [GAMMA] * 6)  # f_eq = W T  (Eq. 6)


def moment_matrix(c: float = 1.0, rows_123_only: bool = False) -> np.ndarray:
    """Eq. 11.  ``c`` scales the whole matrix, or only the flux rows."""
    M = np.array([[1, 1, 1, 1, 1, 1, 1],
                  [0, 1, -1, 0, 0, 0, 0],
                  [0, 0, 0, 1, -1, 0, 0],
                  [0, 0, 0, 0, 0, 1, -1],
                  [6, -1, -1, -1, -1, -1, -1],
                  [0, 2, 2, -1, -1, -1, -1],
                  [0, 0, 0, 1, 1, -1, -1]], dtype=np.float64)
    if rows_123_only:
        M[1:4] *= c
    else:
        M *= c
    return M


def omega(tau3, tau_rest=(1.0, 1.0, 1.0, 1.0), c: float = 1.0, rows_123_only: bool = False) -> np.ndarray:
    """Omega = M^-1 S M with S the matrix inverse of Eq. 12's S^-1."""
    Sinv = np.zeros((7, 7))
    Sinv[0, 0] = tau_rest[0]
    Sinv[1:4, 1:4] = tau3
    Sinv[4, 4], Sinv[5, 5], Sinv[6, 6] = tau_rest[1], tau_rest[2], tau_rest[3]
    M = moment_matrix(c, rows_123_only)
    return np.linalg.inv(M) @ np.linalg.inv(Sinv) @ M


def collision_block(tau3, tau_rest=(1.0, 1.0, 1.0, 1.0)) -> np.ndarray:
    """P with f_hat = P f (Eq. 5): P = I - Omega (I - W 1^T)."""
    Om = omega(tau3, tau_rest)
    return np.eye(7) - Om @ (np.eye(7) - np.outer(W, np.ones(7)))


def scale_for(k6, dmax: float = 1.0) -> float:
    """s such that max eigenvalue of tau - I/2 = D/eps = s k/eps is dmax."""
    lmax = max(np.linalg.eigvalsh(_full(r)).max() for r in k6)
    return dmax * EPS / lmax


def _full(r):
    xx, yy, zz, xy, xz, yz = r
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]], dtype=np.float64)


def tau_of(k6row, s: float) -> np.ndarray:
    """Eq. 13 in lattice units: tau = I/2 + s k / eps."""
    return 0.5 * np.eye(3) + s * _full(k6row) / EPS


def affine_step(phase: np.ndarray, k6, dmax: float, grad_axis: int, t_hot: float, t_cold: float,
                sides, tau_rest=(1.0, 1.0, 1.0, 1.0)):
    """Return (L, b, s) of the one-step map on the pre-collision state.

    ``sides[a]`` for non-gradient axes: 0 periodic, 1 adiabatic.  The
    gradient axis has Dirichlet walls, t_hot on its index-0 face."""
    nz, ny, nx = phase.shape
    dims = (nx, ny, nz)
    N = phase.size
    s = scale_for(k6, dmax)
    blocks = [collision_block(tau_of(r, s), tau_rest) for r in k6]
    C = np.zeros((7 * N, 7 * N))
    flat = phase.reshape(-1)
    for x in range(N):
        Pb = blocks[flat[x]]
        idx = np.arange(7) * N + x
        C[np.ix_(idx, idx)] = Pb
    S = np.zeros((7 * N, 7 * N))
    b = np.zeros(7 * N)

    def lin(p):
        return (p[2] * ny + p[1]) * nx + p[0]

    for z in range(nz):
        for y in range(ny):
            for xx in range(nx):
                p = (xx, y, z)
                src = lin(p)
                S[src, src] = 1.0  # rest population
                for i in range(1, 7):
                    a = (i - 1) // 2
                    q = [p[0] + E[i, 0], p[1] + E[i, 1], p[2] + E[i, 2]]
                    if 0 <= q[a] < dims[a] or (a != grad_axis and sides[a] == 0):
                        q[a] %= dims[a]
                        S[i * N + lin(q), i * N + src] = 1.0
                    elif a != grad_axis:  # adiabatic bounce-back
                        S[OPP[i] * N + src, i * N + src] = 1.0
                    else:  # Dirichlet anti-bounce-back
                        S[OPP[i] * N + src, i * N + src] = -1.0
                        tw = t_hot if E[i, a] < 0 else t_cold
                        b[OPP[i] * N + src] += EPS * tw
    return S @ C, b, s


def fixed_point(phase, k6, dmax, grad_axis, t_hot, t_cold, sides, tau_rest=(1.0, 1.0, 1.0, 1.0)):
    """Steady pre-collision state f* (7, nz, ny, nx) from (I - L) f* = b."""
    L, b, s = affine_step(phase, k6, dmax, grad_axis, t_hot, t_cold, sides, tau_rest)
    f = np.linalg.solve(np.eye(L.shape[0]) - L, b)
    return f.reshape((7,) + phase.shape), s
