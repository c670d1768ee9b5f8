"""FP64 reference of the warm-start network's layers (NumPy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Layout: activations are channels-last, x[n, D, H, W, C] with D = z, H = y,
W = x; a 3x3x3 convolution's weights are w[cout, 3, 3, 3, cin] indexed
(dz, dy, dx) in {0, 1, 2} for offsets -1, 0, +1 (cross-correlation, as in
deep-learning convolutions).  ``circ`` = (x, y, z) flags: True wraps that axis
periodically, False pads it with zeros.
"""

from __future__ import annotations

import numpy as np


def _pad(x, circ):
    """Pad the three spatial axes of x[n, D, H, W, C] by one cell."""
    cx, cy, cz = circ
    for ax, c in ((1, cz), (2, cy), (3, cx)):
        widths = [(0, 0)] * 5
        widths[ax] = (1, 1)
        x = np.pad(x, widths, mode="wrap" if c else "constant")
    return x


def conv3d(x, w, b, circ):
    """y[n, p, co] = b[co] + sum_{tap, ci} w[co, tap, ci] x[n, p + off(tap), ci]."""
    n, D, H, W, ci = x.shape
    co = w.shape[0]
    xp = _pad(np.asarray(x, np.float64), circ)
    y = np.zeros((n, D, H, W, co))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                patch = xp[:, dz:dz + D, dy:dy + H, dx:dx + W, :]
                y += patch @ np.asarray(w[:, dz, dy, dx, :], np.float64).T
    return y + np.asarray(b, np.float64)


def conv3d_backward(x, w, dy, circ):
    """Gradients of sum(dy * conv3d(x, w, b)) w.r.t. x, w and b."""
    n, D, H, W, ci = x.shape
    xp = _pad(np.asarray(x, np.float64), circ)
    dy = np.asarray(dy, np.float64)
    dw = np.zeros(w.shape)
    dxp = np.zeros(xp.shape)
    for dz in range(3):
        for dyy in range(3):
            for dx in range(3):
                patch = xp[:, dz:dz + D, dyy:dyy + H, dx:dx + W, :]
                dw[:, dz, dyy, dx, :] = np.einsum("nzyxo,nzyxi->oi", dy, patch)
                dxp[:, dz:dz + D, dyy:dyy + H, dx:dx + W, :] += dy @ np.asarray(w[:, dz, dyy, dx, :], np.float64)
    # fold the padding back (wrap adds onto the opposite face, zeros drop)
    cx, cy, cz = circ
    for ax, c in ((1, cz), (2, cy), (3, cx)):
        sl = [slice(None)] * 5
        if c:
            lo = [slice(None)] * 5
            hi = [slice(None)] * 5
            lo[ax] = 0
            hi[ax] = -1
            first = [slice(None)] * 5
            last = [slice(None)] * 5
            first[ax] = -2
            last[ax] = 1
            dxp[tuple(first)] += dxp[tuple(lo)]
            dxp[tuple(last)] += dxp[tuple(hi)]
        sl[ax] = slice(1, -1)
        dxp = dxp[tuple(sl)]
    db = dy.sum(axis=(0, 1, 2, 3))
    return dxp, dw, db


def relu(x):
    return np.maximum(x, 0.0)


def pool2(x):
    """2x2x2 average pooling."""
    n, D, H, W, c = x.shape
    return x.reshape(n, D // 2, 2, H // 2, 2, W // 2, 2, c).mean(axis=(2, 4, 6))


def pool2_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up2(x):
    """Nearest-neighbour 2x upsampling."""
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up2_backward(dy):
    n, D, H, W, c = dy.shape
    return dy.reshape(n, D // 2, 2, H // 2, 2, W // 2, 2, c).sum(axis=(2, 4, 6))


def box_resample(x, shape):
    """Resample x[D, H, W, C] to a (Dc, Hc, Wc) grid spanning the same box.

    Fine voxel i of n along an axis has its centre at (i + 1/2)/n of the box
    and belongs to coarse voxel floor((i + 1/2) nc / n); each coarse voxel is
    the mean of its fine voxels, or, when it has none (refinement), the fine
    voxel under its own centre."""
    D, H, W, C = x.shape
    out = np.zeros(tuple(shape) + (C,))
    owner = [[(2 * i + 1) * nc // (2 * n) for i in range(n)] for n, nc in zip((D, H, W), shape)]
    for cz in range(shape[0]):
        zs = [i for i in range(D) if owner[0][i] == cz] or [(2 * cz + 1) * D // (2 * shape[0])]
        for cy in range(shape[1]):
            ys = [i for i in range(H) if owner[1][i] == cy] or [(2 * cy + 1) * H // (2 * shape[1])]
            for cx in range(shape[2]):
                xs = [i for i in range(W) if owner[2][i] == cx] or [(2 * cx + 1) * W // (2 * shape[2])]
                out[cz, cy, cx] = x[np.ix_(zs, ys, xs)].reshape(-1, C).mean(axis=0)
    return out


def interp_to_fine(p, shape):
    """Trilinear interpolation of p[Dc, Hc, Wc] at the voxel centres of a
    (D, H, W) grid spanning the same box.  A fine centre sits at coarse
    coordinate (i + 1/2) nc / n - 1/2 (coarse centres at integers); y and z
    wrap periodically, x is clamped to the first and last coarse centre."""
    Dc, Hc, Wc = p.shape
    D, H, W = shape
    out = np.zeros(shape)
    for z in range(D):
        for y in range(H):
            for x in range(W):
                c = [(x + 0.5) * Wc / W - 0.5, (y + 0.5) * Hc / H - 0.5, (z + 0.5) * Dc / D - 0.5]
                base = [int(np.floor(v)) for v in c]
                t = [v - b for v, b in zip(c, base)]
                acc = 0.0
                for dz in (0, 1):
                    for dy in (0, 1):
                        for dx in (0, 1):
                            ix = min(max(base[0] + dx, 0), Wc - 1)
                            iy = (base[1] + dy) % Hc
                            iz = (base[2] + dz) % Dc
                            wgt = (t[0] if dx else 1 - t[0]) * (t[1] if dy else 1 - t[1]) * (t[2] if dz else 1 - t[2])
                            acc += wgt * p[iz, iy, ix]
                out[z, y, x] = acc
    return out


def mse(pred, target):
    d = np.asarray(pred, np.float64) - np.asarray(target, np.float64)
    return float((d * d).mean()), 2.0 * d / d.size


def adam(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
