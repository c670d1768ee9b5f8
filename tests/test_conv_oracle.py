"""Pins of the FP64 warm-start-network reference (oracle/conv.py).

Forward convolution against brute-force loops and scipy.ndimage.correlate;
every backward against central finite differences of a scalar loss; pooling
and upsampling by adjointness; Adam against torch.optim.Adam.
"""

import numpy as np
import pytest

from oracle import conv as C


def brute_conv(x, w, b, circ):
    n, D, H, W, ci = x.shape
    co = w.shape[0]
    y = np.zeros((n, D, H, W, co))
    dims = (W, H, D)
    for nn in range(n):
        for z in range(D):
            for yy in range(H):
                for xx in range(W):
                    acc = np.array(b, dtype=np.float64).copy()
                    for dz in range(3):
                        for dy in range(3):
                            for dx in range(3):
                                p = [xx + dx - 1, yy + dy - 1, z + dz - 1]
                                ok = True
                                for a in range(3):
                                    if not 0 <= p[a] < dims[a]:
                                        if circ[a]:
                                            p[a] %= dims[a]
                                        else:
                                            ok = False
                                if ok:
                                    acc += w[:, dz, dy, dx, :] @ x[nn, p[2], p[1], p[0], :]
                    y[nn, z, yy, xx] = acc
    return y


@pytest.mark.parametrize("circ", [(False, True, True), (True, False, True), (False, False, False)])
def test_conv_forward_brute_force(circ):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 4, 5, 3))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    assert np.allclose(C.conv3d(x, w, b, circ), brute_conv(x, w, b, circ), atol=1e-12)


@pytest.mark.parametrize("mode", ["wrap", "constant"])
def test_conv_forward_matches_scipy_correlate(mode):
    from scipy import ndimage

    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 5, 6, 7, 1))
    w = rng.standard_normal((1, 3, 3, 3, 1))
    circ = (mode == "wrap",) * 3
    y = C.conv3d(x, w, [0.0], circ)
    ref = ndimage.correlate(x[0, :, :, :, 0], w[0, :, :, :, 0], mode=mode, cval=0.0)
    assert np.allclose(y[0, :, :, :, 0], ref, atol=1e-12)


@pytest.mark.parametrize("circ", [(False, True, True), (True, True, False)])
def test_conv_backward_finite_differences(circ):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 4, 4, 2))
    w = rng.standard_normal((3, 3, 3, 3, 2))
    b = rng.standard_normal(3)
    r = rng.standard_normal((2, 3, 4, 4, 3))

    def loss(x_, w_, b_):
        return float((C.conv3d(x_, w_, b_, circ) * r).sum())

    dx, dw, db = C.conv3d_backward(x, w, r, circ)
    h = 1e-6
    for _ in range(12):
        i = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        assert abs((loss(xp, w, b) - loss(xm, w, b)) / (2 * h) - dx[i]) < 1e-6
        j = tuple(rng.integers(0, s) for s in w.shape)
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        assert abs((loss(x, wp, b) - loss(x, wm, b)) / (2 * h) - dw[j]) < 1e-6
    for k in range(3):
        bp, bm = b.copy(), b.copy()
        bp[k] += h
        bm[k] -= h
        assert abs((loss(x, w, bp) - loss(x, w, bm)) / (2 * h) - db[k]) < 1e-6


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 4, 6, 8, 3))
    y = rng.standard_normal((2, 2, 3, 4, 3))
    assert np.isclose((C.pool2(x) * y).sum(), (x * C.pool2_backward(y)).sum())
    assert np.isclose((C.up2(y) * x).sum(), (y * C.up2_backward(x)).sum())
    assert np.allclose(C.pool2(C.up2(y)), y)


def test_box_resample_pins():
    from scipy import ndimage

    rng = np.random.default_rng(5)
    x = rng.standard_normal((6, 8, 12, 3))
    # equal sizes: identity; halving: the 2x2x2 mean (numpy reshape)
    assert np.array_equal(C.box_resample(x, (6, 8, 12)), x)
    half = x.reshape(3, 2, 4, 2, 6, 2, 3).mean(axis=(1, 3, 5))
    assert np.allclose(C.box_resample(x, (3, 4, 6)), half, rtol=0, atol=1e-14)
    # ratio 1.5 along x (12 -> 8): fine centres 0..11 fall in coarse cells
    # 0,0,1,1,2,...; cell c takes fine voxels {floor(1.5c + 0.25) .. }: brute
    # force from the centre positions in floating point
    y = C.box_resample(x, (6, 8, 8))
    for cx in range(8):
        members = [i for i in range(12) if int(np.floor((i + 0.5) / 12 * 8)) == cx]
        assert np.allclose(y[:, :, cx], x[:, :, members].mean(axis=2), atol=1e-14)
    # uniform refinement (6 -> 12 along z): every coarse voxel has no member
    # and takes the fine voxel under its centre = nearest-neighbour zoom
    z = C.box_resample(x, (12, 8, 12))
    assert np.array_equal(z, ndimage.zoom(x, (2, 1, 1, 1), order=0, mode="grid-constant", grid_mode=True))
    # the mean is preserved whenever every coarse voxel has equally many members
    assert np.isclose(C.box_resample(x, (3, 2, 4)).mean(), x.mean())


def test_interp_to_fine_pins():
    from scipy import ndimage

    rng = np.random.default_rng(6)
    p = rng.standard_normal((4, 6, 8))
    assert np.allclose(C.interp_to_fine(p, p.shape), p, atol=1e-15)
    # library: pad y, z periodically and x by edge values, then linear
    # map_coordinates at the fine centres' coarse coordinates
    shape = (6, 9, 13)
    padded = np.pad(np.pad(p, ((1, 1), (1, 1), (0, 0)), mode="wrap"), ((0, 0), (0, 0), (1, 1)), mode="edge")
    zz, yy, xx = np.meshgrid(*[(np.arange(n) + 0.5) * nc / n - 0.5 for n, nc in zip(shape, p.shape)], indexing="ij")
    xx = np.clip(xx, 0, p.shape[2] - 1)
    ref = ndimage.map_coordinates(padded, [zz + 1, yy + 1, xx + 1], order=1, mode="nearest")
    assert np.allclose(C.interp_to_fine(p, shape), ref, atol=1e-13)
    # a profile linear in x is reproduced between the first and last centre
    lin = np.broadcast_to(np.arange(8, dtype=float) * 0.3 - 1.0, (4, 6, 8))
    f = C.interp_to_fine(lin, (4, 6, 32))
    xs = (np.arange(32) + 0.5) * 8 / 32 - 0.5
    inside = (xs >= 0) & (xs <= 7)
    assert np.allclose(f[..., inside], xs[inside] * 0.3 - 1.0, atol=1e-14)


def test_mse_gradient():
    rng = np.random.default_rng(5)
    p = rng.standard_normal(20)
    t = rng.standard_normal(20)
    L, g = C.mse(p, t)
    assert np.isclose(L, np.mean((p - t) ** 2))
    h = 1e-6
    for i in range(5):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        assert abs((C.mse(pp, t)[0] - C.mse(pm, t)[0]) / (2 * h) - g[i]) < 1e-7


def test_adam_matches_torch():
    import torch

    rng = np.random.default_rng(6)
    w0 = rng.standard_normal(10)
    grads = [rng.standard_normal(10) for _ in range(4)]
    p = torch.nn.Parameter(torch.tensor(w0))
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(10), np.zeros(10)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
        w, m, v = C.adam(w, g, m, v, t, lr=1e-2)
    assert np.allclose(w, p.detach().numpy(), atol=1e-12)
