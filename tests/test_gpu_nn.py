"""Warm-start network kernels (BF16 MFMA, FP32 accumulation) against the FP64
reference of oracle/conv.py.

Inputs are drawn, rounded to BF16 on the host, and the same rounded values
feed both sides, so the differences are the GPU's FP32 accumulation and its
BF16 outputs.  Bars: relative L2 <= 1e-2 and cosine >= 0.999 for BF16
outputs, relative L2 <= 1e-4 for FP32 outputs of exact-BF16 inputs.
"""

import ctypes

import numpy as np
import pytest

from oracle import conv as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no HIP device")
    from paper_1503_08718_amd import load

    L = load()
    return L, torch


def bf(torch, a):
    """Round to BF16; return (device tensor, float64 numpy copy of the rounded values)."""
    t = torch.tensor(np.asarray(a, np.float32)).to(torch.bfloat16)
    return t.cuda(), t.float().numpy().astype(np.float64)


def P(t):
    return ctypes.c_void_p(t.data_ptr())


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def cosine(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def circ_bits(circ):
    return int(circ[0]) | (int(circ[1]) << 1) | (int(circ[2]) << 2)


def pack_w(L, w):
    """oracle weights [cout, 3, 3, 3, cin] -> GPU rows [cout][kpad]."""
    cout, cin = w.shape[0], w.shape[-1]
    kpad = L.mrtlbm_nn_kpad(cin)
    out = np.zeros((cout, kpad), np.float32)
    out[:, :27 * cin] = w.reshape(cout, 27 * cin)
    return out


SHAPES = [
    # (n, D, H, W, cin, cout, circ)
    (2, 4, 6, 10, 8, 16, (False, True, True)),
    (1, 8, 8, 8, 16, 32, (True, True, True)),
    (2, 6, 4, 8, 32, 64, (False, False, False)),
    (1, 4, 4, 4, 128, 128, (False, True, True)),
    (1, 6, 10, 4, 64, 16, (True, False, True)),
    # channel counts of the generic forward kernel (24 in the forward pass, 48
    # in the input gradient of the second); the others have kernels of their own
    (2, 4, 6, 8, 24, 32, (False, True, True)),
    (1, 6, 4, 8, 32, 48, (True, True, False)),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s[:6])))
def test_conv_forward(env, shape):
    L, torch = env
    n, D, H, W, cin, cout, circ = shape
    rng = np.random.default_rng(cin * 7 + cout)
    xd, x = bf(torch, rng.standard_normal((n, D, H, W, cin)))
    w = rng.standard_normal((cout, 3, 3, 3, cin)) * 0.2
    wd, wq = bf(torch, pack_w(L, w))
    w_or = wq[:, :27 * cin].reshape(cout, 3, 3, 3, cin)
    b = torch.tensor(rng.standard_normal(cout).astype(np.float32)).cuda()
    ref = C.conv3d(x, w_or, b.cpu().numpy().astype(np.float64), circ)
    out32 = torch.empty((n * D * H * W, cout), dtype=torch.float32, device="cuda")
    assert L.mrtlbm_nn_conv3d_fwd(P(xd), n, D, H, W, cin, P(wd), P(b), cout, circ_bits(circ), 0, None, P(out32),
                                  None) == 0
    assert rel_l2(out32.cpu().numpy(), ref) < 1e-5
    outb = torch.empty((n * D * H * W, cout), dtype=torch.bfloat16, device="cuda")
    assert L.mrtlbm_nn_conv3d_fwd(P(xd), n, D, H, W, cin, P(wd), P(b), cout, circ_bits(circ), 1, P(outb), None,
                                  None) == 0
    got = outb.float().cpu().numpy()
    r = C.relu(ref)
    assert rel_l2(got, r) < 1e-2 and cosine(got, r) > 0.999


@pytest.mark.parametrize("cin,cout", [(64, 64), (128, 128), (16, 64)])
def test_conv_tile_choice_leaves_results_unchanged(env, cin, cout):
    """The launcher shrinks the tiles of a wave for small launches (8^3 x 1:
    16 x 16 tiles) and keeps them large for big ones (64 copies of the same
    grid): every copy's output equals the single grid's bit for bit, as each
    output element sums the same products in the same k order."""
    L, torch = env
    D = H = W = 8
    rng = np.random.default_rng(cin + cout)
    xd, _ = bf(torch, rng.standard_normal((1, D, H, W, cin)))
    wd, _ = bf(torch, pack_w(L, rng.standard_normal((cout, 3, 3, 3, cin)) * 0.2))
    b = torch.tensor(rng.standard_normal(cout).astype(np.float32)).cuda()
    one = torch.empty((D * H * W, cout), dtype=torch.float32, device="cuda")
    assert L.mrtlbm_nn_conv3d_fwd(P(xd), 1, D, H, W, cin, P(wd), P(b), cout, 0b110, 0, None, P(one), None) == 0
    many_in = xd.repeat(64, 1, 1, 1, 1).contiguous()
    many = torch.empty((64 * D * H * W, cout), dtype=torch.float32, device="cuda")
    assert L.mrtlbm_nn_conv3d_fwd(P(many_in), 64, D, H, W, cin, P(wd), P(b), cout, 0b110, 0, None, P(many),
                                  None) == 0
    torch.cuda.synchronize()
    assert torch.equal(many.view(64, D * H * W, cout), one.view(1, D * H * W, cout).expand(64, -1, -1))


@pytest.mark.parametrize("shape", [s for s in SHAPES if s[4] % 16 == 0], ids=lambda s: "x".join(map(str, s[:6])))
def test_conv_backward(env, shape):
    L, torch = env
    n, D, H, W, cin, cout, circ = shape
    rng = np.random.default_rng(cin + 3 * cout)
    xd, x = bf(torch, rng.standard_normal((n, D, H, W, cin)))
    w = rng.standard_normal((cout, 3, 3, 3, cin)) * 0.2
    wd, wq = bf(torch, pack_w(L, w))
    w_or = wq[:, :27 * cin].reshape(cout, 3, 3, 3, cin)
    dyd, dy = bf(torch, rng.standard_normal((n, D, H, W, cout)))
    dx_ref, dw_ref, db_ref = C.conv3d_backward(x, w_or, dy, circ)
    wt = torch.empty(cin * L.mrtlbm_nn_kpad(cout), dtype=torch.bfloat16, device="cuda")
    dx = torch.empty((n * D * H * W, cin), dtype=torch.bfloat16, device="cuda")
    assert L.mrtlbm_nn_conv3d_dgrad(P(dyd), n, D, H, W, cin, P(wd), cout, circ_bits(circ), P(wt), P(dx), None) == 0
    got = dx.float().cpu().numpy()
    assert rel_l2(got, dx_ref) < 1e-2 and cosine(got, dx_ref) > 0.999
    nbytes = L.mrtlbm_nn_wgrad_scratch_bytes(n, D, H, W, cin, cout)
    scratch = torch.empty(nbytes // 4 + 1, dtype=torch.float32, device="cuda")
    dw = torch.empty((cout, L.mrtlbm_nn_kpad(cin)), dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    assert L.mrtlbm_nn_conv3d_wgrad(P(xd), P(dyd), n, D, H, W, cin, cout, circ_bits(circ), P(scratch), P(dw), P(db),
                                    None) == 0
    dwg = dw.cpu().numpy()
    assert np.all(dwg[:, 27 * cin:] == 0)
    assert rel_l2(dwg[:, :27 * cin], dw_ref.reshape(cout, -1)) < 1e-4
    assert rel_l2(db.cpu().numpy(), db_ref) < 1e-4


def test_pool_upsample_add_relu(env):
    L, torch = env
    rng = np.random.default_rng(9)
    n, D, H, W, c = 2, 4, 6, 8, 16
    xd, x = bf(torch, rng.standard_normal((n, D, H, W, c)))
    out = torch.empty((n * D * H * W // 8, c), dtype=torch.bfloat16, device="cuda")
    assert L.mrtlbm_nn_pool2(1, P(xd), n, D, H, W, c, P(out), None) == 0
    assert rel_l2(out.float().cpu().numpy(), C.pool2(x)) < 5e-3
    yd, y = bf(torch, rng.standard_normal((n, D // 2, H // 2, W // 2, c)))
    back = torch.empty((n * D * H * W, c), dtype=torch.bfloat16, device="cuda")
    assert L.mrtlbm_nn_pool2(0, P(yd), n, D, H, W, c, P(back), None) == 0
    assert rel_l2(back.float().cpu().numpy(), C.pool2_backward(y)) < 5e-3
    up = torch.empty((n * D * H * W, c), dtype=torch.bfloat16, device="cuda")
    assert L.mrtlbm_nn_up2(1, P(yd), n, D // 2, H // 2, W // 2, c, P(up), None) == 0
    assert np.array_equal(up.float().cpu().numpy().reshape(n, D, H, W, c), C.up2(y))
    dn = torch.empty((n * D * H * W // 8, c), dtype=torch.bfloat16, device="cuda")
    assert L.mrtlbm_nn_up2(0, P(xd), n, D // 2, H // 2, W // 2, c, P(dn), None) == 0
    assert rel_l2(dn.float().cpu().numpy(), C.up2_backward(x)) < 5e-3
    s = torch.empty_like(xd)
    assert L.mrtlbm_nn_add(P(xd), P(xd), P(s), xd.numel(), None) == 0
    assert np.array_equal(s.float().cpu().numpy(), 2 * x)
    g = torch.empty_like(xd)
    assert L.mrtlbm_nn_relu_bwd(P(xd), P(xd), P(g), xd.numel(), None) == 0
    assert np.array_equal(g.float().cpu().numpy(), np.where(x > 0, x, 0))
    # the one-element kernels behind the 8-channel ones: a count that is not
    # a multiple of 8, and an output that is not 16-byte aligned
    m = xd.numel() - 3
    s2 = torch.empty_like(xd)
    assert L.mrtlbm_nn_add(P(xd), P(xd), P(s2), m, None) == 0
    assert np.array_equal(s2.float().cpu().numpy().ravel()[:m], 2 * x.ravel()[:m])
    g2 = torch.empty_like(xd)
    assert L.mrtlbm_nn_relu_bwd(P(xd), P(xd), P(g2), m, None) == 0
    assert np.array_equal(g2.float().cpu().numpy().ravel()[:m], np.where(x > 0, x, 0).ravel()[:m])
    up_u = torch.empty(n * D * H * W * c + 1, dtype=torch.bfloat16, device="cuda")
    assert L.mrtlbm_nn_up2(1, P(yd), n, D // 2, H // 2, W // 2, c, ctypes.c_void_p(up_u.data_ptr() + 2), None) == 0
    assert np.array_equal(up_u[1:].float().cpu().numpy().reshape(n, D, H, W, c), C.up2(y))


def test_mse_and_adam(env):
    L, torch = env
    rng = np.random.default_rng(10)
    nv = 5000
    pred = torch.tensor(rng.standard_normal((nv, 16)).astype(np.float32)).cuda()
    tgt = torch.tensor(rng.standard_normal(nv).astype(np.float32)).cuda()
    dpred = torch.empty((nv, 16), dtype=torch.bfloat16, device="cuda")
    scratch = torch.empty(1024, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    assert L.mrtlbm_nn_mse(P(pred), 16, P(tgt), nv, P(dpred), P(scratch), P(loss), None) == 0
    lref, gref = C.mse(pred.cpu().numpy()[:, 0], tgt.cpu().numpy())
    assert abs(loss.item() - lref) < 1e-5 * lref
    d = dpred.float().cpu().numpy()
    assert rel_l2(d[:, 0], gref) < 5e-3 and np.all(d[:, 1:] == 0)
    w0 = rng.standard_normal(777)
    w = torch.tensor(w0.astype(np.float32)).cuda()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    wb = torch.empty(777, dtype=torch.bfloat16, device="cuda")
    wr, mr, vr = w0.copy(), np.zeros(777), np.zeros(777)
    for t in range(1, 4):
        gnp = rng.standard_normal(777)
        g = torch.tensor(gnp.astype(np.float32)).cuda()
        assert L.mrtlbm_nn_adam(P(w), P(g), P(m), P(v), 777, 1e-2, 0.9, 0.999, 1e-8, t, P(wb), None) == 0
        wr, mr, vr = C.adam(wr, gnp.astype(np.float32).astype(np.float64), mr, vr, t, lr=1e-2)
    assert np.allclose(w.cpu().numpy(), wr, atol=1e-5)
    assert rel_l2(wb.float().cpu().numpy(), wr) < 5e-3


def _q(a):
    """Round to BF16 (the precision the GPU stores activations and their
    gradients in), keep FP64 arithmetic otherwise."""
    import torch

    return torch.tensor(np.asarray(a, np.float32)).to(torch.bfloat16).double().numpy()


def _oracle_net(x, W, B, target, keep=False):
    """FP64 forward/backward of the warm-start network with the same weights.
    Every tensor the GPU stores in BF16 is rounded to BF16 at the same point,
    so that both sides take the same ReLU decisions."""
    circ = (False, True, True)
    f = {}

    def conv(name, inp, relu=True):
        y = C.conv3d(inp, W[name], B[name], circ)
        return _q(C.relu(y)) if relu else y

    f["a00"] = conv("c00", x)
    f["e0"] = conv("c01", f["a00"])
    f["p1"] = _q(C.pool2(f["e0"]))
    f["a10"] = conv("c10", f["p1"])
    f["e1"] = conv("c11", f["a10"])
    f["p2"] = _q(C.pool2(f["e1"]))
    f["a20"] = conv("c20", f["p2"])
    f["e2"] = conv("c21", f["a20"])
    f["p3"] = _q(C.pool2(f["e2"]))
    f["a30"] = conv("c30", f["p3"])
    f["e3"] = conv("c31", f["a30"])
    f["u2"] = C.up2(f["e3"])
    f["b2"] = conv("c22", f["u2"])
    f["s2"] = _q(f["b2"] + f["e2"])
    f["d2"] = conv("c23", f["s2"])
    f["u1"] = C.up2(f["d2"])
    f["b1"] = conv("c12", f["u1"])
    f["s1"] = _q(f["b1"] + f["e1"])
    f["d1"] = conv("c13", f["s1"])
    f["u0"] = C.up2(f["d1"])
    f["b0"] = conv("c02", f["u0"])
    f["s0"] = _q(f["b0"] + f["e0"])
    f["d0"] = conv("c03", f["s0"])
    out = conv("c04", f["d0"], relu=False)  # FP32 output on the GPU
    loss, dpred = C.mse(out[..., 0].ravel(), target)
    grads = {}

    def back(name, inp, y, dy, relu=True):
        dpre = _q(dy * (y > 0)) if relu else dy
        dx, dw, db = C.conv3d_backward(inp, W[name], dpre, circ)
        grads[name] = (dw, db)
        return _q(dx)

    dout = np.zeros(out.shape)
    dout[..., 0] = dpred.reshape(out.shape[:-1])
    dout = _q(dout)
    g_d0 = back("c04", f["d0"], out, dout, relu=False)
    g_s0 = back("c03", f["s0"], f["d0"], g_d0)
    g_u0 = back("c02", f["u0"], f["b0"], g_s0)
    g_d1 = _q(C.up2_backward(g_u0))
    g_s1 = back("c13", f["s1"], f["d1"], g_d1)
    g_u1 = back("c12", f["u1"], f["b1"], g_s1)
    g_d2 = _q(C.up2_backward(g_u1))
    g_s2 = back("c23", f["s2"], f["d2"], g_d2)
    g_u2 = back("c22", f["u2"], f["b2"], g_s2)
    g_e3 = _q(C.up2_backward(g_u2))
    g_a30 = back("c31", f["a30"], f["e3"], g_e3)
    g_p3 = back("c30", f["p3"], f["a30"], g_a30)
    g_e2 = _q(_q(C.pool2_backward(g_p3)) + g_s2)
    g_a20 = back("c21", f["a20"], f["e2"], g_e2)
    g_p2 = back("c20", f["p2"], f["a20"], g_a20)
    g_e1 = _q(_q(C.pool2_backward(g_p2)) + g_s1)
    g_a10 = back("c11", f["a10"], f["e1"], g_e1)
    g_p1 = back("c10", f["p1"], f["a10"], g_a10)
    g_e0 = _q(_q(C.pool2_backward(g_p1)) + g_s0)
    g_a00 = back("c01", f["a00"], f["e0"], g_e0)
    back("c00", x, f["a00"], g_a00)
    return (loss, out, grads, f) if keep else (loss, out, grads)


# every layer of the network: (input activation, output activation, upstream
# gradient, where its input gradient goes), as Net.forward / Net.backward
# store them
TEACHER = {
    "c00": ("x", "a00", ("grad", "a00"), None, 0),
    "c01": ("a00", "e0", ("grad", "e0"), "a00", 0),
    "c10": ("p1", "a10", ("grad", "a10"), "p1", 1),
    "c11": ("a10", "e1", ("grad", "e1"), "a10", 1),
    "c20": ("p2", "a20", ("grad", "a20"), "p2", 2),
    "c21": ("a20", "e2", ("grad", "e2"), "a20", 2),
    "c30": ("p3", "a30", ("grad", "a30"), "p3", 3),
    "c31": ("a30", "e3", ("grad", "e3"), "a30", 3),
    "c22": ("u2", "b2", ("grad", "s2"), "u2", 2),
    "c23": ("s2", "d2", ("grad", "d2"), "s2", 2),
    "c12": ("u1", "b1", ("grad", "s1"), "u1", 1),
    "c13": ("s1", "d1", ("grad", "d1"), "s1", 1),
    "c02": ("u0", "b0", ("grad", "s0"), "u0", 0),
    "c03": ("s0", "d0", ("grad", "d0"), "s0", 0),
    "c04": ("d0", None, ("act", "dout"), "d0", 0),
}


def _trained_net_pass(env, n=32, grid=None):
    L, torch = env
    from paper_1503_08718_amd import warmstart as ws

    net = ws.Net(n=n, batch=1, seed=3)
    if grid is not None:
        net.set_grid(*grid)
    nv = int(np.prod(net.grid))
    rng = np.random.default_rng(11)
    xd, x = bf(torch, np.concatenate([rng.uniform(-1, 1, (nv, 7)), np.zeros((nv, 1))], axis=1))
    net.act["x"].copy_(xd)
    tgt = rng.uniform(-1, 1, nv).astype(np.float32)
    net.target.copy_(torch.tensor(tgt).cuda())
    net.forward()
    net.loss_and_grad()
    net.backward()
    torch.cuda.synchronize()
    W, B = {}, {}
    for name, cin, cout, _ in ws.LAYERS:
        wq = net.wbf[name].float().cpu().numpy().astype(np.float64)
        W[name] = wq[:, :27 * cin].reshape(cout, 3, 3, 3, cin)
        B[name] = net.b32[name].cpu().numpy().astype(np.float64)
    return net, ws, x, tgt, W, B


@pytest.mark.parametrize("grid", [(32, 32, 32), (16, 24, 32)], ids=lambda g: "x".join(map(str, g)))
def test_every_layer_teacher_forced(env, grid):
    """Each of the 15 layers of one forward and backward pass, on the 32^3
    training-shaped grid and on an uneven (z, y, x) = 16 x 24 x 32 grid such
    as uneven cells are predicted on (coarse levels down to 2 x 3 x 4), fed
    with the GPU's own stored BF16 input activation and upstream gradient:
    the FP64 oracle's output, input gradient (BF16 on the GPU: relative L2
    <= 1e-2, cosine >= 0.999) and weight and bias gradients (FP32 on the GPU
    from exact BF16 operands: relative L2 <= 1e-4) -- the per-kernel bars,
    layer by layer, so that an indexing or adjoint fault in any one layer
    cannot hide behind the BF16 rounding of the layers before it."""
    L, torch = env
    net, ws, _, _, W, B = _trained_net_pass(env, grid=grid)
    assert net.grid == grid
    circ = (False, True, True)

    def host(t, lv, c):
        d, h, w = (e >> lv for e in grid)
        return t.float().cpu().numpy().astype(np.float64).reshape(1, d, h, w, -1)[..., :c]

    report = []
    for name, cin, cout, relu in ws.LAYERS:
        src, dst, (kind, gname), dxname, lv = TEACHER[name]
        xin = host(net.act[src], lv, cin)
        dy = host((net.grad if kind == "grad" else net.act)[gname], lv, cout)
        y_or = C.conv3d(xin, W[name], B[name], circ)
        if relu:
            y_gpu = host(net.act[dst], lv, cout)
            y_ref = _q(C.relu(y_or))
            assert rel_l2(y_gpu, y_ref) <= 1e-2 and cosine(y_gpu, y_ref) >= 0.999, (name, "forward")
            dpre = _q(dy * (y_gpu > 0))  # the GPU's own ReLU decisions
        else:
            out = net.out.cpu().numpy().astype(np.float64).reshape((1,) + grid + (cout,))
            assert rel_l2(out, y_or) <= 1e-4, (name, "forward")
            dpre = dy
        dx, dw, db = C.conv3d_backward(xin, W[name], dpre, circ)
        gw = net.gw[name].cpu().numpy()[:, :27 * cin].astype(np.float64)
        gb = net.gb[name].cpu().numpy().astype(np.float64)
        rw, rb = rel_l2(gw, dw.reshape(cout, -1)), rel_l2(gb, db)
        line = [name, rw, rb]
        assert rw <= 1e-4 and rb <= 1e-4, (name, rw, rb)
        if dxname is not None:
            g_dx = host(net.grad[dxname], lv, cin)
            rx, cx = rel_l2(g_dx, dx), cosine(g_dx, dx)
            line += [rx, cx]
            assert rx <= 1e-2 and cx >= 0.999, (name, "input gradient", rx, cx)
        report.append(line)
    print("layer: weight-grad rel L2, bias-grad rel L2, [input-grad rel L2, cosine]")
    for line in report:
        print(" ".join(f"{v:.3e}" if isinstance(v, float) else v for v in line))


def test_whole_network_forward_and_gradients(env):
    """The whole pass against an FP64 oracle that runs the network on its own,
    rounding to BF16 wherever the GPU stores.  The forward output and the
    loss agree closely; deep in the backward pass, the two sides' ReLU
    decisions part where a pre-activation lies within BF16 rounding of zero,
    so the end-to-end weight gradients are held only to a direction (cosine
    > 0.99); each layer meets the per-kernel bars in the teacher-forced test
    above.  The share of ReLU decisions that differ is measured and bounded."""
    L, torch = env
    net, ws, x, tgt, W, B = _trained_net_pass(env)
    n = net.n
    loss, out, grads, fwd = _oracle_net(x.reshape(1, n, n, n, 8), W, B, tgt.astype(np.float64), keep=True)
    got_out = net.out.cpu().numpy()[:, 0]
    assert cosine(got_out, out[..., 0].ravel()) > 0.999
    assert abs(net.loss.item() - loss) < 0.02 * loss
    flips, total = 0, 0
    for name, cin, cout, relu in ws.LAYERS:
        if not relu:
            continue
        src, dst, _, _, lv = TEACHER[name]
        d = n >> lv
        yg = net.act[dst].float().cpu().numpy().reshape(1, d, d, d, -1)[..., :cout] > 0
        flips += int(np.count_nonzero(yg != (fwd[dst] > 0)))
        total += yg.size
    print(f"ReLU decisions that differ: {flips} of {total}")
    assert flips <= 2e-3 * total  # measured: 1783 of 2768896 (6.4e-4)
    for name, cin, cout, _ in ws.LAYERS:
        gw = net.gw[name].cpu().numpy()[:, :27 * cin]
        rw = grads[name][0].reshape(cout, -1)
        assert cosine(gw, rw) > 0.99, name


@pytest.mark.parametrize("coarse", [(10, 12, 20), (5, 6, 10), (8, 8, 8), (16, 16, 16), (4, 12, 7)],
                         ids=lambda s: "x".join(map(str, s)))
def test_resampled_features(env, coarse):
    L, torch = env
    rng = np.random.default_rng(21)
    D, H, W = 10, 12, 20
    phase = rng.integers(0, 5, (D, H, W)).astype(np.uint8)
    feat = rng.uniform(-1, 1, (5, 6)).astype(np.float32)
    out = torch.empty((int(np.prod(coarse)), 8), dtype=torch.bfloat16, device="cuda")
    ph, fd = torch.from_numpy(phase).cuda(), torch.from_numpy(feat).cuda()
    assert L.mrtlbm_nn_features_resampled(P(ph), D, H, W, P(fd), *coarse, P(out), None) == 0
    got = out.float().cpu().numpy().astype(np.float64).reshape(coarse + (8,))
    ref = C.box_resample(feat.astype(np.float64)[phase], coarse)
    # one BF16 rounding of an FP32 mean
    assert np.all(np.abs(got[..., :6] - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-6)
    xc = (np.arange(coarse[2]) + 0.5) / coarse[2] - 0.5
    assert np.allclose(got[..., 6], np.broadcast_to(xc, coarse), atol=2.0 ** -9)
    assert not got[..., 7].any()


@pytest.mark.parametrize("grids", [((8, 8, 8), (8, 8, 8)), ((4, 6, 8), (6, 9, 13)), ((8, 8, 8), (12, 16, 24)),
                                   ((8, 8, 8), (4, 8, 6))], ids=lambda g: "x".join(map(str, g[0] + g[1])))
def test_start_field_interpolation(env, grids):
    L, torch = env
    (Dc, Hc, Wc), fine = grids
    rng = np.random.default_rng(22)
    scale, margin = 10.0, 0.05
    pred = rng.uniform(-0.2, 0.2, (Dc, Hc, Wc, 16)).astype(np.float32)
    pred[Dc // 2, Hc // 3, Wc // 2, 0] = 30.0  # pushes part of the field out of range
    T = torch.empty(fine, dtype=torch.float32, device="cuda")
    scratch = torch.empty(2048, dtype=torch.int32, device="cuda")
    bad = ctypes.c_longlong()
    pd = torch.from_numpy(pred).cuda()
    assert L.mrtlbm_nn_to_temperature(P(pd), 16, Dc, Hc, Wc, *fine, scale, margin, P(T), P(scratch),
                                      ctypes.byref(bad), None) == 0
    W = fine[2]
    tlin = 1.0 - (np.arange(W) + 0.5) / W
    ref = tlin + C.interp_to_fine(pred[..., 0].astype(np.float64), fine) / scale
    assert np.abs(T.cpu().numpy() - ref).max() < 1e-5
    out = (ref < -margin) | (ref > 1 + margin)
    edge = np.minimum(np.abs(ref + margin), np.abs(ref - 1 - margin))
    assert edge.min() > 1e-4  # no value sits within rounding of a threshold
    assert bad.value == int(out.sum()) and bad.value > 0


def test_feature_table_spacing(env):
    L, torch = env
    rng = np.random.default_rng(23)
    A = rng.standard_normal((4, 3, 3))
    K = A @ A.transpose(0, 2, 1) + 0.3 * np.eye(3)
    k6 = np.stack([K[:, 0, 0], K[:, 1, 1], K[:, 2, 2], K[:, 0, 1], K[:, 0, 2], K[:, 1, 2]], axis=1)

    def table(k, sp):
        k = np.ascontiguousarray(k, np.float64)
        sp = np.ascontiguousarray(sp, np.float64)
        out = np.empty((k.shape[0], 6), np.float32)
        dp = ctypes.POINTER(ctypes.c_double)
        st = L.mrtlbm_nn_feature_table(k.ctypes.data_as(dp), k.shape[0], sp.ctypes.data_as(dp),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        return st, out

    sp = (1.5, 1.0, 2.0)
    st, got = table(k6, sp)
    assert st == 0
    S = np.diag(1.0 / np.asarray(sp))
    Kt = S @ K @ S  # K'_ab = K_ab / (s_a s_b)
    ref = np.stack([Kt[:, 0, 0], Kt[:, 1, 1], Kt[:, 2, 2], Kt[:, 0, 1], Kt[:, 0, 2], Kt[:, 1, 2]], axis=1)
    ref /= np.linalg.eigvalsh(Kt).max()
    assert np.allclose(got, ref, rtol=1e-6, atol=1e-7)
    # a uniform power-of-two spacing changes nothing, bit for bit
    assert np.array_equal(table(k6, (1, 1, 1))[1], table(k6, (2, 2, 2))[1])
    bad = k6.copy()
    bad[1, 3] = 10.0 * np.sqrt(bad[1, 0] * bad[1, 1])
    assert table(bad, sp)[0] == -2  # E_TENSOR


def test_training_resumes_bit_for_bit(env, tmp_path):
    """A checkpoint holds the master weights, Adam's moments and step count
    and the batch-order generator: 3 iterations, save, load into a fresh
    network, 3 more, equal 6 iterations straight through, bit for bit."""
    L, torch = env
    from paper_1503_08718_amd import warmstart as ws

    n, S = 16, 5
    g = torch.Generator().manual_seed(4)
    phases = torch.randint(0, 3, (S, n ** 3), generator=g, dtype=torch.uint8).cuda()
    feats = (torch.rand((S, 3, 6), generator=g) - 0.5).cuda()
    targets = (torch.rand((S, n ** 3), generator=g) * 0.2).cuda()
    data = (phases, feats, targets)
    quiet = lambda *a, **k: None  # noqa: E731
    a = ws.Net(n=n, batch=2, seed=5)
    ws.train(a, data, iters=6, seed=9, log=quiet)
    b = ws.Net(n=n, batch=2, seed=5)
    ws.train(b, data, iters=3, seed=9, log=quiet, horizon=6)
    path = str(tmp_path / "ckpt.pt")
    b.save(path)
    c = ws.Net.from_file(path, batch=2)
    assert c.t == 3 and c.rng_state is not None
    ws.train(c, data, iters=6, seed=9, log=quiet)
    torch.cuda.synchronize()
    for name, _, _, _ in ws.LAYERS:
        assert torch.equal(a.w32[name], c.w32[name]), name
        assert torch.equal(a.b32[name], c.b32[name]), name
        assert torch.equal(a.vw[name], c.vw[name]), name


def test_training_over_shape_groups(env):
    """Training data of two cell shapes (a 16^3 group and an uneven
    (z, y, x) = 8 x 16 x 24 group): every batch comes from one group, the
    network switches grids between iterations, and the run is deterministic
    -- two fresh networks trained alike end with identical weights; the
    grouped evaluation is finite."""
    L, torch = env
    from paper_1503_08718_amd import warmstart as ws

    g = torch.Generator().manual_seed(8)
    data = []
    for shape, S in (((16, 16, 16), 3), ((8, 16, 24), 4)):
        nv = shape[0] * shape[1] * shape[2]
        data.append((shape, torch.randint(0, 3, (S, nv), generator=g, dtype=torch.uint8).cuda(),
                     (torch.rand((S, 3, 6), generator=g) - 0.5).cuda(),
                     (torch.rand((S, nv), generator=g) * 0.2).cuda()))
    quiet = lambda *a, **k: None  # noqa: E731
    nets = []
    for _ in range(2):
        net = ws.Net(n=16, batch=2, seed=5)
        ws.train(net, data, iters=8, seed=3, log=quiet)
        nets.append(net)
    torch.cuda.synchronize()
    for name, _, _, _ in ws.LAYERS:
        assert torch.equal(nets[0].w32[name], nets[1].w32[name]), name
    loss = ws.evaluate(nets[0], data)
    assert np.isfinite(loss) and loss > 0
    with pytest.raises(ValueError):
        ws.train(ws.Net(n=16, batch=4, seed=5), data, iters=1, log=quiet)  # a group smaller than the batch

