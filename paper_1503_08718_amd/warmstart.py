"""Learned warm start for the lattice Boltzmann solver.

A 3-D convolutional encoder-decoder (four resolution levels, skip additions,
~1.3 M parameters) maps a voxel medium -- per voxel the six conductivity-
tensor entries of its phase and the coordinate along the gradient axis -- to
the steady temperature's deviation from the linear wall-to-wall profile.  The
solver then starts from that field (with the matching non-equilibrium flux
part) instead of from zero; it still iterates to its own stop rule, so the
network only changes how many steps that takes, never the answer.

Every layer -- BF16 implicit-GEMM convolutions on the matrix cores with FP32
accumulation, their input and weight gradients, pooling, upsampling, the loss
and Adam -- runs in the HIP library (include/mrtlbm_nn.h); this module only
allocates buffers with torch, orders the calls and keeps the training loop.

Media are canonicalised so that the gradient runs along x: a solve along z
is the x-solve of the medium with x and z exchanged (the lattice is exactly
symmetric under axis permutations).  The x axis is zero-padded (walls), y and
z wrap (periodic cell sides).
"""

from __future__ import annotations

import ctypes
import os
import time

import numpy as np
import torch

from . import _lib
from ._lib import check, load

CIRC = 0b110  # y and z periodic, x walls
SCALE = 10.0  # target = SCALE * (T - T_lin)
MARGIN = 0.05  # a start field outside [T_cold - MARGIN, T_hot + MARGIN] is rejected

# (name, cin, cout, relu)
LAYERS = [
    ("c00", 8, 16, True), ("c01", 16, 16, True),
    ("c10", 16, 32, True), ("c11", 32, 32, True),
    ("c20", 32, 64, True), ("c21", 64, 64, True),
    ("c30", 64, 128, True), ("c31", 128, 128, True),
    ("c22", 128, 64, True), ("c23", 64, 64, True),
    ("c12", 64, 32, True), ("c13", 32, 32, True),
    ("c02", 32, 16, True), ("c03", 16, 16, True),
    ("c04", 16, 16, False),
]


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def canonical_media(m):
    """(x-solve medium, z-solve medium) of a cell, both with the gradient along x."""
    return m, m.permuted((2, 1, 0))


def feature_table(k6: np.ndarray, spacing=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Per-phase input features: the tensor entries, mapped to a grid whose
    voxels are spacing (x, y, z) times the medium's, over the largest
    eigenvalue (mrtlbm_nn_feature_table)."""
    k = np.ascontiguousarray(k6, dtype=np.float64)
    sp = np.ascontiguousarray(spacing, dtype=np.float64)
    out = np.empty((k.shape[0], 6), np.float32)
    dp, fp = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)
    check(load().mrtlbm_nn_feature_table(k.ctypes.data_as(dp), k.shape[0], sp.ctypes.data_as(dp),
                                         out.ctypes.data_as(fp)))
    return out


class Net:
    def __init__(self, n: int = 64, batch: int = 4, seed: int = 0, device="cuda:0"):
        L = load()
        self.L = L
        self.dev = torch.device(device)
        self.n = n  # training grid n^3
        self.grid = (n, n, n)  # (z, y, x) extents of the level-0 activations
        self.batch = batch
        self.stream = torch.cuda.current_stream(self.dev).cuda_stream
        rng = np.random.default_rng(seed)
        self.w32, self.b32, self.wbf, self.gw, self.gb, self.mw, self.vw, self.mb, self.vb = ({} for _ in range(9))
        for name, cin, cout, relu in LAYERS:
            kpad = L.mrtlbm_nn_kpad(cin)
            w = np.zeros((cout, kpad), np.float32)
            std = np.sqrt(2.0 / (27 * cin)) if relu else np.sqrt(1.0 / (27 * cin))
            if name == "c04":
                std *= 0.1  # start close to the linear profile
            w[:, :27 * cin] = rng.standard_normal((cout, 27 * cin)).astype(np.float32) * std
            self.w32[name] = torch.from_numpy(w).to(self.dev)
            self.b32[name] = torch.zeros(cout, dtype=torch.float32, device=self.dev)
            self.wbf[name] = torch.empty((cout, kpad), dtype=torch.bfloat16, device=self.dev)
            check(L.mrtlbm_nn_to_bf16(_p(self.w32[name]), w.size, _p(self.wbf[name]), self.stream))
            self.gw[name] = torch.zeros_like(self.w32[name])
            self.gb[name] = torch.zeros_like(self.b32[name])
            for d, ref in ((self.mw, self.w32), (self.vw, self.w32), (self.mb, self.b32), (self.vb, self.b32)):
                d[name] = torch.zeros_like(ref[name])
        self.t = 0
        self.rng_state = None  # batch-order generator state of train(), kept in checkpoints
        self._store = None
        self._alloc(batch)

    # -- buffers -------------------------------------------------------------
    _ACTS = (("x", 0, 8), ("a00", 0, 16), ("e0", 0, 16), ("p1", 1, 16), ("a10", 1, 32), ("e1", 1, 32),
             ("p2", 2, 32), ("a20", 2, 64), ("e2", 2, 64), ("p3", 3, 64), ("a30", 3, 128),
             ("e3", 3, 128), ("u2", 2, 128), ("b2", 2, 64), ("s2", 2, 64), ("d2", 2, 64),
             ("u1", 1, 64), ("b1", 1, 32), ("s1", 1, 32), ("d1", 1, 32), ("u0", 0, 32),
             ("b0", 0, 16), ("s0", 0, 16), ("d0", 0, 16), ("dout", 0, 16))

    def _alloc(self, batch):
        """Activation, gradient and scratch buffers for the current grid.
        Storage is kept between grids and only grown (the tensors used by
        the layers are views of the first voxels of it), so that training
        over cells of several shapes does not reallocate every iteration."""
        (d0, h0, w0), dev, bf = self.grid, self.dev, torch.bfloat16
        if batch != self.batch:
            self._store = None
        self.batch = batch
        vox = [batch * (d0 >> lv) * (h0 >> lv) * (w0 >> lv) for lv in range(4)]
        ws = 0
        for _, cin, cout, _ in LAYERS:
            for lv in range(4):
                ws = max(ws, self.L.mrtlbm_nn_wgrad_scratch_bytes(batch, d0 >> lv, h0 >> lv, w0 >> lv, cin, cout))
        st = getattr(self, "_store", None)
        if st is None or st["vox"] < vox[0] or st["ws"] < ws:
            cap = max(vox[0], st["vox"] if st else 0)
            capv = [cap >> (3 * lv) for lv in range(4)]  # extents are multiples of 8: exact
            wsb = max(ws, st["ws"] if st else 0)
            st = {"vox": cap, "ws": wsb,
                  # forward activations (channels-last, flattened voxels)
                  "act": {k: torch.empty((capv[lv], c), dtype=bf, device=dev) for k, lv, c in self._ACTS},
                  # gradient buffers, one per activation shape class
                  "grad": {k: torch.empty((capv[lv], c), dtype=bf, device=dev) for k, lv, c in self._ACTS},
                  "tmp": {lv: torch.empty((capv[lv], 128), dtype=bf, device=dev) for lv in range(4)},
                  "out": torch.empty((cap, 16), dtype=torch.float32, device=dev),
                  "target": torch.empty(cap, dtype=torch.float32, device=dev),
                  "wscratch": torch.empty(wsb // 4 + 1, dtype=torch.float32, device=dev)}
            self._store = st
        lvl = {k: lv for k, lv, _ in self._ACTS}
        self.act = {k: t[:vox[lvl[k]]] for k, t in st["act"].items()}
        self.grad = {k: t[:vox[lvl[k]]] for k, t in st["grad"].items()}
        self.tmp = {lv: t[:vox[lv]] for lv, t in st["tmp"].items()}
        self.out = st["out"][:vox[0]]
        self.target = st["target"][:vox[0]]
        self.wscratch = st["wscratch"]
        if not hasattr(self, "loss"):
            self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
            self.mse_scratch = torch.empty(1024, dtype=torch.float32, device=dev)
            wt = max(cin * self.L.mrtlbm_nn_kpad(cout) for _, cin, cout, _ in LAYERS)
            self.wt = torch.empty(wt, dtype=bf, device=dev)

    def set_grid(self, d: int, h: int, w: int):
        """Run on a (d, h, w) = (z, y, x) grid instead of the training n^3
        (the network is convolutional throughout; three 2x poolings need
        extents that are multiples of 8)."""
        if min(d, h, w) < 8 or (d | h | w) & 7:
            raise ValueError(f"grid {d}x{h}x{w}: extents must be multiples of 8")
        if (d, h, w) != self.grid:
            self.grid = (d, h, w)
            self._alloc(self.batch)

    # -- layer calls -------------------------------------------------------------
    def _dims(self, lv):
        d, h, w = self.grid
        return self.batch, d >> lv, h >> lv, w >> lv

    def _conv(self, name, src, dst, lv, out_f32=None):
        _, cin, cout, relu = next(l for l in LAYERS if l[0] == name)
        b, d, h, w = self._dims(lv)
        check(self.L.mrtlbm_nn_conv3d_fwd(_p(src), b, d, h, w, cin, _p(self.wbf[name]), _p(self.b32[name]), cout,
                                          CIRC, int(relu), _p(dst) if out_f32 is None else None,
                                          _p(out_f32), self.stream))

    def _pool(self, src, dst, lv_fine, c):
        b, d, h, w = self._dims(lv_fine)
        check(self.L.mrtlbm_nn_pool2(1, _p(src), b, d, h, w, c, _p(dst), self.stream))

    def _up(self, src, dst, lv_coarse, c):
        b, d, h, w = self._dims(lv_coarse)
        check(self.L.mrtlbm_nn_up2(1, _p(src), b, d, h, w, c, _p(dst), self.stream))

    def _add(self, a, b, out):
        check(self.L.mrtlbm_nn_add(_p(a), _p(b), _p(out), a.numel(), self.stream))

    def forward(self):
        A = self.act
        self._conv("c00", A["x"], A["a00"], 0)
        self._conv("c01", A["a00"], A["e0"], 0)
        self._pool(A["e0"], A["p1"], 0, 16)
        self._conv("c10", A["p1"], A["a10"], 1)
        self._conv("c11", A["a10"], A["e1"], 1)
        self._pool(A["e1"], A["p2"], 1, 32)
        self._conv("c20", A["p2"], A["a20"], 2)
        self._conv("c21", A["a20"], A["e2"], 2)
        self._pool(A["e2"], A["p3"], 2, 64)
        self._conv("c30", A["p3"], A["a30"], 3)
        self._conv("c31", A["a30"], A["e3"], 3)
        self._up(A["e3"], A["u2"], 3, 128)
        self._conv("c22", A["u2"], A["b2"], 2)
        self._add(A["b2"], A["e2"], A["s2"])
        self._conv("c23", A["s2"], A["d2"], 2)
        self._up(A["d2"], A["u1"], 2, 64)
        self._conv("c12", A["u1"], A["b1"], 1)
        self._add(A["b1"], A["e1"], A["s1"])
        self._conv("c13", A["s1"], A["d1"], 1)
        self._up(A["d1"], A["u0"], 1, 32)
        self._conv("c02", A["u0"], A["b0"], 0)
        self._add(A["b0"], A["e0"], A["s0"])
        self._conv("c03", A["s0"], A["d0"], 0)
        self._conv("c04", A["d0"], None, 0, out_f32=self.out)
        return self.out

    def _wgrad(self, name, x, dy, lv):
        _, cin, cout, _ = next(l for l in LAYERS if l[0] == name)
        b, d, h, w = self._dims(lv)
        check(self.L.mrtlbm_nn_conv3d_wgrad(_p(x), _p(dy), b, d, h, w, cin, cout, CIRC, _p(self.wscratch),
                                            _p(self.gw[name]), _p(self.gb[name]), self.stream))

    def _dgrad(self, name, dy, dx, lv):
        _, cin, cout, _ = next(l for l in LAYERS if l[0] == name)
        b, d, h, w = self._dims(lv)
        check(self.L.mrtlbm_nn_conv3d_dgrad(_p(dy), b, d, h, w, cin, _p(self.wbf[name]), cout, CIRC, _p(self.wt),
                                            _p(dx), self.stream))

    def _relu_bwd(self, y, dy, dx):
        check(self.L.mrtlbm_nn_relu_bwd(_p(y), _p(dy), _p(dx), y.numel(), self.stream))

    def _block_bwd(self, name, x, y, dy, lv, dx):
        """Backward of y = relu(conv(x)): weight grads, and dx if wanted."""
        t = self.tmp[lv].view(-1)[: y.numel()].view(y.shape)
        self._relu_bwd(y, dy, t)
        self._wgrad(name, x, t, lv)
        if dx is not None:
            self._dgrad(name, t, dx, lv)

    def backward(self):
        A, G = self.act, self.grad
        # head (no activation): dout holds dL/d(out) in BF16
        self._wgrad("c04", A["d0"], A["dout"], 0)
        self._dgrad("c04", A["dout"], G["d0"], 0)
        self._block_bwd("c03", A["s0"], A["d0"], G["d0"], 0, G["s0"])
        self._block_bwd("c02", A["u0"], A["b0"], G["s0"], 0, G["u0"])
        b, d, h, w = self._dims(1)
        check(self.L.mrtlbm_nn_up2(0, _p(G["u0"]), b, d, h, w, 32, _p(G["d1"]), self.stream))
        self._block_bwd("c13", A["s1"], A["d1"], G["d1"], 1, G["s1"])
        self._block_bwd("c12", A["u1"], A["b1"], G["s1"], 1, G["u1"])
        b, d, h, w = self._dims(2)
        check(self.L.mrtlbm_nn_up2(0, _p(G["u1"]), b, d, h, w, 64, _p(G["d2"]), self.stream))
        self._block_bwd("c23", A["s2"], A["d2"], G["d2"], 2, G["s2"])
        self._block_bwd("c22", A["u2"], A["b2"], G["s2"], 2, G["u2"])
        b, d, h, w = self._dims(3)
        check(self.L.mrtlbm_nn_up2(0, _p(G["u2"]), b, d, h, w, 128, _p(G["e3"]), self.stream))
        self._block_bwd("c31", A["a30"], A["e3"], G["e3"], 3, G["a30"])
        self._block_bwd("c30", A["p3"], A["a30"], G["a30"], 3, G["p3"])
        # e2 receives the pooled path and the skip from s2
        b, d, h, w = self._dims(2)
        check(self.L.mrtlbm_nn_pool2(0, _p(G["p3"]), b, d, h, w, 64, _p(G["e2"]), self.stream))
        self._add(G["e2"], G["s2"], G["e2"])
        self._block_bwd("c21", A["a20"], A["e2"], G["e2"], 2, G["a20"])
        self._block_bwd("c20", A["p2"], A["a20"], G["a20"], 2, G["p2"])
        b, d, h, w = self._dims(1)
        check(self.L.mrtlbm_nn_pool2(0, _p(G["p2"]), b, d, h, w, 32, _p(G["e1"]), self.stream))
        self._add(G["e1"], G["s1"], G["e1"])
        self._block_bwd("c11", A["a10"], A["e1"], G["e1"], 1, G["a10"])
        self._block_bwd("c10", A["p1"], A["a10"], G["a10"], 1, G["p1"])
        b, d, h, w = self._dims(0)
        check(self.L.mrtlbm_nn_pool2(0, _p(G["p1"]), b, d, h, w, 16, _p(G["e0"]), self.stream))
        self._add(G["e0"], G["s0"], G["e0"])
        self._block_bwd("c01", A["a00"], A["e0"], G["e0"], 0, G["a00"])
        self._block_bwd("c00", A["x"], A["a00"], G["a00"], 0, None)

    def loss_and_grad(self):
        nvox = self.target.numel()
        check(self.L.mrtlbm_nn_mse(_p(self.out), 16, _p(self.target), nvox, _p(self.act["dout"]),
                                   _p(self.mse_scratch), _p(self.loss), self.stream))

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        for name, _, _, _ in LAYERS:
            check(self.L.mrtlbm_nn_adam(_p(self.w32[name]), _p(self.gw[name]), _p(self.mw[name]), _p(self.vw[name]),
                                        self.w32[name].numel(), lr, b1, b2, eps, self.t, _p(self.wbf[name]),
                                        self.stream))
            check(self.L.mrtlbm_nn_adam(_p(self.b32[name]), _p(self.gb[name]), _p(self.mb[name]), _p(self.vb[name]),
                                        self.b32[name].numel(), lr, b1, b2, eps, self.t, None, self.stream))

    def set_input(self, b: int, phase_dev: torch.Tensor, feat_dev: torch.Tensor, shape=None):
        """Features of sample b of the batch from a cell of shape (z, y, x)
        (default the training n^3), which becomes the network's grid."""
        d, h, w = shape or (self.n,) * 3
        self.set_grid(d, h, w)
        nv = d * h * w
        dst = self.act["x"][b * nv:(b + 1) * nv]
        check(self.L.mrtlbm_nn_features(_p(phase_dev), d, h, w, _p(feat_dev), _p(dst), self.stream))

    # -- persistence -----------------------------------------------------------
    def state_dict(self, optimizer: bool = True):
        """FP32 master weights and biases, and with optimizer (a training
        checkpoint) everything training needs to continue bit for bit: Adam's
        moments and step count and the state of the batch-order generator
        (set by train())."""
        cpu = lambda d: {k: v.cpu() for k, v in d.items()}  # noqa: E731
        sd = {"w": cpu(self.w32), "b": cpu(self.b32), "n": self.n}
        if optimizer:
            sd["t"] = self.t
            sd["adam"] = {"mw": cpu(self.mw), "vw": cpu(self.vw), "mb": cpu(self.mb), "vb": cpu(self.vb)}
            if self.rng_state is not None:
                sd["rng"] = self.rng_state
        return sd

    def load_state_dict(self, sd):
        for name, _, _, _ in LAYERS:
            self.w32[name].copy_(sd["w"][name].to(self.dev))
            self.b32[name].copy_(sd["b"][name].to(self.dev))
            check(self.L.mrtlbm_nn_to_bf16(_p(self.w32[name]), self.w32[name].numel(), _p(self.wbf[name]),
                                           self.stream))
            if "adam" in sd:
                for key, d in (("mw", self.mw), ("vw", self.vw), ("mb", self.mb), ("vb", self.vb)):
                    d[name].copy_(sd["adam"][key][name].to(self.dev))
        self.t = int(sd.get("t", 0))
        self.rng_state = sd.get("rng")

    def save(self, path, optimizer: bool = True):
        torch.save(self.state_dict(optimizer), path)

    @classmethod
    def from_file(cls, path, batch=1, device="cuda:0"):
        sd = torch.load(path, map_location="cpu", weights_only=True)
        net = cls(n=int(sd["n"]), batch=batch, device=device)
        net.load_state_dict(sd)
        return net


# ---------------------------------------------------------------------------
# data, training, inference
# ---------------------------------------------------------------------------


def _gen_braid(spec):
    import workloads

    # one thread per worker process: the pool already spreads the cells
    m = workloads.braid(spec["nx"], spec["ny"], spec["nz"], spec["gamma"], spec["v"], workers=1)
    return m.phase, m.k


def generate_media(specs, workers: int = 8):
    """Voxelise braided cells on the CPU, in worker processes.  Call it before
    the process first touches the GPU: the workers are forked copies."""
    import workloads

    if workers <= 1:
        return [workloads.braid(s["nx"], s["ny"], s["nz"], s["gamma"], s["v"]) for s in specs]
    from concurrent.futures import ProcessPoolExecutor

    with ProcessPoolExecutor(workers) as ex:
        out = list(ex.map(_gen_braid, specs, chunksize=4))
    return [workloads.Medium(p, k) for p, k in out]


def linear_start(shape, device, dtype=torch.float32):
    """T_lin = 1 - (x + 1/2) / nx on a (nz, ny, nx) grid (walls 1 -> 0)."""
    nx = shape[2]
    x = (torch.arange(nx, dtype=torch.float64) + 0.5) / nx
    return (1.0 - x).to(dtype).view(1, 1, nx).expand(*shape).contiguous().to(device)


def solve_fields(media, tol=1e-4, check_every=1000, max_steps=5_000_000, start="linear", net=None, batch=True,
                 precision="f32", storage="populations", keep_fields=True, tune=False, grid="isotropic"):
    """Steady x-gradient fields of canonical media (periodic sides).

    start: "zero", "linear" or "learned" (needs net; grid: the inference grid
    of predict_start); tune: pick the batched step's shape for this set first
    (batch only).  Returns (temperature tensors or None, results, setup
    seconds, number of rejected predictions)."""
    from .solver import Medium, batch_autotune, batch_solve

    cells = []
    t0 = time.perf_counter()
    fallbacks = 0
    for m in media:
        g = Medium(m.phase, m.k, precision=precision, storage=storage)
        g.set_bc(0, 1.0, 0.0, ("periodic",) * 3)
        cells.append(g)
    if batch and tune:
        batch_autotune(cells)
    for m, g in zip(media, cells):
        if start == "zero":
            g.init()
        elif start == "linear":
            g.init(linear_start(g.shape, g.device), flux=True)
        else:
            T0, bad = predict_start(net, m, g, grid)
            if bad:
                fallbacks += 1
                g.init()
            else:
                g.init(T0.to(g.dtype), flux=True)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    if batch:
        res, _ = batch_solve(cells, tol=tol, kind="keff", max_steps=max_steps, check_every=check_every)
    else:
        res = [g.solve(tol, "keff", max_steps, check_every=check_every) for g in cells]
    temps = [g.temperature() for g in cells] if keep_fields else None
    return temps, res, setup, fallbacks


def inference_grid(shape, n: int) -> tuple[int, int, int]:
    """(z, y, x) grid the network runs on for a cell of shape (nz, ny, nx):
    one common coarsening factor, max(shape) / n, on every axis (so that the
    voxels stay as nearly cubic as extents that are multiples of 8 allow and
    the largest extent is the training size n), each extent rounded to a
    multiple of 8, at least 8."""
    f = max(shape) / n
    return tuple(max(8, int(round(e / f / 8.0)) * 8) for e in shape)


def predict_start(net: Net, m, g, grid: str = "isotropic") -> tuple[torch.Tensor, int]:
    """Network start field for medium m on solver medium g (x gradient).
    The cell is resampled to the inference grid (a box average of the
    per-voxel features, with the tensors mapped to the new voxel spacing),
    and the prediction is interpolated back to the cell's own grid.
    grid: "isotropic" (inference_grid: one coarsening factor on all axes) or
    "cube" (the training n^3 whatever the cell's shape).
    Returns (T0, number of rejected values)."""
    L = net.L
    nz, ny, nx = m.phase.shape
    if grid == "isotropic":
        dc, hc, wc = inference_grid((nz, ny, nx), net.n)
    elif grid == "cube":
        dc = hc = wc = net.n
    else:
        raise ValueError(f"unknown inference grid {grid!r}")
    net.set_grid(dc, hc, wc)
    s = net.stream
    feat = torch.from_numpy(feature_table(m.k, (nx / wc, ny / hc, nz / dc))).to(net.dev)
    check(L.mrtlbm_nn_features_resampled(_p(g.phase), nz, ny, nx, _p(feat), dc, hc, wc, _p(net.act["x"]), s))
    net.forward()
    T0 = torch.empty((nz, ny, nx), dtype=torch.float32, device=net.dev)
    bad_scratch = torch.empty(2048, dtype=torch.int32, device=net.dev)
    bad = ctypes.c_longlong()
    check(L.mrtlbm_nn_to_temperature(_p(net.out), 16, dc, hc, wc, nz, ny, nx, SCALE, MARGIN, _p(T0),
                                     _p(bad_scratch), ctypes.byref(bad), s))
    return T0, bad.value


def make_dataset(media, tol=1e-5, chunk=128, log=print):
    """Steady fields of braided cells (already voxelised); each cell gives two
    samples (x- and z-solve, canonicalised).  Returns the samples grouped by
    shape, as a list of (shape (z, y, x), phases uint8 [S, voxels], feature
    tables [S, nphase, 6], targets [S, voxels]) on the device, and
    statistics."""
    canon = [mm for m in media for mm in canonical_media(m)]
    groups = {}
    steps = []
    t0 = time.perf_counter()
    for c0 in range(0, len(canon), chunk):
        part = canon[c0:c0 + chunk]
        temps, res, _, _ = solve_fields(part, tol=tol, start="linear", storage="moments")
        for m, T, r in zip(part, temps, res):
            d, h, w = m.phase.shape
            tgt = torch.empty(d * h * w, dtype=torch.float32, device=T.device)
            check(load().mrtlbm_nn_target(_p(T), d, h, w, SCALE, _p(tgt), torch.cuda.current_stream().cuda_stream))
            gr = groups.setdefault((d, h, w), ([], [], []))
            gr[0].append(torch.from_numpy(m.phase.reshape(-1)).to(T.device))
            gr[1].append(torch.from_numpy(feature_table(m.k)).to(T.device))
            gr[2].append(tgt)
            steps.append(r["steps"])
        log(f"dataset: {min(c0 + chunk, len(canon))}/{len(canon)} fields, {time.perf_counter() - t0:.1f} s")
    data = [(shape, torch.stack(g[0]), torch.stack(g[1]), torch.stack(g[2])) for shape, g in sorted(groups.items())]
    return data, dict(seconds=time.perf_counter() - t0, mean_steps=float(np.mean(steps)),
                      shapes=len(data), samples=len(steps))


def _groups(net: Net, data):
    """Dataset as shape groups: a (phases, feats, targets) tuple of cubic
    samples on the training grid is one group."""
    if isinstance(data, tuple):
        return [((net.n,) * 3,) + tuple(data)]
    return list(data)


# resolution level of each convolution (grid n >> level)
LEVEL = {"c00": 0, "c01": 0, "c10": 1, "c11": 1, "c20": 2, "c21": 2, "c30": 3, "c31": 3, "c22": 2, "c23": 2,
         "c12": 1, "c13": 1, "c02": 0, "c03": 0, "c04": 0}


def layer_flops(net: Net) -> dict:
    """Algorithmic FLOPs of each convolution's forward pass on the current
    grid: 2 * voxels * 27 * C_in * C_out (the K padding of the MFMA tiles not
    counted)."""
    d, h, w = net.grid
    return {name: 2.0 * net.batch * (d >> LEVEL[name]) * (h >> LEVEL[name]) * (w >> LEVEL[name]) * 27 * cin * cout
            for name, cin, cout, _ in LAYERS}


def forward_flops(net: Net) -> float:
    """Matrix-core FLOPs of one forward pass (inference)."""
    return sum(layer_flops(net).values())


def iteration_flops(net: Net) -> float:
    """Matrix-core FLOPs of one training iteration (forward, input and weight
    gradients; the first layer has no input gradient)."""
    return sum(f * (2 if name == "c00" else 3) for name, f in layer_flops(net).items())


def train(net: Net, data, iters=2000, lr=1e-3, seed=0, log=print, log_every=100, horizon=None):
    """Adam iterations net.t + 1 .. iters, the learning rate decaying from lr
    to lr / 10 over `horizon` iterations (default iters).  A batch is drawn
    from one shape group (chosen with probability proportional to its size
    when there are several), without replacement within it.  A network
    loaded from a checkpoint continues where it stopped, with the same
    batches and learning rates when given the same horizon."""
    horizon = horizon or iters
    groups = _groups(net, data)
    sizes = np.array([g[1].shape[0] for g in groups], dtype=np.float64)
    if any(sz < net.batch for sz in sizes):
        raise ValueError(f"a shape group has fewer samples than the batch ({net.batch})")
    rng = np.random.default_rng(seed)
    if net.rng_state is not None:
        rng.bit_generator.state = net.rng_state
    losses = []
    t0 = time.perf_counter()
    first = net.t + 1
    flops = 0.0
    for it in range(first, iters + 1):
        gi = 0 if len(groups) == 1 else int(rng.choice(len(groups), p=sizes / sizes.sum()))
        shape, phases, feats, targets = groups[gi]
        idx = rng.choice(phases.shape[0], size=net.batch, replace=False)
        net.rng_state = rng.bit_generator.state
        nv = shape[0] * shape[1] * shape[2]
        for b, i in enumerate(idx):
            net.set_input(b, phases[i], feats[i], shape)
            net.target[b * nv:(b + 1) * nv].copy_(targets[i])
        net.forward()
        net.loss_and_grad()
        net.backward()
        cur_lr = lr * (0.1 ** (it / horizon))  # exponential decay to lr / 10
        net.adam(lr=cur_lr)
        flops += iteration_flops(net)
        if it % log_every == 0 or it == iters:
            loss = float(net.loss.item())
            losses.append((it, loss))
            dt = time.perf_counter() - t0
            log(f"train it {it}: loss {loss:.3e}  ({dt:.1f} s, {flops / dt / 1e12:.2f} TFLOP/s)")
    return losses


def evaluate(net: Net, data) -> float:
    """Mean loss over the batches of every shape group, in order; a group's
    last batch is filled up with its first samples again."""
    tot, nb = 0.0, 0
    for shape, phases, feats, targets in _groups(net, data):
        nv = shape[0] * shape[1] * shape[2]
        S = phases.shape[0]
        for i0 in range(0, S, net.batch):
            for b in range(net.batch):
                i = (i0 + b) % S
                net.set_input(b, phases[i], feats[i], shape)
                net.target[b * nv:(b + 1) * nv].copy_(targets[i])
            net.forward()
            net.loss_and_grad()
            tot += float(net.loss.item())
            nb += 1
    return tot / max(1, nb)


def bench(args) -> dict:
    """Held-out cells solved from zero, linear and learned starts (same stop
    rule, FP32, periodic sides, x and z solves of every cell in one batched
    run per start), each against an FP64 reference."""
    import workloads

    specs = workloads.warmstart_cells(args.seed if args.seed != 1503 else 8719, args.cells, args.n)
    t_gen = time.perf_counter()
    media = generate_media(specs)
    canon = [mm for m in media for mm in canonical_media(m)]
    t_gen = time.perf_counter() - t_gen
    net = Net.from_file(args.model, batch=1)
    out = {"mode": "warmstart", "cells": len(media), "size": args.n, "tol": args.tol, "solves_per_cell": 2,
           "storage": args.storage, "seconds_geometry": round(t_gen, 2)}
    # reference: FP64, tolerance 100x tighter, from the zero start (or the
    # linear profile); the network never seeds the solve that judges it
    ref_start = getattr(args, "ref_start", "zero")
    if getattr(args, "ref_in", ""):
        import json

        with open(args.ref_in) as fh:
            saved = json.load(fh)
        assert saved["mode"] == "warmstart" and saved["size"] == args.n and saved["cells"] == len(media), \
            "reference file of another workload"
        ref = saved["keff"]
        out["reference"] = {k: saved[k] for k in ("precision", "tol", "start", "all_converged", "seconds")}
        out["reference"]["file"] = os.path.basename(args.ref_in)
    else:
        t0 = time.perf_counter()
        _, rres, _, _ = solve_fields(canon, tol=args.tol / 100, start=ref_start, net=net, batch=True,
                                     precision="f64", max_steps=20_000_000, storage=args.storage, keep_fields=False)
        ref = [r["keff"] for r in rres]
        out["reference"] = {"precision": "f64", "tol": args.tol / 100, "start": ref_start,
                            "all_converged": all(r["converged"] for r in rres),
                            "seconds": round(time.perf_counter() - t0, 1), "keff": ref,
                            "steps": [r["steps"] for r in rres]}
        if getattr(args, "ref_out", ""):
            import json

            with open(args.ref_out, "w") as fh:
                json.dump(dict(out["reference"], mode="warmstart", size=args.n, cells=len(media)), fh)
        print("warmstart reference done", flush=True)
    starts = [] if getattr(args, "ref_only", False) else \
        [x for x in (getattr(args, "start", "") or "zero,linear,learned").split(",") if x]
    for start in starts:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, res, setup, fb = solve_fields(canon, tol=args.tol, start=start, net=net, batch=True,
                                         storage=args.storage, keep_fields=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ks = [r["keff"] for r in res]
        rec = {"steps_mean": float(np.mean([r["steps"] for r in res])),
               "steps": [r["steps"] for r in res], "seconds": round(wall, 2), "setup_seconds": round(setup, 2),
               "cells_per_hour": round(len(media) / ((wall + t_gen) / 3600.0), 1), "fallbacks": fb,
               "all_converged": all(r["converged"] for r in res)}
        errs = [abs(a - b) / abs(b) for a, b in zip(ks, ref)]
        rec["max_rel_err_vs_reference"] = float(max(errs))
        rec["mean_rel_err_vs_reference"] = float(np.mean(errs))
        rec["rel_err_vs_reference"] = [float(f"{e:.3g}") for e in errs]  # every solve, (x, z) per cell
        out[start] = rec
        print(f"warmstart {start}: mean steps {rec['steps_mean']:.0f}, {wall:.1f} s", flush=True)
    return out


def main():
    import argparse
    import json

    p = argparse.ArgumentParser(description="generate data, train and save the warm-start network")
    p.add_argument("--cells", type=int, default=1000, help="cubic training cells (two fields each: x and z solves)")
    p.add_argument("--mixed-cells", type=int, default=1000,
                   help="training cells whose extents are drawn per axis from --mixed-sizes")
    p.add_argument("--mixed-sizes", default="32,40,48,64")
    p.add_argument("--tol", type=float, default=1e-5, help="k_eff tolerance of the target fields")
    p.add_argument("--val-cells", type=int, default=16)
    p.add_argument("--size", type=int, default=64)
    p.add_argument("--iters", type=int, default=40000)
    p.add_argument("--batch", type=int, default=4)
    p.add_argument("--lr", type=float, default=5e-4)
    p.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "warmstart_model.pt"),
                   help="the trained weights (what inference loads)")
    p.add_argument("--checkpoint", default="", help="also write a full training checkpoint (Adam state, batch order)")
    p.add_argument("--workers", type=int, default=8)
    a = p.parse_args()
    import workloads

    # voxelise every cell before the GPU is touched (forked workers)
    sizes = tuple(int(v) for v in a.mixed_sizes.split(",") if v)
    train_specs = workloads.warmstart_cells(8718, a.cells, a.size)
    val_specs = workloads.warmstart_cells(8720, a.val_cells, a.size)
    if a.mixed_cells:
        train_specs += workloads.warmstart_cells_mixed(8721, a.mixed_cells, sizes)
        val_specs += workloads.warmstart_cells_mixed(8722, a.val_cells, sizes)
    train_media = generate_media(train_specs, a.workers)
    val_media = generate_media(val_specs, a.workers)
    _lib.load()
    _lib.set_progress(lambda msg: print(msg, flush=True), 30.0)
    data, st = make_dataset(train_media, tol=a.tol)
    val, _ = make_dataset(val_media, tol=a.tol)
    net = Net(n=a.size, batch=a.batch, seed=0)
    before = evaluate(net, val)
    t0 = time.perf_counter()
    losses = train(net, data, iters=a.iters, lr=a.lr)
    t_train = time.perf_counter() - t0
    after = evaluate(net, val)
    net.save(a.out, optimizer=False)
    if a.checkpoint:
        net.save(a.checkpoint)
    print(json.dumps({"train_samples": st["samples"], "shapes": st["shapes"], "target_tol": a.tol,
                      "cubic_cells": a.cells, "mixed_cells": a.mixed_cells, "mixed_sizes": sizes,
                      "data_seconds": round(st["seconds"], 1),
                      "data_mean_steps": st["mean_steps"], "train_seconds": round(t_train, 1),
                      "val_loss_before": before, "val_loss_after": after, "losses": losses[-5:], "out": a.out}))


if __name__ == "__main__":
    main()
