"""Learned primal-dual reconstruction driven by the library's kernels.

The unrolled scheme of Sec. 4.2.1 of Hauptmann, Kunyansky & Poimala (arXiv
2510.24687), eqs. eq:LPD_dual and eq:LPD_primal, with residual updates and one
set of weights shared by all iterations:

    q_{k+1} = q_k + Gamma(q_k, s_A A f_k, s_A y)
    f_{k+1} = f_k + Lambda(f_k, s_U A* q_{k+1}),      k = 0 .. K-1,  f_0 = q_0 = 0,

Gamma and Lambda are 3-layer 3x3 CNNs (cin -> 32 -> 32 -> 1, PReLU after the
first two layers).  s_A and s_U are fixed normalisations of the operator
outputs (chosen once from data so that every input plane has the RMS of f).
Training minimises the mean squared error of f_K against the phantom (the
empirical loss eq:emp_loss divided by the number of pixels).

Everything that computes runs in libpat.so: A, A* (pat_forward_batched /
pat_adjoint_batched), the BF16-MFMA convolutions with fused bias / PReLU /
residual, the explicit reverse sweep (input-gradient convolutions with the
PReLU backward fused into their epilogue, weight gradients, 4K operator
applications per step as the paper counts), the loss gradient (pat_axpby) and Adam.  The whole training step or
inference pass is a fixed launch sequence, captured once in a HIP graph
(torch.cuda.CUDAGraph) and replayed.  Python allocates buffers and marshals
pointers only.
"""
from __future__ import annotations

import ctypes
import math
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch

from .pat import ConvDesc, Plan, _check, load

HID = 32
_VP = ctypes.c_void_p


def _p(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def param_layout(dual_in: int = 3, primal_in: int = 2, arch: str = "cnn") -> List[Tuple[str, tuple]]:
    """Names and shapes of the flat parameter vector, in storage order.  For
    the 3-layer CNN each layer's bias is followed by its PReLU slopes (the
    PReLU backward writes both gradients as one 64-float block); ``arch =
    "unet"`` gives the U-Net layout of unet.layout per network."""
    if arch == "unet":
        from . import unet as U
        return [(net + "." + name, shape) for net, cin in (("dual", dual_in), ("primal", primal_in))
                for name, shape in U.layout(cin)]
    if arch != "cnn":
        raise ValueError("arch must be 'cnn' or 'unet'")
    out = []
    for net, cin in (("dual", dual_in), ("primal", primal_in)):
        out += [(net + ".w1", (HID, cin, 3, 3)), (net + ".b1", (HID,)), (net + ".a1", (HID,)),
                (net + ".w2", (HID, HID, 3, 3)), (net + ".b2", (HID,)), (net + ".a2", (HID,)),
                (net + ".w3", (1, HID, 3, 3)), (net + ".b3", (1,))]
    return out


def init_params(seed: int, dual_in: int = 3, primal_in: int = 2, arch: str = "cnn") -> np.ndarray:
    """Seeded initial weights: He-uniform for the hidden layers, PReLU slopes
    0.25, zero biases, and a last layer scaled down so that the untrained
    network starts close to the identity update (U-Net: unet.init_values)."""
    rng = np.random.default_rng(seed)
    parts = []
    if arch == "unet":
        from . import unet as U
        for name, shape in param_layout(dual_in, primal_in, arch):
            parts.append(U.init_values(name, shape, rng))
        return np.concatenate(parts).astype(np.float32)
    for name, shape in param_layout(dual_in, primal_in):
        size = int(np.prod(shape))
        kind = name.split(".")[1]
        if kind.startswith("w"):
            fan_in = shape[1] * 9
            bound = math.sqrt(6.0 / fan_in) * (0.1 if kind == "w3" else 1.0)
            parts.append(rng.uniform(-bound, bound, size))
        elif kind.startswith("a"):
            parts.append(np.full(size, 0.25))
        else:
            parts.append(np.zeros(size))
    return np.concatenate(parts).astype(np.float32)


def unpack(flat, dual_in: int = 3, primal_in: int = 2, arch: str = "cnn") -> Dict[str, np.ndarray]:
    out, o = {}, 0
    flat = np.asarray(flat)
    for name, shape in param_layout(dual_in, primal_in, arch):
        size = int(np.prod(shape))
        out[name] = flat[o:o + size].reshape(shape)
        o += size
    return out


class _Layer:
    """One convolution of a block: weights (views into the flat vectors) and
    its packed bf16 forward / input-gradient weights."""

    def __init__(self, lib, params, grads, offs, net, idx, cin, cout, in_planar, out_planar, dev):
        self.cin, self.cout, self.in_planar, self.out_planar = cin, cout, in_planar, out_planar
        self.w = params[offs[net + ".w%d" % idx]:][:cout * cin * 9]
        self.gw = grads[offs[net + ".w%d" % idx]:][:cout * cin * 9]
        self.b = params[offs[net + ".b%d" % idx]:][:cout]
        self.gb = grads[offs[net + ".b%d" % idx]:]  # bias grad (+ slopes grad right after it)
        self.a = params[offs[net + ".a%d" % idx]:][:cout] if not out_planar else None
        nf = lib.pat_conv_packed_size(cout, cin, int(in_planar))
        # input gradient: effective conv cout -> cin, its input is this layer's output layout
        nb = lib.pat_conv_packed_size(cin, cout, int(out_planar))
        if nf < 0 or nb < 0:
            raise ValueError("unsupported layer shape")
        self.wf = torch.empty(nf, dtype=torch.int16, device=dev)
        self.wb = torch.empty(nb, dtype=torch.int16, device=dev)

    def pack(self, lib, st):
        _check(lib.pat_conv_pack_weights(_p(self.w), self.cout, self.cin, 0, int(self.in_planar), _p(self.wf), st),
               "pat_conv_pack_weights")
        _check(lib.pat_conv_pack_weights(_p(self.w), self.cout, self.cin, 1, int(self.out_planar), _p(self.wb), st),
               "pat_conv_pack_weights")


def _desc(B, H, W, cin, cout, in_planar, out_planar, inp, out, weight, bias=None, alpha=None, pre=None,
          residual=None, scale=None, bwd_pre=None, partials=None, grad_bias_alpha=None, accumulate=0):
    d = ConvDesc()
    d.B, d.H, d.W, d.cin, d.cout = B, H, W, cin, cout
    d.in_planar, d.out_planar = int(in_planar), int(out_planar)
    for i, t in enumerate(inp):
        d.inp[i] = _p(t)
    for i, t in enumerate(out):
        d.out[i] = _p(t)
    for i, t in enumerate(residual or []):
        d.residual[i] = _p(t)
    for i in range(4):
        d.scale[i] = 1.0
    for i, s in enumerate(scale or []):
        d.scale[i] = float(s)
    d.weight, d.bias, d.alpha, d.pre = _p(weight), _p(bias), _p(alpha), _p(pre)
    d.bwd_pre, d.partials, d.grad_bias_alpha = _p(bwd_pre), _p(partials), _p(grad_bias_alpha)
    d.accumulate = int(accumulate)
    return d


class _Block:
    """A 3-layer CNN on one domain (H x W) with cin planar inputs and a
    residual 1-channel planar output; keeps its activations for K iterations."""

    def __init__(self, lib, params, grads, offs, net, cin, B, H, W, K, dev, train):
        self.lib, self.cin, self.B, self.H, self.W, self.K = lib, cin, B, H, W, K
        self.l1 = _Layer(lib, params, grads, offs, net, 1, cin, HID, True, False, dev)
        self.l2 = _Layer(lib, params, grads, offs, net, 2, HID, HID, False, False, dev)
        self.l3 = _Layer(lib, params, grads, offs, net, 3, HID, 1, False, True, dev)
        nk = K if train else 1
        shp = (nk, B, H, W, HID)
        # hidden activations and gradients are bf16 (int16 storage); the
        # pre-activations the PReLU backward needs stay FP32 (training only)
        self.act1 = torch.empty(shp, dtype=torch.int16, device=dev)
        self.act2 = torch.empty(shp, dtype=torch.int16, device=dev)
        self.pre1 = torch.empty(shp, dtype=torch.float32, device=dev) if train else None
        self.pre2 = torch.empty(shp, dtype=torch.float32, device=dev) if train else None
        if train:
            self.g1 = torch.empty((B, H, W, HID), dtype=torch.int16, device=dev)
            self.g2 = torch.empty((B, H, W, HID), dtype=torch.int16, device=dev)
            self.rows = max(1, min(H, 2048 // W))
            need = 0
            for l in (self.l1, self.l2, self.l3):
                d = _desc(B, H, W, l.cin, l.cout, l.in_planar, l.out_planar, [], [], None)
                need = max(need, lib.pat_conv_wgrad_partials(ctypes.byref(d), self.rows))
            d = _desc(B, H, W, HID, HID, False, False, [], [], None)
            need = max(need, lib.pat_conv_bwd_partials(ctypes.byref(d)))
            self.part = torch.empty(max(need, 64 * 1024), dtype=torch.float32, device=dev)
            self.nred = 512

    def layers(self):
        return (self.l1, self.l2, self.l3)

    def forward(self, k, planes, scales, state_in, state_out, st):
        lib, B, H, W = self.lib, self.B, self.H, self.W
        j = min(k, self.act1.shape[0] - 1)
        l1, l2, l3 = self.layers()
        pre1 = None if self.pre1 is None else self.pre1[j]
        pre2 = None if self.pre2 is None else self.pre2[j]
        d = _desc(B, H, W, self.cin, HID, True, False, planes, [self.act1[j]], l1.wf, l1.b, l1.a, pre1, scale=scales)
        _check(lib.pat_conv3x3(ctypes.byref(d), st), "pat_conv3x3")
        d = _desc(B, H, W, HID, HID, False, False, [self.act1[j]], [self.act2[j]], l2.wf, l2.b, l2.a, pre2)
        _check(lib.pat_conv3x3(ctypes.byref(d), st), "pat_conv3x3")
        d = _desc(B, H, W, HID, 1, False, True, [self.act2[j]], [state_out], l3.wf, l3.b, residual=[state_in])
        _check(lib.pat_conv3x3(ctypes.byref(d), st), "pat_conv3x3")

    def backward(self, k, planes, scales, g_out, g_planes, g_residual, acc, st):
        """g_out: gradient of the block output (planar).  Writes the gradients
        of the input planes: g_planes[c] = g_residual[c] + d loss / d plane_c
        (g_planes[c] None = not needed).  Weight gradients accumulate if acc."""
        lib, B, H, W = self.lib, self.B, self.H, self.W
        l1, l2, l3 = self.layers()
        npix = B * H * W
        a = int(acc)
        # layer 3 (no activation): bias, weights; its input gradient goes through
        # the PReLU of layer 2 in the same launch (bias / slope gradients of layer 2)
        _check(lib.pat_plane_sum(npix, _p(g_out), _p(self.part), self.nred, _p(l3.gb), a, st), "pat_plane_sum")
        d3 = _desc(B, H, W, HID, 1, False, True, [self.act2[k]], [], l3.wf)
        _check(lib.pat_conv3x3_wgrad(ctypes.byref(d3), _p(g_out), self.rows, _p(self.part), _p(l3.gw), a, st),
               "pat_conv3x3_wgrad")
        d = _desc(B, H, W, 1, HID, True, False, [g_out], [self.g1], l3.wb, alpha=l2.a, bwd_pre=self.pre2[k],
                  partials=self.part, grad_bias_alpha=l2.gb, accumulate=a)
        _check(lib.pat_conv3x3(ctypes.byref(d), st), "pat_conv3x3")
        # layer 2: weights; input gradient through the PReLU of layer 1
        d2 = _desc(B, H, W, HID, HID, False, False, [self.act1[k]], [], l2.wf)
        _check(lib.pat_conv3x3_wgrad(ctypes.byref(d2), _p(self.g1), self.rows, _p(self.part), _p(l2.gw), a, st),
               "pat_conv3x3_wgrad")
        d = _desc(B, H, W, HID, HID, False, False, [self.g1], [self.g2], l2.wb, alpha=l1.a, bwd_pre=self.pre1[k],
                  partials=self.part, grad_bias_alpha=l1.gb, accumulate=a)
        _check(lib.pat_conv3x3(ctypes.byref(d), st), "pat_conv3x3")
        # layer 1: weights and the gradients of the input planes
        d1 = _desc(B, H, W, self.cin, HID, True, False, planes, [], l1.wf, scale=scales)
        _check(lib.pat_conv3x3_wgrad(ctypes.byref(d1), _p(self.g2), self.rows, _p(self.part), _p(l1.gw), a, st),
               "pat_conv3x3_wgrad")
        d = _desc(B, H, W, HID, self.cin, False, True, [self.g2], g_planes, l1.wb, residual=g_residual, scale=scales)
        _check(lib.pat_conv3x3(ctypes.byref(d), st), "pat_conv3x3")


class LPD:
    """Learned primal-dual reconstructor for one geometry and batch size.

    ``plan``: an FP32 Plan (max_batch >= batch).  ``params``: flat FP32
    initial weights (init_params).  ``train``: keep the activations of all K
    iterations and allocate gradients / Adam state.  ``arch``: "cnn" (3-layer
    CNNs) or "unet" (the paper's U-Nets, unet.UNetBlock, with batch
    normalisation; ``stats``: flat running statistics of every unrolled
    iteration, unet.init_stats(iters)).
    """

    def __init__(self, plan: Plan, batch: int, iters: int = 10, params=None, seed: int = 0, train: bool = True,
                 s_A: float = 1.0, s_U: float = 1.0, arch: str = "cnn", stats=None):
        if plan.dtype != torch.float32:
            raise TypeError("the learned reconstructor runs on an FP32 plan")
        if batch > plan.max_batch:
            raise ValueError("batch exceeds the plan's max_batch")
        self.lib = load()
        self.plan, self.B, self.K, self.train_mode = plan, batch, iters, train
        dev = plan.device
        self.dev = dev
        self.arch = arch
        self.layout = param_layout(arch=arch)
        self.shapes = dict(self.layout)
        self.offs, o = {}, 0
        for name, shape in self.layout:
            self.offs[name] = o
            o += int(np.prod(shape))
        self.nparams = o
        p0 = init_params(seed, arch=arch) if params is None else np.asarray(params, dtype=np.float32)
        if p0.size != o:
            raise ValueError("expected %d parameters" % o)
        self.params = torch.tensor(p0, device=dev)
        self.grads = torch.zeros(o, dtype=torch.float32, device=dev)
        self.s_A, self.s_U = float(s_A), float(s_U)
        n, nt, m, B, K = plan.n, plan.nt, plan.m, batch, iters
        z = lambda *s: torch.zeros(s, dtype=torch.float32, device=dev)
        self.y = z(B, nt, m)
        self.target = z(B, n, n)
        self.q = z(K + 1, B, nt, m)
        self.f = z(K + 1, B, n, n)
        self.Af = z(K, B, nt, m)
        self.u = z(K, B, n, n)
        if arch == "unet":
            from . import unet as U
            slay = U.stats_layout(K)
            self.soffs, so = {}, 0
            for name, c in slay:
                self.soffs[name] = so
                so += c
            st0 = U.init_stats(K) if stats is None else np.asarray(stats, dtype=np.float32)
            if st0.size != so:
                raise ValueError("expected %d running statistics" % so)
            self.stats = torch.tensor(st0, device=dev)
            mk = lambda net, cin, H, W: U.UNetBlock(self.lib, self.params, self.grads, self.offs, self.shapes,
                                                    self.stats, self.soffs, net, cin, B, H, W, K, dev, train)
            self.dual = mk("dual", 3, nt, m)
            self.primal = mk("primal", 2, n, n)
        else:
            self.stats = None
            self.dual = _Block(self.lib, self.params, self.grads, self.offs, "dual", 3, B, nt, m, K, dev, train)
            self.primal = _Block(self.lib, self.params, self.grads, self.offs, "primal", 2, B, n, n, K, dev, train)
        if train:
            self.dq = z(B, nt, m)
            self.dq2 = z(B, nt, m)
            self.df = z(B, n, n)
            self.df2 = z(B, n, n)
            self.dAf = z(B, nt, m)
            self.du = z(B, n, n)
            self.tmp_g = z(B, nt, m)
            self.tmp_f = z(B, n, n)
            self.adam_m = torch.zeros_like(self.params)
            self.adam_v = torch.zeros_like(self.params)
            self.step_count = torch.zeros(1, dtype=torch.int32, device=dev)
            self.adam_scratch = torch.zeros(128, dtype=torch.float64, device=dev)
        plan.workspace(B)
        self.graph_fwd = None
        self.graph_train = None
        self.opt = dict(lr=1e-3, lr_min=1e-5, total=1000, beta1=0.9, beta2=0.99, eps=1e-8, clip=1.0)

    # ---- launch sequences -------------------------------------------------
    def _st(self):
        return _VP(torch.cuda.current_stream(self.dev).cuda_stream)

    def pack(self):
        st = self._st()
        for blk in (self.dual, self.primal):
            for l in blk.layers():
                l.pack(self.lib, st)

    def _axpby(self, count, a, x, b, y, r):
        _check(self.lib.pat_axpby(self.plan._h, count, float(a), _p(x), float(b), _p(y), _p(r), self._st()),
               "pat_axpby")

    def forward_pass(self):
        """f_K from y (self.y): K unrolled dual / primal steps (weights packed first)."""
        self.pack()
        st = self._st()
        P, K = self.plan, self.K
        for k in range(K):
            if k > 0:
                P.forward(self.f[k], out=self.Af[k])
            self.dual.forward(k, [self.q[k], self.Af[k], self.y], [1.0, self.s_A, self.s_A], self.q[k], self.q[k + 1], st)
            P.adjoint(self.q[k + 1], out=self.u[k])
            self.primal.forward(k, [self.f[k], self.u[k]], [1.0, self.s_U], self.f[k], self.f[k + 1], st)
        return self.f[K]

    def backward_pass(self):
        """Gradients of mean((f_K - target)^2) into self.grads (overwritten)."""
        P, K, B = self.plan, self.K, self.B
        n2 = B * P.n * P.n
        st = self._st()
        s = P.adjoint_scale
        # d loss / d f_K
        self._axpby(n2, 2.0 / n2, self.f[K], -2.0 / n2, self.target, self.df)
        df, df_next = self.df, self.df2
        dq, dq_next = self.dq, self.dq2
        for k in range(K - 1, -1, -1):
            first = k == K - 1
            # primal block: f_{k+1} = f_k + Lambda(f_k, s_U u_k), u_k = A* q_{k+1}
            self.primal.backward(k, [self.f[k], self.u[k]], [1.0, self.s_U], df, [df_next, self.du], [df, None],
                                 acc=not first, st=st)
            # d q_{k+1} += s A du   (u = s A^T q)
            P.forward(self.du, out=self.tmp_g)
            if first:
                self._axpby(self.tmp_g.numel(), s, self.tmp_g, 0.0, None, dq)
            else:
                self._axpby(self.tmp_g.numel(), s, self.tmp_g, 1.0, dq, dq)
            # dual block: q_{k+1} = q_k + Gamma(q_k, s_A A f_k, s_A y)
            want_af = k > 0
            self.dual.backward(k, [self.q[k], self.Af[k], self.y], [1.0, self.s_A, self.s_A], dq,
                               [dq_next, self.dAf if want_af else None, None], [dq, None, None], acc=not first, st=st)
            if want_af:
                # d f_k += A^T dAf = A* dAf / s
                P.adjoint(self.dAf, out=self.tmp_f)
                self._axpby(self.tmp_f.numel(), 1.0 / s, self.tmp_f, 1.0, df_next, df_next)
            df, df_next = df_next, df
            dq, dq_next = dq_next, dq
        return self.grads

    def adam(self):
        o = self.opt
        _check(self.lib.pat_adam(self.nparams, _p(self.params), _p(self.grads), _p(self.adam_m), _p(self.adam_v),
                                 _p(self.step_count), o["lr"], o["lr_min"], int(o["total"]), o["beta1"], o["beta2"],
                                 o["eps"], o["clip"], _p(self.adam_scratch), self._st()), "pat_adam")

    def train_step(self):
        self.forward_pass()
        self.backward_pass()
        self.adam()

    # ---- graphs -----------------------------------------------------------
    def _capture(self, fn):
        fn()  # warm-up outside capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        return g

    def capture_forward(self):
        self.graph_fwd = self._capture(self.forward_pass)
        return self.graph_fwd

    def capture_train(self):
        """Capture one training step.  The warm-up call performs a real step;
        the optimiser state (and the U-Net's running statistics) is reset
        afterwards so replays start from the initial weights."""
        p0 = self.params.clone()
        s0 = None if self.stats is None else self.stats.clone()
        self.graph_train = self._capture(self.train_step)
        self.params.copy_(p0)
        if s0 is not None:
            self.stats.copy_(s0)
        self.adam_m.zero_()
        self.adam_v.zero_()
        self.step_count.zero_()
        torch.cuda.synchronize()
        return self.graph_train

    def set_batch(self, y, target=None):
        self.y.copy_(y)
        if target is not None:
            self.target.copy_(target)

    def reconstruct(self, y):
        self.set_batch(y)
        if self.graph_fwd is not None:
            self.graph_fwd.replay()
        else:
            self.forward_pass()
        return self.f[self.K]

    def loss(self) -> float:
        """Mean squared error of f_K (reporting only)."""
        return float(torch.mean((self.f[self.K] - self.target) ** 2))


# ---- data, training and evaluation ------------------------------------------

def psnr(x: torch.Tensor, ref: torch.Tensor) -> torch.Tensor:
    """Per image 10 log10(1 / MSE) (images with peak value 1)."""
    mse = torch.mean((x.double() - ref.double()) ** 2, dim=(-2, -1))
    return 10.0 * torch.log10(1.0 / mse)


def make_dataset(plan: Plan, seeds, noise: float, noise_seed: int, chunk: int = 256) -> dict:
    """Random-ellipse phantoms (parameters drawn per seed, rasterised on the
    device) and their data y = A f + noise, with A the plan's forward
    operator and noise of relative L2 level ``noise`` per instance (the noise
    model of Sec. 4.3), drawn from a seeded device generator."""
    from . import phantoms as PH
    seeds = [int(s) for s in seeds]
    N, n, dev = len(seeds), plan.n, plan.device
    f = torch.empty((N, n, n), dtype=torch.float32, device=dev)
    y = torch.empty((N, plan.nt, plan.m), dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(noise_seed))
    for s in range(0, N, chunk):
        e = min(N, s + chunk)
        prm = np.stack([PH.ellipse_params(sd) for sd in seeds[s:e]])
        f[s:e] = PH.ellipse_images(prm, n, plan.geom["a"], device=dev)
        plan.forward(f[s:e], out=y[s:e])
        eps = torch.randn(y[s:e].shape, generator=gen, device=dev, dtype=torch.float32)
        ny = torch.linalg.vector_norm(y[s:e].flatten(1), dim=1)
        ne = torch.linalg.vector_norm(eps.flatten(1), dim=1)
        y[s:e] += (noise * ny / ne).view(-1, 1, 1) * eps
    return {"f": f, "y": y, "seeds": seeds}


def input_scales(plan: Plan, ds: dict, count: int = 64):
    """s_A, s_U that give A f (and y) and A* y the RMS of f on the first
    ``count`` training pairs."""
    f, y = ds["f"][:count], ds["y"][:count]
    u = plan.adjoint(y.contiguous())
    rms = lambda t: float(torch.sqrt(torch.mean(t.double() ** 2)))
    return rms(f) / rms(y), rms(f) / rms(u)


def train(net: LPD, ds: dict, steps: int, lr: float = 1e-3, lr_min: float = 1e-5, seed: int = 0,
          log_every: int = 50, log=None, clip: float = 1.0):
    """Adam with cosine decay and global-norm gradient clipping over ``steps``
    captured training steps, batches drawn as epochs of a seeded permutation.
    Returns [(step, loss)]."""
    net.opt.update(lr=lr, lr_min=lr_min, total=steps, clip=clip)
    N, B = ds["f"].shape[0], net.B
    rng = np.random.default_rng(seed)
    order, pos = rng.permutation(N), 0
    idx0 = torch.tensor(order[:B], device=net.dev)
    net.set_batch(ds["y"][idx0], ds["f"][idx0])
    if net.graph_train is None:
        net.capture_train()
    out = []
    for it in range(steps):
        if pos + B > N:
            order, pos = rng.permutation(N), 0
        idx = torch.tensor(order[pos:pos + B], device=net.dev)
        pos += B
        torch.index_select(ds["y"], 0, idx, out=net.y)
        torch.index_select(ds["f"], 0, idx, out=net.target)
        net.graph_train.replay()
        if (it + 1) % log_every == 0 or it == steps - 1:
            out.append((it + 1, net.loss()))
            if log is not None:
                log(it + 1, out[-1][1])
    return out


def evaluate(net: LPD, ds: dict, per_image: bool = False):
    """Mean PSNR of the reconstructions of a dataset (batches of net.B)."""
    vals = []
    N, B = ds["f"].shape[0], net.B
    for s in range(0, N - B + 1, B):
        fk = net.reconstruct(ds["y"][s:s + B])
        vals.append(psnr(fk, ds["f"][s:s + B]))
    v = torch.cat(vals).cpu().numpy()
    return v if per_image else float(v.mean())


def backprojection_psnr(plan: Plan, ds: dict, s_U: float) -> float:
    """Mean PSNR of the normalised back-projection s_U A* y clipped to [0, 1]."""
    u = plan.adjoint(ds["y"].contiguous())
    plan.scale_(u, s_U)
    return float(psnr(torch.clamp(u, 0.0, 1.0), ds["f"]).mean())
