"""CPU FP64 oracle of the learned primal-dual reconstructor.

TEST INFRASTRUCTURE ONLY (imported by ``tests/``; the product never imports
it).  Plain PyTorch CPU float64 with autograd, following Sec. 4.2.1 of
Hauptmann, Kunyansky & Poimala (arXiv 2510.24687): the unrolled updates of
eqs. eq:LPD_dual / eq:LPD_primal in residual form with one set of weights
shared by all iterations, and the squared-error loss of eq:emp_loss (taken
as a mean over pixels).  The operators A and A* inside are this package's
direct-quadrature ``forward`` / ``adjoint``.

Network (the reading used throughout): Gamma and Lambda are 3-layer 3x3
convolution stacks cin -> 32 -> 32 -> 1 with zero padding 1 (the
cross-correlation convention of torch.nn.functional.conv2d), PReLU with one
slope per channel after the first two layers, inputs [q, s_A A f, s_A y] and
[f, s_U A* q]:

    q_{k+1} = q_k + Gamma(q_k, s_A A f_k, s_A y)
    f_{k+1} = f_k + Lambda(f_k, s_U A* q_{k+1}),   f_0 = q_0 = 0.

Precision: the matrix products of the convolutions take operands rounded to
bfloat16 (round to nearest even, via torch's own float32 -> bfloat16 cast),
as the GPU kernels do: in the forward product (input, weight), in the input
gradient (output gradient, weight) and in the weight gradient (output
gradient, input).  Sums are exact-ish (float64).  ``rounding=False`` gives
the plain FP64 network, whose gradients torch.autograd.gradcheck verifies.

``perturb`` (a Perturb) multiplies every operator output (A f, A* q and
their transposes in the backward pass) and every convolution product by
(1 + level * xi), xi i.i.d. N(0,1) from a seeded generator: a model of FP32
arithmetic noise.  The tests use an ensemble of such runs to measure how far
FP32-level differences alone move the bf16-rounded network (roundings that
land on the other side of a midpoint), which sets their tolerance for the
GPU network; it is never part of the network's definition.
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

from . import adjoint as _adjoint_np
from . import adjoint_scale
from . import forward as _forward_np

HID = 32


class Perturb:
    """Seeded relative noise for operator outputs (op) and convolution products (conv)."""

    def __init__(self, seed: int, op: float = 1e-6, conv: float = 1e-7):
        self.gen = torch.Generator().manual_seed(int(seed))
        self.op, self.conv = float(op), float(conv)

    def apply(self, x: torch.Tensor, level: float) -> torch.Tensor:
        if level <= 0:
            return x
        return x * (1.0 + level * torch.randn(x.shape, generator=self.gen, dtype=torch.float64))


def bf16(x: torch.Tensor) -> torch.Tensor:
    """Round float values to bfloat16 (through float32) and return float64."""
    return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)


class _Conv3x3(torch.autograd.Function):
    """conv2d(x, w, b, padding=1) with bf16-rounded operands in every product."""

    @staticmethod
    def forward(ctx, x, w, b, rounding, perturb):
        xr, wr = (bf16(x), bf16(w)) if rounding else (x, w)
        ctx.save_for_backward(xr, wr)
        ctx.rounding = rounding
        ctx.perturb = perturb
        y = F.conv2d(xr, wr, b, padding=1)
        return perturb.apply(y, perturb.conv) if perturb is not None else y

    @staticmethod
    def backward(ctx, gy):
        xr, wr = ctx.saved_tensors
        gyr = bf16(gy) if ctx.rounding else gy
        gx = F.conv_transpose2d(gyr, wr, padding=1)
        gw = torch.nn.grad.conv2d_weight(xr, wr.shape, gyr, padding=1)
        gb = gy.sum(dim=(0, 2, 3))
        pt = ctx.perturb
        if pt is not None:
            gx, gw = pt.apply(gx, pt.conv), pt.apply(gw, pt.conv)
        return gx, gw, gb, None, None


def conv3x3(x, w, b=None, rounding=True, perturb=None):
    """x: (B, cin, H, W), w: (cout, cin, 3, 3), b: (cout,) or None."""
    if b is None:
        b = torch.zeros(w.shape[0], dtype=x.dtype)
    return _Conv3x3.apply(x, w, b, rounding, perturb)


def prelu(x, alpha):
    """max(x, 0) + alpha min(x, 0), one slope per channel (dim 1)."""
    return torch.where(x > 0, x, alpha.view(1, -1, 1, 1) * x)


def _op_noise(x, perturb):
    return perturb.apply(x, perturb.op) if perturb is not None else x


class _A(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, geom, perturb):
        ctx.geom = geom
        ctx.perturb = perturb
        out = [_forward_np(geom, fi.detach().numpy()) for fi in f]
        return _op_noise(torch.tensor(np.stack(out), dtype=torch.float64), perturb)

    @staticmethod
    def backward(ctx, g):
        s = adjoint_scale(ctx.geom)
        out = [_adjoint_np(ctx.geom, gi.numpy()) / s for gi in g]
        return _op_noise(torch.tensor(np.stack(out), dtype=torch.float64), ctx.perturb), None, None


class _Astar(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g, geom, perturb):
        ctx.geom = geom
        ctx.perturb = perturb
        out = [_adjoint_np(geom, gi.detach().numpy()) for gi in g]
        return _op_noise(torch.tensor(np.stack(out), dtype=torch.float64), perturb)

    @staticmethod
    def backward(ctx, f):
        s = adjoint_scale(ctx.geom)
        out = [s * _forward_np(ctx.geom, fi.numpy()) for fi in f]
        return _op_noise(torch.tensor(np.stack(out), dtype=torch.float64), ctx.perturb), None, None


def block(x, P, net, rounding=True, perturb=None):
    """3-layer CNN: conv-PReLU, conv-PReLU, conv.  P: dict of float64 tensors."""
    h = prelu(conv3x3(x, P[net + ".w1"], P[net + ".b1"], rounding, perturb), P[net + ".a1"])
    h = prelu(conv3x3(h, P[net + ".w2"], P[net + ".b2"], rounding, perturb), P[net + ".a2"])
    return conv3x3(h, P[net + ".w3"], P[net + ".b3"], rounding, perturb)


def _network(x, P, net, rounding, arch, running, training, perturb=None):
    if arch == "unet":
        from .unet import unet
        return unet(x, P, net + ".", running, training, rounding, perturb=perturb)
    return block(x, P, net, rounding, perturb)


def reconstruct(geom, P, y, iters, s_A=1.0, s_U=1.0, rounding=True, ops=None, arch="cnn", running=None,
                training=True, perturb=None):
    """f_K for data y (B, nt, m).  ``ops`` = (A, A*) callables on batches may
    replace the direct-quadrature operators (used by gradcheck on tiny
    explicit matrices).  ``arch = "unet"``: the U-Nets of oracle/unet.py with
    running statistics ``running[k]`` for unrolled iteration k (keys
    "dual.<layer>", "primal.<layer>"; batch statistics and updated averages
    in training, the averages otherwise)."""
    A, As = ops if ops is not None else ((lambda f: _A.apply(f, geom, perturb)),
                                         (lambda g: _Astar.apply(g, geom, perturb)))
    B = y.shape[0]
    n = geom["n"]
    q = torch.zeros_like(y)
    f = torch.zeros((B, n, n), dtype=torch.float64)
    for k in range(iters):
        Af = A(f)
        run_k = None if running is None else running[k]
        q = q + _network(torch.stack([q, s_A * Af, s_A * y], dim=1), P, "dual", rounding, arch, run_k,
                         training, perturb)[:, 0]
        u = As(q)
        f = f + _network(torch.stack([f, s_U * u], dim=1), P, "primal", rounding, arch, run_k, training,
                         perturb)[:, 0]
    return f


def loss_and_grads(geom, P, y, target, iters, s_A=1.0, s_U=1.0, rounding=True, arch="cnn", running=None,
                   perturb=None):
    """mean((f_K - target)^2) and its gradient with respect to every parameter."""
    Pt = {k: torch.tensor(np.asarray(v, dtype=np.float64), requires_grad=True) for k, v in P.items()}
    yt = torch.tensor(np.asarray(y, dtype=np.float64))
    tt = torch.tensor(np.asarray(target, dtype=np.float64))
    fK = reconstruct(geom, Pt, yt, iters, s_A, s_U, rounding, arch=arch, running=running, perturb=perturb)
    loss = torch.mean((fK - tt) ** 2)
    loss.backward()
    return float(loss.detach()), fK.detach().numpy(), {k: v.grad.numpy() for k, v in Pt.items()}


def adam_reference(p, g, m, v, t, lr0, lr_min, total, b1=0.9, b2=0.999, eps=1e-8, clip=0.0):
    """One Adam step (Kingma & Ba, bias-corrected moments) with the step size
    lr_min + (lr0 - lr_min) (1 + cos(pi min(1, (t-1)/(total-1)))) / 2, after
    scaling g by min(1, clip / ||g||_2) when clip > 0."""
    if clip > 0:
        g = g * min(1.0, clip / float(np.sqrt(np.sum(np.asarray(g, dtype=np.float64) ** 2))))
    frac = min(1.0, (t - 1) / max(total - 1, 1))
    lr = lr_min + 0.5 * (lr0 - lr_min) * (1 + math.cos(math.pi * frac))
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return p, m, v
