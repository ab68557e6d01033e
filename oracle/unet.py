"""CPU FP64 oracle of the U-Net networks of the learned primal-dual reconstructor.

TEST INFRASTRUCTURE ONLY (imported by ``tests/``; the product never imports
it).  Plain PyTorch CPU float64 with autograd, following Sec. 4.2.1 of
Hauptmann, Kunyansky & Poimala (arXiv 2510.24687): the networks Gamma and
Lambda are U-Nets with four scales, three down- and up-sampling steps of
window 2, two 3x3 convolutions per scale each followed by batch normalisation
and ReLU, 32 filters at the first scale, doubled at every down-sampling (256
at the coarsest), the same architecture for both networks apart from the
number of input channels.

Readings (where the paper leaves the layer details open, the usual U-Net):
  * down-sampling: 2x2 max pooling; the first maximum of a window, in the
    order (0,0), (0,1), (1,0), (1,1), receives the gradient;
  * up-sampling: 2x2 transposed convolution of stride 2 halving the channels
    (weight layout [in][out][2][2]), then concatenation [skip, up-sampled];
  * convolutions: zero padding 1, cross-correlation (the convention of
    torch.nn.functional.conv2d), no bias (the batch normalisation that
    follows removes any constant); the up-sampling has no bias either;
  * batch normalisation: batch statistics (mean, biased variance over batch
    and pixels, eps = 1e-5) in training, running averages with momentum 0.1
    (unbiased variance) updated at every application and used at inference,
    gamma = 1 and beta = 0 initially; inside the unrolled reconstructor each
    iteration keeps its own running averages (buffers, not parameters: the
    parameters stay shared), since the iterations' activations have
    different statistics;
  * output: a 1x1 convolution 32 -> 1 with bias.
With these readings the two networks (3 and 2 input channels) hold 3.85e6
parameters, in line with the paper's count of about 3.9e6.

Precision: with ``rounding=True`` the oracle stores what the GPU stores in
bfloat16 (network inputs, activations after batch normalisation and ReLU,
up-sampled maps) rounded to bfloat16 and rounds the operands of every
convolution product (forward, input gradient, weight gradient) to bfloat16,
as the matrix-core kernels do; sums are float64.  The storage rounding passes
gradients through unchanged (the GPU keeps activation gradients in FP32; only
the gradients that enter a product are rounded, inside the products).
``rounding=False`` is the plain FP64 network.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Tuple

import numpy as np
import torch
import torch.nn.functional as F

from .lpd import bf16, conv3x3

WIDTHS = (32, 64, 128, 256)
BN_EPS = 1e-5
BN_MOMENTUM = 0.1


def layout(cin: int) -> List[Tuple[str, tuple]]:
    """Parameter names and shapes of one U-Net with ``cin`` input channels."""
    out = []
    c_in = cin
    for s, c in enumerate(WIDTHS):
        for j in (1, 2):
            out += [("e%dc%d.w" % (s, j), (c, c_in if j == 1 else c, 3, 3)),
                    ("e%dc%d.g" % (s, j), (c,)), ("e%dc%d.b" % (s, j), (c,))]
        c_in = c
    for s in (2, 1, 0):
        c = WIDTHS[s]
        out.append(("u%d.w" % s, (2 * c, c, 2, 2)))
        for j in (1, 2):
            out += [("d%dc%d.w" % (s, j), (c, 2 * c if j == 1 else c, 3, 3)),
                    ("d%dc%d.g" % (s, j), (c,)), ("d%dc%d.b" % (s, j), (c,))]
    out += [("head.w", (1, WIDTHS[0], 1, 1)), ("head.b", (1,))]
    return out


def bn_layers() -> List[Tuple[str, int]]:
    """(name, channels) of the batch-normalised convolutions, in order."""
    out = []
    for s, c in enumerate(WIDTHS):
        out += [("e%dc1" % s, c), ("e%dc2" % s, c)]
    for s in (2, 1, 0):
        out += [("d%dc1" % s, WIDTHS[s]), ("d%dc2" % s, WIDTHS[s])]
    return out


def count_params(cin: int) -> int:
    return int(sum(np.prod(shape) for _, shape in layout(cin)))


def fresh_running() -> Dict[str, Dict[str, torch.Tensor]]:
    """Running statistics at their initial values (mean 0, variance 1)."""
    return {name: {"mean": torch.zeros(c, dtype=torch.float64), "var": torch.ones(c, dtype=torch.float64)}
            for name, c in bn_layers()}


def batch_norm_relu(z, gamma, beta, running=None, training=True, momentum=BN_MOMENTUM, eps=BN_EPS):
    """max(0, gamma (z - mean) / sqrt(var + eps) + beta) per channel (dim 1);
    training: batch mean and biased variance over dims (0, 2, 3), running
    averages updated in place; otherwise the running averages are used."""
    if training:
        mean = z.mean(dim=(0, 2, 3))
        var = ((z - mean.view(1, -1, 1, 1)) ** 2).mean(dim=(0, 2, 3))
        if running is not None:
            count = z.numel() // z.shape[1]
            running["mean"] = (1 - momentum) * running["mean"] + momentum * mean.detach()
            running["var"] = (1 - momentum) * running["var"] + momentum * var.detach() * count / max(count - 1, 1)
    else:
        mean, var = running["mean"], running["var"]
    xh = (z - mean.view(1, -1, 1, 1)) / torch.sqrt(var.view(1, -1, 1, 1) + eps)
    return torch.relu(gamma.view(1, -1, 1, 1) * xh + beta.view(1, -1, 1, 1))


def maxpool2(x):
    """2x2 max pooling, stride 2; the gradient goes to the first maximum of
    each window in the order (0,0), (0,1), (1,0), (1,1)."""
    B, C, H, W = x.shape
    win = x.reshape(B, C, H // 2, 2, W // 2, 2).permute(0, 1, 2, 4, 3, 5).reshape(B, C, H // 2, W // 2, 4)
    idx = torch.argmax(win, dim=-1, keepdim=True)
    return torch.gather(win, -1, idx).squeeze(-1)


class _TConv2(torch.autograd.Function):
    """2x2 stride-2 transposed convolution without bias, w: (cin, cout, 2, 2):
    out[b, o, 2y+i, 2x+j] = sum_c x[b, c, y, x] w[c, o, i, j]; bf16 operands
    in every product when rounding."""

    @staticmethod
    def forward(ctx, x, w, rounding, perturb):
        xr, wr = (bf16(x), bf16(w)) if rounding else (x, w)
        ctx.save_for_backward(xr, wr)
        ctx.rounding = rounding
        ctx.perturb = perturb
        y = F.conv_transpose2d(xr, wr, stride=2)
        return perturb.apply(y, perturb.conv) if perturb is not None else y

    @staticmethod
    def backward(ctx, gy):
        xr, wr = ctx.saved_tensors
        gyr = bf16(gy) if ctx.rounding else gy
        B, Co, H2, W2 = gyr.shape
        gx = F.conv2d(gyr, wr, stride=2)
        g6 = gyr.reshape(B, Co, H2 // 2, 2, W2 // 2, 2)
        gw = torch.einsum("bchw,bdhiwj->cdij", xr, g6)
        pt = ctx.perturb
        if pt is not None:
            gx, gw = pt.apply(gx, pt.conv), pt.apply(gw, pt.conv)
        return gx, gw, None, None


def tconv2(x, w, rounding=True, perturb=None):
    return _TConv2.apply(x, w, rounding, perturb)


def stored_bf16(x):
    """bf16 storage of a value: rounded forward, gradient passed through."""
    return x + (bf16(x.detach()) - x.detach())


def unet(x, P: dict, prefix: str, running: Optional[dict] = None, training: bool = True, rounding: bool = True,
         perturb=None):
    """The U-Net on x (B, cin, H, W), H and W divisible by 8; parameters
    P[prefix + name] (float64 tensors); running statistics
    running[prefix + layer] (updated in training).  Returns (B, 1, H, W).
    ``perturb``: the FP32 noise model of oracle/lpd.py (tests only)."""
    store = stored_bf16 if rounding else (lambda t: t)

    def cbr(name, h):
        z = conv3x3(h, P[prefix + name + ".w"], None, rounding, perturb)
        r = None if running is None else running[prefix + name]
        return store(batch_norm_relu(z, P[prefix + name + ".g"], P[prefix + name + ".b"], r, training))

    h = store(x)
    skips = []
    for s in range(4):
        h = cbr("e%dc2" % s, cbr("e%dc1" % s, h))
        if s < 3:
            skips.append(h)
            h = maxpool2(h)
    for s in (2, 1, 0):
        up = store(tconv2(h, P[prefix + "u%d.w" % s], rounding, perturb))
        h = torch.cat([skips[s], up], dim=1)
        h = cbr("d%dc2" % s, cbr("d%dc1" % s, h))
    return F.conv2d(h, P[prefix + "head.w"], P[prefix + "head.b"])

