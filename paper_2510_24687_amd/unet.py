"""U-Net networks for the learned primal-dual reconstructor, driven by the
library's kernels.

The architecture of Sec. 4.2.1 of Hauptmann, Kunyansky & Poimala (arXiv
2510.24687): four scales, three window-2 down- and up-sampling steps, two 3x3
convolutions per scale each followed by batch normalisation and ReLU, 32
filters at the first scale doubled at every down-sampling (256 at the
coarsest), the same network for the dual and the primal update apart from the
input channels.  Layer details (the usual U-Net): 2x2 max pooling; 2x2
stride-2 transposed convolutions halving the channels, concatenated after
the skip connection; bias-free convolutions (batch normalisation follows);
batch statistics in training, running averages (momentum 0.1) at inference; a
1x1 output convolution with bias.  Both networks together hold 3.85e6
parameters, shared by all unrolled iterations.  The running averages are
buffers, not parameters, and the activations of the K unrolled iterations
have different statistics, so each iteration keeps its own running averages
(one shared set would average over all iterations and normalise none of them
as in training).

Every step runs in libpat.so: the generic implicit-GEMM convolution on the
BF16 matrix cores (pat_gconv) for the 3x3 convolutions, the transposed
convolutions and all their input gradients, pat_gconv_wgrad for the weight
gradients, pat_bn_forward / pat_bn_backward, pat_maxpool2(_backward), the
input packing and the 1x1 head.  Python allocates buffers and marshals
pointers only.  Activations are NHWC bfloat16, convolution outputs and
activation gradients NHWC FP32.
"""
from __future__ import annotations

import ctypes
import math
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch

from .pat import GConvDesc, _check

WIDTHS = (32, 64, 128, 256)
CPAD = 16                      # padded channels of the network input
BN_EPS = 1e-5
BN_MOMENTUM = 0.1
TAPS3 = [(t // 3 - 1, t % 3 - 1) for t in range(9)]
TAPS_UP = [(0, 0), (0, 1), (1, 0), (1, 1)]


def _p(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def layout(cin: int) -> List[Tuple[str, tuple]]:
    """Parameter names and shapes of one U-Net with ``cin`` input channels,
    in storage order (convolutions [out][in][3][3], transposed convolutions
    [in][out][2][2], batch-normalisation scale g and shift b)."""
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
    out = []
    for s, c in enumerate(WIDTHS):
        out += [("e%dc1" % s, c), ("e%dc2" % s, c)]
    for s in (2, 1, 0):
        out += [("d%dc1" % s, WIDTHS[s]), ("d%dc2" % s, WIDTHS[s])]
    return out


def stats_layout(iters: int, nets=(("dual", 3), ("primal", 2))) -> List[Tuple[str, int]]:
    """Running statistics "<net>.it<k>.<layer>.mean|var": per network,
    unrolled iteration k < iters and layer, mean then variance."""
    out = []
    for net, _ in nets:
        for k in range(iters):
            for name, c in bn_layers():
                key = "%s.it%d.%s" % (net, k, name)
                out += [(key + ".mean", c), (key + ".var", c)]
    return out


def init_stats(iters: int, nets=(("dual", 3), ("primal", 2))) -> np.ndarray:
    return np.concatenate([np.zeros(c) if name.endswith(".mean") else np.ones(c)
                           for name, c in stats_layout(iters, nets)]).astype(np.float32)


def init_values(name: str, shape: tuple, rng) -> np.ndarray:
    """He-uniform convolutions (fan-in = inputs x taps; the transposed
    convolutions: their input channels), g = 1, b = 0, the output layer
    scaled by 0.1 with a zero bias so that the untrained network is close to
    the identity update."""
    size = int(np.prod(shape))
    kind = name.split(".")[-1]
    if kind == "w":
        base = name.split(".")[-2]
        fan_in = shape[0] if base.startswith("u") else shape[1] * shape[2] * shape[3]
        bound = math.sqrt(6.0 / fan_in) * (0.1 if base == "head" else 1.0)
        return rng.uniform(-bound, bound, size)
    if kind == "g":
        return np.ones(size)
    return np.zeros(size)


class _Conv:
    """One bias-free 3x3 convolution + batch normalisation + ReLU."""

    def __init__(self, lib, P, name, srcs, cout, dev):
        self.name, self.srcs, self.cout = name, list(srcs), cout   # srcs: real channel counts of the sources
        self.cin_real = sum(srcs)
        self.cip = [max(c, CPAD) if len(srcs) == 1 else c for c in srcs]  # padded source pitches
        self.cin_pad = sum(self.cip)
        w, gw = P.view(name + ".w")
        self.w, self.gw = w, gw
        self.g, self.gg = P.view(name + ".g")
        self.b, self.gb = P.view(name + ".b")
        self.wf = torch.empty(lib.pat_gconv_packed_size(cout, self.cin_pad, 9), dtype=torch.int16, device=dev)
        self.cout_t = self.cin_pad                                     # input gradient: columns = input channels
        self.wb = torch.empty(lib.pat_gconv_packed_size(self.cout_t, cout, 9), dtype=torch.int16, device=dev)

    def pack(self, lib, st):
        ci = self.cin_real
        _check(lib.pat_gconv_pack(_p(self.w), self.cout, ci, self.cout, self.cin_pad, 9, 0, ci * 9, 9, 1, 0,
                                  _p(self.wf), st), "pat_gconv_pack")
        # W_e[ci][co][t] = w[co][ci][8 - t]
        _check(lib.pat_gconv_pack(_p(self.w), ci, self.cout, self.cout_t, self.cout, 9, 0, 9, ci * 9, 1, 1,
                                  _p(self.wb), st), "pat_gconv_pack")


class _Up:
    """2x2 stride-2 transposed convolution cin -> cout (no bias)."""

    def __init__(self, lib, P, name, cin, cout, dev):
        self.name, self.cin, self.cout = name, cin, cout
        self.w, self.gw = P.view(name + ".w")
        n1 = lib.pat_gconv_packed_size(cout, cin, 1)
        self.wf = torch.empty((4, n1), dtype=torch.int16, device=dev)
        self.wb = torch.empty(lib.pat_gconv_packed_size(cin, cout, 4), dtype=torch.int16, device=dev)

    def pack(self, lib, st):
        for p in range(4):
            # parity p = 2 i + j: W_e[co][ci] = w[ci][co][i][j]
            _check(lib.pat_gconv_pack(_p(self.w), self.cout, self.cin, self.cout, self.cin, 1, p, 4, self.cout * 4, 0,
                                      0, _p(self.wf[p]), st), "pat_gconv_pack")
        # input gradient, tap t = 2 i + j read at stride 2: W_e[ci][co][t] = w[ci][co][t]
        _check(lib.pat_gconv_pack(_p(self.w), self.cin, self.cout, self.cin, self.cout, 4, 0, self.cout * 4, 4, 1, 0,
                                  _p(self.wb), st), "pat_gconv_pack")


class _ParamViews:
    def __init__(self, params, grads, offs, prefix, shapes):
        self.params, self.grads, self.offs, self.prefix, self.shapes = params, grads, offs, prefix, shapes

    def view(self, name):
        o = self.offs[self.prefix + name]
        size = int(np.prod(self.shapes[self.prefix + name]))
        return self.params[o:o + size], self.grads[o:o + size]


def _gdesc(B, H, W, srcs, Hs, Ws, istr, taps, weight, cout, dsts, Ho, Wo, ostr=1, oy=0, ox=0):
    """srcs: [(tensor, channels)], dsts: [(tensor, channels, bf16, accumulate)]."""
    d = GConvDesc()
    d.B, d.H, d.W = B, H, W
    for i, (t, c) in enumerate(srcs):
        d.src[i] = _p(t)
        d.csrc[i] = c
    d.Hs, d.Ws, d.in_stride = Hs, Ws, istr
    d.ntaps = len(taps)
    for i, (dy, dx) in enumerate(taps):
        d.dy[i], d.dx[i] = dy, dx
    d.weight = _p(weight)
    d.cout = cout
    for i, (t, c, bf, acc) in enumerate(dsts):
        d.dst[i] = _p(t)
        d.cdst[i] = c
        d.dst_bf16[i] = int(bf)
        d.accumulate[i] = int(acc)
    d.Ho, d.Wo, d.out_stride, d.oy, d.ox = Ho, Wo, ostr, oy, ox
    return d


class UNetBlock:
    """One U-Net (dual or primal) on a B x H x W domain (H, W divisible by 8)
    with cin planar inputs and a residual 1-channel planar output; keeps what
    the backward needs for K applications (training) or one (inference)."""

    def __init__(self, lib, params, grads, offs, shapes, stats, soffs, net, cin, B, H, W, K, dev, train):
        if H % 8 or W % 8:
            raise ValueError("the U-Net needs H and W divisible by 8 (three 2x down-samplings)")
        self.lib, self.net, self.cin, self.B, self.H, self.W, self.K, self.train = (
            lib, net, cin, B, H, W, K, train)
        P = _ParamViews(params, grads, offs, net + ".", shapes)
        self.convs: Dict[str, _Conv] = {}
        c_in = [cin]
        for s, c in enumerate(WIDTHS):
            self.convs["e%dc1" % s] = _Conv(lib, P, "e%dc1" % s, c_in, c, dev)
            self.convs["e%dc2" % s] = _Conv(lib, P, "e%dc2" % s, [c], c, dev)
            c_in = [c]
        self.ups: Dict[int, _Up] = {}
        for s in (2, 1, 0):
            c = WIDTHS[s]
            self.ups[s] = _Up(lib, P, "u%d" % s, 2 * c, c, dev)
            self.convs["d%dc1" % s] = _Conv(lib, P, "d%dc1" % s, [c, c], c, dev)
            self.convs["d%dc2" % s] = _Conv(lib, P, "d%dc2" % s, [c], c, dev)
        self.head_w, self.head_gw = P.view("head.w")
        self.head_b, self.head_gb = P.view("head.b")
        self.stats = []
        for k in range(K):
            d = {}
            for name, c in bn_layers():
                key = "%s.it%d.%s" % (net, k, name)
                o_m, o_v = soffs[key + ".mean"], soffs[key + ".var"]
                d[name] = (stats[o_m:o_m + c], stats[o_v:o_v + c])
            self.stats.append(d)
        self.hs = [H >> s for s in range(4)]
        self.ws = [W >> s for s in range(4)]
        self.rows = [B * self.hs[s] * self.ws[s] for s in range(4)]
        nk = K if train else 1
        i16 = lambda *s: torch.empty(s, dtype=torch.int16, device=dev)
        f32 = lambda *s: torch.empty(s, dtype=torch.float32, device=dev)
        self.x0 = [i16(self.rows[0], CPAD) for _ in range(nk)]
        self.z, self.a, self.mean, self.invstd = {}, {}, {}, {}
        for name, c in bn_layers():
            s = self._scale(name)
            self.z[name] = [f32(self.rows[s], c) for _ in range(nk)]
            self.a[name] = [i16(self.rows[s], c) for _ in range(nk)]
            self.mean[name] = [f32(c) for _ in range(nk)]
            self.invstd[name] = [f32(c) for _ in range(nk)]
        self.pool = {s: [i16(self.rows[s + 1], WIDTHS[s]) for _ in range(nk)] for s in range(3)}
        self.up = {s: [i16(self.rows[s], WIDTHS[s]) for _ in range(nk)] for s in range(3)}
        bnp = max(lib.pat_bn_partials(self.rows[s], WIDTHS[s]) for s in range(4))
        self.bn_part = torch.empty(max(bnp, lib.pat_head_partials(self.rows[0], WIDTHS[0])), dtype=torch.float64,
                                   device=dev)
        if train:
            self.gA = [f32(self.rows[s], WIDTHS[s]) for s in range(4)]
            self.gB = [f32(self.rows[s], WIDTHS[s]) for s in range(4)]
            self.gS = [f32(self.rows[s], WIDTHS[s]) for s in range(3)]
            self.gz = [i16(self.rows[s], WIDTHS[s]) for s in range(4)]
            self.gup = [i16(self.rows[s], WIDTHS[s]) for s in range(3)]
            self.gx0 = f32(self.rows[0], CPAD)
            need = 0
            for name, L in self.convs.items():
                d = self._fwd_desc(L, 0)
                need = max(need, lib.pat_gconv_wgrad_partials(ctypes.byref(d), self._chunks(d)))
            for s, U in self.ups.items():
                d = self._up_desc(U, s, 0, 0)
                need = max(need, lib.pat_gconv_wgrad_partials(ctypes.byref(d), self._chunks(d)))
            self.wpart = f32(max(need, 1))

    # ---- geometry helpers ---------------------------------------------------
    @staticmethod
    def _scale(name):
        return int(name[1])

    def _chunks(self, d):
        K = d.ntaps * (d.csrc[0] + d.csrc[1])
        tiles = ((K + 63) // 64) * ((d.cout + 63) // 64)
        rows = d.B * d.H * d.W
        return int(max(1, min((rows + 255) // 256, 2048 // tiles)))

    def _sources(self, name, j):
        """(tensor, pitch) sources of convolution ``name`` in application j."""
        s = self._scale(name)
        kind, idx = name[0], name[3]
        if name == "e0c1":
            return [(self.x0[j], CPAD)]
        if idx == "2":
            return [(self.a[name[:3] + "1"][j], WIDTHS[s])]
        if kind == "e":
            return [(self.pool[s - 1][j], WIDTHS[s - 1])]
        return [(self.a["e%dc2" % s][j], WIDTHS[s]), (self.up[s][j], WIDTHS[s])]

    def _fwd_desc(self, L, j, dsts=None):
        s = self._scale(L.name)
        B, H, W = self.B, self.hs[s], self.ws[s]
        return _gdesc(B, H, W, self._sources(L.name, j), H, W, 1, TAPS3, L.wf, L.cout, dsts or [], H, W)

    def _up_desc(self, U, s, j, p, dsts=None):
        """Transposed convolution u_s, output parity p = 2 i + j: iteration grid
        = its input (scale s + 1)."""
        src = self.a["e3c2"][j] if s == 2 else self.a["d%dc2" % (s + 1)][j]
        B, H, W = self.B, self.hs[s + 1], self.ws[s + 1]
        return _gdesc(B, H, W, [(src, U.cin)], H, W, 1, [(0, 0)], U.wf[p], U.cout, dsts or [],
                      self.hs[s], self.ws[s], 2, p // 2, p % 2)

    def layers(self):
        return list(self.convs.values()) + list(self.ups.values())

    def forward_flops(self) -> float:
        """Multiply-add flops (2 per product) of one application's matrix-core
        products (3x3 and transposed convolutions, real channels only)."""
        total = 0.0
        for name, L in self.convs.items():
            total += 2.0 * self.rows[self._scale(name)] * L.cout * 9 * L.cin_real
        for s, U in self.ups.items():
            total += 2.0 * self.rows[s + 1] * 4 * U.cout * U.cin
        return total

    # ---- forward ------------------------------------------------------------
    def _conv_bn(self, name, j, k, bn_train, st):
        lib, L = self.lib, self.convs[name]
        s = self._scale(name)
        d = self._fwd_desc(L, j, [(self.z[name][j], L.cout, False, False)])
        _check(lib.pat_gconv(ctypes.byref(d), st), "pat_gconv")
        rm, rv = self.stats[k][name]
        _check(lib.pat_bn_forward(self.rows[s], L.cout, _p(self.z[name][j]), _p(L.g), _p(L.b), _p(self.mean[name][j]),
                                  _p(self.invstd[name][j]), _p(rm), _p(rv), BN_MOMENTUM, BN_EPS, int(bn_train),
                                  _p(self.a[name][j]), _p(self.bn_part), st), "pat_bn_forward")

    def forward(self, k, planes, scales, state_in, state_out, st):
        """state_out = state_in + U-Net(scales * planes) for application
        (unrolled iteration) k, normalised with iteration k's statistics."""
        lib = self.lib
        j = min(k, len(self.x0) - 1)
        bn_train = self.train
        vpa = (ctypes.c_void_p * 4)(*([_p(t) for t in planes] + [None] * (4 - len(planes))))
        sca = (ctypes.c_float * 4)(*([float(v) for v in scales] + [1.0] * (4 - len(scales))))
        _check(lib.pat_nhwc_pack(self.rows[0], self.cin, CPAD, vpa, sca, _p(self.x0[j]), st), "pat_nhwc_pack")
        for s in range(4):
            self._conv_bn("e%dc1" % s, j, k, bn_train, st)
            self._conv_bn("e%dc2" % s, j, k, bn_train, st)
            if s < 3:
                _check(lib.pat_maxpool2(self.B, self.hs[s], self.ws[s], WIDTHS[s], _p(self.a["e%dc2" % s][j]),
                                        _p(self.pool[s][j]), st), "pat_maxpool2")
        for s in (2, 1, 0):
            U = self.ups[s]
            for p in range(4):
                d = self._up_desc(U, s, j, p, [(self.up[s][j], U.cout, True, False)])
                _check(lib.pat_gconv(ctypes.byref(d), st), "pat_gconv")
            self._conv_bn("d%dc1" % s, j, k, bn_train, st)
            self._conv_bn("d%dc2" % s, j, k, bn_train, st)
        _check(lib.pat_head_forward(self.rows[0], WIDTHS[0], _p(self.a["d0c2"][j]), _p(self.head_w), _p(self.head_b),
                                    _p(state_in), _p(state_out), st), "pat_head_forward")

    # ---- backward -----------------------------------------------------------
    def _conv_bwd(self, name, k, ga, dsts, acc, st):
        """Batch-norm backward of layer ``name`` from ga (FP32 gradient of its
        activation), its weight gradient, and its input gradient into dsts."""
        lib, L = self.lib, self.convs[name]
        s = self._scale(name)
        gz = self.gz[s]
        _check(lib.pat_bn_backward(self.rows[s], L.cout, _p(self.z[name][k]), _p(ga), _p(L.g), _p(L.b),
                                   _p(self.mean[name][k]), _p(self.invstd[name][k]), _p(gz), _p(L.gg), _p(L.gb),
                                   int(acc), _p(self.bn_part), st), "pat_bn_backward")
        d = self._fwd_desc(L, k)
        ci = L.cin_real
        _check(lib.pat_gconv_wgrad(ctypes.byref(d), _p(gz), self._chunks(d), _p(self.wpart), _p(L.gw), ci, 0, ci * 9, 9,
                                   1, int(acc), st), "pat_gconv_wgrad")
        H, W = self.hs[s], self.ws[s]
        d = _gdesc(self.B, H, W, [(gz, L.cout)], H, W, 1, TAPS3, L.wb, L.cout_t, dsts, H, W)
        _check(lib.pat_gconv(ctypes.byref(d), st), "pat_gconv")

    def _up_bwd(self, s, k, dst, acc, st):
        lib, U = self.lib, self.ups[s]
        g = self.gup[s]
        for p in range(4):
            d = self._up_desc(U, s, k, p)
            _check(lib.pat_gconv_wgrad(ctypes.byref(d), _p(g), self._chunks(d), _p(self.wpart), _p(U.gw), U.cin, p,
                                       4, U.cout * 4, 0, int(acc), st), "pat_gconv_wgrad")
        H, W = self.hs[s + 1], self.ws[s + 1]
        d = _gdesc(self.B, H, W, [(g, U.cout)], self.hs[s], self.ws[s], 2, TAPS_UP, U.wb, U.cin,
                   [(dst, U.cin, False, False)], H, W)
        _check(lib.pat_gconv(ctypes.byref(d), st), "pat_gconv")

    def backward(self, k, planes, scales, g_out, g_planes, g_residual, acc, st):
        """g_out: gradient of the block output (planar).  Writes
        g_planes[c] = g_residual[c] + d loss / d plane_c (None = not needed);
        parameter gradients accumulate if acc."""
        lib = self.lib
        a = int(acc)
        gA, gB, gS, gup = self.gA, self.gB, self.gS, self.gup
        _check(lib.pat_head_backward(self.rows[0], WIDTHS[0], _p(self.a["d0c2"][k]), _p(self.head_w), _p(g_out),
                                     _p(gA[0]), _p(self.head_gw), a, _p(self.bn_part), st), "pat_head_backward")
        top = gA[0]
        for s in (0, 1, 2):
            c = WIDTHS[s]
            self._conv_bwd("d%dc2" % s, k, top, [(gB[s], c, False, False)], acc, st)
            self._conv_bwd("d%dc1" % s, k, gB[s], [(gS[s], c, False, False), (gup[s], c, True, False)], acc, st)
            self._up_bwd(s, k, gA[s + 1], acc, st)
            top = gA[s + 1]
        self._conv_bwd("e3c2", k, gA[3], [(gB[3], WIDTHS[3], False, False)], acc, st)
        for s in (3, 2, 1):
            # the input gradient of e{s}c1 is the gradient of the pooled map
            # (WIDTHS[s-1] channels at scale s), routed back into the skip
            # gradient of scale s - 1
            self._conv_bwd("e%dc1" % s, k, gB[s], [(gA[s], WIDTHS[s - 1], False, False)], acc, st)
            _check(lib.pat_maxpool2_backward(self.B, self.hs[s - 1], self.ws[s - 1], WIDTHS[s - 1],
                                             _p(self.a["e%dc2" % (s - 1)][k]), _p(gA[s]), _p(gS[s - 1]), st),
                   "pat_maxpool2_backward")
            self._conv_bwd("e%dc2" % (s - 1), k, gS[s - 1], [(gB[s - 1], WIDTHS[s - 1], False, False)], acc, st)
        self._conv_bwd("e0c1", k, gB[0], [(self.gx0, CPAD, False, False)], acc, st)
        sca = (ctypes.c_float * 4)(*([float(v) for v in scales] + [1.0] * (4 - len(scales))))
        gp = (ctypes.c_void_p * 4)(*([_p(t) for t in g_planes] + [None] * (4 - len(g_planes))))
        rp = (ctypes.c_void_p * 4)(*([_p(t) for t in g_residual] + [None] * (4 - len(g_residual))))
        _check(lib.pat_nhwc_unpack_grad(self.rows[0], self.cin, CPAD, _p(self.gx0), sca, gp, rp, st),
               "pat_nhwc_unpack_grad")
