"""GPU parity of the U-Net kernels (pat_gconv, pat_gconv_wgrad, batch
normalisation, max pooling, input packing, head) and of a whole U-Net's
forward and backward against the FP64 oracle (oracle/unet.py).

Unit tests feed bf16-representable operands, so both sides multiply the same
numbers and differ only by FP32 versus FP64 accumulation (relative 1e-5 of
the largest entry).  bf16 outputs are compared within one bf16 rounding
(2^-8 relative).  The whole network is compared with the oracle in its bf16
storage mode.  There the two sides agree only statistically: FP32 versus FP64
accumulation flips a few bf16 roundings, and each flipped value perturbs
~sqrt(9 C) values of the next layer enough to flip their roundings too, so
flips multiply through the 14 batch-normalised layers until the GPU result is
another draw of the same bf16 rounding noise (measured: with batch-norm shifts
of +2, where ReLU masks rarely flip, the GPU is 0.99 % from the rounded oracle
and the rounded oracle 0.92 % from the unrounded one).  Flips also move ReLU
masks and max-pooling choices, which reroute gradients by O(1) amounts, so
with zero shifts the bf16 effect on gradients is ~36 %.  The bar is measured
on the oracle side alone: an ensemble of rounded oracle runs whose
convolution products (and, in the unrolled network, operator outputs) carry
seeded relative noise at FP32 level (oracle.lpd.Perturb: 1e-7 and 1e-6),
each compared with the unperturbed run.  The GPU is one more such draw, so
every compared quantity must lie within twice the largest distance of the
ensemble (twice covers the sampling error of a maximum over the draws), or
within FLOOR = 1e-5 for quantities that the flips cannot reach (the head's
bias gradient is a plain sum, equal in every draw): FP32 against FP64
accumulation, the bar of the unit tests.  The shifted case is the
discriminating one: a wrong connection, term or sign gives O(1) errors
there."""
import ctypes

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle as O
import oracle.unet as OU
from oracle import lpd as OL
from oracle.lpd import bf16 as obf16
from paper_2510_24687_amd import lpd as LPDM
from paper_2510_24687_amd import pat
from paper_2510_24687_amd import phantoms as PH
from paper_2510_24687_amd import unet as UN

pytestmark = pytest.mark.gpu

DEV = "cuda"
FLOOR = 1e-5  # FP32 vs FP64 accumulation: the floor under every ensemble-derived bar


def within(err, spread):
    """The GPU's distance against twice the ensemble's largest, never below FLOOR."""
    return err < max(2 * spread, FLOOR)


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return pat.load()


def st():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def bfrand(shape, gen, scale=1.0):
    """bf16-representable values: (float64 CPU copy, int16 device storage)."""
    x = (torch.randn(shape, generator=gen, dtype=torch.float32) * scale).to(torch.bfloat16)
    return x.to(torch.float64), x.view(torch.int16).to(DEV)


def from_bf(t16):
    return t16.cpu().view(torch.bfloat16).to(torch.float64)


def nchw(t):
    return t.permute(0, 3, 1, 2)


def nhwc(t):
    return t.permute(0, 2, 3, 1)


def rel_max(got, ref):
    return float((got - ref).abs().max() / ref.abs().max())


def pack(lib, w, co_e, ci_e, cout, cip, ntaps, off, s_co, s_ci, s_t, flip):
    dst = torch.empty(lib.pat_gconv_packed_size(cout, cip, ntaps), dtype=torch.int16, device=DEV)
    rc = lib.pat_gconv_pack(w.data_ptr(), co_e, ci_e, cout, cip, ntaps, off, s_co, s_ci, s_t, flip, dst.data_ptr(), st())
    assert rc == 0, lib.pat_last_error()
    return dst


def run(lib, d):
    rc = lib.pat_gconv(ctypes.byref(d), st())
    assert rc == 0, lib.pat_last_error()


@pytest.mark.parametrize("c0,c1,co", [(32, 16, 48), (64, 32, 64)])
def test_gconv_3x3_two_sources_split_destinations(lib, c0, c1, co):
    """(32, 16): the 16-deep instruction path; (64, 32): the 32-deep one."""
    g = torch.Generator().manual_seed(0)
    B, H, W = 2, 12, 20                                   # 480 rows: 7.5 tiles of 64
    x0, x0d = bfrand((B, H, W, c0), g)
    x1, x1d = bfrand((B, H, W, c1), g)
    w = torch.randn((co, c0 + c1, 3, 3), generator=g) * 0.1
    wd = w.to(DEV)
    wf = pack(lib, wd, co, c0 + c1, co, c0 + c1, 9, 0, (c0 + c1) * 9, 9, 1, 0)
    out0 = torch.full((B, H, W, 32), 0.5, device=DEV)
    out1 = torch.empty((B, H, W, co - 32), dtype=torch.int16, device=DEV)
    d = UN._gdesc(B, H, W, [(x0d, c0), (x1d, c1)], H, W, 1, UN.TAPS3, wf, co,
                  [(out0, 32, False, True), (out1, co - 32, True, False)], H, W)
    run(lib, d)
    ref = nhwc(F.conv2d(nchw(torch.cat([x0, x1], dim=3)), obf16(w.double()), padding=1))
    got0 = out0.cpu().double() - 0.5
    assert rel_max(got0, ref[..., :32]) < 1e-5
    got1 = from_bf(out1)
    assert float(((got1 - ref[..., 32:]).abs() / ref[..., 32:].abs().clamp_min(1e-3)).max()) < 2 ** -8


@pytest.mark.parametrize("B,H,W,c0,c1,co", [(2, 13, 128, 32, 32, 64), (1, 20, 96, 64, 0, 32), (3, 7, 48, 32, 0, 96),
                                              (2, 9, 64, 128, 128, 128)])
def test_gconv_3x3_lds_tiles(lib, B, H, W, c0, c1, co):
    """The LDS-tiled 3x3 path (W divisible by 16, 32-multiple channels): tile
    widths 64 / 32 / 16, rows that do not fill the last tile, one or two
    sources, 2 or 4 column tiles per block, split destinations."""
    g = torch.Generator().manual_seed(H * W + co)
    x0, x0d = bfrand((B, H, W, c0), g)
    srcs, xs = [(x0d, c0)], x0
    if c1:
        x1, x1d = bfrand((B, H, W, c1), g)
        srcs, xs = [(x0d, c0), (x1d, c1)], torch.cat([x0, x1], dim=3)
    ci = c0 + c1
    w = torch.randn((co, ci, 3, 3), generator=g) * 0.1
    wf = pack(lib, w.to(DEV), co, ci, co, ci, 9, 0, ci * 9, 9, 1, 0)
    d0 = co - 16
    out0 = torch.full((B, H, W, d0), -0.25, device=DEV)
    out1 = torch.empty((B, H, W, 16), dtype=torch.int16, device=DEV)
    run(lib, UN._gdesc(B, H, W, srcs, H, W, 1, UN.TAPS3, wf, co, [(out0, d0, False, True), (out1, 16, True, False)],
                       H, W))
    ref = nhwc(F.conv2d(nchw(xs), obf16(w.double()), padding=1))
    assert rel_max(out0.cpu().double() + 0.25, ref[..., :d0]) < 1e-5
    got1 = from_bf(out1)
    assert float(((got1 - ref[..., d0:]).abs() / ref[..., d0:].abs().clamp_min(1e-3)).max()) < 2 ** -8


def test_gconv_input_gradient_is_the_transposed_convolution(lib):
    g = torch.Generator().manual_seed(1)
    B, H, W, cin, co = 2, 8, 24, 3, 32                   # first-layer shape: 3 real inputs padded to 16
    gz, gzd = bfrand((B, H, W, co), g)
    w = torch.randn((co, cin, 3, 3), generator=g) * 0.2
    wb = pack(lib, w.to(DEV), cin, co, 16, co, 9, 0, 9, cin * 9, 1, 1)
    gx = torch.empty((B, H, W, 16), device=DEV)
    run(lib, UN._gdesc(B, H, W, [(gzd, co)], H, W, 1, UN.TAPS3, wb, 16, [(gx, 16, False, False)], H, W))
    ref = nhwc(F.conv_transpose2d(nchw(gz), obf16(w.double()), padding=1))
    got = gx.cpu().double()
    assert rel_max(got[..., :cin], ref) < 1e-5
    assert float(got[..., cin:].abs().max()) == 0.0


def test_transposed_convolution_forward_backward_and_weight_gradient(lib):
    g = torch.Generator().manual_seed(2)
    B, H, W, cin, co = 2, 4, 6, 64, 32                    # up-sampling 64 -> 32 channels, 4x6 -> 8x12
    x, xd = bfrand((B, H, W, cin), g)
    w = torch.randn((cin, co, 2, 2), generator=g) * 0.1
    wd = w.to(DEV)
    up = torch.empty((B, 2 * H, 2 * W, co), dtype=torch.int16, device=DEV)
    for p in range(4):
        wf = pack(lib, wd, co, cin, co, cin, 1, p, 4, co * 4, 0, 0)
        run(lib, UN._gdesc(B, H, W, [(xd, cin)], H, W, 1, [(0, 0)], wf, co, [(up, co, True, False)],
                           2 * H, 2 * W, 2, p // 2, p % 2))
    ref = nhwc(F.conv_transpose2d(nchw(x), obf16(w.double()), stride=2))
    got = from_bf(up)
    assert float(((got - ref).abs() / ref.abs().clamp_min(1e-3)).max()) < 2 ** -8
    # input gradient: 4 taps read at stride 2
    gy, gyd = bfrand((B, 2 * H, 2 * W, co), g)
    wb = pack(lib, wd, cin, co, cin, co, 4, 0, co * 4, 4, 1, 0)
    gx = torch.empty((B, H, W, cin), device=DEV)
    run(lib, UN._gdesc(B, H, W, [(gyd, co)], 2 * H, 2 * W, 2, UN.TAPS_UP, wb, cin, [(gx, cin, False, False)], H, W))
    refx = nhwc(F.conv2d(nchw(gy), obf16(w.double()), stride=2))
    assert rel_max(gx.cpu().double(), refx) < 1e-5
    # weight gradient, one parity at a time, into w's own layout
    gw = torch.zeros((cin, co, 2, 2), device=DEV)
    for p in range(4):
        d = UN._gdesc(B, H, W, [(xd, cin)], H, W, 1, [(0, 0)], wb, co, [], 2 * H, 2 * W, 2, p // 2, p % 2)
        part = torch.empty(lib.pat_gconv_wgrad_partials(ctypes.byref(d), 3), device=DEV)
        rc = lib.pat_gconv_wgrad(ctypes.byref(d), gyd.data_ptr(), 3, part.data_ptr(), gw.data_ptr(), cin, p, 4, co * 4,
                                 0, 0, st())
        assert rc == 0, lib.pat_last_error()
    g6 = nchw(gy).reshape(B, co, H, 2, W, 2)
    refw = torch.einsum("bchw,bdhiwj->cdij", nchw(x), g6)
    assert rel_max(gw.cpu().double(), refw) < 1e-5


@pytest.mark.parametrize("shape", [(2, 10, 14, 16, 32, 1), (3, 16, 8, 64, 64, 1), (2, 6, 10, 32, 16, 2)])
def test_3x3_weight_gradient(lib, shape):
    B, H, W, cin, co, nsrc = shape
    g = torch.Generator().manual_seed(3 + cin)
    x, xd = bfrand((B, H, W, cin), g)
    gz, gzd = bfrand((B, H, W, co), g)
    if nsrc == 2:       # concatenated sources [x | x2]
        x2, x2d = bfrand((B, H, W, cin), g)
        srcs, xs, ct = [(xd, cin), (x2d, cin)], torch.cat([x, x2], dim=3), 2 * cin
    else:
        srcs, xs, ct = [(xd, cin)], x, cin
    real = 3 if cin == 16 else ct                         # 16 = a padded first-layer input with 3 real channels
    gw = torch.full((co, real, 3, 3), 0.25, device=DEV)
    d = UN._gdesc(B, H, W, srcs, H, W, 1, UN.TAPS3, gzd, co, [], H, W)
    for chunks in (1, 5):
        part = torch.empty(lib.pat_gconv_wgrad_partials(ctypes.byref(d), chunks), device=DEV)
        rc = lib.pat_gconv_wgrad(ctypes.byref(d), gzd.data_ptr(), chunks, part.data_ptr(), gw.data_ptr(), real, 0,
                                 real * 9, 9, 1, 1, st())
        assert rc == 0, lib.pat_last_error()
    refw = torch.nn.grad.conv2d_weight(nchw(xs[..., :real]), (co, real, 3, 3), nchw(gz), padding=1)
    assert rel_max(gw.cpu().double() - 0.25, 2 * refw) < 1e-5


def test_batch_norm_forward_backward(lib):
    g = torch.Generator().manual_seed(4)
    B, H, W, C = 2, 12, 10, 64
    R = B * H * W
    z = torch.randn((B, H, W, C), generator=g) * 1.7 + 0.4
    gamma = 1 + 0.2 * torch.randn(C, generator=g)
    beta = 0.3 * torch.randn(C, generator=g)
    ga = torch.randn((B, H, W, C), generator=g)
    zd, gmd, btd, gad = (t.to(DEV) for t in (z, gamma, beta, ga))
    mean, inv = torch.empty(C, device=DEV), torch.empty(C, device=DEV)
    rm, rv = torch.zeros(C, device=DEV), torch.ones(C, device=DEV)
    out = torch.empty((B, H, W, C), dtype=torch.int16, device=DEV)
    part = torch.empty(lib.pat_bn_partials(R, C), dtype=torch.float64, device=DEV)
    rc = lib.pat_bn_forward(R, C, zd.data_ptr(), gmd.data_ptr(), btd.data_ptr(), mean.data_ptr(), inv.data_ptr(),
                            rm.data_ptr(), rv.data_ptr(), 0.1, 1e-5, 1, out.data_ptr(), part.data_ptr(), st())
    assert rc == 0, lib.pat_last_error()
    zt = nchw(z.double()).requires_grad_(True)
    gt, bt = gamma.double().requires_grad_(True), beta.double().requires_grad_(True)
    run_ = {"mean": torch.zeros(C, dtype=torch.float64), "var": torch.ones(C, dtype=torch.float64)}
    y = OU.batch_norm_relu(zt, gt, bt, run_, training=True)
    got = from_bf(out)
    ref = nhwc(y.detach())
    assert float((got - ref).abs().max()) <= 2 ** -8 * float(ref.abs().max())
    assert rel_max(rm.cpu().double(), run_["mean"]) < 1e-6 and rel_max(rv.cpu().double(), run_["var"]) < 1e-6
    # backward
    (y * nchw(ga.double())).sum().backward()
    gz = torch.empty((B, H, W, C), dtype=torch.int16, device=DEV)
    dg, db = torch.zeros(C, device=DEV), torch.zeros(C, device=DEV)
    rc = lib.pat_bn_backward(R, C, zd.data_ptr(), gad.data_ptr(), gmd.data_ptr(), btd.data_ptr(), mean.data_ptr(),
                             inv.data_ptr(), gz.data_ptr(), dg.data_ptr(), db.data_ptr(), 0, part.data_ptr(), st())
    assert rc == 0, lib.pat_last_error()
    refz = nhwc(zt.grad)
    assert float((from_bf(gz) - refz).abs().max()) <= 2 ** -7 * float(refz.abs().max())
    assert rel_max(dg.cpu().double(), gt.grad) < 1e-5 and rel_max(db.cpu().double(), bt.grad) < 1e-5
    # inference with the running statistics
    out_e = torch.empty_like(out)
    rc = lib.pat_bn_forward(R, C, zd.data_ptr(), gmd.data_ptr(), btd.data_ptr(), mean.data_ptr(), inv.data_ptr(),
                            rm.data_ptr(), rv.data_ptr(), 0.1, 1e-5, 0, out_e.data_ptr(), None, st())
    assert rc == 0, lib.pat_last_error()
    ref_e = nhwc(OU.batch_norm_relu(nchw(z.double()), gamma.double(), beta.double(), run_, training=False))
    assert float((from_bf(out_e) - ref_e).abs().max()) <= 2 ** -8 * float(ref_e.abs().max())


def test_max_pooling_exact(lib):
    g = torch.Generator().manual_seed(5)
    B, H, W, C = 2, 8, 12, 32
    x, xd = bfrand((B, H, W, C), g)
    xd_relu = torch.clamp(x, min=0.0)                   # ReLU outputs: many exact ties at 0
    xr = xd_relu.to(torch.float32).to(torch.bfloat16).view(torch.int16).to(DEV)
    out = torch.empty((B, H // 2, W // 2, C), dtype=torch.int16, device=DEV)
    assert lib.pat_maxpool2(B, H, W, C, xr.data_ptr(), out.data_ptr(), st()) == 0
    xt = nchw(xd_relu).clone().requires_grad_(True)
    ref = OU.maxpool2(xt)
    assert torch.equal(from_bf(out), nhwc(ref.detach()))
    go = torch.randn((B, H // 2, W // 2, C), generator=g)
    gin0 = torch.randn((B, H, W, C), generator=g)
    gin = gin0.to(DEV)
    assert lib.pat_maxpool2_backward(B, H, W, C, xr.data_ptr(), go.to(DEV).data_ptr(), gin.data_ptr(), st()) == 0
    (ref * nchw(go.double())).sum().backward()
    assert torch.equal(gin.cpu(), (gin0.double() + nhwc(xt.grad)).float())


def test_input_packing_and_head(lib):
    g = torch.Generator().manual_seed(6)
    B, H, W = 2, 8, 16
    R = B * H * W
    planes = [torch.randn((B, H, W), generator=g) for _ in range(3)]
    pd = [p.to(DEV) for p in planes]
    scales = [1.0, 0.5, 3.0]
    x0 = torch.empty((B, H, W, 16), dtype=torch.int16, device=DEV)
    vp = (ctypes.c_void_p * 4)(*[p.data_ptr() for p in pd], None)
    sc = (ctypes.c_float * 4)(*scales, 1.0)
    assert lib.pat_nhwc_pack(R, 3, 16, vp, sc, x0.data_ptr(), st()) == 0
    ref = torch.stack([obf16(planes[c].double() * scales[c]) for c in range(3)], dim=3)
    got = from_bf(x0)
    assert torch.equal(got[..., :3], ref) and float(got[..., 3:].abs().max()) == 0.0
    # unpack of a gradient, with a residual on plane 0 and plane 2 skipped
    gx = torch.randn((B, H, W, 16), generator=g)
    res = torch.randn((B, H, W), generator=g)
    outs = [torch.empty((B, H, W), device=DEV) for _ in range(2)]
    gp = (ctypes.c_void_p * 4)(outs[0].data_ptr(), outs[1].data_ptr(), None, None)
    resd = res.to(DEV)
    rp = (ctypes.c_void_p * 4)(resd.data_ptr(), None, None, None)
    assert lib.pat_nhwc_unpack_grad(R, 3, 16, gx.to(DEV).data_ptr(), sc, gp, rp, st()) == 0
    assert torch.allclose(outs[0].cpu(), res + 1.0 * gx[..., 0], rtol=1e-6, atol=1e-6)
    assert torch.allclose(outs[1].cpu(), 0.5 * gx[..., 1], rtol=1e-6, atol=1e-6)
    # head: 1x1 convolution 32 -> 1 with bias and residual, and its backward
    act, actd = bfrand((B, H, W, 32), g)
    w = torch.randn(32, generator=g) * 0.3
    b = torch.tensor([0.7])
    out = torch.empty((B, H, W), device=DEV)
    assert lib.pat_head_forward(R, 32, actd.data_ptr(), w.to(DEV).data_ptr(), b.to(DEV).data_ptr(), resd.data_ptr(),
                                out.data_ptr(), st()) == 0
    refh = res.double() + 0.7 + (act * w.double()).sum(dim=3)
    assert rel_max(out.cpu().double(), refh) < 1e-5
    go = torch.randn((B, H, W), generator=g)
    gact = torch.empty((B, H, W, 32), device=DEV)
    gwb = torch.full((33,), 1.0, device=DEV)
    part = torch.empty(lib.pat_head_partials(R, 32), dtype=torch.float64, device=DEV)
    assert lib.pat_head_backward(R, 32, actd.data_ptr(), w.to(DEV).data_ptr(), go.to(DEV).data_ptr(),
                                 gact.data_ptr(), gwb.data_ptr(), 1, part.data_ptr(), st()) == 0
    assert torch.allclose(gact.cpu(), w * go[..., None], rtol=1e-6, atol=1e-7)
    refw = (act * go.double()[..., None]).sum(dim=(0, 1, 2))
    assert rel_max(gwb.cpu().double()[:32] - 1.0, refw) < 1e-5
    assert abs(float(gwb[32]) - 1.0 - float(go.double().sum())) < 1e-4 * float(go.abs().sum())


# ---- whole network ------------------------------------------------------------

def _block(lib, cin, B, H, W, seed, train=True, shift=0.0):
    layout = LPDM.param_layout(arch="unet")
    offs, o = {}, 0
    for name, shape in layout:
        offs[name] = o
        o += int(np.prod(shape))
    p0 = LPDM.init_params(seed, arch="unet")
    rng = np.random.default_rng(seed + 1)
    for name, shape in layout:           # perturb g, b and the head so that every path carries signal
        size = int(np.prod(shape))
        if name.endswith(".g"):
            p0[offs[name]:offs[name] + size] += 0.1 * rng.standard_normal(size).astype(np.float32)
        elif name.endswith(".b"):
            p0[offs[name]:offs[name] + size] = shift + 0.1 * rng.standard_normal(size).astype(np.float32)
        elif name.endswith("head.w"):
            p0[offs[name]:offs[name] + size] *= 10.0
    params = torch.tensor(p0, device=DEV)
    grads = torch.zeros_like(params)
    soffs, so = {}, 0
    for name, c in UN.stats_layout(1):
        soffs[name] = so
        so += c
    stats = torch.tensor(UN.init_stats(1), device=DEV)
    net = "dual" if cin == 3 else "primal"
    blk = UN.UNetBlock(lib, params, grads, offs, dict(layout), stats, soffs, net, cin, B, H, W, 1, DEV, train)
    return blk, params, grads, stats, offs, soffs, dict(layout), net


def _oracle_params(p0, offs, shapes, net, requires_grad=True):
    P = {}
    for name, shape in shapes.items():
        if name.startswith(net + "."):
            size = int(np.prod(shape))
            v = torch.tensor(p0[offs[name]:offs[name] + size].reshape(shape), dtype=torch.float64)
            P[name] = v.requires_grad_(requires_grad)
    return P


@pytest.mark.parametrize("cin,B,H,W,shift", [(2, 2, 32, 32, 0.0), (3, 2, 48, 24, 0.0), (2, 2, 32, 32, 2.0),
                                             (2, 1, 256, 256, 2.0), (3, 1, 512, 256, 2.0)])
def test_unet_forward_backward_against_the_oracle(lib, cin, B, H, W, shift):
    """shift: every batch-normalisation shift beta raised by this much, so that
    ReLU masks rarely sit near a flip (a less chaotic regime, tighter bar).
    The 256 x 256 (primal) and 512 x 256 (dual) cases are the networks of the
    time-to-PSNR workload at their real sizes, on the LDS-tiled path."""
    blk, params, grads, stats, offs, soffs, shapes, net = _block(lib, cin, B, H, W, seed=10 + cin, shift=shift)
    g = torch.Generator().manual_seed(20 + cin)
    planes = [torch.randn((B, H, W), generator=g) for _ in range(cin)]
    scales = [1.0, 0.7, 1.3][:cin]
    res = torch.randn((B, H, W), generator=g)
    gout = torch.randn((B, H, W), generator=g)
    pd = [p.to(DEV) for p in planes]
    resd, goutd = res.to(DEV), gout.to(DEV)
    out = torch.empty((B, H, W), device=DEV)
    for layer in blk.layers():
        layer.pack(lib, st())
    blk.forward(0, pd, scales, resd, out, st())
    gpl = [torch.empty((B, H, W), device=DEV) for _ in range(cin)]
    blk.backward(0, pd, scales, goutd, gpl, [None] * cin, False, st())
    torch.cuda.synchronize()
    p0 = params.cpu().numpy()

    def oracle(perturb=None):
        P = _oracle_params(p0, offs, shapes, net)
        xs = [planes[c].double().requires_grad_(True) for c in range(cin)]
        x = torch.stack([scales[c] * xs[c] for c in range(cin)], dim=1)
        running = {net + "." + k: v for k, v in OU.fresh_running().items()}
        y = OU.unet(x, P, net + ".", running, training=True, rounding=True, perturb=perturb)[:, 0] + res.double()
        (y * gout.double()).sum().backward()
        return y.detach(), P, xs, running

    def gradients(P):
        return {name: P[name].grad.numpy().ravel() for name in P}

    y_r, P_r, xs_r, run_r = oracle()
    g_r = gradients(P_r)
    rel = lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    nrel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
    allr = np.concatenate([g_r[k] for k in P_r])
    # the FP32-noise ensemble of the rounded oracle (fewer draws at the full sizes)
    draws = 8 if H * W <= 4096 else 3
    s_out, s_g, s_blk, s_x = 0.0, 0.0, {k: 0.0 for k in P_r}, [0.0] * cin
    for d in range(draws):
        y_p, P_p, xs_p, _ = oracle(OL.Perturb(2000 + d, op=0.0, conv=1e-7))
        g_p = gradients(P_p)
        s_out = max(s_out, rel(y_p - res.double(), y_r - res.double()))
        s_g = max(s_g, nrel(np.concatenate([g_p[k] for k in P_r]), allr))
        for k in P_r:
            s_blk[k] = max(s_blk[k], nrel(g_p[k], g_r[k]))
        for c in range(cin):
            s_x[c] = max(s_x[c], rel(xs_p[c].grad, xs_r[c].grad))
    e_out = rel(out.cpu().double() - res.double(), y_r - res.double())
    print("output: gpu vs oracle %.3e, flip spread %.3e" % (e_out, s_out))
    # running statistics
    e_stats = 0.0
    for name, c in UN.bn_layers():
        o = soffs[net + ".it0." + name + ".mean"]
        e_stats = max(e_stats, rel_max(stats[o:o + c].cpu().double(), run_r[net + "." + name]["mean"]))
    print("running means: max relative deviation %.3e" % e_stats)
    # parameter gradients, whole vector and per tensor
    gcpu = grads.cpu().double().numpy()
    gg, blocks = [], {}
    for name in P_r:
        size = int(np.prod(shapes[name]))
        gg.append(gcpu[offs[name]:offs[name] + size])
        blocks[name] = (nrel(gg[-1], g_r[name]), s_blk[name])
    worst = sorted(blocks.items(), key=lambda kv: -kv[1][0] / max(kv[1][1], 1e-30))[:5]
    print("worst blocks (gpu, flip spread):", ["%s %.2e %.2e" % (k, a, b) for k, (a, b) in worst])
    e_g = nrel(np.concatenate(gg), allr)
    print("parameter gradient: gpu vs oracle %.3e, flip spread %.3e" % (e_g, s_g))
    ex = []
    for c in range(cin):
        e_x = rel(gpl[c].cpu().double(), xs_r[c].grad)
        ex.append((e_x, s_x[c]))
        print("input gradient %d: gpu vs oracle %.3e, flip spread %.3e" % (c, e_x, s_x[c]))
    # see the module docstring: within twice the ensemble's largest distance
    assert within(e_out, s_out)
    assert e_stats < 5e-2
    assert within(e_g, s_g)
    for name, (a, b) in blocks.items():
        assert within(a, b), (name, a, b)
    for e_x, s in ex:
        assert within(e_x, s)


def test_unet_forward_backward_is_bit_reproducible(lib):
    """No atomics and fixed summation orders: two runs of the same forward
    and backward give identical outputs, input gradients, parameter
    gradients and running statistics."""
    B, H, W, cin = 2, 64, 32, 2
    g = torch.Generator().manual_seed(99)
    planes = [torch.randn((B, H, W), generator=g).to(DEV) for _ in range(cin)]
    res = torch.randn((B, H, W), generator=g).to(DEV)
    gout = torch.randn((B, H, W), generator=g).to(DEV)
    results = []
    for _ in range(2):
        blk, params, grads, stats, *_ = _block(lib, cin, B, H, W, seed=5, shift=0.5)
        for layer in blk.layers():
            layer.pack(lib, st())
        out = torch.empty((B, H, W), device=DEV)
        blk.forward(0, planes, [1.0, 0.8], res, out, st())
        gpl = [torch.empty((B, H, W), device=DEV) for _ in range(cin)]
        blk.backward(0, planes, [1.0, 0.8], gout, gpl, [None] * cin, False, st())
        torch.cuda.synchronize()
        results.append([out.clone(), grads.clone(), stats.clone()] + [t.clone() for t in gpl])
    for a, b in zip(*results):
        assert torch.equal(a, b)


# ---- the learned primal-dual reconstructor with U-Nets -------------------------

def _rel(a, b):
    a, b = np.ravel(np.asarray(a, dtype=np.float64)), np.ravel(np.asarray(b, dtype=np.float64))
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _cuda32(x):
    return torch.tensor(np.asarray(x, dtype=np.float32), device=DEV)


def _tiny(K):
    """n = 16 on a 180-degree arc with m = 16, nt = 32 (the dual U-Net runs on
    32 x 16 traces, the primal on 16 x 16 images), batch 2."""
    geom = PH.top_arc(16, 16, 32, 180.0)
    plan = pat.Plan(geom, torch.float32, max_batch=2)
    f_true = PH.ellipse_batch(16, [21, 22])
    y = np.stack([PH.add_noise(O.forward(geom, fi), 0.02, 30 + i) for i, fi in enumerate(f_true)])
    params = LPDM.init_params(9, arch="unet")
    Pd = LPDM.unpack(params, arch="unet")
    for k in ("dual.head.w", "primal.head.w"):      # visible gradients in every layer
        Pd[k][...] *= 10
    for k in Pd:                                    # ReLU masks away from their flips (see the module docstring)
        if k.endswith(".b"):
            Pd[k][...] = 2.0
    params = np.concatenate([Pd[k].ravel() for k, _ in LPDM.param_layout(arch="unet")]).astype(np.float32)
    return geom, plan, f_true.astype(np.float32), y.astype(np.float32), params


def _oracle_running(K):
    """Per unrolled iteration, fresh running statistics of both networks."""
    return [{net + "." + k: v for net in ("dual", "primal") for k, v in OU.fresh_running().items()}
            for _ in range(K)]


def _running_from(stats_np, K):
    run = [{} for _ in range(K)]
    o = 0
    for name, c in UN.stats_layout(K):
        net_, it, layer, kind = name.split(".")
        run[int(it[2:])].setdefault(net_ + "." + layer, {})[kind] = torch.tensor(stats_np[o:o + c].astype(np.float64))
        o += c
    return run


def test_unet_lpd_loss_gradient_against_the_oracle():
    """f_K, the loss and the whole parameter gradient of K = 2 unrolled
    iterations with U-Nets (batch-norm shifts +2) against the oracle run on
    its own A / A* with the same bf16 storage.  Roundings that flip between
    the two sides feed forward (module docstring), so the bar is the spread
    of an FP32-noise ensemble of the rounded oracle (8 draws): f_K, the loss,
    the whole gradient and each block within twice its largest distance."""
    K = 2
    geom, plan, f_true, y, params = _tiny(K)
    s_A, s_U = 0.9, 1.7
    net = LPDM.LPD(plan, 2, iters=K, params=params, s_A=s_A, s_U=s_U, arch="unet")
    net.set_batch(_cuda32(y), _cuda32(f_true))
    net.forward_pass()
    net.backward_pass()
    torch.cuda.synchronize()
    Pd = {k: v.astype(np.float64) for k, v in LPDM.unpack(params, arch="unet").items()}
    run_o = _oracle_running(K)
    loss_o, fK_o, g_o = OL.loss_and_grads(geom, Pd, y, f_true, K, s_A, s_U, rounding=True, arch="unet",
                                          running=run_o)
    allo = np.concatenate([np.ravel(g_o[k]) for k in g_o])
    s_l, s_f, s_g, s_blk = 0.0, 0.0, 0.0, {k: 0.0 for k in g_o}
    for d in range(8):
        l_p, f_p, g_p = OL.loss_and_grads(geom, Pd, y, f_true, K, s_A, s_U, rounding=True, arch="unet",
                                          running=_oracle_running(K), perturb=OL.Perturb(3000 + d))
        s_l = max(s_l, abs(l_p - loss_o) / loss_o)
        s_f = max(s_f, _rel(f_p, fK_o))
        s_g = max(s_g, _rel(np.concatenate([np.ravel(g_p[k]) for k in g_o]), allo))
        for k in g_o:
            s_blk[k] = max(s_blk[k], _rel(g_p[k], g_o[k]))
    grads = LPDM.unpack(net.grads.cpu().numpy(), arch="unet")
    fK = net.f[K].cpu().numpy()
    e_f = _rel(fK, fK_o)
    allg = np.concatenate([np.ravel(grads[k]) for k in g_o])
    print("K=%d f_K: gpu %.2e, flip spread %.2e; gradient: gpu %.2e, flip spread %.2e"
          % (K, e_f, s_f, _rel(allg, allo), s_g))
    assert within(e_f, s_f)
    assert within(abs(net.loss() - loss_o) / loss_o, s_l)
    assert within(_rel(allg, allo), s_g)
    for k in g_o:
        e = _rel(grads[k], g_o[k])
        assert within(e, s_blk[k]), (k, e, s_blk[k])
    # running statistics of every iteration after one application each
    got = _running_from(net.stats.cpu().numpy(), K)
    for k in range(K):
        for key, v in run_o[k].items():
            for kind in ("mean", "var"):
                assert _rel(got[k][key][kind].numpy(), v[kind].numpy()) < 5e-2, (k, key, kind)


def test_unet_lpd_graph_replay_and_inference():
    """Captured training steps equal eager ones (parameters and running
    statistics bit for bit); the inference network (running statistics) equals
    the oracle's inference mode and its replayed graph equals its eager pass."""
    K = 2
    geom, plan, f_true, y, params = _tiny(K)
    a = LPDM.LPD(plan, 2, iters=K, params=params, arch="unet")
    b = LPDM.LPD(plan, 2, iters=K, params=params, arch="unet")
    for net in (a, b):
        net.opt.update(lr=1e-3, total=10)
        net.set_batch(_cuda32(y), _cuda32(f_true))
    for _ in range(3):
        a.train_step()
    b.capture_train()
    for _ in range(3):
        b.graph_train.replay()
    torch.cuda.synchronize()
    assert torch.equal(a.params, b.params) and torch.equal(a.stats, b.stats)
    # inference with the trained weights and running statistics
    inf = LPDM.LPD(plan, 2, iters=K, params=a.params.cpu().numpy(), stats=a.stats.cpu().numpy(), train=False,
                   arch="unet")
    inf.set_batch(_cuda32(y))
    f_e = inf.forward_pass().clone()
    torch.cuda.synchronize()
    Pd = {k: v.astype(np.float64) for k, v in LPDM.unpack(a.params.cpu().numpy(), arch="unet").items()}
    run = _running_from(a.stats.cpu().numpy(), K)
    Pt = {k: torch.tensor(v) for k, v in Pd.items()}
    yt = torch.tensor(y.astype(np.float64))
    with torch.no_grad():
        f_o = OL.reconstruct(geom, Pt, yt, K, rounding=True, arch="unet", running=run, training=False).numpy()
        spread = max(_rel(OL.reconstruct(geom, Pt, yt, K, rounding=True, arch="unet", running=run, training=False,
                                         perturb=OL.Perturb(4000 + d)).numpy(), f_o) for d in range(8))
    e = _rel(f_e.cpu().numpy(), f_o)
    print("inference f_K: gpu %.2e, flip spread %.2e" % (e, spread))
    assert within(e, spread)
    inf.capture_forward()
    for _ in range(2):
        inf.f[K].zero_()
        torch.cuda.synchronize()
        inf.graph_fwd.replay()
        torch.cuda.synchronize()
        assert torch.equal(inf.f[K], f_e)


def test_unet_lpd_training_gains():
    """300 steps on 256 phantoms (n = 32, 180-degree arc, K = 5) raise the
    held-out PSNR of the U-Net network (inference mode, running statistics)
    well above the untrained network and above K projected-gradient steps."""
    from paper_2510_24687_amd import solvers as S
    geom = PH.top_arc(32, 32, 64, 180.0)
    plan = pat.Plan(geom, torch.float32, max_batch=16)
    ds = LPDM.make_dataset(plan, range(256), noise=0.02, noise_seed=5)
    test = LPDM.make_dataset(plan, range(10 ** 6, 10 ** 6 + 16), noise=0.02, noise_seed=6)
    s_A, s_U = LPDM.input_scales(plan, ds)
    K = 5
    net = LPDM.LPD(plan, 8, iters=K, s_A=s_A, s_U=s_U, seed=1, arch="unet")
    inf0 = LPDM.LPD(plan, 8, iters=K, params=net.params.cpu().numpy(), stats=net.stats.cpu().numpy(),
                    s_A=s_A, s_U=s_U, train=False, arch="unet")
    base = LPDM.evaluate(inf0, test)
    log = LPDM.train(net, ds, steps=300, lr=1e-3)
    inf = LPDM.LPD(plan, 8, iters=K, params=net.params.cpu().numpy(), stats=net.stats.cpu().numpy(),
                   s_A=s_A, s_U=s_U, train=False, arch="unet")
    after = LPDM.evaluate(inf, test)
    sol = S.BatchedSolver([(plan, test["y"], None)], method="nnls")
    for _ in range(K):
        sol.step()
    nnls = float(LPDM.psnr(sol.groups[0].f, test["f"]).mean())
    print("U-Net LPD: untrained %.2f dB, trained %.2f dB, NNLS(%d) %.2f dB, loss %s" % (base, after, K, nnls, log[-3:]))
    assert after > base + 8.0
    assert after > nnls + 3.0
