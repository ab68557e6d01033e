"""Learned primal-dual kernels on the GPU against the CPU oracle (oracle/lpd.py):
BF16-MFMA convolutions (forward, input gradient, weight gradient), PReLU
backward, bias sums, Adam, the whole unrolled network's loss gradient, graph
replay, and what training gains over the untrained network."""
import ctypes
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from oracle import lpd as OL  # noqa: E402
from paper_2510_24687_amd import lpd as L  # noqa: E402
from paper_2510_24687_amd import pat  # noqa: E402
from paper_2510_24687_amd import phantoms as P  # noqa: E402

pytestmark = pytest.mark.gpu

# FP32 accumulation of <= 288 bf16 x bf16 products (exact in FP32) against an
# FP64 sum of the same products: |error| <~ 288 * 2^-24 * sum |terms|.
TOL_CONV = 2e-5


def rel(a, b):
    a, b = np.ravel(np.asarray(a, dtype=np.float64)), np.ravel(np.asarray(b, dtype=np.float64))
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def st():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def cuda32(x):
    return torch.tensor(np.asarray(x, dtype=np.float32), device="cuda")


def planes_to_nchw(planes):
    return np.stack([p for p in planes], axis=1)


def nhwc_to_nchw(x):
    return np.transpose(x, (0, 3, 1, 2))


def pack(lib, w, cout, cin, transpose, in_planar):
    coe, cie = (cin, cout) if transpose else (cout, cin)
    n = lib.pat_conv_packed_size(coe, cie, int(in_planar))
    dst = torch.empty(n, dtype=torch.int16, device="cuda")
    pat._check(lib.pat_conv_pack_weights(w.data_ptr(), cout, cin, transpose, int(in_planar), dst.data_ptr(), st()),
               "pack")
    return dst


def f32(x):
    """values representable in FP32 (inputs of both sides)"""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def bfv(x):
    """values representable in bf16 (the NHWC tensors are stored as bf16)"""
    return OL.bf16(torch.tensor(np.asarray(x, dtype=np.float64))).numpy()


def cuda16(x):
    """NHWC bf16 device tensor (int16 storage) holding the bf16 values x"""
    return torch.tensor(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).view(torch.int16).to("cuda")


def host16(t):
    return t.view(torch.bfloat16).float().cpu().numpy().astype(np.float64)


# bf16 storage of an FP32 result: relative L2 of the rounding is ~2^-9 / sqrt(3)
TOL_BF16 = 3e-3


@pytest.mark.parametrize("B,H,W", [(2, 19, 300), (1, 7, 33)])
def test_conv_forward_variants_vs_oracle(B, H, W):
    lib = pat.load()
    rng = np.random.default_rng(B * 100 + W)
    # planar 3 -> NHWC 32 with input scales, bias, PReLU and pre-activation copy
    x = f32(rng.standard_normal((B, 3, H, W)))
    w1 = f32(0.3 * rng.standard_normal((32, 3, 3, 3)))
    b1 = f32(0.1 * rng.standard_normal(32))
    a1 = f32(0.2 + 0.1 * rng.random(32))
    scales = [1.0, 0.5, 2.0]
    xs = [cuda32(x[:, c]) for c in range(3)]  # kept alive: descriptors hold raw pointers
    w1g, b1g, a1g = cuda32(w1), cuda32(b1), cuda32(a1)
    out = torch.zeros((B, H, W, 32), dtype=torch.int16, device="cuda")
    pre = torch.zeros((B, H, W, 32), device="cuda")
    wf = pack(lib, w1g, 32, 3, 0, True)
    d = L._desc(B, H, W, 3, 32, True, False, xs, [out], wf, b1g, a1g, pre, scale=scales)
    pat._check(lib.pat_conv3x3(ctypes.byref(d), st()), "conv")
    xsc = x * np.array(scales).reshape(1, 3, 1, 1)
    ref_pre = OL.conv3x3(torch.tensor(xsc), torch.tensor(w1), torch.tensor(b1)).numpy()
    ref = OL.prelu(torch.tensor(ref_pre), torch.tensor(a1)).numpy()
    got_pre = pre.cpu()
    assert rel(nhwc_to_nchw(got_pre.numpy()), ref_pre) < TOL_CONV
    assert rel(nhwc_to_nchw(host16(out)), ref) < TOL_BF16
    # the stored activation is exactly the nearest-even bf16 of PReLU(pre)
    act = torch.where(got_pre > 0, got_pre, torch.tensor(a1, dtype=torch.float32) * got_pre)
    assert torch.equal(act.to(torch.bfloat16).view(torch.int16), out.cpu())
    # NHWC 32 -> NHWC 32, no bias, no activation
    h = bfv(rng.standard_normal((B, H, W, 32)))
    w2 = f32(0.1 * rng.standard_normal((32, 32, 3, 3)))
    out2 = torch.zeros((B, H, W, 32), dtype=torch.int16, device="cuda")
    w2g = cuda32(w2)
    hg = cuda16(h)
    d = L._desc(B, H, W, 32, 32, False, False, [hg], [out2], pack(lib, w2g, 32, 32, 0, False))
    pat._check(lib.pat_conv3x3(ctypes.byref(d), st()), "conv")
    ref2 = OL.conv3x3(torch.tensor(nhwc_to_nchw(h)), torch.tensor(w2)).numpy()
    assert rel(nhwc_to_nchw(host16(out2)), ref2) < TOL_BF16
    # NHWC 32 -> planar 1 with bias and residual
    w3 = f32(0.1 * rng.standard_normal((1, 32, 3, 3)))
    b3 = f32([0.37])
    res = f32(rng.standard_normal((B, H, W)))
    out3 = torch.zeros((B, H, W), device="cuda")
    w3g, b3g, resg = cuda32(w3), cuda32(b3), cuda32(res)
    d = L._desc(B, H, W, 32, 1, False, True, [hg], [out3], pack(lib, w3g, 1, 32, 0, False), b3g, residual=[resg])
    pat._check(lib.pat_conv3x3(ctypes.byref(d), st()), "conv")
    ref3 = res + OL.conv3x3(torch.tensor(nhwc_to_nchw(h)), torch.tensor(w3), torch.tensor(b3)).numpy()[:, 0]
    assert rel(out3.cpu().numpy(), ref3) < TOL_CONV


@pytest.mark.parametrize("B,H,W", [(2, 19, 300)])
def test_input_gradient_convolutions_vs_oracle(B, H, W):
    """pat_conv3x3 with transposed packing = conv_transpose2d of the oracle,
    with the PReLU backward fused into the NHWC epilogue."""
    lib = pat.load()
    rng = np.random.default_rng(7)
    part = torch.zeros(1 << 20, device="cuda")
    gba = torch.full((64,), 5.0, device="cuda")
    # layer 3 type: planar 1 -> NHWC 32, then back through a PReLU (slopes al, pre-activation xp)
    w3 = f32(0.2 * rng.standard_normal((1, 32, 3, 3)))
    gy = f32(rng.standard_normal((B, H, W)))
    xp = f32(rng.standard_normal((B, H, W, 32)))
    al = f32(0.1 + 0.3 * rng.random(32))
    gx = torch.zeros((B, H, W, 32), dtype=torch.int16, device="cuda")
    gyg, w3g, xpg, alg = cuda32(gy), cuda32(w3), cuda32(xp), cuda32(al)
    d = L._desc(B, H, W, 1, 32, True, False, [gyg], [gx], pack(lib, w3g, 1, 32, 1, True), alpha=alg, bwd_pre=xpg,
                partials=part, grad_bias_alpha=gba, accumulate=0)
    assert lib.pat_conv_bwd_partials(ctypes.byref(d)) <= part.numel()
    pat._check(lib.pat_conv3x3(ctypes.byref(d), st()), "conv")
    ga = torch.nn.functional.conv_transpose2d(OL.bf16(torch.tensor(gy[:, None])), OL.bf16(torch.tensor(w3)),
                                              padding=1).numpy()
    xpn = nhwc_to_nchw(xp)
    aln = al.reshape(1, 32, 1, 1)
    ref_gx = np.where(xpn > 0, ga, aln * ga)
    assert rel(nhwc_to_nchw(host16(gx)), ref_gx) < TOL_BF16
    assert rel(gba[:32].cpu().numpy(), ref_gx.sum(axis=(0, 2, 3))) < 1e-4
    assert rel(gba[32:].cpu().numpy(), np.where(xpn > 0, 0.0, ga * xpn).sum(axis=(0, 2, 3))) < 1e-4
    # accumulate adds
    d.accumulate = 1
    pat._check(lib.pat_conv3x3(ctypes.byref(d), st()), "conv")
    assert rel(gba[:32].cpu().numpy(), 2 * ref_gx.sum(axis=(0, 2, 3))) < 1e-4
    # layer 2 type: NHWC -> NHWC (plain epilogue: the bf16 input gradient itself)
    w2 = f32(0.1 * rng.standard_normal((32, 32, 3, 3)))
    g2 = bfv(rng.standard_normal((B, H, W, 32)))
    gx2 = torch.zeros((B, H, W, 32), dtype=torch.int16, device="cuda")
    g2g, w2g = cuda16(g2), cuda32(w2)
    d = L._desc(B, H, W, 32, 32, False, False, [g2g], [gx2], pack(lib, w2g, 32, 32, 1, False))
    pat._check(lib.pat_conv3x3(ctypes.byref(d), st()), "conv")
    ref = torch.nn.functional.conv_transpose2d(torch.tensor(nhwc_to_nchw(g2)), OL.bf16(torch.tensor(w2)),
                                               padding=1).numpy()
    assert rel(nhwc_to_nchw(host16(gx2)), ref) < TOL_BF16
    # layer 1 type: NHWC -> planar 3 with output scales, residual on plane 0, plane 2 skipped
    w1 = f32(0.3 * rng.standard_normal((32, 3, 3, 3)))
    res = f32(rng.standard_normal((B, H, W)))
    o0 = torch.zeros((B, H, W), device="cuda")
    o1 = torch.zeros((B, H, W), device="cuda")
    w1g, resg = cuda32(w1), cuda32(res)
    d = L._desc(B, H, W, 32, 3, False, True, [g2g], [o0, o1, None], pack(lib, w1g, 32, 3, 1, False),
                residual=[resg, None, None], scale=[1.0, 0.5, 2.0])
    pat._check(lib.pat_conv3x3(ctypes.byref(d), st()), "conv")
    ref = torch.nn.functional.conv_transpose2d(torch.tensor(nhwc_to_nchw(g2)), OL.bf16(torch.tensor(w1)),
                                               padding=1).numpy()
    assert rel(o0.cpu().numpy(), res + ref[:, 0]) < TOL_CONV
    assert rel(o1.cpu().numpy(), 0.5 * ref[:, 1]) < TOL_CONV


def test_weight_gradients_vs_oracle():
    lib = pat.load()
    rng = np.random.default_rng(11)
    B, H, W, rows = 2, 19, 300, 5      # ragged chunks of rows and a ragged row tail
    part = torch.zeros(4 << 20, device="cuda")
    # planar 3 (scaled) -> 32
    x = f32(rng.standard_normal((B, 3, H, W)))
    g = bfv(rng.standard_normal((B, H, W, 32)))
    gw = torch.zeros(32 * 3 * 9, device="cuda")
    scales = [1.0, 0.5, 2.0]
    xg = [cuda32(x[:, c]) for c in range(3)]
    gg = cuda16(g)
    d = L._desc(B, H, W, 3, 32, True, False, xg, [], None, scale=scales)
    d.weight = 1  # not read by the weight gradient; must be non-null for validation
    assert lib.pat_conv_wgrad_partials(ctypes.byref(d), rows) <= part.numel()
    pat._check(lib.pat_conv3x3_wgrad(ctypes.byref(d), gg.data_ptr(), rows, part.data_ptr(), gw.data_ptr(), 0,
                                     st()), "wgrad")
    xsc = x * np.array(scales).reshape(1, 3, 1, 1)
    ref = torch.nn.grad.conv2d_weight(OL.bf16(torch.tensor(xsc)), (32, 3, 3, 3), torch.tensor(nhwc_to_nchw(g)),
                                      padding=1).numpy()
    assert rel(gw.cpu().numpy(), ref) < TOL_CONV
    # accumulate: a second call adds
    pat._check(lib.pat_conv3x3_wgrad(ctypes.byref(d), gg.data_ptr(), rows, part.data_ptr(), gw.data_ptr(), 1,
                                     st()), "wgrad")
    assert rel(gw.cpu().numpy(), 2 * ref) < TOL_CONV
    # NHWC 32 -> 32
    h = bfv(rng.standard_normal((B, H, W, 32)))
    gw2 = torch.zeros(32 * 32 * 9, device="cuda")
    hg = cuda16(h)
    d = L._desc(B, H, W, 32, 32, False, False, [hg], [], None)
    d.weight = 1
    pat._check(lib.pat_conv3x3_wgrad(ctypes.byref(d), gg.data_ptr(), rows, part.data_ptr(), gw2.data_ptr(), 0,
                                     st()), "wgrad")
    ref2 = torch.nn.grad.conv2d_weight(torch.tensor(nhwc_to_nchw(h)), (32, 32, 3, 3),
                                       torch.tensor(nhwc_to_nchw(g)), padding=1).numpy()
    assert rel(gw2.cpu().numpy(), ref2) < TOL_CONV
    # NHWC 32 -> planar 1
    g1 = f32(rng.standard_normal((B, H, W)))
    gw3 = torch.zeros(32 * 9, device="cuda")
    g1g = cuda32(g1)
    d = L._desc(B, H, W, 32, 1, False, True, [hg], [], None)
    d.weight = 1
    pat._check(lib.pat_conv3x3_wgrad(ctypes.byref(d), g1g.data_ptr(), rows, part.data_ptr(), gw3.data_ptr(), 0,
                                     st()), "wgrad")
    ref3 = torch.nn.grad.conv2d_weight(torch.tensor(nhwc_to_nchw(h)), (1, 32, 3, 3),
                                       OL.bf16(torch.tensor(g1[:, None])), padding=1).numpy()
    assert rel(gw3.cpu().numpy(), ref3) < TOL_CONV


def test_plane_sums():
    lib = pat.load()
    rng = np.random.default_rng(3)
    part = torch.zeros(64 * 37, device="cuda")
    s = torch.zeros(1, device="cuda")
    v = f32(rng.standard_normal(12345))
    vg = cuda32(v)
    pat._check(lib.pat_plane_sum(v.size, vg.data_ptr(), part.data_ptr(), 37, s.data_ptr(), 0, st()), "sum")
    pat._check(lib.pat_plane_sum(v.size, vg.data_ptr(), part.data_ptr(), 37, s.data_ptr(), 1, st()), "sum")
    assert abs(float(s) - 2 * v.sum()) < 1e-4 * np.abs(v).sum()


@pytest.mark.parametrize("clip", [0.0, 30.0])
def test_adam_matches_reference(clip):
    lib = pat.load()
    rng = np.random.default_rng(4)
    n = 5000
    p = f32(rng.standard_normal(n))
    pg, mg, vg = cuda32(p), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    scratch = torch.zeros(128, dtype=torch.float64, device="cuda")
    m, v, q = np.zeros(n), np.zeros(n), p.copy()
    for t in range(1, 6):
        g = f32(rng.standard_normal(n) * (1 + t))   # ||g|| ~ 70 (1 + t): clipped when clip = 30
        gg = cuda32(g)
        pat._check(lib.pat_adam(n, pg.data_ptr(), gg.data_ptr(), mg.data_ptr(), vg.data_ptr(), step.data_ptr(),
                                1e-2, 1e-4, 8, 0.9, 0.999, 1e-8, clip, scratch.data_ptr(), st()), "adam")
        q, m, v = OL.adam_reference(q, g, m, v, t, 1e-2, 1e-4, 8, clip=clip)
    assert int(step) == 5
    assert np.max(np.abs(pg.cpu().numpy() - q)) < 1e-6
    assert rel(mg.cpu().numpy(), m) < 1e-5


def _tiny_setup(K=3):
    geom = P.top_arc(16, 16, 32, 180.0)
    plan = pat.Plan(geom, torch.float32, max_batch=2)
    f_true = P.ellipse_batch(16, [21, 22])
    y = np.stack([P.add_noise(O.forward(geom, fi), 0.02, 30 + i) for i, fi in enumerate(f_true)])
    params = L.init_params(9)
    # a larger last layer so that every layer carries a visible gradient
    Pd = L.unpack(params)
    Pd["dual.w3"][...] *= 10
    Pd["primal.w3"][...] *= 10
    params = np.concatenate([Pd[k].ravel() for k, _ in L.param_layout()]).astype(np.float32)
    return geom, plan, f32(f_true), f32(y), params, K


ENSEMBLE = 16  # perturbed oracle runs that measure the bf16 rounding-flip spread
FLOOR = 1e-5   # FP32 vs FP64 accumulation: the floor under every ensemble-derived bar


def within(err, spread):
    """The GPU's distance against twice the ensemble's largest, never below FLOOR."""
    return err < max(2 * spread, FLOOR)


def flip_spread(geom, Pd, y, f_true, K, s_A, s_U, ref_loss, ref_fK, ref_g, draws=ENSEMBLE):
    """The spread that FP32-level differences alone cause in the bf16-rounded
    oracle network: ``draws`` runs with every operator output perturbed by
    1e-6 and every convolution product by 1e-7 relative (seeded Gaussian
    noise, oracle.lpd.Perturb), each compared with the unperturbed run.
    Returns the largest relative loss difference, f_K distance and
    whole-gradient distance and the largest distance of each parameter block
    over the draws."""
    e_l, e_f, e_all, e_blk = 0.0, 0.0, 0.0, {k: 0.0 for k in ref_g}
    allo = np.concatenate([np.ravel(ref_g[k]) for k in ref_g])
    for s in range(draws):
        lo, fk, g = OL.loss_and_grads(geom, Pd, y, f_true, K, s_A, s_U, rounding=True,
                                      perturb=OL.Perturb(1000 + s, op=1e-6, conv=1e-7))
        e_l = max(e_l, abs(lo - ref_loss) / ref_loss)
        e_f = max(e_f, rel(fk, ref_fK))
        e_all = max(e_all, rel(np.concatenate([np.ravel(g[k]) for k in ref_g]), allo))
        for k in ref_g:
            e_blk[k] = max(e_blk[k], rel(g[k], ref_g[k]))
    return e_l, e_f, e_all, e_blk


@pytest.mark.parametrize("K", [1, 3])
def test_lpd_loss_gradient_vs_oracle(K):
    """Loss, f_K and every parameter gradient of K unrolled iterations at
    n = 16 (m = 16 on a 180-degree arc, nt = 32, batch 2) against the oracle
    network run on the oracle's A / A* with the same bf16 rounding.

    Tolerances.  Both sides round the convolution operands to bf16 from FP32
    values that differ by the operators' FP32 error and by FP32 accumulation,
    so a few roundings land on the other side of a midpoint, each moving one
    operand by up to 2^-8 relative.  With one iteration the results agree to
    ~2e-5 (bar 1e-4).  Every further iteration feeds the flipped values
    through the network and flips more roundings, so at K = 3 both sides are
    draws of the same bf16 noise.  The bar there is measured on the oracle
    side alone: an ensemble of oracle runs whose operator outputs (1e-6) and
    convolution products (1e-7) carry seeded relative noise, compared with
    the unperturbed run (flip_spread; the spread hardly depends on the noise
    level, 1e-5 gives the same).  The GPU is one more such draw: f_K, the
    whole gradient and each parameter block must lie within twice the
    largest distance of the ensemble (16 draws; twice covers the sampling
    error of a maximum), never below 1e-5 (FP32 against FP64 accumulation,
    for quantities the flips cannot reach).  A wrong term or sign gives O(1)
    errors."""
    geom, plan, f_true, y, params, _ = _tiny_setup()
    s_A, s_U = 0.9, 1.7
    net = L.LPD(plan, 2, iters=K, params=params, s_A=s_A, s_U=s_U)
    yg, fg = cuda32(y), cuda32(f_true)
    net.set_batch(yg, fg)
    net.forward_pass()
    net.backward_pass()
    torch.cuda.synchronize()
    Pd = {k: v.astype(np.float64) for k, v in L.unpack(params).items()}
    loss_o, fK_o, g_o = OL.loss_and_grads(geom, Pd, y, f_true, K, s_A, s_U, rounding=True)
    grads = L.unpack(net.grads.cpu().numpy())
    fK = net.f[K].cpu().numpy()
    e_f = rel(fK, fK_o)
    e_g = {k: rel(grads[k], g_o[k]) for k in g_o}
    allg = np.concatenate([np.ravel(grads[k]) for k in g_o])
    allo = np.concatenate([np.ravel(g_o[k]) for k in g_o])
    if K == 1:
        print("K=1 f_K: gpu %.2e" % e_f)
        assert e_f < 1e-4
        assert abs(net.loss() - loss_o) < 1e-4 * loss_o
        for k in g_o:
            assert e_g[k] < 1e-4, k
        return
    s_l, s_f, s_all, s_blk = flip_spread(geom, Pd, y, f_true, K, s_A, s_U, loss_o, fK_o, g_o)
    print("K=%d f_K: gpu %.2e, flip spread %.2e; gradient: gpu %.2e, flip spread %.2e"
          % (K, e_f, s_f, rel(allg, allo), s_all))
    for k in g_o:
        print("  %-10s gpu %.2e  flip spread %.2e" % (k, e_g[k], s_blk[k]))
    assert within(e_f, s_f)
    assert within(abs(net.loss() - loss_o) / loss_o, s_l)
    assert within(rel(allg, allo), s_all)
    for k in g_o:
        assert within(e_g[k], s_blk[k]), k


def test_lpd_graph_replay_equals_eager_training():
    geom, plan, f_true, y, params, K = _tiny_setup(K=2)
    a = L.LPD(plan, 2, iters=K, params=params)
    b = L.LPD(plan, 2, iters=K, params=params)
    for net in (a, b):
        net.opt.update(lr=1e-3, total=10)
        net.set_batch(cuda32(y), cuda32(f_true))
    for _ in range(3):
        a.train_step()
    b.capture_train()
    for _ in range(3):
        b.graph_train.replay()
    torch.cuda.synchronize()
    assert torch.equal(a.params, b.params)
    assert int(b.step_count) == 3


def test_inference_network_equals_training_network():
    """An inference-only network (one set of activations, reused by every
    iteration) gives f_K identical to the training network's, eager and as a
    captured, replayed graph."""
    geom, plan, f_true, y, params, K = _tiny_setup(K=3)
    a = L.LPD(plan, 2, iters=K, params=params, s_A=0.9, s_U=1.7)
    b = L.LPD(plan, 2, iters=K, params=params, s_A=0.9, s_U=1.7, train=False)
    for net in (a, b):
        net.set_batch(cuda32(y), cuda32(f_true))
    fa = a.forward_pass().clone()
    fb = b.forward_pass().clone()
    torch.cuda.synchronize()
    assert torch.equal(fa, fb)
    b.capture_forward()
    for _ in range(2):
        b.f[K].zero_()
        torch.cuda.synchronize()
        b.graph_fwd.replay()
        torch.cuda.synchronize()
        assert torch.equal(b.f[K], fa)


def test_training_gains_over_untrained_network():
    """800 steps on 256 phantoms (n = 32, 180-degree arc) raise the held-out
    PSNR well above the untrained network and above the method without the
    learned part: the same number (K = 5) of projected-gradient (NNLS)
    iterations with the same operators."""
    from paper_2510_24687_amd import solvers as S
    geom = P.top_arc(32, 32, 64, 180.0)
    plan = pat.Plan(geom, torch.float32, max_batch=16)
    ds = L.make_dataset(plan, range(256), noise=0.02, noise_seed=5)
    test = L.make_dataset(plan, range(10 ** 6, 10 ** 6 + 16), noise=0.02, noise_seed=6)
    s_A, s_U = L.input_scales(plan, ds)
    K = 5
    net = L.LPD(plan, 8, iters=K, s_A=s_A, s_U=s_U, seed=1)
    base = L.evaluate(net, test)
    log = L.train(net, ds, steps=800, lr=3e-3)
    after = L.evaluate(net, test)
    sol = S.BatchedSolver([(plan, test["y"], None)], method="nnls")
    for _ in range(K):
        sol.step()
    nnls = float(L.psnr(sol.groups[0].f, test["f"]).mean())
    bp = L.backprojection_psnr(plan, test, s_U)
    print("untrained %.2f dB, trained %.2f dB, NNLS(%d) %.2f dB, back-projection %.2f dB, loss %s"
          % (base, after, K, nnls, bp, log[-3:]))
    assert after > base + 8.0
    assert after > nnls + 3.0
    assert after > bp
