"""Pins of the learned primal-dual oracle (oracle/lpd.py) against things other
than itself: brute-force convolution sums, the bfloat16 rounding rule on
hand-picked ties, finite-difference gradients (torch.autograd.gradcheck) of
the whole unrolled network, and closed forms of the Adam step."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from oracle import lpd as OL  # noqa: E402
from paper_2510_24687_amd import phantoms as P  # noqa: E402


def test_conv3x3_matches_brute_force_sums():
    rng = np.random.default_rng(0)
    B, cin, cout, H, W = 2, 3, 4, 5, 7
    x = rng.standard_normal((B, cin, H, W))
    w = rng.standard_normal((cout, cin, 3, 3))
    b = rng.standard_normal(cout)
    ref = np.zeros((B, cout, H, W))
    for bb in range(B):
        for co in range(cout):
            for yy in range(H):
                for xx in range(W):
                    s = b[co]
                    for ci in range(cin):
                        for ky in range(3):
                            for kx in range(3):
                                sy, sx = yy + ky - 1, xx + kx - 1
                                if 0 <= sy < H and 0 <= sx < W:
                                    s += w[co, ci, ky, kx] * x[bb, ci, sy, sx]
                    ref[bb, co, yy, xx] = s
    got = OL.conv3x3(torch.tensor(x), torch.tensor(w), torch.tensor(b), rounding=False).numpy()
    assert np.max(np.abs(got - ref)) < 1e-12


def test_bf16_rounding_is_nearest_even():
    e = 2.0 ** -8
    vals = torch.tensor([1 + e, 1 + 3 * e, 1 + e + 2.0 ** -20, -(1 + e), 3.0, 1 + 2 * e])
    want = [1.0, 1 + 4 * e, 1 + 2 * e, -1.0, 3.0, 1 + 2 * e]
    assert OL.bf16(vals).tolist() == want


def _tiny_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    P_ = {}
    for net, cin in (("dual", 3), ("primal", 2)):
        P_[net + ".w1"] = scale * rng.standard_normal((32, cin, 3, 3)) / 3
        P_[net + ".b1"] = 0.1 * rng.standard_normal(32)
        P_[net + ".a1"] = 0.25 + 0.05 * rng.standard_normal(32)
        P_[net + ".w2"] = scale * rng.standard_normal((32, 32, 3, 3)) / 17
        P_[net + ".b2"] = 0.1 * rng.standard_normal(32)
        P_[net + ".a2"] = 0.25 + 0.05 * rng.standard_normal(32)
        P_[net + ".w3"] = scale * rng.standard_normal((1, 32, 3, 3)) / 17
        P_[net + ".b3"] = 0.1 * rng.standard_normal(1)
    return P_


def test_unrolled_network_gradients_match_finite_differences():
    """gradcheck of the FP64 network (rounding off) with small explicit
    operator matrices, with respect to a subset of every kind of parameter
    and the data y."""
    rng = np.random.default_rng(1)
    n, nt, m, B, K = 5, 6, 4, 2, 2
    M = torch.tensor(rng.standard_normal((nt * m, n * n)) / 5)
    s = 0.7
    ops = (lambda f: (f.reshape(f.shape[0], -1) @ M.T).reshape(f.shape[0], nt, m),
           lambda g: s * (g.reshape(g.shape[0], -1) @ M).reshape(g.shape[0], n, n))
    P0 = {k: torch.tensor(v) for k, v in _tiny_params(2).items()}
    y0 = torch.tensor(rng.standard_normal((B, nt, m)))
    geom = {"n": n}
    names = ["dual.w1", "dual.a2", "dual.b3", "primal.w3", "primal.b1", "primal.a1"]

    def fn(y, *vals):
        Pd = dict(P0)
        Pd.update(dict(zip(names, vals)))
        return OL.reconstruct(geom, Pd, y, K, 0.8, 1.3, rounding=False, ops=ops)

    inputs = [y0.clone().requires_grad_(True)] + [P0[k].clone().requires_grad_(True) for k in names]
    assert torch.autograd.gradcheck(fn, inputs, eps=1e-6, atol=1e-6, rtol=1e-4)


def test_direct_quadrature_operators_backward_is_their_transpose():
    geom = P.top_arc(6, 8, 8, 180.0)
    f = torch.tensor(P.randn((1, 6, 6), 3), requires_grad=True)
    g = torch.tensor(P.randn((1, 8, 8), 4), requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: OL._A.apply(x, geom, None), (f,), eps=1e-6, atol=1e-8, rtol=1e-6)
    assert torch.autograd.gradcheck(lambda x: OL._Astar.apply(x, geom, None), (g,), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_rounded_network_gradient_is_close_to_exact():
    """bf16 rounding of the products perturbs the loss gradient by ~1e-2, not more."""
    geom = P.top_arc(8, 8, 16, 180.0)
    Pn = _tiny_params(5)
    f_true = P.ellipse_batch(8, [1, 2])
    y = np.stack([O.forward(geom, fi) for fi in f_true])
    l1, f1, g1 = OL.loss_and_grads(geom, Pn, y, f_true, 2, rounding=True)
    l0, f0, g0 = OL.loss_and_grads(geom, Pn, y, f_true, 2, rounding=False)
    for k in g0:
        rel = np.linalg.norm(g1[k] - g0[k]) / np.linalg.norm(g0[k])
        assert rel < 5e-2, (k, rel)
    assert abs(l1 - l0) < 2e-2 * l0


def test_adam_reference_closed_forms():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    p1, m1, v1 = OL.adam_reference(p, g, np.zeros(3), np.zeros(3), 1, 1e-2, 1e-4, 10, eps=1e-12)
    # first step: m_hat = g, v_hat = g^2, so the update is lr * sign(g)
    assert np.allclose(p1, p - 1e-2 * np.sign(g), rtol=0, atol=1e-9)
    # at the last scheduled step the rate is lr_min; a constant gradient keeps
    # m_hat = g, v_hat = g^2, so the update is lr_min * sign(g)
    m, v, q = np.zeros(3), np.zeros(3), p.copy()
    for t in range(1, 11):
        q_prev = q
        q, m, v = OL.adam_reference(q, g, m, v, t, 1e-2, 1e-4, 10, eps=1e-12)
    assert np.allclose(q_prev - q, 1e-4 * np.sign(g), rtol=1e-9, atol=1e-12)
    # halfway (t - 1 = (total - 1)/2) the cosine rate is the mean of the two
    frac_mid = 0.5 * (1e-2 + 1e-4)
    qa, _, _ = OL.adam_reference(p, g, g, g * g, 6, 1e-2, 1e-4, 11, eps=1e-12)
    mh = g / (1 - 0.9 ** 6)
    vh = g * g / (1 - 0.999 ** 6)
    assert np.allclose(p - qa, frac_mid * mh / np.sqrt(vh), rtol=1e-9)
    assert math.isclose(0.5 * (1e-2 - 1e-4) * (1 + math.cos(math.pi * 0.5)) + 1e-4, frac_mid)


def test_adam_reference_clipping():
    g = np.array([3.0, 4.0])                      # ||g|| = 5
    _, m1, v1 = OL.adam_reference(np.zeros(2), g, np.zeros(2), np.zeros(2), 1, 1e-2, 1e-4, 10, clip=1.0)
    assert np.allclose(m1, 0.1 * g / 5.0) and np.allclose(v1, 0.001 * (g / 5.0) ** 2)
    _, m2, _ = OL.adam_reference(np.zeros(2), g, np.zeros(2), np.zeros(2), 1, 1e-2, 1e-4, 10, clip=10.0)
    assert np.allclose(m2, 0.1 * g)               # below the threshold: unchanged
