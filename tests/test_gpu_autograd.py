"""Differentiation through the HIP operators: gradcheck in FP64 and the FP32
data-fidelity gradient 2 A^T (A f - g) against the CPU FP64 oracle."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2510_24687_amd import autograd as AG  # noqa: E402
from paper_2510_24687_amd import pat  # noqa: E402
from paper_2510_24687_amd import phantoms as P  # noqa: E402

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def test_gradcheck_fp64_forward_and_transpose():
    """torch.autograd.gradcheck at n=32, m=64, nt=64 with N(0,1) inputs."""
    geom = P.full_circle(32, 64, 64)
    plan = pat.Plan(geom, torch.float64, max_batch=2)
    f = torch.tensor(P.randn((32, 32), 3), dtype=torch.float64, device="cuda", requires_grad=True)
    g = torch.tensor(P.randn((64, 64), 4), dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: AG.forward(x, plan), (f,), eps=1e-6, atol=1e-7, rtol=1e-5)
    assert torch.autograd.gradcheck(lambda x: AG.transpose(x, plan), (g,), eps=1e-6, atol=1e-7, rtol=1e-5)
    assert torch.autograd.gradcheck(lambda x: AG.adjoint(x, plan), (g,), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_gradgradcheck_fp64():
    """Second derivatives through A, A^T and A*: the backward passes are built
    from the opposite operators, so double backward (create_graph=True) is
    exact, checked by torch.autograd.gradgradcheck at n=32, m=64, nt=64."""
    geom = P.full_circle(32, 64, 64)
    plan = pat.Plan(geom, torch.float64, max_batch=2)
    f = torch.tensor(P.randn((32, 32), 13), dtype=torch.float64, device="cuda", requires_grad=True)
    g = torch.tensor(P.randn((64, 64), 14), dtype=torch.float64, device="cuda", requires_grad=True)
    y = torch.tensor(P.randn((64, 64), 15), dtype=torch.float64, device="cuda")
    # a nonlinear loss, so the second derivative is not zero
    loss_f = lambda x: (AG.forward(x, plan) - y).pow(3).sum()  # noqa: E731
    loss_g = lambda x: AG.transpose(x, plan).pow(3).sum()  # noqa: E731
    loss_a = lambda x: AG.adjoint(x, plan).pow(3).sum()  # noqa: E731
    for fn, x in ((loss_f, f), (loss_g, g), (loss_a, g)):
        assert torch.autograd.gradgradcheck(fn, (x,), eps=1e-6, atol=1e-6, rtol=1e-5)
    # Hessian-vector product of 1/2 ||A f - y||^2 is A^T A v
    v = torch.tensor(P.randn((32, 32), 16), dtype=torch.float64, device="cuda")
    loss = 0.5 * (AG.forward(f, plan) - y).pow(2).sum()
    (grad,) = torch.autograd.grad(loss, f, create_graph=True)
    (hv,) = torch.autograd.grad((grad * v).sum(), f)
    want = plan.transpose(plan.forward(v))
    assert torch.allclose(hv, want, rtol=1e-12, atol=1e-12 * float(want.abs().max()))


def test_transpose_is_exact_in_fp64():
    geom = P.top_arc(32, 32, 40, 180.0)
    plan = pat.Plan(geom, torch.float64)
    f = torch.tensor(P.randn((32, 32), 5), dtype=torch.float64, device="cuda")
    g = torch.tensor(P.randn((40, 32), 6), dtype=torch.float64, device="cuda")
    lhs = torch.sum(plan.forward(f) * g).item()
    rhs = torch.sum(f * plan.transpose(g)).item()
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_fp32_data_fidelity_gradient_vs_oracle_n64():
    """grad of ||A f - g||^2 equals 2 A_o^T (A_o f - g) of the oracle."""
    geom = P.full_circle(64, 128, 128)
    plan = pat.Plan(geom, torch.float32)
    f_np = P.ellipse_phantom(64, 7)
    g_np = P.randn((128, 128), 8)
    f = torch.tensor(f_np, dtype=torch.float32, device="cuda", requires_grad=True)
    g = torch.tensor(g_np, dtype=torch.float32, device="cuda")
    loss = ((AG.forward(f, plan) - g) ** 2).sum()
    loss.backward()
    ref = 2 * O.adjoint(geom, O.forward(geom, f_np) - g_np) / O.adjoint_scale(geom)
    assert rel(f.grad.double().cpu().numpy(), ref) <= 1e-4


def test_fp32_batched_gradient_n256_phantom_data_vs_oracle():
    """The differentiation workload at full size: batch of 16 at n=256,
    m=512, nt=512, f = random-ellipse phantoms, g = A f' + noise (f' other
    phantoms, noise sigma * eps as stored with the oracle's values); the
    gradient of ||A f - g||^2 is compared on the oracle's pixel samples of
    image 0, every other image against 2 A^T (A f - g) of its own."""
    path = os.path.join(HERE, "golden", "grad_full_n256.npz")
    z = np.load(path)
    geom = P.full_circle(256, 512, 512)
    B = 16
    fs = [int(z["f_seed"])] + [720 + b for b in range(B - 1)]
    fps = [int(z["fp_seed"])] + [820 + b for b in range(B - 1)]
    ns = [int(z["noise_seed"])] + [920 + b for b in range(B - 1)]
    sigma = float(z["sigma"])
    plan = pat.Plan(geom, torch.float32, max_batch=B)
    f = torch.tensor(P.ellipse_batch(256, fs), dtype=torch.float32, device="cuda", requires_grad=True)
    fp = torch.tensor(P.ellipse_batch(256, fps), dtype=torch.float32, device="cuda")
    eps = torch.tensor(np.stack([P.randn((512, 512), s) for s in ns]), dtype=torch.float32, device="cuda")
    with torch.no_grad():
        g = plan.forward(fp) + sigma * eps
    loss = ((AG.forward(f, plan) - g) ** 2).sum()
    loss.backward()
    got = f.grad[0].double().cpu().numpy().ravel()[z["pix"]]
    e0 = rel(got, z["grad"])
    print("gradient vs oracle samples %.3e" % e0, flush=True)
    assert e0 <= 1e-4
    with torch.no_grad():
        one = 2 * plan.transpose(plan.forward(f[9].detach()) - g[9])
    assert rel(f.grad[9].double().cpu().numpy(), one.double().cpu().numpy()) <= 1e-6


def test_fp32_batched_gradient_n256_vs_oracle_samples():
    """Batch of 16 at n=256, m=512, nt=512: with f = 0 the gradient of
    ||A f - g||^2 is -2 A^T g, compared on the oracle's stored pixel samples."""
    z = np.load(os.path.join(HERE, "golden", "full_n256.npz"))
    geom = P.full_circle(256, 512, 512)
    plan = pat.Plan(geom, torch.float32, max_batch=16)
    g_np = np.stack([P.randn((512, 512), 1)] + [P.randn((512, 512), 700 + b) for b in range(15)])
    f = torch.zeros((16, 256, 256), dtype=torch.float32, device="cuda", requires_grad=True)
    g = torch.tensor(g_np, dtype=torch.float32, device="cuda")
    loss = ((AG.forward(f, plan) - g) ** 2).sum()
    loss.backward()
    got = f.grad[0].double().cpu().numpy().ravel()[z["pix"]]
    ref = -2 * z["adjoint"] / O.adjoint_scale(geom)
    assert rel(got, ref) <= 1e-4
    # every image of the batch sees the same operator
    one = -2 * plan.transpose(g[5]).double().cpu().numpy()
    assert rel(f.grad[5].double().cpu().numpy(), one) <= 1e-6
