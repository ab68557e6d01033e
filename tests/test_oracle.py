"""Pins of the CPU FP64 oracle against things other than itself.

Every check compares the oracle with an independent mathematical fact:
two closed forms, a different discretisation of the same definition, a
brute-force PDE solve, exact discrete symmetries, or the adjoint identity.
Citations refer to Hauptmann, Kunyansky & Poimala, arXiv 2510.24687.
"""
import numpy as np
import pytest

import oracle as O
from paper_2510_24687_amd import phantoms as P


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _detectors(g):
    th = g["theta0"] + np.arange(g["m"]) * g["arc"] / g["m"]
    return np.stack([g["R"] * np.cos(th), g["R"] * np.sin(th)], axis=1)


def _times(g):
    return (np.arange(g["nt"]) + 1) * g["T"] / g["nt"]


def test_taper_shape():
    """W = 1 up to rho*Lambda, 0 from Lambda on, monotone in between; the C
    and numpy implementations agree."""
    Lam, rho = 100.0, 0.8
    lam = np.linspace(0, 110, 2201)
    w_c = O.taper(lam, Lam, rho)
    w_np = O._taper_np(lam, Lam, rho)
    assert np.max(np.abs(w_c - w_np)) < 1e-15
    assert np.all(w_c[lam <= rho * Lam] == 1.0)
    assert np.all(w_c[lam >= Lam] == 0.0)
    assert np.all(np.diff(w_c) <= 1e-15)
    assert abs(O.taper(90.0, Lam, rho) - 0.5) < 1e-15  # symmetric smooth step


def test_gaussian_semiclosed_form_vs_poisson():
    """Semi-closed J0 form (E:kwave + Jacobi-Anger E:Anger) against the 2D
    Poisson formula for E:wave-eq/E:Cauchy in circular means (no Fourier
    transform, no Bessel J): agreement to 1e-12."""
    g = P.full_circle(64, 12, 16, T=2.0, c=1.3)
    blobs = P.gaussian_blobs(11, count=4)
    ga = O.gauss_forward(g, blobs)
    gp = O.poisson_gauss(blobs, _times(g), _detectors(g), c=g["c"])
    assert np.max(np.abs(ga - gp)) / np.max(np.abs(gp)) < 1e-12


def test_fd_wave_propagation_converges_to_semiclosed_form():
    """Brute-force leapfrog finite differences (Sec. 2.1.1) on three grids
    converge to the semi-closed form at second order."""
    blobs = np.array([[0.2, -0.1, 0.12, 1.0], [-0.3, 0.25, 0.1, 0.6]])
    dets = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)]
    times = [0.5, 1.0, 1.5]
    g = dict(P.full_circle(8, 4, 3, T=1.5), theta0=0.0)
    ref = O.gauss_forward(g, blobs)  # detectors at angles 0, pi/2, pi, 3pi/2
    errs, fds = [], []
    for dx in (0.04, 0.02, 0.01):
        fd = O.fd_gauss(blobs, dets, times, dx=dx, box=3.0)
        fds.append(fd)
        errs.append(np.max(np.abs(fd - ref)) / np.max(np.abs(ref)))
    order = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert errs[2] < 5e-3
    assert 1.5 < order[0] < 2.5 and 1.8 < order[1] < 2.2
    richardson = (4 * fds[2] - fds[1]) / 3
    assert np.max(np.abs(richardson - ref)) / np.max(np.abs(ref)) < 3e-4


def test_grid_model_matches_semiclosed_form_for_resolved_gaussians():
    """For samples of Gaussians with sigma >= 4h lying >= 7 sigma inside the
    box, the band-limited grid model equals the tapered semi-closed form."""
    n = 96
    g = P.full_circle(n, 16, 24, T=2.0)
    blobs = np.array([[0.1, -0.15, 0.09, 1.0], [-0.2, 0.05, 0.085, 0.7], [0.0, 0.2, 0.1, 0.4]])
    f = P.sample_blobs(blobs, n)
    a = O.forward(g, f)
    b = O.gauss_forward(g, blobs, taper_grid=True)
    assert np.max(np.abs(a - b)) / np.max(np.abs(b)) < 1e-10


def test_late_time_closed_form_of_kernel():
    """For c t well beyond every distance, Q(t,d) -> (h^2/2pi)(-ct)/((ct)^2-d^2)^{3/2},
    the exact value of int_0^inf l J0(l d) cos(c l t) dl (time derivative of the
    2D fundamental solution of E:green_conv).  Pins normalisation, sign, the
    factor lambda, the Bessel order and the placement of c."""
    n = 64
    g = P.full_circle(n, 8, 16, T=16.0, c=1.5)
    f = P.sample_blobs(P.gaussian_blobs(4, count=5, sigma=(0.08, 0.15)), n)
    out = O.forward(g, f)
    h = 2.0 / n
    xs = P.pixel_centres(n)
    X, Y = np.meshgrid(xs, xs)
    z = _detectors(g)
    t = _times(g)
    for j in (9, 12, 15):
        tau = g["c"] * t[j]
        ref = np.array([np.sum(f * (h * h / (2 * np.pi)) * (-tau) /
                               (tau * tau - ((zx - X) ** 2 + (zy - Y) ** 2)) ** 1.5) for zx, zy in z])
        assert np.max(np.abs(out[j] - ref)) / np.max(np.abs(ref)) < 1e-9


def test_oracle_matches_kspace_route():
    """The paper's unaccelerated Fourier route (E:kwave), discretised by a 2D
    trapezoid rule in xi, agrees with the J0 quadrature on an arbitrary image."""
    n = 32
    g = P.full_circle(n, 16, 16, T=2.0, c=1.1, R=1.05)
    f = P.randn((n, n), 5)
    a = O.forward(g, f)
    delta = 2 * np.pi / (g["R"] + np.sqrt(2) + g["c"] * g["T"] + 26.0)
    b = O.kspace_forward(g, f, delta=delta)
    assert _rel(a, b) < 1e-10


def test_adjoint_identity():
    """<A f, g>_Y = <f, A* g>_X with the rectangle-rule inner products of
    eqn:innerProducts."""
    n = 24
    g = P.top_arc(n, 20, 18, arc_deg=180.0, T=2.0)
    f = P.randn((n, n), 1)
    y = P.randn((g["nt"], g["m"]), 2)
    Af = O.forward(g, f)
    Aty = O.adjoint(g, y)
    h = 2.0 / n
    lhs = np.sum(Af * y) * (g["T"] / g["nt"]) * (g["R"] * g["arc"] / g["m"])
    rhs = np.sum(f * Aty) * h * h
    assert abs(lhs - rhs) / (np.linalg.norm(Af) * np.linalg.norm(y)) < 1e-14
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


def test_rotation_and_mirror_symmetry():
    """Rotating the image by 90 degrees shifts the detectors by m/4; mirroring
    y -> -y maps theta -> -theta (cell-centred grid, full circle, 4 | m)."""
    n, m = 16, 16
    g = P.full_circle(n, m, 12, T=2.0)
    f = P.randn((n, n), 3)
    a = O.forward(g, f)
    # counter-clockwise rotation f'(x, y) = f(y, -x): new[p, q] = f[n-1-q, p]
    rot = np.array([[f[n - 1 - q, p] for q in range(n)] for p in range(n)])
    b = O.forward(g, rot)
    assert np.max(np.abs(b - np.roll(a, m // 4, axis=1))) < 1e-12 * np.max(np.abs(a))
    mir = f[::-1, :]
    c = O.forward(g, mir)
    idx = (-np.arange(m)) % m
    assert np.max(np.abs(c - a[:, idx])) < 1e-12 * np.max(np.abs(a))


def test_sampled_entries_match_full_tensor_and_mask():
    n = 16
    g = P.full_circle(n, 12, 10, T=2.0, mask_radius=0.7)
    f = P.randn((n, n), 7)
    y = P.randn((g["nt"], g["m"]), 8)
    full = O.forward(g, f)
    dets = [0, 5, 11]
    assert np.array_equal(O.forward(g, f, dets=dets), full[:, dets])
    fa = O.adjoint(g, y)
    pix = [0, 37, 100, 255]
    assert np.allclose(O.adjoint(g, y, pix=pix), fa.ravel()[pix], rtol=0, atol=1e-15 * np.abs(fa).max())
    xs = P.pixel_centres(n)
    X, Y = np.meshgrid(xs, xs)
    inside = X * X + Y * Y <= 0.7 ** 2
    unmasked = dict(g, mask_radius=0.0)
    assert np.allclose(full, O.forward(unmasked, f * inside), rtol=0, atol=1e-14 * np.abs(full).max())
    assert np.all(fa[~inside] == 0.0)


def test_quadrature_panel_refinement():
    """Halving the Gauss-Legendre panels changes nothing at 1e-13."""
    n = 32
    g = P.full_circle(n, 8, 16, T=2.0)
    f = P.randn((n, n), 9)
    a = O.forward(g, f)
    b = O.forward(g, f, phase_per_panel=5.0)
    assert _rel(a, b) < 1e-13
