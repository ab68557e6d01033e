"""CPU FP64 iterations of the variational reconstructions of Sec. 4.2.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): imported by
``tests/`` to check the library's solver kernels, never by the product.

The TV-regularised least-squares problem of eq. E:minim with the total
variation regulariser of Sec. 4.2,

    min_{f >= 0}  1/2 ||A f - g||_Y^2 + lam * h^2 * sum_pixels |grad_h f|,

in the weighted L2 spaces of eq. eqn:innerProducts (X: weight h^2 per pixel,
Y: weight (T/nt)(R arc/m) per trace sample, so the gradient of the data term
is A*(A f - g) with the weighted adjoint A*).  The paper's PDHG (eqs.
eqn:PDHG-dual, eqn:PDHG-primal, eqn:PDHG-relaxation) takes the TV term by a
proximal operator that is itself a denoising problem; this module follows
the fully split reading: the primal-dual method of Chambolle and Pock for
K = [A; mu grad_h], F(y1, y2) = 1/2 ||y1 - g||^2 + (lam/mu) ||y2||_{1,2},
G = indicator of f >= 0 (times an optional support mask), and the standard
relaxation fbar = f_new + theta (f_new - f) (the paper prints the opposite
sign).  The TV dual of mu grad_h is kept as p = mu r, so its step uses
sigma mu^2 and its projection radius is lam.

grad_h: forward differences divided by h, the last difference in each
direction zero (Neumann boundary); div_h = -(grad_h)^T.
"""
from __future__ import annotations

import numpy as np


def grad_h(f: np.ndarray, h: float) -> np.ndarray:
    """(2, n, n): x-differences (along the last axis) and y-differences."""
    out = np.zeros((2,) + f.shape)
    out[0][:, :-1] = (f[:, 1:] - f[:, :-1]) / h
    out[1][:-1, :] = (f[1:, :] - f[:-1, :]) / h
    return out


def div_h(p: np.ndarray, h: float) -> np.ndarray:
    """Minus the transpose of grad_h (plain sums: <grad_h f, p> = -<f, div_h p>)."""
    px, py = p[0], p[1]
    n1, n2 = px.shape
    d = np.zeros((n1, n2))
    # column c receives +px[c-1]/h (as the right end of difference c-1) and -px[c]/h
    for c in range(n2):
        if c < n2 - 1:
            d[:, c] += px[:, c] / h
        if c > 0:
            d[:, c] -= px[:, c - 1] / h
    for r in range(n1):
        if r < n1 - 1:
            d[r, :] += py[r, :] / h
        if r > 0:
            d[r, :] -= py[r - 1, :] / h
    return d


def project_tv_dual(p: np.ndarray, lam: float) -> np.ndarray:
    """Pointwise projection of the (2, n, n) field onto |p_pixel| <= lam."""
    mag = np.sqrt(p[0] ** 2 + p[1] ** 2)
    scale = np.where(mag > lam, lam / np.where(mag > 0, mag, 1.0), 1.0)
    return p * scale


def tv_objective(A, f: np.ndarray, g: np.ndarray, lam: float, h: float, wy: float) -> float:
    """1/2 ||A f - g||_Y^2 + lam h^2 sum |grad_h f| (A a callable)."""
    r = A(f) - g
    gr = grad_h(f, h)
    return 0.5 * wy * float(np.sum(r * r)) + lam * h * h * float(np.sum(np.sqrt(gr[0] ** 2 + gr[1] ** 2)))


def cp_tv(A, Astar, g: np.ndarray, n: int, h: float, lam: float, tau: float, sigma: float, mu: float,
          iters: int, theta: float = 1.0, support=None, history: bool = False):
    """Fully split Chambolle-Pock for the TV problem above, started from zero.

    A, Astar: callables for the forward operator and its weighted adjoint.
    Each iteration, in the order of eqs. eqn:PDHG-dual, eqn:PDHG-primal,
    eqn:PDHG-relaxation:
      q    <- (q + sigma (A fbar - g)) / (1 + sigma)          (data dual)
      p    <- project_{|p| <= lam}(p + sigma mu^2 grad_h fbar) (TV dual, stored as mu r)
      f'   <- max(0, f - tau (A* q - div_h p)) [* support]    (primal)
      fbar <- f' + theta (f' - f)                              (relaxation)
    Returns f (and the list of iterates if ``history``)."""
    f = np.zeros((n, n))
    fbar = np.zeros((n, n))
    q = np.zeros_like(g, dtype=np.float64)
    p = np.zeros((2, n, n))
    hist = []
    for _ in range(iters):
        q = (q + sigma * (A(fbar) - g)) / (1.0 + sigma)
        p = project_tv_dual(p + sigma * mu * mu * grad_h(fbar, h), lam)
        f_new = np.maximum(0.0, f - tau * (Astar(q) - div_h(p, h)))
        if support is not None:
            f_new = f_new * support
        fbar = f_new + theta * (f_new - f)
        f = f_new
        if history:
            hist.append(f.copy())
    return (f, hist) if history else f


def nnls_pg(A, Astar, g: np.ndarray, n: int, tau: float, iters: int, support=None) -> np.ndarray:
    """Projected-gradient NNLS of eqs. eqn:NNLS / eq:NNLS-projstep from f = 0:
    f <- max(0, f - tau A*(A f - g)) [* support]."""
    f = np.zeros((n, n))
    for _ in range(iters):
        f = np.maximum(0.0, f - tau * Astar(A(f) - g))
        if support is not None:
            f = f * support
    return f
