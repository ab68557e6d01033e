"""Pins of the oracle's solver iterations (oracle/solvers.py) against
independent solutions of the same convex problems (Sec. 4.2, eq. E:minim).

The problems are tiny (n = 6, 8 detectors on the 180-degree arc, 12 times),
so the oracle's operator is taken as its explicit matrix: the columns are
the oracle's forward images of the unit pixels, and A* = s A^T with the
oracle's adjoint scale s.
"""
import numpy as np
import pytest
import scipy.optimize as so

import oracle as O
from oracle import solvers as S
from paper_2510_24687_amd import phantoms as P

N_IMG, NT, M = 6, 12, 8


@pytest.fixture(scope="module")
def problem():
    n = N_IMG
    geom = P.top_arc(n, M, NT, 180.0)
    cols = []
    for i in range(n * n):
        e = np.zeros(n * n)
        e[i] = 1.0
        cols.append(O.forward(geom, e.reshape(n, n)).ravel())
    Am = np.array(cols).T
    s = O.adjoint_scale(geom)
    h = 2.0 * geom["a"] / n
    wy = s * h * h          # Y weight: A* = (wy / h^2) A^T
    A = lambda f: (Am @ f.ravel()).reshape(NT, M)  # noqa: E731
    As = lambda g: s * (Am.T @ g.ravel()).reshape(n, n)  # noqa: E731
    f_true = P.ellipse_phantom(n, 3)
    g0 = A(f_true)
    g = g0 + 0.05 * np.linalg.norm(g0) * P.randn((NT, M), 4) / np.sqrt(NT * M)
    # ||A||_{X->Y} = sqrt(wy) sigma_max(Am) / h
    L = np.sqrt(wy) * np.linalg.svd(Am, compute_uv=False)[0] / h
    mu = L / (np.sqrt(8.0) / h)
    Kn = np.sqrt(2.0) * L
    return dict(n=n, h=h, wy=wy, Am=Am, A=A, As=As, g=g, tau=0.99 / (L * Kn), sigma=0.99 * L / Kn, mu=mu)


def test_grad_div_are_adjoint_and_neumann():
    rng = np.random.default_rng(0)
    f = rng.standard_normal((7, 5))
    p = rng.standard_normal((2, 7, 5))
    h = 0.3
    lhs = float(np.sum(S.grad_h(f, h) * p))
    rhs = -float(np.sum(f * S.div_h(p, h)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    gr = S.grad_h(f, h)
    assert np.all(gr[0][:, -1] == 0) and np.all(gr[1][-1, :] == 0)
    # a linear ramp in x has the constant slope away from the last column
    ramp = np.tile(np.arange(5.0), (7, 1))
    assert np.allclose(S.grad_h(ramp, 0.5)[0][:, :-1], 2.0) and np.all(S.grad_h(ramp, 0.5)[1] == 0)


def test_tv_dual_projection():
    p = np.zeros((2, 1, 3))
    p[0, 0] = [3.0, 0.1, 0.0]
    p[1, 0] = [4.0, 0.0, -2.0]
    q = S.project_tv_dual(p, 1.0)
    assert np.allclose(q[:, 0, 0], [0.6, 0.8]) and np.allclose(q[:, 0, 1], [0.1, 0.0])
    assert np.allclose(q[:, 0, 2], [0.0, -1.0])


def test_cp_without_tv_converges_to_nnls(problem):
    """lam = 0: the minimiser is the non-negative least-squares solution
    (scipy.optimize.nnls on the explicit matrix; the weights are scalars)."""
    pb = problem
    f = S.cp_tv(pb["A"], pb["As"], pb["g"], pb["n"], pb["h"], 0.0, pb["tau"], pb["sigma"], pb["mu"], 20000)
    ref, _ = so.nnls(pb["Am"], pb["g"].ravel(), maxiter=10000)
    assert np.linalg.norm(f.ravel() - ref) <= 1e-6 * np.linalg.norm(ref)
    # projected-gradient NNLS reaches the same point
    L2 = (pb["wy"] / pb["h"] ** 2) * np.linalg.svd(pb["Am"], compute_uv=False)[0] ** 2
    fn = S.nnls_pg(pb["A"], pb["As"], pb["g"], pb["n"], 1.0 / L2, 20000)
    assert np.linalg.norm(fn.ravel() - ref) <= 1e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("frac", [0.02, 0.2])
def test_cp_tv_reaches_the_dual_optimum(problem, frac):
    """The CP-TV limit has the optimal value of the TV problem, certified by
    an independent solve of its dual (a concave quadratic over (q, p) with
    A* q - div_h p >= 0 and |p_pixel| <= lam, SLSQP): weak duality puts the
    dual value below every primal value, so equal values pin the minimiser."""
    pb = problem
    n, h, wy, g = pb["n"], pb["h"], pb["wy"], pb["g"]
    lam = frac * float(np.abs(pb["As"](g)).max())
    f = S.cp_tv(pb["A"], pb["As"], g, n, h, lam, pb["tau"], pb["sigma"], pb["mu"], 20000)
    primal = S.tv_objective(pb["A"], f, g, lam, h, wy)
    nq = NT * M

    def dual_neg(x):
        q = x[:nq]
        return wy * float(np.dot(q, g.ravel())) + 0.5 * wy * float(np.dot(q, q))

    def dual_neg_jac(x):
        return np.concatenate([wy * (g.ravel() + x[:nq]), np.zeros(2 * n * n)])

    def feas_lin(x):
        return (pb["As"](x[:nq].reshape(NT, M)) - S.div_h(x[nq:].reshape(2, n, n), h)).ravel()

    def feas_ball(x):
        p = x[nq:].reshape(2, n, n)
        return (lam ** 2 - (p[0] ** 2 + p[1] ** 2)).ravel()

    res = so.minimize(dual_neg, np.zeros(nq + 2 * n * n), jac=dual_neg_jac, method="SLSQP",
                      constraints=[{"type": "ineq", "fun": feas_lin}, {"type": "ineq", "fun": feas_ball}],
                      options={"ftol": 1e-16, "maxiter": 10000})
    dual = -res.fun
    assert feas_lin(res.x).min() >= -1e-9 and feas_ball(res.x).min() >= -1e-12
    assert abs(primal - dual) <= 1e-9 * primal, (primal, dual)
    # the TV term is active: the solution differs from the NNLS one
    f0 = S.cp_tv(pb["A"], pb["As"], g, n, h, 0.0, pb["tau"], pb["sigma"], pb["mu"], 20000)
    assert np.linalg.norm(f - f0) > 1e-3 * np.linalg.norm(f0)
