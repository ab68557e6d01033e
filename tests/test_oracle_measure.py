"""Pins of the measurement-operator oracle (eq. E:real_meas: attenuation
e^{-gamma t} and a 1D Fourier filter eta in t): a brute-force circular
convolution with the explicitly summed impulse response, the closed forms of
the identity, pure attenuation and an integer delay, and the adjoint
identity."""
import numpy as np
import pytest

import oracle as O
from paper_2510_24687_amd import phantoms as P

NT, M = 10, 6
GEOM = P.full_circle(8, M, NT, T=2.0)


def _traces(seed):
    return np.random.default_rng(seed).standard_normal((NT, M))


def test_filter_length():
    assert [O.filter_length(n) for n in (1, 2, 3, 10, 512, 513, 1024)] == [2, 4, 8, 32, 1024, 2048, 2048]


def test_against_brute_force_convolution():
    N = O.filter_length(NT)
    eta = O.transducer_response(NT, GEOM["T"], 2.0, 1.5)
    H = O.response_full(eta, N)
    # impulse response summed term by term
    d = np.array([sum(H[k] * np.exp(2j * np.pi * j * k / N) for k in range(N)) / N for j in range(N)])
    assert np.max(np.abs(d.imag)) < 1e-12          # a real filter
    gamma = 0.4
    g = _traces(1)
    t = (np.arange(NT) + 1) * GEOM["T"] / NT
    want = np.zeros((NT, M))
    for i in range(M):
        for j in range(NT):
            want[j, i] = sum(d[(j - jp) % N].real * np.exp(-gamma * t[jp]) * g[jp, i] for jp in range(NT))
    assert np.max(np.abs(O.measure(GEOM, g, gamma, eta) - want)) < 1e-12


def test_closed_forms():
    N = O.filter_length(NT)
    g = _traces(2)
    t = (np.arange(NT) + 1) * GEOM["T"] / NT
    ones = np.ones(N // 2 + 1)
    assert np.allclose(O.measure(GEOM, g, 0.0, ones), g, rtol=0, atol=1e-13)
    assert np.allclose(O.measure(GEOM, g, 0.7, ones), np.exp(-0.7 * t)[:, None] * g, rtol=0, atol=1e-13)
    # eta = e^{-i xi s dt}: a delay by s samples (zeros enter at the start)
    s = 3
    delay = np.exp(-2j * np.pi * np.arange(N // 2 + 1) * s / N)
    want = np.zeros_like(g)
    want[s:] = (np.exp(-0.2 * t)[:, None] * g)[:-s]
    assert np.allclose(O.measure(GEOM, g, 0.2, delay), want, rtol=0, atol=1e-13)
    # its adjoint advances: rows shift up, the first s rows fall off the start
    want_a = np.zeros_like(g)
    want_a[:-s] = g[s:]
    assert np.allclose(O.measure(GEOM, g, 0.0, delay, adjoint=True), want_a, rtol=0, atol=1e-13)


@pytest.mark.parametrize("gamma", [0.0, 0.9])
def test_adjoint_identity(gamma):
    eta = O.transducer_response(NT, GEOM["T"], 1.0, 2.0)
    g1, g2 = _traces(3), _traces(4)
    lhs = np.sum(O.measure(GEOM, g1, gamma, eta) * g2)
    rhs = np.sum(g1 * O.measure(GEOM, g2, gamma, eta, adjoint=True))
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(g1) * np.linalg.norm(g2)
