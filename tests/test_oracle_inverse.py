"""Pins of the approximate-inverse oracle (Sec. 3.3, Alg. 3): the direct J1
form of the back-projection against an independent Fourier-integral route,
the left-inverse property of the universal back-projection formula (eq.
E:inverse) on exact wave data, and the constant of eq. E:silly_integral."""
import numpy as np
import pytest

import oracle as O
from paper_2510_24687_amd import phantoms as P


def _blob_image(n, blobs):
    h = 2.0 / n
    xc = -1 + (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(xc, xc)
    return sum(b[3] * np.exp(-((X - b[0]) ** 2 + (Y - b[1]) ** 2) / (2 * b[2] ** 2)) for b in blobs)


@pytest.mark.parametrize("geom", [
    P.full_circle(8, 16, 16),
    P.top_arc(8, 12, 20, 180.0, c=1.3, R=1.1),
    P.full_circle(10, 20, 14, T=1.5, mask_radius=0.8, c=0.9, R=1.2, theta0=0.3),
])
def test_ubp_direct_form_matches_fourier_route(geom):
    """Same operator by two derivations: the J1 kernel of the normal
    derivative (C) and the 2D Fourier integral of that derivative on a polar
    grid (numpy, no Bessel functions)."""
    g = np.random.default_rng(3).standard_normal((geom["nt"], geom["m"]))
    v = O.ubp(geom, g)
    k = O.kspace_ubp(geom, g)
    assert np.abs(v - k).max() < 1e-12 * np.abs(v).max()
    # pixel subsets give the same values
    pix = np.array([0, 5, geom["n"] ** 2 - 1, 17])
    assert np.allclose(O.ubp(geom, g, pix=pix), v.ravel()[pix], rtol=0, atol=1e-14 * np.abs(v).max())


@pytest.mark.parametrize("c,R,T,nt,m", [(1.0, 1.0, 8.0, 320, 128), (1.5, 1.3, 6.0, 320, 160)])
def test_backprojection_is_a_left_inverse(c, R, T, nt, m):
    """Exact wave data of two resolved Gaussians supported well inside the
    disk (semi-closed form, no taper): the back-projection returns them to
    ~1e-5 (the finite-T truncation), with the right sign and scale; a
    longer record reduces the error."""
    n = 32
    blobs = np.array([[0.1, -0.05, 0.14, 1.0], [-0.12, 0.1, 0.12, -0.5]])
    f = _blob_image(n, blobs)
    geom = P.full_circle(n, m, nt, T=T, mask_radius=0.9, c=c, R=R)
    om0, _ = O.support_masks(geom)
    v = O.ubp(geom, O.gauss_forward(geom, blobs))
    err = np.linalg.norm((v - f)[om0]) / np.linalg.norm(f[om0])
    assert err < 3e-5, err
    if c == 1.0:
        geom2 = dict(geom, T=12.0, nt=480)
        v2 = O.ubp(geom2, O.gauss_forward(geom2, blobs))
        err2 = np.linalg.norm((v2 - f)[om0]) / np.linalg.norm(f[om0])
        assert err2 < 0.5 * err, (err, err2)


def test_constant_and_restriction():
    geom = P.full_circle(16, 32, 32, mask_radius=0.7)
    g = np.random.default_rng(5).standard_normal((32, 32))
    v = O.ubp(geom, g)
    om0, ann = O.support_masks(geom)
    assert ann.sum() > 0 and not (om0 & ann).any()
    C = O.ubp_constant(geom, v)
    # eq. E:silly_integral: the midpoint sum of v + C over Omega \ Omega_0 vanishes
    assert abs(np.sum(v[ann] + C)) < 1e-12 * np.abs(v).sum()
    f = O.inverse(geom, g)
    assert np.all(f[~om0] == 0.0)
    assert np.allclose(f[om0], v[om0] + C, rtol=0, atol=1e-14)
    # no mask: Omega_0 is the whole image, so there is no annulus and no constant
    geom0 = P.full_circle(16, 32, 32)
    assert O.ubp_constant(geom0, v) == 0.0
    assert np.array_equal(O.inverse(geom0, g), O.ubp(geom0, g))
