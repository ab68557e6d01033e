"""CPU FP64 oracle for the circular-geometry photoacoustic operators A and A*.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product package never
imports, links or runs anything here, and nothing here imports the product
package: the two share no code.  Inputs arrive as plain numpy arrays and a
plain ``dict`` geometry with keys

    n, a, R, c, m, theta0, arc, nt, T, rho, mask_radius

(pixel centres x_pq = -a + (index + 1/2) h with h = 2a/n; detectors
theta_i = theta0 + i*arc/m on the circle of radius R; times t_j = (j+1) T/nt).

Routes (each cites the passage of Hauptmann, Kunyansky & Poimala,
arXiv 2510.24687, that it follows):

* ``forward`` / ``adjoint`` -- the primary oracle (C, ``pat_oracle.c``):
  direct Gauss-Legendre quadrature of the J0 form of the band-limited model
  of eq. E:kwave (Sec. 2.1.1), and the exact weighted transpose under the
  rectangle-rule discretisation of the inner products eqn:innerProducts.
* ``gauss_forward`` -- semi-closed form for a sum of Gaussians: the same J0
  integral with the Gaussian's analytic transform (eq. E:kwave + E:Anger).
* ``poisson_gauss`` -- an independent physical-space route: the 2D Poisson
  (Kirchhoff) solution of the Cauchy problem E:wave-eq / E:Cauchy written
  with circular means, for Gaussian data.  Pins ``gauss_forward``.
* ``kspace_forward`` -- the paper's own verification route (the
  unaccelerated Fourier algorithm of eq. E:kwave, Sec. 2.1.1) evaluated with
  a 2D trapezoid rule in xi and a direct sum at the detectors.  Pins
  ``forward`` on arbitrary images.
* ``fd_gauss`` -- brute-force second-order leapfrog in time with a 4th-order
  Laplacian (the finite-difference approach of Sec. 2.1.1) for Gaussian data
  on a small box.  Pins the physics of ``gauss_forward``.
* ``ubp`` / ``inverse`` -- the approximate inverse of Sec. 3.3 (Alg. 3): the
  back-projection of eq. E:approx_UBP with the band-limited fundamental
  solution (C, direct quadrature of its J1 form), the constant of eq.
  E:silly_integral and the restriction to the support.
* ``measure`` -- the measurement operator B of eq. E:real_meas (Sec. 2):
  attenuation e^{-gamma t}, then the 1D Fourier filter eta in t per detector
  trace (numpy FFT of the zero-extended trace), and its adjoint.
* ``kspace_ubp`` -- an independent route to the same back-projection: the
  2D Fourier integral of the normal derivative of G (eq. E:Fourier_Green)
  evaluated on a polar quadrature grid, with no Bessel functions.  Pins
  ``ubp``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pat_oracle.c")
_LIB = os.path.join(_HERE, "libpat_oracle.so")
_lib = None


class _Geom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("a", ctypes.c_double), ("R", ctypes.c_double),
                ("c", ctypes.c_double), ("m", ctypes.c_int), ("theta0", ctypes.c_double),
                ("arc", ctypes.c_double), ("nt", ctypes.c_int), ("T", ctypes.c_double),
                ("rho", ctypes.c_double), ("mask_radius", ctypes.c_double)]


GEOM_DEFAULTS = dict(a=1.0, R=1.0, c=1.0, theta0=0.0, arc=2 * np.pi, T=2.0, rho=0.8, mask_radius=0.0)


def build(force: bool = False) -> str:
    """Compile the C oracle (plain gcc, IEEE arithmetic, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        gp = ctypes.POINTER(_Geom)
        lib.ora_forward.argtypes = [gp, dp, ctypes.c_int, dp, dp, ctypes.c_int, ip, dp]
        lib.ora_adjoint.argtypes = [gp, dp, ctypes.c_int, dp, dp, ctypes.c_int, ip, dp]
        lib.ora_ubp.argtypes = [gp, dp, ctypes.c_int, dp, dp, ctypes.c_int, ip, dp]
        lib.ora_gauss.argtypes = [gp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_int, dp, dp, ctypes.c_int, ip, dp]
        lib.ora_taper.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.ora_taper.restype = ctypes.c_double
        _lib = lib
    return _lib


def full_geom(geom: dict) -> dict:
    g = dict(GEOM_DEFAULTS)
    g.update(geom)
    return g


def _cgeom(geom: dict) -> _Geom:
    g = full_geom(geom)
    return _Geom(int(g["n"]), float(g["a"]), float(g["R"]), float(g["c"]), int(g["m"]),
                 float(g["theta0"]), float(g["arc"]), int(g["nt"]), float(g["T"]),
                 float(g["rho"]), float(g["mask_radius"]))


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def taper(lam, Lam, rho):
    """W(lambda) of the band-limited model (scalar or array)."""
    lib = _load()
    return np.vectorize(lambda x: lib.ora_taper(float(x), float(Lam), float(rho)))(lam)


def gl_nodes(lmax: float, phase_rate: float, phase_per_panel: float = 10.0, nodes: int = 20,
             refine=None):
    """Composite Gauss-Legendre nodes/weights on [0, lmax]; each panel spans at
    most ``phase_per_panel`` radians of an oscillation with rate ``phase_rate``.
    ``refine=(lo, hi)`` halves the panel width inside [lo, hi]."""
    width = phase_per_panel / max(phase_rate, 1e-300)
    edges = [0.0]
    while edges[-1] < lmax:
        w = width
        if refine is not None and refine[0] <= edges[-1] < refine[1]:
            w = width / 2
        edges.append(min(lmax, edges[-1] + w))
    x, w = np.polynomial.legendre.leggauss(nodes)
    lam, wt = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        lam.append(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
        wt.append(0.5 * (hi - lo) * w)
    return np.concatenate(lam), np.concatenate(wt)


def quad_nodes(geom: dict, phase_per_panel: float = 10.0, nodes: int = 20):
    """Nodes for Q(t,d) on [0, Lambda]: the integrand oscillates at most at rate
    d_max + cT with d_max = R + sqrt(2) a; panels are halved in the taper zone."""
    g = full_geom(geom)
    h = 2 * g["a"] / g["n"]
    Lam = np.pi / h
    rate = g["R"] + np.sqrt(2) * g["a"] + g["c"] * g["T"]
    return gl_nodes(Lam, rate, phase_per_panel, nodes, refine=(g["rho"] * Lam, Lam))


def forward(geom: dict, f, dets=None, phase_per_panel: float = 10.0, nodes: int = 20):
    """[A f]_{j,i} for all t_j and the listed detectors (all if None).
    Returns an (nt, ndet) array."""
    lib = _load()
    g = full_geom(geom)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(g["n"], g["n"])
    lam, wl = quad_nodes(g, phase_per_panel, nodes)
    d = None if dets is None else np.ascontiguousarray(dets, dtype=np.int32)
    nd = g["m"] if d is None else len(d)
    out = np.zeros((g["nt"], nd))
    rc = lib.ora_forward(ctypes.byref(_cgeom(g)), _dptr(f), len(lam), _dptr(lam), _dptr(wl),
                         nd, _iptr(d), _dptr(out))
    if rc != 0:
        raise RuntimeError("ora_forward failed")
    return out


def adjoint(geom: dict, gtr, pix=None, phase_per_panel: float = 10.0, nodes: int = 20):
    """[A* g]_pq (weighted adjoint) on the listed flat pixel indices (all if None).
    Returns an (n, n) array when pix is None, else a vector."""
    lib = _load()
    g = full_geom(geom)
    gtr = np.ascontiguousarray(gtr, dtype=np.float64).reshape(g["nt"], g["m"])
    lam, wl = quad_nodes(g, phase_per_panel, nodes)
    p = None if pix is None else np.ascontiguousarray(pix, dtype=np.int32)
    npix = g["n"] ** 2 if p is None else len(p)
    out = np.zeros(npix)
    rc = lib.ora_adjoint(ctypes.byref(_cgeom(g)), _dptr(gtr), len(lam), _dptr(lam), _dptr(wl),
                         npix, _iptr(p), _dptr(out))
    if rc != 0:
        raise RuntimeError("ora_adjoint failed")
    return out.reshape(g["n"], g["n"]) if p is None else out


def adjoint_scale(geom: dict) -> float:
    """s with A* = s A^T: (T/nt) (R arc/m) / h^2 (rectangle-rule weights of eqn:innerProducts)."""
    g = full_geom(geom)
    h = 2 * g["a"] / g["n"]
    return (g["T"] / g["nt"]) * (g["R"] * g["arc"] / g["m"]) / h ** 2


def ubp(geom: dict, gtr, pix=None, phase_per_panel: float = 10.0, nodes: int = 20):
    """Back-projection v of eq. E:approx_UBP (Sec. 3.3) on the listed flat pixel
    indices (all if None), before the constant and the restriction:

        v(x) = 2 c^2 w_t w_th sum_{j,i} g[j][i] d/dn(z_i) G_W(t_j, x - z_i),

    G_W the fundamental solution of the band-limited model (spectrum
    W(|xi|) sin(c|xi|t) / (2 pi c |xi|)) and n(z_i) = -z_i/R the normal
    pointing into the disk (the sign with which the formula is a left
    inverse; the sign of eq. E:Four_coef_v).  Arc data count as the full
    circle extended by zero (Alg. 3, first step).  Returns (n, n) or a
    vector."""
    lib = _load()
    g = full_geom(geom)
    gtr = np.ascontiguousarray(gtr, dtype=np.float64).reshape(g["nt"], g["m"])
    lam, wl = quad_nodes(g, phase_per_panel, nodes)
    p = None if pix is None else np.ascontiguousarray(pix, dtype=np.int32)
    npix = g["n"] ** 2 if p is None else len(p)
    out = np.zeros(npix)
    rc = lib.ora_ubp(ctypes.byref(_cgeom(g)), _dptr(gtr), len(lam), _dptr(lam), _dptr(wl),
                     npix, _iptr(p), _dptr(out))
    if rc != 0:
        raise RuntimeError("ora_ubp failed")
    return out.reshape(g["n"], g["n"]) if p is None else out


def support_masks(geom: dict):
    """(omega0, annulus) boolean n x n masks: omega0 is the support Omega_0 of
    f (the disk of radius mask_radius, or the whole image without a mask);
    annulus = pixel centres in the detector disk Omega (|x| <= R) outside
    Omega_0, where eq. E:silly_integral asks v + C to integrate to zero."""
    g = full_geom(geom)
    n = g["n"]
    h = 2 * g["a"] / n
    c = -g["a"] + (np.arange(n) + 0.5) * h
    r2 = c[None, :] ** 2 + c[:, None] ** 2
    omega0 = r2 <= g["mask_radius"] ** 2 if g["mask_radius"] > 0 else np.ones((n, n), bool)
    annulus = (r2 <= g["R"] ** 2) & ~omega0
    return omega0, annulus


def ubp_constant(geom: dict, v) -> float:
    """C of eq. E:silly_integral: the pixel-sum (midpoint rule) of v + C over
    Omega minus Omega_0 vanishes; 0 when that set holds no pixel centre."""
    _, ann = support_masks(geom)
    cnt = int(ann.sum())
    return 0.0 if cnt == 0 else -float(np.sum(np.asarray(v)[ann])) / cnt


def inverse(geom: dict, gtr):
    """Approximate inverse of Alg. 3: Pi_{Omega_0}(v + C) on the n x n grid."""
    v = ubp(geom, gtr)
    om0, _ = support_masks(geom)
    return np.where(om0, v + ubp_constant(geom, v), 0.0)


def kspace_ubp(geom: dict, gtr, pix=None, n_phi: int = 0, phase_per_panel: float = 10.0, nodes: int = 20):
    """The back-projection v of ``ubp`` by another route: G_W(t, y) is the
    inverse 2D transform (Sec. 2.1.1) of W sin(c|xi|t)/(2 pi c|xi|) (eq.
    E:Fourier_Green with its 1/(2 pi)), so

      d/dn(z) G_W(t, x - z) = (2 pi)^-2 int W(|xi|) sin(c|xi|t)/(c|xi|) (-i n.xi) e^{i xi.(x - z)} dxi,

    and, with the inward normal n_i = -z_i/R, v(x) = int V(xi) e^{i xi.x} dxi,
      V(xi) = 2 i c w_t w_th (2 pi)^-2 W(|xi|) sum_{j,i} g[j][i] sin(c|xi|t_j) (z_i.xi/(R|xi|)) e^{-i xi.z_i}.
    The xi integral runs over the disk |xi| < Lambda in polar coordinates:
    composite Gauss-Legendre in |xi| (``quad_nodes``) and the trapezoid rule
    in angle (exact for the trigonometric polynomials of degree < n_phi that
    appear).  Plain numpy, meant for small n."""
    g = full_geom(geom)
    n, m, nt = g["n"], g["m"], g["nt"]
    h = 2 * g["a"] / n
    Lam = np.pi / h
    if n_phi <= 0:
        n_phi = int(2 * np.ceil(Lam * (g["R"] + np.sqrt(2) * g["a"])) + 40)
    lam, wl = quad_nodes(g, phase_per_panel, nodes)
    Wl = np.array([_taper_np(x, Lam, g["rho"]) for x in lam])
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    gtr = np.asarray(gtr, dtype=np.float64).reshape(nt, m)
    th = g["theta0"] + np.arange(m) * g["arc"] / m
    zx, zy = g["R"] * np.cos(th), g["R"] * np.sin(th)
    t = (np.arange(nt) + 1) * g["T"] / nt
    xc = -g["a"] + (np.arange(n) + 0.5) * h
    if pix is None:
        pix = np.arange(n * n)
    pix = np.asarray(pix)
    px, py = xc[pix % n], xc[pix // n]
    wt, wth = g["T"] / nt, g["R"] * g["arc"] / m
    pref = 2j * g["c"] * wt * wth / (2 * np.pi) ** 2
    out = np.zeros(len(pix), dtype=complex)
    for l in range(len(lam)):
        xi_x, xi_y = lam[l] * np.cos(phi), lam[l] * np.sin(phi)          # (n_phi,)
        sj = np.sin(g["c"] * lam[l] * t)                                  # (nt,)
        gi = sj @ gtr                                                     # (m,): sum_j g[j][i] sin
        nxi = np.cos(th)[None, :] * np.cos(phi)[:, None] + np.sin(th)[None, :] * np.sin(phi)[:, None]
        ez = np.exp(-1j * (xi_x[:, None] * zx[None, :] + xi_y[:, None] * zy[None, :]))
        V = pref * Wl[l] * ((nxi * ez) @ gi)                              # (n_phi,)
        ex = np.exp(1j * (px[:, None] * xi_x[None, :] + py[:, None] * xi_y[None, :]))
        out += wl[l] * lam[l] * (2 * np.pi / n_phi) * (ex @ V)
    return out.real.reshape(n, n) if len(pix) == n * n else out.real


def gauss_forward(geom: dict, blobs, taper_grid: bool = False, dets=None,
                  phase_per_panel: float = 10.0, nodes: int = 20):
    """Semi-closed form for f = sum_b amp_b exp(-|x-c_b|^2/(2 s_b^2)).
    blobs: (nb, 4) rows (cx, cy, sigma, amp).  With ``taper_grid`` the radial
    taper W of the n x n grid is applied (the band-limited model of that grid);
    otherwise W = 1 (the exact wave solution)."""
    lib = _load()
    g = full_geom(geom)
    blobs = np.ascontiguousarray(blobs, dtype=np.float64).reshape(-1, 4)
    smin = blobs[:, 2].min()
    lmax = 9.5 / smin
    Lam = np.pi / (2 * g["a"] / g["n"])
    if taper_grid:
        lmax = min(lmax, Lam)
    dmax = g["R"] + np.abs(blobs[:, :2]).sum(axis=1).max()
    lam, wl = gl_nodes(lmax, dmax + g["c"] * g["T"], phase_per_panel, nodes)
    d = None if dets is None else np.ascontiguousarray(dets, dtype=np.int32)
    nd = g["m"] if d is None else len(d)
    out = np.zeros((g["nt"], nd))
    rc = lib.ora_gauss(ctypes.byref(_cgeom(g)), len(blobs), _dptr(blobs), int(bool(taper_grid)),
                       float(Lam), len(lam), _dptr(lam), _dptr(wl), nd, _iptr(d), _dptr(out))
    if rc != 0:
        raise RuntimeError("ora_gauss failed")
    return out


def poisson_gauss(blobs, t, z, c: float = 1.0, panels: int = 4000, nodes: int = 16):
    """Pressure p(t, z) of the Cauchy problem E:wave-eq/E:Cauchy with Gaussian
    initial data, from the 2D Poisson formula in circular means:

        p(t,z) = int_0^{pi/2} sin(a) [d/dr (r M(r))]_{r = c t sin a} da,

    M(r) = mean of f over the circle of radius r about z.  For one Gaussian at
    distance d from z, M(r) = amp exp(-(r-d)^2/(2s^2)) I0e(r d/s^2), so
    d(rM)/dr = amp exp(-(r-d)^2/(2s^2)) [ (1 - r^2/s^2) I0e(x) + (r d/s^2) I1e(x) ],
    x = r d / s^2.  No Fourier transform or Bessel J enters."""
    from scipy.special import i0e, i1e
    blobs = np.asarray(blobs, dtype=np.float64).reshape(-1, 4)
    x, w = np.polynomial.legendre.leggauss(nodes)
    edges = np.linspace(0.0, np.pi / 2, panels + 1)
    lo, hi = edges[:-1, None], edges[1:, None]
    al = (0.5 * (hi - lo) * x + 0.5 * (hi + lo)).ravel()
    wa = (0.5 * (hi - lo) * w).ravel()
    out = np.zeros((len(t), len(z)))
    for ti, tv in enumerate(t):
        r = c * tv * np.sin(al)
        for zi, zv in enumerate(z):
            acc = np.zeros_like(r)
            for cx, cy, s, amp in blobs:
                d = np.hypot(zv[0] - cx, zv[1] - cy)
                xx = r * d / s ** 2
                acc += amp * np.exp(-(r - d) ** 2 / (2 * s * s)) * ((1 - r * r / s ** 2) * i0e(xx) + xx * i1e(xx))
            out[ti, zi] = np.sum(wa * np.sin(al) * acc)
    return out


def kspace_forward(geom: dict, f, dets=None, delta=None, chunk: int = 4096):
    """The unaccelerated Fourier route (eq. E:kwave, Sec. 2.1.1):
        g(t,z) = (1/2pi) int W(|xi|) F(xi) cos(c|xi|t) exp(i xi.z) dxi,
    F(xi) = (h^2/2pi) sum f_pq exp(-i xi.x_pq), evaluated by the trapezoid rule
    on the lattice xi = delta*(k1,k2), |xi| < Lambda (spectrally accurate: the
    integrand is smooth and compactly supported), and a direct sum at each
    detector.  Returns (nt, ndet)."""
    g = full_geom(geom)
    n, a = g["n"], g["a"]
    h = 2 * a / n
    Lam = np.pi / h
    if delta is None:
        delta = 2 * np.pi / (g["R"] + np.sqrt(2) * a + g["c"] * g["T"] + 8.0)
    kmax = int(np.ceil(Lam / delta))
    k = np.arange(-kmax, kmax + 1) * delta
    KX, KY = np.meshgrid(k, k)
    keep = np.hypot(KX, KY) < Lam
    xi_x, xi_y = KX[keep], KY[keep]
    rad = np.hypot(xi_x, xi_y)
    Wv = taper(rad, Lam, g["rho"]) if len(rad) < 2000 else _taper_np(rad, Lam, g["rho"])
    xs = -a + (np.arange(n) + 0.5) * h
    f = np.asarray(f, dtype=np.float64).reshape(n, n)
    if g["mask_radius"] > 0:
        X, Y = np.meshgrid(xs, xs)
        f = f * (X * X + Y * Y <= g["mask_radius"] ** 2)
    # F on the lattice, separable in x and y
    F = np.empty(len(xi_x), complex)
    for s0 in range(0, len(xi_x), chunk):
        ex = np.exp(-1j * np.outer(xi_x[s0:s0 + chunk], xs))  # (c, q)
        ey = np.exp(-1j * np.outer(xi_y[s0:s0 + chunk], xs))  # (c, p)
        F[s0:s0 + chunk] = np.einsum("cp,pq,cq->c", ey, f, ex)
    F *= h * h / (2 * np.pi)
    th = g["theta0"] + np.arange(g["m"]) * g["arc"] / g["m"]
    if dets is not None:
        th = th[np.asarray(dets)]
    t = (np.arange(g["nt"]) + 1) * g["T"] / g["nt"]
    zx, zy = g["R"] * np.cos(th), g["R"] * np.sin(th)
    out = np.zeros((g["nt"], len(th)))
    for s0 in range(0, len(xi_x), chunk):
        sl = slice(s0, s0 + chunk)
        A = np.cos(g["c"] * np.outer(t, rad[sl])) * (Wv[sl] * F[sl])[None, :]
        E = np.exp(1j * (np.outer(xi_x[sl], zx) + np.outer(xi_y[sl], zy)))
        out += (A @ E).real
    return out * delta * delta / (2 * np.pi)


def _taper_np(lam, Lam, rho):
    lam = np.asarray(lam, dtype=np.float64)
    W = np.where(lam <= rho * Lam, 1.0, 0.0)
    mid = (lam > rho * Lam) & (lam < Lam)
    u = (Lam - lam[mid]) / ((1 - rho) * Lam)
    e1, e2 = np.exp(-1 / u), np.exp(-1 / (1 - u))
    W[mid] = e1 / (e1 + e2)
    return W


def fd_gauss(blobs, dets_xy, times, dx: float, box: float, c: float = 1.0, nu: float = 0.5):
    """Brute-force leapfrog solution of E:wave-eq/E:Cauchy for Gaussian data on
    [-box, box]^2 with zero Dirichlet boundary, 4th-order central Laplacian,
    Courant number nu = c dt/dx, first step from the Taylor expansion
    p(dt) = p0 + (c dt)^2/2 Lap p0 (p_t(0) = 0).  Detectors must lie on grid
    points; ``times`` must be multiples of dt.  Returns (len(times), ndet)."""
    blobs = np.asarray(blobs, dtype=np.float64).reshape(-1, 4)
    N = int(round(2 * box / dx)) + 1
    xs = -box + np.arange(N) * dx
    X, Y = np.meshgrid(xs, xs)
    p0 = np.zeros((N, N))
    for cx, cy, s, amp in blobs:
        p0 += amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
    dt = nu * dx / c

    def lap(u):
        L = np.zeros_like(u)
        ci = slice(2, -2)
        L[ci, ci] = (-u[ci, 4:] + 16 * u[ci, 3:-1] - 30 * u[ci, ci] + 16 * u[ci, 1:-3] - u[ci, :-4]
                     - u[4:, ci] + 16 * u[3:-1, ci] - 30 * u[ci, ci] + 16 * u[1:-3, ci] - u[:-4, ci]) / (12 * dx * dx)
        return L

    idx = [(int(round((zy + box) / dx)), int(round((zx + box) / dx))) for zx, zy in dets_xy]
    steps = [int(round(tv / dt)) for tv in times]
    for tv, st in zip(times, steps):
        if abs(st * dt - tv) > 1e-9:
            raise ValueError("times must be multiples of dt")
    out = np.zeros((len(times), len(idx)))
    prev = p0
    cur = p0 + 0.5 * (c * dt) ** 2 * lap(p0)
    k = 1
    want = {st: i for i, st in enumerate(steps)}
    if 0 in want:
        out[want[0]] = [p0[i] for i in idx]
    while k <= max(steps):
        if k in want:
            out[want[k]] = [cur[i] for i in idx]
        nxt = 2 * cur - prev + (c * dt) ** 2 * lap(cur)
        prev, cur = cur, nxt
        k += 1
    return out


# ---------------------------------------------------------------------------
# Measurement operator B of eq. E:real_meas (Sec. 2): attenuation e^{-gamma t}
# and a transducer response eta applied as a 1D Fourier filter in t.
# ---------------------------------------------------------------------------
def filter_length(nt: int) -> int:
    """Length N of the discrete transform in t: the smallest power of two
    >= 2 nt (each trace is zero-extended from nt to N samples, so the filter's
    wrap-around never mixes the end of a record into its start)."""
    N = 1
    while N < 2 * nt:
        N *= 2
    return N


def response_full(eta, N: int):
    """eta at the N frequencies of the DFT, xi_k = 2 pi k / (N dt): the given
    values for k = 0..N/2 and eta(-xi) = conj(eta(xi)) (a real filter) above;
    eta_0 and eta_{N/2} contribute their real parts."""
    eta = np.asarray(eta, dtype=complex)
    if eta.shape != (N // 2 + 1,):
        raise ValueError("eta must hold N/2 + 1 values")
    H = np.zeros(N, dtype=complex)
    H[:N // 2 + 1] = eta
    H[0], H[N // 2] = eta[0].real, eta[N // 2].real
    H[N // 2 + 1:] = np.conj(eta[1:N // 2][::-1])
    return H


def measure(geom: dict, g, gamma: float, eta, adjoint: bool = False):
    """B (or its adjoint) on traces g (nt x m, time-major):

        B g = D(e^{-gamma t} g),   D h = F^-1(eta F h)  per detector trace,

    eq. E:real_meas with F the DFT of the trace zero-extended to
    N = filter_length(nt) samples (t_j = (j+1) T/nt), the result cut back to
    the nt measured samples.  Under the trace inner product (the same
    weights w_t w_th on both sides) the adjoint is
    B* g = e^{-gamma t} F^-1(conj(eta) F g), with the same extension and cut."""
    gg = full_geom(geom)
    nt, m = gg["nt"], gg["m"]
    g = np.asarray(g, dtype=np.float64).reshape(nt, m)
    N = filter_length(nt)
    H = response_full(eta, N)
    e = np.exp(-gamma * (np.arange(nt) + 1) * gg["T"] / nt)[:, None]
    h = g if adjoint else e * g
    pad = np.zeros((N, m))
    pad[:nt] = h
    out = np.fft.ifft((np.conj(H) if adjoint else H)[:, None] * np.fft.fft(pad, axis=0), axis=0).real[:nt]
    return e * out if adjoint else out


def transducer_response(nt: int, T: float, f0: float, bw: float):
    """A smooth band-pass response for tests and benchmarks (the paper leaves
    eta open): eta(xi) = exp(-(|xi| - 2 pi f0)^2 / (2 (2 pi bw)^2)) -
    exp(-(|xi| + 2 pi f0)^2 / ...) times a half-sample delay phase, at the
    N/2 + 1 non-negative DFT frequencies of filter_length(nt)."""
    N = filter_length(nt)
    dt = T / nt
    xi = 2 * np.pi * np.arange(N // 2 + 1) / (N * dt)
    w0, s = 2 * np.pi * f0, 2 * np.pi * bw
    mag = np.exp(-(xi - w0) ** 2 / (2 * s * s)) - np.exp(-(xi + w0) ** 2 / (2 * s * s))
    return mag * np.exp(-0.5j * xi * dt)
