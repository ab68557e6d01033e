"""Seeded synthetic inputs: phantoms, Gaussian blobs, noise, random traces.

This module holds input generators only -- none of the operators' arithmetic.
It is shared by the GPU path's tests/benchmarks and by the oracle's tests, so
that both sides see identical inputs.  All randomness is numpy PCG64
(``numpy.random.default_rng(seed)``), reproducible across machines.

The paper (Hauptmann, Kunyansky & Poimala, arXiv 2510.24687, Sec. 4.1 and
Sec. 4.2.1) describes its phantoms only in words (smoothed characteristic
functions of circles; random ellipses with smoothed boundaries) and does not
ship them, so the recipes below are synthetic stand-ins with the stated
sizes and value ranges.
"""
from __future__ import annotations

import numpy as np


def pixel_centres(n: int, a: float = 1.0) -> np.ndarray:
    """Cell-centred coordinates -a + (k + 1/2) h, h = 2a/n."""
    h = 2.0 * a / n
    return -a + (np.arange(n) + 0.5) * h


def gaussian_blobs(seed: int, count: int = 5, radius: float = 0.8, sigma=(0.03, 0.1),
                   amp=(0.2, 1.0)) -> np.ndarray:
    """Blob parameters, rows (cx, cy, sigma, amp): centres uniform in the disk
    of the given radius (r = radius*sqrt(U), angle 2 pi V), sigma and amplitude
    uniform in the given ranges."""
    rng = np.random.default_rng(seed)
    out = np.zeros((count, 4))
    for b in range(count):
        r = radius * np.sqrt(rng.random())
        ang = 2 * np.pi * rng.random()
        out[b] = (r * np.cos(ang), r * np.sin(ang), rng.uniform(*sigma), rng.uniform(*amp))
    return out


def sample_blobs(blobs: np.ndarray, n: int, a: float = 1.0) -> np.ndarray:
    """Point samples of sum_b amp_b exp(-|x-c_b|^2/(2 s_b^2)) at pixel centres,
    f[p, q] with p indexing y and q indexing x."""
    xs = pixel_centres(n, a)
    X, Y = np.meshgrid(xs, xs)
    f = np.zeros((n, n))
    for cx, cy, s, amp in np.asarray(blobs).reshape(-1, 4):
        f += amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
    return f


def ellipse_params(seed: int, count: int = 10, support: float = 0.9, axes=(0.05, 0.4)) -> np.ndarray:
    """Random-ellipse parameters, rows (cx, cy, semi-axis 1, semi-axis 2,
    rotation, intensity): per ellipse, semi-axes uniform in ``axes``, rotation
    uniform in [0, pi), intensity uniform in [0, 1]; the centre is
    rejection-sampled until |c| + max(semi-axes) <= support."""
    rng = np.random.default_rng(seed)
    out = np.zeros((count, 6))
    for e in range(count):
        ax1, ax2 = rng.uniform(*axes), rng.uniform(*axes)
        rot = rng.uniform(0.0, np.pi)
        val = rng.uniform(0.0, 1.0)
        lim = support - max(ax1, ax2)
        while True:
            c = rng.uniform(-lim, lim, size=2)
            if np.hypot(*c) <= lim:
                break
        out[e] = (c[0], c[1], ax1, ax2, rot, val)
    return out


def ellipse_phantom(n: int, seed: int, count: int = 10, support: float = 0.9,
                    axes=(0.05, 0.4), a: float = 1.0) -> np.ndarray:
    """Random-ellipse phantom from ellipse_params: the ellipses are summed
    (pixel-centre inclusion) and the result clipped to [0, 1]."""
    xs = pixel_centres(n, a)
    X, Y = np.meshgrid(xs, xs)
    f = np.zeros((n, n))
    for cx, cy, ax1, ax2, rot, val in ellipse_params(seed, count, support, axes):
        cr, sr = np.cos(rot), np.sin(rot)
        u = (X - cx) * cr + (Y - cy) * sr
        v = -(X - cx) * sr + (Y - cy) * cr
        f += val * ((u / ax1) ** 2 + (v / ax2) ** 2 <= 1.0)
    return np.clip(f, 0.0, 1.0)


def ellipse_images(params: np.ndarray, n: int, a: float = 1.0, device="cuda", edge: float = 0.0):
    """The same rasterisation as ellipse_phantom for a stack of parameter sets
    (N, count, 6), done with torch on ``device`` in float64 and returned as
    float32 (N, n, n).  Used to generate large training sets in device memory;
    pixels on an ellipse boundary may differ from the numpy version by the
    last-bit differences of the two sine/cosine implementations.

    ``edge`` > 0 smooths the boundaries (the smoothed ellipses of the paper's
    training data, Sec. 4.2.1): each ellipse contributes
    val * (1 + tanh((1 - rho) sqrt(a1 a2) / edge)) / 2 with
    rho = sqrt((u/a1)^2 + (v/a2)^2) its normalised radius, so the boundary
    layer is about ``edge`` wide (in the units of a)."""
    import torch
    xs = torch.tensor(pixel_centres(n, a), dtype=torch.float64, device=device)
    Y, X = torch.meshgrid(xs, xs, indexing="ij")
    prm = torch.tensor(np.asarray(params, dtype=np.float64), device=device)
    f = torch.zeros((prm.shape[0], n, n), dtype=torch.float64, device=device)
    for e in range(prm.shape[1]):
        cx, cy, ax1, ax2, rot, val = [prm[:, e, i].view(-1, 1, 1) for i in range(6)]
        cr, sr = torch.cos(rot), torch.sin(rot)
        u = (X - cx) * cr + (Y - cy) * sr
        v = -(X - cx) * sr + (Y - cy) * cr
        rho2 = (u / ax1) ** 2 + (v / ax2) ** 2
        if edge > 0:
            f += val * 0.5 * (1.0 + torch.tanh((1.0 - torch.sqrt(rho2)) * torch.sqrt(ax1 * ax2) / edge))
        else:
            f += val * (rho2 <= 1.0)
    return torch.clamp(f, 0.0, 1.0).to(torch.float32)


def ellipse_batch(n: int, seeds, **kw) -> np.ndarray:
    return np.stack([ellipse_phantom(n, int(s), **kw) for s in seeds])


def randn(shape, seed: int) -> np.ndarray:
    """i.i.d. N(0, 1) array."""
    return np.random.default_rng(seed).standard_normal(shape)


def add_noise(g: np.ndarray, level: float, seed: int) -> np.ndarray:
    """g + level * ||g||_2 * e / ||e||_2 with e i.i.d. N(0,1) (relative L2 noise
    level, the noise model described in Sec. 4.3)."""
    e = np.random.default_rng(seed).standard_normal(np.shape(g))
    return g + level * np.linalg.norm(g) * e / np.linalg.norm(e)


def full_circle(n: int, m: int, nt: int, T: float = 2.0, **extra) -> dict:
    """Geometry dict for m equispaced detectors on the whole circle."""
    g = dict(n=n, m=m, nt=nt, T=T, a=1.0, R=1.0, c=1.0, theta0=0.0, arc=2 * np.pi,
             rho=0.8, mask_radius=0.0)
    g.update(extra)
    return g


def top_arc(n: int, m: int, nt: int, arc_deg: float, T: float = 2.0, **extra) -> dict:
    """Geometry dict for m detectors on an arc of the given width centred on the
    top of the circle: theta_i = pi/2 - arc/2 + (i + 1/2) arc/m."""
    arc = np.deg2rad(arc_deg)
    g = dict(n=n, m=m, nt=nt, T=T, a=1.0, R=1.0, c=1.0, theta0=np.pi / 2 - arc / 2 + arc / (2 * m),
             arc=arc, rho=0.8, mask_radius=0.0)
    g.update(extra)
    return g
