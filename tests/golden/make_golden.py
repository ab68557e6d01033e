"""Write sampled oracle values for the large parity cases.

Calls only the CPU FP64 oracle (``oracle/``) and the seeded input generators;
nothing here touches the GPU library.  Each case stores, for a seeded input,
the oracle's forward traces at a seeded subset of detectors (all times) and
the oracle's weighted adjoint of seeded N(0,1) traces at a seeded subset of
pixels.  The ``inv_*`` cases store the back-projection v of the approximate
inverse (before its constant; no mask) of seeded N(0,1) traces at a seeded
subset of pixels.  The ``grad_*`` cases store the gradient of the data
fidelity ||A f - g||^2 with g = A f' + noise at a seeded subset of pixels.
Run from the repository root:
python tests/golden/make_golden.py [case names]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2510_24687_amd import phantoms as P  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# name -> (geometry, image seed, trace seed, detectors sampled, pixels sampled)
CASES = {
    "full_n256": (P.full_circle(256, 512, 512, T=2.0), 0, 1, 8, 256),
    "arc180_n256": (P.top_arc(256, 256, 512, 180.0, T=2.0), 2, 3, 8, 256),
    "arc180_n128": (P.top_arc(128, 256, 256, 180.0, T=2.0), 4, 5, 8, 256),
    "full_n512": (P.full_circle(512, 1024, 1024, T=2.0), 0, 1, 8, 256),
}


# name -> (geometry, trace seed, pixels sampled)
INV_CASES = {
    "inv_full_n256": (P.full_circle(256, 512, 512, T=2.0), 21, 128),
    "inv_full_n512": (P.full_circle(512, 1024, 1024, T=2.0), 22, 128),
}


# name -> (geometry, image seeds f and f' of batch image 0, noise seed, pixels sampled)
# Data-fidelity gradient of the differentiation workload: g = A f' + noise, the
# gradient of ||A f - g||^2 at f is 2 A^T (A f - g).  The noise is sigma * eps,
# eps i.i.d. N(0,1) (seeded), sigma = 5 % of the RMS of the oracle's A f' on
# eight sampled detectors; sigma is stored so that both sides use the same
# noise vector.
GRAD_CASES = {
    "grad_full_n256": (P.full_circle(256, 512, 512, T=2.0), 710, 810, 910, 256),
}


def make_gradient(name):
    geom, fseed, fpseed, nseed, npix = GRAD_CASES[name]
    n, m, nt = geom["n"], geom["m"], geom["nt"]
    rng = np.random.default_rng(3000 + fseed)
    pix = np.sort(rng.choice(n * n, size=npix, replace=False)).astype(np.int32)
    dets = np.sort(rng.choice(m, size=8, replace=False)).astype(np.int32)
    f, fp = P.ellipse_phantom(n, fseed), P.ellipse_phantom(n, fpseed)
    t0 = time.time()
    sigma = 0.05 * float(np.sqrt(np.mean(oracle.forward(geom, fp, dets=dets) ** 2)))
    eps = P.randn((nt, m), nseed)
    # A f - g = A (f - f') - sigma eps (linearity of the oracle's A)
    r = oracle.forward(geom, f - fp) - sigma * eps
    grad = 2.0 * oracle.adjoint(geom, r, pix=pix) / oracle.adjoint_scale(geom)
    np.savez(os.path.join(HERE, name + ".npz"), pix=pix, grad=grad, sigma=sigma, f_seed=fseed, fp_seed=fpseed,
             noise_seed=nseed, geometry=np.array(repr(sorted(geom.items()))))
    print("%s: gradient %.1fs" % (name, time.time() - t0), flush=True)


def make_inverse(name):
    geom, gseed, npix = INV_CASES[name]
    n, m, nt = geom["n"], geom["m"], geom["nt"]
    rng = np.random.default_rng(2000 + gseed)
    pix = np.sort(rng.choice(n * n, size=npix, replace=False)).astype(np.int32)
    y = P.randn((nt, m), gseed)
    t0 = time.time()
    v = oracle.ubp(geom, y, pix=pix)
    np.savez(os.path.join(HERE, name + ".npz"), pix=pix, ubp=v, trace_seed=gseed,
             geometry=np.array(repr(sorted(geom.items()))))
    print("%s: back-projection %.1fs" % (name, time.time() - t0), flush=True)


def make(name):
    geom, fseed, gseed, ndet, npix = CASES[name]
    n, m, nt = geom["n"], geom["m"], geom["nt"]
    rng = np.random.default_rng(1000 + fseed)
    dets = np.sort(rng.choice(m, size=ndet, replace=False)).astype(np.int32)
    pix = np.sort(rng.choice(n * n, size=npix, replace=False)).astype(np.int32)
    f = P.ellipse_phantom(n, fseed)
    y = P.randn((nt, m), gseed)
    t0 = time.time()
    g_s = oracle.forward(geom, f, dets=dets)
    t1 = time.time()
    a_s = oracle.adjoint(geom, y, pix=pix)
    t2 = time.time()
    np.savez(os.path.join(HERE, name + ".npz"), dets=dets, pix=pix, forward=g_s, adjoint=a_s,
             image_seed=fseed, trace_seed=gseed, geometry=np.array(repr(sorted(geom.items()))))
    print("%s: forward %.1fs adjoint %.1fs" % (name, t1 - t0, t2 - t1), flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES) + list(INV_CASES) + list(GRAD_CASES)):
        if name in INV_CASES:
            make_inverse(name)
        elif name in GRAD_CASES:
            make_gradient(name)
        else:
            make(name)
