"""Write sampled oracle values for the large parity cases.

Calls only the CPU FP64 oracle (``oracle/``) and the seeded input generators;
nothing here touches the GPU library.  Each case stores, for a seeded input,
the oracle's forward traces at a seeded subset of detectors (all times) and
the oracle's weighted adjoint of seeded N(0,1) traces at a seeded subset of
pixels.  The ``inv_*`` cases store the back-projection v of the approximate
inverse (before its constant; no mask) of seeded N(0,1) traces at a seeded
subset of pixels.  Run from the repository root:
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
    for name in (sys.argv[1:] or list(CASES) + list(INV_CASES)):
        if name in INV_CASES:
            make_inverse(name)
        else:
            make(name)
