"""Reconstruction experiments in the style of the paper's Table 1 (Secs.
4.3-4.5): the acquisition schemes 360 degrees, 180 degrees with a support
that satisfies the visibility condition ("partial"), 180 and 120 degrees
with a support that does not ("incomplete"), clean or with 30 % noise, each
reconstructed by the approximate inverse (Alg. 3), projected-gradient NNLS,
Chambolle-Pock TV and the learned primal-dual network, with the paper's
stopping rule for the iterations (the update's L2 norm below 0.3 % of the
first non-zero iterate's).

The paper's phantom and its k-Wave data are not published; the phantoms here
are the seeded random-ellipse images (characteristic functions of ellipses,
inside the disk |x| <= 0.9), and the data come from the library's forward
operator on a grid twice as fine as the reconstruction grid (n_data = 2n,
same detectors and times), so reconstructions do not see their own
discretisation ("inverse crime").  Errors are relative L2 and L-infinity
norms over the whole n x n image, as in the table.

Everything numerical runs in the library (operators, update kernels,
reductions); this module chooses geometries, seeds and parameters and
records times and errors.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional

import numpy as np
import torch

from . import phantoms as PH
from .pat import Plan
from . import solvers as S

SUPPORT_RADIUS = 0.98   # the disk D of Sec. 4.4

# name -> (arc in degrees, support kind, relative noise, methods); "smooth" schemes
# use ellipses with smoothed boundaries (boundary layer about EDGE wide)
EDGE = 0.03
SCHEMES = {
    "360, no noise": (360.0, "disk", 0.0, ("inverse",)),
    "360, no noise, smooth edges": (360.0, "disk smooth", 0.0, ("inverse",)),
    "360, 30% noise": (360.0, "disk", 0.3, ("inverse", "tv")),
    "180 (partial), no noise": (180.0, "upper", 0.0, ("inverse", "nnls")),
    "180 (partial), 30% noise": (180.0, "upper", 0.3, ("nnls", "tv")),
    "180 (incomplete), 30% noise": (180.0, "disk", 0.3, ("inverse", "nnls", "tv", "lpd")),
    "120 (incomplete), 30% noise": (120.0, "disk", 0.3, ("inverse", "nnls", "tv", "lpd")),
}


def detectors(arc_deg: float, n: int) -> int:
    """2n detectors on the full circle, n on a 180- or 120-degree arc centred
    on the top (full-circle grids of 2n and 3n points)."""
    return 2 * n if arc_deg >= 360.0 else n


def geometry(arc_deg: float, n: int, m: int, nt: int, T: float) -> dict:
    if arc_deg >= 360.0:
        return PH.full_circle(n, m, nt, T=T, mask_radius=SUPPORT_RADIUS)
    return PH.top_arc(n, m, nt, arc_deg, T=T, mask_radius=SUPPORT_RADIUS)


def support(kind: str, n: int, device) -> torch.Tensor:
    """Omega_0 as a 0/1 image: the disk D, or its upper half (Sec. 4.4)."""
    xs = torch.tensor(PH.pixel_centres(n, 1.0), dtype=torch.float64, device=device)
    Y, X = torch.meshgrid(xs, xs, indexing="ij")
    m = (X * X + Y * Y) <= SUPPORT_RADIUS ** 2
    if kind.startswith("upper"):
        m &= Y > 0
    return m.to(torch.float32)


def phantoms(seeds, n: int, kind: str, device) -> torch.Tensor:
    prm = np.stack([PH.ellipse_params(int(s)) for s in seeds])
    f = PH.ellipse_images(prm, n, 1.0, device=device, edge=EDGE if "smooth" in kind else 0.0)
    return f * support(kind, n, device)


def measured_data(arc_deg, kind, seeds, n, nt, T, noise, noise_seed, device):
    """Traces of the phantoms rasterised at 2n (the same ellipses), from the
    forward operator of a 2n plan, plus noise of relative L2 level ``noise``
    per instance (reading of Sec. 4.3: white Gaussian noise scaled to the
    trace norm), from a seeded device generator."""
    g_hi = geometry(arc_deg, 2 * n, detectors(arc_deg, n), nt, T)
    plan_hi = Plan(g_hi, torch.float32, max_batch=len(seeds), device=device)
    f_hi = phantoms(seeds, 2 * n, kind, device)
    y = plan_hi.forward(f_hi)
    if noise > 0:
        gen = torch.Generator(device=device)
        gen.manual_seed(int(noise_seed))
        eps = torch.randn(y.shape, generator=gen, device=device, dtype=torch.float32)
        ny = torch.linalg.vector_norm(y.flatten(1), dim=1)
        ne = torch.linalg.vector_norm(eps.flatten(1), dim=1)
        y = y + (noise * ny / ne).view(-1, 1, 1) * eps
    del plan_hi
    return y


def errors(f: torch.Tensor, ref: torch.Tensor) -> Dict[str, float]:
    d = (f.double() - ref.double())
    r = ref.double()
    return {"l2": float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(r)),
            "linf": float(d.abs().max() / r.abs().max()),
            "psnr": float(10 * torch.log10(1.0 / torch.mean(d * d)))}


def run_inverse(plan: Plan, y: torch.Tensor):
    plan.inverse(y)                                   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f = plan.inverse(y)
    torch.cuda.synchronize()
    return f, 1, time.perf_counter() - t0


def run_iterative(plan: Plan, y: torch.Tensor, method: str, supp: torch.Tensor, lam: float = 0.0,
                  opnorm: Optional[float] = None, max_iter: int = 1000, tol: float = 3e-3):
    """One instance (y: nt x m) until the stopping rule; returns
    (f, iterations, seconds).  The time covers the iterations only (plan,
    operator norm and graph capture are set up before)."""
    sol = S.BatchedSolver([(plan, y.unsqueeze(0), supp.unsqueeze(0).contiguous())], method=method, lam=lam,
                          opnorms=[opnorm] if opnorm else None)
    rule = S.StoppingRule(sol, tol)
    rule.capture()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, _ = rule.run(max_iter)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return sol.groups[0].f[0].clone(), iters[0], dt


def train_lpd(plan: Plan, kind: str, noise: float, steps: int, n_train: int, lr: float, log=None,
              arch: str = "cnn"):
    """A learned primal-dual network (K = 10, batch 8) for one scheme, trained
    on phantoms of the scheme's support with data from the plan's operator
    (``arch``: "cnn" 3-layer networks or the paper's "unet")."""
    from . import lpd as L
    seeds = list(range(n_train))
    f = phantoms(seeds, plan.n, kind, plan.device)
    y = torch.empty((n_train, plan.nt, plan.m), dtype=torch.float32, device=plan.device)
    gen = torch.Generator(device=plan.device)
    gen.manual_seed(77)
    for s in range(0, n_train, 256):
        e = min(n_train, s + 256)
        plan.forward(f[s:e], out=y[s:e])
        eps = torch.randn(y[s:e].shape, generator=gen, device=plan.device, dtype=torch.float32)
        ny = torch.linalg.vector_norm(y[s:e].flatten(1), dim=1)
        ne = torch.linalg.vector_norm(eps.flatten(1), dim=1)
        y[s:e] += (noise * ny / ne).view(-1, 1, 1) * eps
    ds = {"f": f, "y": y}
    s_A, s_U = L.input_scales(plan, ds)
    net = L.LPD(plan, 8, 10, s_A=s_A, s_U=s_U, seed=0, arch=arch)
    t0 = time.perf_counter()
    hist = L.train(net, ds, steps, lr=lr, log_every=max(1, steps // 10), log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    params = net.params.cpu().numpy()
    stats = None if net.stats is None else net.stats.cpu().numpy()
    del net, ds
    torch.cuda.empty_cache()
    inf = L.LPD(plan, 1, 10, params=params, stats=stats, train=False, s_A=s_A, s_U=s_U, arch=arch)
    inf.capture_forward()
    return inf, {"steps": steps, "phantoms": n_train, "seconds": train_s, "loss_last": hist[-1][1] if hist else None,
                 "arch": arch}


def run_lpd(net, y: torch.Tensor):
    net.reconstruct(y.unsqueeze(0))                   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f = net.reconstruct(y.unsqueeze(0))
    torch.cuda.synchronize()
    return f[0].clone(), 10, time.perf_counter() - t0


def methods_filter(methods, selected):
    """The scheme's methods that are also selected (all of them when none are)."""
    if not selected:
        return tuple(methods)
    return tuple(m for m in methods if m in selected)


def run_suite(n: int = 256, nt: int = 512, T: float = 4.0, tests: int = 4, schemes: Optional[List[str]] = None,
              lpd_steps: int = 3000, lpd_train: int = 4000, lpd_lr: float = 1e-3,
              tv_lams=(1e-4, 3e-4, 1e-3, 3e-3, 1e-2), max_iter: int = 1000, device="cuda", log=None,
              lpd_arch: str = "cnn", methods: Optional[List[str]] = None, train_log=None) -> dict:
    """Runs the schemes; per method the mean over ``tests`` held-out phantoms
    of iterations, time, time per iteration and errors.  The TV weight is
    chosen per scheme from ``tv_lams`` on a separate validation phantom.
    ``methods`` restricts every scheme to those methods; ``lpd_arch`` picks
    the learned networks (the paper's Table 1 uses U-Nets); ``train_log(step,
    loss)`` receives the training progress."""
    device = torch.device(device)
    methods_sel = list(methods) if methods else []
    out = {"grid": n, "data_grid": 2 * n, "nt": nt, "T": T, "test_phantoms": tests, "rows": []}
    test_seeds = [10 ** 6 + i for i in range(tests)]
    val_seed = [2 * 10 ** 6]
    for name in (schemes or list(SCHEMES)):
        arc, kind, noise, methods = SCHEMES[name]
        methods = methods_filter(methods, methods_sel)
        if not methods:
            continue
        geom = geometry(arc, n, detectors(arc, n), nt, T)
        t0 = time.perf_counter()
        plan = Plan(geom, torch.float32, max_batch=8, device=device)
        plan_s = time.perf_counter() - t0
        supp = support(kind, n, device)
        truth = phantoms(test_seeds, n, kind, device)
        y = measured_data(arc, kind, test_seeds, n, nt, T, noise, 11, device)
        L = plan.opnorm(30)
        lam = None
        sweep = {}
        if "tv" in methods:
            fv = phantoms(val_seed, n, kind, device)
            yv = measured_data(arc, kind, val_seed, n, nt, T, noise, 12, device)
            for lm in tv_lams:
                fr, it, _ = run_iterative(plan, yv[0], "tv", supp, lam=lm, opnorm=L, max_iter=max_iter)
                sweep["%g" % lm] = errors(fr, fv[0])["l2"]
            lam = float(min(tv_lams, key=lambda v: sweep["%g" % v]))
        net, train_info = None, None
        if "lpd" in methods:
            net, train_info = train_lpd(plan, kind, noise, lpd_steps, lpd_train, lpd_lr, log=train_log, arch=lpd_arch)
        for meth in methods:
            recs = []
            for i in range(tests):
                if meth == "inverse":
                    fr, it, dt = run_inverse(plan, y[i])
                elif meth == "lpd":
                    fr, it, dt = run_lpd(net, y[i])
                else:
                    fr, it, dt = run_iterative(plan, y[i], meth, supp, lam=lam or 0.0, opnorm=L, max_iter=max_iter)
                e = errors(fr, truth[i])
                recs.append(dict(e, iterations=it, seconds=dt))
            row = {"scheme": name, "method": meth if meth != "lpd" else "lpd (%s)" % lpd_arch,
                   "iterations": float(np.mean([r["iterations"] for r in recs])),
                   "seconds": float(np.mean([r["seconds"] for r in recs])),
                   "seconds_per_iteration": float(np.mean([r["seconds"] / r["iterations"] for r in recs])),
                   "l2_pct": 100 * float(np.mean([r["l2"] for r in recs])),
                   "linf_pct": 100 * float(np.mean([r["linf"] for r in recs])),
                   "psnr": float(np.mean([r["psnr"] for r in recs])),
                   "plan_seconds": plan_s}
            if meth == "tv":
                row["tv_lambda"] = lam
                row["tv_sweep_val_l2"] = sweep
            if meth == "lpd":
                row["training"] = train_info
            out["rows"].append(row)
            if log is not None:
                log(row)
        del plan, net
        torch.cuda.empty_cache()
    return out
