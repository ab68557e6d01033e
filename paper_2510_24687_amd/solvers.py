"""Batched variational reconstructions driven by the HIP operators.

Projected-gradient NNLS (eq. eqn:NNLS with the projection step eq:NNLS-projstep /
eqn:projectionHalfCircle) and Chambolle-Pock TV-regularised least squares
(eqs. eqn:PDHG-dual, eqn:PDHG-primal, eqn:PDHG-relaxation) of Hauptmann,
Kunyansky & Poimala (arXiv 2510.24687, Sec. 4.2), for

    min_{f >= 0}  1/2 ||A f - g||_Y^2  [+ lam * h^2 sum |grad_h f|]

in the weighted L2 spaces X, Y of eq. eqn:innerProducts, so the gradient of the
data term is A*(A f - g) with the library's weighted adjoint A*.  The
extrapolation uses the standard Chambolle-Pock form fbar = f_new + theta
(f_new - f), theta = 1.

One iteration for every instance of a batch -- several plans of different
image sizes, each with its own batch -- is a fixed sequence of launches on one
stream (A, fused update kernels, A*), captured once in a HIP graph
(torch.cuda.CUDAGraph) and replayed.  Python only marshals pointers.
"""
from __future__ import annotations

import ctypes
import math
from typing import List, Optional

import torch

from .pat import Group, Plan, load, _check

_VP = ctypes.c_void_p


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else _VP(t.data_ptr())


def _bind(lib):
    if getattr(lib, "_solver_bound", False):
        return lib
    D, L, I = ctypes.c_double, ctypes.c_long, ctypes.c_int
    lib.pat_axpby.argtypes = [_VP, L, D, _VP, D, _VP, _VP, _VP]
    lib.pat_nnls_update.argtypes = [_VP, I, _VP, _VP, D, _VP, _VP]
    lib.pat_cp_dual_data.argtypes = [_VP, I, _VP, _VP, _VP, D, _VP]
    lib.pat_cp_dual_tv.argtypes = [_VP, I, _VP, _VP, D, D, _VP]
    lib.pat_cp_primal.argtypes = [_VP, I, _VP, _VP, _VP, _VP, D, D, _VP, _VP]
    lib.pat_dot_batched.argtypes = [_VP, I, L, L, _VP, _VP, _VP, _VP, _VP]
    lib.pat_dot_batched_noalloc.argtypes = [_VP, I, L, L, _VP, _VP, _VP, _VP]
    lib.pat_forward_residual.argtypes = [_VP, I, _VP, _VP, _VP, _VP, _VP]
    lib.pat_forward_cp_dual.argtypes = [_VP, I, _VP, _VP, _VP, D, _VP, _VP]
    lib.pat_adjoint_nnls.argtypes = [_VP, I, _VP, _VP, D, _VP, _VP, _VP]
    lib.pat_adjoint_cp_primal.argtypes = [_VP, I, _VP, _VP, _VP, _VP, D, D, _VP, _VP, _VP]
    lib._solver_bound = True
    return lib


def opnorm(plan: Plan, iters: int = 30, seed: int = 0) -> float:
    """||A||_{X->Y} by power iteration on A*A (pat_opnorm_estimate)."""
    return plan.opnorm(iters)


def tv_norm_bound(plan: Plan) -> float:
    """||grad_h||^2 <= 8/h^2 (forward differences in two directions)."""
    h = 2.0 * plan.geom["a"] / plan.n
    return math.sqrt(8.0) / h


class _Group:
    """State of one plan's batch of instances."""

    def __init__(self, plan: Plan, g: torch.Tensor, support: Optional[torch.Tensor]):
        self.plan = plan
        self.B = g.shape[0]
        self.g = g.contiguous()
        self.support = support
        dt, dev, n, nt, m = plan.dtype, plan.device, plan.n, plan.nt, plan.m
        self.f = torch.zeros((self.B, n, n), dtype=dt, device=dev)
        self.fbar = torch.zeros_like(self.f)
        self.grad = torch.zeros_like(self.f)
        self.Af = torch.zeros((self.B, nt, m), dtype=dt, device=dev)
        self.q = torch.zeros_like(self.Af)
        self.p = torch.zeros((self.B, 2, n, n), dtype=dt, device=dev)
        plan.workspace(self.B)


class BatchedSolver:
    """NNLS or CP-TV over groups of instances (one Plan per image size).

    ``groups`` is a list of (plan, g, support) with g of shape (B, nt, m).
    """

    def __init__(self, groups, method: str = "nnls", lam: float = 1e-3, opnorms=None, grouped: bool = False,
                 fused: bool = True):
        """grouped: run the operators of all plans as one grouped launch per
        stage (pat_group_forward / pat_group_adjoint) instead of one launch
        chain per plan.  fused (per-plan chains only): the data-term updates
        run inside the operators' last launches (pat_forward_residual /
        pat_adjoint_nnls, pat_forward_cp_dual / pat_adjoint_cp_primal)
        instead of as separate kernels."""
        if method not in ("nnls", "tv"):
            raise ValueError("method must be 'nnls' or 'tv'")
        self.method, self.lam = method, float(lam)
        self.fused = bool(fused) and not grouped
        self.lib = _bind(load())
        self.groups: List[_Group] = [_Group(p, g, s) for p, g, s in groups]
        self.opgroup = Group([G.plan for G in self.groups]) if grouped else None
        self.norms = opnorms or [opnorm(G.plan) for G in self.groups]
        self.graph = None
        self.stream = torch.cuda.current_stream()
        for G, L in zip(self.groups, self.norms):
            if method == "nnls":
                G.tau = 1.0 / (L * L)
            else:
                # K = [A; mu grad_h] with mu = ||A|| / ||grad_h|| so both blocks have norm ||A||
                # (||K|| = sqrt(2) ||A||); the TV dual is stored as mu * p, so its update uses
                # sigma * mu^2 and the projection radius stays lam.  Steps tau = s/||K||,
                # sigma = 1/(s ||K||) with s = 1/||A|| (tau sigma ||K||^2 = 0.98 < 1).
                mu = L / tv_norm_bound(G.plan)
                Kn = math.sqrt(2.0) * L
                G.tau = 0.99 / (L * Kn)
                G.sigma = 0.99 * L / Kn
                G.sigma_tv = G.sigma * mu * mu

    def _step_group(self, G: _Group):
        lib, P, st = self.lib, G.plan, _VP(torch.cuda.current_stream().cuda_stream)
        h = P._h
        if self.fused:
            ws = _ptr(P.workspace(G.B))
            if self.method == "nnls":
                _check(lib.pat_forward_residual(h, G.B, _ptr(G.f), _ptr(G.g), _ptr(G.Af), ws, st), "pat_forward_residual")
                _check(lib.pat_adjoint_nnls(h, G.B, _ptr(G.Af), _ptr(G.f), G.tau, _ptr(G.support), ws, st),
                       "pat_adjoint_nnls")
            else:
                _check(lib.pat_forward_cp_dual(h, G.B, _ptr(G.fbar), _ptr(G.g), _ptr(G.q), G.sigma, ws, st),
                       "pat_forward_cp_dual")
                _check(lib.pat_cp_dual_tv(h, G.B, _ptr(G.p), _ptr(G.fbar), G.sigma_tv, self.lam, st), "pat_cp_dual_tv")
                _check(lib.pat_adjoint_cp_primal(h, G.B, _ptr(G.q), _ptr(G.p), _ptr(G.f), _ptr(G.fbar), G.tau, 1.0,
                                                 _ptr(G.support), ws, st), "pat_adjoint_cp_primal")
            return
        if self.method == "nnls":
            P.forward(G.f, out=G.Af)
            _check(lib.pat_axpby(h, G.Af.numel(), 1.0, _ptr(G.Af), -1.0, _ptr(G.g), _ptr(G.Af), st), "pat_axpby")
            P.adjoint(G.Af, out=G.grad)
            _check(lib.pat_nnls_update(h, G.B, _ptr(G.f), _ptr(G.grad), G.tau, _ptr(G.support), st), "pat_nnls_update")
        else:
            P.forward(G.fbar, out=G.Af)
            _check(lib.pat_cp_dual_data(h, G.B, _ptr(G.q), _ptr(G.Af), _ptr(G.g), G.sigma, st), "pat_cp_dual_data")
            _check(lib.pat_cp_dual_tv(h, G.B, _ptr(G.p), _ptr(G.fbar), G.sigma_tv, self.lam, st), "pat_cp_dual_tv")
            P.adjoint(G.q, out=G.grad)
            _check(lib.pat_cp_primal(h, G.B, _ptr(G.f), _ptr(G.fbar), _ptr(G.grad), _ptr(G.p), G.tau, 1.0,
                                     _ptr(G.support), st), "pat_cp_primal")

    def _updates(self, G: _Group, phase: int):
        lib, P, st = self.lib, G.plan, _VP(torch.cuda.current_stream().cuda_stream)
        h = P._h
        if self.method == "nnls":
            if phase == 0:
                _check(lib.pat_axpby(h, G.Af.numel(), 1.0, _ptr(G.Af), -1.0, _ptr(G.g), _ptr(G.Af), st), "pat_axpby")
            else:
                _check(lib.pat_nnls_update(h, G.B, _ptr(G.f), _ptr(G.grad), G.tau, _ptr(G.support), st),
                       "pat_nnls_update")
        elif phase == 0:
            _check(lib.pat_cp_dual_data(h, G.B, _ptr(G.q), _ptr(G.Af), _ptr(G.g), G.sigma, st), "pat_cp_dual_data")
            _check(lib.pat_cp_dual_tv(h, G.B, _ptr(G.p), _ptr(G.fbar), G.sigma_tv, self.lam, st), "pat_cp_dual_tv")
        else:
            _check(lib.pat_cp_primal(h, G.B, _ptr(G.f), _ptr(G.fbar), _ptr(G.grad), _ptr(G.p), G.tau, 1.0,
                                     _ptr(G.support), st), "pat_cp_primal")

    def step(self):
        """One iteration of every instance, launched eagerly."""
        if self.opgroup is None:
            for G in self.groups:
                self._step_group(G)
            return
        src = [G.f if self.method == "nnls" else G.fbar for G in self.groups]
        self.opgroup.forward(src, [G.Af for G in self.groups])
        for G in self.groups:
            self._updates(G, 0)
        self.opgroup.adjoint([G.Af if self.method == "nnls" else G.q for G in self.groups],
                             [G.grad for G in self.groups])
        for G in self.groups:
            self._updates(G, 1)

    def capture(self):
        """Capture one iteration of every instance in a HIP graph."""
        self.step()  # warm-up outside capture (allocators, first launches)
        torch.cuda.synchronize()
        self.reset()
        self.graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(self.graph, stream=s):
                self.step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.reset()
        return self.graph

    def replay(self, iters: int = 1):
        for _ in range(iters):
            self.graph.replay()

    def reset(self):
        for G in self.groups:
            for t in (G.f, G.fbar, G.grad, G.Af, G.q, G.p):
                t.zero_()

    def objective(self) -> List[torch.Tensor]:
        """Per instance: 1/2 ||A f - g||_Y^2 (+ lam * h^2 sum |grad_h f| for TV); reporting only."""
        out = []
        for G in self.groups:
            P = G.plan
            r = P.forward(G.f) - G.g
            wy = (P.geom["T"] / P.nt) * (P.geom["R"] * P.geom["arc"] / P.m)
            val = 0.5 * wy * (r.double() ** 2).sum(dim=(1, 2))
            if self.method == "tv":
                h = 2.0 * P.geom["a"] / P.n
                f = G.f.double()
                gx = torch.zeros_like(f)
                gy = torch.zeros_like(f)
                gx[:, :, :-1] = (f[:, :, 1:] - f[:, :, :-1]) / h
                gy[:, :-1, :] = (f[:, 1:, :] - f[:, :-1, :]) / h
                val = val + self.lam * h * h * torch.sqrt(gx * gx + gy * gy).sum(dim=(1, 2))
            out.append(val)
        return out


class StoppingRule:
    """Iterate a one-group solver until the update is small (Sec. 4.3): stop
    after iteration k when ||f_k - f_{k-1}||_2 < tol ||f_1||_2, f_1 the first
    non-zero iterate, per instance.  One captured HIP graph per iteration
    holds the copy of the previous iterate, the solver's iteration, the
    difference (pat_axpby) and its squared norm per instance
    (pat_dot_batched); the host reads B doubles per iteration."""

    def __init__(self, solver: BatchedSolver, tol: float = 3e-3):
        if len(solver.groups) != 1:
            raise ValueError("one group of instances")
        self.solver, self.tol = solver, float(tol)
        G = solver.groups[0]
        self.G = G
        self.prev = torch.zeros_like(G.f)
        self.diff = torch.zeros_like(G.f)
        self.out = torch.zeros(G.B, dtype=torch.float64, device=G.f.device)
        self.scratch = torch.zeros(64 * G.B, dtype=torch.float64, device=G.f.device)
        self.lib = solver.lib
        self.graph = None

    def _iteration(self):
        lib, G = self.lib, self.G
        P = G.plan
        st = _VP(torch.cuda.current_stream().cuda_stream)
        cnt = G.f.numel()
        _check(lib.pat_axpby(P._h, cnt, 1.0, _ptr(G.f), 0.0, None, _ptr(self.prev), st), "pat_axpby")
        self.solver.step()
        _check(lib.pat_axpby(P._h, cnt, 1.0, _ptr(G.f), -1.0, _ptr(self.prev), _ptr(self.diff), st), "pat_axpby")
        img = P.n * P.n
        _check(lib.pat_dot_batched(P._h, G.B, img, img, _ptr(self.diff), _ptr(self.diff), _ptr(self.out),
                                   _ptr(self.scratch), st), "pat_dot_batched")

    def capture(self):
        self._iteration()
        torch.cuda.synchronize()
        self.solver.reset()
        self.graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(self.graph, stream=s):
                self._iteration()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.solver.reset()

    def run(self, max_iter: int = 1000):
        """Returns (iterations per instance, final update norms); the
        instances' iterates stay in solver.groups[0].f.  All instances
        iterate until every one has stopped, so run one instance per call
        when per-instance iterates at their own stopping points matter."""
        if self.graph is None:
            self.capture()
        B = self.G.B
        first = None
        stopped = [0] * B
        last = None
        for k in range(1, max_iter + 1):
            self.graph.replay()
            d = self.out.sqrt().cpu().numpy()
            last = d
            if first is None:
                first = d.copy()
                continue
            for b in range(B):
                if not stopped[b] and d[b] <= self.tol * first[b]:
                    stopped[b] = k
            if all(stopped):
                break
        return [s if s else max_iter for s in stopped], last
