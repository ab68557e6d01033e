"""Grouped launches of plans with different image sizes (pat_group_*): one
launch per stage for the whole group gives results identical, bit for bit, to
per-plan calls (same kernel bodies, same per-block work), also when captured
in a HIP graph and replayed, and the grouped solvers match the per-plan ones."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2510_24687_amd import pat  # noqa: E402
from paper_2510_24687_amd import phantoms as P  # noqa: E402
from paper_2510_24687_amd import solvers as S  # noqa: E402

pytestmark = pytest.mark.gpu


def setup(dtype, batches=(2, 3, 1)):
    geoms = [P.full_circle(32, 64, 64), P.top_arc(48, 64, 80, 180.0), P.full_circle(64, 128, 96, mask_radius=0.9)]
    plans = [pat.Plan(g, dtype, max_batch=4) for g in geoms]
    fs, gs = [], []
    for k, (p, B) in enumerate(zip(plans, batches)):
        fs.append(torch.tensor(np.stack([P.ellipse_phantom(p.n, 10 * k + b) for b in range(B)]), dtype=dtype,
                               device="cuda"))
        gs.append(torch.tensor(np.stack([P.randn((p.nt, p.m), 100 * k + b) for b in range(B)]), dtype=dtype,
                               device="cuda"))
    return geoms, plans, fs, gs


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_group_equals_per_plan_calls(dtype):
    geoms, plans, fs, gs = setup(dtype)
    grp = pat.Group(plans)
    outg = [torch.full((f.shape[0], p.nt, p.m), float("nan"), dtype=dtype, device="cuda") for p, f in zip(plans, fs)]
    outf = [torch.full((g.shape[0], p.n, p.n), float("nan"), dtype=dtype, device="cuda") for p, g in zip(plans, gs)]
    grp.forward(fs, outg)
    grp.adjoint(gs, outf)
    torch.cuda.synchronize()
    for p, f, g, og, of in zip(plans, fs, gs, outg, outf):
        assert torch.equal(og, p.forward(f))
        assert torch.equal(of, p.adjoint(g))
    # and the group meets the parity bar on its own (first image of each plan)
    tol = 1e-8 if dtype == torch.float64 else 1e-4
    for geom, f, g, og, of in zip(geoms, fs, gs, outg, outf):
        ref_f = O.forward(geom, f[0].double().cpu().numpy())
        ref_a = O.adjoint(geom, g[0].double().cpu().numpy())
        assert np.linalg.norm(og[0].double().cpu().numpy() - ref_f) <= tol * np.linalg.norm(ref_f)
        assert np.linalg.norm(of[0].double().cpu().numpy() - ref_a) <= tol * np.linalg.norm(ref_a)


def test_group_graph_replay():
    geoms, plans, fs, gs = setup(torch.float32, batches=(4, 2, 3))
    grp = pat.Group(plans)
    outg = [torch.zeros((f.shape[0], p.nt, p.m), device="cuda") for p, f in zip(plans, fs)]
    outf = [torch.zeros((g.shape[0], p.n, p.n), device="cuda") for p, g in zip(plans, gs)]
    grp.forward(fs, outg)
    grp.adjoint(gs, outf)
    torch.cuda.synchronize()
    eager_g = [t.clone() for t in outg]
    eager_f = [t.clone() for t in outf]
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            grp.forward(fs, outg)
            grp.adjoint(gs, outf)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for t in outg + outf:
            t.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(outg + outf, eager_g + eager_f):
            assert torch.equal(a, b), rep


@pytest.mark.parametrize("method", ["nnls", "tv"])
def test_grouped_solver_matches_per_plan_solver(method):
    geoms = [P.top_arc(32, 32, 64, 180.0), P.top_arc(64, 64, 128, 180.0)]
    groups = []
    for k, geom in enumerate(geoms):
        plan = pat.Plan(geom, torch.float32, max_batch=2)
        f = torch.tensor(P.ellipse_batch(plan.n, [k, k + 7]), dtype=torch.float32, device="cuda")
        groups.append((plan, plan.forward(f), None))
    norms = [p.opnorm(20) for p, _, _ in groups]
    a = S.BatchedSolver(groups, method=method, opnorms=norms)
    b = S.BatchedSolver(groups, method=method, opnorms=norms, grouped=True)
    for _ in range(5):
        a.step()
        b.step()
    torch.cuda.synchronize()
    for Ga, Gb in zip(a.groups, b.groups):
        assert torch.equal(Ga.f, Gb.f)
