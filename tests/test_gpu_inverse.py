"""The approximate inverse A^-1 of Sec. 3.3 (Alg. 3) on the GPU, through the
C ABI (pat_inverse / pat_inverse_batched), against the CPU FP64 oracle
(oracle.inverse / oracle.ubp): full tensors at small sizes (with and without
the mask that brings in the constant of eq. E:silly_integral), sampled
back-projection values at n = 256 and 512, batching, graph replay, and the
left-inverse property on the GPU's own forward data.  Tolerances: FP32
relative L2 <= 1e-4, FP64 <= 1e-8, as for A and A*."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2510_24687_amd import pat  # noqa: E402
from paper_2510_24687_amd import phantoms as P  # noqa: E402

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {"f32": 1e-4, "f64": 1e-8}


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def tdt(dt):
    return torch.float64 if dt == "f64" else torch.float32


def on_gpu(x, dt):
    return torch.tensor(np.asarray(x), dtype=tdt(dt), device="cuda")


CASES = [
    ("f64_n32_mask", "f64", P.full_circle(32, 64, 64, mask_radius=0.9)),
    ("f64_n25_odd", "f64", P.full_circle(25, 64, 41, T=1.7, c=1.2, R=1.1, mask_radius=0.7)),
    ("f32_n64_mask", "f32", P.full_circle(64, 128, 128, mask_radius=0.9)),
    ("f32_n64_nomask", "f32", P.full_circle(64, 128, 128)),
    ("f32_arc180_n48", "f32", P.top_arc(48, 64, 96, 180.0, mask_radius=0.8)),
    ("f64_arc90_n32", "f64", P.top_arc(32, 32, 64, 90.0)),
    ("f32_arc120_n32", "f32", P.top_arc(32, 32, 64, 120.0, mask_radius=0.9)),
]


@pytest.mark.parametrize("cid,dt,geom", CASES, ids=[c[0] for c in CASES])
def test_inverse_parity(cid, dt, geom):
    print("case", cid, flush=True)
    n, m, nt = geom["n"], geom["m"], geom["nt"]
    plan = pat.Plan(geom, tdt(dt), max_batch=2)
    y = P.randn((nt, m), 31)
    got = plan.inverse(on_gpu(y, dt)).double().cpu().numpy()
    v = O.ubp(geom, y)
    om0, ann = O.support_masks(geom)
    ref = np.where(om0, v + O.ubp_constant(geom, v), 0.0)    # = O.inverse(geom, y)
    e = rel(got, ref)
    print("  inverse rel %.3e  constant %.3e" % (e, O.ubp_constant(geom, v)), flush=True)
    assert e <= TOL[dt]
    assert np.all(got[~om0] == 0.0)
    if ann.any():
        # the constant: the GPU output minus the oracle's v on Omega_0 is one number
        d = got[om0] - v[om0]
        assert abs(d.mean() - O.ubp_constant(geom, v)) <= TOL[dt] * np.abs(v).max()


def test_inverse_of_phantom_data_f32():
    """Realistic input: the oracle's traces of an ellipse phantom."""
    geom = P.full_circle(48, 128, 96, mask_radius=0.9)
    f = P.ellipse_phantom(48, 3)
    g = O.forward(geom, f)
    plan = pat.Plan(geom, torch.float32)
    got = plan.inverse(on_gpu(g, "f32")).double().cpu().numpy()
    assert rel(got, O.inverse(geom, g)) <= 1e-4


@pytest.mark.parametrize("name,B", [("inv_full_n256", 3), ("inv_full_n512", 16)])
def test_sampled_inverse_parity_at_full_size(name, B):
    """Oracle back-projection samples at the full sizes (no mask, so the
    output is v), in a batch; then the masked plan's output differs from v by
    the constant computed from v's own annulus, on every pixel of Omega_0."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    geom, gseed, _ = mod.INV_CASES[name]
    z = np.load(os.path.join(HERE, "golden", name + ".npz"))
    print("case", name, "B", B, flush=True)
    n, m, nt = geom["n"], geom["m"], geom["nt"]
    plan = pat.Plan(geom, torch.float32, max_batch=B)
    y = np.stack([P.randn((nt, m), gseed)] + [P.randn((nt, m), 700 + b) for b in range(B - 1)])
    yg = on_gpu(y, "f32")
    v = plan.inverse(yg).double().cpu().numpy()
    e = rel(v[0].ravel()[z["pix"]], z["ubp"])
    print("  back-projection rel %.3e" % e, flush=True)
    assert e <= 1e-4
    geom_m = dict(geom, mask_radius=0.9)
    plan_m = pat.Plan(geom_m, torch.float32, max_batch=B)
    f = plan_m.inverse(yg).double().cpu().numpy()
    om0, ann = O.support_masks(geom_m)
    for b in (0, B - 1):
        C = -v[b][ann].mean()
        assert np.all(f[b][~om0] == 0.0)
        assert np.max(np.abs(f[b][om0] - v[b][om0] - C)) <= 1e-5 * np.abs(v[b]).max()


def test_batched_inverse_equals_single_calls():
    geom = P.top_arc(64, 64, 128, 180.0, mask_radius=0.85)
    plan = pat.Plan(geom, torch.float32, max_batch=4)
    y = on_gpu(np.stack([P.randn((128, 64), 40 + b) for b in range(4)]), "f32")
    batch = plan.inverse(y)
    plan1 = pat.Plan(geom, torch.float32, max_batch=1)
    for b in range(4):
        one = plan1.inverse(y[b])
        assert float((one - batch[b]).abs().max()) <= 1e-6 * float(one.abs().max())
    assert torch.equal(plan.inverse(y), batch)                # deterministic
    assert float(plan.inverse(torch.zeros_like(y)).abs().max()) == 0.0


def test_inverse_graph_replay():
    geom = P.full_circle(64, 128, 128, mask_radius=0.9)
    plan = pat.Plan(geom, torch.float32, max_batch=2)
    y = on_gpu(np.stack([P.randn((128, 128), 50), P.randn((128, 128), 51)]), "f32")
    out = torch.zeros((2, 64, 64), device="cuda")
    plan.inverse(y, out=out)
    torch.cuda.synchronize()
    eager = out.clone()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            plan.inverse(y, out=out)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        out.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager)


def test_left_inverse_of_the_gpu_forward():
    """A^-1 A f ~ f for a smooth phantom well inside the disk, full circle,
    T = 8 (the truncation error of the formula falls with T)."""
    n = 64
    geom = P.full_circle(n, 256, 512, T=8.0, mask_radius=0.9)
    plan = pat.Plan(geom, torch.float64)
    blobs = np.array([[0.1, -0.05, 0.14, 1.0], [-0.12, 0.1, 0.12, -0.5], [0.3, 0.3, 0.08, 0.7]])
    h = 2.0 / n
    xc = -1 + (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(xc, xc)
    f = sum(b[3] * np.exp(-((X - b[0]) ** 2 + (Y - b[1]) ** 2) / (2 * b[2] ** 2)) for b in blobs)
    back = plan.inverse(plan.forward(on_gpu(f, "f64"))).cpu().numpy()
    om0, _ = O.support_masks(geom)
    e = rel(back[om0], f[om0])
    print("A^-1 A f: rel %.3e" % e)
    assert e < 1e-3


@pytest.mark.parametrize("wave", [1, 0])
def test_inverse_with_and_without_the_wave_sine_transform(tmp_path, wave):
    """At n = 64 (M = 384 admits the one-wave transform) the approximate inverse
    runs its sine transform on the wave kernel (dct_wave = 1) or on the
    generic column kernel (dct_wave = 0), forced through the tuning cache:
    both meet the FP32 bar against the oracle and agree with each other."""
    geom = P.full_circle(64, 128, 128)
    B = 2
    path = str(tmp_path / "t.txt")
    pat.Plan(geom, torch.float32, max_batch=B, tuning_cache=path)
    key = open(path).read().splitlines()[0].split(" | ")[0]
    outs = {}
    g = np.stack([P.randn((128, 128), 900 + s) for s in range(B)])
    for flag in (wave, 1 - wave):
        cache = str(tmp_path / ("c%d.txt" % flag))
        with open(cache, "w") as fh:
            fh.write(key + " | cols_cw=1 dct_cw=1 ring_group=2 spread_images=16 fft_radix_log2=4 ms=1.0 "
                     "twiddle_table=0 spread_staged=2 dct_wave=%d wave_fft=1\n" % flag)
        plan = pat.Plan(geom, torch.float32, max_batch=B, tuning_cache=cache)
        assert plan.info["tuned"] == 2 and plan.info["tune_dct_wave"] == flag
        outs[flag] = plan.inverse(torch.tensor(g, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    ref = O.inverse(geom, g[0])
    assert rel(outs[wave][0], ref) <= 1e-4
    for b in range(B):
        assert rel(outs[1][b], outs[0][b]) <= 1e-5

