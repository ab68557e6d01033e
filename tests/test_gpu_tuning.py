"""The launch-shape autotuner and its cache: a plan created with a cache path
times the candidates and appends one line; a second plan with the same key
reads it back; every non-default launch shape (read from a hand-written cache
line) still meets the parity bar against the FP64 oracle, batched, with a
batch that is not a multiple of the image groups."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2510_24687_amd import pat  # noqa: E402
from paper_2510_24687_amd import phantoms as P  # noqa: E402

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def test_tuner_measures_stores_and_reuses(tmp_path):
    path = str(tmp_path / "tune.txt")
    geom = P.top_arc(64, 64, 128, 180.0)
    a = pat.Plan(geom, torch.float32, max_batch=5, tuning_cache=path)
    assert a.info["tuned"] == 1 and a.info["tuned_ms"] > 0
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and " | " in lines[0]
    b = pat.Plan(geom, torch.float32, max_batch=5, tuning_cache=path)
    assert b.info["tuned"] == 2
    keys = ["tune_fft_radix_log2", "tune_twiddle_table", "tune_cols_per_block", "tune_dct_cols_per_block",
            "tune_ring_images", "tune_spread_images", "tune_spread_staged"]
    assert [a.info[k] for k in keys] == [b.info[k] for k in keys]
    assert len(open(path).read().splitlines()) == 1
    # another batch size is another key
    pat.Plan(geom, torch.float32, max_batch=2, tuning_cache=path)
    assert len(open(path).read().splitlines()) == 2


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_every_launch_shape_meets_parity(tmp_path, dt):
    tdt = torch.float64 if dt == "f64" else torch.float32
    tol = 1e-8 if dt == "f64" else 1e-4
    geom = P.full_circle(48, 64, 80)
    B = 5
    f_np = np.stack([P.ellipse_phantom(48, s) for s in range(B)])
    g_np = np.stack([P.randn((80, 64), 50 + s) for s in range(B)])
    ref_f = np.stack([O.forward(geom, f) for f in f_np])
    ref_a = np.stack([O.adjoint(geom, g) for g in g_np])
    base = pat.Plan(geom, tdt, max_batch=B)
    # the key the library writes, taken from a measured entry
    path = str(tmp_path / "t.txt")
    pat.Plan(geom, tdt, max_batch=B, tuning_cache=path)
    key = open(path).read().splitlines()[0].split(" | ")[0]
    bcl = base.info["tune_spread_images"]
    # (radix, cols, dct cols, ring images, spread images, twiddle table, spread form
    #  (0 unstaged, 1 staged tiles, 2 binned), wave cosine transform, wave FFT kernels)
    shapes = [(3, 1, 1, 1, bcl // 2, 1, 0, 0, 0), (4, 1, base.info["tune_dct_cols_per_block"], 2, bcl, 0, 1, 0, 0),
              (3, base.info["tune_cols_per_block"], 1, base.info["tune_ring_images"], bcl // 2, 0, 1, 0, 0),
              (4, base.info["tune_cols_per_block"], base.info["tune_dct_cols_per_block"], 1, bcl, 1, 0, 0, 0),
              (3, 1, 1, 1, bcl, 0, 1, 1, 1), (4, 1, 1, 2, bcl // 2, 0, 0, 1, 0), (3, 1, 1, 1, bcl // 2, 0, 1, 0, 1)]
    if dt == "f32":
        # the binned spread (FP32 only), both image groups
        shapes += [(3, 1, 1, 1, bcl, 0, 2, 1, 1), (4, base.info["tune_cols_per_block"], 1, 2, bcl // 2, 1, 2, 0, 0),
                   (3, 1, 1, 4, bcl, 0, 2, 1, 1)]
    f = torch.tensor(f_np, dtype=tdt, device="cuda")
    g = torch.tensor(g_np, dtype=tdt, device="cuda")
    for lr, cw, dw, rg, sb, tt, ss, dwv, wf in shapes:
        with open(path, "a") as fp:
            fp.write("%s | cols_cw=%d dct_cw=%d ring_group=%d spread_images=%d fft_radix_log2=%d ms=1.0 "
                     "twiddle_table=%d spread_staged=%d dct_wave=%d wave_fft=%d\n"
                     % (key, cw, dw, rg, sb, lr, tt, ss, dwv, wf))
        plan = pat.Plan(geom, tdt, max_batch=B, tuning_cache=path)
        got = [plan.info[k] for k in ("tune_fft_radix_log2", "tune_cols_per_block", "tune_dct_cols_per_block",
                                      "tune_ring_images", "tune_spread_images", "tune_twiddle_table",
                                      "tune_spread_staged")]
        assert plan.info["tuned"] == 2 and got == [lr, cw, dw, rg, sb, tt, ss]
        ef = rel(plan.forward(f).cpu().numpy(), ref_f)
        ea = rel(plan.adjoint(g).cpu().numpy(), ref_a)
        print(dt, (lr, cw, dw, rg, sb, tt, ss, dwv, wf), "forward %.2e adjoint %.2e" % (ef, ea))
        assert ef < tol and ea < tol


def test_invalid_cache_lines_are_ignored(tmp_path):
    geom = P.full_circle(32, 64, 64)
    path = str(tmp_path / "bad.txt")
    pat.Plan(geom, torch.float32, max_batch=1, tuning_cache=path)
    key = open(path).read().splitlines()[0].split(" | ")[0]
    with open(path, "a") as fp:
        fp.write("%s | cols_cw=3 dct_cw=1 ring_group=1 spread_images=16 fft_radix_log2=4 ms=1.0\n" % key)
        fp.write("%s | garbage\n" % key)
    plan = pat.Plan(geom, torch.float32, max_batch=1, tuning_cache=path)
    assert plan.info["tuned"] == 2            # the first (valid) line is used
    assert plan.info["tune_cols_per_block"] != 3
