"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every symbol the header declares, validates geometries, and its plan logic
(parameter choices, Bessel recurrence) is sound."""
import ctypes
import json
import math
import os
import re

import numpy as np
import pytest

from paper_2510_24687_amd import pat
from paper_2510_24687_amd import phantoms as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pat.LIB_PATH):
        from paper_2510_24687_amd import build
        build.build()
    return pat.load()


def header_functions():
    src = open(os.path.join(ROOT, "include", "pat.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pat_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(pat.EXPORTED) <= set(names)


def test_status_strings(lib):
    assert lib.pat_status_string(0) == b"ok"
    for code in (-1, -2, -3, -4, -5):
        assert lib.pat_status_string(code) not in (b"ok", b"unknown status")


def test_null_arguments_are_rejected_without_device_work(lib):
    vp = ctypes.c_void_p
    assert lib.pat_forward(None, None, None, None, None) == -1
    assert lib.pat_adjoint_batched(None, 1, None, 0, None, 0, None, None) == -1
    assert lib.pat_plan_destroy(None) == -1
    out = vp()
    assert lib.pat_plan_create(ctypes.byref(out), None, 0, 1, None) == -1
    assert b"NULL" in lib.pat_last_error()


@pytest.mark.parametrize("bad,code", [
    (dict(n=4), -1), (dict(c=-1.0), -1), (dict(rho=1.0), -1), (dict(m=360), -2), (dict(m=80), -2),
    (dict(arc=2.0), -1), (dict(mask_radius=-0.1), -1), (dict(nt=0), -1),
])
def test_invalid_geometries(lib, bad, code):
    g = P.full_circle(64, 128, 128)
    g.update(bad)
    info = pat.PlanInfo()
    rc = lib.pat_plan_query(ctypes.byref(pat.make_geometry(g)), 0, ctypes.byref(info))
    assert rc == code, lib.pat_last_error()


def test_plan_parameters_for_the_workloads(lib):
    m512 = pat.plan_query(P.full_circle(512, 1024, 1024), "f32")
    assert m512["grid"] == 1024 and m512["stencil"] == 6 and m512["m_full"] == 1024
    # M is the smallest 2^a or 3*2^a that covers the band and the time samples:
    # 1536 here, so the period 2 M c T/nt is 6 and L = M/2 rings
    assert abs(m512["period"] - 6.0) < 1e-12
    assert m512["rings"] == 768 and m512["dct_half"] == 1536
    assert 820 <= m512["kmax"] <= 900                    # Lambda R = 804 plus the Bessel transition zone
    assert m512["max_ring"] == 2048
    arc = pat.plan_query(P.top_arc(256, 256, 512, 180.0), "f32")
    assert arc["m_full"] == 512
    # a 120-degree arc: the full-circle grid has 3 m = 3 * 2^8 points
    assert pat.plan_query(P.top_arc(256, 256, 512, 120.0), "f32")["m_full"] == 768
    c1 = pat.plan_query(P.full_circle(64, 128, 128), "f64")
    assert c1["stencil"] == 13 and c1["period"] >= 16.0
    # the period always leaves room for the compact part of every harmonic's time signal
    for g, dt in [(P.full_circle(32, 64, 64), "f32"), (P.full_circle(128, 256, 256), "f32"),
                  (P.top_arc(128, 256, 256, 180.0), "f64")]:
        q = pat.plan_query(g, dt)
        assert q["period"] > g["T"] + 1 + math.sqrt(2)
        assert q["rings"] * q["dlam"] >= q["lambda_max"] - 1e-9
        M = q["dct_half"]
        assert M >= g["nt"] and (M & (M - 1) == 0 or (M % 3 == 0 and (M // 3) & (M // 3 - 1) == 0))


def test_bessel_recurrence_against_mpmath(lib):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30
    for x in (0.0, 0.37, 5.5, 63.0, 401.3, 804.2):
        K = 900
        J = pat.debug_bessel(x, K)
        scale = np.max(np.abs(J))
        for k in (0, 1, 2, 7, 60, int(x), int(x) + 20, 880):
            ref = float(mpmath.besselj(k, x))
            assert abs(J[k] - ref) <= 5e-15 * max(scale, 1e-300) + 1e-300, (x, k, J[k], ref)


def test_product_package_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2510_24687_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "pat_oracle" not in text, fn


def test_plan_needs_a_gpu_and_says_so():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError, match="GPU"):
        pat.Plan(P.full_circle(32, 64, 64))


def test_bench_measures_one_gpu_only():
    """The benchmark runs on one GPU; asked for more it exits with status 2
    and says why, before touching any device."""
    import subprocess
    import sys
    for n in (2, 8):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                           capture_output=True, text=True, timeout=120, cwd=ROOT)
        assert r.returncode == 2, (n, r.returncode, r.stderr)
        assert "one GPU" in r.stderr and r.stdout == ""


def test_gconv_rejects_mixed_channel_packing_without_device_work(lib):
    """Two 16-channel sources total 32 channels, whose weights pack for the
    32-deep instruction; the kernel needs every source to be a multiple of 32,
    so the call is refused before any launch."""
    d = pat.GConvDesc()
    d.B, d.H, d.W, d.Hs, d.Ws, d.Ho, d.Wo = 1, 8, 8, 8, 8, 8, 8
    d.src[0], d.src[1] = 16, 32            # never dereferenced: rejected on the host
    d.csrc[0], d.csrc[1] = 16, 16
    d.in_stride, d.out_stride, d.ntaps = 1, 1, 1
    d.weight, d.cout = 64, 16
    d.dst[0], d.cdst[0] = 128, 16
    assert lib.pat_gconv(ctypes.byref(d), None) == -2
    assert b"multiple of 32" in lib.pat_last_error()
    d.csrc[1] = 0
    d.cout = 24
    assert lib.pat_gconv(ctypes.byref(d), None) == -2      # cout not a multiple of 16
    assert lib.pat_gconv(None, None) == -1


def test_unet_entry_points_validate_on_the_host(lib):
    """Unsupported channel counts and bad shapes are refused before any launch."""
    assert lib.pat_bn_partials(1000, 48) == -1          # channels must divide 256
    assert lib.pat_bn_partials(0, 32) == -1
    assert lib.pat_bn_partials(1000, 32) > 0
    assert lib.pat_head_partials(100, 33) == -1
    assert lib.pat_gconv_packed_size(24, 32, 9) == -1   # cout not a multiple of 16
    assert lib.pat_gconv_packed_size(32, 32, 10) == -1  # at most 9 taps
    assert lib.pat_gconv_packed_size(32, 48, 9) == 32 * 48 * 9
    assert lib.pat_maxpool2(1, 7, 8, 32, 16, 32, None) == -1     # odd H
    assert lib.pat_bn_forward(1000, 48, 16, 16, 16, 16, 16, None, None, 0.1, 1e-5, 1, 16, 16, None) == -2
    assert lib.pat_bn_forward(1000, 32, 16, 16, 16, 16, 16, None, None, 0.1, 1e-5, 0, 16, 16, None) == -1
    assert lib.pat_gconv_pack(None, 16, 16, 16, 16, 9, 0, 1, 1, 1, 0, 16, None) == -1
    assert lib.pat_nhwc_pack(10, 5, 16, None, None, 16, None) == -1


def test_suite_method_selection():
    from paper_2510_24687_amd import experiments as X
    meths = ("inverse", "nnls", "tv", "lpd")
    assert X.methods_filter(meths, []) == meths
    assert X.methods_filter(meths, ["lpd"]) == ("lpd",)
    assert X.methods_filter(("inverse",), ["lpd", "tv"]) == ()
    assert X.methods_filter(meths, ["tv", "inverse"]) == ("inverse", "tv")   # the scheme's order


def test_bench_byte_model_and_traffic_record():
    """The benchmark's algorithmic bytes for the cosine transform at n = 512,
    m = 1024, nt = 1024, batch 16 are the harmonic columns' ring values read
    and time values written once (complex64), and the committed HBM traffic
    record is used only for the batch, launch shape and kernel sources it was
    taken with."""
    import bench
    geom = P.full_circle(512, 1024, 1024)
    info = pat.plan_query(geom)
    per = bench.stage_bytes(info, 16, geom)
    assert per["dct_fwd"] == per["dct_adj"] == 16 * 8 * (info["rings"] + 1024) * info["kpad"]
    assert per["spread_adj"] == 16 * 8 * (info["ring_points"] + info["grid"] * (info["grid"] // 2 + 1 + 2 * ((info["stencil"] + 1) // 2)))
    assert bench.measured_traffic("dct_fwd", 8) is None                     # other batch
    z = json.load(open(os.path.join(ROOT, "profiles", "traffic_n512.json")))
    shapes = dict(z["launch_shapes"])
    if z["source_hash"] != bench.kernel_source_hash():
        assert bench.measured_traffic("dct_fwd", 16, shapes) is None
        pytest.skip("kernel sources changed since the traffic record was taken")
    t = bench.measured_traffic("dct_fwd", 16, shapes)
    assert 0.95 * per["dct_fwd"] <= t <= 1.05 * per["dct_fwd"]               # no re-reads
    shapes["tune_dct_cols_per_block"] += 1
    # the wave cosine transform fixes its own columns per block
    assert (bench.measured_traffic("dct_fwd", 16, shapes) is None) == (shapes["tune_dct_wave"] != 1)
    shapes["tune_dct_wave"] = 1 - shapes["tune_dct_wave"]
    assert bench.measured_traffic("dct_fwd", 16, shapes) is None            # other launch shape
    assert bench.measured_traffic("rows_fwd", 16, shapes) is not None       # shape irrelevant to it


def test_device_code_has_no_packed_fp32_arithmetic(tmp_path):
    """Every HIP source, compiled for gfx950 with the library's own flags,
    contains no packed FP32 add / multiply / fma instruction (the build turns
    that target feature off; without it the compiler emits them from plain
    float code)."""
    import subprocess
    from paper_2510_24687_amd import build as Bd
    if not os.path.exists(Bd.HIPCC):
        pytest.skip("hipcc not installed")
    packed = re.compile(r"\bv_pk_(fma|mul|add)_f32\b")
    for src in Bd.SOURCES:
        if not src.endswith(".hip"):
            continue
        out = tmp_path / (os.path.basename(src) + ".s")
        subprocess.check_call([Bd.HIPCC] + Bd.FLAGS + ["--cuda-device-only", "-S", "-w", "-o", str(out), src],
                              timeout=900)
        hits = [ln for ln in open(out) if packed.search(ln)]
        assert not hits, (src, hits[:3])
