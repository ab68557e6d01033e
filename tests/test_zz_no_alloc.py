"""pat_dot_batched_noalloc (static device scratch, no allocation) against
pat_dot_batched (caller's scratch): bit-identical results on two calls in a
row, the second with a smaller input, and the batch limit."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2510_24687_amd import pat  # noqa: E402
from paper_2510_24687_amd import phantoms as P  # noqa: E402
from paper_2510_24687_amd import solvers as S  # noqa: E402

pytestmark = pytest.mark.gpu


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_dot_matches_scratch_variant(dtype):
    lib = S._bind(pat.load())
    plan = pat.Plan(P.top_arc(32, 32, 64, 180.0), dtype, max_batch=4)
    # first call: 40 images of 5000 values (stride 5003); second: 3 of 1000 (stride 1000)
    for B, count, stride, seed in ((40, 5000, 5003, 1), (3, 1000, 1000, 2)):
        print("noalloc dot: B %d count %d stride %d" % (B, count, stride), flush=True)
        x = torch.tensor(P.randn((B, stride), seed), dtype=dtype, device="cuda")
        y = torch.tensor(P.randn((B, stride), seed + 10), dtype=dtype, device="cuda")
        out_ref = torch.zeros(B, dtype=torch.float64, device="cuda")
        scr = torch.zeros(64 * B, dtype=torch.float64, device="cuda")
        rc = lib.pat_dot_batched(plan._h, B, count, stride, _vp(x), _vp(y), _vp(out_ref), _vp(scr), None)
        assert rc == 0
        out = torch.full((B,), float("nan"), dtype=torch.float64, device="cuda")
        rc = lib.pat_dot_batched_noalloc(plan._h, B, count, stride, _vp(x), _vp(y), _vp(out), None)
        assert rc == 0, pat.load().pat_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out, out_ref)
        want = (x[:, :count].double() * y[:, :count].double()).sum(dim=1)
        assert torch.allclose(out, want, rtol=1e-12, atol=1e-12)


def test_noalloc_dot_rejects_batches_beyond_the_scratch():
    lib = S._bind(pat.load())
    plan = pat.Plan(P.top_arc(32, 32, 64, 180.0), torch.float32)
    x = torch.zeros(8, dtype=torch.float32, device="cuda")
    out = torch.zeros(4097, dtype=torch.float64, device="cuda")
    # B = 4097 exceeds the 4096-image limit: rejected before any launch (stride 0
    # would also be invalid, so no kernel could read past x)
    rc = lib.pat_dot_batched_noalloc(plan._h, 4097, 1, 1, _vp(x), _vp(x), _vp(out), None)
    assert rc == -1
    assert b"scratch" in lib.pat_last_error()
