"""The Table-1 experiment driver end to end at a tiny size: every method of
an incomplete-data scheme runs through the library (inverse, NNLS and TV with
the stopping rule, a briefly trained LPD) and reports finite errors, with the
regularised methods ahead of the plain inverse."""
import math

import pytest

torch = pytest.importorskip("torch")

from paper_2510_24687_amd import experiments as X  # noqa: E402

pytestmark = pytest.mark.gpu


def test_suite_runs_every_method():
    res = X.run_suite(n=32, nt=64, T=4.0, tests=2, schemes=["180 (incomplete), 30% noise"], lpd_steps=30,
                      lpd_train=64, tv_lams=(1e-4, 1e-3), max_iter=300)
    rows = {r["method"]: r for r in res["rows"]}
    assert set(rows) == {"inverse", "nnls", "tv", "lpd (cnn)"}
    for r in rows.values():
        assert math.isfinite(r["l2_pct"]) and math.isfinite(r["linf_pct"]) and r["seconds"] > 0
    assert rows["inverse"]["iterations"] == 1 and rows["lpd (cnn)"]["iterations"] == 10
    assert 2 <= rows["nnls"]["iterations"] <= 300 and 2 <= rows["tv"]["iterations"] <= 300
    assert rows["tv"]["l2_pct"] < rows["inverse"]["l2_pct"]
    assert rows["nnls"]["l2_pct"] < rows["inverse"]["l2_pct"]


def test_suite_lpd_rows_with_unets():
    """The learned rows with the paper's U-Nets, alone (method selection)."""
    res = X.run_suite(n=32, nt=64, T=4.0, tests=2, schemes=["120 (incomplete), 30% noise"], lpd_steps=20,
                      lpd_train=64, methods=["lpd"], lpd_arch="unet")
    assert [r["method"] for r in res["rows"]] == ["lpd (unet)"]
    r = res["rows"][0]
    assert r["iterations"] == 10 and math.isfinite(r["l2_pct"]) and r["training"]["arch"] == "unet"
