"""The whole privacy-preserving PCA pipeline from a raw dataset (homomorphic
means and covariance, PowerMethod, EigenShift) with the accuracy metrics of
section 7.2: the decrypted components give the same R2(X) and R2(V) as the
FP64 replay of the same algorithm."""
import pytest

pytestmark = pytest.mark.gpu


def test_pppca_accuracy_pipeline_small():
    from paper_2305_17341_amd import pca
    res = pca.accuracy_bench(cases=[("s200_lE2_lP4", 200, 2, 4)], seed=7, log=print)
    r = res["rows"][0]
    assert r["max_abs_err_vs_replay"] < 1e-3
    assert abs(r["r2_x"] - r["r2_x_fp64_replay"]) < 1e-3
    assert abs(r["r2_v"] - r["r2_v_fp64_replay"]) < 1e-3
    assert r["refreshes"] > 0 and 0.0 < r["r2_x"] <= r["r2_x_exact_pca"] + 1e-3
