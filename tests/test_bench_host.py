"""Host arithmetic of bench.py's roofline (CPU only): the algorithmic-bytes
model behind `roofline.frac`, pinned to its per-evaluation totals at 15
entries per row, and the fraction that follows from it."""
import numpy as np
import pytest

import bench


def sizes(N, Nt, z=15, zl=15):
    return {"N": N, "Nt": Nt, "nnz_magnet": z * N, "nnz_potential": zl * Nt}


@pytest.mark.parametrize("seed", range(5))
def test_bytes_model_reduces_to_the_per_evaluation_totals(seed):
    # with 15 entries per row the per-row model sums, per evaluation with k
    # CG iterations, to 1256 N + (224 + 288 k) N_t bytes in FP64 and to
    # 696 N + (144 + 176 k) N_t in the FP32 form
    rng = np.random.default_rng(seed)
    N, Nt = int(rng.integers(1, 10**6)), int(rng.integers(0, 3 * 10**6))
    evals = int(rng.integers(1, 10**4))
    pcg = int(rng.integers(0, 20 * evals))
    sz = sizes(N, Nt)
    b64 = evals * (1256 * N + 224 * Nt) + 288 * pcg * Nt
    b32 = evals * (696 * N + 144 * Nt) + 176 * pcg * Nt
    assert bench.bytes_per_evaluation_model(sz, evals, pcg, fp64=True) == pytest.approx(b64, rel=1e-12)
    assert bench.bytes_per_evaluation_model(sz, evals, pcg, fp64=False) == pytest.approx(b32, rel=1e-12)


def test_bytes_model_is_linear_in_the_row_lengths():
    # one more entry per magnet row costs 64 bytes per magnet node and
    # evaluation in FP64 (36 in FP32); one more per potential row costs 12
    # bytes per potential row for the solve's start and per CG iteration (8)
    N, Nt, evals, pcg = 1000, 3000, 7, 50
    for fp64, dm, dl in ((True, 64, 12), (False, 36, 8)):
        b = bench.bytes_per_evaluation_model(sizes(N, Nt), evals, pcg, fp64)
        bm = bench.bytes_per_evaluation_model(sizes(N, Nt, z=16), evals, pcg, fp64)
        bl = bench.bytes_per_evaluation_model(sizes(N, Nt, zl=16), evals, pcg, fp64)
        assert bm - b == pytest.approx(dm * N * evals, rel=1e-12)
        assert bl - b == pytest.approx(dl * Nt * (evals + pcg), rel=1e-12)


def test_roofline_fraction_is_model_bytes_over_time_over_peak():
    N, Nt, evals, pcg = 68921, 250047, 337, 5452
    tm = {"launches": 46880, "ms": 579.0, "bytes": 1.5e12}
    ro = bench.roofline_of(tm, "k_step<double,4>", sizes(N, Nt), evals, pcg, fp64=True, traffic=3.5e7)
    B = evals * (1256 * N + 224 * Nt) + 288 * pcg * Nt
    secs = 0.579
    assert ro["achieved"] == pytest.approx(B / secs / 1e9, rel=1e-12)
    assert ro["frac"] == pytest.approx(B / secs / 1e9 / 8000.0, rel=1e-12)
    assert ro["peak"] == 8000.0 and ro["unit"] == "GB/s" and ro["bound"] == "hbm"
    assert ro["avg_launch_us"] == pytest.approx(579.0e3 / 46880, rel=1e-12)
    assert ro["alg_bytes_per_launch"] == pytest.approx(B / 46880, rel=1e-12)
    assert ro["phase_model"]["frac"] == pytest.approx(1.5e12 / secs / 1e9 / 8000.0, rel=1e-12)
    assert ro["traffic"] == 3.5e7
    # no launches timed: no roofline
    assert bench.roofline_of({"launches": 0, "ms": 0.0, "bytes": 0.0}, "k") is None
