"""Synthetic generators: shapes, laws and bit-for-bit reproducibility."""
import numpy as np
import pytest

from paper_1206_6409_amd import synth


def _valid_csc(P):
    assert P.col_ptr.dtype == np.int64 and P.row_idx.dtype == np.int32 and P.val.dtype == np.float32
    assert P.col_ptr[0] == 0 and np.all(np.diff(P.col_ptr) >= 0) and P.col_ptr[-1] == P.row_idx.size
    for j in range(P.k):
        r = P.row_idx[P.col_ptr[j]:P.col_ptr[j + 1]]
        assert np.all(np.diff(r) > 0)  # sorted, unique
    assert P.row_idx.min(initial=0) >= 0 and P.row_idx.max(initial=0) < P.n


@pytest.mark.parametrize("gen", [synth.c1_ccd_logistic, synth.c2_zipf_logistic,
                                 synth.c3_zipf_lasso, synth.c4_binary_path])
def test_generators_valid_and_reproducible(gen):
    a = gen(scale=0.02)
    b = gen(scale=0.02)
    _valid_csc(a)
    for f in ("col_ptr", "row_idx", "val", "y"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    if a.loss == synth.LOGISTIC:
        assert set(np.unique(a.y).tolist()) <= {-1.0, 1.0}


def test_c1_density_and_values():
    P = synth.c1_ccd_logistic()
    assert (P.n, P.k) == (2000, 5000)
    assert abs(P.nnz / (P.n * P.k) - 0.01) < 0.0005
    assert abs(P.val.std() - 1.0) < 0.02


def test_c2_zipf_shape_small():
    P = synth.c2_zipf_logistic(scale=0.05)
    nnz = np.diff(P.col_ptr)
    rows_len = np.bincount(P.row_idx, minlength=P.n)
    assert abs(rows_len.mean() - 50) < 1.5
    # heavy head: the largest column is nearly dense, many columns are empty
    assert nnz.max() > 0.8 * P.n
    assert (nnz == 0).mean() > 0.1
    # rows are L2-normalised
    ss = np.bincount(P.row_idx, weights=P.val.astype(np.float64) ** 2, minlength=P.n)
    np.testing.assert_allclose(ss[rows_len > 0], 1.0, rtol=1e-5)


def test_c4_binary():
    P = synth.c4_binary_path(scale=0.1)
    assert np.all(P.val == 1.0)
    g = synth.lambda_grid(2.0)
    assert g.size == 64 and g[0] == 2.0 and abs(g[-1] - 2e-3) < 1e-15 and np.all(np.diff(g) < 0)


def test_request_stream():
    rs = synth.c5_request_stream(count=50, rate=10.0)
    assert len(rs) == 50
    assert all(1000 <= r.n <= 50000 and 1000 <= r.k <= 200000 for r in rs)
    assert all(0.001 <= r.density <= 0.02 and 1e-3 <= r.lambda_ratio <= 0.5 for r in rs)
    t = np.array([r.arrival for r in rs])
    assert np.all(np.diff(t) >= 0)
