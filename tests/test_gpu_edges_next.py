"""Degenerate cases of Top-Greedy, Block Shotgun, the fused iteration and
improve-delta on the GPU, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1206_6409_amd import gencd as G
from paper_1206_6409_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _solve(P, lam, tol=1e-8, max_epochs=200000, **kw):
    params = G.make_params(P.loss, lam, seed=2, tol=tol, max_epochs=max_epochs, **kw)
    return G.solve(G.Matrix.of(P), torch.as_tensor(P.y, device=DEV), params)


def _ref(P, lam):
    Xo = O.Matrix.of(P)
    r = O.solve(Xo, P.y, P.loss, lam, O.CYCLIC, tol=1e-11, max_epochs=500000)
    assert r.converged
    return Xo, r


def _assert_optimum(P, lam, res, Xo, ref, kkt=1e-8):
    assert res.status == G.OK and res.stats["kkt_max"] <= kkt
    oc = O.check(Xo, P.y, P.loss, lam, res.w.cpu().numpy().astype(np.float64))
    assert abs(oc.objective - ref.objective) <= 1e-6 * abs(ref.objective)


@pytest.fixture(scope="module")
def small():
    P = synth.c1_ccd_logistic(scale=0.1)
    lam = 0.1 * O.lambda_max(O.Matrix.of(P), P.y, P.loss)
    Xo, ref = _ref(P, lam)
    return P, lam, Xo, ref


def test_block_shotgun_one_column_per_block(small):
    # every block a single column: P_b* = 1, windows of one column
    P, lam, Xo, ref = small
    kl = int(np.sum(np.diff(P.col_ptr) > 0))
    rho, ps = G.estimate_block_rho(G.Matrix.of(P), kl, 20, G.make_params(0, 0.0, seed=2))
    np.testing.assert_allclose(rho, 1.0, rtol=1e-12)
    assert set(ps) == {1}
    res = _solve(P, lam, rule=G.BLOCK_SHOTGUN, block=kl)
    _assert_optimum(P, lam, res, Xo, ref)
    assert res.stats["iters"] == kl * res.stats["epochs"]


def test_block_shotgun_more_blocks_than_columns_clamps(small):
    P, lam, Xo, ref = small
    kl = int(np.sum(np.diff(P.col_ptr) > 0))
    res = _solve(P, lam, rule=G.BLOCK_SHOTGUN, block=min(4096, kl + 50))
    _assert_optimum(P, lam, res, Xo, ref)


def test_top_greedy_window_smaller_than_accept_count(small):
    P, lam, Xo, ref = small
    res = _solve(P, lam, rule=G.TOP_GREEDY, select_size=37, block=1000)
    _assert_optimum(P, lam, res, Xo, ref)


@pytest.mark.parametrize("rule,kw", [(G.SHOTGUN, dict(select_size=1)), (G.SHOTGUN, dict(select_size=10**6)),
                                     (G.CYCLIC, dict()), (G.BLOCK_SHOTGUN, dict(block=3))])
def test_fused_extreme_windows(small, rule, kw):
    P, lam, Xo, ref = small
    res = _solve(P, lam, rule=rule, flags=G.FUSED | G.USE_GRAPH, **kw)
    _assert_optimum(P, lam, res, Xo, ref)


def test_single_column_logistic_improve_is_the_minimiser():
    # k = 1: one improved coordinate step solves the problem (1-D logistic)
    rng = np.random.default_rng(4)
    n = 300
    x = rng.normal(size=n).astype(np.float32)
    y = np.where(rng.random(n) < 1 / (1 + np.exp(-0.7 * x)), 1.0, -1.0).astype(np.float32)
    col_ptr = np.array([0, n], dtype=np.int64)
    P = synth.Problem(n, 1, col_ptr, np.arange(n, dtype=np.int32), x, y, O.LOGISTIC,
                      np.zeros(1), "one column")
    lam = 0.01
    Xo, ref = _ref(P, lam)
    res = _solve(P, lam, rule=G.CYCLIC, improve=500, max_epochs=3, tol=1e-7)
    assert res.stats["epochs"] == 1  # converged at the first check (FP32 floor ~1e-8)
    oc = O.check(Xo, P.y, P.loss, lam, res.w.cpu().numpy().astype(np.float64))
    assert abs(oc.objective - ref.objective) <= 1e-7 * abs(ref.objective)


def test_empty_matrix_new_rules():
    n, k = 20, 6
    P = synth.Problem(n, k, np.zeros(k + 1, np.int64), np.zeros(0, np.int32),
                      np.zeros(0, np.float32), np.where(np.arange(n) % 2, 1.0, -1.0).astype(np.float32),
                      O.LOGISTIC, np.zeros(k), "empty")
    for kw in (dict(rule=G.TOP_GREEDY, select_size=4, block=2), dict(rule=G.BLOCK_SHOTGUN, block=2),
               dict(rule=G.SHOTGUN, select_size=4, flags=G.FUSED), dict(rule=G.SHOTGUN, select_size=0),
               dict(rule=G.SHOTGUN, select_size=4, improve=10)):
        res = _solve(P, 0.1, **kw)
        assert res.status == G.OK and np.all(res.w.cpu().numpy() == 0)


@pytest.mark.parametrize("flags", [0, G.USE_GRAPH])
def test_divergence_guard_halves_the_selection_and_converges(flags):
    """Jacobi Shotgun over every column of strongly correlated columns
    overshoots; the guard restores the last checked point, halves |J| and
    rebuilds the selection order, and the solve still reaches the optimum."""
    rng = np.random.default_rng(5)
    n, k = 200, 64
    # a shared component correlates every pair of columns (rho ~ 14 on the
    # normalised Gram matrix, so only |J| <= 8 is stable)
    dense = rng.standard_normal((n, k)) + 0.5 * rng.standard_normal((n, 1))
    y = (dense[:, :5] @ rng.standard_normal(5) + 0.1 * rng.standard_normal(n)).astype(np.float32)
    col_ptr = np.arange(0, n * k + 1, n, dtype=np.int64)
    row_idx = np.tile(np.arange(n, dtype=np.int32), k)
    val = dense.T.reshape(-1).astype(np.float32)
    P = synth.Problem(n, k, col_ptr, row_idx, val, y, synth.SQUARED, name="correlated")
    lam = 0.05 * O.lambda_max(O.Matrix.of(P), P.y, P.loss)
    Xo, ref = _ref(P, lam)
    res = _solve(P, lam, tol=1e-7, rule=G.SHOTGUN, select_size=k, flags=flags)
    assert res.stats["select_size"] < k  # the guard fired
    _assert_optimum(P, lam, res, Xo, ref, kkt=1e-7)


@pytest.mark.parametrize("m,K,neg", [(700, 64, 0), (4096, 300, 10), (3000, 1, 0), (4096, 4096, 5)])
def test_top_greedy_ties_go_to_the_lowest_positions(m, K, neg):
    """At lambda >= lambda_max from w = 0 every proxy is exactly 0; a few
    columns are then made to propose by a nonzero start.  Top-Greedy takes
    the proposals with phi < 0 and, among the tied zeros, the lowest window
    positions, whatever the number of ties."""
    print("CASE top-greedy ties", m, K, neg, flush=True)
    P = synth.c2_zipf_logistic(scale=0.02)
    Xo = O.Matrix.of(P)
    lam = 2.0 * O.lambda_max(Xo, P.y, P.loss)
    live = np.nonzero(np.diff(P.col_ptr) > 0)[0]
    rng = np.random.default_rng(3)
    J = rng.choice(live, size=min(m, live.size), replace=False).astype(np.int32)
    m = J.size
    w = np.zeros(P.k, dtype=np.float32)
    w[J[rng.choice(m, size=neg, replace=False)]] = 0.5  # these propose moving back to 0
    oc = O.check(Xo, P.y, P.loss, 0.0, w.astype(np.float64))
    z_hi = oc.z.astype(np.float32)
    z_lo = (oc.z - z_hi.astype(np.float64)).astype(np.float32)
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    params = G.make_params(P.loss, lam, rule=G.TOP_GREEDY, select_size=m, block=K)
    res = G.step(X, y, params, torch.as_tensor(J, device=DEV), torch.as_tensor(w, device=DEV),
                 torch.as_tensor(z_hi, device=DEV), torch.as_tensor(z_lo, device=DEV))
    torch.cuda.synchronize()
    acc = res.accepted.cpu().numpy()
    phi = res.phi.cpu().numpy()
    assert acc.sum() == min(K, m)
    below = np.nonzero(phi < 0)[0]
    assert below.size == neg and np.all(acc[below] == 1)
    zeros = np.nonzero(phi == 0)[0]
    take = min(K, m) - below.size
    assert np.array_equal(np.nonzero(acc[zeros])[0], np.arange(take))  # the first tied positions
