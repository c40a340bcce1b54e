"""Spectral-radius estimate (section 4.1's P* = k / (2 rho)) on the GPU
against the FP64 oracle, and solves that take |J| from it.

Both sides run the same power iteration in FP64; only the summation order
differs (atomics on the device), so every iterate agrees to 1e-10 relative.
The derived |J| = floor(k_live / (2 rho)) is compared exactly unless
k_live / (2 rho) is within 1e-8 of an integer, where either neighbour is
accepted.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1206_6409_amd import gencd as G
from paper_1206_6409_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(*a):
    print("CASE", *a, flush=True)


def _empty_tail(P, extra):
    """P with `extra` empty columns appended."""
    col_ptr = np.concatenate([P.col_ptr, np.full(extra, P.col_ptr[-1], dtype=P.col_ptr.dtype)])
    return synth.Problem(P.n, P.k + extra, col_ptr, P.row_idx, P.val, P.y, P.loss,
                         np.concatenate([P.w_true, np.zeros(extra)]), P.name + "+empty")


def _request(seed):
    r = synth.c5_request_stream(count=1, rate=1.0, seed=seed, n_range=(2000, 4000),
                                k_range=(3000, 8000), d_range=(0.002, 0.01))[0]
    return synth.request_problem(r, support=30)


PROBLEMS = {
    "c1": lambda: synth.c1_ccd_logistic(scale=0.5),
    "c2": lambda: synth.c2_zipf_logistic(scale=0.02),
    "c3": lambda: synth.c3_zipf_lasso(scale=0.005),
    "c4": lambda: synth.c4_binary_path(scale=0.1),
    "c5": lambda: _request(7),
    "orth": lambda: synth.orthogonal_design(3000, 700, 0, 3),
    "empty": lambda: _empty_tail(synth.c1_ccd_logistic(scale=0.2), 37),
}


def _pstar_ok(gpu_sel, k_live, rho):
    q = k_live / (2.0 * rho)
    want = O.pstar(k_live, rho)
    if abs(q - round(q)) < 1e-8 * max(q, 1.0):
        return abs(gpu_sel - want) <= 1
    return gpu_sel == want


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("piece,group", [(0, 0), (64, 4), (256, 32)])
def test_rho_matches_oracle(name, piece, group):
    _case("rho", name, piece, group)
    P = PROBLEMS[name]()
    X = G.Matrix.of(P, DEV)
    params = G.make_params(0, 0.0, piece=piece, group=group)
    r = G.estimate_rho(X, 20, params)
    ro, ho, klo = O.rho(O.Matrix.of(P), 20)
    assert r.k_live == klo
    np.testing.assert_allclose(r.history, ho, rtol=1e-10)
    assert np.all(np.diff(r.history) >= -1e-10 * r.rho)  # monotone lower bounds
    assert _pstar_ok(r.select_size, r.k_live, r.rho)
    if name == "orth":
        np.testing.assert_allclose(r.history, 1.0, rtol=1e-12)


def test_rho_edge_cases():
    _case("rho edge")
    # every column empty: no iteration, rho 0, |J| = 1
    n, k = 50, 9
    P = synth.Problem(n, k, np.zeros(k + 1, np.int64), np.zeros(0, np.int32),
                      np.zeros(0, np.float32), np.ones(n, np.float32), 0, np.zeros(k), "empty")
    r = G.estimate_rho(G.Matrix.of(P, DEV), 5)
    assert r.k_live == 0 and r.rho == 0.0 and r.select_size == 1
    # one column: G = [1]
    P1 = synth.orthogonal_design(40, 1, 0, 1)
    r = G.estimate_rho(G.Matrix.of(P1, DEV), 3)
    assert r.k_live == 1 and r.history == pytest.approx([1.0] * 3, rel=1e-14)
    # iteration count outside 1..1024
    X = G.Matrix.of(P1, DEV)
    for bad in (0, 1025):
        with pytest.raises(G.GencdError):
            G.estimate_rho(X, bad)


@pytest.mark.parametrize("seed,rule", [(7, G.SHOTGUN), (8, G.SHOTGUN), (9, G.THREAD_GREEDY)])
def test_solve_with_select_size_from_rho(seed, rule):
    _case("auto |J| solve", seed, rule)
    P = _request(seed)
    X = G.Matrix.of(P, DEV)
    y = torch.from_numpy(P.y).to(DEV)
    Xo = O.Matrix.of(P)
    lam = 0.1 * O.lambda_max(Xo, P.y, P.loss)
    params = G.make_params(P.loss, lam, rule=rule, select_size=0, block=16, seed=5, tol=1e-8,
                           max_epochs=20000)
    res = G.solve(X, y, params)
    st = res.stats
    ro, _, klo = O.rho(Xo, 20)
    assert abs(st["rho"] - ro) <= 1e-10 * ro
    assert _pstar_ok(st["select_size"], klo, ro)
    assert res.status == 0 and st["kkt_max"] <= 1e-8
    # the oracle's own |J| from its own rho estimate
    ref = O.solve(Xo, P.y, P.loss, lam, O.SHOTGUN, select_size=O.pstar(klo, ro), seed=5,
                  tol=1e-10, max_epochs=200000)
    assert abs(st["objective"] - ref.objective) <= 1e-6 * abs(ref.objective)
