"""GPU colouring: bit-exact against the sequential greedy oracle, and the
Coloring rule end to end (atomic-free updates, bit-identical reruns)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1206_6409_amd import gencd as G
from paper_1206_6409_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _pattern(n, k, pairs):
    rows = np.array([p[0] for p in pairs], dtype=np.int64)
    cols = np.array([p[1] for p in pairs], dtype=np.int64)
    return synth.coo_to_csc(n, k, rows, cols, np.ones(len(pairs), np.float32))


def _gpu_color(n, k, cp, ri, va):
    X = G.Matrix.from_numpy(n, k, cp, ri, va)
    c, nc = G.color(X)
    return c.cpu().numpy(), nc


CASES = {
    "c3_small": lambda: synth.c3_zipf_lasso(scale=0.005),
    "c3_mid": lambda: synth.c3_zipf_lasso(scale=0.05),
    "c2_small": lambda: synth.c2_zipf_logistic(scale=0.02),
    "c1": lambda: synth.c1_ccd_logistic(),
    "c4_small": lambda: synth.c4_binary_path(scale=0.1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_color_bit_exact(name):
    print("CASE color", name, flush=True)
    P = CASES[name]()
    got, nc = _gpu_color(P.n, P.k, P.col_ptr, P.row_idx, P.val)
    exp, nce, _ = O.color(P.n, P.k, P.col_ptr, P.row_idx)
    assert nc == nce
    assert np.array_equal(got, exp)


def test_color_adversarial():
    # clique (one row holds every column), star, empty columns, single column
    cp, ri, va = _pattern(1, 300, [(0, j) for j in range(300)])
    got, nc = _gpu_color(1, 300, cp, ri, va)
    assert nc == 300 and np.array_equal(got, O.color(1, 300, cp, ri)[0])
    pairs = [(i, 0) for i in range(50)] + [(i, i + 1) for i in range(50)]
    cp, ri, va = _pattern(50, 51, pairs)
    got, nc = _gpu_color(50, 51, cp, ri, va)
    assert got[0] == 0 and np.all(got[1:] == 1) and nc == 2
    cp, ri, va = _pattern(3, 6, [(0, 1), (1, 1), (1, 3)])
    got, nc = _gpu_color(3, 6, cp, ri, va)
    assert np.array_equal(got, O.color(3, 6, cp, ri)[0])
    cp = np.zeros(5, np.int64)
    got, nc = _gpu_color(4, 4, cp, np.zeros(0, np.int32), np.zeros(0, np.float32))
    assert nc == 1 and np.all(got == 0)
    # many rows shared by few columns (long chains of ties in nnz)
    rng = np.random.default_rng(0)
    pairs = list({(int(rng.integers(0, 30)), int(rng.integers(0, 200))) for _ in range(900)})
    cp, ri, va = _pattern(30, 200, pairs)
    got, nc = _gpu_color(30, 200, cp, ri, va)
    exp, nce, _ = O.color(30, 200, cp, ri)
    assert nc == nce and np.array_equal(got, exp)


@pytest.mark.parametrize("scale", [0.005, 0.02])
def test_coloring_solve_parity_and_determinism(scale):
    print("CASE coloring solve", scale, flush=True)
    P = synth.c3_zipf_lasso(scale=scale)
    Xo = O.Matrix.of(P)
    lam = 0.1 * O.lambda_max(Xo, P.y, P.loss)
    ref = O.solve(Xo, P.y, P.loss, lam, O.CYCLIC, tol=1e-10, max_epochs=200000)
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    colors, nc = G.color(X)
    runs = []
    for rep in range(2):
        params = G.make_params(P.loss, lam, rule=G.COLORING, colors=colors, num_colors=nc,
                               seed=5, tol=1e-6, max_epochs=20000, piece=64)
        res = G.solve(X, y, params)
        assert res.status == G.OK, res.stats
        runs.append(res.w.cpu().numpy())
    # Coloring uses no atomics on z: reruns are bit-identical
    assert np.array_equal(runs[0], runs[1])
    oc = O.check(Xo, P.y, P.loss, lam, runs[0].astype(np.float64))
    assert oc.kkt <= 1e-6 * (1 + 1e-9)
    assert abs(oc.objective - ref.objective) <= 1e-6 * abs(ref.objective)


def test_coloring_step_matches_sequential_ccd():
    """One Coloring iteration over a colour class equals the oracle's
    sequential updates of the class members (disjoint rows)."""
    P = synth.c3_zipf_lasso(scale=0.01)
    X = G.Matrix.of(P)
    Xo = O.Matrix.of(P)
    colors, nc = G.color(X)
    cols = colors.cpu().numpy()
    nnz = np.diff(P.col_ptr)
    sizes = np.bincount(cols[nnz > 0], minlength=nc)
    c = int(np.argmax(sizes))
    J = np.nonzero((cols == c) & (nnz > 0))[0].astype(np.int32)
    assert J.size >= 8
    lam = 0.01 * O.lambda_max(Xo, P.y, P.loss)
    rng = np.random.default_rng(3)
    w = np.zeros(P.k, dtype=np.float32)
    half = J.size // 2
    w[J[:half]] = rng.normal(size=half).astype(np.float32) * 0.5
    z64 = O.check(Xo, P.y, P.loss, 0.0, w.astype(np.float64)).z
    zh = z64.astype(np.float32)
    zl = (z64 - zh).astype(np.float32)
    wd, zhd, zld = (torch.as_tensor(a, device=DEV) for a in (w, zh, zl))
    G.step(X, torch.as_tensor(P.y, device=DEV), G.make_params(P.loss, lam, rule=G.COLORING,
                                                               colors=colors, num_colors=nc),
           torch.as_tensor(J, device=DEV), wd, zhd, zld)
    wo, zo = w.astype(np.float64), zh.astype(np.float64) + zl.astype(np.float64)
    for j in J:
        O.step(Xo, P.y, P.loss, lam, [j], wo, zo)
    zg = zhd.cpu().numpy().astype(np.float64) + zld.cpu().numpy().astype(np.float64)
    scale = np.abs(zo) + np.sqrt(np.mean(zo ** 2))
    assert np.sqrt(np.mean(zo ** 2)) > 0
    assert np.all(np.abs(zg - zo) <= 1e-5 * scale)
    np.testing.assert_allclose(wd.cpu().numpy(), wo, rtol=1e-5, atol=1e-7)


def test_coloring_graph_replays_bit_identical():
    """Coloring uses no atomics: the captured-epoch path must reproduce the
    plain path bit for bit over many replays."""
    P = synth.c3_zipf_lasso(scale=0.01)
    Xo = O.Matrix.of(P)
    lam = 0.1 * O.lambda_max(Xo, P.y, P.loss)
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    colors, nc = G.color(X)
    ws = []
    for flags in (0, G.USE_GRAPH, G.USE_GRAPH):
        params = G.make_params(P.loss, lam, rule=G.COLORING, colors=colors, num_colors=nc,
                               seed=5, tol=1e-7, max_epochs=5000, piece=64, flags=flags)
        res = G.solve(X, y, params)
        assert res.status == G.OK and res.stats["epochs"] > 2
        ws.append(res.w.cpu().numpy())
    assert np.array_equal(ws[0], ws[1]) and np.array_equal(ws[1], ws[2])


@pytest.mark.parametrize("cap", [0, 1, 5, 10**9])
def test_balanced_colouring_bit_exact(cap):
    """Balanced colouring on the GPU equals the oracle's bit for bit, and the
    Coloring solve on it reaches the optimum."""
    print("CASE balance", cap, flush=True)
    P = synth.c3_zipf_lasso(scale=0.003)
    X = G.Matrix.of(P)
    colors, nc = G.color(X)
    bal, nb = G.balance_colors(X, colors, nc, cap)
    ocol, onc, _ = O.color(P.n, P.k, P.col_ptr, P.row_idx)
    obal, onb = O.balance_colors(P.k, P.col_ptr, ocol, onc, cap)
    assert nb == onb and np.array_equal(bal.cpu().numpy(), obal)
    if cap == 0:
        Xo = O.Matrix.of(P)
        lam = 0.1 * O.lambda_max(Xo, P.y, P.loss)
        ref = O.solve(Xo, P.y, P.loss, lam, O.CYCLIC, tol=1e-11, max_epochs=500000)
        params = G.make_params(P.loss, lam, rule=G.COLORING, colors=bal, num_colors=nb, seed=3,
                               tol=1e-7, max_epochs=20000)
        res = G.solve(X, torch.as_tensor(P.y, device="cuda"), params)
        assert res.status == G.OK
        oc = O.check(Xo, P.y, P.loss, lam, res.w.cpu().numpy().astype(np.float64))
        assert abs(oc.objective - ref.objective) <= 1e-6 * abs(ref.objective)


def test_balanced_colouring_rejects_out_of_range():
    P = synth.c3_zipf_lasso(scale=0.003)
    X = G.Matrix.of(P)
    colors, nc = G.color(X)
    with pytest.raises(G.GencdError):
        G.balance_colors(X, colors, max(1, nc - 1), 0)
