"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances (FP32 path against FP64 oracle):
  * selection permutation, accepted positions: bit-exact (integer work);
  * lambda_max, FP64 check (objective, KKT, z = Xw): relative 1e-12
    (both sides FP64, different summation order);
  * one iteration from a shared state: z within 1e-5 (|z_or| + rms(z_or));
    g within 1e-5 of max|g| and delta within 1e-5 of max|delta| (FP32 sums);
  * end-to-end: solved to FP64 KKT <= 1e-8 (re-checked by the oracle at the
    GPU's w), the objective is within 1e-6 relative of the oracle's optimum.
    KKT <= 1e-6 alone does not pin the objective that tightly on k >> n
    logistic problems (the objective error is about quadratic in the KKT
    violation: ~1e-4 relative at 1e-6 on the binary workload), so solves at
    1e-6 are checked for KKT and for an objective within 2e-4.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1206_6409_amd import gencd as G
from paper_1206_6409_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _print_case(*args):
    print("CASE", *args, flush=True)


def rel_close(a, b, rtol, scale=None):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    s = np.abs(b) + (np.sqrt(np.mean(b ** 2)) if scale is None else scale)
    return np.all(np.abs(a - b) <= rtol * s + 1e-30), np.max(np.abs(a - b) / (s + 1e-300))


@pytest.fixture(scope="module")
def problems():
    return {
        "c1": synth.c1_ccd_logistic(scale=0.5),
        "c2": synth.c2_zipf_logistic(scale=0.02),
        "c3": synth.c3_zipf_lasso(scale=0.005),
        "c4": synth.c4_binary_path(scale=0.1),
        "c1s": synth.c1_ccd_logistic(scale=0.05),
    }


# --------------------------------------------------------------------------
# selection, lambda_max, FP64 check
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m", [1, 2, 7, 1000, 4097, 65536, 300001])
def test_select_permutation_bit_exact(m):
    _print_case("perm", m)
    for e in (0, 1, 17):
        got = G.select_perm(m, 102, e).cpu().numpy()
        if m <= 5000:
            exp = O.perm(m, 102, e)
            assert np.array_equal(got, exp)
        else:
            idx = np.random.default_rng(e).choice(m, 2000, replace=False)
            L = O.lib()
            exp = np.array([L.orc_perm(m, 102, e, int(p)) for p in idx])
            assert np.array_equal(got[idx], exp)
            assert np.array_equal(np.sort(got), np.arange(m))


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4"])
def test_lambda_max_and_check(problems, name):
    _print_case("check", name)
    P = problems[name]
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    Xo = O.Matrix.of(P)
    lm_gpu = G.lambda_max(X, y, P.loss)
    lm_or = O.lambda_max(Xo, P.y, P.loss)
    assert lm_gpu == pytest.approx(lm_or, rel=1e-12)
    rng = np.random.default_rng(1)
    w = np.zeros(P.k, dtype=np.float32)
    sup = rng.choice(P.k, size=min(P.k, 300), replace=False)
    w[sup] = rng.normal(size=sup.size).astype(np.float32) * 0.3
    lam = 0.1 * lm_or
    gc = G.check(X, y, P.loss, lam, torch.as_tensor(w, device=DEV))
    oc = O.check(Xo, P.y, P.loss, lam, w.astype(np.float64))
    assert gc.objective == pytest.approx(oc.objective, rel=1e-12)
    assert gc.kkt == pytest.approx(oc.kkt, rel=1e-10, abs=1e-15)
    assert gc.nnz_w == oc.nnz_w
    gap_or, _ = O.duality_gap(Xo, P.y, P.loss, lam, w.astype(np.float64))
    assert gc.gap == pytest.approx(gap_or, rel=1e-9, abs=1e-13)
    np.testing.assert_allclose(gc.z64.cpu().numpy(), oc.z, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gc.g64.cpu().numpy(), oc.g, rtol=1e-9, atol=1e-14)


# --------------------------------------------------------------------------
# one iteration from a shared state
# --------------------------------------------------------------------------

def _state(P, rng, frac=0.05):
    w = np.zeros(P.k, dtype=np.float32)
    nz = np.nonzero(np.diff(P.col_ptr) > 0)[0]
    sup = rng.choice(nz, size=max(1, int(frac * nz.size)), replace=False)
    w[sup] = (rng.normal(size=sup.size) * 0.2).astype(np.float32)
    return w


def _split(z64):
    hi = z64.astype(np.float32)
    lo = (z64 - hi.astype(np.float64)).astype(np.float32)
    return hi, lo


STEP_CASES = [
    ("c1", G.SHOTGUN, 0, 8, 64), ("c1", G.SHOTGUN, 0, 16, 64),
    ("c2", G.SHOTGUN, 0, 8, 1024), ("c2", G.SHOTGUN, 0, 4, 64), ("c2", G.SHOTGUN, 0, 32, 128),
    ("c2", G.THREAD_GREEDY, 64, 8, 256), ("c2", G.THREAD_GREEDY, 7, 16, 64),
    ("c2", G.GREEDY, 0, 8, 1024), ("c2", G.GREEDY, 0, 4, 64),
    ("c3", G.SHOTGUN, 0, 8, 64), ("c4", G.SHOTGUN, 0, 4, 64), ("c4", G.THREAD_GREEDY, 16, 8, 64),
    ("c2", G.SHOTGUN, 0, 8, 256, G.EXACT_ACCUM), ("c2", G.THREAD_GREEDY, 64, 8, 256, G.EXACT_ACCUM),
    ("c2", G.TOP_GREEDY, 64, 8, 256), ("c2", G.TOP_GREEDY, 1, 16, 64), ("c4", G.TOP_GREEDY, 100, 8, 64),
    ("c1", G.TOP_GREEDY, 100000, 4, 128),
    # J = every live column: the whole-window accept runs in two stages
    # (chunk winners, then the best of them)
    ("c2", G.GREEDY, 0, 8, 256, 0, 100000), ("c4", G.GREEDY, 0, 8, 256, 0, 100000),
    ("c2", G.THREAD_GREEDY, 100000, 8, 256, 0, 100000),
]
# Propose from the refreshed residual vector (2) and per entry (1), whatever
# the automatic choice would be for the case
STEP_CASES += [c[:5] + ((c[5] if len(c) > 5 else 0), (c[6] if len(c) > 6 else 700), r)
               for c in [("c1", G.SHOTGUN, 0, 8, 64), ("c2", G.SHOTGUN, 0, 8, 1024),
                         ("c2", G.THREAD_GREEDY, 64, 8, 256), ("c2", G.GREEDY, 0, 8, 256, 0, 100000),
                         ("c3", G.SHOTGUN, 0, 8, 64), ("c4", G.TOP_GREEDY, 100, 8, 64),
                         ("c2", G.SHOTGUN, 0, 8, 256, G.EXACT_ACCUM)]
               for r in (1, 2)]


@pytest.mark.parametrize("case", STEP_CASES)
def test_step_parity(problems, case):
    name, rule, block, group, piece = case[:5]
    flags = case[5] if len(case) > 5 else 0
    m_cap = case[6] if len(case) > 6 else 700
    residual = case[7] if len(case) > 7 else 0
    _print_case("step", name, rule, block, group, piece, flags, m_cap, residual)
    P = problems[name]
    X = G.Matrix.of(P)
    Xo = O.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    rng = np.random.default_rng(7)
    w = _state(P, rng)
    oc = O.check(Xo, P.y, P.loss, 0.0, w.astype(np.float64))
    z_hi, z_lo = _split(oc.z)
    lam = 0.1 * O.lambda_max(Xo, P.y, P.loss)
    live = np.nonzero(np.diff(P.col_ptr) > 0)[0]
    # J: random live columns, plus the heaviest column so split columns are covered
    m = min(live.size, m_cap)
    J = rng.choice(live, size=m, replace=False).astype(np.int32)
    heavy = int(np.argmax(np.diff(P.col_ptr)))
    if heavy not in J:
        J[0] = heavy
    params = G.make_params(P.loss, lam, rule=rule, select_size=m, block=block, group=group,
                           piece=piece, flags=flags, residual=residual)
    w_d = torch.as_tensor(w, device=DEV)
    zh_d = torch.as_tensor(z_hi, device=DEV)
    zl_d = torch.as_tensor(z_lo, device=DEV)
    res = G.step(X, y, params, torch.as_tensor(J, device=DEV), w_d, zh_d, zl_d)
    torch.cuda.synchronize()
    # oracle from the same state (z as the FP64 value of z_hi + z_lo)
    wo = w.astype(np.float64)
    zo = z_hi.astype(np.float64) + z_lo.astype(np.float64)
    oblock = block if rule == G.THREAD_GREEDY else (m if rule == G.GREEDY else 0)
    otop = min(block, m) if rule == G.TOP_GREEDY else 0
    g_gpu = res.g.cpu().numpy().astype(np.float64)
    d_gpu = res.delta.cpu().numpy().astype(np.float64)
    acc_gpu = res.accepted.cpu().numpy()
    # propose parity (state at entry)
    probe = O.step(Xo, P.y, P.loss, lam, J, wo.copy(), zo.copy(), block=oblock, top=otop)
    gs = np.abs(probe.g).max()
    assert np.max(np.abs(g_gpu - probe.g)) <= 1e-5 * gs
    ds = max(np.abs(probe.delta).max(), 1e-30)
    assert np.max(np.abs(d_gpu - probe.delta)) <= 1e-5 * ds + 1e-6 * np.abs(wo[J]).max()
    forced = None
    if oblock > 0:
        nb = (m + oblock - 1) // oblock
        forced = np.full(nb, -1, dtype=np.int32)
        for b in range(nb):
            lo, hi = b * oblock, min(m, (b + 1) * oblock)
            gpos = lo + int(np.argmax(acc_gpu[lo:hi]))
            assert acc_gpu[lo:hi].sum() == 1
            opos = lo + int(np.argmax(probe.accepted[lo:hi]))
            if gpos != opos:  # near tie: accept only if the proxies agree to 1e-6
                assert probe.phi[gpos] - probe.phi[opos] <= 1e-6 * abs(probe.phi[opos])
            forced[b] = gpos
    elif otop > 0:
        # the otop smallest proxies of the window; where FP32 and FP64 order
        # differ, the GPU's extra picks must tie the oracle's last pick to 1e-6
        assert acc_gpu.sum() == otop
        gset, oset = np.nonzero(acc_gpu)[0], np.nonzero(probe.accepted)[0]
        kth = np.sort(probe.phi)[otop - 1]
        for q in np.setdiff1d(gset, oset):
            assert probe.phi[q] - kth <= 1e-6 * abs(kth)
        forced = gset.astype(np.int32)
    else:
        assert np.all(acc_gpu == 1)
    O.step(Xo, P.y, P.loss, lam, J, wo, zo, block=oblock, forced=forced, top=otop)
    z_gpu = zh_d.cpu().numpy().astype(np.float64) + zl_d.cpu().numpy().astype(np.float64)
    ok, worst = rel_close(z_gpu, zo, 1e-5)
    assert ok, f"z mismatch {worst}"
    np.testing.assert_allclose(w_d.cpu().numpy(), wo, rtol=1e-5, atol=1e-6 * max(1e-30, np.abs(wo).max()))


# --------------------------------------------------------------------------
# end to end
# --------------------------------------------------------------------------

SOLVE_CASES = [
    ("c1", G.SHOTGUN, dict(select_size=256)),
    ("c1", G.THREAD_GREEDY, dict(select_size=1024, block=8)),
    ("c2", G.SHOTGUN, dict(select_size=512)),
    ("c2", G.THREAD_GREEDY, dict(select_size=2048, block=16)),
    ("c1", G.TOP_GREEDY, dict(select_size=1024, block=64)),
    ("c2", G.TOP_GREEDY, dict(select_size=2048, block=256)),
    ("c3", G.SHOTGUN, dict(select_size=256)),
    ("c4", G.SHOTGUN, dict(select_size=256)),
    ("c1s", G.STOCHASTIC, dict()),
    ("c2", G.SHOTGUN, dict(select_size=512, residual=1)),
    ("c2", G.SHOTGUN, dict(select_size=512, residual=2)),
    ("c3", G.SHOTGUN, dict(select_size=256, residual=2)),
]
LAM_FRAC = {"c1": 0.1, "c2": 0.05, "c3": 0.1, "c4": 0.05, "c1s": 0.1}


@pytest.fixture(scope="module")
def optima(problems):
    out = {}
    for name, P in problems.items():
        Xo = O.Matrix.of(P)
        lam = LAM_FRAC[name] * O.lambda_max(Xo, P.y, P.loss)
        r = O.solve(Xo, P.y, P.loss, lam, O.CYCLIC, tol=1e-11, max_epochs=500000)
        assert r.converged
        out[name] = (lam, r)
    return out


# A float32 weight cannot move by less than half an ulp, so the KKT violation
# of a float32 solution is floored near c_j * ulp(|w_j|) / 2; on the Lasso
# workload (c_j ~ 1, |w_j| ~ 1) that is ~6e-8, so its tight level is 1e-7.
TIGHT = {"c3": 1e-7}


@pytest.mark.parametrize("name,rule,kw", SOLVE_CASES)
@pytest.mark.parametrize("level", ["tight", "1e-6"])
def test_solve_parity(problems, optima, name, rule, kw, level):
    kkt = TIGHT.get(name, 1e-8) if level == "tight" else 1e-6
    _print_case("solve", name, rule, kw, kkt)
    P = problems[name]
    lam, ref = optima[name]
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    params = G.make_params(P.loss, lam, rule=rule, seed=3, tol=kkt, max_epochs=20000, **kw)
    res = G.solve(X, y, params)
    st = res.stats
    print("STATS", name, rule, {k: st[k] for k in ("epochs", "iters", "objective", "kkt_max", "gap",
                                                  "nnz_w", "seconds")}, "ref", ref.objective,
          flush=True)
    assert res.status == G.OK, res.stats
    assert st["converged"] == 1 and st["kkt_max"] <= kkt
    w = res.w.cpu().numpy().astype(np.float64)
    oc = O.check(O.Matrix.of(P), P.y, P.loss, lam, w)
    assert oc.kkt <= kkt * (1 + 1e-6)
    assert st["objective"] == pytest.approx(oc.objective, rel=1e-12)
    gap_or, _ = O.duality_gap(O.Matrix.of(P), P.y, P.loss, lam, w)
    assert st["gap"] == pytest.approx(gap_or, rel=1e-6, abs=1e-12)
    assert oc.objective - ref.objective >= -1e-12 * abs(ref.objective)
    bound = 1e-6 if level == "tight" else 2e-4
    assert abs(oc.objective - ref.objective) <= bound * abs(ref.objective)
    z = res.z.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(z, oc.z, rtol=1e-6, atol=1e-6 * np.abs(oc.z).max())


def test_solve_lambda_above_max_is_zero(problems):
    P = problems["c1"]
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    lm = G.lambda_max(X, y, P.loss)
    res = G.solve(X, y, G.make_params(P.loss, lm * 1.000001, rule=G.SHOTGUN, select_size=64))
    assert res.status == G.OK and res.stats["epochs"] == 0
    assert torch.count_nonzero(res.w).item() == 0


def test_solve_edge_shapes():
    # empty columns, |J| larger than the live count, a ragged last window
    n, k = 50, 40
    rng = np.random.default_rng(0)
    rows, cols = [], []
    for j in range(0, k, 3):  # two thirds of the columns are empty
        r = rng.choice(n, size=rng.integers(1, 6), replace=False)
        rows += list(r)
        cols += [j] * r.size
    cp, ri, va = synth.coo_to_csc(n, k, np.array(rows), np.array(cols),
                                  rng.normal(size=len(rows)).astype(np.float32))
    yv = np.where(rng.random(n) < 0.5, 1.0, -1.0).astype(np.float32)
    X = G.Matrix.from_numpy(n, k, cp, ri, va)
    y = torch.as_tensor(yv, device=DEV)
    Xo = O.Matrix(n, k, cp, ri, va)
    lam = 0.05 * O.lambda_max(Xo, yv, O.LOGISTIC)
    ref = O.solve(Xo, yv, O.LOGISTIC, lam, O.CYCLIC, tol=1e-10, max_epochs=100000)
    for sel in (5, 13, 100):
        res = G.solve(X, y, G.make_params(O.LOGISTIC, lam, rule=G.SHOTGUN, select_size=sel,
                                          max_epochs=100000))
        assert res.status == G.OK
        assert abs(res.stats["objective"] - ref.objective) <= 1e-6 * ref.objective
    # all columns empty: nothing to do, w = 0 is optimal
    X0 = G.Matrix.from_numpy(n, k, np.zeros(k + 1, np.int64), np.zeros(0, np.int32),
                             np.zeros(0, np.float32))
    res = G.solve(X0, y, G.make_params(O.LOGISTIC, 0.01, rule=G.SHOTGUN, select_size=4))
    assert res.status == G.OK and torch.count_nonzero(res.w).item() == 0


def test_error_paths():
    P = synth.c1_ccd_logistic(scale=0.05)
    X = G.Matrix.of(P)
    ybad = torch.as_tensor(P.y * 0.5, device=DEV)
    with pytest.raises(G.GencdError) as e:
        G.solve(X, ybad, G.make_params(P.loss, 0.01, rule=G.SHOTGUN, select_size=8))
    assert e.value.status == -3
    # an invalid matrix is caught by device validation
    ri = P.row_idx.copy()
    ri[3] = P.n + 5
    Xb = G.Matrix.from_numpy(P.n, P.k, P.col_ptr, ri, P.val)
    y = torch.as_tensor(P.y, device=DEV)
    with pytest.raises(G.GencdError) as e:
        G.solve(Xb, y, G.make_params(P.loss, 0.01, rule=G.SHOTGUN, select_size=8,
                                     flags=G.VALIDATE_DEVICE))
    assert e.value.status == -2


@pytest.mark.parametrize("name,rule,kw", [("c2", G.SHOTGUN, dict(select_size=512)),
                                          ("c2", G.THREAD_GREEDY, dict(select_size=2048, block=16)),
    ("c1", G.TOP_GREEDY, dict(select_size=1024, block=64)),
    ("c2", G.TOP_GREEDY, dict(select_size=2048, block=256)),
                                          ("c4", G.SHOTGUN, dict(select_size=256))])
def test_graph_path_matches_plain(problems, optima, name, rule, kw):
    """The captured epoch is replayed once per epoch, with the eager FP64
    check and host synchronisations between replays; every replay must give
    the plain path's result (same objective and KKT level)."""
    _print_case("graph", name, rule, kw)
    P = problems[name]
    lam, ref = optima[name]
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    out = {}
    for flags in (0, G.USE_GRAPH, G.USE_GRAPH | G.EXACT_ACCUM):
        params = G.make_params(P.loss, lam, rule=rule, seed=3, tol=1e-8, max_epochs=20000,
                               flags=flags, **kw)
        res = G.solve(X, y, params)
        assert res.status == G.OK, res.stats
        out[flags] = res
    a, b = out[0], out[G.USE_GRAPH]
    assert b.stats["epochs"] > 3
    c = out[G.USE_GRAPH | G.EXACT_ACCUM]
    assert abs(c.stats["objective"] - ref.objective) <= 1e-6 * abs(ref.objective)
    assert abs(a.stats["objective"] - b.stats["objective"]) <= 1e-9 * abs(ref.objective)
    assert abs(b.stats["objective"] - ref.objective) <= 1e-6 * abs(ref.objective)
    assert b.stats["kkt_max"] <= 1e-8
