"""Batched regularisation path on the GPU against independent oracle solves."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1206_6409_amd import gencd as G
from paper_1206_6409_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def binary_problem():
    P = synth.c4_binary_path(scale=0.05)
    Xo = O.Matrix.of(P)
    lm = O.lambda_max(Xo, P.y, P.loss)
    return P, Xo, lm


@pytest.mark.parametrize("B,L,flags,stagger,every", [
    (16, 20, 0, 0, 1), (32, 12, 0, 0, 1), (64, 6, 0, 0, 1),
    (16, 20, G.FUSED, 0, 1), (64, 6, G.FUSED, 0, 1),
    (16, 20, G.USE_GRAPH, 0, 1), (64, 6, G.USE_GRAPH, 0, 1),
    (32, 12, G.FUSED | G.USE_GRAPH, 0, 1),
    # staggered admission (a lambda enters once its predecessor ran 3 epochs)
    # and the adaptive check interval
    (64, 20, G.USE_GRAPH, 3, 0), (16, 20, 0, 5, 0), (32, 12, G.FUSED, 2, 1),
    # the whole epoch in one launch of |J| workgroups
    (16, 20, G.FUSED | G.FUSED_EPOCH, 0, 1), (64, 6, G.FUSED | G.FUSED_EPOCH | G.USE_GRAPH, 0, 0),
    (32, 12, G.FUSED | G.FUSED_EPOCH | G.USE_GRAPH, 3, 0)])
def test_path_matches_independent_solves(binary_problem, B, L, flags, stagger, every):
    print("CASE path", B, L, flags, stagger, every, flush=True)
    P, Xo, lm = binary_problem
    lams = synth.lambda_grid(lm, count=L, ratio=0.1)
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    params = G.make_params(P.loss, 0.0, rule=G.SHOTGUN, select_size=256, seed=4, tol=1e-8,
                           max_epochs=20000, flags=flags, stagger=stagger, check_every=every)
    res = G.solve_path(X, y, params, lams, B=B)
    assert res.status == G.OK
    W = res.W.cpu().numpy().astype(np.float64)
    w_or = None  # the oracle's own warm-started chain along the path
    for t, lam in enumerate(lams):
        st = res.stats[t]
        assert st["converged"] == 1 and st["kkt_max"] <= 1e-8, (t, st)
        oc = O.check(Xo, P.y, P.loss, lam, W[t])
        assert oc.kkt <= 1e-8 * (1 + 1e-6)
        assert st["objective"] == pytest.approx(oc.objective, rel=1e-12)
        ref = O.solve(Xo, P.y, P.loss, lam, O.CYCLIC, tol=1e-11, max_epochs=500000, w0=w_or)
        w_or = ref.w
        assert abs(oc.objective - ref.objective) <= 1e-6 * abs(ref.objective), t


@pytest.mark.parametrize("B,L,flags,steps", [
    (16, 20, G.FUSED | G.FUSED_EPOCH, 50), (32, 12, 0, 20), (64, 6, G.FUSED | G.USE_GRAPH, 5),
    (16, 20, G.USE_GRAPH, 1), (64, 6, G.FUSED | G.FUSED_EPOCH | G.USE_GRAPH, 500)])
def test_path_improve_matches_independent_solves(binary_problem, B, L, flags, steps):
    """"Improve delta_j" (Algorithm 3, section 4.1) on every slot of the
    batched path: each lambda's result passes the oracle's KKT test and its
    objective is within 1e-6 of the oracle's own optimum."""
    print("CASE path improve", B, L, flags, steps, flush=True)
    P, Xo, lm = binary_problem
    lams = synth.lambda_grid(lm, count=L, ratio=0.1)
    params = G.make_params(P.loss, 0.0, rule=G.SHOTGUN, select_size=256, seed=4, tol=1e-8,
                           max_epochs=20000, flags=flags, improve=steps)
    res = G.solve_path(G.Matrix.of(P), torch.as_tensor(P.y, device=DEV), params, lams, B=B)
    assert res.status == G.OK
    W = res.W.cpu().numpy().astype(np.float64)
    w_or = None
    for t, lam in enumerate(lams):
        st = res.stats[t]
        assert st["converged"] == 1 and st["kkt_max"] <= 1e-8, (t, st)
        oc = O.check(Xo, P.y, P.loss, lam, W[t])
        assert oc.kkt <= 1e-8 * (1 + 1e-6)
        assert st["objective"] == pytest.approx(oc.objective, rel=1e-12)
        ref = O.solve(Xo, P.y, P.loss, lam, O.CYCLIC, tol=1e-11, max_epochs=500000, w0=w_or)
        w_or = ref.w
        assert abs(oc.objective - ref.objective) <= 1e-6 * abs(ref.objective), t


def test_path_improve_single_lambda_equals_solve(binary_problem):
    """One lambda with improve steps: the batched path and gencd_solve (the
    same Jacobi windows, the improvement from the state at the window's
    start) reach the same objective."""
    P, Xo, lm = binary_problem
    lam = 0.05 * lm
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    kw = dict(rule=G.SHOTGUN, select_size=256, seed=4, tol=1e-8, max_epochs=20000, improve=20)
    single = G.solve(X, y, G.make_params(P.loss, lam, **kw))
    path = G.solve_path(X, y, G.make_params(P.loss, 0.0, **kw), [lam], B=16)
    assert single.status == G.OK and path.status == G.OK
    assert path.stats[0]["converged"] == 1
    assert abs(path.stats[0]["objective"] - single.stats["objective"]) <= 1e-7 * single.stats["objective"]


def test_path_improve_takes_fewer_epochs(binary_problem):
    """At the small lambdas of the logistic path the quadratic bound's step
    is far shorter than the coordinate minimiser's; improving each increment
    cuts the epochs to a tight KKT tolerance (the reason the paper offers the
    option): without it, three times the epochs the improved solve needed
    leave some lambda unconverged."""
    P, Xo, lm = binary_problem
    lams = synth.lambda_grid(lm, count=64, ratio=1e-3)[60:]
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)

    def run(steps, max_epochs):
        params = G.make_params(P.loss, 0.0, rule=G.SHOTGUN, select_size=256, seed=4, tol=1e-8,
                               max_epochs=max_epochs, improve=steps)
        return G.solve_path(X, y, params, lams, B=16)

    imp = run(50, 100000)
    assert imp.status == G.OK and all(st["converged"] for st in imp.stats)
    e50 = max(st["epochs"] for st in imp.stats)
    plain = run(0, 3 * e50)
    assert plain.status == G.NOT_CONVERGED, e50
    assert not all(st["converged"] for st in plain.stats)


def test_path_single_lambda_equals_solve(binary_problem):
    P, Xo, lm = binary_problem
    lam = 0.1 * lm
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    params = G.make_params(P.loss, lam, rule=G.SHOTGUN, select_size=256, seed=4, tol=1e-8,
                           max_epochs=20000)
    single = G.solve(X, y, params)
    path = G.solve_path(X, y, G.make_params(P.loss, 0.0, rule=G.SHOTGUN, select_size=256, seed=4,
                                            tol=1e-8, max_epochs=20000), [lam], B=16)
    assert path.status == G.OK
    assert abs(path.stats[0]["objective"] - single.stats["objective"]) <= 1e-7 * single.stats["objective"]


def test_path_rejects_bad_args(binary_problem):
    P, Xo, lm = binary_problem
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    with pytest.raises(G.GencdError):
        G.solve_path(X, y, G.make_params(P.loss, 0.0, rule=G.THREAD_GREEDY, select_size=64, block=8),
                     [0.1 * lm], B=16)
    with pytest.raises(G.GencdError):
        G.solve_path(X, y, G.make_params(P.loss, 0.0, rule=G.SHOTGUN, select_size=64), [0.1 * lm], B=24)
    with pytest.raises(G.GencdError) as e:  # one launch per epoch only in the fused form
        G.solve_path(X, y, G.make_params(P.loss, 0.0, rule=G.SHOTGUN, select_size=64,
                                         flags=G.FUSED_EPOCH), [0.1 * lm], B=16)
    assert e.value.status == G.ERR_UNSUPPORTED
    for steps in (-1, 1000001):
        with pytest.raises(G.GencdError) as e:
            G.solve_path(X, y, G.make_params(P.loss, 0.0, rule=G.SHOTGUN, select_size=64,
                                             improve=steps), [0.1 * lm], B=16)
        assert e.value.status == G.ERR_INVALID_ARG


@pytest.mark.parametrize("loss,B,flags", [(synth.SQUARED, 32, G.USE_GRAPH), (synth.SQUARED, 64, 0),
                                          (synth.LOGISTIC, 16, G.USE_GRAPH)])
def test_path_check_statistics_match_oracle(loss, B, flags):
    """Every per-slot statistic of the batched FP64 check (objective, KKT,
    duality gap, nnz(w)) against the oracle evaluated at the returned w."""
    print("CASE path check stats", loss, B, flags, flush=True)
    P = synth.make_bernoulli_problem(1500, 4000, 0.004, loss, seed=31, support=30)
    Xo = O.Matrix.of(P)
    lm = O.lambda_max(Xo, P.y, P.loss)
    lams = synth.lambda_grid(lm, count=B + 5, ratio=0.05)
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    params = G.make_params(P.loss, 0.0, rule=G.SHOTGUN, select_size=128, seed=2, tol=1e-7,
                           max_epochs=20000, flags=flags)
    res = G.solve_path(X, y, params, lams, B=B, want_z=True)
    assert res.status == G.OK
    W = res.W.cpu().numpy().astype(np.float64)
    Z = res.Z.cpu().numpy().astype(np.float64)
    for t, lam in enumerate(lams):
        st = res.stats[t]
        oc = O.check(Xo, P.y, P.loss, lam, W[t])
        # Z[t] = X W[t]: the FP32 rounding of an FP64 product (summation order differs)
        scale = np.abs(oc.z) + np.sqrt(np.mean(oc.z ** 2)) + 1e-300
        assert np.max(np.abs(Z[t] - oc.z) / scale) <= 1e-6, t
        gap, prim = O.duality_gap(Xo, P.y, P.loss, lam, W[t])
        assert st["objective"] == pytest.approx(oc.objective, rel=1e-12), t
        assert st["kkt_max"] == pytest.approx(oc.kkt, rel=1e-9, abs=1e-15), t
        assert st["gap"] == pytest.approx(gap, rel=1e-6, abs=1e-12 * abs(prim)), t
        assert st["nnz_w"] == int(np.count_nonzero(W[t])), t


@pytest.mark.parametrize("flags", [G.FUSED | G.FUSED_EPOCH, G.FUSED, 0])
def test_path_profile_events(binary_problem, flags):
    """GENCD_PROFILE on the batched path: HIP events around every fused (or
    Propose and Update) launch, totals in stats[0]; one fused launch per
    epoch covers every live column, so its bytes per launch are exactly the
    stated count."""
    print("CASE path profile", flags, flush=True)
    P, Xo, lm = binary_problem
    lams = synth.lambda_grid(lm, count=6, ratio=0.1)
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    B = 16
    base = G.make_params(P.loss, 0.0, rule=G.SHOTGUN, select_size=256, seed=4, tol=1e-7,
                         max_epochs=20000, flags=flags)
    ref = G.solve_path(X, y, base, lams, B=B)
    res = G.solve_path(X, y, G.make_params(P.loss, 0.0, rule=G.SHOTGUN, select_size=256, seed=4,
                                           tol=1e-7, max_epochs=20000, flags=flags | G.PROFILE),
                       lams, B=B)
    assert res.status == G.OK
    for a, b in zip(ref.stats, res.stats):
        assert abs(a["objective"] - b["objective"]) <= 1e-6 * abs(a["objective"])
    s0 = res.stats[0]
    epochs = max(s["epochs"] for s in res.stats)
    assert s0["prof_launches"] >= epochs and s0["prof_kernel_ms"] > 0.0
    k_live = int(np.count_nonzero(np.diff(P.col_ptr)))
    if flags & G.FUSED_EPOCH:
        per = P.nnz * (12 + 16 * B) + k_live * (20 + 8 * B)
        assert s0["prof_bytes"] == pytest.approx(s0["prof_launches"] * per, rel=1e-9)
        assert s0["prof_update_launches"] == 0
    elif flags & G.FUSED:
        assert s0["prof_update_launches"] == 0
    else:
        assert s0["prof_update_launches"] == s0["prof_launches"] and s0["prof_update_ms"] > 0.0
    for s in res.stats[1:]:
        assert s["prof_launches"] == 0
