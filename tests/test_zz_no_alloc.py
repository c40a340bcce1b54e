"""gencd_solve_noalloc (static device scratch instead of a caller workspace)
against gencd_solve on the same problems, two calls in a row on one
device, the second with a smaller problem; and its host-side size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
from paper_1206_6409_amd import gencd as G
from paper_1206_6409_amd import synth

DEV = "cuda"


def _solve_both(P, lam, rule, **kw):
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    prm = dict(rule=rule, seed=3, tol=1e-8, max_epochs=50000, **kw)
    ref = G.solve(X, y, G.make_params(P.loss, lam, **prm))
    got = G.solve_noalloc(X, y, G.make_params(P.loss, lam, **prm))
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.gpu
def test_noalloc_matches_solve_twice_shrinking():
    # first call: the larger problem; second call: a smaller one, so the
    # scratch still holds the first call's (larger) contents
    cases = [(synth.make_bernoulli_problem(3000, 9000, 0.003, synth.LOGISTIC, seed=71, support=40),
              G.SHOTGUN, dict(select_size=512)),
             (synth.make_bernoulli_problem(1200, 2500, 0.005, synth.SQUARED, seed=72, support=20),
              G.SHOTGUN, dict(select_size=128))]
    for P, rule, kw in cases:
        print("CASE noalloc", P.name, flush=True)
        Xo = O.Matrix.of(P)
        lam = 0.1 * O.lambda_max(Xo, P.y, P.loss)
        ref, got = _solve_both(P, lam, rule, **kw)
        assert ref.status == G.OK and got.status == G.OK
        opt = O.solve(Xo, P.y, P.loss, lam, O.CYCLIC, tol=1e-11, max_epochs=500000)
        for r in (ref, got):
            assert r.stats["kkt_max"] <= 1e-8
            chk = O.check(Xo, P.y, P.loss, lam, r.w.double().cpu().numpy())
            assert chk.kkt <= 1e-8 * (1 + 1e-6)
            assert abs(chk.objective - opt.objective) <= 1e-6 * abs(opt.objective)
        assert abs(got.stats["objective"] - ref.stats["objective"]) <= 1e-7 * abs(ref.stats["objective"])
        z_ref = ref.z.double().cpu().numpy()
        z_got = got.z.double().cpu().numpy()
        scale = np.abs(z_ref) + np.sqrt(np.mean(z_ref ** 2))
        assert np.max(np.abs(z_got - z_ref) / scale) <= 1e-5


@pytest.mark.gpu
def test_noalloc_rejects_graph_and_profile_flags():
    P = synth.make_bernoulli_problem(500, 800, 0.01, synth.SQUARED, seed=73, support=10)
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    for fl in (G.USE_GRAPH, G.PROFILE):
        with pytest.raises(G.GencdError) as e:
            G.solve_noalloc(X, y, G.make_params(P.loss, 0.01, rule=G.SHOTGUN, select_size=64,
                                                flags=fl))
        assert e.value.status == G.ERR_UNSUPPORTED


def test_noalloc_rejects_problems_beyond_the_scratch():
    # host-only: the size check precedes any HIP call; pointers are never used
    X = G.Csc(100000, 500000, 5000000, 0x1000, 0x2000, 0x3000)
    p = G.make_params(G.LOGISTIC, 0.1, rule=G.SHOTGUN, select_size=4096)
    need = C.c_size_t()
    assert G.lib().gencd_workspace_bytes(C.byref(X), C.byref(p), C.byref(need)) == 0
    assert need.value > (64 << 20)
    w = C.c_void_p(0x4000)
    rc = G.lib().gencd_solve_noalloc(C.byref(X), C.c_void_p(0x5000), C.byref(p), w, None, None, None)
    assert rc == G.ERR_TOO_LARGE
    assert "static scratch" in G.status_string(rc)
