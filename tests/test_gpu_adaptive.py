"""Adaptive FP64 check interval (check_every = 0): the stopping rule is the
same KKT test, evaluated at epochs spaced by a tenth of the epochs run, so
the solve ends at most about 10% (plus one epoch) after the first epoch at
which a per-epoch check would have stopped it; check_every = -m spaces them
by an m-th (at most about 1/m later)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1206_6409_amd import gencd as G
from paper_1206_6409_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.mark.parametrize("loss,flags", [(synth.LOGISTIC, 0), (synth.SQUARED, G.USE_GRAPH),
                                        (synth.LOGISTIC, G.FUSED)])
def test_adaptive_checks_stop_on_the_same_test(loss, flags):
    print("CASE adaptive checks", loss, flags, flush=True)
    P = synth.make_bernoulli_problem(2500, 6000, 0.004, loss, seed=61, support=30)
    Xo = O.Matrix.of(P)
    lam = 0.02 * O.lambda_max(Xo, P.y, P.loss)
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    ref = O.solve(Xo, P.y, P.loss, lam, O.CYCLIC, tol=1e-11, max_epochs=500000)
    res = {}
    for every in (1, 0, -3):
        prm = G.make_params(P.loss, lam, rule=G.SHOTGUN, select_size=256, seed=3, tol=1e-8,
                            max_epochs=100000, check_every=every, flags=flags)
        r = G.solve(X, y, prm)
        assert r.status == G.OK
        chk = O.check(Xo, P.y, P.loss, lam, r.w.double().cpu().numpy())
        assert chk.kkt <= 1e-8 * (1 + 1e-6)
        assert abs(chk.objective - ref.objective) <= 1e-6 * abs(ref.objective)
        res[every] = r.stats["epochs"]
    print("epochs: every epoch", res[1], "adaptive", res[0], "a third", res[-3], flush=True)
    assert res[0] <= 1.1 * res[1] + 2
    assert res[-3] <= 1.34 * res[1] + 2


def test_check_every_below_minus_1000_is_rejected():
    P = synth.make_bernoulli_problem(300, 500, 0.02, synth.SQUARED, seed=62, support=5)
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device=DEV)
    with pytest.raises(G.GencdError) as e:
        G.solve(X, y, G.make_params(P.loss, 0.1, rule=G.SHOTGUN, select_size=16,
                                    check_every=-1001))
    assert e.value.status == G.ERR_INVALID_ARG
