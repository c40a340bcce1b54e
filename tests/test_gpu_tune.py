"""Autotuner: picks a valid schedule, caches it, and the schedule solves correctly."""
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_1206_6409_amd import gencd as G
from paper_1206_6409_amd import synth

pytestmark = pytest.mark.gpu


def test_autotune_cache_and_correctness(tmp_path):
    P = synth.c2_zipf_logistic(scale=0.02)
    Xo = O.Matrix.of(P)
    lam = 0.05 * O.lambda_max(Xo, P.y, P.loss)
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device="cuda")
    params = G.make_params(P.loss, lam, rule=G.SHOTGUN, select_size=512, seed=2, tol=1e-8,
                           max_epochs=20000)
    cache = str(tmp_path / "tune.jsonl")
    s1 = G.autotune(X, y, params, epochs=3, cache_path=cache)
    assert s1["group"] in (4, 8, 16) and s1["piece"] in (128, 256, 512) and s1["residual"] in (1, 2)
    assert s1["from_cache"] == 0 and s1["seconds_per_epoch"] > 0
    assert os.path.getsize(cache) > 0
    s2 = G.autotune(X, y, params, epochs=3, cache_path=cache)
    assert s2["from_cache"] == 1
    assert (s2["group"], s2["piece"], s2["flags"], s2["residual"]) == \
        (s1["group"], s1["piece"], s1["flags"], s1["residual"])
    res = G.solve(X, y, G.apply_schedule(params, s1))
    assert res.status == G.OK
    ref = O.solve(Xo, P.y, P.loss, lam, O.CYCLIC, tol=1e-11, max_epochs=500000)
    assert abs(res.stats["objective"] - ref.objective) <= 1e-6 * ref.objective
    # a different problem signature is not answered from the cache
    P2 = synth.c2_zipf_logistic(scale=0.01)
    X2 = G.Matrix.of(P2)
    s3 = G.autotune(X2, torch.as_tensor(P2.y, device="cuda"), params, epochs=2, cache_path=cache)
    assert s3["from_cache"] == 0


@pytest.mark.parametrize("group,piece", [(4, 256), (8, 512), (16, 1024), (32, 64), (8, 128)])
def test_every_tunable_schedule_is_correct(group, piece):
    P = synth.c2_zipf_logistic(scale=0.02)
    Xo = O.Matrix.of(P)
    lam = 0.05 * O.lambda_max(Xo, P.y, P.loss)
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device="cuda")
    for flags in (0, G.USE_GRAPH):
        params = G.make_params(P.loss, lam, rule=G.SHOTGUN, select_size=512, seed=2, tol=1e-8,
                               max_epochs=20000, group=group, piece=piece, flags=flags)
        res = G.solve(X, y, params)
        assert res.status == G.OK
        oc = O.check(Xo, P.y, P.loss, lam, res.w.cpu().numpy().astype(np.float64))
        assert oc.kkt <= 1e-8 * (1 + 1e-6)


def test_path_autotune_picks_a_candidate_and_caches(tmp_path):
    P = synth.c4_binary_path(scale=0.05)
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device="cuda")
    lm = G.lambda_max(X, y, P.loss)
    lams = synth.lambda_grid(lm, count=12, ratio=0.1)
    params = G.make_params(P.loss, 0.0, rule=G.SHOTGUN, select_size=256, seed=4, tol=1e-6,
                           max_epochs=20000)
    cache = str(tmp_path / "tune.jsonl")
    s1 = G.autotune_path(X, y, params, lams, cache_path=cache)
    assert s1["B"] in (16, 32, 64) and s1["flags"] in (0, G.FUSED, G.FUSED | G.FUSED_EPOCH) and s1["from_cache"] == 0
    s2 = G.autotune_path(X, y, params, lams, cache_path=cache)
    assert s2["from_cache"] == 1 and (s2["B"], s2["flags"]) == (s1["B"], s1["flags"])
    # the chosen schedule solves the path
    params.flags |= s1["flags"]
    res = G.solve_path(X, y, params, lams, B=s1["B"])
    assert res.status == G.OK
