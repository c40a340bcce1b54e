"""The continuous-batching server on the GPU: every result equals the same
solve run alone (objective within 1e-6 of it and of the oracle), under
concurrency, backpressure and failures."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1206_6409_amd import gencd as G
from paper_1206_6409_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _requests(count, seed):
    stream = synth.c5_request_stream(count=count, rate=100.0, seed=seed, n_range=(400, 3000),
                                     k_range=(400, 6000), d_range=(0.005, 0.02),
                                     ratio_range=(0.05, 0.5))
    out = []
    for r in stream:
        P = synth.request_problem(r, support=20)
        Xo = O.Matrix.of(P)
        lam = r.lambda_ratio * O.lambda_max(Xo, P.y, P.loss)
        out.append((r, P, Xo, lam))
    return out


def _params(P, lam, flags=0):
    return G.make_params(P.loss, lam, rule=G.SHOTGUN, select_size=256, seed=9, tol=1e-8,
                         max_epochs=50000, flags=flags)


@pytest.fixture(scope="module")
def reqs():
    return _requests(14, 55)


def test_server_results_equal_alone(reqs):
    dev = []
    for r, P, Xo, lam in reqs:
        X = G.Matrix.of(P)
        y = torch.as_tensor(P.y, device=DEV)
        dev.append((X, y))
    alone = []
    for (r, P, Xo, lam), (X, y) in zip(reqs, dev):
        res = G.solve(X, y, _params(P, lam))
        assert res.status == G.OK
        alone.append(res.stats["objective"])
    biggest = max(G.workspace_bytes(X, _params(P, lam)) for (r, P, Xo, lam), (X, y) in zip(reqs, dev))
    srv = G.Server(arena_bytes=3 * biggest + (1 << 20), max_slots=4)
    ws = []
    for i, ((r, P, Xo, lam), (X, y)) in enumerate(zip(reqs, dev)):
        w = torch.empty(P.k, dtype=torch.float32, device=DEV)
        ws.append(w)
        srv.submit(X, y, _params(P, lam), w, tag=i)
    results = []
    while len(results) < len(reqs):
        results += srv.poll(wait_for=1)
    srv.close()
    assert sorted(r["user_tag"] for r in results) == list(range(len(reqs)))
    overlap = False
    for res in results:
        i = res["user_tag"]
        r, P, Xo, lam = reqs[i]
        assert res["status"] == G.OK, res
        st = res["stats"]
        assert st["kkt_max"] <= 1e-8
        assert abs(st["objective"] - alone[i]) <= 1e-6 * abs(alone[i])
        oc = O.check(Xo, P.y, P.loss, lam, ws[i].cpu().numpy().astype(np.float64))
        assert oc.kkt <= 1e-8 * (1 + 1e-6)
        assert res["start_s"] >= res["submit_s"] and res["finish_s"] >= res["start_s"]
    # several requests ran at the same time
    iv = sorted((r["start_s"], r["finish_s"]) for r in results)
    overlap = any(b[0] < a[1] for a, b in zip(iv[:-1], iv[1:]))
    assert overlap


def test_server_backpressure_and_failures(reqs):
    r0, P0, Xo0, lam0 = reqs[0]
    X = G.Matrix.of(P0)
    y = torch.as_tensor(P0.y, device=DEV)
    need = G.workspace_bytes(X, _params(P0, lam0))
    # an arena for exactly one request at a time: requests are serialised
    srv = G.Server(arena_bytes=need + 4096, max_slots=4)
    ws = [torch.empty(P0.k, dtype=torch.float32, device=DEV) for _ in range(3)]
    for i in range(3):
        srv.submit(X, y, _params(P0, lam0), ws[i], tag=i)
    # a request larger than the arena is rejected at submit
    big = reqs[int(np.argmax([p.nnz + p.k + p.n for _, p, _, _ in reqs]))]
    Xb = G.Matrix.of(big[1])
    if G.workspace_bytes(Xb, _params(big[1], big[3])) > need + 4096:
        with pytest.raises(G.GencdError) as e:
            srv.submit(Xb, torch.as_tensor(big[1].y, device=DEV), _params(big[1], big[3]),
                       torch.empty(big[1].k, dtype=torch.float32, device=DEV))
        assert e.value.status == -8
    res = []
    while len(res) < 3:
        res += srv.poll(wait_for=1)
    srv.close()
    res.sort(key=lambda r: r["user_tag"])
    for a, b in zip(res[:-1], res[1:]):
        assert b["start_s"] >= a["finish_s"] - 1e-6  # one at a time
    for r in res:
        assert r["status"] == G.OK
    # a failing request fails alone
    srv = G.Server(arena_bytes=8 * need, max_slots=4)
    lg = [(p, xo, l) for (_, p, xo, l) in reqs if p.loss == G.LOGISTIC]
    Pl, _, laml = lg[0]
    Xl = G.Matrix.of(Pl)
    good = torch.as_tensor(Pl.y, device=DEV)
    bad = torch.as_tensor(Pl.y * 0.5, device=DEV)
    wg = torch.empty(Pl.k, dtype=torch.float32, device=DEV)
    wb = torch.empty(Pl.k, dtype=torch.float32, device=DEV)
    srv.submit(Xl, bad, _params(Pl, laml), wb, tag=1)
    srv.submit(Xl, good, _params(Pl, laml), wg, tag=2)
    out = []
    while len(out) < 2:
        out += srv.poll(wait_for=1)
    srv.close()
    st = {r["user_tag"]: r["status"] for r in out}
    assert st[1] == -3 and st[2] == G.OK
