"""Writes c4_path_optima.txt: the oracle's optimum of Eq. (1) for each of the
64 lambdas of the binary regularisation-path workload (n = 50,000,
k = 200,000, density 0.05 %, binary values, logistic loss; lambdas geometric
from lambda_max down to 1e-3 lambda_max, the decreasing path of section 4.1).

Only the FP64 oracle runs here: cyclic coordinate descent (section 2.1) whose
accepted increments are refined by up to 50 further quadratic-approximation
steps along their column (the "improve delta_j" option of section 4.1; the
optimum of Eq. (1) does not depend on the rule, and at the small lambdas the
refined steps reach a tight KKT level many times sooner than one bound-based
step per coordinate).  A first warm-started pass along the path solves each
lambda to KKT <= min(1e-6, lambda / 10); every lambda is then solved from that
point to FP64 KKT <= 1e-10, in parallel over lambdas.  Each row records the
KKT level and the l1 norm reached, so that a test can bound the objective
error of any other point a by convexity: |P(a) - P(b)| <= max(KKT(a),
KKT(b)) (|a|_1 + |b|_1).

Usage: python tests/golden/make_c4_path_optima.py [--workers 6]
"""
import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1206_6409_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "c4_path_optima.txt")
TOL = 1e-10
IMPROVE = 50
MAX_EPOCHS = 20000

_G = {}


def _problem():
    if "P" not in _G:
        P = synth.c4_binary_path()
        _G["P"] = P
        _G["X"] = O.Matrix.of(P)
        _G["y"] = P.y.astype(np.float64)
    return _G["P"], _G["X"], _G["y"]


def _tight(args):
    t, lam, w0 = args
    P, X, y = _problem()
    t0 = time.time()
    r = O.solve(X, y, P.loss, float(lam), O.CYCLIC, tol=TOL, max_epochs=MAX_EPOCHS, w0=w0,
                check_every=5, improve=IMPROVE)
    return (t, float(lam), r.objective, r.kkt, int(r.nnz_w), float(np.abs(r.w).sum()), r.epochs,
            bool(r.converged), time.time() - t0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    args = ap.parse_args()
    print("starting points: warm-started pass to KKT min(1e-6, lambda/10)", flush=True)
    P, X, y = _problem()
    lm = O.lambda_max(X, y, P.loss)
    lams = synth.lambda_grid(lm, count=64, ratio=1e-3)
    starts, w0 = [], None
    for t, lam in enumerate(lams):  # warm-started pass: starting points only
        t0 = time.time()
        r = O.solve(X, y, P.loss, float(lam), O.CYCLIC, tol=min(1e-6, 0.1 * float(lam)),
                    max_epochs=MAX_EPOCHS, w0=w0, check_every=5, improve=IMPROVE)
        w0 = r.w
        starts.append(r.w.copy())
        print(f"start {t:2d}: kkt {r.kkt:.2e} epochs {r.epochs} ({time.time() - t0:.0f} s)",
              flush=True)
    jobs = [(t, lams[t], starts[t]) for t in range(len(lams))]
    jobs.sort(key=lambda j: -j[0])  # the slow small lambdas first
    rows = []
    with mp.Pool(args.workers) as pool:
        for row in pool.imap_unordered(_tight, jobs):
            rows.append(row)
            print(f"lambda {row[0]:2d}: objective {row[2]:.15e} kkt {row[3]:.2e} "
                  f"epochs {row[6]} ({row[8]:.0f} s)", flush=True)
    rows.sort()
    with open(OUT, "w") as f:
        f.write("# Oracle optima of Eq. (1) on the binary regularisation-path workload\n")
        f.write(f"# (synth.c4_binary_path(), seed 104: n={P.n} k={P.k} nnz={P.nnz}, logistic),\n")
        f.write(f"# lambda_t = lambda_max * 1e-3^(t/63), lambda_max = {lm!r}.\n")
        f.write("# Written by tests/golden/make_c4_path_optima.py: FP64 oracle, cyclic CD to\n")
        f.write(f"# KKT <= {TOL:g} (improve {IMPROVE}, at most {MAX_EPOCHS} epochs) from a\n")
        f.write("# warm-started pass to KKT <= min(1e-6, lambda/10) (section 4.1).\n")
        f.write("# t lambda objective kkt nnz_w l1_w epochs converged\n")
        for t, lam, obj, kkt, nz, l1, ep, conv, _ in rows:
            f.write(f"{t} {lam!r} {obj!r} {kkt:.6e} {nz} {l1!r} {ep} {int(conv)}\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
