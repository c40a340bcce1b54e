"""Seeded synthetic inputs for l1-regularised regression (Eq. 1 of the paper).

This module only draws data.  It contains none of the coordinate-descent
arithmetic (no gradients, no lambda_max, no steps): both the HIP library and
the FP64 oracle consume what it returns, and each side derives everything else
on its own.

Every matrix is returned as CSC with ``col_ptr`` int64[k+1], ``row_idx``
int32[nnz] (rows sorted and unique within a column) and ``val`` float32[nnz].
Labels ``y`` are float32 (logistic labels are exactly -1.0 / +1.0).

The shapes stand in for the paper's two datasets (section 4.4), which are not
available: ``zipf_rows`` is tf-idf-like (heavy-tailed column counts, like the
Reuters text data), ``bernoulli_csc`` with binary values is DOROTHEA-like.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SQUARED = 0
LOGISTIC = 1


@dataclass
class Problem:
    n: int
    k: int
    col_ptr: np.ndarray  # int64[k+1]
    row_idx: np.ndarray  # int32[nnz]
    val: np.ndarray      # float32[nnz]
    y: np.ndarray        # float32[n]
    loss: int
    w_true: np.ndarray = field(default=None)  # float64[k], the generating weights
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col_ptr[-1])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def coo_to_csc(n: int, k: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    """Sort (row, col, val) triplets into CSC.  Duplicate (row, col) pairs are an error."""
    key = cols.astype(np.int64) * n + rows.astype(np.int64)
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size > 1 and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate (row, col) entries")
    cols_s = cols[order]
    counts = np.bincount(cols_s, minlength=k).astype(np.int64)
    col_ptr = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(counts, out=col_ptr[1:])
    return col_ptr, rows[order].astype(np.int32), vals[order].astype(np.float32)


def _uniform_positions(rng: np.random.Generator, total_cells: int, m: int) -> np.ndarray:
    """m distinct uniform integers from [0, total_cells), sorted."""
    if m == 0:
        return np.zeros(0, dtype=np.int64)
    got = np.zeros(0, dtype=np.int64)
    while got.size < m:
        extra = int((m - got.size) * 1.02) + 64
        got = np.unique(np.concatenate([got, rng.integers(0, total_cells, size=extra, dtype=np.int64)]))
    if got.size > m:
        keep = np.sort(rng.choice(got.size, size=m, replace=False))
        got = got[keep]
    return got


def bernoulli_pattern(rng: np.random.Generator, n: int, k: int, density: float):
    """Entries present independently with probability ``density``.

    Drawn as a Binomial total followed by a uniform set of that many distinct
    cells, which has the same law as independent Bernoulli entries.
    Returns (rows, cols) in CSC order.
    """
    total = int(rng.binomial(n * k, density))
    pos = _uniform_positions(rng, n * k, total)
    cols = (pos // n).astype(np.int64)
    rows = (pos % n).astype(np.int64)
    return rows, cols


def _zipf_cdf(k: int, a: float) -> np.ndarray:
    p = np.arange(1, k + 1, dtype=np.float64) ** (-a)
    c = np.cumsum(p)
    return c / c[-1]


def zipf_rows(rng: np.random.Generator, n: int, k: int, a: float, mean_len: int):
    """Rows of length 1 + Poisson(mean_len - 1); each row holds distinct column
    ranks drawn from Zipf(a) truncated to [1, k] (repeats rejected and
    redrawn); ranks map to columns through a seeded permutation."""
    lens = 1 + rng.poisson(mean_len - 1, size=n).astype(np.int64)
    lens = np.minimum(lens, k)
    cdf = _zipf_cdf(k, a)
    rank_to_col = rng.permutation(k).astype(np.int64)
    have = np.zeros(0, dtype=np.int64)  # sorted distinct keys row * k + rank
    deficit = lens.copy()
    while True:
        need = int(deficit.sum())
        if need == 0:
            break
        r = np.repeat(np.arange(n, dtype=np.int64), deficit)
        u = rng.random(need)
        rank = np.searchsorted(cdf, u, side="right").astype(np.int64)
        rank = np.minimum(rank, k - 1)
        new = np.unique(r * k + rank)
        if have.size:
            at = np.minimum(np.searchsorted(have, new), have.size - 1)
            new = new[have[at] != new]
        # two sorted runs: the stable sort merges them in linear time
        have = np.sort(np.concatenate([have, new]), kind="stable")
        cnt = np.bincount(new // k, minlength=n).astype(np.int64)
        deficit = deficit - cnt
    rows = have // k
    cols = rank_to_col[have % k]
    return rows, cols


def _row_normalise(n: int, rows: np.ndarray, vals: np.ndarray) -> np.ndarray:
    ss = np.bincount(rows, weights=vals.astype(np.float64) ** 2, minlength=n)
    nrm = np.sqrt(ss)
    nrm[nrm == 0] = 1.0
    return vals.astype(np.float64) / nrm[rows]


def _pick_support(rng, col_ptr, count):
    nonempty = np.nonzero(np.diff(col_ptr) > 0)[0]
    count = min(count, nonempty.size)
    return np.sort(rng.choice(nonempty, size=count, replace=False))


def _xw(n, col_ptr, row_idx, val, w):
    """X @ w in FP64 for generating responses (data synthesis only)."""
    z = np.zeros(n, dtype=np.float64)
    nzc = np.nonzero(w)[0]
    for j in nzc:
        a, b = col_ptr[j], col_ptr[j + 1]
        z[row_idx[a:b]] += w[j] * val[a:b].astype(np.float64)
    return z


def _logistic_labels(rng, z):
    p = 1.0 / (1.0 + np.exp(-z))
    return np.where(rng.random(z.size) < p, 1.0, -1.0).astype(np.float32)


def make_bernoulli_problem(n, k, density, loss, seed, support=50, binary=False,
                           noise_sd=0.1, name=""):
    rng = _rng(seed)
    rows, cols = bernoulli_pattern(rng, n, k, density)
    if binary:
        vals = np.ones(rows.size, dtype=np.float32)
    else:
        vals = rng.standard_normal(rows.size).astype(np.float32)
    col_ptr, row_idx, val = coo_to_csc(n, k, rows, cols, vals)
    w = np.zeros(k)
    sup = _pick_support(rng, col_ptr, support)
    w[sup] = rng.standard_normal(sup.size)
    z = _xw(n, col_ptr, row_idx, val, w)
    if loss == LOGISTIC:
        y = _logistic_labels(rng, z)
    else:
        y = (z + noise_sd * rng.standard_normal(n)).astype(np.float32)
    return Problem(n, k, col_ptr, row_idx, val, y, loss, w, name)


def make_zipf_problem(n, k, a, mean_len, loss, seed, support, values="lognormal",
                      row_normalise=True, noise_sd=0.1, name=""):
    rng = _rng(seed)
    rows, cols = zipf_rows(rng, n, k, a, mean_len)
    if values == "lognormal":
        vals = np.exp(rng.standard_normal(rows.size))
    else:
        vals = rng.standard_normal(rows.size)
    if row_normalise:
        vals = _row_normalise(n, rows, vals)
    col_ptr, row_idx, val = coo_to_csc(n, k, rows, cols, vals.astype(np.float32))
    w = np.zeros(k)
    sup = _pick_support(rng, col_ptr, support)
    w[sup] = rng.standard_normal(sup.size)
    z = _xw(n, col_ptr, row_idx, val, w)
    if loss == LOGISTIC:
        y = _logistic_labels(rng, z)
    else:
        y = (z + noise_sd * rng.standard_normal(n)).astype(np.float32)
    return Problem(n, k, col_ptr, row_idx, val, y, loss, w, name)


# ---------------------------------------------------------------------------
# The five workloads.  ``scale`` < 1 shrinks n and k proportionally (same
# densities / row lengths) for tests that the CPU oracle must finish quickly.
# ---------------------------------------------------------------------------

def c1_ccd_logistic(scale=1.0, seed=101):
    """Cyclic CD workload: n=2000, k=5000, density 1%, N(0,1) values,
    logistic labels from a 50-sparse w*; solved at 0.1*lambda_max."""
    n, k = max(8, int(2000 * scale)), max(8, int(5000 * scale))
    return make_bernoulli_problem(n, k, 0.01, LOGISTIC, seed, support=50,
                                  name=f"ccd-logistic n={n} k={k} d=1%")


def c2_zipf_logistic(scale=1.0, seed=102):
    """Shotgun / Thread-Greedy workload: n=1e5, k=5e5, Zipf(1.1) column
    popularity, ~50 nnz per row, lognormal values, rows L2-normalised,
    logistic labels from a 500-sparse w*; solved at 0.05*lambda_max."""
    n, k = max(16, int(100_000 * scale)), max(16, int(500_000 * scale))
    return make_zipf_problem(n, k, 1.1, 50, LOGISTIC, seed, support=500,
                             values="lognormal", row_normalise=True,
                             name=f"zipf1.1-logistic n={n} k={k}")


def c3_zipf_lasso(scale=1.0, seed=103):
    """Coloring workload: n=2e5, k=1e6, Zipf(1.2), ~30 nnz per row, N(0,1)
    values, y = X w* + N(0, 0.01) with 1000-sparse w*; 0.1*lambda_max."""
    n, k = max(16, int(200_000 * scale)), max(16, int(1_000_000 * scale))
    return make_zipf_problem(n, k, 1.2, 30, SQUARED, seed, support=1000,
                             values="normal", row_normalise=False, noise_sd=0.1,
                             name=f"zipf1.2-lasso n={n} k={k}")


def c4_binary_path(scale=1.0, seed=104):
    """Regularisation-path workload: n=5e4, k=2e5, density 0.05%, binary
    values, logistic labels from a 200-sparse w*; 64 lambdas."""
    n, k = max(16, int(50_000 * scale)), max(16, int(200_000 * scale))
    return make_bernoulli_problem(n, k, 5e-4, LOGISTIC, seed, support=200, binary=True,
                                  name=f"binary-path n={n} k={k} d=0.05%")


def lambda_grid(lam_max: float, count: int = 64, ratio: float = 1e-3) -> np.ndarray:
    """Geometric grid from lam_max down to ratio*lam_max (decreasing)."""
    t = np.arange(count, dtype=np.float64)
    return lam_max * ratio ** (t / max(count - 1, 1))


@dataclass
class Request:
    ticket: int
    arrival: float
    loss: int
    n: int
    k: int
    density: float
    lambda_ratio: float
    seed: int


def c5_request_stream(count=2000, rate=1.0, seed=105, arrival_seed=1050,
                      n_range=(1000, 50000), k_range=(1000, 200000),
                      d_range=(0.001, 0.02), ratio_range=(1e-3, 0.5)):
    """Serving workload: Poisson arrivals; per request loss ~ Bernoulli(1/2),
    n ~ U{n_range}, k ~ U{k_range}, density ~ U[d_range], lambda/lambda_max
    log-uniform over ratio_range."""
    rng = _rng(seed)
    arng = _rng(arrival_seed)
    gaps = arng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        loss = int(rng.integers(0, 2))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        d = float(rng.uniform(d_range[0], d_range[1]))
        lr = float(np.exp(rng.uniform(np.log(ratio_range[0]), np.log(ratio_range[1]))))
        out.append(Request(i, float(t[i]), loss, n, k, d, lr, int(rng.integers(0, 2**62))))
    return out


def request_problem(req: Request, support=50):
    """Materialise one serving request on the host."""
    return make_bernoulli_problem(req.n, req.k, req.density, req.loss, req.seed,
                                  support=support, name=f"request {req.ticket}")


# ---------------------------------------------------------------------------
# Small structured matrices used by tests.
# ---------------------------------------------------------------------------

def orthogonal_design(n, k, loss, seed):
    """One nonzero per row, every column non-empty when n >= k: columns have
    disjoint supports."""
    rng = _rng(seed)
    cols = np.concatenate([np.arange(k), rng.integers(0, k, size=n - k)]) if n >= k else rng.integers(0, k, size=n)
    rows = np.arange(n)
    vals = rng.standard_normal(n).astype(np.float32)
    vals[vals == 0] = 1.0
    col_ptr, row_idx, val = coo_to_csc(n, k, rows, cols, vals)
    w = np.zeros(k)
    w[rng.choice(k, size=min(k, 3), replace=False)] = rng.standard_normal(min(k, 3)) * 2
    z = _xw(n, col_ptr, row_idx, val, w)
    if loss == LOGISTIC:
        y = _logistic_labels(rng, z)
    else:
        y = (z + 0.1 * rng.standard_normal(n)).astype(np.float32)
    return Problem(n, k, col_ptr, row_idx, val, y, loss, w, "orthogonal")


def dense_small(n, k, loss, seed, density=1.0):
    """Small (possibly dense) problem for brute-force checks."""
    return make_bernoulli_problem(n, k, density, loss, seed, support=max(1, k // 2),
                                  name=f"small n={n} k={k}")
