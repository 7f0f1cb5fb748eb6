"""Seeded generators of sparse irregular slices (inputs only, no method arithmetic).

Recipe (shapes follow the paper's synthetic experiment, Sec. "SPARTan is fast
and memory-efficient", Table "table:synthetic": one million subjects, five
thousand variables, at most one hundred observations per subject):

* every subject k gets I_k rows, drawn uniformly from an inclusive range;
* every row gets at least one nonzero (the paper's structured-sparsity premise,
  Sec. "Challenges of PARAFAC2 on sparse data": all rows of X_k are nonzero);
* the columns of a row are distinct and sorted (canonical CSR);
* columns are drawn either uniformly over J or from a bounded Zipf law over J
  (P(rank r) proportional to r^-s, r = 1..J, sampled by inverse CDF on the
  J-entry table) followed by a fixed seeded permutation of the column ids,
  so that the hot columns are not the low ids;
* values are 1 - U[0,1), i.e. in (0, 1], stored as float32.

Subjects are generated in chunks of CHUNK subjects; chunk c draws from child
c of SeedSequence([ROOT_SEED, cfg]).  The first n chunks of a configuration
therefore do not depend on K, which makes K-subsamples of the large
configurations bit-identical to the leading subjects of the full input.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Callable, Optional

import numpy as np

ROOT_SEED = 170304219
CHUNK = 10_000


@dataclasses.dataclass
class Slices:
    """K sparse slices X_k (I_k x J) in one concatenated CSR (0-based).

    Subject k owns rows [subj_ptr[k], subj_ptr[k+1]); row i owns nonzeros
    [row_ptr[i], row_ptr[i+1]).  Columns are strictly increasing in a row.
    """

    J: int
    subj_ptr: np.ndarray  # int64 [K+1]
    row_ptr: np.ndarray  # int64 [n_rows+1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float32 [nnz]

    @property
    def K(self) -> int:
        return int(self.subj_ptr.shape[0] - 1)

    @property
    def n_rows(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def I(self) -> np.ndarray:
        return np.diff(self.subj_ptr)


# ---------------------------------------------------------------------------
# samplers
# ---------------------------------------------------------------------------

def _zipf_table(J: int, s: float) -> np.ndarray:
    w = np.arange(1, J + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


def make_col_sampler(J: int, dist: str, zipf_s: float = 1.1, perm_seed=None):
    if dist == "uniform":
        def draw(rng, n):
            return rng.integers(0, J, size=n, dtype=np.int64)
        return draw
    if dist == "zipf":
        cdf = _zipf_table(J, zipf_s)
        perm = np.random.default_rng(perm_seed).permutation(J).astype(np.int64)

        def draw(rng, n):
            u = rng.random(n)
            r = np.searchsorted(cdf, u, side="right")
            np.minimum(r, J - 1, out=r)
            return perm[r]
        return draw
    raise ValueError(dist)


def _distinct_sorted_rows(rng, row_id: np.ndarray, J: int, draw) -> np.ndarray:
    """Draw one column per entry of row_id so that columns are distinct within a
    row (duplicates are redrawn), and return the columns sorted by (row, col)."""
    n = row_id.shape[0]
    cols = draw(rng, n)
    for _ in range(10_000):
        key = row_id * J + cols
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(n, dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            return (ks - row_id[order] * J).astype(np.int32)
        idx = order[dup]
        cols[idx] = draw(rng, idx.shape[0])
    raise RuntimeError("could not draw distinct columns")


def _gpu_runtime_started() -> bool:
    import sys
    torch = sys.modules.get("torch")
    try:
        return bool(torch is not None and torch.cuda.is_initialized())
    except Exception:
        return True


def _gen_chunk(args):
    """One chunk of subjects (runs in a worker process for large inputs)."""
    (child, nk, take, J, ik_range, nnz_row, col_dist, zipf_s, perm_seed, ik_draw, val_draw) = args
    draw = make_col_sampler(J, col_dist, zipf_s, perm_seed=perm_seed)
    rng = np.random.default_rng(child)
    if ik_draw is None:
        Ik = rng.integers(ik_range[0], ik_range[1] + 1, size=nk, dtype=np.int64)
    else:
        Ik = np.asarray(ik_draw(rng, nk), dtype=np.int64)
    nr = int(Ik.sum())
    rl = np.asarray(nnz_row(rng, nr), dtype=np.int64)
    np.clip(rl, 1, J, out=rl)
    row_id = np.repeat(np.arange(nr, dtype=np.int64), rl)
    cols = _distinct_sorted_rows(rng, row_id, J, draw)
    if val_draw is None:
        vals = (1.0 - rng.random(cols.shape[0])).astype(np.float32)
    else:
        vals = np.asarray(val_draw(rng, cols.shape[0]), dtype=np.float32)
    if take < nk:
        nr_t = int(Ik[:take].sum())
        nz_t = int(rl[:nr_t].sum())
        Ik, rl, cols, vals = Ik[:take], rl[:nr_t], cols[:nz_t], vals[:nz_t]
    return Ik, rl, cols, vals


def gen_slices(
    K: int,
    J: int,
    ik_range: tuple[int, int],
    nnz_row: Callable[[np.random.Generator, int], np.ndarray],
    col_dist: str,
    seed,
    zipf_s: float = 1.1,
    chunk: int = CHUNK,
    k_limit: Optional[int] = None,
    workers: Optional[int] = None,
    ik_draw=None,
    val_draw=None,
) -> Slices:
    """Generate K slices chunk by chunk.  seed is a sequence of ints; chunk c uses
    child c of SeedSequence(seed); the column permutation uses seed + [2].
    Chunks are independent, so large inputs are drawn by a process pool; the
    result does not depend on the number of workers."""
    seed = list(seed)
    n_chunks = (K + chunk - 1) // chunk
    children = np.random.SeedSequence(seed).spawn(n_chunks)
    perm_seed = np.random.SeedSequence(seed + [2])
    k_stop = K if k_limit is None else min(K, k_limit)
    jobs = []
    for c in range((k_stop + chunk - 1) // chunk):
        nk = min(chunk, K - c * chunk)
        take = min(nk, k_stop - c * chunk)
        jobs.append((children[c], nk, take, J, ik_range, nnz_row, col_dist, zipf_s, perm_seed,
                     ik_draw, val_draw))
    if workers is None:
        workers = min(16, os.cpu_count() or 1) if len(jobs) >= 8 else 1
        if _gpu_runtime_started():
            workers = 1  # never fork a process that holds a GPU context
    if workers > 1:
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
            parts = list(ex.map(_gen_chunk, jobs, chunksize=1))
    else:
        parts = [_gen_chunk(j) for j in jobs]
    Ik = np.concatenate([q[0] for q in parts])
    rl = np.concatenate([q[1] for q in parts])
    subj_ptr = np.zeros(Ik.shape[0] + 1, dtype=np.int64)
    np.cumsum(Ik, out=subj_ptr[1:])
    row_ptr = np.zeros(rl.shape[0] + 1, dtype=np.int64)
    np.cumsum(rl, out=row_ptr[1:])
    return Slices(J, subj_ptr, row_ptr, np.concatenate([q[2] for q in parts]),
                  np.concatenate([q[3] for q in parts]))


class _poisson_plus_one:
    """1 + Poisson(lam) nonzeros per row."""

    def __init__(self, lam):
        self.lam = lam

    def __call__(self, rng, n):
        return 1 + rng.poisson(self.lam, size=n)


class _geometric_rows:
    """lo + Geometric(p) - 1 rows, truncated at hi (many subjects with few
    observations, a long tail of frequent ones)."""

    def __init__(self, lo, hi, p):
        self.lo, self.hi, self.p = lo, hi, p

    def __call__(self, rng, n):
        return np.minimum(self.lo - 1 + rng.geometric(self.p, size=n), self.hi)


class _half_stars:
    """Values in {0.5, 1.0, ..., 5.0}, uniform (rating-like)."""

    def __call__(self, rng, n):
        return 0.5 * rng.integers(1, 11, size=n)


class _uniform_int:
    """Uniform integer count in [lo, hi]."""

    def __init__(self, lo, hi):
        self.lo, self.hi = lo, hi

    def __call__(self, rng, n):
        return rng.integers(self.lo, self.hi + 1, size=n)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

CONFIGS = {
    # small: the oracle runs 20 iterations in seconds
    1: dict(name="c1_small_R5", K=200, J=100, R=5, ik=(5, 20), nnz_row=("poisson1", 4.0), cols="uniform"),
    # single large decomposition, R=10, ~63M nnz
    2: dict(name="c2_K1M_J5000_R10_63Mnnz", K=1_000_000, J=5000, R=10, ik=(10, 100),
            nnz_row=("poisson1", 0.145), cols="zipf"),
    # scaled to ~490M nnz, R=40
    3: dict(name="c3_K1M_J5000_R40_490Mnnz", K=1_000_000, J=5000, R=40, ik=(40, 100),
            nnz_row=("poisson1", 6.0), cols="zipf"),
    # the shape of the paper's EHR data (Table "table:data_stats": 464,900
    # subjects, 1,328 variables, at most 166 observations, 12.3M nonzeros):
    # I_k = 2 + Geometric(1/7) - 1 truncated at 166 (mean about 8), 1 +
    # Poisson(2.3) codes per weekly observation at Zipf(1.1) columns
    6: dict(name="c6_ehr_like_K465K_J1328_R10", K=464_900, J=1328, R=10, ik=(2, 166),
            ik_draw=("geometric", 2, 166, 1.0 / 7.0), nnz_row=("poisson1", 2.3), cols="zipf"),
    # the shape of the paper's ratings data (25,249 users, 26,096 movies, at
    # most 19 yearly observations, 8.9M nonzeros): I_k uniform in [2, 19],
    # 1 + Poisson(32.5) ratings per year at Zipf(1.1) columns, values in
    # half stars
    7: dict(name="c7_ratings_like_K25K_J26096_R10", K=25_249, J=26_096, R=10, ik=(2, 19),
            nnz_row=("poisson1", 32.5), cols="zipf", vals="half_stars"),
}


def _nnz_sampler(spec):
    kind, a = spec[0], spec[1:]
    if kind == "poisson1":
        return _poisson_plus_one(a[0])
    if kind == "uniform":
        return _uniform_int(a[0], a[1])
    raise ValueError(kind)


def gen_config(cfg: int, k_limit: Optional[int] = None) -> tuple[Slices, int]:
    """Slices of configuration cfg (1..3, 6, 7), optionally only the first k_limit
    subjects (identical to the leading subjects of the full input)."""
    c = CONFIGS[cfg]
    ik_draw = None
    if "ik_draw" in c:
        kind, lo, hi, p = c["ik_draw"]
        assert kind == "geometric"
        ik_draw = _geometric_rows(lo, hi, p)
    val_draw = _half_stars() if c.get("vals") == "half_stars" else None
    X = gen_slices(c["K"], c["J"], c["ik"], _nnz_sampler(c["nnz_row"]), c["cols"],
                   [ROOT_SEED, cfg], k_limit=k_limit, ik_draw=ik_draw, val_draw=val_draw)
    return X, c["R"]


def gen_init(J: int, K: int, R: int, seed) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Default initial state: H0 = I_R, W0 = ones (K x R), V0 ~ U[0,1) (J x R).
    V0 is rounded to float32 values (held in float64), so that a float32 copy
    of it is exact."""
    rng = np.random.default_rng(np.random.SeedSequence(list(seed)))
    V0 = rng.random((J, R)).astype(np.float32).astype(np.float64)
    return np.eye(R), V0, np.ones((K, R))


def take_subjects(X: Slices, k0: int, k1: int) -> Slices:
    """Subjects [k0, k1) as a Slices of their own (same J)."""
    r0, r1 = int(X.subj_ptr[k0]), int(X.subj_ptr[k1])
    z0, z1 = int(X.row_ptr[r0]), int(X.row_ptr[r1])
    return Slices(X.J, X.subj_ptr[k0:k1 + 1] - r0, X.row_ptr[r0:r1 + 1] - z0,
                  X.col[z0:z1].copy(), X.val[z0:z1].copy())


def concat_slices(parts: list) -> Slices:
    J = parts[0].J
    sp, rp = [np.zeros(1, np.int64)], [np.zeros(1, np.int64)]
    ro, zo = 0, 0
    for p in parts:
        assert p.J == J
        sp.append(p.subj_ptr[1:] + ro)
        rp.append(p.row_ptr[1:] + zo)
        ro += p.n_rows
        zo += p.nnz
    return Slices(J, np.concatenate(sp), np.concatenate(rp),
                  np.concatenate([p.col for p in parts]), np.concatenate([p.val for p in parts]))


# ---------------------------------------------------------------------------
# planted (noise-free) PARAFAC2 data, for recovery tests
# ---------------------------------------------------------------------------

def gen_planted(K: int, J: int, R: int, ik_range, seed, col_blocks: bool = False,
                s_off_frac: float = 0.0):
    """Dense noise-free slices X_k = Q*_k H* S*_k V*^T with orthonormal Q*_k,
    returned as a Slices plus the true factors.  This is the model of the
    paper's Sec. "Model" evaluated forward on random factors; with
    col_blocks=True every column of V* is supported on its own block of
    columns (so the slices are column-sparse), and with s_off_frac > 0 that
    fraction of the entries of S*_k is zero."""
    rng = np.random.default_rng(np.random.SeedSequence(list(seed)))
    H = rng.standard_normal((R, R))
    if col_blocks:
        V = np.zeros((J, R))
        edges = np.linspace(0, J, R + 1).astype(int)
        for r in range(R):
            V[edges[r]:edges[r + 1], r] = 0.5 + rng.random(edges[r + 1] - edges[r])
    else:
        V = rng.random((J, R))
    W = 0.5 + rng.random((K, R))
    if s_off_frac > 0:
        W[rng.random((K, R)) < s_off_frac] = 0.0
        W[np.arange(K), rng.integers(0, R, K)] = 1.0
    Qs, rows = [], []
    for k in range(K):
        Ik = int(rng.integers(ik_range[0], ik_range[1] + 1))
        Q, _ = np.linalg.qr(rng.standard_normal((Ik, R)))
        Qs.append(Q)
        rows.append((Q @ H) * W[k] @ V.T)
    Ik = np.array([r.shape[0] for r in rows], dtype=np.int64)
    subj_ptr = np.zeros(K + 1, np.int64)
    np.cumsum(Ik, out=subj_ptr[1:])
    dense = np.concatenate(rows).astype(np.float32)
    nzr, nzc = np.nonzero(dense)
    row_ptr = np.zeros(dense.shape[0] + 1, np.int64)
    np.cumsum(np.bincount(nzr, minlength=dense.shape[0]), out=row_ptr[1:])
    X = Slices(J, subj_ptr, row_ptr, nzc.astype(np.int32), dense[nzr, nzc].astype(np.float32))
    return X, dict(H=H, V=V, W=W, Q=Qs)


# ---------------------------------------------------------------------------
# batched workload: 64 independent problems of different sizes
# ---------------------------------------------------------------------------

def gen_limits_case(big_nnz: int = 65535, J: int = 65536, K: int = 16, R: int = 4,
                    seed=(ROOT_SEED, 9)) -> Slices:
    """An input at the limits of the compact on-device encoding: J columns
    (65536 by default, with the top column J - 1 used) and subject 0 holding
    exactly big_nnz nonzeros in rows of about 50; subjects 1.. have I_k in
    [R, R + 10] and 1-6 uniform distinct columns per row.  Values in (0, 1]."""
    rng = np.random.default_rng(list(seed))
    rows = []  # one (sorted distinct columns) array per row
    subj_ptr = [0]
    n0 = -(-big_nnz // 50)
    base, extra = divmod(big_nnz, n0)
    for i in range(n0):
        m = base + (1 if i < extra else 0)
        cols = np.sort(rng.choice(J, size=m, replace=False))
        if i == 0 and cols[-1] != J - 1:
            cols[-1] = J - 1
            cols = np.unique(cols)
            while cols.shape[0] < m:  # keep the row length after the swap
                extra_col = int(rng.integers(0, J - 1))
                if extra_col not in cols:
                    cols = np.sort(np.append(cols, extra_col))
        rows.append(cols)
    subj_ptr.append(len(rows))
    for _ in range(1, K):
        ik = int(rng.integers(R, R + 11))
        for _ in range(ik):
            m = int(rng.integers(1, 7))
            rows.append(np.sort(rng.choice(J, size=m, replace=False)))
        subj_ptr.append(len(rows))
    row_ptr = np.zeros(len(rows) + 1, np.int64)
    row_ptr[1:] = np.cumsum([r.shape[0] for r in rows])
    col = np.concatenate(rows).astype(np.int32)
    val = (1.0 - rng.random(col.shape[0])).astype(np.float32)
    return Slices(J, np.asarray(subj_ptr, np.int64), row_ptr, col, val)


def gen_batched_specs(n_problems: int = 64, seed=(ROOT_SEED, 4), k_scale: float = 1.0):
    """Sizes of the batched workload: K log-uniform in [1000, 50000] (times
    k_scale), J in {500,1000,2000,5000}, R in {5,10,20}, I_k in [R,100],
    3..12 nonzeros per row at uniform distinct columns."""
    rng = np.random.default_rng(np.random.SeedSequence(list(seed)))
    specs = []
    for p in range(n_problems):
        K = int(round(math.exp(rng.uniform(math.log(1000), math.log(50000))) * k_scale))
        K = max(K, 1)
        J = int(rng.choice([500, 1000, 2000, 5000]))
        R = int(rng.choice([5, 10, 20]))
        specs.append(dict(K=K, J=J, R=R, seed=[*seed, 100 + p]))
    return specs


def gen_batched_problem(spec) -> Slices:
    return gen_slices(spec["K"], spec["J"], (spec["R"], 100), _uniform_int(3, 12), "uniform",
                      spec["seed"])


# ---------------------------------------------------------------------------
# serving workload: fixed phenotypes and a Poisson stream of new subjects
# ---------------------------------------------------------------------------

def gen_serving_model(J: int = 5000, R: int = 40, density: float = 0.05, seed=(ROOT_SEED, 5)):
    """Fixed V (J x R, each entry nonzero with probability density, U[0,1))
    and H (R x R, standard normal)."""
    rng = np.random.default_rng(np.random.SeedSequence(list(seed) + [1]))
    V = rng.random((J, R)) * (rng.random((J, R)) < density)
    H = rng.standard_normal((R, R))
    return V.astype(np.float32), H


def gen_serving_requests(n: int, J: int = 5000, R: int = 40, rate: float = 2000.0,
                         seed=(ROOT_SEED, 5)):
    """n requests: arrival times (Poisson process at `rate` per second) and one
    slice each with I_k in [R, 100] rows and 1..50 nonzeros per row at uniform
    distinct columns."""
    rng = np.random.default_rng(np.random.SeedSequence(list(seed) + [2]))
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    X = gen_slices(n, J, (max(R, 40), 100), _uniform_int(1, 50), "uniform", list(seed) + [3])
    return t, X
