"""Process-pool driver of the FP64 oracle for inputs of up to a million subjects.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): only tests/, the smoke
check, bench.py's CPU baseline and the scripts under tests/golden/ use it.

It runs one PARAFAC2-ALS iteration (Algorithm "PARAFAC2-ALS" body with one
Algorithm "CP-ALS" iteration) with the functions of parafac2_oracle and no
arithmetic of its own beyond adding partial results:

* the Q-step and Y_k are per subject (the algorithm's loops over k), so any
  range of subjects can be done on its own;
* each MTTKRP is the plain definition Y_(n) (Khatri-Rao) of
  parafac2_oracle.mttkrp.  The columns of Y_(1) and Y_(2), and the rows of
  Y_(3), are grouped by subject, so the definition's sum over the columns of
  Y_(1) (Y_(2)) splits into one sum per range of subjects, and Y_(3)'s rows
  are the subjects themselves.  Each worker evaluates the definition on its
  range; the parent adds the partial M1 and M2 (in range order) and stacks
  the rows of M3;
* the R x R least-squares updates, the normalisation and the expanded loss
  are the single-process functions, called once in the parent.

Workers recompute the Q-step of their range for each of the three MTTKRPs
(the step depends only on the input state, so every pass sees the same Y_k)
rather than hold Y between passes.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np

from . import parafac2_oracle as O

_X = None  # (subj_ptr, row_ptr, col, val, J) of the worker's input
_BLAS_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")


def default_workers() -> int:
    """Worker processes: the CPUs this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _init(subj_ptr, row_ptr, col, val, J):
    global _X
    _X = (subj_ptr, row_ptr, col, val, J)


def _slices(k0, k1):
    subj_ptr, row_ptr, col, val, J = _X
    r0, r1 = int(subj_ptr[k0]), int(subj_ptr[k1])
    return O.slices_to_list(subj_ptr[k0:k1 + 1] - r0, row_ptr[r0:r1 + 1], col, val, J)


def _ys(Xs, H, V, W):
    return [O.y_slice(O.procrustes_q(Xk, H, W[k], V), Xk) for k, Xk in enumerate(Xs)]


def _task(args):
    kind, k0, k1, H0, V0, W0r, extra = args
    Xs = _slices(k0, k1)
    if kind == "nx2":
        return O.norm_x_sq(Xs)
    Ys = _ys(Xs, H0, V0, W0r)
    if kind == "m1":
        return O.mttkrp(Ys, H0, V0, W0r, 1)
    if kind == "m2":
        return O.mttkrp(Ys, extra[0], V0, W0r, 2)
    if kind == "m3":
        return O.mttkrp(Ys, extra[0], extra[1], W0r, 3)
    if kind == "dloss":
        # sum_k ||X_k - Q_k H1 S1_k V1^T||_F^2 over the range, densely
        H1, V1, W1 = extra
        Qs = [O.procrustes_q(Xk, H0, W0r[k], V0) for k, Xk in enumerate(Xs)]
        return O.loss_dense(Xs, Qs, H1, V1, W1[k0:k1])
    if kind == "kappa":
        # condition number of B_k = X_k V S_k H^T at the input state, over the
        # singular values above cut * sigma_max (0 for B_k = 0)
        out = np.zeros(len(Xs))
        for k, Xk in enumerate(Xs):
            B = np.asarray(Xk @ (V0 * W0r[k]) @ H0.T)
            s = np.linalg.svd(B, compute_uv=False)
            if s[0] > 0:
                s = s[s > extra[0] * s[0]]
                out[k] = s[0] / s[-1]
        return out
    raise ValueError(kind)


class Pool:
    """A pool of workers holding one input collection (the concatenated CSR)."""

    def __init__(self, subj_ptr, row_ptr, col, val, J, workers=None, chunk=None):
        self.K = int(len(subj_ptr) - 1)
        self.workers = default_workers() if workers is None else int(workers)
        if chunk is None:  # about four ranges per worker, at most 2000 subjects each
            chunk = max(1, min(2000, -(-self.K // (4 * self.workers))))
        self.ranges = [(k0, min(self.K, k0 + chunk)) for k0 in range(0, self.K, chunk)]
        args = (np.asarray(subj_ptr, np.int64), np.asarray(row_ptr, np.int64),
                np.asarray(col), np.asarray(val), int(J))
        # spawned workers (the parent may hold a GPU context, which must not be
        # forked), each with one BLAS thread: the environment is read when a
        # worker first imports numpy
        saved = {v: os.environ.get(v) for v in _BLAS_VARS}
        os.environ.update({v: "1" for v in _BLAS_VARS})
        try:
            self._pool = mp.get_context("spawn").Pool(self.workers, initializer=_init,
                                                      initargs=args)
        finally:
            for v, old in saved.items():
                if old is None:
                    os.environ.pop(v, None)
                else:
                    os.environ[v] = old

    def close(self):
        self._pool.close()
        self._pool.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _map(self, kind, H0, V0, W0, extra=()):
        jobs = [(kind, k0, k1, H0, V0, W0[k0:k1], extra) for k0, k1 in self.ranges]
        return self._pool.map(_task, jobs, chunksize=1)

    def norm_x_sq(self):
        return float(sum(self._map("nx2", None, None, np.zeros((self.K, 0)))))

    def kappa(self, H0, V0, W0, cut=0.0):
        """Condition numbers of B_k = X_k V S_k H^T for every subject, over its
        singular values above cut * sigma_max (0 where B_k = 0)."""
        return np.concatenate(self._map("kappa", H0, V0, W0, (cut,)))

    def iterate(self, H0, V0, W0, nx2=None, nonneg=False, dense_loss=False):
        """One PARAFAC2-ALS iteration from (H0, V0, W0), as
        parafac2_oracle.iterate (nonneg: V and W by NNLS, in the parent;
        dense_loss: the loss from the dense residuals, else the expanded
        formula, which assumes Q_k^T Q_k = I).  Returns (H1, V1, W1, info)
        with info = M1, M2, M3, loss, fit, seconds."""
        t0 = time.perf_counter()
        if nx2 is None:
            nx2 = self.norm_x_sq()
        M1 = np.zeros((H0.shape[0], H0.shape[0]))
        for part in self._map("m1", H0, V0, W0):
            M1 += part
        H1 = O.normalize_cols(M1 @ O.pinv_sym((W0.T @ W0) * (V0.T @ V0)))
        M2 = np.zeros(V0.shape)
        for part in self._map("m2", H0, V0, W0, (H1,)):
            M2 += part
        N2 = (W0.T @ W0) * (H1.T @ H1)
        V1 = O.normalize_cols(O.nnls_rows(N2, M2) if nonneg else M2 @ O.pinv_sym(N2))
        M3 = np.concatenate(self._map("m3", H0, V0, W0, (H1, V1)))
        N3 = (V1.T @ V1) * (H1.T @ H1)
        W1 = O.nnls_rows(N3, M3) if nonneg else M3 @ O.pinv_sym(N3)
        if dense_loss:
            loss = float(sum(self._map("dloss", H0, V0, W0, (H1, V1, W1))))
        else:
            loss = O.loss_expanded(nx2, M3, W1, V1, H1)
        return H1, V1, W1, dict(M1=M1, M2=M2, M3=M3, loss=loss, fit=1.0 - loss / nx2,
                                nx2=nx2, seconds=time.perf_counter() - t0)
