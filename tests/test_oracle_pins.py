"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test ties one part of the oracle to something other than itself: a dense
brute-force construction of the tensor unfoldings, the textbook properties of
the orthogonal Procrustes solution, least squares on the explicit Khatri-Rao
product, the monotone ALS objective, a closed form at R = 1, exact recovery of
planted noise-free models, and hand-derived values in tests/golden/.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from datagen import gen_config, gen_init, gen_planted, gen_slices, take_subjects
from datagen.synth import _poisson_plus_one
from oracle import parafac2_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _xs(X):
    return O.slices_to_list(X.subj_ptr, X.row_ptr, X.col, X.val, X.J)


def _small(K=12, J=9, R=3, ik=(3, 6), lam=2.0, seed=7):
    X = gen_slices(K, J, ik, _poisson_plus_one(lam), "uniform", [seed])
    return X, R


def _dense_tensor(Ys, R, J):
    K = len(Ys)
    T = np.zeros((R, J, K))
    for k, (cj, Yk) in enumerate(Ys):
        T[:, cj, k] = Yk
    return T


def _unfold_dense(T, n):
    # Kolda's mode-n unfolding: mode-n fibers become columns, remaining indices
    # in increasing order with the first varying fastest (Fortran order).
    return np.reshape(np.moveaxis(T, n - 1, 0), (T.shape[n - 1], -1), order="F")


def _kr_dense(A, B):
    # column r of A (.) B is kron(A[:, r], B[:, r])
    return np.stack([np.kron(A[:, r], B[:, r]) for r in range(A.shape[1])], axis=1)


def _state(X, R, seed=3):
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((R, R))
    V = rng.random((X.J, R))
    W = 0.5 + rng.random((X.K, R))
    return H, V, W


# ---------------------------------------------------------------------------
# P-1: the three MTTKRPs against a dense brute force
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [1, 2])
def test_mttkrp_matches_dense_bruteforce(seed):
    X, R = _small(seed=seed)
    Xs = _xs(X)
    H, V, W = _state(X, R, seed)
    Qs = [O.procrustes_q(Xk, H, W[k], V) for k, Xk in enumerate(Xs)]
    Ys = [O.y_slice(Qs[k], Xk) for k, Xk in enumerate(Xs)]
    T = _dense_tensor(Ys, R, X.J)
    # the dense tensor's slices are Q_k^T X_k on all columns
    for k, Xk in enumerate(Xs):
        np.testing.assert_allclose(T[:, :, k], Qs[k].T @ Xk.toarray(), atol=1e-13)
    bf = {1: _unfold_dense(T, 1) @ _kr_dense(W, V),
          2: _unfold_dense(T, 2) @ _kr_dense(W, H),
          3: _unfold_dense(T, 3) @ _kr_dense(V, H)}
    for n in (1, 2, 3):
        M = O.mttkrp(Ys, H, V, W, n)
        Mps = O.mttkrp_per_slice(Ys, H, V, W, n)
        scale = np.linalg.norm(bf[n])
        assert np.linalg.norm(M - bf[n]) <= 1e-12 * scale
        assert np.linalg.norm(Mps - bf[n]) <= 1e-12 * scale


def test_mode3_is_columnwise_inner_product():
    # equation (mttkrp3_colwise): M3(k, r) = H(:, r)^T Y_k V(:, r)
    X, R = _small(seed=5)
    Xs = _xs(X)
    H, V, W = _state(X, R, 5)
    Ys = [O.y_slice(O.procrustes_q(Xk, H, W[k], V), Xk) for k, Xk in enumerate(Xs)]
    M3 = O.mttkrp(Ys, H, V, W, 3)
    T = _dense_tensor(Ys, R, X.J)
    for k in range(X.K):
        for r in range(R):
            assert abs(M3[k, r] - H[:, r] @ T[:, :, k] @ V[:, r]) <= 1e-12 * (1 + abs(M3[k, r]))


# ---------------------------------------------------------------------------
# P-2: orthogonal Procrustes
# ---------------------------------------------------------------------------

def _rand_orth(rng, n, r):
    q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return q


def test_procrustes_textbook_properties():
    rng = np.random.default_rng(11)
    I, J, R = 9, 7, 4
    Xd = rng.random((I, J))
    X = sp.csr_matrix(Xd)
    H = rng.standard_normal((R, R))
    w = 0.5 + rng.random(R)
    V = rng.random((J, R))
    Q = O.procrustes_q(X, H, w, V)
    B = Xd @ V @ np.diag(w) @ H.T  # the matrix whose polar factor Q is
    np.testing.assert_allclose(Q.T @ Q, np.eye(R), atol=1e-13)
    s = np.linalg.svd(B, compute_uv=False)
    assert abs(np.trace(Q.T @ B) - s.sum()) <= 1e-12 * s.sum()
    for _ in range(100):
        Qp = _rand_orth(rng, I, R)
        assert np.trace(Qp.T @ B) <= np.trace(Q.T @ B) + 1e-12
    # full rank: Q = B (B^T B)^{-1/2}
    lam, E = np.linalg.eigh(B.T @ B)
    np.testing.assert_allclose(Q, B @ (E / np.sqrt(lam)) @ E.T, atol=1e-11)
    # the Procrustes objective itself: Q minimises ||X - Q H S V^T||
    obj = np.linalg.norm(Xd - Q @ H @ np.diag(w) @ V.T)
    for _ in range(50):
        Qp = _rand_orth(rng, I, R)
        assert obj <= np.linalg.norm(Xd - Qp @ H @ np.diag(w) @ V.T) + 1e-12


def test_procrustes_special_cases():
    rng = np.random.default_rng(12)
    # R = 1: Q = b / ||b||
    Xd = rng.random((6, 5))
    V = rng.random((5, 1))
    Q = O.procrustes_q(sp.csr_matrix(Xd), np.array([[2.0]]), np.array([0.7]), V)
    b = Xd @ V
    np.testing.assert_allclose(Q, b / np.linalg.norm(b), atol=1e-14)
    # B already orthonormal: Q = B
    Qo = _rand_orth(rng, 8, 3)
    # X V = Qo with X = Qo V^+ for V with orthonormal columns, H = I, w = 1
    Vo = _rand_orth(rng, 6, 3)
    Xd = Qo @ Vo.T
    Q = O.procrustes_q(sp.csr_matrix(Xd), np.eye(3), np.ones(3), Vo)
    np.testing.assert_allclose(Q, Qo, atol=1e-13)


def test_procrustes_ambiguous_case_keeps_objective():
    # w with a zero entry makes B rank deficient: several Q are optimal, check
    # only the invariant tr(Q^T B) = ||B||_* and orthonormality
    rng = np.random.default_rng(13)
    Xd = rng.random((7, 6))
    H = rng.standard_normal((3, 3))
    V = rng.random((6, 3))
    w = np.array([1.0, 0.0, 0.5])
    Q = O.procrustes_q(sp.csr_matrix(Xd), H, w, V)
    B = Xd @ V @ np.diag(w) @ H.T
    np.testing.assert_allclose(Q.T @ Q, np.eye(3), atol=1e-13)
    assert abs(np.trace(Q.T @ B) - np.linalg.svd(B, compute_uv=False).sum()) <= 1e-12 * np.abs(B).sum()


# ---------------------------------------------------------------------------
# P-3: least-squares updates against lstsq on the explicit Khatri-Rao product
# ---------------------------------------------------------------------------

def test_updates_are_least_squares_on_explicit_kr():
    X, R = _small(K=10, J=8, R=3, seed=21)
    Xs = _xs(X)
    H, V, W = _state(X, R, 21)
    H1, V1, W1, info = O.iterate(Xs, H, V, W, normalize=False)
    T = _dense_tensor(info["Y"], R, X.J)
    # H solves min ||Y_(1) - H (W (.) V)^T||
    Hl = np.linalg.lstsq(_kr_dense(W, V), _unfold_dense(T, 1).T, rcond=None)[0].T
    np.testing.assert_allclose(H1, Hl, rtol=1e-9, atol=1e-10)
    # V solves min ||Y_(2) - V (W (.) H1)^T||
    Vl = np.linalg.lstsq(_kr_dense(W, H1), _unfold_dense(T, 2).T, rcond=None)[0].T
    np.testing.assert_allclose(V1, Vl, rtol=1e-9, atol=1e-10)
    # W solves min ||Y_(3) - W (V1 (.) H1)^T||
    Wl = np.linalg.lstsq(_kr_dense(V1, H1), _unfold_dense(T, 3).T, rcond=None)[0].T
    np.testing.assert_allclose(W1, Wl, rtol=1e-9, atol=1e-10)


# ---------------------------------------------------------------------------
# P-4, P-5, P-6: objective, fit formula, normalisation
# ---------------------------------------------------------------------------

def test_loss_monotone_config1():
    X, R = gen_config(1)
    Xs = _xs(X)
    H, V, W = gen_init(X.J, X.K, R, [170304219, 1, 1])
    H, V, W, hist = O.run(Xs, H, V, W, 20)
    losses = [h["loss"] for h in hist]
    for a, b in zip(losses, losses[1:]):
        assert b <= a * (1 + 1e-12)
    assert 0.0 < hist[-1]["fit"] < 1.0


def test_dense_loss_equals_expanded_formula():
    X, R = gen_config(1)
    Xs = _xs(X)
    H, V, W = gen_init(X.J, X.K, R, [170304219, 1, 1])
    nx2 = O.norm_x_sq(Xs)
    for _ in range(3):
        H, V, W, info = O.iterate(Xs, H, V, W, nx2, dense_loss=True)
        le = O.loss_expanded(nx2, info["M3"], W, V, H)
        assert abs(le - info["loss"]) <= 1e-10 * nx2


def test_normalisation_does_not_change_the_model():
    X, R = _small(K=15, J=10, R=3, seed=31)
    Xs = _xs(X)
    H, V, W = _state(X, R, 31)
    Ha, Va, Wa, ia = O.iterate(Xs, H, V, W, normalize=True)
    Hb, Vb, Wb, ib = O.iterate(Xs, H, V, W, normalize=False)
    for k in range(X.K):
        Ua = ia["Q"][k] @ Ha @ np.diag(Wa[k]) @ Va.T
        Ub = ib["Q"][k] @ Hb @ np.diag(Wb[k]) @ Vb.T
        np.testing.assert_allclose(Ua, Ub, rtol=1e-10, atol=1e-12)
    assert abs(ia["loss"] - ib["loss"]) <= 1e-10 * ia["loss"]


# ---------------------------------------------------------------------------
# P-7: recovery of planted noise-free models (PARAFAC2 unique for K >= 4)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("col_blocks", [False, True])
def test_planted_model_recovered_from_near_truth(col_blocks):
    X, truth = gen_planted(K=8, J=30, R=3, ik_range=(5, 12), seed=[41], col_blocks=col_blocks)
    Xs = _xs(X)
    rng = np.random.default_rng(0)
    H = truth["H"] + 1e-2 * rng.standard_normal(truth["H"].shape)
    V = truth["V"] + 1e-2 * rng.standard_normal(truth["V"].shape)
    W = truth["W"] + 1e-2 * rng.standard_normal(truth["W"].shape)
    H, V, W, hist = O.run(Xs, H, V, W, 300, dense_loss=False)
    # ALS converges linearly here; the float32 rounding of the inputs alone
    # would only cap the fit near 1 - 1e-15
    assert hist[-1]["fit"] >= 1 - 1e-8
    fits = [h["fit"] for h in hist]
    assert all(b >= a - 1e-13 for a, b in zip(fits, fits[1:]))
    # the recovered V spans the true columns (up to scale and sign)
    Vt = truth["V"] / np.linalg.norm(truth["V"], axis=0)
    cong = np.abs(Vt.T @ V)
    assert np.all(cong.max(axis=1) > 0.999)


def test_planted_model_recovered_from_default_init():
    # From the default start (H = I, W = 1, V random) PARAFAC2-ALS passes through
    # a long swamp before it reaches the planted model; this recorded seed
    # reaches it within 2000 iterations.
    X, truth = gen_planted(K=50, J=30, R=3, ik_range=(6, 12), seed=[45], col_blocks=True)
    Xs = _xs(X)
    H, V, W = gen_init(X.J, X.K, 3, [45, 1])
    H, V, W, hist = O.run(Xs, H, V, W, 2000, dense_loss=False)
    assert hist[-1]["fit"] >= 1 - 1e-10
    Vt = truth["V"] / np.linalg.norm(truth["V"], axis=0)
    cong = np.abs(Vt.T @ V)
    assert np.all(cong.max(axis=1) > 0.9999)


# ---------------------------------------------------------------------------
# P-8: R = 1 closed form
# ---------------------------------------------------------------------------

def test_rank_one_closed_form():
    # With R = 1, min sum_k ||X_k - c_k q_k v^T|| over unit q_k, v gives the top
    # eigenvector v of sum_k X_k^T X_k and fit* = lambda_max / ||X||^2.
    X = gen_slices(60, 40, (3, 8), _poisson_plus_one(3.0), "uniform", [51])
    Xs = _xs(X)
    G = sum((Xk.T @ Xk).toarray() for Xk in Xs)
    lam, E = np.linalg.eigh(G)
    nx2 = O.norm_x_sq(Xs)
    fit_star = lam[-1] / nx2
    H, V, W = gen_init(X.J, X.K, 1, [51, 1])
    H, V, W, hist = O.run(Xs, H, V, W, 300, dense_loss=False)
    assert abs(hist[-1]["fit"] - fit_star) <= 1e-7
    assert abs(abs(float(E[:, -1] @ V[:, 0])) - 1.0) <= 1e-6


def test_golden_hand_derived_cases():
    with open(os.path.join(GOLDEN, "rank_one_hand.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        K = len(c["slices"])
        J = len(c["slices"][0][0])
        Xs = [sp.csr_matrix(np.array(s, dtype=np.float64)) for s in c["slices"]]
        H, V, W = np.eye(1), np.array(c["v0"], dtype=np.float64).reshape(J, 1), np.ones((K, 1))
        H, V, W, hist = O.run(Xs, H, V, W, c["iters"], dense_loss=True)
        assert abs(hist[-1]["fit"] - c["fit"]) <= c["tol"], c["name"]


# ---------------------------------------------------------------------------
# P-9, P-10: structure
# ---------------------------------------------------------------------------

def test_mode2_rows_outside_nonzero_columns_are_zero():
    X, R = _small(K=5, J=60, R=3, lam=0.5, seed=61)
    Xs = _xs(X)
    H, V, W = _state(X, R, 61)
    _, _, _, info = O.iterate(Xs, H, V, W)
    used = np.zeros(X.J, bool)
    used[np.unique(X.col)] = True
    assert not used.all()
    assert np.all(info["M2"][~used] == 0.0)


def test_subject_permutation_invariance():
    X, R = _small(K=10, J=9, R=3, seed=71)
    Xs = _xs(X)
    H, V, W = _state(X, R, 71)
    perm = np.random.default_rng(1).permutation(X.K)
    a = O.iterate(Xs, H, V, W)
    b = O.iterate([Xs[p] for p in perm], H, V, W[perm])
    np.testing.assert_allclose(b[0], a[0], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(b[1], a[1], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(b[2], a[2][perm], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(b[3]["M3"], a[3]["M3"][perm], rtol=1e-11, atol=1e-12)


def test_zero_weight_subject_contributes_nothing():
    # a subject with w_k = 0 has H S_k V^T X_k^T = 0; taking Q_k = 0 it must
    # leave M1, M2, H, V and every other subject's W row exactly as if it were
    # absent (W^T W, M1 and M2 weight it by w_k = 0), and its own M3 and W rows
    # are then zero (Y_k = 0)
    X, R = _small(K=12, J=9, R=3, seed=81)
    Xs = _xs(X)
    H, V, W = _state(X, R, 81)
    dead = [2, 7]
    W[dead] = 0.0
    live = [k for k in range(X.K) if k not in dead]
    a = O.iterate(Xs, H, V, W)
    b = O.iterate([Xs[k] for k in live], H, V, W[live])
    for k in dead:
        assert not np.any(a[3]["Q"][k])
        assert not np.any(a[3]["Y"][k][1])
    np.testing.assert_allclose(a[3]["M1"], b[3]["M1"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(a[3]["M2"], b[3]["M2"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(a[2][live], b[2], rtol=1e-11, atol=1e-12)
    assert not np.any(a[3]["M3"][dead]) and not np.any(a[2][dead])
    # the loss counts the dead subjects' whole norm, in both loss formulas
    nx_dead = sum(float(Xs[k].multiply(Xs[k]).sum()) for k in dead)
    np.testing.assert_allclose(a[3]["loss"], b[3]["loss"] + nx_dead, rtol=1e-12)


# ---------------------------------------------------------------------------
# P-12: projection of new subjects onto fixed (V, H)
# ---------------------------------------------------------------------------

def test_projection_recovers_planted_weights():
    X, truth = gen_planted(K=6, J=25, R=3, ik_range=(6, 10), seed=[81])
    Xs = _xs(X)
    for k in range(X.K):
        Q, w, loss = O.project(Xs[k], truth["V"], truth["H"], n_steps=200)
        nk = float(Xs[k].data @ Xs[k].data)
        assert loss <= 1e-12 * nk
        np.testing.assert_allclose(w, truth["W"][k], rtol=1e-5)


def test_projection_loss_monotone_over_steps():
    X, R = _small(K=4, J=12, R=3, seed=91)
    Xs = _xs(X)
    rng = np.random.default_rng(91)
    V, H = rng.random((X.J, R)), rng.standard_normal((R, R))
    for k in range(X.K):
        losses = [O.project(Xs[k], V, H, n_steps=s)[2] for s in range(1, 8)]
        for a, b in zip(losses, losses[1:]):
            assert b <= a * (1 + 1e-12) + 1e-14


# ---------------------------------------------------------------------------
# input decoding, projection brute force, economy Procrustes, convergence, U_k
# ---------------------------------------------------------------------------

def test_slices_to_list_stacks_back_to_the_concatenated_csr():
    # the per-subject slices, stacked in order, are the concatenated CSR itself
    # (built here straight from the arrays, without the oracle's decoding)
    X = gen_slices(37, 23, (1, 9), _poisson_plus_one(2.0), "zipf", [4711])
    Xs = _xs(X)
    assert len(Xs) == X.K
    assert [x.shape for x in Xs] == [(int(i), X.J) for i in X.I()]
    whole = sp.csr_matrix((X.val.astype(np.float64), X.col, X.row_ptr), shape=(X.n_rows, X.J))
    stacked = sp.vstack(Xs).tocsr()
    assert (stacked != whole).nnz == 0
    # and each slice is the rows of its subject, densely
    dense = whole.toarray()
    for k in (0, 5, X.K - 1):
        np.testing.assert_array_equal(Xs[k].toarray(), dense[X.subj_ptr[k]:X.subj_ptr[k + 1]])


def _project_bruteforce(Xd, V, H, n_steps):
    """n_steps alternations, each written out from scratch: the polar factor of
    B = X V diag(w) H^T from a full SVD, then w from least squares of X on the
    R rank-one terms (Q H(:, r)) V(:, r)^T."""
    R = H.shape[0]
    w = np.ones(R)
    Q = None
    for _ in range(n_steps):
        B = Xd @ V @ np.diag(w) @ H.T
        U, s, Vt = np.linalg.svd(B, full_matrices=False)
        Q = U @ Vt
        terms = np.stack([np.outer(Q @ H[:, r], V[:, r]).ravel() for r in range(R)], axis=1)
        w = np.linalg.lstsq(terms, Xd.ravel(), rcond=None)[0]
    return Q, w, float(np.sum((Xd - Q @ H @ np.diag(w) @ V.T) ** 2))


def test_projection_matches_svd_lstsq_bruteforce():
    X, R = _small(K=5, J=14, R=3, ik=(5, 9), seed=93)
    Xs = _xs(X)
    rng = np.random.default_rng(93)
    V, H = rng.random((X.J, R)), rng.standard_normal((R, R))
    for k in range(X.K):
        Q, w, loss = O.project(Xs[k], V, H, n_steps=10)
        Qb, wb, lb = _project_bruteforce(Xs[k].toarray(), V, H, 10)
        np.testing.assert_allclose(w, wb, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(Q, Qb, rtol=1e-10, atol=1e-12)
        assert abs(loss - lb) <= 1e-10 * max(lb, 1.0)


def test_procrustes_economy_when_fewer_rows_than_rank():
    # I_k < R: the thin SVD has I_k singular values; Q_k has orthonormal rows
    # and attains tr(Q^T B) = ||B||_* over all matrices with orthonormal rows
    rng = np.random.default_rng(14)
    I, J, R = 3, 9, 5
    Xd = rng.random((I, J))
    H = rng.standard_normal((R, R))
    w = 0.5 + rng.random(R)
    V = rng.random((J, R))
    Q = O.procrustes_q(sp.csr_matrix(Xd), H, w, V)
    B = Xd @ V @ np.diag(w) @ H.T
    assert Q.shape == (I, R)
    np.testing.assert_allclose(Q @ Q.T, np.eye(I), atol=1e-13)
    nuc = np.linalg.svd(B, compute_uv=False).sum()
    assert abs(np.trace(Q.T @ B) - nuc) <= 1e-12 * nuc
    for _ in range(100):
        Qp = _rand_orth(rng, R, I).T  # orthonormal rows
        assert np.trace(Qp.T @ B) <= nuc + 1e-12
    # and it is the economy polar factor B (B^T B)^{+1/2} on B's row space
    lam, E = np.linalg.eigh(B.T @ B)
    keep = lam > 1e-12 * lam.max()
    Gm = (E[:, keep] / np.sqrt(lam[keep])) @ E[:, keep].T
    np.testing.assert_allclose(Q, B @ Gm, atol=1e-11)


def test_economy_subjects_keep_the_loss_monotone():
    # subjects with I_k < R mixed with taller ones: the ALS objective still
    # never increases (each step minimises it over its own block)
    X = gen_slices(30, 12, (1, 8), _poisson_plus_one(3.0), "uniform", [4713])
    assert (X.I() < 4).any()
    Xs = _xs(X)
    H, V, W = gen_init(X.J, X.K, 4, [4713, 1])
    _, _, _, hist = O.run(Xs, H, V, W, 25, dense_loss=True)
    losses = [h["loss"] for h in hist]
    for a, b in zip(losses, losses[1:]):
        assert b <= a * (1 + 1e-12)
    # the dense loss and the expanded formula (which assumes Q_k^T Q_k = I)
    # differ once some Q_k has orthonormal rows only: the oracle's dense loss
    # is the objective itself
    Hn, Vn, Wn, info = O.iterate(Xs, H, V, W, dense_loss=True)
    assert info["loss"] >= 0.0


def test_run_until_stops_on_the_relative_loss_change():
    X, R = gen_config(1)
    Xs = _xs(X)
    H, V, W = gen_init(X.J, X.K, R, [170304219, 1, 1])
    tol = 1e-3
    _, _, _, hist = O.run_until(Xs, H, V, W, 200, tol)
    _, _, _, full = O.run(Xs, H, V, W, len(hist) + 1, dense_loss=False)
    losses = [h["loss"] for h in full]
    n = len(hist)
    assert 2 <= n < 200
    # the same iterates as a plain run of that length
    np.testing.assert_allclose([h["loss"] for h in hist], losses[:n], rtol=1e-12)
    # the criterion holds at the stop and at no earlier iteration
    rel = [abs(a - b) / a for a, b in zip(losses, losses[1:])]
    assert rel[n - 2] <= tol
    assert all(r > tol for r in rel[:n - 2])


def test_u_factors_reconstruct_the_model():
    # U_k S_k V^T equals Q_k H S_k V^T (Sec. "Model"), and U_k^T U_k = H^T H
    # is the same for every subject (the PARAFAC2 constraint)
    X, R = _small(K=6, J=10, R=3, seed=95)
    Xs = _xs(X)
    H, V, W = _state(X, R, 95)
    H1, V1, W1, info = O.iterate(Xs, H, V, W)
    Us = O.u_factors(info["Q"], H1)
    for k in range(X.K):
        np.testing.assert_allclose(Us[k] @ np.diag(W1[k]) @ V1.T,
                                   info["Q"][k] @ H1 @ np.diag(W1[k]) @ V1.T, atol=1e-13)
        np.testing.assert_allclose(Us[k].T @ Us[k], H1.T @ H1, atol=1e-12)


# ---------------------------------------------------------------------------
# N1: non-negative least squares on the normal equations (V and S_k >= 0)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_nnls_normal_matches_scipy_and_kkt(seed):
    # min_{x >= 0} ||y - Z x|| from (Z^T Z, Z^T y) against scipy's NNLS on Z, y
    # itself, and the KKT conditions: x >= 0, gradient w = m - N x <= 0 where
    # x = 0 and = 0 where x > 0
    from scipy.optimize import nnls
    rng = np.random.default_rng(500 + seed)
    n, R = 30, [3, 5, 10, 16][seed % 4]
    Z = rng.standard_normal((n, R)) + (0.5 if seed % 2 else 0.0)
    y = rng.standard_normal(n)
    N, m = Z.T @ Z, Z.T @ y
    x = O.nnls_normal(N, m)
    xs, _ = nnls(Z, y)
    np.testing.assert_allclose(x, xs, rtol=1e-9, atol=1e-11)
    assert np.all(x >= 0)
    w = m - N @ x
    scale = np.abs(m).max()
    assert np.all(w[x == 0] <= 1e-10 * scale)
    assert np.all(np.abs(w[x > 0]) <= 1e-10 * scale)
    # an unconstrained minimiser that is already >= 0 is returned as is
    yp = Z @ (0.5 + rng.random(R))
    np.testing.assert_allclose(O.nnls_normal(N, Z.T @ yp), np.linalg.solve(N, Z.T @ yp),
                               rtol=1e-9)
    # m <= 0 everywhere with N having non-negative entries: x = 0
    Zp = np.abs(Z)
    assert not np.any(O.nnls_normal(Zp.T @ Zp, -np.abs(Zp.T @ y)))


def test_nonnegative_iteration_keeps_factors_nonnegative_and_loss_monotone():
    # the constrained ALS: V and W stay >= 0, the objective never increases,
    # and each V and W row is the NNLS solution of its normal equations
    X, R = gen_config(1)
    Xs = _xs(X)
    H, V, W = _state(X, R, 17)  # Gaussian H: unconstrained updates go negative
    H1, V1, W1, info = O.iterate(Xs, H, V, W, nonneg=True)
    assert np.all(V1 >= 0) and np.all(W1 >= 0)
    assert (V1 == 0).any()  # the constraint binds on V
    Hu, Vu, Wu, _ = O.iterate(Xs, H, V, W)
    assert (Vu < 0).any()
    N2 = (W.T @ W) * (H1.T @ H1)
    # V rows before the column normalisation: the KKT conditions of each row
    # with a zero (gradient <= 0 at the zeros, = 0 on the support), and the
    # same zero pattern as the normalised V
    for j in np.nonzero((V1 == 0).any(axis=1))[0][:5]:
        v = O.nnls_normal(N2, info["M2"][j])
        np.testing.assert_array_equal(v == 0, V1[j] == 0)
        g = info["M2"][j] - N2 @ v
        assert np.all(v >= 0)
        assert np.all(g[v == 0] <= 1e-9 * max(np.abs(info["M2"][j]).max(), 1e-300))
        assert np.all(np.abs(g[v > 0]) <= 1e-9 * max(np.abs(info["M2"][j]).max(), 1e-300))
    _, _, _, hist = O.run(Xs, H, V, W, 15, dense_loss=True, nonneg=True)
    losses = [h["loss"] for h in hist]
    for a, b in zip(losses, losses[1:]):
        assert b <= a * (1 + 1e-12)


def test_procrustes_economy_rank_deficient_keeps_the_row_space():
    # I_k < R with two proportional rows: B has rank I_k - 1; the truncated
    # factor maps onto range(B) only (Q Q^T = projector onto range(B), Q^T Q
    # = projector onto the row space of B) and still attains ||B||_*
    rng = np.random.default_rng(15)
    R, J = 5, 8
    x = rng.random(J)
    Xd = np.vstack([x, 2.5 * x, rng.random(J)])
    H = rng.standard_normal((R, R))
    w = 0.5 + rng.random(R)
    V = rng.random((J, R))
    Q = O.procrustes_q(sp.csr_matrix(Xd), H, w, V)
    B = Xd @ V @ np.diag(w) @ H.T
    U, s, Vt = np.linalg.svd(B, full_matrices=False)
    r = int((s > 1e-10 * s[0]).sum())
    assert r == 2
    np.testing.assert_allclose(Q @ Q.T, U[:, :r] @ U[:, :r].T, atol=1e-12)
    np.testing.assert_allclose(Q.T @ Q, Vt[:r].T @ Vt[:r], atol=1e-12)
    assert abs(np.trace(Q.T @ B) - s.sum()) <= 1e-12 * s.sum()
