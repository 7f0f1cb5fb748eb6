"""Plain FP64 CPU oracle for one PARAFAC2-ALS iteration on sparse irregular slices.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: it exists so that tests/, the smoke check and the CPU
baseline of the benchmark can check the HIP path against a slow, obviously
correct implementation written from the paper (Perros et al., "SPARTan:
Scalable PARAFAC2 for Large & Sparse Data", KDD'17).  It shares no code with
the HIP path.

Everything is float64 (the input values are float32 and are upcast exactly).
The oracle follows the paper's algorithms in their order and notation:

* the Q-step is the orthogonal Procrustes solution of Sec. "Classical
  Algorithm for PARAFAC2", objective (procrustes_obj): SVD of H S_k V^T X_k^T,
  Q_k = Z_k P_k^T (Algorithm "PARAFAC2-ALS", the first loop over k);
* Y_k = Q_k^T X_k is formed explicitly (same algorithm, second loop over k);
* the MTTKRPs are computed from their plain definitions, equations (mttkrp1),
  (mttkrp2), (mttkrp3): M^(n) = Y_(n) (Khatri-Rao product), with the
  matricizations of Sec. "Tensors and Tensor Operations" written out as
  sparse matrices (only the nonzero columns of each Y_k are stored, as the
  overview of Sec. "The SPARTan approach" notes they are the only nonzeros);
* one CP-ALS iteration (Algorithm "CP-ALS") updates H, V, W with
  pseudo-inverses of the Hadamard products of Grams.

Readings of points the paper leaves open (each is listed in the design notes):

* Q-step SVD (garbled in the text): the SVD of the R x I_k matrix
  H S_k V^T X_k^T is written P diag(sigma) Z^T, and Q_k = Z P^T; the rank-R
  truncation is the thin SVD.  For I_k < R the thin SVD has I_k singular
  values and Q_k (I_k x R) has orthonormal rows instead of columns; there
  the truncation also drops singular values at or below 10^-6.5 sigma_max
  (numerically zero: rows of X_k that are multiples of each other), because
  with orthonormal rows ||Q_k H S_k V^T|| and so the loss would depend on the
  arbitrary completion of the missing directions.
* Normalisation (Algorithm "CP-ALS", "Normalize columns"): H and V get unit
  2-norm columns after their updates and the norms are dropped; W is not
  normalised (S_k = diag(W(k,:)) carries the scale, Sec. "CP Decomposition").
  Dropping the norms does not change the iterate after the next least-squares
  update, because each update absorbs a column scaling of the factors it holds
  fixed.
* Pseudo-inverse: eigen-decomposition of the symmetric R x R matrix,
  eigenvalues <= R * eps64 * lambda_max are dropped.
* Loss and fit: loss = sum_k ||X_k - Q_k H S_k V^T||_F^2 (the objective of
  Sec. "Classical Algorithm for PARAFAC2"), fit = 1 - loss / sum_k ||X_k||_F^2,
  evaluated after the W update of the iteration.
* Projection of new subjects (serving) is not in the paper: with V and H
  fixed, alternate the same Q-step and the least-squares update of one row of
  W (the mode-3 MTTKRP row, equation (mttkrp3_row_wise), times the
  pseudo-inverse of (V^T V) * (H^T H)), starting from w = 1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

EPS64 = np.finfo(np.float64).eps


# ---------------------------------------------------------------------------
# input slices
# ---------------------------------------------------------------------------

def slices_to_list(subj_ptr, row_ptr, col, val, J):
    """The collection {X_k} as scipy CSR matrices in float64."""
    out = []
    K = len(subj_ptr) - 1
    for k in range(K):
        r0, r1 = int(subj_ptr[k]), int(subj_ptr[k + 1])
        z0, z1 = int(row_ptr[r0]), int(row_ptr[r1])
        out.append(sp.csr_matrix(
            (np.asarray(val[z0:z1], dtype=np.float64), np.asarray(col[z0:z1]),
             np.asarray(row_ptr[r0:r1 + 1] - row_ptr[r0])), shape=(r1 - r0, J)))
    return out


def norm_x_sq(Xs):
    """sum_k ||X_k||_F^2."""
    return float(sum(float(X.data @ X.data) for X in Xs))


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def khatri_rao(A, B):
    """Column-wise Kronecker product A (.) B: row k*B.shape[0] + j is
    A[k, :] * B[j, :] (Sec. "Tensors and Tensor Operations")."""
    K, R = A.shape
    J = B.shape[0]
    return (A[:, None, :] * B[None, :, :]).reshape(K * J, R)


def pinv_sym(N):
    """Moore-Penrose pseudo-inverse of a symmetric PSD matrix via its
    eigen-decomposition; eigenvalues <= R * eps * lambda_max are dropped."""
    lam, E = np.linalg.eigh(N)
    lmax = max(float(lam.max()), 0.0)
    keep = lam > N.shape[0] * EPS64 * lmax
    inv = np.zeros_like(lam)
    inv[keep] = 1.0 / lam[keep]
    return (E * inv) @ E.T


def nnls_normal(N, m, max_outer=None):
    """min_{x >= 0} ||y - Z x||^2 given only N = Z^T Z (symmetric positive
    definite, R x R) and m = Z^T y: the active-set method of Lawson and
    Hanson in the form that works on the cross products (the fast NNLS of Bro
    and De Jong, which the paper uses for the non-negative S_k and V, Sec.
    "Setup").  P is the passive set (free variables), the others are held at
    zero.
      x = 0, w = m - N x
      while some j outside P has w_j > tol:
          move the j with the largest w_j into P
          s = solution of N[P,P] s_P = m_P, s = 0 outside P
          while some s_j <= 0 on P:
              step x towards s as far as x stays >= 0 (alpha = min over
              those j of x_j / (x_j - s_j)); variables that reach 0 leave P;
              solve again on the new P
          x = s, w = m - N x
    tol is 10 R eps times the scale of m and N x."""
    N = np.asarray(N, np.float64)
    m = np.asarray(m, np.float64)
    R = m.shape[0]
    eps = EPS64
    x = np.zeros(R)
    P = np.zeros(R, dtype=bool)
    max_outer = 3 * R if max_outer is None else max_outer

    def solve(Pm):
        s = np.zeros(R)
        idx = np.nonzero(Pm)[0]
        if idx.size:
            s[idx] = np.linalg.solve(N[np.ix_(idx, idx)], m[idx])
        return s

    scale = max(float(np.max(np.abs(m))), np.finfo(np.float64).tiny)
    tol = 10.0 * R * eps * scale
    w = m - N @ x
    blocked = np.zeros(R, dtype=bool)  # entered and left again without a step
    for _ in range(max_outer):
        cand = np.where(~P & ~blocked, w, -np.inf)
        j = int(np.argmax(cand))
        if not (cand[j] > tol):
            break
        P[j] = True
        s = solve(P)
        for _ in range(R + 1):
            bad = np.nonzero(P & (s <= 0))[0]
            if bad.size == 0:
                break
            d = x[bad] - s[bad]
            ratio = np.where(d > 0, x[bad] / np.where(d > 0, d, 1.0), 0.0)
            q = int(np.argmin(ratio))
            alpha = ratio[q]
            x = x + alpha * (s - x)
            x[bad[q]] = 0.0  # the variable that limits the step reaches zero
            P &= ~(x <= 10.0 * eps * max(float(np.max(np.abs(x))), 1e-300))
            x[~P] = 0.0
            if alpha > 0:
                blocked[:] = False
            elif not P[j]:
                blocked[j] = True  # rounding: w_j > tol but its solve was <= 0
            s = solve(P)
        x = s
        w = m - N @ x
        scale = max(scale, float(np.max(np.abs(N @ x))))
        tol = 10.0 * R * eps * scale
    return x


def nnls_rows(N, M):
    """Row by row: X(i, :) = argmin over x >= 0 of the least-squares problem
    with normal equations N x = M(i, :) (nnls_normal)."""
    return np.array([nnls_normal(N, M[i]) for i in range(M.shape[0])]).reshape(M.shape)


def procrustes_q(X, H, w, V):
    """Q-step for one subject (Sec. "Classical Algorithm for PARAFAC2",
    objective (procrustes_obj)): SVD of H S_k V^T X_k^T = P diag(s) Z^T,
    Q_k = Z P^T (I_k x R; orthonormal columns, or orthonormal rows when
    I_k < R)."""
    # H S_k V^T X_k^T, R x I_k, associated as H S_k (X_k V)^T so that only the
    # rows of V at X_k's nonzero columns enter
    M = ((np.asarray(X @ V) * w) @ H.T).T
    if not np.any(M):
        # H S_k V^T X_k^T = 0 (e.g. w_k = 0): every Q_k attains the objective,
        # and this reading takes Q_k = 0, so that the subject contributes
        # nothing (Y_k = 0) rather than an arbitrary orthonormal completion
        return np.zeros((X.shape[0], H.shape[0]))
    P, s, Zt = np.linalg.svd(M, full_matrices=False)
    if X.shape[0] < H.shape[0]:
        keep = s > s[0] * 10.0 ** -6.5
        P, Zt = P[:, keep], Zt[keep]
    return Zt.T @ P.T


def y_slice(Q, X):
    """Y_k = Q_k^T X_k restricted to the nonzero columns of X_k (the other
    columns of Y_k are exactly zero).  Returns (cols, Y_k[:, cols])."""
    cols = np.unique(X.indices)
    Xd = X[:, cols].toarray()
    return cols, Q.T @ Xd


# ---------------------------------------------------------------------------
# matricizations of Y (R x J x K) and the plain MTTKRP definitions
# ---------------------------------------------------------------------------

def unfold_coo(Ys, R, J, n):
    """The nonzeros of the mode-n matricization of the intermediate tensor Y
    (R x J x K), with Kolda's column ordering (Sec. "Tensors and Tensor
    Operations"):
      n=1: R x (J*K), column j + J*k;
      n=2: J x (R*K), column r + R*k;
      n=3: K x (R*J), column r + R*j.
    Returns (rows, cols, vals, shape); only the nonzero columns of each Y_k
    are stored (all other entries of Y are zero)."""
    K = len(Ys)
    rows, cols, vals = [np.zeros(0, np.int64)], [np.zeros(0, np.int64)], [np.zeros(0)]
    for k, (cj, Yk) in enumerate(Ys):
        c = len(cj)
        rr = np.repeat(np.arange(R, dtype=np.int64), c)
        jj = np.tile(np.asarray(cj, np.int64), R)
        v = Yk.reshape(-1)
        if n == 1:
            rows.append(rr); cols.append(jj + J * k)
        elif n == 2:
            rows.append(jj); cols.append(rr + R * k)
        else:
            rows.append(np.full(R * c, k, dtype=np.int64)); cols.append(rr + R * jj)
        vals.append(v)
    shape = {1: (R, J * K), 2: (J, R * K), 3: (K, R * J)}[n]
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), shape


def unfold_y(Ys, R, J, n):
    """Mode-n matricization of Y as a sparse matrix (see unfold_coo)."""
    rows, cols, vals, shape = unfold_coo(Ys, R, J, n)
    return sp.csr_matrix((vals, (rows, cols)), shape=shape)


def khatri_rao_rows(A, B, idx):
    """Rows idx of the Khatri-Rao product A (.) B: row k*B.shape[0] + j is
    A[k, :] * B[j, :]."""
    nb = B.shape[0]
    idx = np.asarray(idx, np.int64)
    return A[idx // nb] * B[idx % nb]


def mttkrp(Ys, H, V, W, n):
    """Plain definitions: M1 = Y_(1)(W (.) V) (mttkrp1), M2 = Y_(2)(W (.) H)
    (mttkrp2), M3 = Y_(3)(V (.) H) (mttkrp3).  The product is taken over the
    columns of Y_(n) that hold a nonzero, with the matching rows of the
    Khatri-Rao product; the other rows of that product multiply zero columns
    of Y_(n) and are not formed (for a million subjects the full product has
    K*J rows)."""
    R, J = H.shape[0], V.shape[0]
    rows, cols, vals, shape = unfold_coo(Ys, R, J, n)
    used, inv = np.unique(cols, return_inverse=True)
    Yu = sp.csr_matrix((vals, (rows, inv.reshape(-1))), shape=(shape[0], used.shape[0]))
    if n == 1:
        kr = khatri_rao_rows(W, V, used)
    elif n == 2:
        kr = khatri_rao_rows(W, H, used)
    else:
        kr = khatri_rao_rows(V, H, used)
    return np.asarray(Yu @ kr)


def mttkrp_per_slice(Ys, H, V, W, n):
    """The per-slice forms of Sec. "Methodology" (Algorithm "MTTKRP for
    SPARTan"): (mttkrp1_3), (mttkrp2_3), (mttkrp3_row_wise).  Used only by
    the oracle's own self-tests, as a second route to the same numbers."""
    R, J, K = H.shape[0], V.shape[0], W.shape[0]
    if n == 1:
        M = np.zeros((R, R))
        for k, (cj, Yk) in enumerate(Ys):
            M += (Yk @ V[cj]) * W[k]
        return M
    if n == 2:
        M = np.zeros((J, R))
        for k, (cj, Yk) in enumerate(Ys):
            M[cj] += (Yk.T @ H) * W[k]
        return M
    M = np.zeros((K, R))
    for k, (cj, Yk) in enumerate(Ys):
        M[k] = np.sum(H * (Yk @ V[cj]), axis=0)
    return M


# ---------------------------------------------------------------------------
# one PARAFAC2-ALS iteration
# ---------------------------------------------------------------------------

def normalize_cols(A):
    n = np.linalg.norm(A, axis=0)
    n = np.where(n > 1e-300, n, 1.0)
    return A / n


def loss_dense(Xs, Qs, H, V, W):
    """sum_k ||X_k - Q_k H S_k V^T||_F^2, computed densely."""
    tot = 0.0
    for k, X in enumerate(Xs):
        D = X.toarray() - Qs[k] @ ((H * W[k]) @ V.T)
        tot += float(np.sum(D * D))
    return tot


def loss_expanded(nx2, M3, W, V, H):
    """The same loss when every Q_k has orthonormal columns:
    ||X||^2 - 2 <W, M3> + sum_k w_k^T ((V^T V) * (H^T H)) w_k."""
    N3 = (V.T @ V) * (H.T @ H)
    return nx2 - 2.0 * float(np.sum(W * M3)) + float(np.sum((W @ N3) * W))


def iterate(Xs, H, V, W, nx2=None, dense_loss=True, normalize=True, nonneg=False):
    """One PARAFAC2-ALS iteration (Algorithm "PARAFAC2-ALS" body: Q-step,
    build {Y_k}, one CP-ALS iteration (Algorithm "CP-ALS"), S_k <- diag(W(k,:))).
    nonneg: V and W (the diagonals of S_k) are updated by non-negative least
    squares on the same normal equations (the constraints of the paper's
    experiments, Sec. "Classical Algorithm for PARAFAC2" and Sec. "Setup");
    H stays unconstrained.
    Returns the new (H, V, W) and a dict with Q, Y, M1, M2, M3, loss, fit."""
    R = H.shape[0]
    if nx2 is None:
        nx2 = norm_x_sq(Xs)
    Qs = [procrustes_q(X, H, W[k], V) for k, X in enumerate(Xs)]
    Ys = [y_slice(Qs[k], X) for k, X in enumerate(Xs)]
    # mode 1: H <- Y_(1)(W (.) V)(W^T W * V^T V)^+, normalise
    M1 = mttkrp(Ys, H, V, W, 1)
    H1 = M1 @ pinv_sym((W.T @ W) * (V.T @ V))
    if normalize:
        H1 = normalize_cols(H1)
    # mode 2: V <- Y_(2)(W (.) H)(W^T W * H^T H)^+, normalise
    M2 = mttkrp(Ys, H1, V, W, 2)
    N2 = (W.T @ W) * (H1.T @ H1)
    V1 = nnls_rows(N2, M2) if nonneg else M2 @ pinv_sym(N2)
    if normalize:
        V1 = normalize_cols(V1)
    # mode 3: W <- Y_(3)(V (.) H)(V^T V * H^T H)^+
    M3 = mttkrp(Ys, H1, V1, W, 3)
    N3 = (V1.T @ V1) * (H1.T @ H1)
    W1 = nnls_rows(N3, M3) if nonneg else M3 @ pinv_sym(N3)
    if dense_loss:
        loss = loss_dense(Xs, Qs, H1, V1, W1)
    else:
        loss = loss_expanded(nx2, M3, W1, V1, H1)
    return H1, V1, W1, dict(Q=Qs, Y=Ys, M1=M1, M2=M2, M3=M3, loss=loss, fit=1.0 - loss / nx2)



def run(Xs, H, V, W, n_iter, dense_loss=True, nonneg=False):
    """n_iter iterations from (H, V, W); returns the final state and the list
    of per-iteration info dicts."""
    nx2 = norm_x_sq(Xs)
    hist = []
    for _ in range(n_iter):
        H, V, W, info = iterate(Xs, H, V, W, nx2, dense_loss, nonneg=nonneg)
        hist.append(info)
    return H, V, W, hist


def run_until(Xs, H, V, W, max_iter, tol, dense_loss=False):
    """Iterate while the convergence criterion is not met (Algorithm
    "PARAFAC2-ALS"; the paper leaves the criterion open).  The reading taken
    here: stop after iteration t >= 2 once the loss decreased by at most
    tol * loss_{t-1} (or reached 0), else after max_iter iterations."""
    nx2 = norm_x_sq(Xs)
    hist = []
    for t in range(max_iter):
        H, V, W, info = iterate(Xs, H, V, W, nx2, dense_loss)
        hist.append(info)
        if t > 0:
            prev, cur = hist[-2]["loss"], info["loss"]
            if cur <= 0.0 or abs(prev - cur) <= tol * abs(prev):
                break
    return H, V, W, hist


def u_factors(Qs, H):
    """U_k = Q_k H for every subject (Algorithm "PARAFAC2-ALS", after the
    loop; Sec. "Model": X_k is approximated by U_k S_k V^T)."""
    return [Q @ H for Q in Qs]


# ---------------------------------------------------------------------------
# projection of a new subject onto fixed (V, H)
# ---------------------------------------------------------------------------

def project(X, V, H, n_steps=10, w0=None):
    """Alternate, n_steps times, the Q-step for this subject and the
    least-squares update of its row of W with V and H fixed:
    w <- diag(H^T Y V) ((V^T V) * (H^T H))^+   (equation (mttkrp3_row_wise)).
    Returns (Q, w, loss) with Q from the last Q-step and w from the last
    update."""
    R = H.shape[0]
    w = np.ones(R) if w0 is None else np.asarray(w0, dtype=np.float64).copy()
    N3p = pinv_sym((V.T @ V) * (H.T @ H))
    Q = None
    for _ in range(n_steps):
        Q = procrustes_q(X, H, w, V)
        cj, Y = y_slice(Q, X)
        m3 = np.sum(H * (Y @ V[cj]), axis=0)
        w = m3 @ N3p
    D = X.toarray() - Q @ ((H * w) @ V.T)
    return Q, w, float(np.sum(D * D))
