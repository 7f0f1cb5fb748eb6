"""Element-by-element comparison of a GPU iteration with the FP64 oracle.

Shared outputs (M1, M2, H, V): the largest entrywise error, relative to the
largest entry of the oracle's matrix, is at most 1e-4.

Per-subject outputs (rows of M3 and W): each row's relative error
||row_gpu - row_oracle|| / ||row_oracle|| is checked against the condition
number kappa of that subject's Procrustes matrix B_k = X_k V S_k H^T (over its
numerically nonzero singular values).  The Q-step takes the polar factor of
B_k, whose sensitivity to a relative perturbation e of B_k is about kappa * e
to first order; the float32 sparse product X_k V perturbs B_k by about 1e-7.
The bar is therefore 1e-4 for subjects with kappa <= 1e3, and 1e-4 * kappa /
1e3 above (the same first-order bound, scaled).  A subject with B_k = 0
(kappa reported as 0) must match to 1e-6 absolute (both sides give zero rows).
"""
import numpy as np

SHARED_TOL = 1e-4
ROW_TOL = 1e-4
KAPPA_KNEE = 1e3
BINS = (0.0, 1e1, 1e2, 1e3, 1e4, 1e5, np.inf)


def kappa_of(Xs, H, V, W, cut=1e-8):
    """kappa(B_k) per subject (plain, single process; for small inputs)."""
    out = np.zeros(len(Xs))
    for k, Xk in enumerate(Xs):
        B = np.asarray(Xk @ (V * W[k]) @ H.T)
        s = np.linalg.svd(B, compute_uv=False)
        if s[0] > 0:
            s = s[s > cut * s[0]]
            out[k] = s[0] / s[-1]
    return out


def shared_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def row_errs(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    num = np.linalg.norm(a - b, axis=1)
    den = np.linalg.norm(b, axis=1)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)


def row_bar(kappa):
    kappa = np.asarray(kappa, np.float64)
    return np.where(kappa <= 0, 1e-6, ROW_TOL * np.maximum(1.0, kappa / KAPPA_KNEE))


def kappa_table(name, errs, kappa):
    """Per condition-number bin: subjects, median and worst row error."""
    lines = [f"{name}: per-subject relative row error by kappa(B_k)"]
    for lo, hi in zip(BINS[:-1], BINS[1:]):
        m = (kappa >= lo) & (kappa < hi) if lo > 0 else (kappa < hi)
        if not np.any(m):
            continue
        lines.append(f"  kappa in [{lo:.0e}, {hi:.0e}): {int(m.sum()):7d} subjects, "
                     f"median {np.median(errs[m]):.2e}, worst {np.max(errs[m]):.2e}")
    return "\n".join(lines)


def check_rows(name, got, want, kappa):
    """Assert every row within its kappa bar; print the per-bin table."""
    e = row_errs(got, want)
    print(kappa_table(name, e, kappa), flush=True)
    bar = row_bar(kappa)
    bad = np.nonzero(e > bar)[0]
    assert bad.size == 0, (name, [(int(k), float(e[k]), float(kappa[k])) for k in bad[:10]])
    return e


def check_shared(errs: dict, name, got, want, tol=SHARED_TOL):
    e = shared_err(got, want)
    errs[name] = e
    assert e <= tol, (name, e)
    return e
