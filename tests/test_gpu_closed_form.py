"""GPU against a closed form at a size the oracle cannot reach (pin P-8).

At R = 1 the PARAFAC2 problem min sum_k ||X_k - c_k q_k v^T||^2 with unit q_k
and v has the solution v = top eigenvector of sum_k X_k^T X_k, c_k = ||X_k v||
and fit* = lambda_max / sum_k ||X_k||^2 (a rank-one fit of each slice along a
shared right vector).  ALS converges to it geometrically, at the rate of the
eigenvalue gap (lambda_2 / lambda_1 ~ 0.47 on this input).

The input is the first 100,000 subjects of the K = 1M, R = 10 workload (Zipf
columns, about 6.3M nonzeros), run at R = 1.  The expected values come from
scipy's Lanczos solver on the J x J Gram, not from the oracle.
"""
import numpy as np
import pytest

from datagen import gen_config

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1703_04219_amd import binding as B  # noqa: E402


def test_rank_one_reaches_the_closed_form_at_scale():
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    X, _ = gen_config(2, k_limit=100_000)
    M = sp.csr_matrix((X.val.astype(np.float64), X.col, X.row_ptr), shape=(X.n_rows, X.J))
    lam, vec = sla.eigsh((M.T @ M).tocsr(), k=1, which="LA")
    v_star = vec[:, 0] / np.linalg.norm(vec[:, 0])
    fit_star = float(lam[0] / (X.val.astype(np.float64) ** 2).sum())

    rng = np.random.default_rng([170304219, 8, 1])
    H0 = np.ones((1, 1))
    V0 = rng.random((X.J, 1)).astype(np.float32)
    W0 = np.ones((X.K, 1), np.float32)
    print(f"K={X.K} nnz={X.nnz}: fit* = {fit_star:.10f}", flush=True)
    ctx = B.Context(B.DeviceSlices.from_slices(X), 1, H0, V0, W0)
    fits = ctx.iterate(150)
    torch.cuda.synchronize()
    v = ctx.V.cpu().numpy().astype(np.float64)[:, 0]
    align = abs(float(v @ v_star)) / np.linalg.norm(v)
    print(f"GPU fit {fits[-1]:.10f} (after 50: {fits[49]:.10f}); |v . v*| = {align:.10f}", flush=True)
    # the fit never decreases (loss is monotone), up to FP32 rounding of the factors
    assert np.all(np.diff(fits) >= -1e-6)
    assert abs(fits[-1] - fit_star) <= 1e-6
    assert align >= 1 - 1e-6
