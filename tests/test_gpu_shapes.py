"""GPU parity on subjects with fewer rows than the rank (the economy
Procrustes factor, Q_k with orthonormal rows) and on the EHR-like and
ratings-like workloads that the paper's real data shape (Table
"table:data_stats"), against the FP64 oracle with its dense loss."""
import numpy as np
import pytest

from datagen import gen_config, gen_init, take_subjects
from oracle import parafac2_oracle as O

from _cmp import check_rows, check_shared, kappa_of

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1703_04219_amd import binding as B  # noqa: E402


def _xs(X):
    return O.slices_to_list(X.subj_ptr, X.row_ptr, X.col, X.val, X.J)


def _compare(X, R, H0, V0, W0, pool=False):
    if pool:
        from oracle.parallel import Pool
        with Pool(X.subj_ptr, X.row_ptr, X.col, X.val, X.J) as p:
            H1, V1, W1, info = p.iterate(H0, V0, W0, dense_loss=True)
            kap = p.kappa(H0, V0, W0, cut=1e-8)
    else:
        Xs = _xs(X)
        H1, V1, W1, info = O.iterate(Xs, H0, V0, W0, dense_loss=True)
        kap = kappa_of(Xs, H0, V0, W0)
    ctx = B.Context(B.DeviceSlices.from_slices(X), R, H0, V0, W0)
    fit = ctx.iterate(1)[0]
    torch.cuda.synchronize()
    M1, M2, M3 = (t.cpu().numpy() for t in ctx.mttkrp())
    errs = {}
    check_shared(errs, "M1", M1, info["M1"])
    check_shared(errs, "M2", M2, info["M2"])
    check_shared(errs, "H", ctx.H.cpu().numpy(), H1)
    check_shared(errs, "V", ctx.V.cpu().numpy(), V1)
    e3 = check_rows("M3", M3, info["M3"], kap)
    ew = check_rows("W", ctx.W.cpu().numpy(), W1, kap)
    errs["fit"] = abs(fit - info["fit"])
    n_econ = int((X.I() < R).sum())
    print(f"K={X.K} R={R}, {n_econ} subjects with I_k < R: " +
          ", ".join(f"{k}={v:.2e}" for k, v in errs.items()) +
          f", M3 rows {e3.max():.2e}, W rows {ew.max():.2e}", flush=True)
    assert errs["fit"] <= 1e-5
    return ctx


@pytest.mark.parametrize("R", [8, 12])
def test_fewer_rows_than_rank_config1(R):
    # the 200-subject workload has I_k in [5, 20]: at R = 8 and 12 part of
    # the subjects get Q_k with orthonormal rows
    X, _ = gen_config(1)
    assert (X.I() < R).any() and (X.I() >= R).any()
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, 1, 1])
    ctx = _compare(X, R, H0, V0, W0)
    Q = ctx.q(0, X.K).cpu().numpy().astype(np.float64)
    worst = 0.0
    for k in np.nonzero(X.I() < R)[0]:
        Qk = Q[X.subj_ptr[k]:X.subj_ptr[k + 1]]
        worst = max(worst, float(np.abs(Qk @ Qk.T - np.eye(Qk.shape[0])).max()))
    print("Q_k Q_k^T - I over the short subjects:", worst, flush=True)
    assert worst <= 1e-5


def test_fewer_rows_than_rank_fit_trajectory():
    X, _ = gen_config(1)
    R = 8
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, 1, 1])
    _, _, _, hist = O.run(_xs(X), H0, V0, W0, 15, dense_loss=True)
    ofits = np.array([h["fit"] for h in hist])
    ctx = B.Context(B.DeviceSlices.from_slices(X), R, H0, V0, W0)
    gfits = ctx.iterate(15)
    print("fit oracle", ofits[[0, 7, 14]], "gpu", gfits[[0, 7, 14]], flush=True)
    assert np.max(np.abs(gfits - ofits)) <= 1e-5
    assert np.all(np.diff(gfits) >= -1e-6)


@pytest.mark.parametrize("cfg,R,k_limit", [(6, 10, 20000), (6, 40, 5000), (7, 10, 5000),
                                           (7, 40, 2000)])
def test_real_data_shaped_workloads(cfg, R, k_limit):
    # EHR-like (464,900 x 1,328, I_k 2..166, mostly short) and ratings-like
    # (25,249 x 26,096, I_k 2..19) subsamples at R = 10 and 40
    X, _ = gen_config(cfg, k_limit=k_limit)
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, cfg, 1])
    _compare(X, R, H0, V0, W0, pool=True)
