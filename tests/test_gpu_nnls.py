"""GPU parity of the non-negative V and S_k (NNLS rows, parafac2_opts.nonneg)
against the FP64 oracle, element by element (tests/_cmp.py bars), plus the
KKT conditions of the GPU's own W rows."""
import numpy as np
import pytest

from datagen import gen_config, gen_init, gen_planted
from oracle import parafac2_oracle as O

from _cmp import check_rows, check_shared, kappa_of

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1703_04219_amd import binding as B  # noqa: E402


def _xs(X):
    return O.slices_to_list(X.subj_ptr, X.row_ptr, X.col, X.val, X.J)


def _gauss_state(X, R, seed):
    # a Gaussian H makes the unconstrained V update go negative, so the
    # constraint binds; the state is rounded to the float32 values the GPU holds
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((R, R))
    V = rng.random((X.J, R)).astype(np.float32).astype(np.float64)
    W = (0.5 + rng.random((X.K, R))).astype(np.float32).astype(np.float64)
    return H, V, W


def _compare(X, R, H0, V0, W0, pool=False):
    if pool:
        from oracle.parallel import Pool
        with Pool(X.subj_ptr, X.row_ptr, X.col, X.val, X.J) as p:
            H1, V1, W1, info = p.iterate(H0, V0, W0, nonneg=True)
            kap = p.kappa(H0, V0, W0, cut=1e-8)
    else:
        Xs = _xs(X)
        H1, V1, W1, info = O.iterate(Xs, H0, V0, W0, dense_loss=False, nonneg=True)
        kap = kappa_of(Xs, H0, V0, W0)
    ctx = B.Context(B.DeviceSlices.from_slices(X), R, H0, V0, W0, B.make_opts(nonneg=True))
    fit = ctx.iterate(1)[0]
    torch.cuda.synchronize()
    M1, M2, M3 = (t.cpu().numpy() for t in ctx.mttkrp())
    V, W = ctx.V.cpu().numpy(), ctx.W.cpu().numpy()
    errs = {}
    check_shared(errs, "M1", M1, info["M1"])
    check_shared(errs, "M2", M2, info["M2"])
    check_shared(errs, "H", ctx.H.cpu().numpy(), H1)
    check_shared(errs, "V", V, V1)
    check_rows("M3", M3, info["M3"], kap)
    ew = check_rows("W", W, W1, kap)
    errs["fit"] = abs(fit - info["fit"])
    print(f"K={X.K} R={R} nonneg: zeros V {(V1 == 0).sum()} (gpu {(V == 0).sum()}), "
          f"W {(W1 == 0).sum()} (gpu {(W == 0).sum()}); errors " +
          ", ".join(f"{k}={v:.2e}" for k, v in errs.items()) + f", W rows {ew.max():.2e}",
          flush=True)
    assert np.all(V >= 0) and np.all(W >= 0)
    assert errs["fit"] <= 1e-5
    return ctx, info


def test_nonneg_one_iteration_config1():
    X, R = gen_config(1)
    H0, V0, W0 = _gauss_state(X, R, 17)
    _compare(X, R, H0, V0, W0)


@pytest.mark.parametrize("R", [3, 10, 20, 40])
def test_nonneg_planted_sparse_weights(R):
    # a planted model whose S_k have zero entries: the W rows' constraint
    # binds; one iteration from a perturbed truth
    X, truth = gen_planted(K=120, J=60, R=R, ik_range=(R, R + 10), seed=[600 + R],
                           s_off_frac=0.4)
    rng = np.random.default_rng(R)
    H0 = truth["H"] + 0.05 * rng.standard_normal(truth["H"].shape)
    V0 = np.abs(truth["V"] + 0.05 * rng.standard_normal(truth["V"].shape))
    W0 = np.abs(truth["W"] + 0.05 * rng.standard_normal(truth["W"].shape))
    V0 = V0.astype(np.float32).astype(np.float64)
    W0 = W0.astype(np.float32).astype(np.float64)
    ctx, info = _compare(X, R, H0, V0, W0)
    # KKT of the GPU's W rows with its own N3 = (V^T V) * (H^T H)
    V = ctx.V.cpu().numpy().astype(np.float64)
    H = ctx.H.cpu().numpy()
    W = ctx.W.cpu().numpy().astype(np.float64)
    M3 = ctx.mttkrp()[2].cpu().numpy().astype(np.float64)
    N3 = (V.T @ V) * (H.T @ H)
    G = M3 - W @ N3
    scale = np.abs(M3).max(axis=1, keepdims=True)
    if R >= 10:  # at R = 3 the planted zeros are not reached in one step
        assert (W == 0).any()
    assert np.all(G[W == 0] <= 1e-4 * np.broadcast_to(scale, W.shape)[W == 0])
    assert np.all(np.abs(G[W > 0]) <= 1e-4 * np.broadcast_to(scale, W.shape)[W > 0])


def test_nonneg_fit_trajectory_config1():
    X, R = gen_config(1)
    H0, V0, W0 = _gauss_state(X, R, 18)
    _, _, _, hist = O.run(_xs(X), H0, V0, W0, 20, dense_loss=True, nonneg=True)
    ofits = np.array([h["fit"] for h in hist])
    ctx = B.Context(B.DeviceSlices.from_slices(X), R, H0, V0, W0, B.make_opts(nonneg=True))
    gfits = ctx.iterate(20)
    print("nonneg fit oracle", ofits[[0, 9, 19]], "gpu", gfits[[0, 9, 19]], flush=True)
    assert np.max(np.abs(gfits - ofits)) <= 1e-5
    assert np.all(np.diff(gfits) >= -1e-6)
    assert np.all(ctx.V.cpu().numpy() >= 0) and np.all(ctx.W.cpu().numpy() >= 0)


def test_nonneg_large_subsample():
    X, R = gen_config(2, k_limit=20000)
    H0, V0, W0 = _gauss_state(X, R, 19)
    _compare(X, R, H0, V0, W0, pool=True)


def test_nonneg_batch_mixed_with_unconstrained():
    # a batch holding a constrained and an unconstrained problem of one rank:
    # each matches the same problem run alone
    X, R = gen_config(1)
    H0, V0, W0 = _gauss_state(X, R, 21)
    alone = []
    for nn in (True, False):
        c = B.Context(B.DeviceSlices.from_slices(X), R, H0, V0, W0, B.make_opts(nonneg=nn))
        c.iterate(3)
        alone.append(tuple(t.cpu().numpy().copy() for t in (c.H, c.V, c.W)))
    ctxs = [B.Context(B.DeviceSlices.from_slices(X), R, H0, V0, W0, B.make_opts(nonneg=nn))
            for nn in (True, False)]
    batch = B.Batch(ctxs)
    batch.iterate(3)
    torch.cuda.synchronize()
    for c, ref in zip(ctxs, alone):
        for got, want in zip((c.H, c.V, c.W), ref):
            got = got.cpu().numpy().astype(np.float64)
            assert np.max(np.abs(got - want)) <= 1e-5 * max(np.abs(want).max(), 1e-30)
