"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle,
element by element on the same seeded inputs.

Tolerances (float32 sparse products, float64 R x R algebra; tests/_cmp.py):
  * M1, M2, H, V after one iteration from the same state: largest entrywise
    error <= 1e-4 of the largest entry;
  * rows of M3 and W: relative error per subject <= 1e-4 where the subject's
    Procrustes matrix has condition number kappa <= 1e3, scaled by kappa / 1e3
    above (first-order sensitivity of the polar factor);
  * fit per iteration: absolute error <= 1e-5;
  * projection: relative error of each request's w <= 1e-4 (kappa <= 1e3)
    and of all requests' w together <= 1e-4.
"""
import numpy as np
import pytest

from datagen import gen_config, gen_init, gen_planted, gen_slices, take_subjects
from datagen.synth import _poisson_plus_one, _uniform_int, gen_serving_model, gen_serving_requests
from oracle import parafac2_oracle as O

from _cmp import check_rows, check_shared, kappa_of

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1703_04219_amd import binding as B  # noqa: E402


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _xs(X):
    return O.slices_to_list(X.subj_ptr, X.row_ptr, X.col, X.val, X.J)


def _gpu_run(X, R, H0, V0, W0, n, **opts):
    ctx = B.Context(B.DeviceSlices.from_slices(X), R, H0, V0, W0,
                    B.make_opts(**opts) if opts else None)
    fits = ctx.iterate(n)
    torch.cuda.synchronize()
    return ctx, fits


def _oracle_one_iteration(X, H0, V0, W0, pool=False):
    """(H1, V1, W1, info, kappa) of the oracle; pool=True runs it on the
    process-pool driver (subject ranges on all host cores)."""
    if pool:
        from oracle.parallel import Pool
        with Pool(X.subj_ptr, X.row_ptr, X.col, X.val, X.J) as p:
            H1, V1, W1, info = p.iterate(H0, V0, W0)
            kap = p.kappa(H0, V0, W0, cut=1e-8)
        return H1, V1, W1, info, kap
    Xs = _xs(X)
    H1, V1, W1, info = O.iterate(Xs, H0, V0, W0, dense_loss=False)
    return H1, V1, W1, info, kappa_of(Xs, H0, V0, W0)


def _compare_one_iteration(X, R, H0, V0, W0, fit_tol=1e-5, pool=False, **opts):
    H1, V1, W1, info, kap = _oracle_one_iteration(X, H0, V0, W0, pool)
    ctx, fits = _gpu_run(X, R, H0, V0, W0, 1, **opts)
    M1, M2, M3 = (t.cpu().numpy() for t in ctx.mttkrp())
    errs = {}
    check_shared(errs, "M1", M1, info["M1"])
    check_shared(errs, "M2", M2, info["M2"])
    check_shared(errs, "H", ctx.H.cpu().numpy(), H1)
    check_shared(errs, "V", ctx.V.cpu().numpy(), V1)
    e3 = check_rows("M3", M3, info["M3"], kap)
    ew = check_rows("W", ctx.W.cpu().numpy(), W1, kap)
    errs["M3 rows"], errs["W rows"] = float(e3.max()), float(ew.max())
    errs["fit"] = abs(fits[0] - info["fit"])
    print(f"K={X.K} R={R} {opts or ''} errors: " +
          ", ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    assert errs["fit"] <= fit_tol
    return ctx, info, kap


def test_config1_one_iteration_matches_oracle():
    X, R = gen_config(1)
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, 1, 1])
    _compare_one_iteration(X, R, H0, V0, W0)


def test_config1_fit_trajectory_20_iterations():
    X, R = gen_config(1)
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, 1, 1])
    _, _, _, hist = O.run(_xs(X), H0, V0, W0, 20, dense_loss=True)
    ofits = np.array([h["fit"] for h in hist])
    _, gfits = _gpu_run(X, R, H0, V0, W0, 20)
    print("fit oracle", ofits[[0, 4, 9, 19]], "gpu", gfits[[0, 4, 9, 19]], flush=True)
    assert np.max(np.abs(gfits - ofits)) <= 1e-5
    assert np.all(np.diff(gfits) >= -1e-6)


def _check_q_orthonormal(ctx, X, kap, R, n=2000):
    # Q_k^T Q_k = I for subjects whose B_k has full rank R and condition number
    # kappa <= 1e3 over all R singular values (rank-deficient subjects get
    # Q_k^T Q_k = the projector onto the range of B_k^T on the GPU)
    n = min(n, X.K)
    Q = ctx.q(0, n).cpu().numpy().astype(np.float64)
    worst, counted = 0.0, 0
    for k in range(n):
        if not (0 < kap[k] <= 1e3):
            continue
        r0, r1 = X.subj_ptr[k], X.subj_ptr[k + 1]
        Qk = Q[r0:r1]
        worst = max(worst, float(np.abs(Qk.T @ Qk - np.eye(R)).max()))
        counted += 1
    print(f"Q^T Q - I over {counted} subjects: {worst:.2e}", flush=True)
    assert worst <= 1e-5


@pytest.mark.parametrize("cfg", [2, 3])
def test_large_config_subsample_one_iteration(cfg):
    # the first 20,000 subjects of the R = 10 and R = 40 workloads, as problems
    # of their own (bit-identical to the leading subjects of the full input)
    X, R = gen_config(cfg, k_limit=20000)
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, cfg, 1])
    print(f"config {cfg}: K={X.K} nnz={X.nnz} R={R}", flush=True)
    ctx, _, _ = _compare_one_iteration(X, R, H0, V0, W0, pool=True)
    n = 2000
    head = take_subjects(X, 0, n)
    kap_full = kappa_of(_xs(head), H0, V0, W0[:n], cut=0.0)
    _check_q_orthonormal(ctx, X, kap_full, R, n)


@pytest.mark.parametrize("R,hot_cols", [(10, -1), (10, 1), (10, 2), (20, 1), (20, -1), (32, 1)])
def test_mode2_hot_column_counts(R, hot_cols):
    # fewer LDS-staged hot columns than the columns a lane sums in registers
    # (hot_cols = -1 is none): every column still reaches M2
    X = gen_slices(400, 300, (R, R + 20), _poisson_plus_one(2.0), "zipf", [7100 + R])
    H0, V0, W0 = gen_init(X.J, X.K, R, [7100 + R, 1])
    _compare_one_iteration(X, R, H0, V0, W0, hot_cols=hot_cols)


@pytest.mark.parametrize("R", [r for r in B.SUPPORTED_R if r not in (10, 40)])
def test_other_ranks_one_iteration(R):
    # J = 400 columns: with J = 150 the R = 39 case draws a subject with
    # kappa(B_k) = 8.9e6, whose Procrustes factor alone moves M2 by 8.6e-6
    # and V by 1.8e-4 of their largest entries (the per-subject rows stay
    # within their kappa bars); such subjects are the kappa-binned tests'
    # business, this one covers every rank's kernels
    X = gen_slices(300, 400, (R, R + 12), _poisson_plus_one(3.0), "zipf", [9000 + R])
    H0, V0, W0 = gen_init(X.J, X.K, R, [9000 + R, 1])
    _compare_one_iteration(X, R, H0, V0, W0)


@pytest.mark.parametrize("R", [7, 13, 17, 25, 33, 39])
def test_other_ranks_fit_trajectory(R):
    # after the first iteration each Procrustes step runs inside the mode-3
    # pass of the iteration before: odd ranks and ranks between the built
    # lane-group sizes take that path too
    X = gen_slices(300, 400, (R, R + 12), _poisson_plus_one(3.0), "zipf", [9100 + R])
    H0, V0, W0 = gen_init(X.J, X.K, R, [9100 + R, 1])
    _, _, _, hist = O.run(_xs(X), H0, V0, W0, 4, dense_loss=False)
    ofits = np.array([h["fit"] for h in hist])
    _, gfits = _gpu_run(X, R, H0, V0, W0, 4)
    print(f"R={R} fit oracle", ofits, "gpu", gfits, flush=True)
    assert np.max(np.abs(gfits - ofits)) <= 1e-5


def _with_empty_rows(X, every=3):
    """X with an empty row inserted after every `every`-th row of each subject
    (empty rows are accepted and contribute nothing)."""
    from datagen.synth import Slices
    rp, sp = [0], [0]
    for k in range(X.K):
        r0, r1 = int(X.subj_ptr[k]), int(X.subj_ptr[k + 1])
        n = 0
        for i in range(r0, r1):
            rp.append(int(X.row_ptr[i + 1]))
            n += 1
            if (i - r0) % every == every - 1:
                rp.append(rp[-1])
                n += 1
        sp.append(sp[-1] + n)
    return Slices(X.J, np.array(sp, np.int64), np.array(rp, np.int64), X.col.copy(), X.val.copy())


def test_edge_empty_rows():
    X, R = gen_config(1)
    Xe = _with_empty_rows(X)
    assert Xe.n_rows > X.n_rows and Xe.nnz == X.nnz
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, 1, 1])
    _compare_one_iteration(Xe, R, H0, V0, W0)


def test_edge_single_subject_and_minimal_rows():
    # one subject; and every subject with exactly I_k = R rows
    X = gen_slices(1, 40, (30, 30), _poisson_plus_one(3.0), "uniform", [4242])
    H0, V0, W0 = gen_init(X.J, X.K, 5, [4242, 1])
    _compare_one_iteration(X, 5, H0, V0, W0)
    X = gen_slices(500, 60, (4, 4), _poisson_plus_one(3.0), "uniform", [4343])
    H0, V0, W0 = gen_init(X.J, X.K, 4, [4343, 1])
    _compare_one_iteration(X, 4, H0, V0, W0)


@pytest.mark.parametrize("K", [7, 97, 1001])
def test_edge_ragged_subject_counts(K):
    # subject counts that leave partial tiles, partial bins and idle blocks
    # (a single subject is covered by test_edge_single_subject_and_minimal_rows)
    X = gen_slices(K, 80, (6, 20), _poisson_plus_one(2.0), "zipf", [5000 + K])
    H0, V0, W0 = gen_init(X.J, X.K, 6, [5000 + K, 1])
    _compare_one_iteration(X, 6, H0, V0, W0)


def test_edge_zero_weight_subjects():
    # a zero row of W makes B_k = 0: the GPU's Cholesky finds no positive
    # pivot, so F_k = 0, Q_k = 0 and Y_k = 0 (the oracle's reading of a zero
    # B_k); such subjects contribute nothing and their W rows stay zero
    X, R = gen_config(1)
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, 1, 1])
    W0 = W0.copy()
    dead = [0, 17, 101, X.K - 1]
    W0[dead] = 0.0
    ctx, _, _ = _compare_one_iteration(X, R, H0, V0, W0)
    assert not np.any(ctx.W.cpu().numpy()[dead])
    Q = ctx.q(0, X.K).cpu().numpy()
    for k in dead:
        assert not np.any(Q[X.subj_ptr[k]:X.subj_ptr[k + 1]])
    _, _, _, hist = O.run(_xs(X), H0, V0, W0, 5, dense_loss=True)
    ofits = np.array([h["fit"] for h in hist])
    ctx5, gfits = _gpu_run(X, R, H0, V0, W0, 5)
    print("fit oracle", ofits, "gpu", gfits, flush=True)
    assert np.max(np.abs(gfits - ofits)) <= 1e-5
    assert not np.any(ctx5.W.cpu().numpy()[dead])


def test_edge_encoding_limits():
    # the largest input the compact encoding takes: J = 65536 (16-bit column
    # ids, the top column used) and one subject with exactly 65535 nonzeros
    # (16-bit in-subject offsets) in about 1300 rows
    from datagen.synth import gen_limits_case
    X = gen_limits_case()
    H0, V0, W0 = gen_init(X.J, X.K, 4, [170304219, 9, 1])
    _compare_one_iteration(X, 4, H0, V0, W0)


def test_get_q_matches_oracle_and_is_orthonormal():
    X, R = gen_config(1)
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, 1, 1])
    Xs = _xs(X)
    _, _, _, info = O.iterate(Xs, H0, V0, W0)
    ctx, _ = _gpu_run(X, R, H0, V0, W0, 1)
    Q = ctx.q(0, X.K).cpu().numpy().astype(np.float64)
    worst_orth, worst_q = 0.0, 0.0
    for k in range(X.K):
        r0, r1 = X.subj_ptr[k], X.subj_ptr[k + 1]
        Qk = Q[r0:r1]
        worst_orth = max(worst_orth, np.abs(Qk.T @ Qk - np.eye(R)).max())
        worst_q = max(worst_q, rel(Qk, info["Q"][k]))
    print("Q orth", worst_orth, "Q vs oracle", worst_q, flush=True)
    assert worst_orth <= 1e-5
    assert worst_q <= 1e-4


def test_planted_model_fit_goes_to_one():
    X, truth = gen_planted(K=40, J=30, R=3, ik_range=(6, 12), seed=[45], col_blocks=True)
    H0 = truth["H"] + 1e-2
    V0 = truth["V"] + 1e-2
    W0 = truth["W"] + 1e-2
    _, fits = _gpu_run(X, 3, H0 / np.linalg.norm(H0, axis=0), V0, W0, 100)
    print("planted fit", fits[[0, 9, 99]], flush=True)
    assert fits[-1] >= 1 - 1e-5
    assert np.all(np.diff(fits) >= -1e-6)


def test_subject_permutation_invariance():
    X, R = gen_config(1)
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, 1, 1])
    perm = np.random.default_rng(5).permutation(X.K)
    from datagen import concat_slices
    Xp = concat_slices([take_subjects(X, int(k), int(k) + 1) for k in perm])
    a, _ = _gpu_run(X, R, H0, V0, W0, 1)
    b, _ = _gpu_run(Xp, R, H0, V0, W0[perm], 1)
    Ma, Mb = a.mttkrp(), b.mttkrp()
    assert rel(Mb[0].cpu().numpy(), Ma[0].cpu().numpy()) <= 1e-6
    assert rel(Mb[1].cpu().numpy(), Ma[1].cpu().numpy()) <= 1e-6
    assert rel(Mb[2].cpu().numpy(), Ma[2].cpu().numpy()[perm]) <= 1e-6


def test_projection_matches_oracle():
    V, H = gen_serving_model()
    t, Xr = gen_serving_requests(24)
    model = B.Model(V, H)
    dX = B.DeviceSlices.from_slices(Xr)
    Q, w, loss = model.project(dX, n_steps=10)
    torch.cuda.synchronize()
    w = w.cpu().numpy().astype(np.float64)
    loss = loss.cpu().numpy()
    Xs = _xs(Xr)
    ws, ls = [], []
    for k in range(Xr.K):
        _, wo, lo = O.project(Xs[k], V.astype(np.float64), H, n_steps=10)
        ws.append(wo)
        ls.append(lo)
    ws = np.array(ws)
    err = rel(w, ws)
    print("projection w rel err", err, flush=True)
    assert err <= 1e-4
    # each request's w against the condition number of its final B = X V S H^T
    kap = kappa_of(Xs, H, V.astype(np.float64), ws)
    check_rows("projection w", w, ws, kap)
    nx = np.array([float(x.data @ x.data) for x in Xs])
    assert np.max(np.abs(loss - np.array(ls)) / nx) <= 1e-5


@pytest.mark.parametrize("R", [7, 17, 33])
def test_projection_other_ranks(R):
    V, H = gen_serving_model(J=800, R=R, density=0.2, seed=(170304219, 50 + R))
    _, Xr = gen_serving_requests(16, J=800, R=R, seed=(170304219, 50 + R))
    Q, w, loss = B.Model(V, H).project(B.DeviceSlices.from_slices(Xr), n_steps=10)
    torch.cuda.synchronize()
    w = w.cpu().numpy().astype(np.float64)
    Xs = _xs(Xr)
    ws = np.array([O.project(Xs[k], V.astype(np.float64), H, n_steps=10)[1]
                   for k in range(Xr.K)])
    err = rel(w, ws)
    print(f"R={R} projection w rel err", err, flush=True)
    assert err <= 1e-4
    check_rows("projection w", w, ws, kappa_of(Xs, H, V.astype(np.float64), ws))


def test_projection_alone_equals_in_the_mix():
    # each subject's result depends only on its own slice: projecting a request
    # alone or inside a batch gives the same bits
    V, H = gen_serving_model()
    _, Xr = gen_serving_requests(16)
    model = B.Model(V, H)
    Qb, wb, lb = model.project(B.DeviceSlices.from_slices(Xr), n_steps=10)
    torch.cuda.synchronize()
    for k in (0, 5, 15):
        Xk = take_subjects(Xr, k, k + 1)
        Q1, w1, l1 = model.project(B.DeviceSlices.from_slices(Xk), n_steps=10)
        torch.cuda.synchronize()
        r0, r1 = int(Xr.subj_ptr[k]), int(Xr.subj_ptr[k + 1])
        assert torch.equal(w1[0], wb[k])
        assert torch.equal(l1[0], lb[k])
        assert torch.equal(Q1, Qb[r0:r1])


def test_projection_q_is_orthonormal():
    V, H = gen_serving_model()
    _, Xr = gen_serving_requests(8)
    model = B.Model(V, H)
    Q, w, _ = model.project(B.DeviceSlices.from_slices(Xr), n_steps=10)
    Q = Q.cpu().numpy().astype(np.float64)
    Xs = _xs(Xr)
    for k in range(Xr.K):
        r0, r1 = Xr.subj_ptr[k], Xr.subj_ptr[k + 1]
        Qk = Q[r0:r1]
        assert np.abs(Qk.T @ Qk - np.eye(Qk.shape[1])).max() <= 1e-5
        Qo, _, _ = O.project(Xs[k], V.astype(np.float64), H, n_steps=10)
        assert rel(Qk, Qo) <= 1e-4


def test_invalid_input_is_rejected():
    X, R = gen_config(1)
    bad = X.col.copy()
    bad[5] = X.J + 3
    H0, V0, W0 = gen_init(X.J, X.K, R, [1, 1])
    dX = B.DeviceSlices(X.subj_ptr, X.row_ptr, bad, X.val, X.J)
    with pytest.raises(B.Parafac2Error) as e:
        B.Context(dX, R, H0, V0, W0)
    assert e.value.code == B.P2_EINVAL
    # a subject without rows (checked on the device during init)
    sp = np.concatenate([[0], X.subj_ptr])
    dX = B.DeviceSlices(sp, X.row_ptr, X.col, X.val, X.J)
    with pytest.raises(B.Parafac2Error) as e:
        B.Context(dX, R, np.eye(R), np.ones((X.J, R)), np.ones((X.K + 1, R)))
    assert e.value.code == B.P2_EINVAL and "no rows" in str(e.value)
