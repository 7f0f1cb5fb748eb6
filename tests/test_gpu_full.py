"""GPU parity at the full sizes of the large workloads, in the launch
configurations bench.py times (the schedule its autotuner settles on and the
default one), and of the 64-problem batch against its problems run alone.

The FP64 oracle's first iteration on each full workload (K = 1,000,000
subjects; R = 10 with 63M nonzeros, R = 40 with 490M) is stored in
tests/golden/full_c<cfg>_iter1.npz, written by tests/golden/make_full_golden.py
(which calls only datagen/ and oracle/).  The GPU's first iteration from the
same state is compared with it element by element (tests/_cmp.py):
  * M1, M2, H_{t+1}, V_{t+1} whole: largest entrywise error <= 1e-4 of the
    largest entry;
  * M3 and W_{t+1} rows of 1002 sampled subjects: relative error per subject
    <= 1e-4 for kappa(B_k) <= 1e3, scaled by kappa / 1e3 above;
  * the fit: absolute error <= 1e-5;
  * Q_k^T Q_k = I within 1e-5 for the sampled subjects with kappa <= 1e3.

The inputs are drawn when the module is imported (during collection, before
any test has created a GPU context), so the generator can use its worker pool.
"""
import os

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

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_INPUTS = {cfg: gen_config(cfg) for cfg in (2, 3)}


def _arrays(X):
    return X.subj_ptr, X.row_ptr, X.col, X.val, X.J


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("cfg,sched", [
    (2, dict(tile_rounds=8, dynamic=1, m2_tiles=256)),
    (2, dict()),
    (3, dict(tile_rounds=16, dynamic=1)),
])
def test_full_size_matches_oracle(cfg, sched):
    X, R = _INPUTS[cfg]
    path = os.path.join(GOLDEN, f"full_c{cfg}_iter1.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_full_golden.py {cfg})")
    g = np.load(path, allow_pickle=False)
    assert (int(g["K"]), int(g["J"]), int(g["R"]), int(g["nnz"])) == (X.K, X.J, R, X.nnz)
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, cfg, 1])
    print(f"config {cfg}: K={X.K} nnz={X.nnz} R={R} schedule {sched}", flush=True)
    opts = B.make_opts(sched=B.make_sched(**sched)) if sched else None
    ctx = B.Context(B.DeviceSlices.from_slices(X), R, H0, V0, W0, opts)
    fit = ctx.iterate(1)[0]
    torch.cuda.synchronize()
    M1, M2, M3 = (t.cpu().numpy() for t in ctx.mttkrp())
    errs = {}
    check_shared(errs, "M1", M1, g["M1"])
    check_shared(errs, "M2", M2, g["M2"])
    check_shared(errs, "H", ctx.H.cpu().numpy(), g["H1"])
    check_shared(errs, "V", ctx.V.cpu().numpy(), g["V1"])
    idx, kap = g["idx"], g["kappa_s"]
    e3 = check_rows("M3 (sampled)", M3[idx], g["M3s"], kap)
    ew = check_rows("W (sampled)", ctx.W.cpu().numpy()[idx], g["W1s"], kap)
    errs["fit"] = abs(float(fit) - float(g["fit"]))
    # Q_k^T Q_k = I where B_k has full rank with condition number <= 1e3 over
    # all R singular values (a rank-deficient B_k gives the projector onto its
    # row space on the GPU)
    sub = [O.slices_to_list(*_arrays(take_subjects(X, int(k), int(k) + 1)))[0] for k in idx]
    kap_full = kappa_of(sub, H0, V0, W0[idx], cut=0.0)
    worst = 0.0
    for k, kp in zip(idx, kap_full):
        if 0 < kp <= 1e3:
            Qk = ctx.q(int(k), int(k) + 1).cpu().numpy().astype(np.float64)
            worst = max(worst, float(np.abs(Qk.T @ Qk - np.eye(R)).max()))
    print(f"errors: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()) +
          f", M3 rows {e3.max():.2e}, W rows {ew.max():.2e}, Q^T Q - I {worst:.1e}", flush=True)
    assert errs["fit"] <= 1e-5
    assert worst <= 1e-5


def test_full_size_batch_equals_problems_alone():
    # the 64-problem workload at full size (K log-uniform in [1000, 50000],
    # R in {5, 10, 20}, about 348M nonzeros), batched in the schedule the
    # bench's autotuner settles on (graph replay, dynamic tiles of one round,
    # the default mode-2 blocks), against each problem run on its own
    # context: one
    # iteration from the same state agrees to 1e-5 (only the order of float
    # atomics differs)
    from datagen.synth import gen_batched_problem, gen_batched_specs
    specs = gen_batched_specs(64)
    probs = []
    for i, sp in enumerate(specs):
        X = gen_batched_problem(sp)
        H0, V0, W0 = gen_init(X.J, X.K, sp["R"], [170304219, 4, 7, i])
        probs.append((X, sp["R"], H0, V0, W0))
    nnz = sum(p[0].nnz for p in probs)
    print(f"64 problems, {nnz} nnz", flush=True)
    alone = []
    for X, R, H0, V0, W0 in probs:
        c = B.Context(B.DeviceSlices.from_slices(X), R, H0, V0, W0)
        c.iterate(1)
        alone.append((c.H.cpu().numpy().copy(), c.V.cpu().numpy().copy(),
                      c.W.cpu().numpy().copy()))
        del c
    torch.cuda.synchronize()
    ctxs = [B.Context(B.DeviceSlices.from_slices(X), R, H0, V0, W0)
            for X, R, H0, V0, W0 in probs]
    batch = B.Batch(ctxs, B.make_sched(tile_rounds=1, dynamic=1, graph=1))
    batch.iterate(1)
    torch.cuda.synchronize()
    worst = 0.0
    for c, ref in zip(ctxs, alone):
        got = (c.H.cpu().numpy(), c.V.cpu().numpy(), c.W.cpu().numpy())
        worst = max(worst, max(rel(x, y) for x, y in zip(got, ref)))
    print(f"batched vs alone, worst factor difference {worst:.2e}", flush=True)
    assert worst <= 1e-5
