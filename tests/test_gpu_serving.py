"""GPU: the continuous-batching projection server.

A request's result depends only on its own slice, so the server must return
bitwise the same w, loss and Q as a projection of that request alone,
whatever batches it lands in; against the FP64 oracle the projection bar
holds (w within 1e-4 relative in aggregate)."""
import time

import numpy as np
import pytest

from datagen.synth import gen_serving_model, gen_serving_requests
from oracle import parafac2_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1703_04219_amd import binding as B  # noqa: E402


def _request(X, k):
    r0, r1 = int(X.subj_ptr[k]), int(X.subj_ptr[k + 1])
    rp = X.row_ptr[r0:r1 + 1]
    z0, z1 = int(rp[0]), int(rp[-1])
    return rp - rp[0], X.col[z0:z1], X.val[z0:z1]


def _alone(model, X, k):
    from datagen import take_subjects
    Q, w, loss = model.project(B.DeviceSlices.from_slices(take_subjects(X, k, k + 1)), n_steps=10)
    torch.cuda.synchronize()
    return Q.cpu().numpy(), w[0].cpu().numpy(), float(loss[0].cpu())


def _serve(server, X, order, burst):
    """Submit requests in `order`, `burst` at a time with polls in between;
    returns {id: (w, loss, Q)}."""
    got = {}
    i = 0
    while len(got) < len(order):
        for _ in range(burst):
            if i < len(order):
                assert server.submit(order[i], *_request(X, order[i])) == B.P2_OK
                i += 1
        ids, w, loss, qs = server.poll()
        for j, rid in enumerate(ids):
            got[int(rid)] = (w[j], loss[j], qs[j])
        if len(ids) == 0:
            time.sleep(1e-4)
    return got


@pytest.mark.parametrize("slots,max_requests,burst", [(3, 8, 5), (1, 1, 1), (4, 512, 40)])
def test_served_equals_alone(slots, max_requests, burst):
    V, H = gen_serving_model()
    _, X = gen_serving_requests(40)
    model = B.Model(V, H)
    server = B.Server(model, slots=slots, max_requests=max_requests, want_q=True)
    order = list(np.random.default_rng(3).permutation(X.K))
    got = _serve(server, X, order, burst)
    assert server.pending() == (0, 0, 0)
    for k in range(X.K):
        Qa, wa, la = _alone(model, X, k)
        w, loss, Q = got[k]
        assert np.array_equal(w.view(np.uint32), wa.view(np.uint32)), k
        assert loss == la
        assert np.array_equal(Q.view(np.uint32), Qa.view(np.uint32)), k


def test_served_matches_oracle():
    V, H = gen_serving_model()
    _, X = gen_serving_requests(16)
    model = B.Model(V, H)
    server = B.Server(model, slots=2, max_requests=4)
    got = {}
    for k in range(X.K):
        assert server.submit(k, *_request(X, k)) == B.P2_OK
    server.drain()
    ids, w, loss = server.poll()
    got = {int(i): w[j] for j, i in enumerate(ids)}
    Xs = O.slices_to_list(X.subj_ptr, X.row_ptr, X.col, X.val, X.J)
    wg = np.array([got[k] for k in range(X.K)], np.float64)
    wo = np.array([O.project(Xs[k], V.astype(np.float64), H, n_steps=10)[1] for k in range(X.K)])
    err = np.linalg.norm(wg - wo) / np.linalg.norm(wo)
    print("server w vs oracle", err, flush=True)
    assert err <= 1e-4


def test_server_rejects_bad_requests_and_bounds_the_queue():
    V, H = gen_serving_model()
    _, X = gen_serving_requests(4)
    model = B.Model(V, H)
    server = B.Server(model, slots=1, max_requests=4, max_nnz=4000, max_queue=2)
    rp, col, val = _request(X, 0)
    bad = col.copy()
    bad[0] = X.J
    with pytest.raises(B.Parafac2Error) as e:
        server.submit(0, rp, bad, val)
    assert e.value.code == B.P2_EINVAL
    with pytest.raises(B.Parafac2Error) as e:  # I < R
        server.submit(0, rp[:11] - rp[0], col[:int(rp[10])], val[:int(rp[10])])
    assert e.value.code == B.P2_EINVAL
    big_rp = np.arange(0, 50 * 100 + 1, 50, dtype=np.int64)  # 100 rows x 50 nnz > max_nnz
    with pytest.raises(B.Parafac2Error) as e:
        server.submit(0, big_rp, np.tile(np.arange(50, dtype=np.int32), 100),
                      np.ones(5000, np.float32))
    assert e.value.code == B.P2_EINVAL
    assert server.submit(1, *_request(X, 1)) == B.P2_OK
    assert server.submit(2, *_request(X, 2)) == B.P2_OK
    assert server.submit(3, *_request(X, 3)) == B.P2_EBUSY
    server.drain()
    ids, _, _ = server.poll()
    assert sorted(ids.tolist()) == [1, 2]
