"""The allocation-free projection entry point against the workspace one.

parafac2_project_noalloc builds the model state in the library's device
scratch array; its results must equal those of parafac2_model_create +
parafac2_project on the same inputs (same kernels; the V^T V sums may differ
in rounding order).  Two calls in a row, the second smaller (fewer requests,
smaller J and R), check that the shared scratch is rebuilt per call."""
import numpy as np
import pytest

from datagen import gen_slices
from datagen.synth import _uniform_int, gen_serving_model, gen_serving_requests

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1703_04219_amd import binding as B  # noqa: E402


def _maxrel(a, b):
    a = a.double().cpu()
    b = b.double().cpu()
    return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))


def _both(V, H, X, n_steps=10):
    dev = "cuda"
    Vd = torch.as_tensor(V, dtype=torch.float32, device=dev).contiguous()
    Hd = torch.as_tensor(H, dtype=torch.float64, device=dev).contiguous()
    dX = B.DeviceSlices.from_slices(X)
    R = V.shape[1]
    out = (torch.empty((X.n_rows, R), dtype=torch.float32, device=dev),
           torch.empty((X.K, R), dtype=torch.float32, device=dev),
           torch.empty((X.K,), dtype=torch.float64, device=dev))
    Qn, wn, ln = B.parafac2_project_noalloc(Vd, Hd, dX, n_steps, out=out)
    model = B.Model(V, H)
    Qm, wm, lm = model.project(dX, n_steps=n_steps)
    torch.cuda.synchronize()
    return (Qn, wn, ln), (Qm, wm, lm)


def test_noalloc_projection_equals_the_model_path_twice():
    V, H = gen_serving_model()
    _, X1 = gen_serving_requests(24)
    rng = np.random.default_rng(77)
    V2 = rng.random((3000, 10)).astype(np.float32)
    H2 = rng.standard_normal((10, 10))
    X2 = gen_slices(5, 3000, (10, 30), _uniform_int(1, 20), "uniform", [77])
    for name, (Vx, Hx, Xx) in (("J=5000 R=40, 24 requests", (V, H, X1)),
                               ("J=3000 R=10, 5 requests", (V2, H2, X2))):
        (Qn, wn, ln), (Qm, wm, lm) = _both(Vx, Hx, Xx)
        errs = (_maxrel(wn, wm), _maxrel(ln, lm), _maxrel(Qn, Qm))
        print(f"{name}: w {errs[0]:.1e}, loss {errs[1]:.1e}, Q {errs[2]:.1e}", flush=True)
        assert max(errs) <= 1e-5


def test_noalloc_rejects_model_state_beyond_the_scratch():
    V = torch.zeros((200_000, 40), dtype=torch.float32, device="cuda")
    H = torch.eye(40, dtype=torch.float64, device="cuda")
    X = gen_slices(1, 200_000, (40, 41), _uniform_int(1, 3), "uniform", [78])
    dX = B.DeviceSlices.from_slices(X)
    out = (None, torch.empty((1, 40), device="cuda"), None)
    with pytest.raises(B.Parafac2Error) as e:
        B.parafac2_project_noalloc(V, H, dX, 10, out=out)
    assert e.value.code == B.P2_EINVAL and "scratch" in str(e.value)
