"""Thin ctypes binding of libparafac2.so (argument marshalling only).

Every step of the hot path runs in the HIP library; this module only turns
torch device tensors into pointers and sizes, keeps the workspace alive and
maps status codes to exceptions.  torch is used for device memory and the
current stream, nothing else.  The functions named parafac2_* mirror the C
ABI of include/parafac2.h one to one.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libparafac2.so")

P2_OK, P2_EINVAL, P2_ENOMEM, P2_EDEVICE, P2_ESTATE, P2_ENOTSUP, P2_EBUSY = 0, -1, -2, -3, -4, -5, -6
_STATUS = {P2_EINVAL: "EINVAL", P2_ENOMEM: "ENOMEM", P2_EDEVICE: "EDEVICE",
           P2_ESTATE: "ESTATE", P2_ENOTSUP: "ENOTSUP", P2_EBUSY: "EBUSY"}

SUPPORTED_R = tuple(range(1, 41))


class Parafac2Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class Csr(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int64), ("J", ctypes.c_int64), ("n_rows", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("subj_ptr", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class Sched(ctypes.Structure):
    _fields_ = [("tile_rounds", ctypes.c_int32), ("dynamic", ctypes.c_int32),
                ("m2_tiles", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("m2_threads", ctypes.c_int32), ("m2_blocks", ctypes.c_int32),
                ("warm_polar", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Opts(ctypes.Structure):
    _fields_ = [("tau_polar", ctypes.c_double), ("tau_pinv", ctypes.c_double),
                ("hot_cols", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("sched", Sched), ("m2_capacity", ctypes.c_int32),
                ("keep_bases", ctypes.c_int32), ("nonneg", ctypes.c_int32),
                ("baseline", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_requests", ctypes.c_int32),
                ("max_rows", ctypes.c_int64), ("max_nnz", ctypes.c_int64),
                ("max_queue", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("want_q", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1703_04219_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "parafac2_abi_version": (ctypes.c_int, []),
        "parafac2_last_error": (ctypes.c_char_p, []),
        "parafac2_validate_host": (ctypes.c_int, [P(Csr), i32, ctypes.c_char_p, sz]),
        "parafac2_workspace_size": (ctypes.c_int, [P(Csr), i32, P(Opts), P(sz)]),
        "parafac2_init": (ctypes.c_int, [P(vp), P(Csr), i32, vp, vp, vp, vp, sz, vp, P(Opts)]),
        "parafac2_iterate": (ctypes.c_int, [vp, i32, P(ctypes.c_double), P(ctypes.c_double)]),
        "parafac2_iterate_until": (ctypes.c_int, [vp, i32, ctypes.c_double, P(i32),
                                                  P(ctypes.c_double), P(ctypes.c_double)]),
        "parafac2_get_mttkrp": (ctypes.c_int, [vp, vp, vp, vp]),
        "parafac2_get_q": (ctypes.c_int, [vp, i64, i64, vp]),
        "parafac2_get_u": (ctypes.c_int, [vp, i64, i64, vp]),
        "parafac2_set_profiling": (ctypes.c_int, [vp, i32]),
        "parafac2_get_profile": (ctypes.c_int, [vp, P(ctypes.c_double), P(ctypes.c_int64)]),
        "parafac2_launch_config": (ctypes.c_int, [i32, i32, P(i32), P(i64), P(i32)]),
        "parafac2_destroy": (None, [vp]),
        "parafac2_model_workspace_size": (ctypes.c_int, [i64, i32, P(sz)]),
        "parafac2_model_create": (ctypes.c_int, [P(vp), i64, i32, vp, vp, vp, sz, vp]),
        "parafac2_project": (ctypes.c_int, [vp, P(Csr), i32, vp, vp, vp, vp, vp]),
        "parafac2_model_destroy": (None, [vp]),
        "parafac2_project_noalloc": (ctypes.c_int, [i64, i32, vp, vp, P(Csr), i32, vp, vp, vp,
                                                    vp, vp]),
        "parafac2_set_sched": (ctypes.c_int, [vp, P(Sched)]),
        "parafac2_autotune": (ctypes.c_int, [vp, i32, P(Sched), P(ctypes.c_double)]),
        "parafac2_batch_workspace_size": (ctypes.c_int, [P(vp), i32, P(sz)]),
        "parafac2_batch_create": (ctypes.c_int, [P(vp), P(vp), i32, vp, sz, vp, P(Sched)]),
        "parafac2_batch_iterate": (ctypes.c_int, [vp, i32, P(ctypes.c_double),
                                                  P(ctypes.c_double)]),
        "parafac2_batch_set_sched": (ctypes.c_int, [vp, P(Sched)]),
        "parafac2_batch_autotune": (ctypes.c_int, [vp, i32, P(Sched), P(ctypes.c_double)]),
        "parafac2_batch_set_profiling": (ctypes.c_int, [vp, i32]),
        "parafac2_batch_get_profile": (ctypes.c_int, [vp, P(ctypes.c_double), P(ctypes.c_int64)]),
        "parafac2_batch_destroy": (None, [vp]),
        "parafac2_server_workspace_size": (ctypes.c_int, [vp, P(ServerOpts), P(sz)]),
        "parafac2_server_create": (ctypes.c_int, [P(vp), vp, P(ServerOpts), vp, sz]),
        "parafac2_server_submit": (ctypes.c_int, [vp, i64, i32, vp, vp, vp]),
        "parafac2_server_poll": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, i64, vp, P(i32)]),
        "parafac2_server_pending": (ctypes.c_int, [vp, P(i64), P(i64), P(i64)]),
        "parafac2_server_drain": (ctypes.c_int, [vp]),
        "parafac2_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> list:
    return ["parafac2_abi_version", "parafac2_last_error", "parafac2_validate_host",
            "parafac2_workspace_size", "parafac2_init", "parafac2_iterate",
            "parafac2_iterate_until", "parafac2_get_mttkrp", "parafac2_get_q",
            "parafac2_get_u", "parafac2_set_profiling",
            "parafac2_get_profile", "parafac2_launch_config", "parafac2_destroy",
            "parafac2_model_workspace_size", "parafac2_model_create", "parafac2_project",
            "parafac2_model_destroy", "parafac2_project_noalloc", "parafac2_set_sched", "parafac2_autotune",
            "parafac2_batch_workspace_size", "parafac2_batch_create", "parafac2_batch_iterate",
            "parafac2_batch_set_sched", "parafac2_batch_autotune", "parafac2_batch_set_profiling",
            "parafac2_batch_get_profile", "parafac2_batch_destroy",
            "parafac2_server_workspace_size", "parafac2_server_create", "parafac2_server_submit",
            "parafac2_server_poll", "parafac2_server_pending", "parafac2_server_drain",
            "parafac2_server_destroy"]


def _check(rc: int):
    if rc != P2_OK:
        raise Parafac2Error(rc, load().parafac2_last_error().decode())


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def make_sched(tile_rounds=0, dynamic=0, m2_tiles=0, graph=0, m2_threads=0, m2_blocks=0,
               warm_polar=0) -> Sched:
    return Sched(tile_rounds, dynamic, m2_tiles, graph, m2_threads, m2_blocks, warm_polar)


def make_opts(tau_polar=0.0, tau_pinv=0.0, hot_cols=0, max_sweeps=0, sched=None,
              m2_capacity=0, keep_bases=False, nonneg=False, baseline=False) -> Opts:
    o = Opts()
    o.tau_polar, o.tau_pinv, o.hot_cols, o.max_sweeps = tau_polar, tau_pinv, hot_cols, max_sweeps
    if sched is not None:
        o.sched = sched if isinstance(sched, Sched) else make_sched(**sched)
    o.m2_capacity = m2_capacity
    o.keep_bases = 1 if keep_bases else 0
    o.nonneg = 1 if nonneg else 0
    o.baseline = 1 if baseline else 0
    return o


# ---------------------------------------------------------------------------
# host-side helpers (no GPU)
# ---------------------------------------------------------------------------

def host_csr(subj_ptr: np.ndarray, row_ptr: np.ndarray, col: np.ndarray, val: np.ndarray,
             J: int) -> tuple:
    """A Csr over host numpy arrays (kept alive by the returned tuple)."""
    arrs = (np.ascontiguousarray(subj_ptr, dtype=np.int64),
            np.ascontiguousarray(row_ptr, dtype=np.int64),
            np.ascontiguousarray(col, dtype=np.int32),
            np.ascontiguousarray(val, dtype=np.float32))
    c = Csr(len(arrs[0]) - 1, J, len(arrs[1]) - 1, len(arrs[2]),
            arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data, arrs[3].ctypes.data)
    return c, arrs


def parafac2_validate_host(subj_ptr, row_ptr, col, val, J: int, R: int) -> tuple:
    """Host-only validation; returns (status, message)."""
    c, keep = host_csr(subj_ptr, row_ptr, col, val, J)
    buf = ctypes.create_string_buffer(512)
    rc = load().parafac2_validate_host(ctypes.byref(c), R, buf, 512)
    return rc, buf.value.decode()


def parafac2_workspace_size(K: int, J: int, n_rows: int, nnz: int, R: int,
                            opts: Optional[Opts] = None) -> int:
    c = Csr(K, J, n_rows, nnz, 0, 0, 0, 0)
    n = ctypes.c_size_t(0)
    _check(load().parafac2_workspace_size(ctypes.byref(c), R,
                                          ctypes.byref(opts) if opts is not None else None,
                                          ctypes.byref(n)))
    return n.value


def parafac2_launch_config(R: int, kernel: int) -> tuple:
    """(threads, lds_bytes, max_hot) of a kernel for rank R (no GPU)."""
    t = ctypes.c_int32(0)
    lds = ctypes.c_int64(0)
    mh = ctypes.c_int32(0)
    _check(load().parafac2_launch_config(R, kernel, ctypes.byref(t), ctypes.byref(lds),
                                         ctypes.byref(mh)))
    return t.value, lds.value, mh.value


def parafac2_model_workspace_size(J: int, R: int) -> int:
    n = ctypes.c_size_t(0)
    _check(load().parafac2_model_workspace_size(J, R, ctypes.byref(n)))
    return n.value


# ---------------------------------------------------------------------------
# device objects
# ---------------------------------------------------------------------------

class DeviceSlices:
    """The concatenated CSR of {X_k} as torch device tensors."""

    def __init__(self, subj_ptr, row_ptr, col, val, J: int, device="cuda"):
        import torch
        self.subj_ptr = torch.as_tensor(np.asarray(subj_ptr, np.int64), device=device)
        self.row_ptr = torch.as_tensor(np.asarray(row_ptr, np.int64), device=device)
        self.col = torch.as_tensor(np.asarray(col, np.int32), device=device)
        self.val = torch.as_tensor(np.asarray(val, np.float32), device=device)
        self.J = int(J)

    @classmethod
    def from_slices(cls, X, device="cuda"):
        return cls(X.subj_ptr, X.row_ptr, X.col, X.val, X.J, device)

    @property
    def K(self):
        return int(self.subj_ptr.shape[0] - 1)

    def csr(self) -> Csr:
        return Csr(self.K, self.J, int(self.row_ptr.shape[0] - 1), int(self.col.shape[0]),
                   _ptr(self.subj_ptr), _ptr(self.row_ptr), _ptr(self.col), _ptr(self.val))


def _workspace(nbytes: int, device="cuda"):
    import torch
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


class Context:
    """One decomposition (parafac2_init / parafac2_iterate / ...)."""

    def __init__(self, X: DeviceSlices, R: int, H, V, W, opts: Optional[Opts] = None,
                 stream=None):
        import torch
        self.lib = load()
        self.X, self.R = X, int(R)
        dev = X.val.device
        self.H = torch.as_tensor(H, dtype=torch.float64, device=dev).contiguous().clone()
        self.V = torch.as_tensor(V, dtype=torch.float32, device=dev).contiguous().clone()
        self.W = torch.as_tensor(W, dtype=torch.float32, device=dev).contiguous().clone()
        assert self.H.shape == (R, R) and self.V.shape == (X.J, R) and self.W.shape == (X.K, R)
        csr = X.csr()
        self.opts = opts if opts is not None else make_opts()
        self.ws_bytes = parafac2_workspace_size(csr.K, csr.J, csr.n_rows, csr.nnz, self.R,
                                                self.opts)
        self._ws, wsp = _workspace(self.ws_bytes, dev)
        self.stream = stream
        h = ctypes.c_void_p(0)
        _check(self.lib.parafac2_init(ctypes.byref(h), ctypes.byref(csr), self.R, _ptr(self.H),
                                      _ptr(self.V), _ptr(self.W), wsp, self.ws_bytes,
                                      _stream_handle(stream), ctypes.byref(self.opts)))
        self.handle = h

    def iterate(self, n: int, with_fit: bool = True, with_loss: bool = False):
        """Fits of the n iterations (or None); with_loss: (fits, losses)."""
        fit = (ctypes.c_double * n)() if with_fit else None
        loss = (ctypes.c_double * n)() if with_loss else None
        _check(self.lib.parafac2_iterate(self.handle, n, fit, loss))
        fits = np.array(fit[:], dtype=np.float64) if with_fit else None
        if with_loss:
            return fits, np.array(loss[:], dtype=np.float64)
        return fits

    def iterate_until(self, max_iters: int, tol: float):
        """(fits, losses) of the iterations run until the relative loss change
        is at most tol (parafac2_iterate_until)."""
        fit = (ctypes.c_double * max(max_iters, 1))()
        loss = (ctypes.c_double * max(max_iters, 1))()
        nd = ctypes.c_int32(0)
        _check(self.lib.parafac2_iterate_until(self.handle, max_iters, float(tol),
                                               ctypes.byref(nd), fit, loss))
        n = nd.value
        return np.array(fit[:n], dtype=np.float64), np.array(loss[:n], dtype=np.float64)

    def mttkrp(self):
        import torch
        dev = self.X.val.device
        M1 = torch.empty((self.R, self.R), dtype=torch.float64, device=dev)
        M2 = torch.empty((self.X.J, self.R), dtype=torch.float32, device=dev)
        M3 = torch.empty((self.X.K, self.R), dtype=torch.float32, device=dev)
        _check(self.lib.parafac2_get_mttkrp(self.handle, _ptr(M1), _ptr(M2), _ptr(M3)))
        return M1, M2, M3

    def q(self, k0: int, k1: int):
        import torch
        sp = self.X.subj_ptr
        nrows = int(sp[k1].item() - sp[k0].item())
        Q = torch.empty((nrows, self.R), dtype=torch.float32, device=self.X.val.device)
        _check(self.lib.parafac2_get_q(self.handle, k0, k1, _ptr(Q)))
        return Q

    def u(self, k0: int, k1: int):
        """U_k = Q_k H of subjects [k0, k1) (parafac2_get_u)."""
        import torch
        sp = self.X.subj_ptr
        nrows = int(sp[k1].item() - sp[k0].item())
        U = torch.empty((nrows, self.R), dtype=torch.float32, device=self.X.val.device)
        _check(self.lib.parafac2_get_u(self.handle, k0, k1, _ptr(U)))
        return U

    PHASES = ("alpha", "solve_h", "mode2", "vupdate", "gamma", "fit")

    def set_profiling(self, on: bool):
        _check(self.lib.parafac2_set_profiling(self.handle, 1 if on else 0))

    def profile(self) -> dict:
        ms = (ctypes.c_double * 6)()
        n = (ctypes.c_int64 * 6)()
        _check(self.lib.parafac2_get_profile(self.handle, ms, n))
        return {p: (ms[i], n[i]) for i, p in enumerate(self.PHASES)}

    def set_sched(self, sched: Sched):
        _check(self.lib.parafac2_set_sched(self.handle, ctypes.byref(sched)))

    def autotune(self, iters_per_trial: int = 2) -> tuple:
        """(chosen Sched, ms per iteration); the trials advance the decomposition."""
        sc = Sched()
        ms = ctypes.c_double(0)
        _check(self.lib.parafac2_autotune(self.handle, iters_per_trial, ctypes.byref(sc),
                                          ctypes.byref(ms)))
        return sc, ms.value

    def close(self):
        if getattr(self, "handle", None):
            self.lib.parafac2_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several contexts iterated in lock step (parafac2_batch_*)."""

    def __init__(self, ctxs, sched: Optional[Sched] = None, stream=None):
        import torch
        self.lib = load()
        self.ctxs = list(ctxs)  # keeps the contexts alive
        n = len(self.ctxs)
        self._arr = (ctypes.c_void_p * n)(*[c.handle.value for c in self.ctxs])
        nb = ctypes.c_size_t(0)
        _check(self.lib.parafac2_batch_workspace_size(self._arr, n, ctypes.byref(nb)))
        self.ws_bytes = nb.value
        self._ws, wsp = _workspace(self.ws_bytes, self.ctxs[0].X.val.device)
        h = ctypes.c_void_p(0)
        _check(self.lib.parafac2_batch_create(ctypes.byref(h), self._arr, n, wsp, self.ws_bytes,
                                              _stream_handle(stream),
                                              ctypes.byref(sched) if sched is not None else None))
        self.handle = h

    def iterate(self, n: int, with_fit: bool = True) -> Optional[np.ndarray]:
        """Fits as an (n, len(ctxs)) array (or None)."""
        nc = len(self.ctxs)
        fit = (ctypes.c_double * (n * nc))() if with_fit else None
        _check(self.lib.parafac2_batch_iterate(self.handle, n, fit, None))
        return np.array(fit[:], dtype=np.float64).reshape(n, nc) if with_fit else None

    def set_sched(self, sched: Sched):
        _check(self.lib.parafac2_batch_set_sched(self.handle, ctypes.byref(sched)))

    def autotune(self, iters_per_trial: int = 2) -> tuple:
        sc = Sched()
        ms = ctypes.c_double(0)
        _check(self.lib.parafac2_batch_autotune(self.handle, iters_per_trial, ctypes.byref(sc),
                                                ctypes.byref(ms)))
        return sc, ms.value

    def set_profiling(self, on: bool):
        _check(self.lib.parafac2_batch_set_profiling(self.handle, 1 if on else 0))

    def profile(self) -> dict:
        ms = (ctypes.c_double * 6)()
        n = (ctypes.c_int64 * 6)()
        _check(self.lib.parafac2_batch_get_profile(self.handle, ms, n))
        return {p: (ms[i], n[i]) for i, p in enumerate(Context.PHASES)}

    def close(self):
        if getattr(self, "handle", None):
            self.lib.parafac2_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """Fixed (V, H) for projecting new subjects (parafac2_model_create / parafac2_project)."""

    def __init__(self, V, H, stream=None, device="cuda"):
        import torch
        self.lib = load()
        self.V = torch.as_tensor(V, dtype=torch.float32, device=device).contiguous()
        self.H = torch.as_tensor(H, dtype=torch.float64, device=device).contiguous()
        self.J, self.R = int(self.V.shape[0]), int(self.V.shape[1])
        self.ws_bytes = parafac2_model_workspace_size(self.J, self.R)
        self._ws, wsp = _workspace(self.ws_bytes, device)
        h = ctypes.c_void_p(0)
        _check(self.lib.parafac2_model_create(ctypes.byref(h), self.J, self.R, _ptr(self.V),
                                              _ptr(self.H), wsp, self.ws_bytes,
                                              _stream_handle(stream)))
        self.handle = h

    def project(self, X: DeviceSlices, n_steps: int = 10, w0=None, want_q: bool = True,
                stream=None, out=None):
        """Returns (Q, w, loss) device tensors for the K subjects of X."""
        import torch
        dev = X.val.device
        K = X.K
        n_rows = int(X.row_ptr.shape[0] - 1)
        if out is None:
            Q = torch.empty((n_rows, self.R), dtype=torch.float32, device=dev) if want_q else None
            w = torch.empty((K, self.R), dtype=torch.float32, device=dev)
            loss = torch.empty((K,), dtype=torch.float64, device=dev)
        else:
            Q, w, loss = out
        csr = X.csr()
        _check(self.lib.parafac2_project(self.handle, ctypes.byref(csr), n_steps, _ptr(w0),
                                         _ptr(Q), _ptr(w), _ptr(loss),
                                         _stream_handle(stream)))
        return Q, w, loss

    def close(self):
        if getattr(self, "handle", None):
            self.lib.parafac2_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching projection server over a Model (parafac2_server_*)."""

    def __init__(self, model: Model, slots=0, max_requests=0, max_rows=0, max_nnz=0,
                 max_queue=0, n_steps=0, want_q=False, poll_cap=4096):
        self.lib = load()
        self.model = model  # the model must outlive the server
        self.R = model.R
        self.opts = ServerOpts(slots, max_requests, max_rows, max_nnz, max_queue, n_steps,
                               1 if want_q else 0)
        nb = ctypes.c_size_t(0)
        _check(self.lib.parafac2_server_workspace_size(model.handle, ctypes.byref(self.opts),
                                                       ctypes.byref(nb)))
        self.ws_bytes = nb.value
        self._ws, wsp = _workspace(self.ws_bytes, model.V.device)
        h = ctypes.c_void_p(0)
        _check(self.lib.parafac2_server_create(ctypes.byref(h), model.handle,
                                               ctypes.byref(self.opts), wsp, self.ws_bytes))
        self.handle = h
        self.want_q = bool(want_q)
        self._cap = int(poll_cap)
        self._ids = np.zeros(self._cap, np.int64)
        self._w = np.zeros((self._cap, self.R), np.float32)
        self._loss = np.zeros(self._cap, np.float64)
        self._qrows = np.zeros(self._cap, np.int32)
        self._qcap = self._cap * 128 if want_q else 0
        self._q = np.zeros((max(self._qcap, 1), self.R), np.float32)
        self._n = ctypes.c_int32(0)

    def submit(self, rid: int, row_ptr: np.ndarray, col: np.ndarray, val: np.ndarray) -> int:
        """Queue a request (host arrays, row_ptr from 0); returns the status
        (P2_OK or P2_EBUSY; other errors raise)."""
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float32)
        rc = self.lib.parafac2_server_submit(self.handle, int(rid), int(row_ptr.shape[0] - 1),
                                             row_ptr.ctypes.data, col.ctypes.data,
                                             val.ctypes.data)
        if rc not in (P2_OK, P2_EBUSY):
            _check(rc)
        return rc

    def poll(self):
        """(ids, w, loss[, q list]) of the requests finished since the last poll."""
        _check(self.lib.parafac2_server_poll(
            self.handle, self._cap, self._ids.ctypes.data, self._w.ctypes.data,
            self._loss.ctypes.data, self._q.ctypes.data if self.want_q else None, self._qcap,
            self._qrows.ctypes.data if self.want_q else None, ctypes.byref(self._n)))
        n = self._n.value
        out = (self._ids[:n].copy(), self._w[:n].copy(), self._loss[:n].copy())
        if self.want_q:
            qs, r0 = [], 0
            for r in self._qrows[:n]:
                qs.append(self._q[r0:r0 + r].copy())
                r0 += int(r)
            out = out + (qs,)
        return out

    def pending(self) -> tuple:
        a, b, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
        _check(self.lib.parafac2_server_pending(self.handle, ctypes.byref(a), ctypes.byref(b),
                                                ctypes.byref(c)))
        return a.value, b.value, c.value

    def drain(self):
        _check(self.lib.parafac2_server_drain(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.parafac2_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# C-ABI names at module level -------------------------------------------------

def parafac2_init(X: DeviceSlices, R: int, H, V, W, opts: Optional[Opts] = None,
                  stream=None) -> Context:
    return Context(X, R, H, V, W, opts, stream)


def parafac2_iterate(ctx: Context, n_iters: int, with_fit: bool = True):
    return ctx.iterate(n_iters, with_fit)


def parafac2_get_mttkrp(ctx: Context):
    return ctx.mttkrp()


def parafac2_iterate_until(ctx: Context, max_iters: int, tol: float):
    return ctx.iterate_until(max_iters, tol)


def parafac2_get_q(ctx: Context, k0: int, k1: int):
    return ctx.q(k0, k1)


def parafac2_get_u(ctx: Context, k0: int, k1: int):
    return ctx.u(k0, k1)


def parafac2_set_sched(ctx: Context, sched: Sched):
    return ctx.set_sched(sched)


def parafac2_autotune(ctx: Context, iters_per_trial: int = 2):
    return ctx.autotune(iters_per_trial)


def parafac2_batch_create(ctxs, sched: Optional[Sched] = None, stream=None) -> Batch:
    return Batch(ctxs, sched, stream)


def parafac2_batch_iterate(batch: Batch, n_iters: int, with_fit: bool = True):
    return batch.iterate(n_iters, with_fit)


def parafac2_batch_autotune(batch: Batch, iters_per_trial: int = 2):
    return batch.autotune(iters_per_trial)


def parafac2_model_create(V, H, stream=None) -> Model:
    return Model(V, H, stream)


def parafac2_server_create(model: Model, **opts) -> Server:
    return Server(model, **opts)


def parafac2_project(model: Model, X: DeviceSlices, n_steps: int = 10, w0=None,
                     want_q: bool = True, stream=None):
    return model.project(X, n_steps, w0, want_q, stream)


def parafac2_project_noalloc(V, H, X: DeviceSlices, n_steps: int = 10, w0=None, out=None,
                             stream=None):
    """Projection with the model state in the library's device scratch (no
    workspace); V (J x R float32) and H (R x R float64) are device tensors and
    out = (Q, w, loss) device tensors of the right shapes (Q may be None)."""
    Q, w, loss = out
    csr = X.csr()
    _check(load().parafac2_project_noalloc(int(V.shape[0]), int(V.shape[1]), _ptr(V), _ptr(H),
                                           ctypes.byref(csr), n_steps, _ptr(w0), _ptr(Q),
                                           _ptr(w), _ptr(loss), _stream_handle(stream)))
    return Q, w, loss
