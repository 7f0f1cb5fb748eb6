"""CPU-only checks of the C ABI: the library loads, exports every function that
include/parafac2.h declares, validates inputs on the host, and plans launches
and workspaces that fit the hardware for every rank it is built for."""
import os
import re

import numpy as np
import pytest

from datagen import gen_config
from paper_1703_04219_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LDS_BYTES = 160 * 1024


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "parafac2.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(parafac2_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = B.load()
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(B.exported_symbols())
    assert lib.parafac2_abi_version() == 1


def test_validate_host_accepts_generated_input():
    X, R = gen_config(1)
    rc, msg = B.parafac2_validate_host(X.subj_ptr, X.row_ptr, X.col, X.val, X.J, R)
    assert rc == B.P2_OK and msg == ""


def _mutated(field, fn):
    X, R = gen_config(1)
    arrs = dict(subj_ptr=X.subj_ptr.copy(), row_ptr=X.row_ptr.copy(), col=X.col.copy(),
                val=X.val.copy())
    fn(arrs[field])
    return arrs, X.J, R


@pytest.mark.parametrize("case,field,fn,code,text", [
    ("col out of range", "col", lambda a: a.__setitem__(3, 100), B.P2_EINVAL, "out of range"),
    ("negative col", "col", lambda a: a.__setitem__(3, -1), B.P2_EINVAL, "out of range"),
    ("unsorted", "col", lambda a: a.__setitem__(slice(0, 2), a[0:2][::-1].copy()), B.P2_EINVAL,
     "increasing"),
    ("nan value", "val", lambda a: a.__setitem__(7, np.nan), B.P2_EINVAL, "non-finite"),
    ("inf value", "val", lambda a: a.__setitem__(7, np.inf), B.P2_EINVAL, "non-finite"),
])
def test_validate_host_rejects_bad_input(case, field, fn, code, text):
    arrs, J, R = _mutated(field, fn)
    rc, msg = B.parafac2_validate_host(arrs["subj_ptr"], arrs["row_ptr"], arrs["col"],
                                       arrs["val"], J, R)
    assert rc == code, (case, msg)
    assert text in msg


def test_validate_host_encoding_limits():
    # 16-bit column ids and in-subject nonzero offsets: J = 65536 and a subject
    # with 65535 nonzeros are accepted, one more of either is ENOTSUP
    from datagen.synth import gen_limits_case
    X = gen_limits_case()
    rc, msg = B.parafac2_validate_host(X.subj_ptr, X.row_ptr, X.col, X.val, X.J, 4)
    assert rc == B.P2_OK, msg
    rc, msg = B.parafac2_validate_host(X.subj_ptr, X.row_ptr, X.col, X.val, X.J + 1, 4)
    assert rc == B.P2_ENOTSUP and "J" in msg
    Y = gen_limits_case(big_nnz=65536)
    rc, msg = B.parafac2_validate_host(Y.subj_ptr, Y.row_ptr, Y.col, Y.val, Y.J, 4)
    assert rc == B.P2_ENOTSUP and "65535" in msg


def test_validate_host_subject_count_limit():
    # the per-subject passes visit subjects through a 32-bit position table;
    # the count is checked before any array is read
    import ctypes
    c = B.Csr(2**31, 10, 2**31 * 4, 0, 0, 0, 0, 0)
    buf = ctypes.create_string_buffer(512)
    rc = B.load().parafac2_validate_host(ctypes.byref(c), 4, buf, 512)
    assert rc == B.P2_ENOTSUP and "2^31" in buf.value.decode()
    c = B.Csr(2**31 - 1, 10, (2**31 - 1) * 4, 0, 0, 0, 0, 0)
    rc = B.load().parafac2_validate_host(ctypes.byref(c), 4, buf, 512)
    assert rc == B.P2_EINVAL and "NULL" in buf.value.decode()


def test_validate_host_rank_rules():
    X, _ = gen_config(1)  # I_k in [5, 20]
    # subjects with fewer rows than R are accepted (economy Procrustes factor)
    rc, msg = B.parafac2_validate_host(X.subj_ptr, X.row_ptr, X.col, X.val, X.J, 40)
    assert rc == B.P2_OK, msg
    # a subject with no rows is not
    sp = np.concatenate([[0], X.subj_ptr])
    rc, msg = B.parafac2_validate_host(sp, X.row_ptr, X.col, X.val, X.J, 5)
    assert rc == B.P2_EINVAL and "no rows" in msg
    rc, msg = B.parafac2_validate_host(X.subj_ptr, X.row_ptr, X.col, X.val, X.J, 41)
    assert rc == B.P2_ENOTSUP
    rc, msg = B.parafac2_validate_host(X.subj_ptr, X.row_ptr, X.col, X.val, X.J, 0)
    assert rc == B.P2_EINVAL


def test_validate_host_bad_offsets():
    X, R = gen_config(1)
    sp = X.subj_ptr.copy()
    sp[-1] += 1
    rc, _ = B.parafac2_validate_host(sp, X.row_ptr, X.col, X.val, X.J, R)
    assert rc == B.P2_EINVAL
    rp = X.row_ptr.copy()
    rp[5], rp[6] = rp[6], rp[5]
    rc, _ = B.parafac2_validate_host(X.subj_ptr, rp, X.col, X.val, X.J, R)
    assert rc == B.P2_EINVAL


@pytest.mark.parametrize("R", B.SUPPORTED_R)
def test_launch_plans_fit_the_lds(R):
    for kernel in range(5):
        threads, lds, max_hot = B.parafac2_launch_config(R, kernel)
        assert threads in (64, 128, 256, 512, 1024), (R, kernel, threads)
        assert 0 < lds <= LDS_BYTES, (R, kernel, lds)
        assert max_hot >= 0


@pytest.mark.parametrize("R", B.SUPPORTED_R)
def test_workspace_size_is_sane(R):
    # K=1e6, J=5000, 55M rows, 63M nnz: encoded slices ~0.5 GB plus
    # K*R*R*8 bytes of F per subject and, for the ranks with warm-started
    # eigen-solves, K*NC*R*4 bytes of kept bases; never wrapped around
    base = 63_000_000 * 6 + 55_000_000 * 2
    n = B.parafac2_workspace_size(1_000_000, 5000, 55_000_000, 63_000_000, R)
    f = R * R * 8  # F_k in FP64
    assert base + 1_000_000 * f <= n <= base + 1_000_000 * f + 2e9
    nc = R + (R & 1)
    per_subject = f + (nc * R * 4 if R <= 20 else 0)
    kept = B.parafac2_workspace_size(1_000_000, 5000, 55_000_000, 63_000_000, R,
                                     B.make_opts(keep_bases=True))
    assert base + 1_000_000 * per_subject <= kept <= base + 1_000_000 * per_subject + 2e9
    assert base + 1_000_000 * f <= n
    small = B.parafac2_workspace_size(10, 50, 100, 300, R)
    assert 0 < small < 64 * 2**20


def test_launch_config_rejects_unbuilt_rank():
    for R in (0, 41, 64):
        with pytest.raises(B.Parafac2Error) as e:
            B.parafac2_launch_config(R, 0)
        assert e.value.code in (B.P2_ENOTSUP, B.P2_EINVAL)


def test_init_rejects_a_short_workspace_before_touching_the_gpu():
    # the workspace size is checked on the host, before any HIP call: a buffer
    # one byte short of parafac2_workspace_size() is P2_EINVAL (the pointers
    # are never dereferenced, so placeholders serve on a CPU-only host)
    import ctypes
    X, R = gen_config(1)
    lib = B.load()
    need = B.parafac2_workspace_size(X.K, X.J, X.n_rows, X.nnz, R)
    fake = 1 << 20  # 256-byte aligned, never read
    c = B.Csr(X.K, X.J, X.n_rows, X.nnz, fake, fake, fake, fake)
    h = ctypes.c_void_p(0)
    opts = B.make_opts()
    rc = lib.parafac2_init(ctypes.byref(h), ctypes.byref(c), R, fake, fake, fake, fake, need - 1,
                           None, ctypes.byref(opts))
    assert rc == B.P2_EINVAL
    assert "workspace too small" in lib.parafac2_last_error().decode()
    assert not h.value
    # a misaligned workspace is refused the same way
    rc = lib.parafac2_init(ctypes.byref(h), ctypes.byref(c), R, fake, fake, fake, fake + 8, need,
                           None, ctypes.byref(opts))
    assert rc == B.P2_EINVAL and "aligned" in lib.parafac2_last_error().decode()


@pytest.mark.parametrize("R", [10, 20, 40])
def test_hot_column_requests_are_clamped_to_the_lds_plan(R):
    # a hot-column count above what the mode-2 LDS plan holds is clamped on
    # the host (the workspace of the partial sums is sized by the clamped
    # count), so no launch can be planned over the LDS budget
    _, _, max_hot = B.parafac2_launch_config(R, 2)
    assert 0 < max_hot
    sizes = dict(K=200_000, J=5000, n_rows=1_000_000, nnz=2_000_000, R=R)
    dflt = B.parafac2_workspace_size(**sizes)
    huge = B.parafac2_workspace_size(**sizes, opts=B.make_opts(hot_cols=10**6))
    at_max = B.parafac2_workspace_size(**sizes, opts=B.make_opts(hot_cols=max_hot))
    none = B.parafac2_workspace_size(**sizes, opts=B.make_opts(hot_cols=-1))
    assert huge == at_max == dflt
    assert none < dflt


def test_iterate_rejects_null_handles():
    lib = B.load()
    import ctypes
    nd = ctypes.c_int32(0)
    assert lib.parafac2_iterate(None, 1, None, None) == B.P2_EINVAL
    assert lib.parafac2_iterate_until(None, 5, 1e-3, ctypes.byref(nd), None, None) == B.P2_EINVAL
    assert lib.parafac2_get_u(None, 0, 1, None) == B.P2_EINVAL
