"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

import paper_1512_06500_amd as eda

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eda.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(eda_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return eda.load_library()


@pytest.fixture()
def handle(lib):
    h = ctypes.c_void_p()
    st = lib.eda_create(ctypes.byref(h), None)
    assert st in (eda.EDA_OK, eda.EDA_ERR_HIP)
    assert h.value is not None
    yield h
    lib.eda_destroy(h)


def test_library_exports_every_declared_symbol(lib):
    declared = header_functions()
    assert set(declared) == set(eda.EXPORTED_SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name


def test_strerror_covers_every_status(lib):
    for s in range(8):
        msg = lib.eda_strerror(s).decode()
        assert msg and msg != "unknown status"
    assert lib.eda_strerror(99).decode() == "unknown status"


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


@pytest.mark.parametrize("d,n,k,ldw,ldb,storage", [
    (1, 10, 2, 1, 1, 0),      # d < 2
    (100, 10, 1, 100, 100, 0),  # k < 2
    (100, 3, 4, 100, 100, 0),   # n < k
    (100, 10, 3, 99, 100, 0),   # ldw < d
    (100, 10, 3, 100, 50, 0),   # ldb < d
    (100, 10, 3, 100, 100, 9),  # unknown storage
    (100, 10, 3, 100, 100, 4),  # one past the last storage type
    (5000, 2050, 10, 5000, 5000, 0),  # n > 2048
])
def test_prepare_rejects_bad_arguments(lib, handle, d, n, k, ldw, ldb, storage):
    st = lib.eda_prepare(handle, d, n, k, FAKE, ldw, FAKE, ldb, storage)
    assert st == eda.EDA_ERR_ARG
    assert lib.eda_last_error(handle).decode()


def test_prepare_null_factor(lib, handle):
    assert lib.eda_prepare(handle, 100, 10, 3, None, 100, FAKE, 100, 0) == eda.EDA_ERR_ARG


def test_calls_before_prepare_report_state(lib, handle):
    ls = ctypes.c_double()
    assert lib.eda_expmv(handle, 0, -1.0, 1, FAKE, 10, FAKE, 10, 0, ctypes.byref(ls)) == eda.EDA_ERR_STATE
    assert lib.eda_opmv(handle, 0, 1, FAKE, 10, FAKE, 10, 0, ctypes.byref(ls)) == eda.EDA_ERR_STATE
    assert lib.eda_gram(handle, FAKE, 10) == eda.EDA_ERR_STATE
    o = eda.SolveOpts()
    buf = (ctypes.c_double * 4)()
    info = eda.Info()
    assert lib.eda_solve(handle, 2, 1e-8, ctypes.byref(o), buf, buf, FAKE, 10, buf,
                         ctypes.byref(info)) == eda.EDA_ERR_STATE
    assert lib.eda_solve_direct(handle, 2, buf, buf, FAKE, 10, buf,
                                ctypes.byref(info)) == eda.EDA_ERR_STATE


def test_expmv_rejects_bad_which_and_c(lib, handle):
    ls = ctypes.c_double()
    assert lib.eda_expmv(handle, 5, -1.0, 1, FAKE, 10, FAKE, 10, 0, ctypes.byref(ls)) == eda.EDA_ERR_ARG
    assert lib.eda_expmv(handle, 0, float("nan"), 1, FAKE, 10, FAKE, 10, 0,
                         ctypes.byref(ls)) == eda.EDA_ERR_ARG
    assert lib.eda_opmv(handle, 7, 1, FAKE, 10, FAKE, 10, 0, ctypes.byref(ls)) == eda.EDA_ERR_ARG


@pytest.mark.parametrize("n,lda,ldz", [(0, 1, 1), (3000, 3000, 3000), (10, 9, 10), (10, 10, 9)])
def test_syev_rejects_bad_arguments(lib, handle, n, lda, ldz):
    assert lib.eda_syev(handle, n, FAKE, lda, FAKE, FAKE, ldz) == eda.EDA_ERR_ARG


def test_scatter_rejects_bad_counts(lib, handle):
    counts = (ctypes.c_int64 * 3)(2, 0, 3)
    assert lib.eda_scatter_factors(handle, 10, 5, 3, FAKE, 10, counts, FAKE, 10, FAKE,
                                   10) == eda.EDA_ERR_ARG
    counts = (ctypes.c_int64 * 3)(2, 2, 2)  # sums to 6, not 5
    assert lib.eda_scatter_factors(handle, 10, 5, 3, FAKE, 10, counts, FAKE, 10, FAKE,
                                   10) == eda.EDA_ERR_ARG
    counts = (ctypes.c_int64 * 2)(2, 3)
    assert lib.eda_scatter_factors(handle, 10, 5, 2, FAKE, 9, counts, FAKE, 10, FAKE,
                                   10) == eda.EDA_ERR_ARG


@pytest.mark.parametrize("d,N,b,storage", [
    (0, 100, 8, 0),     # d < 1
    (100, 0, 8, 0),     # N < 1
    (100, 100, 0, 0),   # b < 1
    (100, 100, 17, 0),  # b > 16
    (100, 100, 8, 9),   # unknown storage
])
def test_autotune_rejects_bad_arguments(lib, handle, d, N, b, storage):
    assert lib.eda_autotune(handle, d, N, b, storage, None, None, None) == eda.EDA_ERR_ARG
    assert lib.eda_last_error(handle).decode()


@pytest.mark.parametrize("d,t,ntr,nte,ldx,ldtr,ldte", [
    (0, 1, 4, 4, 1, 1, 1),        # d < 1
    (10, 0, 4, 4, 10, 10, 10),    # t < 1
    (10, 11, 4, 4, 10, 10, 10),   # t > d
    (2000, 1025, 4, 4, 2000, 2000, 2000),  # t > 1024
    (10, 2, 0, 4, 10, 10, 10),    # no training samples
    (10, 2, 4, 0, 10, 10, 10),    # no testing samples
    (10, 2, 4, 4, 9, 10, 10),     # ldx < d
    (10, 2, 4, 4, 10, 9, 10),     # ldtr < d
    (10, 2, 4, 4, 10, 10, 9),     # ldte < d
    (10, 2, 4, 2 ** 31, 10, 10, 10),  # more testing samples than workgroups
])
def test_nn_classify_rejects_bad_arguments(lib, handle, d, t, ntr, nte, ldx, ldtr, ldte):
    st = lib.eda_nn_classify(handle, d, t, FAKE, ldx, ntr, FAKE, ldtr, FAKE, nte, FAKE, ldte,
                             FAKE, FAKE, FAKE)
    assert st == eda.EDA_ERR_ARG
    assert lib.eda_last_error(handle).decode()
    assert lib.eda_nn_classify(handle, 10, 2, None, 10, 4, FAKE, 10, FAKE, 4, FAKE, 10, FAKE,
                               FAKE, FAKE) == eda.EDA_ERR_ARG


def test_null_handle(lib):
    assert lib.eda_prepare(None, 10, 4, 2, FAKE, 10, FAKE, 10, 0) == eda.EDA_ERR_ARG
    assert lib.eda_create(None, None) == eda.EDA_ERR_ARG
    lib.eda_destroy(None)  # no-op


def test_no_cpu_fallback_without_library(monkeypatch, tmp_path):
    """The product path fails loudly when the HIP library is missing."""
    monkeypatch.setattr(eda, "_lib", None)
    monkeypatch.setattr(eda, "library_path", lambda: str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        eda.load_library()


def _problem(eda, d=100, n=10, k=3, t=2, tol=1e-8):
    arr = (eda.Problem * 1)()
    r = (ctypes.c_double * 4)()
    arr[0] = eda.Problem(d, n, k, 0x1000, d, 0x2000, d, t, tol, r, r, 0x3000, d, r)
    return arr


@pytest.mark.parametrize("field,value", [
    ("d", 1), ("k", 1), ("n", 2), ("t", 0), ("t", 200), ("tol", 0.0), ("ldw", 5), ("ldx", 5),
])
def test_solve_batched_rejects_bad_problems(lib, handle, field, value):
    arr = _problem(eda)
    setattr(arr[0], field, value)
    st = lib.eda_solve_batched(handle, 1, arr, 0, None, None, None)
    assert st == eda.EDA_ERR_ARG
    assert lib.eda_last_error(handle).decode()


def test_solve_batched_rejects_bad_calls(lib, handle):
    arr = _problem(eda)
    assert lib.eda_solve_batched(handle, 0, arr, 0, None, None, None) == eda.EDA_ERR_ARG
    assert lib.eda_solve_batched(handle, 1, None, 0, None, None, None) == eda.EDA_ERR_ARG
    assert lib.eda_solve_batched(handle, 1, arr, 9, None, None, None) == eda.EDA_ERR_ARG
    o = eda.SolveOpts()
    o.start_block = 0x1000
    o.ld_start = 100
    assert lib.eda_solve_batched(handle, 1, arr, 0, ctypes.byref(o), None, None) == eda.EDA_ERR_ARG
    o = eda.SolveOpts()
    o.max_basis = 40
    assert lib.eda_solve_batched(handle, 1, arr, 0, ctypes.byref(o), None, None) == eda.EDA_ERR_ARG
    assert lib.eda_solve_batched(None, 1, arr, 0, None, None, None) == eda.EDA_ERR_ARG
