"""The allocation-free product entry point (eda_opmv_noalloc) against
eda_opmv, through the C ABI: identical bits on two calls in a row (the
second with a smaller block), on a second, smaller problem, in both
operator forms, with float32 and bfloat16 blocks and with narrow factors;
oversized products are refused."""
import sys

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    _t.cuda.set_device(0)
    return _t


@pytest.fixture(scope="module")
def eda(torch):
    import paper_1512_06500_amd as m
    m.load_library()
    return m


def _prepared(torch, eda, name, storage="f64"):
    p = datagen.config(name)
    h = eda.Handle()
    Xd = torch.from_numpy(np.ascontiguousarray(p.X.T)).cuda().t()
    HW, HB = h.scatter_factors(Xd, p.counts.tolist())
    h.prepare(HW, HB, storage=storage)
    return h, p


def _block(torch, d, b, seed, dtype):
    g = torch.Generator(device="cuda").manual_seed(seed)
    return torch.randn(b, d, dtype=dtype, device="cuda", generator=g).t()


def _compare(torch, h, form, V, vdtype):
    ref, s_ref = h.opmv(form, V, vdtype=vdtype)
    out = torch.full_like(ref.t(), float("nan")).t()
    s = h.opmv_noalloc(form, V, out, vdtype=vdtype)
    torch.cuda.synchronize()
    assert s == s_ref
    assert torch.equal(out, ref), float((out - ref).abs().max())


def test_noalloc_matches_opmv_two_calls_then_smaller(torch, eda):
    h, p = _prepared(torch, eda, "C2")
    log(f"no-alloc product on d={p.d} N={p.n + p.k}: b=8 then b=3")
    _compare(torch, h, "M", _block(torch, p.d, 8, 1, torch.float64), "f64")
    _compare(torch, h, "M", _block(torch, p.d, 3, 2, torch.float64), "f64")
    _compare(torch, h, "M", _block(torch, p.d, 5, 3, torch.float32), "f32")
    h.opmv("A", _block(torch, p.d, 1, 4, torch.float64))   # builds the Arnoldi core
    _compare(torch, h, "A", _block(torch, p.d, 8, 5, torch.float64), "f64")
    h.close()
    h1, p1 = _prepared(torch, eda, "C1")
    log(f"no-alloc product on the smaller d={p1.d} N={p1.n + p1.k}: b=2")
    _compare(torch, h1, "M", _block(torch, p1.d, 2, 6, torch.float64), "f64")
    h1.close()


@pytest.mark.parametrize("storage,vdtype", [("bf16", "f32"), ("fp8", "bf16"), ("fp8", "f64")])
def test_noalloc_matches_opmv_narrow_storage(torch, eda, storage, vdtype):
    """Narrow factors: the second pass of both entry points takes the same
    kernel (column-split with float32 partials for narrow blocks)."""
    h, p = _prepared(torch, eda, "C3", storage)
    dt = {"f32": torch.float32, "bf16": torch.bfloat16, "f64": torch.float64}[vdtype]
    log(f"no-alloc product, {storage} factor d={p.d} N={p.n + p.k}, {vdtype} blocks b=8 then b=5")
    _compare(torch, h, "M", _block(torch, p.d, 8, 11, torch.float32).to(dt), vdtype)
    _compare(torch, h, "M", _block(torch, p.d, 5, 12, torch.float32).to(dt), vdtype)
    h.close()


def test_noalloc_refuses_oversized_and_unbuilt_core(torch, eda):
    h, p = _prepared(torch, eda, "C1")
    V = _block(torch, p.d, 8, 7, torch.float64)
    out = torch.empty_like(V.t()).t()
    with pytest.raises(eda.EDAError) as ei:
        h.opmv_noalloc("A", V, out)
    assert ei.value.status == eda.EDA_ERR_STATE
    h.close()
    # a product whose row-chunk partials alone exceed the 32 MiB scratch
    # (64 row chunks x 1100 columns x 64 block columns x 8 bytes = 36 MB)
    d, n, k = 65536, 1000, 100
    HW = _block(torch, d, n, 9, torch.float64) / np.sqrt(d)
    HB = _block(torch, d, k, 10, torch.float64) / np.sqrt(d)
    h2 = eda.Handle()
    h2.prepare(HW, HB)
    Vb = _block(torch, d, 64, 8, torch.float64)
    outb = torch.empty_like(Vb.t()).t()
    with pytest.raises(eda.EDAError) as ei:
        h2.opmv_noalloc("M", Vb, outb)
    assert ei.value.status == eda.EDA_ERR_ARG and "scratch" in str(ei.value)
    h2.close()
