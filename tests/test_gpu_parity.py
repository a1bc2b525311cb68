"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances (float64 path):
* exponential products: ||e^s Out - E V||_F <= 1e-13 ||E||_2 ||V||_F, where E
  is the dense exponential of the oracle -- a few hundred ulps of the largest
  term, the rounding of two streamed passes of length d plus the small core;
* Ritz values: relative error <= max(1e-10, 50 u lam_1 / lam_i);
* subspace: sin angle(X, X_oracle) <= max(1e-8, 50 u lam_1 / (lam_t - lam_t+1));
* eigensolver: |w - w_ref| <= 1e-13 ||A||, ||A Z - Z diag(w)|| <= 1e-12 ||A||,
  ||Z^T Z - I|| <= 1e-12.
"""
import sys

import numpy as np
import pytest

import datagen
import oracle as O

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


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


def dev(torch, a):
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


def host(t):
    return t.detach().cpu().numpy()


def rel_op_err(out, ref, E_norm, V):
    return np.linalg.norm(out - ref) / (E_norm * np.linalg.norm(V))


class Case:
    def __init__(self, name, X, counts, t):
        self.name, self.X, self.counts, self.t = name, X, np.asarray(counts), t
        self.H_W, self.H_B = O.scatter_factors(X, counts)
        self.d = X.shape[0]


@pytest.fixture(scope="module")
def c1():
    p = datagen.config("C1")
    return Case("C1", p.X, p.counts, p.t)


@pytest.fixture(scope="module")
def c2():
    p = datagen.config("C2")
    return Case("C2", p.X, p.counts, p.t)


@pytest.fixture(scope="module")
def ragged():
    counts = [2, 3, 4, 1, 5]
    X = datagen.make_samples(333, counts, 12, seed=21)
    return Case("ragged", X, counts, 4)


def prepared(torch, eda, case, storage="f64"):
    h = eda.Handle()
    Xd = dev(torch, case.X)
    H_W, H_B = h.scatter_factors(Xd, case.counts.tolist())
    h.prepare(H_W, H_B, storage=storage)
    return h, H_W, H_B


# ---------------------------------------------------------------------------
# a1 / a2: scatter factors, factor ingest and Gram
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cname", ["c1", "ragged"])
def test_scatter_factors(torch, eda, cname, request):
    case = request.getfixturevalue(cname)
    log(f"scatter factors {case.name} d={case.d} counts={case.counts.tolist()}")
    h, H_W, H_B = prepared(torch, eda, case)
    torch.cuda.synchronize()
    assert np.abs(host(H_W) - case.H_W).max() <= 1e-15 * 4
    assert np.abs(host(H_B) - case.H_B).max() <= 1e-14
    h.close()


def test_scatter_factors_class_sizes(torch, eda):
    """Classes of 1 to 47 samples: those of at most 8, 16, 24 and 32 samples
    are read once with the class held in registers (sizes at both ends of
    each bound), larger ones take the two-pass loop; a ragged d (not a
    multiple of the 256-row workgroup).  Against the oracle's eqs.
    (1.1)-(1.2)."""
    counts = [1, 7, 8, 9, 16, 17, 24, 25, 32, 33, 47]
    X = datagen.make_samples(1003, counts, 24, seed=41)
    case = Case("class sizes", X, counts, 3)
    log(f"scatter factors d=1003 counts={counts}")
    h = eda.Handle()
    H_W, H_B = h.scatter_factors(dev(torch, X), counts)
    torch.cuda.synchronize()
    assert np.abs(host(H_W) - case.H_W).max() <= 1e-15 * 4
    assert np.abs(host(H_B) - case.H_B).max() <= 1e-14
    h.close()


@pytest.mark.parametrize("cname", ["c1", "ragged", "c2"])
def test_gram(torch, eda, cname, request):
    case = request.getfixturevalue(cname)
    log(f"gram {case.name}")
    h, _, _ = prepared(torch, eda, case)
    G = host(h.gram())
    P = np.concatenate([case.H_W, case.H_B], axis=1)
    Gr = P.T @ P
    assert np.array_equal(G, G.T), "Gram must be exactly symmetric"
    assert np.linalg.norm(G - Gr) <= 1e-14 * np.linalg.norm(Gr)
    h.close()


@pytest.mark.parametrize("d,n,k", [(5003, 677, 100), (20000, 1500, 37)])
def test_gram_large_matrix_cores(torch, eda, d, n, k):
    """Gram matrices with N = n + k >= 256 take the matrix-core kernel (64 x
    64 tiles, row chunks, ragged last tile and chunk): exactly symmetric and
    normwise within 1e-14 of P^T P in float64."""
    log(f"gram (matrix cores) d={d} N={n + k}")
    rng = np.random.default_rng(d)
    H_W = rng.standard_normal((d, n)) / np.sqrt(d)
    H_B = rng.standard_normal((d, k)) / np.sqrt(d)
    h = eda.Handle()
    h.prepare(dev(torch, H_W), dev(torch, H_B))
    G = host(h.gram())
    P = np.concatenate([H_W, H_B], axis=1)
    Gr = P.T @ P
    assert np.array_equal(G, G.T), "Gram must be exactly symmetric"
    err = np.linalg.norm(G - Gr) / np.linalg.norm(Gr)
    log(f"  rel err {err:.2e}")
    assert err <= 1e-14
    h.close()


@pytest.mark.parametrize("n,scale", [(1990, 4.0), (2000, 0.9)])
def test_w_cores_with_many_tiles(torch, eda, n, scale):
    """W-cores of n = 2000 columns: 528 lower 64 x 64 tiles per product of
    the matrix polynomial, every tile split along K and reduced (n = 1990:
    ragged last tile).  The scales put the spectral bound of c S_W at about
    2 (no or one doubling) and about 50 (several doublings).  Oracle: the
    closed form of Theorem 3.1 for exp(c S_W) and the composite operator."""
    d, k = 3000, 20
    log(f"W-cores n={n} d={d} k={k} scale={scale}")
    rng = np.random.default_rng(n)
    H_W = rng.standard_normal((d, n)) * (scale / np.sqrt(d))
    H_B = rng.standard_normal((d, k)) * (0.5 / np.sqrt(d))
    h = eda.Handle()
    h.prepare(dev(torch, H_W), dev(torch, H_B))
    V = rng.standard_normal((d, 8))
    for c in (-0.5, -1.0):
        out, s = h.expmv("W", c, dev(torch, V))
        ref = O.exp_action_thm31(H_W, c, V)
        err = rel_op_err(host(out) * np.exp(s), ref, 1.0, V)
        log(f"  W c={c} err={err:.2e}")
        assert err <= 1e-13
    sB = np.linalg.svd(H_B, compute_uv=False) ** 2
    out, s = h.opmv("M", dev(torch, V))
    ref = O.lanczos_action_thm31(H_W, H_B, V)
    err = rel_op_err(host(out) * np.exp(s), ref, np.exp(sB[0]), V)
    log(f"  M err={err:.2e}")
    assert err <= 1e-13
    h.close()


# ---------------------------------------------------------------------------
# a3: symmetric eigensolver
# ---------------------------------------------------------------------------

def check_eig(A, w, Z, tol_res=1e-12):
    nrm = max(np.linalg.norm(A, 2), 1e-300)
    wr = np.linalg.eigvalsh(A)
    assert np.all(np.diff(w) >= -1e-13 * nrm), "eigenvalues must ascend"
    assert np.max(np.abs(w - wr)) <= 1e-13 * nrm
    assert np.linalg.norm(A @ Z - Z * w) <= tol_res * nrm * max(1, np.sqrt(A.shape[0]) / 4)
    assert np.abs(Z.T @ Z - np.eye(A.shape[0])).max() <= 1e-12


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 17, 63, 64, 65, 100, 112, 113, 128, 200, 257,
                               600])
def test_syev_random(torch, eda, n):
    log(f"syev random n={n}")
    rng = np.random.default_rng(100 + n)
    B = rng.standard_normal((n, n))
    A = B + B.T
    h = eda.Handle()
    w, Z = h.syev(dev(torch, A))
    check_eig(A, host(w), host(Z))
    h.close()


def test_syev_special_matrices(torch, eda, c1):
    log("syev special matrices")
    h = eda.Handle()
    cases = {
        "zero": np.zeros((7, 7)),
        "identity": np.eye(9),
        "repeated": np.diag([1.0, 2.0, 2.0, 2.0, 3.0, 3.0, 5.0]),
        "gram_WW": c1.H_W.T @ c1.H_W,       # rank n-k: a zero cluster of size k
        "gram_BB": c1.H_B.T @ c1.H_B,       # rank k-1
    }
    rng = np.random.default_rng(3)
    Q = np.linalg.qr(rng.standard_normal((40, 40)))[0]
    cases["clustered"] = (Q * np.concatenate([np.full(20, 1.0), np.full(10, 1.0 + 1e-9),
                                              np.linspace(2, 3, 10)])) @ Q.T
    for name, A in cases.items():
        log(f"  {name} n={A.shape[0]}")
        w, Z = h.syev(dev(torch, A))
        check_eig(A, host(w), host(Z))
    h.close()


@pytest.mark.parametrize("n,c", [(112, 64), (120, 61), (128, 60), (128, 62), (128, 100)])
def test_syev_large_clusters_in_lds(torch, eda, n, c):
    """Matrices of up to 128 rows stay in LDS; a cluster of c equal
    eigenvalues is orthonormalised by Cholesky QR when its Gram matrix fits
    in the LDS left over by the matrix (64 x 64 up to n = 112, 60 x 60 at
    n = 128) and by Gram-Schmidt otherwise.  Eigenvalues, residuals and
    orthogonality against the definitions (check_eig)."""
    log(f"syev n={n} cluster of {c}")
    rng = np.random.default_rng(n + c)
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    lam = np.concatenate([np.full(c, 0.5), np.linspace(1.0, 2.0, n - c)])
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    h = eda.Handle()
    w, Z = h.syev(dev(torch, A))
    check_eig(A, host(w), host(Z))
    h.close()


# ---------------------------------------------------------------------------
# a4: low-rank exponential apply
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("b", [1, 3, 8, 13])
def test_expmv_c1(torch, eda, c1, b):
    log(f"expmv C1 b={b}")
    h, _, _ = prepared(torch, eda, c1)
    rng = np.random.default_rng(b)
    V = rng.standard_normal((c1.d, b))
    for which, H, c in (("W", c1.H_W, -1.0), ("W", c1.H_W, -0.5), ("W", c1.H_W, 0.7),
                        ("B", c1.H_B, 1.0), ("B", c1.H_B, -1.0)):
        E = O.expm_sym(H @ H.T, c)
        out, s = h.expmv(which, c, dev(torch, V))
        got = host(out) * np.exp(s)
        err = rel_op_err(got, E @ V, np.linalg.norm(E, 2), V)
        log(f"  {which} c={c} s={s:.3f} err={err:.2e}")
        assert err <= 1e-13
    h.close()


@pytest.mark.parametrize("storage,u", [("f32", 2.0 ** -24), ("bf16", 2.0 ** -8)])
def test_expmv_narrow_storage_c1(torch, eda, c1, storage, u):
    """Factor stored in float32 / bfloat16.  Rounding H to the storage type
    moves S = H H^T by ||dS|| <= 2 ||H||_2 ||dH||_2 <= 2 u ||H||_2 ||H||_F, and
    the Frechet derivative of exp at S is bounded by e^{max(c S)} |c| ||dS||;
    relative to ||exp(cS)|| = e^{max(c S)} that gives 2 |c| u ||H||_2 ||H||_F,
    tested with a factor 2 of room (plus the float32 operand rounding)."""
    log(f"expmv C1 with {storage} storage")
    h, _, _ = prepared(torch, eda, c1, storage=storage)
    rng = np.random.default_rng(5)
    V = rng.standard_normal((c1.d, 8))
    for vdt in ("f64", "f32"):
        for which, H, c in (("W", c1.H_W, -0.5), ("B", c1.H_B, 1.0)):
            E = O.expm_sym(H @ H.T, c)
            Vd = dev(torch, V)
            if vdt == "f32":
                Vd = Vd.float()
            out, s = h.expmv(which, c, Vd, vdtype=vdt)
            got = host(out).astype(np.float64) * np.exp(s)
            err = rel_op_err(got, E @ V, np.linalg.norm(E, 2), V)
            bound = 4 * abs(c) * u * np.linalg.norm(H, 2) * np.linalg.norm(H) + (
                4 * 2.0 ** -24 if vdt == "f32" else 0.0)
            log(f"  {which} c={c} vdtype={vdt} err={err:.2e} bound={bound:.2e}")
            assert err <= bound
    h.close()


def _e4m3_factor(rng, d, cols, exps):
    """Columns of exact E4M3 values times 2^exps[j], each holding +-448 once:
    the per-column FP8 scale is then exactly 2^exps[j] and storage is lossless."""
    from oracle.fp8 import e4m3_values
    vals = e4m3_values()
    H = rng.choice(vals, size=(d, cols)) * rng.choice([-1.0, 1.0], size=(d, cols))
    H[rng.integers(0, d, size=cols), np.arange(cols)] = 448.0
    return H * 2.0 ** np.asarray(exps, dtype=np.float64)


def test_expmv_fp8_lossless_factor(torch, eda):
    """FP8 storage of a factor whose entries are exact E4M3 values times a
    power-of-two per column: the stored copy is exact, so both streaming
    passes must reproduce the float64 exponential action to float64
    accuracy.  Pins the decode, the per-column scales and where the passes
    apply them."""
    log("expmv FP8 storage, lossless factor")
    rng = np.random.default_rng(11)
    d, n, k = 700, 24, 5
    H_W = _e4m3_factor(rng, d, n, rng.integers(-11, -8, size=n)) * 0.25
    H_B = _e4m3_factor(rng, d, k, rng.integers(-11, -9, size=k))
    h = eda.Handle()
    h.prepare(dev(torch, H_W), dev(torch, H_B), storage="fp8")
    V = rng.standard_normal((d, 8))
    for vdt in ("f64", "f32"):
        for which, H, c in (("W", H_W, -0.5), ("W", H_W, -1.0), ("B", H_B, 1.0)):
            E = O.expm_sym(H @ H.T, c)
            Vd = dev(torch, V)
            if vdt == "f32":
                Vd = Vd.float()
            out, s = h.expmv(which, c, Vd, vdtype=vdt)
            got = host(out).astype(np.float64) * np.exp(s)
            ref = E @ (V.astype(np.float32).astype(np.float64) if vdt == "f32" else V)
            err = rel_op_err(got, ref, np.linalg.norm(E, 2), V)
            bound = 1e-13 if vdt == "f64" else 64 * 2.0 ** -24
            log(f"  {which} c={c} vdtype={vdt} err={err:.2e} bound={bound:.1e}")
            assert err <= bound
    h.close()


@pytest.mark.parametrize("storage", ["fp8", "bf16"])
@pytest.mark.parametrize("d,n,k,b", [(3001, 150, 7, 8), (20011, 333, 40, 3), (40000, 1216, 38, 8)])
def test_expmv_narrow_lossless_float32_blocks(torch, eda, storage, d, n, k, b):
    """Float32 blocks against FP8 / bfloat16 copies that hold the factor
    exactly (E4M3 values times a power of two per column, or bfloat16
    values): the float32 pass over the narrow copy must give the exact
    exponential action of the float32-rounded block to float32 accuracy.
    The shapes span several 64-column groups with a ragged last group, row
    chunks of several slabs and a ragged row tail."""
    from oracle.bf16 import bf16_round
    log(f"expmv {storage} lossless d={d} n={n} k={k} b={b} float32 block")
    rng = np.random.default_rng(d + n)
    if storage == "fp8":
        H_W = _e4m3_factor(rng, d, n, rng.integers(-13, -10, size=n))
        H_B = _e4m3_factor(rng, d, k, rng.integers(-13, -11, size=k))
    else:
        H_W = bf16_round(rng.standard_normal((d, n)) * 2.0 ** -5)
        H_B = bf16_round(rng.standard_normal((d, k)) * 2.0 ** -6)
    h = eda.Handle()
    h.prepare(dev(torch, H_W), dev(torch, H_B), storage=storage)
    V = rng.standard_normal((d, b)).astype(np.float32).astype(np.float64)
    for which, H, c in (("W", H_W, -0.5), ("B", H_B, 1.0)):
        out, s = h.expmv(which, c, dev(torch, V).float(), vdtype="f32")
        got = host(out).astype(np.float64) * np.exp(s)
        ref = O.exp_action_thm31(H, c, V)
        E_norm = np.exp(max(0.0, c * np.linalg.norm(H, 2) ** 2))
        err = rel_op_err(got, ref, E_norm, V)
        bound = 64 * 2.0 ** -24
        log(f"  {which} c={c} err={err:.2e} bound={bound:.1e}")
        assert err <= bound
    h.close()


@pytest.mark.parametrize("storage", ["fp8", "bf16"])
@pytest.mark.parametrize("d,n,k,b", [(3001, 150, 7, 8), (20011, 333, 40, 3)])
def test_expmv_narrow_bfloat16_blocks(torch, eda, storage, d, n, k, b):
    """bfloat16 blocks against lossless FP8 / bfloat16 copies: the products
    are exact and the sums run in float32 over 32 rows, then float64, so the
    result is the exact exponential action of the block, rounded once to
    bfloat16: within 2^-8 of the oracle normwise, and within one bfloat16
    ulp of the float32-block result rounded to bfloat16, entry by entry."""
    from oracle.bf16 import bf16_round
    log(f"expmv {storage} lossless d={d} n={n} k={k} b={b} bfloat16 block")
    rng = np.random.default_rng(d + 7 * n)
    if storage == "fp8":
        H_W = _e4m3_factor(rng, d, n, rng.integers(-13, -10, size=n))
        H_B = _e4m3_factor(rng, d, k, rng.integers(-13, -11, size=k))
    else:
        H_W = bf16_round(rng.standard_normal((d, n)) * 2.0 ** -5)
        H_B = bf16_round(rng.standard_normal((d, k)) * 2.0 ** -6)
    h = eda.Handle()
    h.prepare(dev(torch, H_W), dev(torch, H_B), storage=storage)
    V = bf16_round(rng.standard_normal((d, b)))
    for which, H, c in (("W", H_W, -0.5), ("B", H_B, 1.0)):
        out, s = h.expmv(which, c, dev(torch, V).to(torch.bfloat16), vdtype="bf16")
        o16 = host(out.float()).astype(np.float64)
        out32, s32 = h.expmv(which, c, dev(torch, V).float(), vdtype="f32")
        assert s == s32
        o32 = bf16_round(host(out32).astype(np.float64))
        ulp = np.abs(o32) * 2.0 ** -7 + 2.0 ** -133
        assert np.all(np.abs(o16 - o32) <= ulp), np.abs(o16 - o32).max()
        ref = O.exp_action_thm31(H, c, V)
        E_norm = np.exp(max(0.0, c * np.linalg.norm(H, 2) ** 2))
        err = rel_op_err(o16 * np.exp(s), ref, E_norm, V)
        log(f"  {which} c={c} err={err:.2e}")
        assert err <= 2.0 ** -8
    h.close()


def test_bfloat16_block_needs_narrow_storage(torch, eda, c1):
    h, _, _ = prepared(torch, eda, c1)
    V = torch.zeros(8, c1.d, dtype=torch.bfloat16, device="cuda").t()
    with pytest.raises(eda.EDAError):
        h.expmv("W", -0.5, V, vdtype="bf16")
    h.close()


def test_expmv_fp8_rounding_c1(torch, eda, c1):
    """FP8 storage of the C1 factors.  The two streaming passes read the
    E4M3 copy (scaled per column, rounded to nearest even) while the core
    phi_c(H^T H) comes from the float64 Gram, so the product equals
    V + Hq G_c Hq^T V with Hq the reference rounding of H and G_c from the
    SVD of H: compared at float64 accuracy, which pins the encoding of every
    entry that feeds the product."""
    from oracle.fp8 import fp8_columns
    log("expmv C1 with FP8 storage against the reference rounding")
    h = eda.Handle()
    h.prepare(dev(torch, c1.H_W), dev(torch, c1.H_B), storage="fp8")
    rng = np.random.default_rng(6)
    V = rng.standard_normal((c1.d, 8))
    for which, H, c in (("W", c1.H_W, -0.5), ("B", c1.H_B, 1.0)):
        Hq, _ = fp8_columns(H)
        _, sig, Vt = np.linalg.svd(H, full_matrices=False)
        lam = sig ** 2
        phi = np.where(lam > 0, np.expm1(c * lam) / np.where(lam > 0, lam, 1.0), c)
        G = Vt.T @ (phi[:, None] * Vt)
        ref = V + Hq @ (G @ (Hq.T @ V))
        out, s = h.expmv(which, c, dev(torch, V))
        got = host(out) * np.exp(s)
        scale = np.linalg.norm(ref) + np.linalg.norm(V)
        err = np.linalg.norm(got - ref) / scale
        E = O.expm_sym(H @ H.T, c)
        drift = rel_op_err(got, E @ V, np.linalg.norm(E, 2), V)
        log(f"  {which} c={c} err vs rounded factor={err:.2e}  vs exact exp={drift:.2e}")
        assert err <= 1e-12
    h.close()


@pytest.fixture(params=["poly", "eig"])
def wcore(request, monkeypatch):
    """W-cores by the matrix polynomial (default) or by eig(H_W^T H_W)."""
    if request.param == "eig":
        monkeypatch.setenv("EDA_WCORE", "eig")
    else:
        monkeypatch.delenv("EDA_WCORE", raising=False)
    return request.param


def test_opmv_c1(torch, eda, c1, wcore):
    log(f"opmv C1 (Lanczos M and Arnoldi A), W-core by {wcore}")
    h, _, _ = prepared(torch, eda, c1)
    V = np.random.default_rng(5).standard_normal((c1.d, 8))
    M = O.lanczos_matrix_dense(c1.H_W, c1.H_B)
    A = O.arnoldi_matrix_dense(c1.H_W, c1.H_B)
    for form, E in (("M", M), ("A", A)):
        out, s = h.opmv(form, dev(torch, V))
        got = host(out) * np.exp(s)
        err = rel_op_err(got, E @ V, np.linalg.norm(E, 2), V)
        log(f"  {form} s={s:.3f} err={err:.2e}")
        assert err <= 1e-13
    h.close()


def test_expmv_opmv_c2_full_size(torch, eda, c2, wcore):
    """d=10304, n=200, k=40 at b=8, the launch shape the solver uses; the
    oracle is the closed form of Theorem 3.1 (QR + SVD), norms from the same."""
    log(f"expmv/opmv C2 full size, W-core by {wcore}")
    h, _, _ = prepared(torch, eda, c2)
    V = np.random.default_rng(9).standard_normal((c2.d, 8))
    sW = np.linalg.svd(c2.H_W, compute_uv=False) ** 2
    sB = np.linalg.svd(c2.H_B, compute_uv=False) ** 2
    for which, H, c, En in (("W", c2.H_W, -0.5, 1.0), ("W", c2.H_W, -1.0, 1.0),
                            ("B", c2.H_B, 1.0, np.exp(sB[0]))):
        out, s = h.expmv(which, c, dev(torch, V))
        ref = O.exp_action_thm31(H, c, V)
        err = rel_op_err(host(out) * np.exp(s), ref, En, V)
        log(f"  {which} c={c} err={err:.2e}")
        assert err <= 1e-13
    out, s = h.opmv("M", dev(torch, V))
    ref = O.lanczos_action_thm31(c2.H_W, c2.H_B, V)
    err = rel_op_err(host(out) * np.exp(s), ref, np.exp(sB[0]), V)
    log(f"  M err={err:.2e}")
    assert err <= 1e-13
    h.close()


@pytest.mark.parametrize("b,storage", [(39, "f64"), (99, "f64"), (39, "f32")])
def test_expmv_opmv_c2_wide_blocks(torch, eda, c2, b, storage):
    """Blocks as wide as the Ritz blocks of the final stage (t = 39 at this
    size, 99 for the large workload), on the full-size factor: the wide
    launch shapes of both passes (matrix-core P Z for float64, the
    40-column vector kernel for float32, three B tiles per workgroup in
    P^T V).  Oracle: the closed form of Theorem 3.1; the float32 bound is
    the storage-rounding bound of the narrow-storage test."""
    log(f"expmv/opmv C2 full size, b={b}, {storage} storage")
    h, _, _ = prepared(torch, eda, c2, storage=storage)
    V = np.random.default_rng(b).standard_normal((c2.d, b))
    sB = np.linalg.svd(c2.H_B, compute_uv=False) ** 2
    u = 2.0 ** -24 if storage == "f32" else 0.0
    for which, H, c, En in (("W", c2.H_W, -0.5, 1.0), ("B", c2.H_B, 1.0, np.exp(sB[0]))):
        out, s = h.expmv(which, c, dev(torch, V))
        ref = O.exp_action_thm31(H, c, V)
        err = rel_op_err(host(out) * np.exp(s), ref, En, V)
        bound = max(1e-13, 4 * abs(c) * u * np.linalg.norm(H, 2) * np.linalg.norm(H))
        log(f"  {which} c={c} err={err:.2e} bound={bound:.2e}")
        assert err <= bound
    if storage == "f64":
        out, s = h.opmv("M", dev(torch, V))
        ref = O.lanczos_action_thm31(c2.H_W, c2.H_B, V)
        err = rel_op_err(host(out) * np.exp(s), ref, np.exp(sB[0]), V)
        log(f"  M err={err:.2e}")
        assert err <= 1e-13
    h.close()


@pytest.fixture(scope="module")
def tall():
    """A factor long enough (d = 40000) for the streaming passes to take
    their 16-column forms, with few columns so that the oracle stays cheap."""
    counts = [25] * 12
    X = datagen.make_samples(40000, counts, 40, seed=31)
    return Case("tall", X, counts, 11)


@pytest.mark.parametrize("b", [12, 16])
def test_expmv_opmv_blocks_of_9_to_16_columns(torch, eda, c2, tall, b):
    """Blocks of 9 to 16 columns: P^T V staged as 16 columns, the 16-column
    streaming P Z (d = 40000) and the column-split core product.  Oracle:
    the closed form of Theorem 3.1."""
    for case in (c2, tall):
        log(f"expmv/opmv {case.name} b={b}")
        h, _, _ = prepared(torch, eda, case)
        V = np.random.default_rng(100 + b).standard_normal((case.d, b))
        sB = np.linalg.svd(case.H_B, compute_uv=False) ** 2
        for which, H, c, En in (("W", case.H_W, -0.5, 1.0), ("B", case.H_B, 1.0, np.exp(sB[0]))):
            out, s = h.expmv(which, c, dev(torch, V))
            ref = O.exp_action_thm31(H, c, V)
            err = rel_op_err(host(out) * np.exp(s), ref, En, V)
            log(f"  {which} c={c} err={err:.2e}")
            assert err <= 1e-13
        out, s = h.opmv("M", dev(torch, V))
        ref = O.lanczos_action_thm31(case.H_W, case.H_B, V)
        err = rel_op_err(host(out) * np.exp(s), ref, np.exp(sB[0]), V)
        log(f"  M err={err:.2e}")
        assert err <= 1e-13
        h.close()


@pytest.mark.parametrize("b", [1, 3, 8])
def test_expmv_opmv_tall_blocks_up_to_8_columns(torch, eda, tall, b):
    """Blocks of 1 to 8 columns at d = 40000: the 8-column streaming P Z,
    whose Z rows are read with scalar loads (whole rows for b = 8, entry by
    entry below), with a ragged last workgroup (40000 is not a multiple of
    its 128 rows).  Oracle: the closed form of Theorem 3.1."""
    case = tall
    log(f"expmv/opmv {case.name} b={b}")
    h, _, _ = prepared(torch, eda, case)
    V = np.random.default_rng(200 + b).standard_normal((case.d, b))
    sB = np.linalg.svd(case.H_B, compute_uv=False) ** 2
    for which, H, c, En in (("W", case.H_W, -0.5, 1.0), ("B", case.H_B, 1.0, np.exp(sB[0]))):
        out, s = h.expmv(which, c, dev(torch, V))
        ref = O.exp_action_thm31(H, c, V)
        err = rel_op_err(host(out) * np.exp(s), ref, En, V)
        log(f"  {which} c={c} err={err:.2e}")
        assert err <= 1e-13
    out, s = h.opmv("M", dev(torch, V))
    ref = O.lanczos_action_thm31(case.H_W, case.H_B, V)
    err = rel_op_err(host(out) * np.exp(s), ref, np.exp(sB[0]), V)
    log(f"  M err={err:.2e}")
    assert err <= 1e-13
    h.close()


@pytest.mark.parametrize("b,max_basis", [(16, 0), (12, 72), (16, 80)])
def test_solve_c2_blocks_above_8(torch, eda, c2, b, max_basis):
    """Block Lanczos with 12 and 16 columns: the full default basis (the
    pivoted Cholesky's correction then spans more rows than one staged
    tile) and small bases with thick restarts.  Oracle: the reduced
    direct solve."""
    log(f"solve C2 b={b} max_basis={max_basis}")
    red = O.eda_reduced(c2.H_W, c2.H_B, c2.t)
    h, _, _ = prepared(torch, eda, c2)
    res = h.solve(c2.t, 1e-10, block=b, max_basis=max_basis, seed=6, max_iter=3000)
    if max_basis:
        assert res.info["restarts"] >= 1
    check_solution(res, red, c2.t, red.lam_all, 1e-10)
    h.close()


def test_solve_tall_block_16(torch, eda, tall):
    """b = 16 at d = 40000: the new block is normalised in place by the
    16-column streaming product.  Oracle: the reduced direct solve."""
    log("solve tall d=40000 t=11 b=16")
    red = O.eda_reduced(tall.H_W, tall.H_B, tall.t)
    h, _, _ = prepared(torch, eda, tall)
    res = h.solve(tall.t, 1e-10, block=16, seed=7)
    check_solution(res, red, tall.t, red.lam_all, 1e-10)
    h.close()


def test_block_width_limits_per_form(torch, eda, c1):
    """Block widths above 16 are rejected; the Arnoldi and Jacobi-Davidson
    forms take at most 8."""
    h, _, _ = prepared(torch, eda, c1)
    for form, b in (("M", 17), ("A", 9), ("JD", 9)):
        res = h.solve(c1.t, 1e-8, block=b, seed=1, form=form, raise_on_error=False)
        assert res.status == 1, (form, b, res.status, res.message)
    h.close()


# ---------------------------------------------------------------------------
# f3: nearest-neighbour classification in the EDA subspace (Section 3.3)
# ---------------------------------------------------------------------------

def _classify(torch, h, V, train, labels, test):
    pred, idx, dist = h.nn_classify(dev(torch, V), dev(torch, train),
                                    torch.as_tensor(np.asarray(labels, dtype=np.int32)).cuda(),
                                    dev(torch, test))
    return host(pred), host(idx), host(dist)


def test_nn_classify_hand_example_and_ties(torch, eda):
    """The hand-computed example of the oracle pins: exact distances, labels,
    and the smallest index on a three-way tie."""
    log("nn_classify hand example")
    h = eda.Handle()
    train = np.array([[1.0, 0.0, 0.0, 0.6], [0.0, 1.0, 0.0, 0.8], [0.0, 0.0, 1.0, 0.0]])
    test = np.array([[0.9, 0.5, 0.0], [0.1, 0.7, 0.0], [0.4, 0.5, 1.0]])
    pred, idx, dist = _classify(torch, h, np.eye(3)[:, :2], train, [10, 11, 12, 13], test)
    assert idx.tolist() == [0, 3, 2] and pred.tolist() == [10, 13, 12]
    np.testing.assert_allclose(dist, [np.sqrt(0.02), np.sqrt(0.02), 0.0], rtol=0, atol=1e-15)
    pred, idx, dist = _classify(torch, h, np.eye(3)[:, 2:3], train, [5, 6, 7, 8],
                                np.array([[0.6], [0.8], [0.0]]))
    assert idx.tolist() == [0] and pred.tolist() == [5] and dist.tolist() == [0.0]
    h.close()


@pytest.mark.parametrize("n_test_per_class", [5, 1])
def test_nn_classify_c2_against_oracle(torch, eda, n_test_per_class):
    """C2-sized split (d = 10304, 200 training samples, 40 classes): the
    oracle's EDA solution on both sides; the nearest index must agree wherever
    the oracle's nearest distance is unique (second nearest more than 1e-10
    away), else be one of the near-tied; distances to 1e-12."""
    p = datagen.config("C2", with_data=False)
    Xtr, Xte, lte = datagen.make_split(p.d, p.counts, np.full(p.k, n_test_per_class), p.r, p.seed)
    log(f"nn_classify C2 split, {Xte.shape[1]} testing samples")
    H_W, H_B = O.scatter_factors(Xtr, p.counts)
    V = O.eda_reduced(H_W, H_B, p.t).X
    lab_o, idx_o, dist_o = O.nn.nn_classify(V, Xtr, p.labels(), Xte)
    D = O.nn.nn_distances(V, Xtr, Xte)
    h = eda.Handle()
    pred, idx, dist = _classify(torch, h, V, Xtr, p.labels(), Xte)
    h.close()
    np.testing.assert_allclose(dist, dist_o, rtol=0, atol=1e-12)
    Ds = np.sort(D, axis=0)
    unique = (Ds[1] - Ds[0]) > 1e-10
    log(f"  unique nearest: {int(unique.sum())}/{unique.size}, accuracy {np.mean(pred == lte):.3f}")
    assert np.array_equal(idx[unique], idx_o[unique])
    near = D[idx, np.arange(D.shape[1])] <= Ds[0] + 1e-10
    assert near.all()
    assert np.array_equal(pred, p.labels()[idx])


def test_nn_distances_within_thm37_bounds(torch, eda):
    """Theorem 3.7 on a solution computed to tol 1e-4: the nearest distances
    measured with it stay within the bounds around those of the exact
    subspace (the oracle's), with sin and cos of the angle between them."""
    p = datagen.config("C2", with_data=False)
    Xtr, Xte, lte = datagen.make_split(p.d, p.counts, np.full(p.k, 2), p.r, p.seed)
    log("nn distances vs Theorem 3.7, tol 1e-4")
    H_W, H_B = O.scatter_factors(Xtr, p.counts)
    V = O.eda_reduced(H_W, H_B, p.t).X
    _, _, d_exact = O.nn.nn_classify(V, Xtr, p.labels(), Xte)
    h = eda.Handle()
    Xd = dev(torch, Xtr)
    H_Wd, H_Bd = h.scatter_factors(Xd, p.counts.tolist())
    h.prepare(H_Wd, H_Bd)
    res = h.solve(p.t, 1e-4, block=8, seed=p.seed)
    assert res.status == 0
    Xt = host(res.X)
    pred, idx, d_approx = _classify(torch, h, Xt, Xtr, p.labels(), Xte)
    h.close()
    s, c = O.sin_angle(V, Xt), O.nn.cos_angle(V, Xt)
    lo, hi = O.nn.thm37_bounds(d_approx, s, c)
    log(f"  sin={s:.2e} cos={c:.6f} max|d~-d|={np.max(np.abs(d_approx - d_exact)):.2e} "
        f"accuracy {np.mean(pred == lte):.3f}")
    assert np.all(lo <= d_exact + 1e-12) and np.all(d_exact <= hi + 1e-12)


# ---------------------------------------------------------------------------
# a5-a7: block Lanczos solve, Rayleigh-Ritz, back-transform + orth
# ---------------------------------------------------------------------------

def check_solution(res, ref, t, lam_all, tol):
    lam = np.array(res.ritz)
    fl = O.accuracy_floor(lam_all, t)
    lam_tol = np.maximum(1e-10, 50 * U * lam_all[0] / ref.lam)
    relerr = np.abs(lam - ref.lam) / ref.lam
    X = host(res.X)
    ang = O.sin_angle(ref.X, X)
    ang_tol = max(1e-8, 50 * fl["span"])
    log(f"  status={res.status} iters={res.info['iters']} restarts={res.info['restarts']} "
        f"lam_err={relerr.max():.2e} sin={ang:.2e} resid={max(res.resid):.2e} "
        f"krylov_ms={res.info['t_krylov_ms']:.2f}")
    assert res.status == 0, res.message
    assert np.all(relerr <= lam_tol)
    assert ang <= ang_tol
    assert np.abs(X.T @ X - np.eye(t)).max() <= 1e-13
    assert np.allclose(np.array(res.ritz_log), np.log(ref.lam), rtol=0, atol=1e-10)
    tol_i = np.maximum(tol, 10 * U * lam[0] / lam)
    assert np.all(np.array(res.resid) <= 10 * tol_i)
    return X


def nu_max(H):
    """Largest eigenvalue of H H^T (through the small Gram matrix)."""
    return float(np.linalg.eigvalsh(H.T @ H)[-1])


def check_floored_solution(res, ref, t, tol, tag="", nu1=None):
    """Bounds for solves stopped at tol (1e-6) whose small pairs sit at their
    attainable floor (graded spectra), all derived from the residuals the
    solver returns:
    * each returned residual meets max(tol, 10 u lam_1 / lam_i) up to the
      rounding of the one product that measures it (a factor 10 of room);
    * Ritz value i is within its residual ||M y_i - theta_i y_i|| of an
      eigenvalue (symmetric M, unit y_i), i.e. within resid_i theta_i of
      lam_i (a factor 2 of room), plus rounding on both sides: the oracle's
      dense N x N pencil solve is backward stable, so its lam_i carries an
      absolute error of about sqrt(N) u lam_1, and the residual the GPU
      measures with one product cannot resolve below that product's own
      rounding, of the same size (10 sqrt(N) u lam_1 / lam_i relative for
      each side);
    * the component of Ritz vector y_i in the eigenspace of the unwanted
      eigenvalues (those <= lam_next = max(lam_{t+1}, 1)) is at most
      ||r_i|| / (theta_i - lam_next), so sin angle(Y, Y_exact) is at most the
      2-norm of those bounds; the back-transform x = exp(-S_W/2) y multiplies
      angles by at most cond(exp(-S_W/2)) = e^{nu_1 / 2}; plus the oracle's
      own span floor."""
    lam = np.array(res.ritz)
    resid = np.array(res.resid)
    N = ref.lam_all.size
    relerr = np.abs(lam - ref.lam) / ref.lam
    X = host(res.X)
    ang = O.sin_angle(ref.X, X)
    fl = O.accuracy_floor(ref.lam_all, t)
    tol_i = np.maximum(tol, 10 * U * lam[0] / lam)
    oracle_pair = max(50.0, 20 * np.sqrt(N)) * U * ref.lam[0] / ref.lam
    lam_tol = 2 * resid * lam / ref.lam + oracle_pair
    lam_next = ref.lam[-1] - fl["gap"]
    comp = resid * lam / np.maximum(lam - lam_next, 1e-300)
    amp = np.exp(nu1 / 2) if nu1 is not None else 1.0
    ang_tol = max(1e-8, 50 * fl["span"]) + 2 * amp * np.linalg.norm(comp)
    log(f"  {tag}: status={res.status} iters={res.info['iters']} restarts={res.info['restarts']} "
        f"passes={res.info['refine_passes']} lam_err={relerr.max():.2e} "
        f"(max err/bound {np.max(relerr / lam_tol):.2e}) sin={ang:.2e} (bound {ang_tol:.1e}) "
        f"max resid/tol_i={np.max(resid / tol_i):.2e} krylov_ms={res.info['t_krylov_ms']:.1f} "
        f"refine_ms={res.info['t_refine_ms']:.1f}")
    assert res.status == 0, res.message
    assert np.all(resid <= 10 * tol_i)
    assert np.all(relerr <= lam_tol), np.argmax(relerr / lam_tol)
    assert ang <= ang_tol
    assert np.abs(X.T @ X - np.eye(t)).max() <= 1e-13
    return X


def test_solve_c1(torch, eda, c1):
    log("solve C1 t=9 b=8 tol=1e-10")
    ref = O.eda_dense(c1.H_W, c1.H_B, c1.t)
    red = O.eda_reduced(c1.H_W, c1.H_B, c1.t)
    h, _, _ = prepared(torch, eda, c1)
    res = h.solve(c1.t, 1e-10, block=8, seed=1)
    X = check_solution(res, ref, c1.t, red.lam_all, 1e-10)
    # per-column agreement (distinct, well separated eigenvalues at C1)
    assert np.abs(X - ref.X).max() <= 1e-8
    h.close()


def test_solve_c2(torch, eda, c2, wcore):
    log(f"solve C2 t=39 b=8 tol=1e-10, W-core by {wcore}")
    red = O.eda_reduced(c2.H_W, c2.H_B, c2.t)
    h, _, _ = prepared(torch, eda, c2)
    sb = datagen.start_block(c2.d, 8, 2)
    res = h.solve(c2.t, 1e-10, block=8, start_block=dev(torch, sb))
    check_solution(res, red, c2.t, red.lam_all, 1e-10)
    h.close()


def test_solve_c2_thick_restart(torch, eda, c2):
    log("solve C2 with a small basis (thick restarts)")
    red = O.eda_reduced(c2.H_W, c2.H_B, c2.t)
    h, _, _ = prepared(torch, eda, c2)
    res = h.solve(c2.t, 1e-10, block=8, max_basis=72, seed=4, max_iter=3000)
    assert res.info["restarts"] >= 1
    check_solution(res, red, c2.t, red.lam_all, 1e-10)
    h.close()


def test_solve_ragged_small_block(torch, eda, ragged):
    log("solve ragged d=333 n=15 k=5 t=4 b=3")
    ref = O.eda_dense(ragged.H_W, ragged.H_B, ragged.t)
    red = O.eda_reduced(ragged.H_W, ragged.H_B, ragged.t)
    h, _, _ = prepared(torch, eda, ragged)
    res = h.solve(ragged.t, 1e-10, block=3, seed=2)
    check_solution(res, ref, ragged.t, red.lam_all, 1e-10)
    h.close()


def test_solve_deterministic(torch, eda, c1):
    log("solve C1 twice: bitwise identical")
    h, _, _ = prepared(torch, eda, c1)
    a = h.solve(c1.t, 1e-10, seed=7)
    Xa = host(a.X).copy()
    b = h.solve(c1.t, 1e-10, seed=7)
    assert a.ritz == b.ritz and np.array_equal(Xa, host(b.X))
    h.close()


def test_solve_iteration_limit_reports_noconv(torch, eda, c2):
    log("solve C2 max_iter=1")
    h, _, _ = prepared(torch, eda, c2)
    res = h.solve(c2.t, 1e-12, max_iter=5, seed=1, check_every=1)
    assert res.status == eda.EDA_ERR_NOCONV
    assert np.all(np.isfinite(res.ritz))
    h.close()


def test_degenerate_t_flag(torch, eda, ragged):
    log("t > k-1 sets the degenerate flag")
    h, _, _ = prepared(torch, eda, ragged)
    res = h.solve(6, 1e-8, block=2, seed=1)
    assert res.info["flags"] & eda.EDA_WARN_DEGENERATE
    h.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "fp8"])
@pytest.mark.parametrize("where", ["W", "B"])
def test_nonfinite_input_rejected(torch, eda, ragged, storage, where):
    """A NaN or Inf anywhere in either factor (checked by the pass that
    copies the factor) makes the preparation fail with EDA_ERR_NONFINITE;
    the same handle then prepares the clean factors."""
    for r, c, v in ((5, 3, np.nan), (ragged.d - 1, -1, np.inf), (0, 0, -np.inf)):
        log(f"{v} in H_{where}[{r}, {c}], {storage} storage")
        h = eda.Handle()
        HW, HB = ragged.H_W.copy(), ragged.H_B.copy()
        (HW if where == "W" else HB)[r, c] = v
        with pytest.raises(eda.EDAError) as ei:
            h.prepare(dev(torch, HW), dev(torch, HB), storage=storage)
        assert ei.value.status == eda.EDA_ERR_NONFINITE
        h.prepare(dev(torch, ragged.H_W), dev(torch, ragged.H_B), storage=storage)
        h.close()


def test_fp32_storage_c2(torch, eda, c2):
    """P stored in float32, float64 basis, no refinement.  Rounding P to
    float32 perturbs S_W, S_B by at most about 2 u32 ||H||^2 in norm, which
    moves log lambda by about 1e-6 (Theorem 3.2 type bound) and the span by
    at most lam_1 * that / gap (Davis-Kahan): tolerances 1e-5 and 1e-2."""
    log("solve C2 with float32 storage, no refinement")
    red = O.eda_reduced(c2.H_W, c2.H_B, c2.t)
    h, _, _ = prepared(torch, eda, c2, storage="f32")
    res = h.solve(c2.t, 1e-8, block=8, seed=2, max_refine=-1)
    lam = np.array(res.ritz)
    relerr = np.max(np.abs(lam - red.lam) / red.lam)
    ang = O.sin_angle(red.X, host(res.X))
    log(f"  status={res.status} lam_err={relerr:.2e} sin={ang:.2e}")
    assert res.status in (0, eda.EDA_ERR_NOCONV)
    assert res.info["refine_passes"] == 0
    assert relerr <= 1e-5 and ang <= 1e-2
    h.close()


# ---------------------------------------------------------------------------
# a8: narrow Krylov phase + float64 refinement
# ---------------------------------------------------------------------------

def errors(res, ref):
    lam = np.array(res.ritz)
    return np.max(np.abs(lam - ref.lam) / ref.lam), O.sin_angle(ref.X, host(res.X))


@pytest.mark.parametrize("storage,basis", [("f64", "f32"), ("f32", "f64"), ("f32", "f32"),
                                           ("bf16", "f64"), ("bf16", "f32"), ("fp8", "f32"),
                                           ("fp8", "f64")])
def test_mixed_refined_c2(torch, eda, c2, storage, basis):
    """The refined result meets the float64 bounds of the float64 solve.
    Before refinement (max_refine < 0) each Ritz value obeys the first-order
    bound of the narrow phase: the phase stops at residual 10 u_lo theta_1 /
    theta_i (u_lo the larger unit roundoff of storage and basis), which moves
    the eigenvalue by at most that much (relative to lam_i), and rounding P
    to the storage type perturbs S_W, S_B by at most 2 u_P ||P||_2 ||P||_F,
    which moves lam_i by at most twice that times lam_1 / lam_i (Frechet
    derivative of exp, as in the narrow-storage product test); a factor 2 of
    room on each term."""
    log(f"solve C2 storage={storage} basis={basis}: before and after refinement")
    red = O.eda_reduced(c2.H_W, c2.H_B, c2.t)
    h, _, _ = prepared(torch, eda, c2, storage=storage)
    pre = h.solve(c2.t, 1e-10, block=8, seed=2, krylov_dtype=basis, max_refine=-1)
    e_lam, e_ang = errors(pre, red)
    uu = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -8, "fp8": 2.0 ** -4}
    u_P = uu[storage] if storage != "f64" else 0.0
    u_lo = max(uu[storage], uu[basis])
    P = np.concatenate([c2.H_W, c2.H_B], axis=1)
    ratio = red.lam[0] / red.lam
    pre_tol = np.maximum(1e-10, 2 * 10 * u_lo * ratio
                         + 2 * 4 * u_P * np.linalg.norm(P, 2) * np.linalg.norm(P) * ratio)
    pre_err = np.abs(np.array(pre.ritz) - red.lam) / red.lam
    log(f"  before: status={pre.status} iters={pre.info['iters']} lam_err={e_lam:.2e} "
        f"(max err/bound {np.max(pre_err / pre_tol):.2e}) sin={e_ang:.2e} "
        f"resid={max(pre.resid):.2e}")
    assert pre.status in (0, eda.EDA_ERR_NOCONV)
    assert np.all(np.isfinite(pre.ritz)) and np.all(pre_err <= pre_tol)
    res = h.solve(c2.t, 1e-10, block=8, seed=2, krylov_dtype=basis)
    log(f"  after: passes={res.info['refine_passes']} refine_ms={res.info['t_refine_ms']:.2f}")
    check_solution(res, red, c2.t, red.lam_all, 1e-10)
    assert res.info["refine_passes"] <= 16
    h.close()


@pytest.mark.parametrize("cname", ["c1", "c2"])
def test_direct_solve_against_oracle(torch, eda, cname, request):
    """Reduced direct solve (row f2): the exact N x N reduction of the pencil
    on the GPU.  Its pairs are exact up to rounding, so they meet the oracle's
    exact reduction at the float64 bounds used for the converged Krylov
    solve, and agree with that solve."""
    case = request.getfixturevalue(cname)
    log(f"direct solve {case.name}")
    red = O.eda_reduced(case.H_W, case.H_B, case.t)
    h, _, _ = prepared(torch, eda, case)
    res = h.solve_direct(case.t)
    log(f"  status={res.status} ms={res.info['t_krylov_ms']:.2f} resid_max={max(res.resid):.2e}")
    check_solution(res, red, case.t, red.lam_all, 1e-12)
    kry = h.solve(case.t, 1e-10, block=8, seed=2)
    lam_d, lam_k = np.array(res.ritz), np.array(kry.ritz)
    lam_tol = np.maximum(1e-10, 100 * U * red.lam_all[0] / red.lam)
    assert np.all(np.abs(lam_d - lam_k) / lam_k <= lam_tol)
    h.close()


def test_direct_solve_rejects_t_above_rank(torch, eda, c1):
    h, _, _ = prepared(torch, eda, c1)
    N = c1.H_W.shape[1] + c1.H_B.shape[1]
    r = np.linalg.matrix_rank(np.concatenate([c1.H_W, c1.H_B], axis=1))
    assert r < N
    res = h.solve_direct(min(r + 1, 128), raise_on_error=False)
    assert res.status == eda.EDA_ERR_ARG and "rank" in res.message
    h.close()


@pytest.mark.parametrize("cname,block", [("c1", 8), ("c2", 8), ("ragged", 2)])
def test_aform_solve_against_oracle(torch, eda, cname, block, request):
    """Arnoldi form (row f1): eigenvectors of A = exp(-S_W) exp(S_B) by block
    Lanczos in the exp(S_W) inner product, returned without back-transform.
    Same bounds against the oracle as the Lanczos form, and the two forms
    agree with each other."""
    case = request.getfixturevalue(cname)
    log(f"A-form solve {case.name} b={block}")
    ref = O.eda_dense(case.H_W, case.H_B, case.t) if case.d <= 2000 else None
    red = O.eda_reduced(case.H_W, case.H_B, case.t)
    h, _, _ = prepared(torch, eda, case)
    res = h.solve(case.t, 1e-10, block=block, seed=3, form="A")
    check_solution(res, ref if ref is not None else red, case.t, red.lam_all, 1e-10)
    kry = h.solve(case.t, 1e-10, block=block, seed=3)
    lam_a, lam_m = np.array(res.ritz), np.array(kry.ritz)
    lam_tol = np.maximum(1e-10, 100 * U * red.lam_all[0] / red.lam)
    assert np.all(np.abs(lam_a - lam_m) / lam_m <= lam_tol)
    fl = O.accuracy_floor(red.lam_all, case.t)
    assert O.sin_angle(host(res.X), host(kry.X)) <= max(1e-8, 100 * fl["span"])
    h.close()


@pytest.mark.parametrize("cname,block", [("c1", 8), ("c2", 8), ("ragged", 3), ("c2", 4)])
def test_jd_solve_against_oracle(torch, eda, cname, block, request):
    """Block Jacobi-Davidson (row f4): the same pairs of e^{-s} M by
    Rayleigh-Ritz, projected correction equations solved by GMRES, and
    restarts to the t + b leading Ritz vectors.  Same bounds against the
    oracle as the Lanczos form, and the two solvers agree."""
    case = request.getfixturevalue(cname)
    log(f"JD solve {case.name} b={block}")
    ref = O.eda_dense(case.H_W, case.H_B, case.t) if case.d <= 2000 else None
    red = O.eda_reduced(case.H_W, case.H_B, case.t)
    h, _, _ = prepared(torch, eda, case)
    res = h.solve(case.t, 1e-10, block=block, seed=5, form="JD")
    check_solution(res, ref if ref is not None else red, case.t, red.lam_all, 1e-10)
    kry = h.solve(case.t, 1e-10, block=block, seed=5)
    lam_j, lam_m = np.array(res.ritz), np.array(kry.ritz)
    lam_tol = np.maximum(1e-10, 100 * U * red.lam_all[0] / red.lam)
    assert np.all(np.abs(lam_j - lam_m) / lam_m <= lam_tol)
    fl = O.accuracy_floor(red.lam_all, case.t)
    assert O.sin_angle(host(res.X), host(kry.X)) <= max(1e-8, 100 * fl["span"])
    h.close()


def test_jd_argument_checks_and_iteration_limit(torch, eda, c1):
    """The Jacobi-Davidson form refuses a float32 basis and reports
    EDA_ERR_NOCONV (outputs still written) when max_iter outer steps do not
    reach the tolerance."""
    h, _, _ = prepared(torch, eda, c1)
    r = h.solve(c1.t, 1e-10, form="JD", krylov_dtype="f32", raise_on_error=False)
    assert r.status == eda.EDA_ERR_ARG
    r = h.solve(c1.t, 1e-14, form="JD", max_iter=1, raise_on_error=False)
    assert r.status == eda.EDA_ERR_NOCONV
    assert r.info["iters"] == 1
    assert np.all(np.isfinite(np.array(r.ritz)))
    h.close()


def test_aform_thick_restart_c2(torch, eda, c2):
    log("A-form solve C2 with a small basis (thick restarts)")
    red = O.eda_reduced(c2.H_W, c2.H_B, c2.t)
    h, _, _ = prepared(torch, eda, c2)
    res = h.solve(c2.t, 1e-10, block=8, max_basis=72, seed=4, max_iter=3000, form="A")
    assert res.info["restarts"] >= 1
    check_solution(res, red, c2.t, red.lam_all, 1e-10)
    h.close()


def test_aform_argument_checks(torch, eda, c1):
    h, _, _ = prepared(torch, eda, c1)
    r = h.solve(c1.t, 1e-10, form="A", krylov_dtype="f32", raise_on_error=False)
    assert r.status == eda.EDA_ERR_ARG and "float64" in r.message
    # the basis may not reach the dimension n - 1 + b of the invariant hull
    r = h.solve(c1.t, 1e-10, form="A", max_basis=48, raise_on_error=False)
    assert r.status == eda.EDA_ERR_ARG and "max_basis" in r.message
    h.close()


def test_mixed_c1_agrees_per_column(torch, eda, c1):
    log("solve C1 with bfloat16 storage and float32 basis, refined")
    ref = O.eda_dense(c1.H_W, c1.H_B, c1.t)
    red = O.eda_reduced(c1.H_W, c1.H_B, c1.t)
    h, _, _ = prepared(torch, eda, c1, storage="bf16")
    res = h.solve(c1.t, 1e-10, block=8, seed=1, krylov_dtype="f32")
    X = check_solution(res, ref, c1.t, red.lam_all, 1e-10)
    assert np.abs(X - ref.X).max() <= 1e-8
    h.close()


def test_mixed_c3_full_size(torch, eda):
    """d = 32256, k = 38, n = 1216, t = 37, tol 1e-6: bfloat16 P, float32
    basis, float64 refinement, against the oracle's exact reduction and the
    float64 GPU solve.  Per-pair bounds follow the attainable floors, which
    are far above 1e-6 for the small pairs of this workload."""
    log("solve C3 full size: float64 and bfloat16+refinement")
    p = datagen.config("C3")
    case = Case("C3", p.X, p.counts, p.t)
    red = O.eda_reduced(case.H_W, case.H_B, p.t)
    for storage, basis in (("f64", "f64"), ("bf16", "f32")):
        h, _, _ = prepared(torch, eda, case, storage=storage)
        res = h.solve(p.t, p.tol, block=8, seed=3, krylov_dtype=basis)
        check_floored_solution(res, red, p.t, p.tol, f"{storage}/{basis}",
                               nu1=nu_max(case.H_W))
        h.close()


def test_mixed_c5_fp8_full_size(torch, eda):
    """d = 65536, k = 100, n = 2000, t = 99, tol 1e-6 (the large FP8
    workload): FP8 E4M3 P with per-column scales, float32 basis, float64
    refinement, against the oracle's exact reduction (and its stored values
    in tests/golden) and the float64 GPU solve."""
    from tests.golden.reader import read as read_golden
    log("solve C5 full size: float64 and fp8+refinement (oracle reduction first)")
    p = datagen.config("C5")
    g = read_golden("C5")
    case = Case("C5", p.X, p.counts, p.t)
    red = O.eda_reduced(case.H_W, case.H_B, p.t)
    # the stored values agree to the per-pair floor u lam_1 / lam_i (the
    # reduced pencil is solved in a different summation order here)
    assert np.all(np.abs(red.lam - g["lam"]) / red.lam
                  <= np.maximum(1e-12, 10 * np.array(g["pair_floor"])))
    log("  oracle done")
    for storage, basis in (("f64", "f64"), ("fp8", "f32")):
        h, _, _ = prepared(torch, eda, case, storage=storage)
        res = h.solve(p.t, p.tol, block=8, seed=3, krylov_dtype=basis)
        check_floored_solution(res, red, p.t, p.tol, f"{storage}/{basis}",
                               nu1=nu_max(case.H_W))
        h.close()


def test_autotune_records_shapes_and_keeps_results(torch, eda, c2, tmp_path, monkeypatch):
    """The autotuner (a9): valid shapes for the ORL-shaped class, written to
    the cache file; the product and the solve after tuning still meet the
    oracle's bounds."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("EDA_TUNE_CACHE", str(cache))
    h, _, _ = prepared(torch, eda, c2)
    V = dev(torch, datagen.start_block(c2.d, 8, 5))
    before, _ = h.opmv("M", V)
    before = host(before)
    r = h.autotune(c2.d, c2.H_W.shape[1] + c2.H_B.shape[1], 8, "f64")
    log(f"  autotune C2 class: {r}")
    assert r["tn_steps"] in (1, 2, 4, 8) and 0 <= r["nn_tile"] < 4
    assert r["tn_us"] > 0 and r["nn_us"] > 0
    lines = cache.read_text().split()
    assert "tn" in lines and "nn" in lines
    after, _ = h.opmv("M", V)
    after = host(after)
    assert np.abs(after - before).max() <= 1e-13 * np.abs(before).max()
    red = O.eda_reduced(c2.H_W, c2.H_B, c2.t)
    res = h.solve(c2.t, 1e-10, block=8, seed=2)
    check_solution(res, red, c2.t, red.lam_all, 1e-10)
    h.close()


# ---------------------------------------------------------------------------
# a9: many problems solved together
# ---------------------------------------------------------------------------

def _small_batch():
    """Uneven small problems: C1, the ragged case and four more shapes."""
    cases = []
    p = datagen.config("C1")
    cases.append(Case("C1", p.X, p.counts, p.t))
    counts = [2, 3, 4, 1, 5]
    cases.append(Case("ragged", datagen.make_samples(333, counts, 12, seed=21), counts, 4))
    rng = np.random.default_rng(77)
    for q in range(4):
        d = int(rng.choice([300, 700, 1500]))
        k = int(rng.integers(3, 12))
        cnt = rng.integers(2, 7, size=k).tolist()
        cases.append(Case(f"s{q}", datagen.make_samples(d, cnt, 24, seed=500 + q), cnt, k - 1))
    return cases


@pytest.mark.parametrize("storage,basis", [("f64", "f64"), ("f32", "f32")])
def test_batched_small_against_oracle(torch, eda, storage, basis):
    """Each problem of a batch meets the float64 bounds of a single solve."""
    log(f"batched solve of 6 uneven problems, storage={storage} basis={basis}")
    cases = _small_batch()
    h = eda.Handle()
    probs = []
    for c in cases:
        HW, HB = h.scatter_factors(dev(torch, c.X), c.counts.tolist())
        probs.append((HW, HB, c.t, 1e-10))
    res, st = h.solve_batched(probs, storage=storage, krylov_dtype=basis, seed=11)
    assert st == 0, res
    for c, r in zip(cases, res):
        red = O.eda_reduced(c.H_W, c.H_B, c.t)
        log(f"  {c.name}: d={c.d} t={c.t}")
        check_solution(r, red, c.t, red.lam_all, 1e-10)
    h.close()


def test_batched_agrees_with_single_solves(torch, eda):
    """Same start blocks (seed + index) and the same kernels: the batch and
    the one-by-one solves agree to rounding (the chunking of the row sums
    may differ with the largest problem of a launch)."""
    log("batched vs single solves")
    cases = _small_batch()[:4]
    h = eda.Handle()
    probs, singles = [], []
    for i, c in enumerate(cases):
        HW, HB = h.scatter_factors(dev(torch, c.X), c.counts.tolist())
        probs.append((HW, HB, c.t, 1e-10))
        hs = eda.Handle()
        hs.prepare(HW, HB)
        singles.append(hs.solve(c.t, 1e-10, seed=5 + i))
        hs.close()
    res, st = h.solve_batched(probs, seed=5)
    assert st == 0
    for c, r, s in zip(cases, res, singles):
        lam_b, lam_s = np.array(r.ritz), np.array(s.ritz)
        rel = np.max(np.abs(lam_b - lam_s) / lam_s)
        ang = O.sin_angle(host(s.X), host(r.X))
        log(f"  {c.name}: lam rel diff {rel:.1e} sin {ang:.1e} iters {r.info['iters']} vs {s.info['iters']}")
        assert rel <= 1e-11 and ang <= 1e-8
    h.close()


@pytest.fixture(scope="module")
def c4_batch():
    """The 64 problems of the batched workload with the oracle's exact
    reduction of each (d in {1024, 4096, 10304}, k in [10, 68], n_j in
    [2, 20], t = k - 1, tol 1e-6)."""
    ps = datagen.batched_configs(64)
    cases, reds = [], []
    for p in ps:
        c = Case(p.name, p.X, p.counts, p.t)
        cases.append(c)
        reds.append(O.eda_reduced(c.H_W, c.H_B, c.t))
    log(f"  oracle reductions of the 64 batched problems done")
    return ps, cases, reds


@pytest.mark.parametrize("storage,basis", [("f32", "f32"), ("f64", "f64")])
def test_batched_c4_all_problems(torch, eda, c4_batch, storage, basis):
    """All 64 problems of the batched workload in one call, every one against
    the oracle's exact reduction: residuals, Ritz values and span as for the
    single floored solves (graded spectra: the small pairs are held to their
    attainable float64 floors u lam_1 / lam_i).  With float32 storage, the
    problems whose float32 phase and refinement stall continue in float64
    (EDA_WARN_FALLBACK) and meet the same bounds."""
    ps, cases, reds = c4_batch
    log(f"batched C4, 64 problems, storage={storage} basis={basis}")
    h = eda.Handle()
    probs = []
    for p, c in zip(ps, cases):
        HW, HB = h.scatter_factors(dev(torch, c.X), c.counts.tolist())
        probs.append((HW, HB, c.t, p.tol))
    res, st = h.solve_batched(probs, storage=storage, krylov_dtype=basis, seed=4000)
    assert st == 0, [r.status for r in res]
    fell = [i for i, r in enumerate(res) if r.info["flags"] & eda.EDA_WARN_FALLBACK]
    log(f"  fell back: {fell}")
    if storage == "f64":
        assert not fell
    for i, (p, c, red, r) in enumerate(zip(ps, cases, reds, res)):
        check_floored_solution(r, red, c.t, p.tol,
                               f"{c.name} d={c.d} N={c.H_W.shape[1] + c.H_B.shape[1]} "
                               f"t={c.t}{' (fallback)' if i in fell else ''}",
                               nu1=nu_max(c.H_W))
    h.close()


def test_batched_float64_continuation(torch, eda, c4_batch):
    """Narrow problems with the float64 refinement switched off stall after
    their bfloat16 phase and continue as float64 block Lanczos solves started
    from their Ritz blocks, on their float64 masters: every one meets the
    floored float64 bounds against the oracle, and none needs more
    iterations than a float64 solve from a random start."""
    ps, cases, reds = c4_batch
    sel = list(range(0, 64, 8))
    log(f"batched float64 continuation, problems {sel}")
    h = eda.Handle()
    probs = []
    for i in sel:
        HW, HB = h.scatter_factors(dev(torch, cases[i].X), cases[i].counts.tolist())
        probs.append((HW, HB, cases[i].t, ps[i].tol))
    res, st = h.solve_batched(probs, storage="bf16", krylov_dtype="f32", seed=4100, max_refine=-1)
    assert st == 0, [r.status for r in res]
    cold, st2 = h.solve_batched(probs, storage="f64", krylov_dtype="f64", seed=4100)
    assert st2 == 0
    fell = [j for j, r in enumerate(res) if r.info["flags"] & eda.EDA_WARN_FALLBACK]
    log(f"  continued in float64: {fell}")
    assert fell, "no problem stalled without refinement"
    for j, i in enumerate(sel):
        r = res[j]
        check_floored_solution(r, reds[i], cases[i].t, ps[i].tol,
                               f"{cases[i].name} continuation={j in fell}", nu1=nu_max(cases[i].H_W))
    h.close()


def test_solve_graph_replays_match_eager(torch, eda, c2, monkeypatch):
    """Block steps replayed from captured graphs give the bitwise result of
    direct launches, on every replay, with other work and synchronisations
    of the program between the replays."""
    log("graph replays vs direct launches (C2)")
    h, _, _ = prepared(torch, eda, c2)
    monkeypatch.setenv("EDA_GRAPHS", "0")
    ref = h.solve(c2.t, 1e-10, seed=9)
    X0 = host(ref.X).copy()
    monkeypatch.setenv("EDA_GRAPHS", "1")
    V = dev(torch, np.random.default_rng(1).standard_normal((c2.d, 4)))
    for rep in range(3):
        r = h.solve(c2.t, 1e-10, seed=9)
        assert r.ritz == ref.ritz, f"replay {rep}"
        assert np.array_equal(host(r.X), X0), f"replay {rep}"
        h.expmv("W", -0.5, V)          # other work of the program in between
        torch.cuda.synchronize()
    h.close()


def test_solve_repair_every_step_matches(torch, eda, c1, monkeypatch):
    """The repair pass is left out away from the Krylov dimension bound; with
    it forced into every step the solve must give the same pairs to
    rounding (C1 reaches the bound, so both modes deflate)."""
    log("repair pass in every step vs only near the bound (C1)")
    ref = O.eda_dense(c1.H_W, c1.H_B, c1.t)
    h, _, _ = prepared(torch, eda, c1)
    a = h.solve(c1.t, 1e-10, seed=1)
    monkeypatch.setenv("EDA_ALWAYS_REPAIR", "1")
    b = h.solve(c1.t, 1e-10, seed=1)
    for r in (a, b):
        assert r.status == 0
        assert np.max(np.abs(np.array(r.ritz) - ref.lam) / ref.lam) <= 1e-10
        assert O.sin_angle(ref.X, host(r.X)) <= 1e-8
    h.close()
