"""GPU parity on cases whose answer the paper (or the format) fixes in closed
form, on the edge cases of the method, and on the byte-level encoding of the
stored factor.  Every case runs through the C ABI; the reference is a closed
form where one exists (Theorem 3.1, the example of Section 2 with H_W = 0,
orthogonal factor spaces), else the FP64 CPU oracle.
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


# ---------------------------------------------------------------------------
# a1: the stored factor, code by code
# ---------------------------------------------------------------------------

def test_factor_codes_bf16_bit_exact(torch, eda):
    """bfloat16 storage: every stored code equals the reference rounding of
    the float64 entry, rounded once with ties to even (oracle/bf16.py).  The
    factor holds exact ties, values just above a tie that the float32 hop
    would move onto it, values just below a tie, subnormals and random
    entries over many binades."""
    from oracle.bf16 import bf16_codes
    log("factor codes, bfloat16 storage")
    rng = np.random.default_rng(41)
    d, n, k = 517, 13, 4
    P = rng.standard_normal((d, n + k)) * 10.0 ** rng.uniform(-6, 3, (d, n + k))
    special = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -30,
                        1 + 2.0 ** -8 - 2.0 ** -40, 3 * 2.0 ** -134, 2.0 ** -134,
                        2.0 ** -134 + 2.0 ** -160, 2.0 ** -133, 0.0, -0.0, np.pi, 1 / 3])
    scales = 2.0 ** rng.integers(-20, 20, special.size)
    for i, v in enumerate(special):
        P[7 + i, i % (n + k)] = v * (scales[i] if abs(v) > 2.0 ** -120 else 1.0)
        P[40 + i, (3 * i) % (n + k)] = -v
    h = eda.Handle()
    h.prepare(dev(torch, P[:, :n]), dev(torch, P[:, n:]), storage="bf16")
    codes, _ = h.factor_codes()
    got = host(codes).view(np.uint16)
    want = bf16_codes(P)
    bad = np.argwhere(got != want)
    log(f"  mismatches: {len(bad)} of {got.size}")
    assert bad.size == 0, [(tuple(ix), P[tuple(ix)], hex(got[tuple(ix)]), hex(want[tuple(ix)]))
                           for ix in bad[:5]]
    h.close()


def _e4m3_codes(vals):
    """Codes of values that are exact E4M3 numbers (index in the table of
    non-negative values, sign bit 0x80)."""
    from oracle.fp8 import e4m3_values
    table = e4m3_values()
    idx = np.searchsorted(table, np.abs(vals))
    assert np.all(table[idx] == np.abs(vals))
    return (idx | np.where(np.signbit(vals), 0x80, 0)).astype(np.uint8)


def test_factor_codes_fp8_bit_exact(torch, eda):
    """FP8 E4M3 storage of the C1 factors and of a ragged factor: the
    per-column scales equal max |P(:, j)| / 448 exactly and every code is the
    reference rounding (nearest, ties to even, oracle/fp8.py) of
    P(:, j) / scale_j."""
    from oracle.fp8 import e4m3_round
    p = datagen.config("C1")
    HW, HB = O.scatter_factors(p.X, p.counts)
    counts = [2, 3, 4, 1, 5]
    HW2, HB2 = O.scatter_factors(datagen.make_samples(333, counts, 12, seed=21), counts)
    for name, H_W, H_B in (("C1", HW, HB), ("ragged", HW2, HB2)):
        log(f"factor codes, FP8 storage, {name}")
        P = np.concatenate([H_W, H_B], axis=1)
        h = eda.Handle()
        h.prepare(dev(torch, H_W), dev(torch, H_B), storage="fp8")
        codes, sc = h.factor_codes()
        mx = np.max(np.abs(P), axis=0)
        s_ref = np.where(mx > 0, mx / 448.0, 1.0)
        assert np.array_equal(host(sc), s_ref)
        want = _e4m3_codes(e4m3_round(P / s_ref))
        got = host(codes)
        # -0 and +0 both decode to zero; compare values for zeros
        zero = (want & 0x7F) == 0
        assert np.array_equal(got[~zero], want[~zero]), int(np.sum(got[~zero] != want[~zero]))
        assert np.all((got[zero] & 0x7F) == 0)
        h.close()


# ---------------------------------------------------------------------------
# Closed forms of Theorem 3.1 and the example of Section 2 on the GPU
# ---------------------------------------------------------------------------

def _check_pairs(res, lam_ref, X_ref, lam_tol, ang_tol):
    lam = np.array(res.ritz)
    relerr = np.abs(lam - lam_ref) / lam_ref
    X = host(res.X)
    ang = O.sin_angle(X_ref, X) if X_ref is not None else 0.0
    log(f"  status={res.status} iters={res.info['iters']} lam_err={relerr.max():.2e} "
        f"sin={ang:.2e} resid={max(res.resid):.2e}")
    assert res.status == 0, res.message
    assert np.all(relerr <= lam_tol), relerr
    assert ang <= ang_tol
    assert np.abs(X.T @ X - np.eye(X.shape[1])).max() <= 1e-13
    return X


def test_example_hw_zero_tiny_direct(torch, eda):
    """The example of Section 2: three samples, one per class, so H_W = 0 and
    the pencil is exp(S_B) x = lam x with lam = exp(sigma_i(H_B)^2) and 1; the
    eigenvectors are the left singular vectors of H_B.  d = 3 leaves no room
    for a Krylov basis, so the reduced direct solve (row f2) takes it."""
    X = np.asfortranarray(np.array([[1.0, 0.2, -0.3], [0.1, 0.9, 0.4], [0.2, -0.5, 1.1]]))
    HW, HB = O.scatter_factors(X, [1, 1, 1])
    assert np.all(HW == 0.0)
    Ub, sb, _ = np.linalg.svd(HB)
    lam_ref = np.exp(sb[:2] ** 2)
    log("H_W = 0, d = 3 (Section 2 example), direct solve")
    h = eda.Handle()
    h.prepare(dev(torch, HW), dev(torch, HB))
    res = h.solve_direct(2)
    _check_pairs(res, lam_ref, O.orth_qr(Ub[:, :2]), 1e-12, 1e-12)
    h.close()


def test_hw_zero_krylov_closed_form(torch, eda):
    """H_W = 0 at d = 300 (one sample per class, k = 12): exp(S_B) only, so
    lam_i = exp(sigma_i(H_B)^2), i <= k-1, and the eigenvectors are H_B's left
    singular vectors; the Krylov space saturates at rank H_B = k-1 (deflation
    on every problem-sized block)."""
    k = 12
    X = datagen.make_samples(300, [1] * k, 16, seed=61)
    HW, HB = O.scatter_factors(X, [1] * k)
    assert np.all(HW == 0.0)
    Ub, sb, _ = np.linalg.svd(HB, full_matrices=False)
    t = k - 1
    lam_ref = np.exp(sb[:t] ** 2)
    log(f"H_W = 0, d = 300, k = {k}, Krylov solve; lam_1/lam_t = {lam_ref[0] / lam_ref[-1]:.1f}")
    h = eda.Handle()
    Hw, Hb = h.scatter_factors(dev(torch, X), [1] * k)
    h.prepare(Hw, Hb)
    res = h.solve(t, 1e-10, block=4, seed=3)
    lam_tol = np.maximum(1e-10, 50 * U * lam_ref[0] / lam_ref)
    _check_pairs(res, lam_ref, O.orth_qr(Ub[:, :t]), lam_tol, 1e-8)
    h.close()


def test_hb_zero_closed_form(torch, eda):
    """H_B = 0 (every class centroid equals the global one): exp(S_B) = I, so
    the pencil is x = lam exp(S_W) x with lam = exp(-nu_i) and 1; the top pairs
    are the unit eigenvalue, whose eigenspace span(H_W)^perp has dimension
    d - rank H_W.  Any orthonormal t vectors of it are correct: the check is
    lam = 1 and X orthogonal to span H_W."""
    rng = np.random.default_rng(62)
    d, k, nj = 250, 4, 4
    base = rng.standard_normal((d, nj // 2))
    cols = []
    for _ in range(k):
        c = rng.standard_normal((d, nj // 2)) * 0.1 + base * 0.05
        cols.append(np.concatenate([c, -c], axis=1))          # class mean 0
    X = np.asfortranarray(np.concatenate(cols, axis=1))
    counts = [nj] * k
    HW, HB = O.scatter_factors(X, counts)
    assert np.abs(HB).max() < 1e-15
    HB = np.zeros_like(HB)
    log("H_B = 0: top pairs are the unit eigenvalue")
    h = eda.Handle()
    h.prepare(dev(torch, HW), dev(torch, HB))
    t = 3
    res = h.solve(t, 1e-12, block=4, seed=5)
    assert res.status == 0, res.message
    Xg = host(res.X)
    log(f"  lam={res.ritz} |H_W^T X|={np.abs(HW.T @ Xg).max():.2e}")
    assert np.all(np.abs(np.array(res.ritz) - 1.0) <= 1e-12)
    # residual 1e-12 leaves components in span H_W of at most 1e-12 / (1 - e^{-nu_min})
    nu = np.linalg.svd(HW, compute_uv=False) ** 2
    nu_min = nu[nu > 1e-10 * nu[0]].min()
    assert np.abs(HW.T @ Xg).max() <= 1e-9 / (1 - np.exp(-nu_min)) * np.linalg.norm(HW, 2)
    assert np.abs(Xg.T @ Xg - np.eye(t)).max() <= 1e-13
    h.close()


def test_orthogonal_factor_spaces_closed_form(torch, eda):
    """span H_W orthogonal to span H_B: S_W S_B = 0, the exponentials commute
    and the spectrum is exp(sigma_B^2), 1 and exp(-sigma_W^2) (Theorem 3.1 on
    each factor); the top k eigenvectors are H_B's left singular vectors."""
    rng = np.random.default_rng(63)
    d, n, k = 2000, 24, 6
    Q = np.linalg.qr(rng.standard_normal((d, n + k)))[0]
    Ob = np.linalg.qr(rng.standard_normal((k, k)))[0]
    Ow = np.linalg.qr(rng.standard_normal((n, n)))[0]
    HB = Q[:, :k] @ (np.linspace(2.0, 0.8, k)[:, None] * Ob)      # sigma_B = 2.0 ... 0.8
    HW = Q[:, k:] @ (np.linspace(1.5, 0.1, n)[:, None] * Ow)      # sigma_W = 1.5 ... 0.1
    Ub, sb, _ = np.linalg.svd(HB, full_matrices=False)
    t = k
    lam_ref = np.exp(sb ** 2)
    log(f"orthogonal factor spaces d={d} n={n} k={k}: lam = {lam_ref.round(3).tolist()}")
    h = eda.Handle()
    h.prepare(dev(torch, HW), dev(torch, HB))
    res = h.solve(t, 1e-11, block=4, seed=6)
    lam_tol = np.maximum(1e-10, 50 * U * lam_ref[0] / lam_ref)
    gap = lam_ref[-1] - 1.0
    _check_pairs(res, lam_ref, O.orth_qr(Ub), lam_tol, max(1e-8, 50 * U * lam_ref[0] / gap))
    # the product itself: exp(S_B) V and exp(-S_W/2) V by the closed form of
    # Theorem 3.1 through each factor's singular vectors
    V = rng.standard_normal((d, 8))
    for which, H, c in (("B", HB, 1.0), ("W", HW, -0.5)):
        Uh, sh, _ = np.linalg.svd(H, full_matrices=False)
        ref = V + Uh @ ((np.exp(c * sh ** 2) - 1.0)[:, None] * (Uh.T @ V))
        out, s = h.expmv(which, c, dev(torch, V))
        err = np.linalg.norm(host(out) * np.exp(s) - ref) / (np.exp(max(0, c) * sh[0] ** 2)
                                                             * np.linalg.norm(V))
        log(f"  product {which} c={c}: err={err:.2e}")
        assert err <= 1e-13
    h.close()


# ---------------------------------------------------------------------------
# Edge cases of the method
# ---------------------------------------------------------------------------

def test_more_samples_than_dimensions(torch, eda):
    """n > d (the small-sample assumption k <= n << d of the cost remark of
    Section 3.1 fails): N = n + k = 330 > d = 200, no unit-eigenvalue
    complement, so the floors use the gap to lam_{t+1} alone; against the
    oracle's dense pencil (Algorithm 1)."""
    counts = [10] * 30
    X = datagen.make_samples(200, counts, 64, seed=64)
    HW, HB = O.scatter_factors(X, counts)
    t = 29
    ref = O.eda_dense(HW, HB, t, full=True)
    fl = O.accuracy_floor(ref.lam_all, t, unit_cluster=False)
    log(f"n > d: d=200 n=300 k=30 t={t}; lam_t={ref.lam[-1]:.3f} lam_t+1={ref.lam_all[t]:.3f}")
    h = eda.Handle()
    Hw, Hb = h.scatter_factors(dev(torch, X), counts)
    h.prepare(Hw, Hb)
    res = h.solve(t, 1e-10, block=8, seed=7)
    lam_tol = np.maximum(1e-10, 50 * U * ref.lam[0] / ref.lam)
    _check_pairs(res, ref.lam, ref.X, lam_tol, max(1e-8, 50 * fl["span"]))
    h.close()


def test_t_above_k_minus_1(torch, eda):
    """t > k - 1: the wanted set takes unit eigenvalues from the degenerate
    eigenspace span(P)^perp, so several results are correct.  Unique parts are
    compared with the oracle (the k - 1 leading eigenvalues and their span);
    the rest must be valid: eigenvalue 1 and the extra columns orthogonal to
    span P = span[H_W H_B]."""
    counts = [2, 3, 4, 1, 5]
    X = datagen.make_samples(333, counts, 12, seed=21)
    HW, HB = O.scatter_factors(X, counts)
    k = len(counts)
    t = 7
    red = O.eda_reduced(HW, HB, k - 1)
    log(f"t={t} > k-1={k - 1}")
    h = eda.Handle()
    Hw, Hb = h.scatter_factors(dev(torch, X), counts)
    h.prepare(Hw, Hb)
    res = h.solve(t, 1e-12, block=3, seed=8)
    assert res.status == 0, res.message
    assert res.info["flags"] & eda.EDA_WARN_DEGENERATE
    lam = np.array(res.ritz)
    Xg = host(res.X)
    P = np.concatenate([HW, HB], axis=1)
    top_err = np.max(np.abs(lam[:k - 1] - red.lam) / red.lam)
    ang = O.sin_angle(red.X, Xg[:, :k - 1])
    extra = np.abs(P.T @ Xg[:, k - 1:]).max() / np.linalg.norm(P, 2)
    log(f"  top lam_err={top_err:.2e} sin={ang:.2e} extra lam={lam[k - 1:]} |P^T X_extra|={extra:.2e}")
    # residual 1e-12 leaves the extra columns within 1e-12 / gap of span(P)^perp,
    # gap = 1 - (largest eigenvalue below 1) of the reduced pencil
    below = red.lam_all[red.lam_all < 1 - 1e-9]
    gap_low = 1.0 - below.max()
    assert top_err <= 1e-10 and ang <= 1e-8
    assert np.all(np.abs(lam[k - 1:] - 1.0) <= 1e-12)
    assert extra <= max(1e-11, 1e-10 / gap_low)
    assert np.abs(Xg.T @ Xg - np.eye(t)).max() <= 1e-13
    h.close()


# ---------------------------------------------------------------------------
# a4 component by component, in the eigenbasis of S (Theorem 3.1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("which,c", [("B", 1.0), ("W", -0.5), ("W", -1.0)])
def test_expmv_components_in_eigenbasis_c2(torch, eda, which, c):
    """exp(cS)V = Q~ e^{cD} Q~^T V + (I - Q~ Q~^T) V (Theorem 3.1) compared
    component by component: the error in eigen-direction i is held to
    1e-13 e^{c mu_i} |q_i^T V| plus the rounding that the largest term leaves
    in every component, N u e^{c mu_1}||V|| (the second pass forms sums of
    N terms whose size is set by the largest exponential); the complement's
    error to the same rounding term."""
    p = datagen.config("C2")
    HW, HB = O.scatter_factors(p.X, p.counts)
    H = HB if which == "B" else HW
    log(f"expmv components C2 which={which} c={c}")
    Qt, D = O.thm31_basis(H)
    keep = D > 1e-12 * D.max()
    Qt, D = Qt[:, keep], D[keep]
    V = np.random.default_rng(19).standard_normal((p.d, 8))
    h = eda.Handle()
    Hw, Hb = h.scatter_factors(dev(torch, p.X), p.counts.tolist())
    h.prepare(Hw, Hb)
    out, s = h.expmv(which, c, dev(torch, V))
    got = host(out) * np.exp(s)
    W = Qt.T @ V
    ref = Qt @ (np.exp(c * D)[:, None] * W) + V - Qt @ W
    err = got - ref
    N = p.n + p.k
    big = N * U * np.exp(max(0.0, c * D.max())) * np.linalg.norm(V, axis=0)
    comp = np.abs(Qt.T @ err)                          # per eigen-direction, per column
    comp_tol = 1e-13 * np.exp(c * D)[:, None] * np.abs(W) + big[None, :]
    perp = np.linalg.norm(err - Qt @ (Qt.T @ err), axis=0)
    log(f"  max comp/tol={np.max(comp / comp_tol):.2e} perp={perp.max():.2e} "
        f"big={big.max():.2e}")
    assert np.all(comp <= comp_tol)
    assert np.all(perp <= big)
    h.close()
