"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types an oracle formula: each compares the oracle with a
different route (a library routine, a 50-digit power series, a closed form,
an identity, a bound, or brute force) so that a dropped term, a wrong sign or
index, or a transposed operand in the oracle fails at least one of them.
The ``TestMutants`` class plants such mistakes in copies of oracle functions
and checks that the pins catch them.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

import datagen
import oracle as O

RNG = np.random.default_rng(12345)


def small_problem(d=40, k=4, counts=None, r=8, seed=7):
    counts = np.asarray(counts if counts is not None else [3] * k)
    X = datagen.make_samples(d, counts, r, seed)
    H_W, H_B = O.scatter_factors(X, counts)
    return X, counts, H_W, H_B


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ----------------------------------------------------------------------------
# Check functions (shared by the pins and by the mutation tests)
# ----------------------------------------------------------------------------

def check_scatter(scatter_factors):
    """S_W + S_B equals the total scatter about the sample mean (a classical
    decomposition that holds only for the sample-weighted global centroid),
    class blocks of H_W sum to zero, and H_B [sqrt(n_j)] = 0."""
    counts = np.array([2, 5, 3, 7])
    X = datagen.make_samples(12, counts, 5, seed=3)
    H_W, H_B = scatter_factors(X, counts)
    m = X.mean(axis=1, keepdims=True)
    S_T = (X - m) @ (X - m).T
    ok = rel(H_W @ H_W.T + H_B @ H_B.T, S_T) < 1e-13
    offs = np.concatenate([[0], np.cumsum(counts)])
    for j in range(counts.size):
        ok &= np.abs(H_W[:, offs[j]:offs[j + 1]].sum(axis=1)).max() < 1e-14
    ok &= np.abs(H_B @ np.sqrt(counts)).max() < 1e-13
    # the sum forms of eqs. (1.1)-(1.2)
    S_W, S_B = O.scatter_sums(X, counts)
    ok &= rel(H_W @ H_W.T, S_W) < 1e-13 and rel(H_B @ H_B.T, S_B) < 1e-13
    return bool(ok)


def check_expm_vs_scipy(expm_sym):
    ok = True
    for trial in range(4):
        A = RNG.standard_normal((7, 7)) * (0.5 + trial)
        S = A + A.T
        for c in (1.0, -1.0, -0.5, 0.3):
            ok &= rel(expm_sym(S, c), scipy.linalg.expm(c * S)) < 1e-12
    return bool(ok)


def check_thm31(exp_action_thm31):
    _, _, H_W, H_B = small_problem(d=30, k=3, counts=[4, 2, 5])
    V = RNG.standard_normal((30, 3))
    ok = True
    for H, c in ((H_W, -1.0), (H_W, -0.5), (H_B, 1.0), (H_W, 2.0)):
        ok &= rel(exp_action_thm31(H, c, V), scipy.linalg.expm(c * H @ H.T) @ V) < 1e-12
    return bool(ok)


def check_example_1_1(eda_dense):
    """Example 1.1: three independent samples, one per class, so H_W = 0 and
    the pencil becomes exp(S_B) x = lam x.  Its eigenvalues are exp(sigma_i^2)
    for the singular values of H_B, together with exp(0) = 1 for the null
    direction, and the eigenvectors are H_B's left singular vectors."""
    X = np.asfortranarray(np.array([[1.0, 0.2, -0.3], [0.1, 0.9, 0.4], [0.2, -0.5, 1.1]]))
    counts = np.array([1, 1, 1])
    H_W, H_B = O.scatter_factors(X, counts)
    if np.abs(H_W).max() != 0.0:
        return False
    U, s, _ = np.linalg.svd(H_B)
    expect = np.sort(np.exp(s ** 2))[::-1]
    res = eda_dense(H_W, H_B, 3)
    ok = rel(res.lam, expect) < 1e-13
    # distinct eigenvalues: columns equal the singular vectors up to sign
    for i in range(3):
        ok &= abs(abs(res.X[:, i] @ U[:, i]) - 1.0) < 1e-12
    return bool(ok)


def check_dense_order(eda_dense):
    _, _, H_W, H_B = small_problem(d=25, k=4, counts=[3, 3, 2, 4])
    full = O.pencil_spectrum(H_W, H_B)
    res = eda_dense(H_W, H_B, 3)
    return bool(rel(res.lam, full[:3]) < 1e-12 and np.all(np.diff(res.lam) < 0))


# ----------------------------------------------------------------------------
# Pins
# ----------------------------------------------------------------------------

def test_scatter_factors_decomposition():
    assert check_scatter(O.scatter_factors)


def test_expm_sym_matches_pade_library():
    assert check_expm_vs_scipy(O.expm_sym)


@pytest.mark.parametrize("c", [1.0, -1.0, -0.5])
def test_expm_sym_matches_50_digit_power_series(c):
    H = RNG.standard_normal((5, 3)) * 0.9
    S = H @ H.T
    ref = O.expm_taylor_mp(S, c, digits=50)
    assert rel(O.expm_sym(S, c), ref) < 1e-14


def test_phi_identity_against_oracle_exponential():
    """exp(c H H^T) = I + H phi_c(H^T H) H^T, phi_c(z) = (e^{cz} - 1)/z,
    phi_c(0) = c: the power series of exp(c H H^T) with one H pulled out on
    each side.  Checked on rank-deficient scatter factors (H_W has rank n-k,
    H_B rank k-1) and on a generic H."""
    _, _, H_W, H_B = small_problem(d=20, k=3, counts=[3, 4, 2])
    for H in (H_W, H_B, RNG.standard_normal((9, 4))):
        lam, V = np.linalg.eigh(H.T @ H)
        for c in (1.0, -1.0, -0.5):
            with np.errstate(divide="ignore", invalid="ignore"):
                phi = np.where(np.abs(lam) > 1e-300, np.expm1(c * lam) / lam, c)
            E = np.eye(H.shape[0]) + H @ (V * phi) @ V.T @ H.T
            assert rel(E, O.expm_sym(H @ H.T, c)) < 1e-13


def test_thm31_route_matches_library_expm():
    assert check_thm31(O.exp_action_thm31)


def test_exp_of_between_scatter_spectrum_closed_form():
    """eig(exp(S_B)) = {exp(sigma_i(H_B)^2)} U {1} (Theorem 3.1, eq. 3.9)."""
    _, _, _, H_B = small_problem(d=30, k=5, counts=[3, 2, 4, 3, 2])
    s = np.linalg.svd(H_B, compute_uv=False)
    expect = np.sort(np.concatenate([np.exp(s ** 2), np.ones(30 - s.size)]))
    got = np.linalg.eigvalsh(O.expm_sym(H_B @ H_B.T, 1.0))
    assert np.max(np.abs(got - expect) / expect) < 1e-13


def test_exp_inverse_and_square_root_identities():
    """exp(S) exp(-S) = I (eq. 2.2) and exp(-S/2)^2 = exp(-S) (eq. 3.11)."""
    _, _, H_W, _ = small_problem(d=25, k=3)
    S = H_W @ H_W.T
    assert np.abs(O.expm_sym(S, 1.0) @ O.expm_sym(S, -1.0) - np.eye(25)).max() < 1e-13
    Eh = O.expm_sym(S, -0.5)
    assert rel(Eh @ Eh, O.expm_sym(S, -1.0)) < 1e-14


def test_lanczos_and_arnoldi_products_match_dense():
    _, _, H_W, H_B = small_problem(d=35, k=4, counts=[3, 2, 4, 3])
    V = RNG.standard_normal((35, 4))
    assert rel(O.lanczos_action_thm31(H_W, H_B, V), O.lanczos_matrix_dense(H_W, H_B) @ V) < 1e-12
    assert rel(O.arnoldi_action_thm31(H_W, H_B, V), O.arnoldi_matrix_dense(H_W, H_B) @ V) < 1e-12
    # and against the library exponential
    M = scipy.linalg.expm(-0.5 * H_W @ H_W.T) @ scipy.linalg.expm(H_B @ H_B.T) @ scipy.linalg.expm(-0.5 * H_W @ H_W.T)
    assert rel(O.lanczos_matrix_dense(H_W, H_B), M) < 1e-12


def test_example_1_1_closed_form():
    assert check_example_1_1(O.eda_dense)


def test_dense_returns_top_t_descending():
    assert check_dense_order(O.eda_dense)


def test_between_scatter_zero_case():
    """Equal class means give H_B = 0; the pencil is then I x = lam exp(S_W) x
    with eigenvalues exp(-sigma_i(H_W)^2) and 1."""
    rng = np.random.default_rng(5)
    d, counts = 10, np.array([3, 3])
    dev = 0.3 * rng.standard_normal((d, 6))
    dev[:, :3] -= dev[:, :3].mean(axis=1, keepdims=True)
    dev[:, 3:] -= dev[:, 3:].mean(axis=1, keepdims=True)
    X = np.asfortranarray(rng.standard_normal((d, 1)) + dev)
    H_W, H_B = O.scatter_factors(X, counts)
    assert np.abs(H_B).max() < 1e-14
    s = np.linalg.svd(H_W, compute_uv=False)
    expect = np.sort(np.concatenate([np.exp(-s ** 2), np.ones(d - s.size)]))[::-1]
    got = O.pencil_spectrum(H_W, H_B)
    assert np.max(np.abs(got - expect) / expect) < 1e-13


def test_orthogonal_factor_spaces_case():
    """If span(H_W) is orthogonal to span(H_B), the spectrum is
    {e^{sigma_B^2}} U {e^{-sigma_W^2}} U {1} (both exponentials act on
    orthogonal invariant subspaces, Theorem 3.1)."""
    rng = np.random.default_rng(6)
    Q = np.linalg.qr(rng.standard_normal((12, 12)))[0]
    H_B = Q[:, :3] @ rng.standard_normal((3, 3)) * 0.6
    H_W = Q[:, 3:7] @ rng.standard_normal((4, 5)) * 0.4
    sB = np.linalg.svd(H_B, compute_uv=False)
    sW = np.linalg.svd(H_W, compute_uv=False)[:4]
    expect = np.sort(np.concatenate([np.exp(sB ** 2), np.exp(-sW ** 2), np.ones(5)]))[::-1]
    got = O.pencil_spectrum(H_W, H_B)
    assert np.max(np.abs(got - expect) / expect) < 1e-12


def test_pencil_eigenvalues_positive_and_bounded_thm32():
    """Generalised eigenvalues are positive (SPD pencil) and satisfy the
    per-index bounds (3.17)-(3.18) of Theorem 3.2."""
    _, _, H_W, H_B = small_problem(d=40, k=4)
    lam = O.pencil_spectrum(H_W, H_B)
    assert np.all(lam > 0)
    mu = np.sort(np.linalg.eigvalsh(H_B @ H_B.T))[::-1]
    nu = np.sort(np.linalg.eigvalsh(H_W @ H_W.T))[::-1]
    lo, hi = O.eig_bounds_thm32(mu, nu)
    assert np.all(lam >= lo * (1 - 1e-12)) and np.all(lam <= hi * (1 + 1e-12))


def test_thm32_bounds_collapse_when_one_factor_vanishes():
    """With S_W = 0 the bounds of Theorem 3.2 pinch to exp(mu_i); with
    S_B = 0 to exp(-nu_{d-i+1}).  This pins the index bookkeeping."""
    mu = np.sort(RNG.uniform(0, 3, 9))[::-1]
    lo, hi = O.eig_bounds_thm32(mu, np.zeros(9))
    assert np.allclose(lo, np.exp(mu), rtol=1e-15) and np.allclose(hi, np.exp(mu), rtol=1e-15)
    nu = np.sort(RNG.uniform(0, 3, 9))[::-1]
    lo, hi = O.eig_bounds_thm32(np.zeros(9), nu)
    assert np.allclose(lo, np.exp(-nu[::-1]), rtol=1e-15) and np.allclose(hi, np.exp(-nu[::-1]), rtol=1e-15)


def test_unit_eigenvalue_count_thm36_and_exact_inertia():
    """Theorem 3.6: at least d-n+1 eigenvalues equal 1 for independent
    samples.  Sharper (Courant-Fischer on span[H_W H_B]): exactly k-1 above 1,
    d-n+1 equal to 1 and n-k below 1."""
    d, k, nj = 40, 4, 3
    _, _, H_W, H_B = small_problem(d=d, k=k, counts=[nj] * k)
    n = k * nj
    above, equal, below = O.inertia(O.pencil_spectrum(H_W, H_B), tol=1e-9)
    assert equal >= d - n + 1
    assert (above, equal, below) == (k - 1, d - n + 1, n - k)


def test_trace_ratio_bruteforce_lemma33_thm34():
    """Lemma 3.3: tr((V^T E_W V)^{-1} V^T E_B V) <= sum of the t largest
    eigenvalues, with equality on the dominant eigenspace.  Brute force over
    4 x 2 matrices (random search + local optimisation from random starts)
    must not beat the oracle, and its maximiser must span the oracle's X.
    Theorem 3.4 bounds the maximum."""
    rng = np.random.default_rng(8)
    d, t = 4, 2
    H_W = rng.standard_normal((d, 3)) * 0.7
    H_B = rng.standard_normal((d, 2)) * 0.8
    E_B, E_W = O.pencil_dense(H_W, H_B)
    res = O.eda_dense(H_W, H_B, t)
    best = res.lam.sum()
    assert abs(O.trace_ratio(res.X, E_B, E_W) - best) < 1e-12 * best
    samples = rng.standard_normal((20000, d, t))
    vals = [O.trace_ratio(V, E_B, E_W) for V in samples]
    assert max(vals) <= best * (1 + 1e-12)
    f = lambda v: -O.trace_ratio(v.reshape(d, t), E_B, E_W)
    opt = min((scipy.optimize.minimize(f, rng.standard_normal(d * t), method="BFGS",
                                       options={"gtol": 1e-12}) for _ in range(12)),
              key=lambda r: r.fun)
    assert abs(-opt.fun - best) < 1e-9 * best
    Vopt = np.linalg.qr(opt.x.reshape(d, t))[0]
    assert O.sin_angle(res.X, Vopt) < 1e-4
    mu = np.sort(np.linalg.eigvalsh(H_B @ H_B.T))[::-1]
    nu = np.sort(np.linalg.eigvalsh(H_W @ H_W.T))[::-1]
    lo, hi = O.rho_bounds_thm34(mu, nu, t)
    assert lo * (1 - 1e-12) <= best <= hi * (1 + 1e-12)


def test_lanczos_arnoldi_pencil_share_spectrum():
    """M, exp(-S_W)exp(S_B) and the pencil have the same eigenvalues, and
    x = exp(-S_W/2) y maps eigenvectors of M to pencil eigenvectors
    (eqs. 3.12-3.14)."""
    _, _, H_W, H_B = small_problem(d=20, k=3, counts=[3, 3, 3])
    M = O.lanczos_matrix_dense(H_W, H_B)
    A = O.arnoldi_matrix_dense(H_W, H_B)
    lm, Y = np.linalg.eigh(M)
    la = np.sort(np.linalg.eigvals(A).real)
    lp = np.sort(O.pencil_spectrum(H_W, H_B))
    assert np.max(np.abs(lm - lp) / lp) < 1e-12 and np.max(np.abs(la - lp) / lp) < 1e-10
    E_B, E_W = O.pencil_dense(H_W, H_B)
    x = O.expm_sym(H_W @ H_W.T, -0.5) @ Y
    R = E_B @ x - (E_W @ x) * lm
    assert np.abs(R).max() < 1e-12 * lm.max()


def test_orth_qr_follows_eigenvalue_order():
    """orth by QR keeps nested spans: span X[:, :i] = span x[:, :i]."""
    _, _, H_W, H_B = small_problem(d=30, k=5, counts=[2, 3, 3, 2, 3])
    res = O.eda_dense(H_W, H_B, 4)
    assert np.abs(res.X.T @ res.X - np.eye(4)).max() < 1e-14
    for i in range(1, 5):
        xi = np.linalg.qr(res.x[:, :i])[0]
        assert O.sin_angle(xi, res.X[:, :i]) < 1e-12
    # sign convention: largest-magnitude entry positive
    idx = np.argmax(np.abs(res.X), axis=0)
    assert np.all(res.X[idx, np.arange(4)] > 0)


def test_sin_angle_known_rotation():
    th = 0.123
    X = np.array([[1.0], [0.0], [0.0]])
    Y = np.array([[np.cos(th)], [np.sin(th)], [0.0]])
    assert abs(O.sin_angle(X, Y) - np.sin(th)) < 1e-15


def test_dense_and_reduced_agree_small():
    _, counts, H_W, H_B = small_problem(d=60, k=5, counts=[3, 4, 2, 5, 3])
    a = O.eda_dense(H_W, H_B, 4)
    b = O.eda_reduced(H_W, H_B, 4)
    assert np.max(np.abs(a.lam - b.lam) / a.lam) < 1e-12
    assert O.sin_angle(a.X, b.X) < 1e-11
    assert np.abs(a.X - b.X).max() < 1e-10  # same sign convention, distinct lam


@pytest.mark.slow
def test_dense_and_reduced_agree_c1():
    """O1 (dense d x d) against O2 (exact reduction) on the d=1024 workload."""
    p = datagen.config("C1")
    H_W, H_B = O.scatter_factors(p.X, p.counts)
    a = O.eda_dense(H_W, H_B, p.t)
    b = O.eda_reduced(H_W, H_B, p.t)
    assert np.max(np.abs(a.lam - b.lam) / a.lam) < 1e-12
    assert O.sin_angle(a.X, b.X) < 1e-10


# ----------------------------------------------------------------------------
# Mutation tests: plausible mistakes planted in copies of oracle functions.
# ----------------------------------------------------------------------------

class TestMutants:
    def test_unweighted_global_mean_is_caught(self):
        def bad(X, counts):
            H_W, H_B = O.scatter_factors(X, counts)
            offs = np.concatenate([[0], np.cumsum(counts)])
            mus = np.stack([X[:, offs[j]:offs[j + 1]].mean(axis=1) for j in range(len(counts))], 1)
            mu_bad = mus.mean(axis=1)
            return H_W, np.sqrt(counts)[None, :] * (mus - mu_bad[:, None])
        assert not check_scatter(bad)

    def test_missing_sqrt_weight_is_caught(self):
        def bad(X, counts):
            H_W, H_B = O.scatter_factors(X, counts)
            return H_W, H_B / np.sqrt(counts)[None, :]
        assert not check_scatter(bad)

    def test_transposed_eigenvectors_are_caught(self):
        def bad(S, c=1.0):
            mu, Z = np.linalg.eigh(S)
            return (Z.T * np.exp(c * mu)) @ Z
        assert not check_expm_vs_scipy(bad)

    def test_wrong_exponent_sign_is_caught(self):
        assert not check_expm_vs_scipy(lambda S, c=1.0: O.expm_sym(S, -c))

    def test_dropped_complement_term_is_caught(self):
        def bad(H, c, V):
            Qt, D = O.thm31_basis(H)
            return Qt @ (np.exp(c * D)[:, None] * (Qt.T @ V))
        assert not check_thm31(bad)

    def test_swapped_pencil_is_caught(self):
        def bad(H_W, H_B, t):
            return O.eda_dense(H_B, H_W, t)
        assert not check_example_1_1(bad)

    def test_ascending_order_is_caught(self):
        def bad(H_W, H_B, t):
            E_B, E_W = O.pencil_dense(H_W, H_B)
            lam, x = scipy.linalg.eigh(E_B, E_W)
            return O.EDAResult(lam=lam[:t], log_lam=np.log(lam[:t]), X=O.orth_qr(x[:, :t]), x=x[:, :t])
        assert not check_dense_order(bad)


# ----------------------------------------------------------------------------
# Stored reference values (tests/golden/oracle_*.txt, written by
# tests/golden/make_golden.py from the oracle) still match the oracle.
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["C1", "C2"])
def test_golden_values_match_oracle(name):
    from tests.golden.reader import read
    g = read(name)
    p = datagen.config(name)
    H_W, H_B = O.scatter_factors(p.X, p.counts)
    red = O.eda_reduced(H_W, H_B, p.t)
    assert np.max(np.abs(red.lam - g["lam"]) / g["lam"]) < 1e-12
    # and the top of the stored values within Theorem 3.2's bounds in reduced form:
    # lam_1 <= exp(mu_1 - nu_d) = exp(sigma_B,max^2) since nu_d = 0 for d > n
    assert g["lam"][0] <= np.exp(g["sigma2_B_max"]) * (1 + 1e-12)


# ----------------------------------------------------------------------------
# Reference E4M3 rounding of the FP8 storage tests (format facts, not paper)
# ----------------------------------------------------------------------------

def test_e4m3_codes():
    """Known codes of the OCP E4M3 format: 1.0 = 0x38, 1.5 = 0x3c, the
    largest finite 448 = 0x7e, the smallest normal 2^-6 = 0x08, the smallest
    subnormal 2^-9 = 0x01, NaN = 0x7f, and 0x80 = -0."""
    from oracle.fp8 import e4m3_decode, e4m3_values
    assert e4m3_decode(0x38) == 1.0
    assert e4m3_decode(0x3C) == 1.5
    assert e4m3_decode(0x7E) == 448.0
    assert e4m3_decode(0x08) == 2.0 ** -6
    assert e4m3_decode(0x01) == 2.0 ** -9
    assert np.isnan(e4m3_decode(0x7F))
    assert e4m3_decode(0x80) == 0.0 and np.signbit(e4m3_decode(0x80))
    v = e4m3_values()
    assert len(v) == 127 and np.all(np.diff(v) > 0)          # monotone, no duplicates
    # spacing: 2^-9 below 2^-5, then 8 values per binade
    assert np.allclose(np.diff(v[:16]), 2.0 ** -9)
    assert np.all(np.diff(v[v >= 1.0][:8]) == 0.125)


def test_e4m3_rounding():
    """Nearest with ties to even, saturation, subnormals, sign symmetry."""
    from oracle.fp8 import e4m3_round
    cases = {
        1.0 + 1.0 / 16: 1.0,        # tie between 1.0 (m=0) and 1.125 (m=1): even
        1.0 + 3.0 / 16: 1.25,       # tie between 1.125 (m=1) and 1.25 (m=2): even
        1.0 + 1.0 / 15: 1.125,      # above the tie
        500.0: 448.0,               # saturates
        460.0: 448.0,
        2.0 ** -10: 0.0,            # half the smallest subnormal: tie to 0
        3 * 2.0 ** -10: 2.0 ** -8,  # 1.5 quanta: tie to 2 quanta
        0.3: 0.3125,                # 0.3 = 1.2 * 2^-2 -> 1.25 * 2^-2
    }
    for x, want in cases.items():
        assert e4m3_round(np.array([x]))[0] == want, x
        assert e4m3_round(np.array([-x]))[0] == -want, -x
    x = RNG.standard_normal(2000) * 10
    r = e4m3_round(x)
    small = np.abs(x) < 2.0 ** -6
    rel_err = np.abs(r - x)[~small] / np.abs(x)[~small]
    assert rel_err.max() <= 2.0 ** -4 * (1 + 1e-12)           # half an ulp of 3 bits
    assert np.abs(r - x)[small].max(initial=0.0) <= 2.0 ** -10


def test_fp8_columns_scale():
    """Each column's largest entry maps to 448 exactly; zero columns keep
    scale 1; exact E4M3 multiples of a power of two survive unchanged."""
    from oracle.fp8 import fp8_columns, e4m3_values
    P = RNG.standard_normal((50, 4))
    P[:, 2] = 0.0
    Q, s = fp8_columns(P)
    assert s[2] == 1.0 and np.all(Q[:, 2] == 0.0)
    for j in (0, 1, 3):
        i = np.argmax(np.abs(P[:, j]))
        assert np.isclose(abs(P[i, j]) / s[j], 448.0)
        assert Q[i, j] == P[i, j] * (1 + 0.0) or np.isclose(Q[i, j], P[i, j], rtol=1e-15)
    vals = e4m3_values()
    E = RNG.choice(vals, size=(30, 3)) * RNG.choice([-1.0, 1.0], size=(30, 3))
    E[0, :] = 448.0
    E *= 2.0 ** np.array([-3, 0, 5])
    Q, s = fp8_columns(E)
    assert np.array_equal(Q, E) and np.array_equal(s, 2.0 ** np.array([-3, 0, 5]))


# ----------------------------------------------------------------------------
# Reference bfloat16 rounding (format facts, not paper): one rounding from
# float64, ties to even.
# ----------------------------------------------------------------------------

def test_bf16_codes_known_values():
    """Codes fixed by the format: 1 = 0x3f80, -2 = 0xc000, the smallest
    subnormal 2^-133 = 0x0001, the smallest normal 2^-126 = 0x0080, the
    largest finite (2 - 2^-7) 2^127 = 0x7f7f, infinity 0x7f80, and the
    nearest values of pi (3.140625 = 0x4049) and 1/3 (0.333984375 = 0x3eab)."""
    from oracle.bf16 import bf16_codes, bf16_decode, BF16_MAX
    cases = {1.0: 0x3F80, -2.0: 0xC000, 2.0 ** -133: 0x0001, 2.0 ** -126: 0x0080,
             BF16_MAX: 0x7F7F, np.inf: 0x7F80, np.pi: 0x4049, 1.0 / 3.0: 0x3EAB,
             0.0: 0x0000}
    for x, code in cases.items():
        assert int(bf16_codes(np.array([x]))[0]) == code, (x, hex(code))
    assert bf16_decode(np.array([0x4049]))[0] == 3.140625
    assert bf16_decode(np.array([0x3EAB]))[0] == 0.333984375
    assert np.signbit(bf16_decode(np.array([0x8000]))[0])


def test_bf16_rounding_ties_and_single_rounding():
    """Ties go to the even significand; a value just above a tie rounds up
    even when its float32 rounding would land on the tie (the double
    rounding float64 -> float32 -> bfloat16 gets that case wrong); overflow
    to infinity happens exactly at the midpoint above the largest finite."""
    from oracle.bf16 import bf16_round, BF16_MAX
    cases = {
        1.0 + 2.0 ** -8: 1.0,                      # tie between m = 0 and m = 1: even
        1.0 + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6,      # tie between m = 1 and m = 2: even
        1.0 + 2.0 ** -8 + 2.0 ** -30: 1.0 + 2.0 ** -7,   # above the tie, below float32's ulp
        1.0 + 2.0 ** -8 - 2.0 ** -40: 1.0,         # below the tie
        3 * 2.0 ** -134: 2.0 ** -132,              # subnormal tie (1.5 quanta): even = 2
        2.0 ** -134: 0.0,                          # half the smallest subnormal: to 0
        2.0 ** -134 + 2.0 ** -160: 2.0 ** -133,    # just above it
        BF16_MAX + 2.0 ** 119: np.inf,             # the midpoint to 2^128: ties to even = inf
        BF16_MAX + 2.0 ** 119 - 2.0 ** 100: BF16_MAX,
    }
    for x, want in cases.items():
        assert bf16_round(np.array([x]))[0] == want, x
        assert bf16_round(np.array([-x]))[0] == -want, -x
    x = np.float64(1.0 + 2.0 ** -8 + 2.0 ** -30)
    assert float(np.float32(x)) == 1.0 + 2.0 ** -8   # float32 hop lands on the tie


def test_bf16_rounding_error_bound_and_idempotence():
    """|round(x) - x| <= 2^-8 |x| for normal x (half an ulp of 7 stored bits),
    rounding is idempotent, monotone, and exact on values with 8 significant
    bits."""
    from oracle.bf16 import bf16_round
    x = RNG.standard_normal(5000) * 10.0 ** RNG.uniform(-30, 30, 5000)
    r = bf16_round(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-15))
    assert np.array_equal(bf16_round(r), r)
    s = np.sort(x)
    assert np.all(np.diff(bf16_round(s)) >= 0)
    m = RNG.integers(128, 256, 1000).astype(np.float64) * 2.0 ** RNG.integers(-40, 40, 1000)
    assert np.array_equal(bf16_round(m), m)


# ----------------------------------------------------------------------------
# The attainable-accuracy report (oracle.accuracy_floor) against Weyl's and
# Davis-Kahan's perturbation theorems on matrices with a chosen spectrum:
# the report claims that an absolute perturbation of size u * lam_1 (one
# product's rounding) moves pair i by at most u lam_1 / lam_i relatively and
# the top-t span by at most u lam_1 / gap.  Both bounds are attained by
# specific perturbations, so a floor that is too small fails the random
# checks and one that is too large fails the attainment checks.
# ----------------------------------------------------------------------------

def _spectral_matrix(spec, rng):
    """Symmetric matrix Q diag(spec) Q^T with a random orthogonal Q."""
    Q = np.linalg.qr(rng.standard_normal((len(spec), len(spec))))[0]
    return (Q * spec) @ Q.T, Q


def _top_span(M, t):
    w, Z = np.linalg.eigh(0.5 * (M + M.T))
    return w[::-1], Z[:, ::-1][:, :t]


def check_accuracy_floor(accuracy_floor):
    """True when accuracy_floor's pair and span floors match the perturbation
    theory of the spectra below (unit cluster present, absent, t = N)."""
    rng = np.random.default_rng(31)
    ok = True
    # (reduced spectrum lam_all, t, multiplicity of the unit eigenvalue in the
    # full problem: d - N complement directions)
    cases = [
        (np.array([400.0, 90.0, 12.0, 3.0, 0.6, 0.4, 0.2]), 3, 4),   # lam_{t+1} > 1
        (np.array([400.0, 90.0, 12.0, 1.3, 0.6, 0.4, 0.2]), 4, 4),   # unit cluster closest
        (np.array([400.0, 90.0, 12.0, 0.8, 0.6]), 3, 3),             # lam_{t+1} < 1 < lam_t
        (np.array([50.0, 7.0, 2.5]), 3, 5),                          # t = N: gap to the unit cluster
        (np.array([50.0, 7.0, 2.5, 0.3]), 2, 0),                     # no complement (d = N)
    ]
    u = 1e-9   # a perturbation level far above float64 rounding
    for lam_all, t, n_unit in cases:
        spec = np.concatenate([lam_all, np.ones(n_unit)])
        fl = accuracy_floor(lam_all, t, u=u, unit_cluster=n_unit > 0)
        M, Q = _spectral_matrix(spec, rng)
        eps = u * lam_all[0]
        order = np.argsort(-spec, kind="stable")
        q = Q[:, order]                           # eigenvectors by decreasing eigenvalue
        _, X0 = _top_span(M, t)
        # Weyl: no perturbation of norm eps moves lam_i by more than eps
        for _ in range(3):
            E = rng.standard_normal(M.shape)
            E = E + E.T
            E *= eps / np.linalg.norm(E, 2)
            w, X = _top_span(M + E, t)
            ok &= np.all(np.abs(w[:t] - lam_all[:t]) / lam_all[:t] <= fl["pair"] * (1 + 1e-6))
            ok &= O.sin_angle(X0, X) <= fl["span"] * (1 + 1e-3)
        # attained: E = eps q_i q_i^T moves lam_i by exactly eps
        for i in range(t):
            w, _ = _top_span(M + eps * np.outer(q[:, i], q[:, i]), t)
            ok &= abs((w[i] - lam_all[i]) / lam_all[i] / fl["pair"][i] - 1.0) < 1e-4
        # attained to first order: coupling q_t with the closest unwanted
        # eigenvector rotates the span by eps / gap
        jn = int(np.argmin(np.abs(spec[order][t:] - lam_all[t - 1]))) + t
        E = eps * (np.outer(q[:, t - 1], q[:, jn]) + np.outer(q[:, jn], q[:, t - 1]))
        _, X = _top_span(M + E, t)
        with np.errstate(divide="ignore"):
            ok &= abs(O.sin_angle(X0, X) / fl["span"] - 1.0) < 1e-3
    return bool(ok)


def test_accuracy_floor_matches_perturbation_theory():
    assert check_accuracy_floor(O.accuracy_floor)


def test_accuracy_floor_hand_values_and_default_unit_roundoff():
    """Hand values: lam = [100, 10, 0.5], t = 2 -> pair floors u [1, 10],
    span u * 100 / (10 - 1) with the unit eigenvalue, u * 100 / 9.5 without;
    the default u is the float64 unit roundoff 2^-53 = eps / 2."""
    lam = np.array([100.0, 10.0, 0.5])
    f = O.accuracy_floor(lam, 2)
    u = np.finfo(np.float64).eps / 2
    assert f["pair"][0] == u and f["pair"][1] == 10 * u
    assert f["span"] == u * 100 / 9.0 and f["gap"] == 9.0
    g = O.accuracy_floor(lam, 2, unit_cluster=False)
    assert g["span"] == u * 100 / 9.5
    h = O.accuracy_floor(np.array([100.0, 10.0]), 2)          # t = N
    assert h["gap"] == 9.0


def test_rho_bounds_thm34_collapse_and_hand_case():
    """Theorem 3.4's bounds on the EDA criterion are the minimum and maximum
    over all V of the trace ratio (Lemma 3.3) when one factor vanishes:
    with S_W = 0 they are the sums of the t smallest and t largest exp(mu_i),
    with S_B = 0 those of exp(-nu_i).  A hand case fixes the index pairing:
    mu = (3, 1, 0), nu = (2, 0.5, 0), t = 2 gives
    lower = max(e^{1-2}, e^{0-0.5}) + max(e^{0-2}, e^{0-2}) = e^{-1/2} + e^{-2},
    upper = min(e^{3-0}, e^{3-0}) + min(e^{1-0}, e^{3-0.5}) = e^3 + e."""
    rng = np.random.default_rng(5)
    d, t = 7, 3
    mu = np.sort(rng.uniform(0, 2, d))[::-1]
    lo, hi = O.rho_bounds_thm34(mu, np.zeros(d), t)
    assert np.isclose(lo, np.exp(mu[-t:]).sum(), rtol=1e-15)
    assert np.isclose(hi, np.exp(mu[:t]).sum(), rtol=1e-15)
    nu = np.sort(rng.uniform(0, 2, d))[::-1]
    lo, hi = O.rho_bounds_thm34(np.zeros(d), nu, t)
    assert np.isclose(lo, np.exp(-nu[:t]).sum(), rtol=1e-15)
    assert np.isclose(hi, np.exp(-nu[-t:]).sum(), rtol=1e-15)
    lo, hi = O.rho_bounds_thm34(np.array([3.0, 1.0, 0.0]), np.array([2.0, 0.5, 0.0]), 2)
    assert np.isclose(lo, np.exp(-0.5) + np.exp(-2.0), rtol=1e-15)
    assert np.isclose(hi, np.exp(3.0) + np.exp(1.0), rtol=1e-15)
    # and on a real problem both bounds contain the extreme trace ratios
    _, _, H_W, H_B = small_problem(d=12, k=3, counts=[2, 2, 2])
    lam = O.pencil_spectrum(H_W, H_B)
    mu = np.sort(np.linalg.eigvalsh(H_B @ H_B.T))[::-1]
    nu = np.sort(np.linalg.eigvalsh(H_W @ H_W.T))[::-1]
    lo, hi = O.rho_bounds_thm34(mu, nu, t)
    assert lo * (1 - 1e-12) <= lam[-t:].sum() and lam[:t].sum() <= hi * (1 + 1e-12)


class TestFloorAndBoundMutants:
    """Plausible slips in the accuracy report and in the criterion bounds."""

    def test_off_by_one_gap_index_is_caught(self):
        def bad(lam_all, t, u=2.0 ** -53, unit_cluster=True):
            f = O.accuracy_floor(lam_all, t, u, unit_cluster)
            nxt = lam_all[t + 1] if lam_all.size > t + 1 else -np.inf
            if unit_cluster:
                nxt = max(nxt, 1.0)
            gap = lam_all[t - 1] - nxt
            return {"pair": f["pair"], "span": u * lam_all[0] / gap, "gap": gap}
        assert not check_accuracy_floor(bad)

    def test_previous_pair_gap_is_caught(self):
        def bad(lam_all, t, u=2.0 ** -53, unit_cluster=True):
            f = O.accuracy_floor(lam_all, t, u, unit_cluster)
            gap = lam_all[t - 2] - lam_all[t - 1]
            return {"pair": f["pair"], "span": u * lam_all[0] / gap, "gap": gap}
        assert not check_accuracy_floor(bad)

    def test_ignored_unit_cluster_is_caught(self):
        def bad(lam_all, t, u=2.0 ** -53, unit_cluster=True):
            return O.accuracy_floor(lam_all, t, u, unit_cluster=False)
        assert not check_accuracy_floor(bad)

    def test_pair_floor_against_lam_t_is_caught(self):
        def bad(lam_all, t, u=2.0 ** -53, unit_cluster=True):
            f = O.accuracy_floor(lam_all, t, u, unit_cluster)
            return {"pair": u * lam_all[0] / lam_all[t - 1] * np.ones(t), "span": f["span"],
                    "gap": f["gap"]}
        assert not check_accuracy_floor(bad)

    def test_wrong_unit_roundoff_is_caught(self):
        import inspect
        default_u = inspect.signature(O.accuracy_floor).parameters["u"].default
        assert default_u == np.finfo(np.float64).eps / 2      # 2^-52 would fail here
        assert 2.0 ** -52 != np.finfo(np.float64).eps / 2

    def test_shifted_mu_index_in_rho_lower_bound_is_caught(self):
        def bad(mu, nu, t):
            d = mu.size
            i = np.arange(1, t + 1)
            lo = np.maximum(np.exp(mu[np.minimum(d - t + i, d - 1)] - nu[0]),
                            np.exp(mu[d - 1] - nu[t - i]))
            return float(lo.sum()), O.rho_bounds_thm34(mu, nu, t)[1]
        mu = np.sort(RNG.uniform(0, 2, 7))[::-1]
        lo, _ = bad(mu, np.zeros(7), 3)
        assert not np.isclose(lo, np.exp(mu[-3:]).sum(), rtol=1e-12)

    def test_reversed_nu_index_in_rho_upper_bound_is_caught(self):
        def bad(mu, nu, t):
            d = mu.size
            i = np.arange(1, t + 1)
            hi = np.minimum(np.exp(mu[i - 1] - nu[d - 1]), np.exp(mu[0] - nu[i - 1]))
            return O.rho_bounds_thm34(mu, nu, t)[0], float(hi.sum())
        nu = np.sort(RNG.uniform(0, 2, 7))[::-1]
        _, hi = bad(np.zeros(7), nu, 3)
        assert not np.isclose(hi, np.exp(-nu[-3:]).sum(), rtol=1e-12)
