"""Plain FP64 reference implementation of EDA (test infrastructure only).

Each function states the passage of the paper it follows.  No blocking,
fusion or reordering beyond the definition: readable against the paper.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.linalg

__all__ = [
    "scatter_factors",
    "scatter_sums",
    "expm_sym",
    "expm_taylor_mp",
    "exp_action_dense",
    "thm31_basis",
    "exp_action_thm31",
    "lanczos_matrix_dense",
    "arnoldi_matrix_dense",
    "lanczos_action_thm31",
    "arnoldi_action_thm31",
    "pencil_dense",
    "EDAResult",
    "eda_dense",
    "eda_reduced",
    "pencil_spectrum",
    "orth_qr",
    "sign_fix",
    "sin_angle",
    "trace_ratio",
    "eig_bounds_thm32",
    "rho_bounds_thm34",
    "inertia",
    "accuracy_floor",
]


# ---------------------------------------------------------------------------
# Scatter factors: Section 1, eqs. (1.1) and (1.2).
# ---------------------------------------------------------------------------

def _class_slices(counts):
    counts = np.asarray(counts, dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(counts)])
    return [slice(int(offs[j]), int(offs[j + 1])) for j in range(counts.size)]


def scatter_factors(X: np.ndarray, counts) -> tuple[np.ndarray, np.ndarray]:
    """H_W (d x n) and H_B (d x k) for samples X grouped class by class.

    Section 1: mu_j is the centroid of class j, mu the global centroid of the
    training set (the mean of all n samples); H_W stacks X_j - mu_j e^T,
    H_B stacks sqrt(n_j) (mu_j - mu), so S_W = H_W H_W^T (eq. 1.1) and
    S_B = H_B H_B^T (eq. 1.2).
    """
    X = np.asarray(X, dtype=np.float64)
    counts = np.asarray(counts, dtype=np.int64)
    mu = X.mean(axis=1)
    H_W = np.empty_like(X, order="F")
    H_B = np.empty((X.shape[0], counts.size), order="F")
    for j, sl in enumerate(_class_slices(counts)):
        mu_j = X[:, sl].mean(axis=1)
        H_W[:, sl] = X[:, sl] - mu_j[:, None]
        H_B[:, j] = np.sqrt(counts[j]) * (mu_j - mu)
    return H_W, H_B


def scatter_sums(X: np.ndarray, counts) -> tuple[np.ndarray, np.ndarray]:
    """S_W and S_B by the sum forms of eqs. (1.1)-(1.2) (outer products)."""
    X = np.asarray(X, dtype=np.float64)
    d = X.shape[0]
    mu = X.mean(axis=1)
    S_W = np.zeros((d, d))
    S_B = np.zeros((d, d))
    for j, sl in enumerate(_class_slices(counts)):
        mu_j = X[:, sl].mean(axis=1)
        for i in range(sl.start, sl.stop):
            dv = X[:, i] - mu_j
            S_W += np.outer(dv, dv)
        dm = mu_j - mu
        S_B += (sl.stop - sl.start) * np.outer(dm, dm)
    return S_W, S_B


# ---------------------------------------------------------------------------
# Matrix exponential: Section 2.
# ---------------------------------------------------------------------------

def expm_sym(S: np.ndarray, c: float = 1.0) -> np.ndarray:
    """exp(c S) for symmetric S via S = Z diag(mu) Z^T (Section 2, eq. 2.3)."""
    S = np.asarray(S, dtype=np.float64)
    mu, Z = np.linalg.eigh(0.5 * (S + S.T))
    return (Z * np.exp(c * mu)) @ Z.T


def expm_taylor_mp(A: np.ndarray, c: float = 1.0, digits: int = 50) -> np.ndarray:
    """exp(c A) by the power series sum_j (cA)^j / j! (Section 2, eq. 2.1).

    Evaluated in mpmath at ``digits`` significant digits until the term is
    below 10^-digits relative to the running sum; tiny inputs only.
    """
    import mpmath

    with mpmath.workdps(digits + 10):
        M = mpmath.matrix(np.asarray(A, dtype=np.float64).tolist()) * mpmath.mpf(c)
        n = M.rows
        term = mpmath.eye(n)
        total = mpmath.eye(n)
        j = 0
        eps = mpmath.mpf(10) ** (-digits)
        while True:
            j += 1
            term = term * M / j
            total = total + term
            if mpmath.mnorm(term, 1) <= eps * mpmath.mnorm(total, 1):
                break
            if j > 10000:
                raise RuntimeError("series did not converge")
        return np.array([[float(total[i, k]) for k in range(n)] for i in range(n)])


def exp_action_dense(H: np.ndarray, c: float, V: np.ndarray) -> np.ndarray:
    """exp(c H H^T) V with the d x d exponential formed densely."""
    return expm_sym(H @ H.T, c) @ V


# ---------------------------------------------------------------------------
# Closed form of Theorem 3.1 / Algorithm 2 (skinny QR, SVD of R).
# ---------------------------------------------------------------------------

def thm31_basis(H: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(Q~, D) with H = Q R (eq. 3.3), R = U Sigma V^T (eq. 3.4),
    Q~ = Q U and D = Sigma^2 (eqs. 3.5-3.6); Algorithm 2, steps 2-4."""
    Q, R = np.linalg.qr(np.asarray(H, dtype=np.float64), mode="reduced")
    U, sig, _ = np.linalg.svd(R)
    return Q @ U, sig ** 2


def exp_action_thm31(H: np.ndarray, c: float, V: np.ndarray) -> np.ndarray:
    """exp(c H H^T) V = Q~ exp(cD) Q~^T V + V - Q~ Q~^T V.

    Theorem 3.1, eqs. (3.9)-(3.11) (c = 1, -1, -1/2), as steps (i)/(ii) of the
    remark after the theorem and steps 7-10 of Algorithm 2.
    """
    Qt, D = thm31_basis(H)
    W = Qt.T @ V
    return Qt @ (np.exp(c * D)[:, None] * W) + V - Qt @ W


def lanczos_matrix_dense(H_W, H_B) -> np.ndarray:
    """M = exp(-S_W/2) exp(S_B) exp(-S_W/2), eq. (3.15), formed densely."""
    Eh = expm_sym(H_W @ H_W.T, -0.5)
    return Eh @ expm_sym(H_B @ H_B.T, 1.0) @ Eh


def arnoldi_matrix_dense(H_W, H_B) -> np.ndarray:
    """A = exp(-S_W) exp(S_B), eq. (3.1), formed densely."""
    return expm_sym(H_W @ H_W.T, -1.0) @ expm_sym(H_B @ H_B.T, 1.0)


def lanczos_action_thm31(H_W, H_B, V) -> np.ndarray:
    """M V by steps (iii)-(v) of Section 3.1 (product eq. 3.16)."""
    V = exp_action_thm31(H_W, -0.5, V)
    V = exp_action_thm31(H_B, 1.0, V)
    return exp_action_thm31(H_W, -0.5, V)


def arnoldi_action_thm31(H_W, H_B, V) -> np.ndarray:
    """A V by steps (i)-(ii) of Section 3.1 (product eq. 3.2)."""
    V = exp_action_thm31(H_B, 1.0, V)
    return exp_action_thm31(H_W, -1.0, V)


# ---------------------------------------------------------------------------
# The EDA eigenproblem: Algorithm 1, pencil (1.7).
# ---------------------------------------------------------------------------

def pencil_dense(H_W, H_B) -> tuple[np.ndarray, np.ndarray]:
    """(exp(S_B), exp(S_W)) formed densely (Algorithm 1, step 1)."""
    return expm_sym(H_B @ H_B.T, 1.0), expm_sym(H_W @ H_W.T, 1.0)


def sign_fix(X: np.ndarray) -> np.ndarray:
    """Flip each column so its largest-magnitude entry is positive."""
    X = np.array(X, dtype=np.float64, order="F", copy=True)
    idx = np.argmax(np.abs(X), axis=0)
    s = np.sign(X[idx, np.arange(X.shape[1])])
    s[s == 0] = 1.0
    return X * s[None, :]


def orth_qr(x: np.ndarray) -> np.ndarray:
    """Orthonormalise the columns in their given order by a QR decomposition
    (Algorithm 1 step 4 / Algorithm 3 step 6; Section 4 says orth is done by
    QR), then fix signs."""
    Q, _ = np.linalg.qr(np.asarray(x, dtype=np.float64), mode="reduced")
    return sign_fix(Q)


@dataclasses.dataclass
class EDAResult:
    lam: np.ndarray        # t dominant generalised eigenvalues, descending
    log_lam: np.ndarray    # their logarithms
    X: np.ndarray          # d x t orthonormal, QR of x in descending-lambda order
    x: np.ndarray          # d x t raw generalised eigenvectors
    lam_all: Optional[np.ndarray] = None  # every eigenvalue computed, descending


def _gen_eig_top(E_B, E_W, t, full=False):
    d = E_B.shape[0]
    if full:
        lam, x = scipy.linalg.eigh(E_B, E_W)
    else:
        lam, x = scipy.linalg.eigh(E_B, E_W, subset_by_index=[d - t, d - 1])
    order = np.argsort(lam)[::-1]
    return lam[order], x[:, order]


def eda_dense(H_W, H_B, t: int, full: bool = False) -> EDAResult:
    """Algorithm 1: form exp(S_B), exp(S_W), solve exp(S_B)x = lam exp(S_W)x
    (eq. 1.7), sort by decreasing lam, orthonormalise the top t.

    The pencil is symmetric-definite (both exponentials are SPD), so the
    symmetric-definite LAPACK driver is used instead of eig of
    exp(S_W)^{-1} exp(S_B); the eigenpairs are the same.
    """
    E_B, E_W = pencil_dense(H_W, H_B)
    lam, x = _gen_eig_top(E_B, E_W, t, full=full)
    lam_t, x_t = lam[:t], x[:, :t]
    return EDAResult(lam=lam_t, log_lam=np.log(lam_t), X=orth_qr(x_t), x=x_t,
                     lam_all=lam if full else None)


def eda_reduced(H_W, H_B, t: int) -> EDAResult:
    """Exact reduction of the pencil to dimension N = n + k (all d).

    With [H_W H_B] = Q_P R (Householder QR, Q_P d x N orthonormal), both
    exp(S_W) and exp(S_B) leave span(Q_P) invariant and equal the identity
    on its orthogonal complement (Theorem 3.1, eqs. 3.7-3.8 with f = exp).
    So the pencil splits into the N x N pencil of R_W = Q_P^T H_W,
    R_B = Q_P^T H_B plus the eigenvalue 1 on the complement.  The N x N
    pencil is solved by ``eda_dense`` unchanged and lifted by x = Q_P z.
    ``lam_all`` holds the full spectrum of the N x N block.
    """
    P = np.concatenate([H_W, H_B], axis=1)
    Q, _ = np.linalg.qr(P, mode="reduced")
    R_W = Q.T @ H_W
    R_B = Q.T @ H_B
    N = P.shape[1]
    if t > N:
        raise ValueError("t exceeds the reduced dimension")
    with np.errstate(invalid="ignore"):
        red = eda_dense(R_W, R_B, N, full=True)
    lam_t = red.lam_all[:t]
    x_t = Q @ red.x[:, :t]
    return EDAResult(lam=lam_t, log_lam=np.log(lam_t), X=orth_qr(x_t), x=x_t,
                     lam_all=red.lam_all)


def pencil_spectrum(H_W, H_B) -> np.ndarray:
    """Every generalised eigenvalue of (exp(S_B), exp(S_W)), descending."""
    E_B, E_W = pencil_dense(H_W, H_B)
    lam = scipy.linalg.eigh(E_B, E_W, eigvals_only=True)
    return np.sort(lam)[::-1]


# ---------------------------------------------------------------------------
# Measures and bounds used as checks.
# ---------------------------------------------------------------------------

def sin_angle(X: np.ndarray, Y: np.ndarray) -> float:
    """sin angle(X, Y) = ||(I - X X^T) Y||_2 for orthonormal X, Y (Section 3.3)."""
    R = Y - X @ (X.T @ Y)
    return float(np.linalg.norm(R, 2))


def trace_ratio(V, E_B, E_W) -> float:
    """The EDA criterion tr((V^T E_W V)^{-1} V^T E_B V) of eq. (1.6)."""
    return float(np.trace(np.linalg.solve(V.T @ E_W @ V, V.T @ E_B @ V)))


def eig_bounds_thm32(mu: np.ndarray, nu: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Bounds (3.17)-(3.18) of Theorem 3.2 on lambda_i(M), i = 1..d.

    mu, nu: eigenvalues of S_B and S_W in decreasing order (length d).
    lower_i = max(e^{mu_i - nu_1}, e^{mu_d - nu_{d-i+1}}),
    upper_i = min(e^{mu_i - nu_d}, e^{mu_1 - nu_{d-i+1}}).
    """
    mu = np.asarray(mu)
    nu = np.asarray(nu)
    d = mu.size
    i = np.arange(1, d + 1)
    lower = np.maximum(np.exp(mu[i - 1] - nu[0]), np.exp(mu[d - 1] - nu[d - i]))
    upper = np.minimum(np.exp(mu[i - 1] - nu[d - 1]), np.exp(mu[0] - nu[d - i]))
    return lower, upper


def rho_bounds_thm34(mu: np.ndarray, nu: np.ndarray, t: int) -> tuple[float, float]:
    """Bounds (3.24)-(3.25) of Theorem 3.4 on the maximal EDA criterion rho."""
    mu = np.asarray(mu)
    nu = np.asarray(nu)
    d = mu.size
    i = np.arange(1, t + 1)
    lo = np.maximum(np.exp(mu[d - t + i - 1] - nu[0]), np.exp(mu[d - 1] - nu[t - i]))
    hi = np.minimum(np.exp(mu[i - 1] - nu[d - 1]), np.exp(mu[0] - nu[d - i]))
    return float(lo.sum()), float(hi.sum())


def inertia(lam: np.ndarray, tol: float = 1e-10) -> tuple[int, int, int]:
    """Counts of eigenvalues above, equal to (within tol) and below 1."""
    lam = np.asarray(lam)
    above = int(np.sum(lam > 1 + tol))
    below = int(np.sum(lam < 1 - tol))
    return above, lam.size - above - below, below


def accuracy_floor(lam_all: np.ndarray, t: int, u: float = 2.0 ** -53,
                   unit_cluster: bool = True) -> dict:
    """Attainable accuracy of any linear-scale FP method at working precision u.

    Every product with M carries an absolute error of order u * lam_1, so the
    relative error of pair i cannot drop below about u lam_1 / lam_i and the
    span error below about u lam_1 / (lam_t - lam_{t+1}).  With
    ``unit_cluster`` the eigenvalue 1 of the complement of span[H_W H_B]
    counts among the unwanted ones.
    """
    lam_all = np.asarray(lam_all)
    lam1 = lam_all[0]
    nxt = lam_all[t] if lam_all.size > t else -np.inf
    if unit_cluster:
        nxt = max(nxt, 1.0)
    gap = lam_all[t - 1] - nxt
    return {
        "pair": u * lam1 / lam_all[:t],
        "span": u * lam1 / gap,
        "gap": gap,
    }
