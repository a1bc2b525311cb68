"""Seeded synthetic inputs for exponential discriminant analysis (EDA).

This module is shared by the FP64 CPU oracle and by the GPU path, and it
holds none of the method's arithmetic: it only draws sample matrices X
(d x n, samples as columns, grouped class by class) together with the class
sizes n_j, and the Gaussian start blocks used by the Krylov solver.  Scatter
factors, exponentials and eigenproblems are computed by each side on its own.

Sample model (the paper's experiments use face images, which are not
available here; these inputs stand in for them with the same shapes):

    U      = orthonormal basis of a seeded d x r Gaussian matrix (QR)
    a_j    ~ N(0, I_r)                     class code of class j
    x      = U (a_j + 0.5 g) + 0.05 eps,   g ~ N(0, I_r), eps ~ N(0, I_d)
    x     <- x / ||x||_2                   every column has unit 2-norm,
                                           as in the paper's experimental setup
                                           (Section 4, setup paragraph)

Draw order from ``numpy.random.default_rng(seed)`` (PCG64): the d x r matrix
for U, then the k x r class codes, then for each class j in order an
n_j x r block of g followed by an n_j x d block of eps.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Problem",
    "make_samples",
    "make_split",
    "start_block",
    "config",
    "batched_configs",
    "CONFIG_NAMES",
]


@dataclasses.dataclass
class Problem:
    """One synthetic EDA input: X (d x n, Fortran order, float64) and n_j."""

    name: str
    d: int
    k: int
    counts: np.ndarray  # int64[k], class sizes n_j, classes stored contiguously
    r: int
    t: int
    seed: int
    X: Optional[np.ndarray] = None
    tol: float = 1e-8
    block: int = 8
    storage: str = "f64"

    @property
    def n(self) -> int:
        return int(self.counts.sum())

    @property
    def N(self) -> int:
        return self.n + self.k

    def labels(self) -> np.ndarray:
        return np.repeat(np.arange(self.k, dtype=np.int32), self.counts)


def make_samples(d: int, counts: Sequence[int], r: int, seed: int,
                 signal: float = 0.5, noise: float = 0.05) -> np.ndarray:
    """Return X (d x n, Fortran order, float64) with unit-norm columns."""
    counts = np.asarray(counts, dtype=np.int64)
    k = counts.size
    n = int(counts.sum())
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((d, r)))[0]
    A = rng.standard_normal((k, r))
    X = np.empty((d, n), dtype=np.float64, order="F")
    col = 0
    for j in range(k):
        nj = int(counts[j])
        G = rng.standard_normal((nj, r))
        E = rng.standard_normal((nj, d))
        Xj = U @ (A[j][None, :] + signal * G).T + noise * E.T
        Xj /= np.linalg.norm(Xj, axis=0, keepdims=True)
        X[:, col:col + nj] = Xj
        col += nj
    return X


def make_split(d: int, counts: Sequence[int], test_counts: Sequence[int], r: int, seed: int,
               signal: float = 0.5, noise: float = 0.05):
    """Training and testing samples of the same classes: X_train equals
    make_samples(d, counts, r, seed); the testing samples (test_counts[j]
    per class, same U and class codes) are drawn after all of it, class by
    class, an m_j x r block of g followed by an m_j x d block of eps.
    Returns (X_train, X_test, test_labels)."""
    counts = np.asarray(counts, dtype=np.int64)
    test_counts = np.asarray(test_counts, dtype=np.int64)
    k = counts.size
    if test_counts.size != k:
        raise ValueError("one test count per class")
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((d, r)))[0]
    A = rng.standard_normal((k, r))

    def draw(cs):
        out = np.empty((d, int(cs.sum())), dtype=np.float64, order="F")
        col = 0
        for j in range(k):
            nj = int(cs[j])
            G = rng.standard_normal((nj, r))
            E = rng.standard_normal((nj, d))
            Xj = U @ (A[j][None, :] + signal * G).T + noise * E.T
            Xj /= np.linalg.norm(Xj, axis=0, keepdims=True)
            out[:, col:col + nj] = Xj
            col += nj
        return out

    X_train = draw(counts)
    X_test = draw(test_counts)
    return X_train, X_test, np.repeat(np.arange(k, dtype=np.int32), test_counts)


def start_block(d: int, b: int, seed: int) -> np.ndarray:
    """Seeded Gaussian d x b start block (Fortran order), rng seed + 100."""
    rng = np.random.default_rng(seed + 100)
    return np.asfortranarray(rng.standard_normal((d, b)))


_SPECS = {
    # name: (d, k, n_j, r, t, tol, storage)
    "C1": (1024, 10, 5, 64, 9, 1e-10, "f64"),
    "C2": (10304, 40, 5, 128, 39, 1e-8, "f64"),
    "C3": (32256, 38, 32, 256, 37, 1e-6, "bf16"),
    "C5": (65536, 100, 20, 512, 99, 1e-6, "fp8"),
}
CONFIG_NAMES = ["C1", "C2", "C3", "C4", "C5"]


def config(name: str, with_data: bool = True) -> Problem:
    """The fixed workloads.

    C1: d=1024 (32x32 images), k=10 classes x 5 samples, t=9, r=64.
    C2: d=10304 (112x92 images), k=40 x 5, t=39, r=128, block 8, tol 1e-8.
    C3: d=32256 (192x168), k=38 x 32, t=37, r=256.
    C5: d=65536 (256x256), k=100 x 20, t=99, r=512.
    C4 is a batch; see ``batched_configs``.
    """
    if name not in _SPECS:
        raise KeyError(name)
    d, k, nj, r, t, tol, storage = _SPECS[name]
    seed = int(name[1:])
    counts = np.full(k, nj, dtype=np.int64)
    p = Problem(name=name, d=d, k=k, counts=counts, r=r, t=t, seed=seed,
                tol=tol, storage=storage)
    if with_data:
        p.X = make_samples(d, counts, r, seed)
    return p


def batched_configs(count: int = 64, with_data: bool = True) -> List[Problem]:
    """C4: independent problems of uneven shape (folds / resampled splits).

    d uniform in {1024, 4096, 10304}, k uniform in [10, 68], n_j uniform in
    [2, 20] per class, t = k - 1, r = 128; shapes drawn from
    default_rng(4), problem p's samples from seed 4000 + p.
    """
    rng = np.random.default_rng(4)
    out = []
    for p in range(count):
        d = int(rng.choice([1024, 4096, 10304]))
        k = int(rng.integers(10, 69))
        counts = rng.integers(2, 21, size=k).astype(np.int64)
        prob = Problem(name=f"C4.{p}", d=d, k=k, counts=counts, r=128,
                       t=k - 1, seed=4000 + p, tol=1e-6, storage="f32")
        if with_data:
            prob.X = make_samples(d, counts, 128, prob.seed)
        out.append(prob)
    return out
