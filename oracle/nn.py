"""Nearest-neighbour classification in the EDA subspace and the distance
bounds of Theorem 3.7 (Section 3.3), in float64.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: the product path never
imports it.

* The distance between a training sample x_i and a testing sample y_j is
  d_ij = ||V^T (x_i - y_j)||_2 for the orthonormal d x t matrix V of the
  computed (or exact) solution (Section 3.3, the distance definition before
  Theorem 3.7).  A testing sample takes the class of its nearest training
  sample (1-NN, Section 3.3).  The paper does not say how ties are broken;
  here the smallest training index wins.
* Theorem 3.7: for unit-norm samples and cos angle(V, W) != 0,
      (dW_ij - 2 sin) / cos <= dV_ij <= dW_ij cos + 2 sin,
  with sin = ||(I - V V^T) W||_2 and cos = ||V^T W||_2 (the theorem's
  definitions; the cosine as in its proof).
"""
from __future__ import annotations

import numpy as np

__all__ = ["nn_distances", "nn_classify", "cos_angle", "thm37_bounds"]


def nn_distances(V: np.ndarray, train: np.ndarray, test: np.ndarray) -> np.ndarray:
    """All d_ij = ||V^T (x_i - y_j)||_2, i over training and j over testing
    columns (n_train x n_test), by brute force over the pairs."""
    V = np.asarray(V, dtype=np.float64)
    P = V.T @ np.asarray(train, dtype=np.float64)   # t x n_train
    Q = V.T @ np.asarray(test, dtype=np.float64)    # t x n_test
    D = np.empty((P.shape[1], Q.shape[1]))
    for j in range(Q.shape[1]):
        diff = P - Q[:, j:j + 1]
        D[:, j] = np.sqrt(np.sum(diff * diff, axis=0))
    return D


def nn_classify(V, train, train_labels, test):
    """1-NN: (predicted labels, index of the nearest training sample, its
    distance) for every testing column; ties go to the smallest index."""
    D = nn_distances(V, train, test)
    idx = np.argmin(D, axis=0)          # first minimum: the smallest index
    labels = np.asarray(train_labels)[idx]
    return labels, idx, D[idx, np.arange(D.shape[1])]


def cos_angle(V: np.ndarray, W: np.ndarray) -> float:
    """cos angle(V, W) = ||V^T W||_2 for orthonormal V, W (proof of Theorem 3.7)."""
    return float(np.linalg.norm(V.T @ W, 2))


def thm37_bounds(dW: np.ndarray, sin: float, cos: float):
    """Lower and upper bounds on d^V_ij from d^W_ij (eq. (3.30))."""
    return (dW - 2.0 * sin) / cos, dW * cos + 2.0 * sin
