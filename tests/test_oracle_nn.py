"""Pins of the nearest-neighbour classifier and of Theorem 3.7 (Section 3.3)
in the oracle: hand-computed distances and labels, closed forms of the
subspace angle, the theorem's bounds on random perturbations, and the
generator's train/test split."""
import numpy as np
import pytest

import datagen
import oracle as O
from oracle import nn


def test_hand_example_distances_and_labels():
    # V spans the first two coordinates; distances are those of the first
    # two entries, worked out by hand
    V = np.eye(3)[:, :2]
    train = np.array([[1.0, 0.0, 0.0, 0.6],
                      [0.0, 1.0, 0.0, 0.8],
                      [0.0, 0.0, 1.0, 0.0]])
    labels = np.array([10, 11, 12, 13])
    test = np.array([[0.9, 0.5, 0.0],
                     [0.1, 0.7, 0.0],
                     [0.4, 0.5, 1.0]])
    D = nn.nn_distances(V, train, test)
    expect = np.array([
        [np.sqrt(0.02), np.sqrt(0.74), 1.0],
        [np.sqrt(1.62), np.sqrt(0.34), 1.0],
        [np.sqrt(0.82), np.sqrt(0.74), 0.0],
        [np.sqrt(0.58), np.sqrt(0.02), 1.0],
    ])
    np.testing.assert_allclose(D, expect, rtol=0, atol=1e-15)
    lab, idx, dist = nn.nn_classify(V, train, labels, test)
    assert idx.tolist() == [0, 3, 2]
    assert lab.tolist() == [10, 13, 12]
    np.testing.assert_allclose(dist, [np.sqrt(0.02), np.sqrt(0.02), 0.0], atol=1e-15)


def test_ties_go_to_the_smallest_index():
    V = np.eye(3)[:, 2:3]            # the third coordinate only
    train = np.array([[1.0, 0.0, 0.0, 0.6],
                      [0.0, 1.0, 0.0, 0.8],
                      [0.0, 0.0, 1.0, 0.0]])
    test = np.array([[0.6], [0.8], [0.0]])   # distance 0 to columns 0, 1 and 3
    lab, idx, dist = nn.nn_classify(V, train, np.array([5, 6, 7, 8]), test)
    assert idx.tolist() == [0] and lab.tolist() == [5] and dist.tolist() == [0.0]


@pytest.mark.parametrize("theta", [0.0, 1e-6, 0.3, 1.2])
def test_angle_closed_form(theta):
    V = np.array([[1.0], [0.0]])
    W = np.array([[np.cos(theta)], [np.sin(theta)]])
    assert abs(O.sin_angle(V, W) - abs(np.sin(theta))) <= 1e-16
    assert abs(nn.cos_angle(V, W) - abs(np.cos(theta))) <= 1e-16
    # unit samples e1 and e2: d^V = 1, d^W = |cos - sin|
    x, y = np.array([[1.0], [0.0]]), np.array([[0.0], [1.0]])
    dV = nn.nn_distances(V, x, y)[0, 0]
    dW = nn.nn_distances(W, x, y)[0, 0]
    assert abs(dV - 1.0) <= 1e-16 and abs(dW - abs(np.cos(theta) - np.sin(theta))) <= 1e-15
    lo, hi = nn.thm37_bounds(dW, abs(np.sin(theta)), abs(np.cos(theta)))
    assert lo <= dV + 1e-15 and dV <= hi + 1e-15


@pytest.mark.parametrize("eps", [1e-8, 1e-4, 1e-2, 0.3])
def test_thm37_bounds_hold_on_perturbed_subspaces(eps):
    rng = np.random.default_rng(int(-np.log10(eps)) + 11)
    d, t = 60, 5
    V = np.linalg.qr(rng.standard_normal((d, t)))[0]
    W = np.linalg.qr(V + eps * rng.standard_normal((d, t)))[0]
    X = rng.standard_normal((d, 12))
    Y = rng.standard_normal((d, 9))
    X /= np.linalg.norm(X, axis=0)
    Y /= np.linalg.norm(Y, axis=0)
    dV = nn.nn_distances(V, X, Y)
    dW = nn.nn_distances(W, X, Y)
    s, c = O.sin_angle(V, W), nn.cos_angle(V, W)
    # principal angles: sin is that of the largest, ||V^T W||_2 the cosine of
    # the smallest (singular values of V^T W)
    sv = np.linalg.svd(V.T @ W, compute_uv=False)
    assert abs(c - sv[0]) <= 1e-14 and abs(s * s + sv[-1] ** 2 - 1.0) <= 1e-12
    lo, hi = nn.thm37_bounds(dW, s, c)
    assert np.all(lo <= dV + 1e-12) and np.all(dV <= hi + 1e-12)
    # the symmetric statement with the roles exchanged
    lo2, hi2 = nn.thm37_bounds(dV, s, c)
    assert np.all(lo2 <= dW + 1e-12) and np.all(dW <= hi2 + 1e-12)


def test_split_shares_the_training_samples_and_classes():
    p = datagen.config("C1", with_data=False)
    Xtr, Xte, lte = datagen.make_split(p.d, p.counts, np.full(p.k, 3), p.r, p.seed)
    np.testing.assert_array_equal(Xtr, datagen.make_samples(p.d, p.counts, p.r, p.seed))
    assert Xte.shape == (p.d, 3 * p.k) and lte.tolist() == np.repeat(np.arange(p.k), 3).tolist()
    np.testing.assert_allclose(np.linalg.norm(Xte, axis=0), 1.0, atol=1e-14)
    # in the EDA subspace of the training set the testing samples of this
    # well-separated model fall next to their own class
    H_W, H_B = O.scatter_factors(Xtr, p.counts)
    V = O.eda_reduced(H_W, H_B, p.t).X
    lab, _, _ = nn.nn_classify(V, Xtr, p.labels(), Xte)
    assert np.mean(lab == lte) >= 0.9
