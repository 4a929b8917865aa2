"""Pins of the oracle's bases and quadrature against textbook facts (CPU only)."""
import math

import numpy as np
import pytest

from oracle.basis import bernstein, gauss_legendre, gll_points, lagrange, tensor_tables


def test_gll_points_closed_forms():
    # GLL points on [-1,1]: k=2: 0; k=3: +-1/sqrt(5); k=4: 0, +-sqrt(3/7)
    assert np.allclose(gll_points(1), [0, 1])
    assert np.allclose(gll_points(2), [0, 0.5, 1], atol=1e-15)
    s5 = 1 / math.sqrt(5)
    assert np.allclose(gll_points(3), [0, (1 - s5) / 2, (1 + s5) / 2, 1], atol=1e-15)
    s = math.sqrt(3 / 7)
    assert np.allclose(gll_points(4), [0, (1 - s) / 2, 0.5, (1 + s) / 2, 1], atol=1e-15)


@pytest.mark.parametrize("n", range(1, 9))
def test_gauss_exactness(n):
    x, w = gauss_legendre(n)
    assert abs(w.sum() - 1) < 1e-15
    for p in range(2 * n):
        assert abs(np.dot(w, x ** p) - 1.0 / (p + 1)) < 1e-14
    # degree 2n is NOT integrated exactly
    assert abs(np.dot(w, x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_lagrange_nodal_and_derivative(k):
    nodes = gll_points(k)
    V, D = lagrange(nodes, nodes)
    assert np.allclose(V, np.eye(k + 1), atol=1e-14)
    t = np.linspace(0.03, 0.97, 11)
    V, D = lagrange(nodes, t)
    # interpolation reproduces polynomials of degree <= k and their derivatives
    for p in range(k + 1):
        assert np.allclose(V @ nodes ** p, t ** p, atol=1e-13)
        dp = p * t ** (p - 1) if p > 0 else 0 * t
        assert np.allclose(D @ nodes ** p, dp, atol=1e-12)
    # derivative against central differences of the values
    h = 1e-6
    Vp, _ = lagrange(nodes, t + h)
    Vm, _ = lagrange(nodes, t - h)
    assert np.allclose((Vp - Vm) / (2 * h), D, atol=1e-8)


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_bernstein_partition_positive_integral(deg):
    t = np.linspace(0, 1, 17)
    B = bernstein(deg, t)
    assert np.allclose(B.sum(1), 1.0, atol=1e-15)
    assert (B >= 0).all()
    x, w = gauss_legendre(deg + 1)
    # each Bernstein polynomial of degree n integrates to 1/(n+1)
    assert np.allclose(w @ bernstein(deg, x), 1.0 / (deg + 1), atol=1e-15)


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3)])
def test_tensor_tables_partition_of_unity(dim, k):
    T = tensor_tables(dim, k)
    assert T["W"].shape == ((2 * k) ** dim, (k + 1) ** dim)
    assert np.allclose(T["W"].sum(1), 1, atol=1e-14)
    assert np.allclose(T["dW"].sum(1), 0, atol=1e-13)
    assert np.allclose(T["Phi"].sum(1), 1, atol=1e-14)
    assert abs(T["qw"].sum() - 1) < 1e-14
    # the H1 tables reproduce the reference coordinates and their gradient (identity)
    ih = T["ih"]
    xi_nodes = np.stack([T["gll"][ih[a]] for a in range(dim)])  # (dim, Nh)
    assert np.allclose(T["W"] @ xi_nodes.T, T["qpts"], atol=1e-14)
    grad = np.einsum("an,qnb->qab", xi_nodes, T["dW"])
    assert np.allclose(grad, np.broadcast_to(np.eye(dim), grad.shape), atol=1e-13)
