"""Pins of the oracle's 1D rules, basis and cell matrix against facts fixed outside it:
numpy's Gauss-Legendre routine, polynomial identities and textbook element matrices."""

import json
import os

import numpy as np
import pytest

from oracle import sbm_oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_rule_matches_numpy_leggauss(n):
    g, w = O.gauss_rule(n)
    x, ww = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(g, (x + 1) / 2, atol=2e-16 * 4)
    np.testing.assert_allclose(w, ww / 2, rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", range(2, 9))
def test_gll_nodes_are_roots_of_legendre_derivative(p):
    z = O.gll_nodes(p)
    r = np.sort(np.polynomial.legendre.Legendre.basis(p).deriv().roots().real)
    assert z[0] == 0.0 and z[-1] == 1.0
    np.testing.assert_allclose(z[1:-1], (r + 1) / 2, atol=1e-14)
    # symmetry of the node set about 1/2
    np.testing.assert_allclose(z + z[::-1], np.ones_like(z), atol=1e-15)


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_reproduces_polynomials_when_extrapolating(p):
    """sum_j l_j(x) = 1 and sum_j z_j^m l_j(x) = x^m for m <= p, for x in [-1.4, 2.4]."""
    z = O.gll_nodes(p)
    x = np.linspace(-1.4, 2.4, 97)
    L = O.lagrange_values(z, x)
    growth = np.abs(L).sum(axis=1)  # Lebesgue function: rounding amplification at x
    for m in range(p + 1):
        ref = x ** m
        err = np.abs(L @ (z ** m) - ref)
        assert np.all(err <= 64 * np.finfo(float).eps * growth * np.maximum(1.0, np.abs(ref)))
    # derivative reproduces m x^(m-1)
    D = O.lagrange_derivatives(z, x)
    dgrowth = np.abs(D).sum(axis=1)
    for m in range(1, p + 1):
        ref = m * x ** (m - 1)
        err = np.abs(D @ (z ** m) - ref)
        assert np.all(err <= 64 * np.finfo(float).eps * dgrowth * np.maximum(1.0, np.abs(ref)))
    # cardinality at the nodes
    np.testing.assert_allclose(O.lagrange_values(z, z), np.eye(p + 1), atol=1e-14)


def _kron_sum(K, M, d):
    if d == 2:
        return np.kron(M, K) + np.kron(K, M)
    return np.kron(M, np.kron(M, K)) + np.kron(M, np.kron(K, M)) + np.kron(K, np.kron(M, M))


def _textbook(p):
    with open(os.path.join(GOLD, "textbook_1d_matrices.json")) as fh:
        t = json.load(fh)
    if p == 1:
        return np.array(t["p1"]["K_hat"], float), np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
    e = t["p2"]
    return np.array(e["K_num"], float) / e["K_den"], np.array(e["M_num"], float) / e["M_den"]


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("h", [1.0, 0.125])
def test_cell_matrix_is_kronecker_sum_of_textbook_matrices(d, p, h):
    """The brute-force quadrature cell matrix equals h^(d-2) sum_k M x .. K_k .. x M built
    from textbook 1D matrices (Gauss with p+1 points integrates degree 2p exactly)."""
    K, M = _textbook(p)
    ls = {"kind": "sphere", "centre": [0.0] * d, "radius": 10.0}
    prob = O.setup(d, 2, 0.0, 2 * h, ls, p)
    A = O.cell_matrix(prob)
    ref = _kron_sum(K, M, d) * h ** (d - 2)
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_q1_laplace_textbook_2d():
    with open(os.path.join(GOLD, "textbook_1d_matrices.json")) as fh:
        t = json.load(fh)["q1_2d_laplace"]
    ref = np.array(t["num"], float) / t["den"]
    ls = {"kind": "sphere", "centre": [0.0, 0.0], "radius": 10.0}
    prob = O.setup(2, 1, 0.0, 0.37, ls, 1)
    np.testing.assert_allclose(O.cell_matrix(prob), ref, atol=1e-15)


@pytest.mark.parametrize("d,p", [(2, 1), (2, 4), (3, 2), (3, 4), (3, 6)])
def test_cell_matrix_annihilates_constants_and_is_spsd(d, p):
    ls = {"kind": "sphere", "centre": [0.0] * d, "radius": 10.0}
    prob = O.setup(d, 2, -1.0, 1.0, ls, p)
    A = O.cell_matrix(prob)
    assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-12 * np.abs(A).max()
    np.testing.assert_allclose(A, A.T, atol=1e-14 * np.abs(A).max())
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > -1e-12 * ev.max()
    # exactly one zero eigenvalue (the constants)
    assert np.sum(ev < 1e-10 * ev.max()) == 1


def test_basis_lexicographic_numbering():
    """Local index i = i1 + (p+1) i2 (+ (p+1)^2 i3): psi_i is 1 at node (z_i1, z_i2, z_i3)."""
    p = 3
    z = O.gll_nodes(p)
    mi = O.local_multi_indices(3, p)
    assert tuple(mi[1]) == (1, 0, 0) and tuple(mi[p + 1]) == (0, 1, 0) and tuple(mi[(p + 1) ** 2]) == (0, 0, 1)
    V = O.basis_values(z, z[mi])
    np.testing.assert_allclose(V, np.eye(V.shape[0]), atol=1e-13)
