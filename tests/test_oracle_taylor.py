"""Pins of the oracle's truncated extension E_m (the Taylor expansion of Sec. 2.1 kept to total
order m) against what the mathematics fixes, each through a route that does not use the
Taylor code itself:

* the Taylor series of a polynomial terminates: m >= d p gives the point value at the
  shifted point (basis_values), i.e. the full extension;
* m = 0 keeps only u(x~): the operator of the unshifted problem (shift_scale = 0);
* m = 1 is value plus gradient, u(x~) + delta . grad u(x~), with the gradient from the
  product-rule derivative (lagrange_derivatives), not from polynomial coefficients;
* E_m reproduces every polynomial of total degree <= m: applied to the interpolant of such a
  polynomial the SBM face term equals that of the full extension;
* and E_m differs from the full extension for a polynomial of total degree m + 1."""

import numpy as np
import pytest

from oracle import sbm_oracle as O
from paper_2507_17053_amd import inputs

DISK = inputs.sphere((0.05, -0.03), 0.7)
BALL = inputs.sphere((0, 0, 0), 0.75)


def _sbm(prob):
    return O.assemble(prob, parts=("sbm",))


def _rel(a, b):
    return np.linalg.norm((a - b).toarray() if hasattr(a, "toarray") else a - b) / max(
        np.linalg.norm(b.toarray() if hasattr(b, "toarray") else b), 1e-300)


@pytest.mark.parametrize("d,n,ls,p,disc", [(2, 8, DISK, 3, "cg"), (2, 6, DISK, 2, "dg"), (3, 8, BALL, 2, "cg")])
def test_full_order_equals_point_evaluation(d, n, ls, p, disc):
    full = O.setup(d, n, -1.0, 1.0, ls, p, disc=disc)
    trunc = O.setup(d, n, -1.0, 1.0, ls, p, disc=disc, taylor_order=d * p)
    assert _rel(_sbm(trunc), _sbm(full)) <= 1e-12
    # one order less is a different operator (the top mixed term is dropped)
    lower = O.setup(d, n, -1.0, 1.0, ls, p, disc=disc, taylor_order=d * p - 1)
    assert _rel(_sbm(lower), _sbm(full)) > 1e-10


@pytest.mark.parametrize("d,n,ls,p,disc", [(2, 8, DISK, 2, "cg"), (3, 8, BALL, 2, "dg")])
def test_order_zero_is_the_unshifted_operator(d, n, ls, p, disc):
    m0 = O.setup(d, n, -1.0, 1.0, ls, p, disc=disc, taylor_order=0)
    unshifted = O.setup(d, n, -1.0, 1.0, ls, p, disc=disc, shift_scale=0.0)
    assert _rel(_sbm(m0), _sbm(unshifted)) <= 1e-13


@pytest.mark.parametrize("d,p", [(2, 2), (2, 4), (3, 3)])
def test_order_one_is_value_plus_gradient(d, p):
    rng = np.random.default_rng(11)
    nodes = O.gll_nodes(p)
    xi0 = rng.uniform(0, 1, (7, d))
    xi = xi0 + rng.uniform(-0.6, 0.6, (7, d))
    got = O.basis_taylor_values(nodes, xi0, xi, 1)
    grad = O.basis_gradients(nodes, xi0)  # (nq, nb, d), product-rule derivatives
    want = O.basis_values(nodes, xi0) + np.einsum("qik,qk->qi", grad, xi - xi0)
    assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))


def _total_degree_poly(d, deg, seed):
    rng = np.random.default_rng(seed)
    exps = [e for e in np.ndindex(*([deg + 1] * d)) if sum(e) <= deg]
    coef = rng.uniform(-1, 1, len(exps))

    def u(x):
        out = np.zeros(x.shape[0])
        for c, e in zip(coef, exps):
            t = np.full(x.shape[0], c)
            for k in range(d):
                t = t * x[:, k] ** e[k]
            out += t
        return out

    return u


@pytest.mark.parametrize("d,n,ls,p,disc,m", [(2, 8, DISK, 3, "cg", 1), (2, 8, DISK, 3, "cg", 2),
                                             (2, 6, DISK, 4, "dg", 3), (3, 8, BALL, 2, "cg", 2)])
def test_reproduces_total_degree_m(d, n, ls, p, disc, m):
    full = O.setup(d, n, -1.0, 1.0, ls, p, disc=disc)
    trunc = O.setup(d, n, -1.0, 1.0, ls, p, disc=disc, taylor_order=m)
    Bf, Bt = _sbm(full), _sbm(trunc)
    u = O.interpolate(full, _total_degree_poly(d, m, 3 + m))
    assert np.linalg.norm(Bt @ u - Bf @ u) <= 1e-11 * np.linalg.norm(Bf @ u)
    # a polynomial of total degree m + 1 (within Q_p) is not reproduced
    if m + 1 <= p:
        w = O.interpolate(full, _total_degree_poly(d, m + 1, 5 + m))
        assert np.linalg.norm(Bt @ w - Bf @ w) > 1e-8 * np.linalg.norm(Bf @ w)


def test_taylor_terms_of_one_basis_function_by_hand():
    """p = 1 on GLL nodes {0, 1}: l_0(x) = 1 - x, l_1(x) = x, so the terms about x0 are
    (1 - x0, -dlt) and (x0, dlt), and every higher order is zero."""
    nodes = O.gll_nodes(1)
    t = O.lagrange_taylor_terms(nodes, np.array([0.3]), np.array([-0.8]), 3)[0]
    np.testing.assert_allclose(t[0], [0.7, 0.3], atol=1e-15)
    np.testing.assert_allclose(t[1], [0.8, -0.8], atol=1e-15)
    np.testing.assert_allclose(t[2:], 0.0, atol=1e-15)


def test_negative_order_rejected():
    with pytest.raises(ValueError):
        O.setup(2, 4, -1.0, 1.0, DISK, 1, taylor_order=-1)


@pytest.mark.parametrize("p", [4, 8])
def test_taylor_terms_against_exact_rational_arithmetic(p):
    """The terms from float inputs (GLL nodes, x0, dlt as stored) against the same terms
    computed exactly with fractions: multiply out prod_{l != j} (x0 - z_l + t dlt) and divide
    by prod_{l != j} (z_j - z_l).  Relative to the largest term, within 1e-14."""
    from fractions import Fraction as Fr
    nodes = O.gll_nodes(p)
    rng = np.random.default_rng(p)
    for _ in range(6):
        x0, dlt = float(rng.uniform(0, 1)), float(rng.uniform(-1.2, 1.2))
        got = O.lagrange_taylor_terms(nodes, np.array([x0]), np.array([dlt]), p)[0]
        for j in range(p + 1):
            others = [Fr(z) for k, z in enumerate(nodes) if k != j]
            den = Fr(1)
            for z in others:
                den *= Fr(nodes[j]) - z
            poly = [Fr(1)]
            for z in others:
                a = Fr(x0) - z
                nxt = [Fr(0)] * (len(poly) + 1)
                for k, c in enumerate(poly):
                    nxt[k] += a * c
                    nxt[k + 1] += Fr(dlt) * c
                poly = nxt
            exact = np.array([float(c / den) for c in poly])
            assert np.max(np.abs(got[:, j] - exact)) <= 1e-14 * np.max(np.abs(exact))
