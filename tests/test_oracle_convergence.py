"""Convergence pin (App. A): on the disk workload's geometry with u* = sin(pi x) cos(pi y),
the SBM solution converges in L2 at about O(h^(p+1)); without the shift (E = identity)
the surrogate-boundary error caps the rate near 2.  A dropped or mis-signed term in the
operator or the right-hand side breaks one of these."""

import numpy as np
import pytest

from oracle import sbm_oracle as O
from paper_2507_17053_amd import inputs


def _errors(p, Ns, shift=1.0, disc="cg"):
    w = inputs.workload("disk2d_q2")
    u, f = inputs.manufactured(2)
    out = []
    for N in Ns:
        prob = O.setup(2, N, w["lo"], w["hi"], w["levelset"], p, disc=disc, shift_scale=shift)
        A = O.assemble(prob)
        x = O.solve_direct(A, O.rhs(prob, f, u))
        out.append(O.l2_error(prob, x, u))
    return np.array(out)


@pytest.mark.parametrize("p,min_rate", [(1, 1.75), (2, 2.4), (3, 3.2)])
def test_l2_rate_near_optimal(p, min_rate):
    Ns = [16, 32, 64]
    e = _errors(p, Ns)
    assert np.all(np.diff(e) < 0)
    rate = np.log2(e[0] / e[-1]) / (len(Ns) - 1)
    assert rate >= min_rate, (e, rate)


def test_dg_converges_like_cg():
    e = _errors(2, [16, 32, 64], disc="dg")
    rate = np.log2(e[0] / e[-1]) / 2
    assert rate >= 2.4, (e, rate)


def test_unshifted_rate_is_lower():
    """p = 2 without the shift stays near second order; with the shift it is clearly above."""
    e0 = _errors(2, [16, 32, 64], shift=0.0)
    e1 = _errors(2, [16, 32, 64], shift=1.0)
    r0 = np.log2(e0[0] / e0[-1]) / 2
    r1 = np.log2(e1[0] / e1[-1]) / 2
    assert r0 < 2.3 and r1 > r0 + 0.3, (r0, r1)
