"""Pins of the oracle's exact closest-point rules against brute-force sampling of each
surface and against the first-order optimality (KKT) conditions."""

import numpy as np
import pytest

from oracle import sbm_oracle as O
from paper_2507_17053_amd import inputs


def _fib_sphere(n):
    i = np.arange(n) + 0.5
    z = 1 - 2 * i / n
    r = np.sqrt(1 - z * z)
    th = np.pi * (1 + 5 ** 0.5) * i
    return np.stack([r * np.cos(th), r * np.sin(th), z], axis=1)


def _surface_samples(ls, d, n=400000):
    k = ls["kind"]
    if k == "sphere":
        c = np.asarray(ls["centre"])[:d]
        if d == 2:
            t = np.linspace(0, 2 * np.pi, n, endpoint=False)
            return c + ls["radius"] * np.stack([np.cos(t), np.sin(t)], 1)
        return c + ls["radius"] * _fib_sphere(n)
    if k == "ellipsoid":
        c = np.asarray(ls["centre"])[:d]
        a = np.asarray(ls["semi_axes"])[:d]
        if d == 2:
            t = np.linspace(0, 2 * np.pi, n, endpoint=False)
            return c + a * np.stack([np.cos(t), np.sin(t)], 1)
        return c + a * _fib_sphere(n)
    if k == "torus":
        m = int(np.sqrt(n))
        u, v = np.meshgrid(np.linspace(0, 2 * np.pi, m, endpoint=False),
                           np.linspace(0, 2 * np.pi, m, endpoint=False))
        u, v = u.ravel(), v.ravel()
        R, r = ls["R"], ls["r"]
        return np.asarray(ls["centre"]) + np.stack([(R + r * np.cos(v)) * np.cos(u),
                                                    (R + r * np.cos(v)) * np.sin(u), r * np.sin(v)], 1)
    if k == "sphere_union":
        cs, rs = np.asarray(ls["centres"])[:, :d], np.asarray(ls["radii"])
        pts = []
        for c, r in zip(cs, rs):
            s = _surface_samples({"kind": "sphere", "centre": c, "radius": r}, d, n // len(rs))
            keep = np.ones(len(s), bool)
            for c2, r2 in zip(cs, rs):
                keep &= np.linalg.norm(s - c2, axis=1) >= r2 * (1 - 1e-12) if not np.all(c2 == c) else keep
            pts.append(s[keep])
        return np.concatenate(pts)
    raise KeyError(k)


CASES = [
    (2, inputs.sphere((0.05, -0.03), 0.7)),
    (2, inputs.ellipsoid((0.02, 0.01), (0.8, 0.45))),
    (2, {"kind": "sphere_union", "centres": np.array([[-0.3, 0.0], [0.35, 0.1], [0.0, 0.4]]),
         "radii": np.array([0.5, 0.45, 0.3])}),
    (3, inputs.sphere((0.0, 0.0, 0.0), 0.75)),
    (3, inputs.ellipsoid((0.0, 0.0, 0.0), (0.8, 0.5, 0.65))),
    (3, inputs.torus(0.6, 0.25)),
    (3, inputs.sphere_union(1)),
]


@pytest.mark.parametrize("d,ls", CASES)
def test_closest_point_is_on_surface_and_nearest(d, ls):
    rng = np.random.default_rng(5)
    # query points near the surface, as surrogate-face points are (inside and outside)
    samp = _surface_samples(ls, d)
    q = samp[rng.integers(0, len(samp), 40)] + rng.normal(0, 0.06, (40, d))
    cp = O.closest_point(ls, q)
    # on the surface
    assert np.abs(O.phi(ls, cp)).max() < 1e-12
    dist = np.linalg.norm(cp - q, axis=1)
    # nearest: no surface sample is closer than the computed point (up to the sampling gap)
    gap = 0.02 if d == 3 else 1e-4
    for i in range(len(q)):
        ds = np.linalg.norm(samp - q[i], axis=1).min()
        assert dist[i] <= ds + 1e-12, (i, dist[i], ds)
        assert dist[i] >= ds - gap, (i, dist[i], ds)


@pytest.mark.parametrize("d,ls", [c for c in CASES if c[1]["kind"] in ("ellipsoid", "torus", "sphere")])
def test_closest_point_kkt(d, ls):
    """x - x~ is parallel to grad phi(x) at the closest point (first-order optimality)."""
    rng = np.random.default_rng(6)
    samp = _surface_samples(ls, d, 20000)
    q = samp[rng.integers(0, len(samp), 50)] + rng.normal(0, 0.05, (50, d))
    cp = O.closest_point(ls, q)
    eps = 1e-6
    g = np.zeros_like(cp)
    for k in range(d):
        e = np.zeros(d)
        e[k] = eps
        g[:, k] = (O.phi(ls, cp + e) - O.phi(ls, cp - e)) / (2 * eps)
    r = cp - q
    if d == 2:
        cross = r[:, 0] * g[:, 1] - r[:, 1] * g[:, 0]
    else:
        cross = np.linalg.norm(np.cross(r, g), axis=1)
    assert np.all(np.abs(cross) <= 1e-7 * np.linalg.norm(r, axis=1) * np.linalg.norm(g, axis=1) + 1e-12)


def test_halfspace_shift_is_normal_offset():
    ls = inputs.halfspace((1.0, 0.0, 0.0), 0.3)
    x = np.array([[0.0, 0.1, 0.2], [-0.5, 0.3, -0.7]])
    cp = O.closest_point(ls, x)
    np.testing.assert_allclose(cp, [[0.3, 0.1, 0.2], [0.3, 0.3, -0.7]], atol=1e-15)


def test_active_cells_lie_inside_convex_domain():
    """For a convex domain the vertex test is exact: every point of an active cell is inside."""
    ls = inputs.ellipsoid((0.0, 0.0, 0.0), (0.8, 0.5, 0.65))
    prob = O.setup(3, 12, -1.0, 1.0, ls, 1)
    g = np.linspace(0, 1, 5)
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    for c in prob.cells:
        x = prob.lo + prob.h * (c + pts)
        assert np.all(O.phi(ls, x) < 1e-15)


def test_callback_newton_projection_is_exact_for_radial_level_sets():
    """The level-set Newton projection (callback kind) moves along grad phi; for a sphere given
    as |x - c| - r or |x - c|^2 - r^2, and a torus given by its distance, the gradient lines
    are straight, so it must land on the exact closest point."""
    rng = np.random.default_rng(5)
    c = np.array([0.1, -0.2, 0.05])
    X = rng.uniform(-1, 1, (200, 3))
    exact = O.closest_point({"kind": "sphere", "centre": list(c), "radius": 0.6}, X)
    for phi, grad in [(lambda Y: np.linalg.norm(Y - c, axis=1) - 0.6,
                       lambda Y: (Y - c) / np.linalg.norm(Y - c, axis=1)[:, None]),
                      (lambda Y: np.sum((Y - c) ** 2, axis=1) - 0.36, lambda Y: 2.0 * (Y - c))]:
        got = O.closest_point(inputs.callback(phi, grad, 3), X)
        assert np.abs(got - exact).max() <= 1e-12

    def tphi(Y):
        rho = np.sqrt(Y[:, 0] ** 2 + Y[:, 1] ** 2)
        return np.sqrt((rho - 0.6) ** 2 + Y[:, 2] ** 2) - 0.25

    def tgrad(Y):
        rho = np.sqrt(Y[:, 0] ** 2 + Y[:, 1] ** 2)
        q = np.sqrt((rho - 0.6) ** 2 + Y[:, 2] ** 2)
        f = (rho - 0.6) / (rho * q)
        return np.stack([f * Y[:, 0], f * Y[:, 1], Y[:, 2] / q], axis=1)

    Xt = X[np.sqrt(X[:, 0] ** 2 + X[:, 1] ** 2) > 0.05]
    exact_t = O.closest_point(inputs.torus(0.6, 0.25), Xt)
    got_t = O.closest_point(inputs.callback(tphi, tgrad, 3), Xt)
    assert np.abs(got_t - exact_t).max() <= 1e-12


def test_callback_newton_projection_lands_on_the_boundary_or_fails():
    """Implicit ellipse: every projected point lies on the boundary to rounding (first-order
    distance |phi| / |grad phi| <= 1e-14); a level set without zeros (phi = |x|^2 + 1) makes the
    projection raise."""
    a = np.array([0.8, 0.45])
    ls = inputs.callback(lambda Y: np.sum((Y / a) ** 2, axis=1) - 1.0, lambda Y: 2.0 * Y / a ** 2, 2)
    X = np.random.default_rng(6).uniform(-1, 1, (100, 2))
    got = O.closest_point(ls, X)
    assert np.max(np.abs(ls["phi"](got)) / np.linalg.norm(ls["grad"](got), axis=1)) <= 1e-14
    none = inputs.callback(lambda Y: np.sum(Y ** 2, axis=1) + 1.0, lambda Y: 2.0 * Y, 2)
    with pytest.raises(ValueError):
        O.closest_point(none, X[:3])


@pytest.mark.parametrize("case", ["scaled-distance", "squared-r10", "squared-c50-r30"])
def test_callback_newton_projection_is_scale_aware(case):
    """The Newton stop is relative to the point and the gradient, so level sets that are
    scaled, or whose values are large near the boundary, project as accurately as a distance
    function: 100 (|x - c| - r), |x|^2 - 10^2 and |x - (50, 50)|^2 - 30^2 all land on the exact
    closest point of their circle (an absolute |phi| stop fails on many of these points)."""
    rng = np.random.default_rng(11)
    if case == "scaled-distance":
        c, r = np.array([0.05, -0.03]), 0.75
        phi = lambda Y: 100.0 * (np.linalg.norm(Y - c, axis=1) - r)
        grad = lambda Y: 100.0 * (Y - c) / np.linalg.norm(Y - c, axis=1)[:, None]
        X = rng.uniform(-1, 1, (300, 2))
    elif case == "squared-r10":
        c, r = np.array([0.0, 0.0]), 10.0
        phi = lambda Y: np.sum((Y - c) ** 2, axis=1) - r * r
        grad = lambda Y: 2.0 * (Y - c)
        X = rng.uniform(-12, 12, (300, 2))
    else:
        c, r = np.array([50.0, 50.0]), 30.0
        phi = lambda Y: np.sum((Y - c) ** 2, axis=1) - r * r
        grad = lambda Y: 2.0 * (Y - c)
        X = rng.uniform(15, 85, (300, 2))
    exact = O.closest_point({"kind": "sphere", "centre": list(c), "radius": r}, X)
    got = O.closest_point(inputs.callback(phi, grad, 2), X)
    assert np.abs(got - exact).max() <= 1e-12 * max(1.0, np.abs(c).max() + r)
