"""FP64 CPU oracle for the shifted-boundary (SBM) Poisson operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link this
module: only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
It shares no code, tables or constants with the HIP library; the two meet only through
seeded inputs (vectors, geometry parameters) generated outside both.

What it computes is the plain definition of the operator of the paper
(Wichrowski, "Matrix-Free Evaluation of High-Order Shifted Boundary Finite Element
Operators"):

* the SBM weak form of Sec. 2.1, Eq. (1): for all v_h,
      a(u,v) = int_{Om~} grad u . grad v
               - int_{Gam~} (grad u . n~) v
               - int_{Gam~} (grad v . n~) E u
               + int_{Gam~} sigma_Gam  E u  v ,
  with the extension E u(x~) taken as the value of the cell polynomial at the
  closest-point image x = x~ + d on the true boundary (Sec. 3.3, Alg. 3);
* the SIPG replacement of the Laplace term for the DG variant (Sec. 2.1, last display;
  Sec. 3.2), with jump [u] = u_K1 - u_K2 and average {du/dn} = (du_K1/dn + du_K2/dn)/2,
  n pointing from K1 to K2;
* tensor-product Lagrange bases with lexicographic local numbering (Sec. 3.1) and
  (p+1)^d Gauss points per cell, (p+1)^(d-1) per face (Sec. 3.1, Sec. 3.3).

Every local matrix is formed by brute-force quadrature, one quadrature point at a
time, with no sum factorisation; the global matrix is the plain sum of the local blocks.
The matrix-free apply must reproduce A @ u up to rounding (the paper validates its
matrix-free products against assembled sparse matrices, Sec. 4 introduction).

Readings of points where the paper is silent or ambiguous (recorded in the design
notes as well):
  R1 E u(x~_q) is the point value u_K(xi_q) of the face's own active cell K, evaluated
     at the reference coordinates xi_q = xi~_q + d_q / h, which lie outside [0,1]^d.
  R2 Active cells: phi < 0 strictly at all 2^d vertices (cells "lying entirely within"
     the domain, Sec. 2).  Surrogate faces: faces of active cells whose neighbour is
     missing or inactive.
  R3 Penalties sigma_Gam = gamma p^2 / h, sigma_F = gamma_F p^2 / h (the paper only says
     "sufficiently large", Sec. 2 and Sec. 3.2).
  R4 Normal derivative and face measure are taken on the surrogate face (Alg. 3).
  R5 Nodes: Gauss-Lobatto-Legendre (GLL) Lagrange basis for CG and DG.
  R6 Global CG numbering: lattice index m = p*c + j; ids are the ranks of touched
     lattice points in lexicographic order, first coordinate fastest.  DG: rank of the
     active cell times (p+1)^d plus the local index.
  R7 Closest points are exact (sphere, torus, ellipsoid, half-space, sphere union);
     see closest_point().
  R8 The truncated extension E_m (the Taylor expansion of Sec. 2.1 kept to total order
     m) expands the same cell polynomial about the surrogate point:
         E_m u(x~) = sum_{|alpha| <= m} D^alpha u_K(x~) d^alpha / alpha!,
     in reference coordinates (D_x^alpha d^alpha = D_xi^alpha delta^alpha with
     delta = xi - xi~).  m = 1 is "values and gradients"; m >= d p is the full
     extension of R1, since u_K has degree at most p in each coordinate.

Parity pins: see tests/test_oracle_*.py.  Functions without an independent pin are
marked "parity unpinned" in their docstrings (none at present).
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

# ----------------------------------------------------------------------------------------
# 1D rules on the reference interval [0, 1]   (Sec. 3.1)
# ----------------------------------------------------------------------------------------


def _legendre(n: int, x: np.ndarray):
    """Legendre polynomial P_n and its derivative on [-1,1] by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    # derivative from n (x P_n - P_{n-1}) / (x^2 - 1); only used away from +-1
    dp = n * (x * p1 - p0) / (x * x - 1.0)
    return p1, dp


def gauss_rule(n: int):
    """n-point Gauss-Legendre rule mapped to [0,1]: (nodes ascending, weights summing to 1).

    Nodes are the roots of P_n found by Newton's method from Chebyshev-type guesses."""
    if n == 1:
        return np.array([0.5]), np.array([1.0])
    i = np.arange(n)
    x = -np.cos(np.pi * (i + 0.75) / (n + 0.5))
    for _ in range(100):
        pn, dpn = _legendre(n, x)
        dx = pn / dpn
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    _, dpn = _legendre(n, x)
    w = 2.0 / ((1.0 - x * x) * dpn * dpn)
    order = np.argsort(x)
    return (x[order] + 1.0) / 2.0, w[order] / 2.0


def gll_nodes(p: int) -> np.ndarray:
    """p+1 Gauss-Lobatto-Legendre nodes on [0,1]: 0, 1 and the roots of P'_p (reading R5)."""
    if p == 1:
        return np.array([0.0, 1.0])
    i = np.arange(1, p)
    x = -np.cos(np.pi * i / p)  # Chebyshev-Gauss-Lobatto guesses, ascending
    for _ in range(100):
        pn, dpn = _legendre(p, x)
        # P''_p from Legendre's equation (1-x^2) P'' - 2x P' + p(p+1) P = 0
        d2 = (2.0 * x * dpn - p * (p + 1) * pn) / (1.0 - x * x)
        dx = dpn / d2
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    nodes = np.concatenate([[-1.0], np.sort(x), [1.0]])
    return (nodes + 1.0) / 2.0


def lagrange_values(nodes: np.ndarray, x) -> np.ndarray:
    """l_j(x) for all nodes j, in product form (stable for x outside [0,1]).  Shape x.shape+(n,)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(nodes)
    out = np.ones(x.shape + (n,))
    for j in range(n):
        for m in range(n):
            if m != j:
                out[..., j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return out


def lagrange_taylor_terms(nodes: np.ndarray, x0, dlt, m: int) -> np.ndarray:
    """Terms l_j^(k)(x0) dlt^k / k! of the Taylor expansion of each 1D Lagrange polynomial
    about x0, for k = 0..m (k > p gives zero).  l_j re-expanded about x0 is
    l_j(x0 + t) = prod_{l != j} (t - (z_l - x0)) / prod_{l != j} (z_j - z_l), whose monomial
    coefficients (numpy's polyfromroots of the shifted roots) are l_j^(k)(x0) / k!.  (Forming
    the coefficients about 0 and differentiating loses about 1e-11 relative at p = 8.)
    x0, dlt: arrays of one shape; result shape x0.shape + (m + 1, n)."""
    P = np.polynomial.polynomial
    x0 = np.asarray(x0, dtype=np.float64)
    dlt = np.asarray(dlt, dtype=np.float64)
    n = len(nodes)
    out = np.zeros(x0.shape + (m + 1, n))
    kmax = min(m, n - 1)
    for idx in np.ndindex(x0.shape):
        for j in range(n):
            others = np.delete(nodes, j)
            c = P.polyfromroots(others - x0[idx]) / np.prod(nodes[j] - others)
            for k in range(kmax + 1):
                out[idx + (k, j)] = c[k] * dlt[idx] ** k
    return out


def basis_taylor_values(nodes: np.ndarray, xi0: np.ndarray, xi: np.ndarray, m: int) -> np.ndarray:
    """E_m psi_i at each point (reading R8): sum over multi-indices alpha with |alpha| <= m
    of prod_k l_{i_k}^(alpha_k)(xi0_k) (xi_k - xi0_k)^alpha_k / alpha_k!.
    xi0, xi: (nq, d); result (nq, n1^d), the truncated counterpart of basis_values(xi)."""
    xi0 = np.atleast_2d(xi0)
    xi = np.atleast_2d(xi)
    d = xi.shape[1]
    p = len(nodes) - 1
    mi = local_multi_indices(d, p)
    km = min(m, p)
    terms = [lagrange_taylor_terms(nodes, xi0[:, k], xi[:, k] - xi0[:, k], km) for k in range(d)]
    out = np.zeros((xi.shape[0], mi.shape[0]))
    for alpha in itertools.product(range(km + 1), repeat=d):
        if sum(alpha) > m:
            continue
        t = np.ones((xi.shape[0], mi.shape[0]))
        for k in range(d):
            t *= terms[k][:, alpha[k], :][:, mi[:, k]]
        out += t
    return out


def lagrange_derivatives(nodes: np.ndarray, x) -> np.ndarray:
    """l'_j(x) by the product rule: sum_k 1/(z_j - z_k) prod_{m != j,k} (x - z_m)/(z_j - z_m)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(nodes)
    out = np.zeros(x.shape + (n,))
    for j in range(n):
        for k in range(n):
            if k == j:
                continue
            term = np.full(x.shape, 1.0 / (nodes[j] - nodes[k]))
            for m in range(n):
                if m != j and m != k:
                    term = term * (x - nodes[m]) / (nodes[j] - nodes[m])
            out[..., j] += term
    return out


# ----------------------------------------------------------------------------------------
# Tensor-product basis on the reference cell [0,1]^d with lexicographic numbering (Sec. 3.1)
# ----------------------------------------------------------------------------------------


def local_multi_indices(d: int, p: int) -> np.ndarray:
    """Row i holds (i_1, ..., i_d) with i = i_1 + (p+1) i_2 + (p+1)^2 i_3 (first index fastest)."""
    n1 = p + 1
    idx = np.array(list(itertools.product(range(n1), repeat=d)))[:, ::-1]
    return idx  # itertools varies the last entry fastest; reversing makes entry 0 fastest


def basis_values(nodes: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """psi_i(xi_q) = prod_k l_{i_k}(xi_qk); xi has shape (nq, d); result (nq, n1^d)."""
    xi = np.atleast_2d(xi)
    d = xi.shape[1]
    mi = local_multi_indices(d, len(nodes) - 1)
    out = np.ones((xi.shape[0], mi.shape[0]))
    for k in range(d):
        lk = lagrange_values(nodes, xi[:, k])  # (nq, n1)
        out *= lk[:, mi[:, k]]
    return out


def basis_gradients(nodes: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Reference gradients d psi_i / d xi_k at xi_q; shape (nq, n1^d, d)."""
    xi = np.atleast_2d(xi)
    d = xi.shape[1]
    mi = local_multi_indices(d, len(nodes) - 1)
    vals = [lagrange_values(nodes, xi[:, k])[:, mi[:, k]] for k in range(d)]
    ders = [lagrange_derivatives(nodes, xi[:, k])[:, mi[:, k]] for k in range(d)]
    out = np.empty((xi.shape[0], mi.shape[0], d))
    for k in range(d):
        g = ders[k].copy()
        for m in range(d):
            if m != k:
                g *= vals[m]
        out[:, :, k] = g
    return out


def tensor_gauss(d: int, n: int):
    """Tensor Gauss rule on [0,1]^d: points (n^d, d) in lexicographic order, weights (n^d,)."""
    g, w = gauss_rule(n)
    mi = np.array(list(itertools.product(range(n), repeat=d)))[:, ::-1]
    pts = g[mi]
    wts = np.prod(w[mi], axis=1)
    return pts, wts


# ----------------------------------------------------------------------------------------
# Level sets and exact closest points (Sec. 2.1: closest-point projection; reading R7)
# ----------------------------------------------------------------------------------------


def phi(ls: dict, x: np.ndarray) -> np.ndarray:
    """Level-set value; the true domain is {phi < 0}.  x has shape (m, d)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    kind = ls["kind"]
    d = x.shape[1]
    if kind == "callback":
        return np.asarray(ls["phi"](x), dtype=np.float64)
    if kind == "sphere":
        c = np.asarray(ls["centre"], dtype=np.float64)[:d]
        s = np.zeros(x.shape[0])
        for k in range(d):
            s += (x[:, k] - c[k]) ** 2
        return np.sqrt(s) - ls["radius"]
    if kind == "ellipsoid":
        c = np.asarray(ls["centre"], dtype=np.float64)[:d]
        a = np.asarray(ls["semi_axes"], dtype=np.float64)[:d]
        s = np.zeros(x.shape[0])
        for k in range(d):
            s += ((x[:, k] - c[k]) / a[k]) ** 2
        return s - 1.0  # sign-equivalent to the distance
    if kind == "torus":
        c = np.asarray(ls["centre"], dtype=np.float64)
        y0, y1, y2 = x[:, 0] - c[0], x[:, 1] - c[1], x[:, 2] - c[2]
        rho = np.sqrt(y0 * y0 + y1 * y1)
        return np.sqrt((rho - ls["R"]) ** 2 + y2 * y2) - ls["r"]
    if kind == "halfspace":
        nrm = np.asarray(ls["normal"], dtype=np.float64)[:d]
        s = np.zeros(x.shape[0])
        for k in range(d):
            s += nrm[k] * x[:, k]
        return s - ls["offset"]
    if kind == "sphere_union":
        cs = np.asarray(ls["centres"], dtype=np.float64)[:, :d]
        rs = np.asarray(ls["radii"], dtype=np.float64)
        out = np.full(x.shape[0], np.inf)
        for i in range(len(rs)):
            s = np.zeros(x.shape[0])
            for k in range(d):
                s += (x[:, k] - cs[i, k]) ** 2
            out = np.minimum(out, np.sqrt(s) - rs[i])
        return out
    raise ValueError(f"unknown level-set kind {kind!r}")


def _norm_rows(v):
    return np.sqrt(np.sum(v * v, axis=1))


def _closest_sphere(c, r, y):
    u = y - c
    nu = _norm_rows(u)
    return c + r * u / nu[:, None]


def _closest_ellipsoid(c, a, y):
    """Closest point on the axis-aligned ellipsoid sum (x_k/a_k)^2 = 1 (centred at c).

    Lagrange condition x_k = a_k^2 y_k / (a_k^2 + t); t is the largest root of
    F(t) = sum (a_k y_k / (a_k^2 + t))^2 - 1, found by bisection on a bracket where
    F changes sign (Eberly, "Distance from a point to an ellipse, an ellipsoid, or a
    hyperellipsoid").  The degenerate branch (y zero along the shortest axis and no
    root) returns the + branch."""
    y = y - c
    m, d = y.shape
    a2 = a * a
    out = np.empty_like(y)
    amin2 = np.min(a2)
    for q in range(m):
        yq = y[q]
        lo = -amin2
        for k in range(d):
            if yq[k] != 0.0:
                lo = max(lo, -a2[k] + a[k] * abs(yq[k]))
        hi = max(0.0, np.sqrt(np.sum(a2 * yq * yq)))

        def F(t):
            s = 0.0
            for k in range(d):
                if yq[k] != 0.0:
                    s += (a[k] * yq[k] / (a2[k] + t)) ** 2
            return s - 1.0

        kmin = int(np.argmin(a2))
        if lo == -amin2 and yq[kmin] == 0.0 and F(lo) <= 0.0:
            x = np.empty(d)
            ssum = 0.0
            for k in range(d):
                if k == kmin:
                    continue
                x[k] = a2[k] * yq[k] / (a2[k] - amin2)
                ssum += (x[k] / a[k]) ** 2
            x[kmin] = a[kmin] * np.sqrt(max(0.0, 1.0 - ssum))
            out[q] = x
            continue
        for _ in range(400):
            mid = 0.5 * (lo + hi)
            if mid <= lo or mid >= hi:
                break
            if F(mid) > 0.0:
                lo = mid
            else:
                hi = mid
        t = 0.5 * (lo + hi)
        out[q] = a2 * yq / (a2 + t)
    return out + c


def _closest_torus(c, R, r, y):
    """Torus with axis z through c: nearest core-circle point, then radial step of length r."""
    y = y - c
    rho = np.sqrt(y[:, 0] ** 2 + y[:, 1] ** 2)
    core = np.stack([R * y[:, 0] / rho, R * y[:, 1] / rho, np.zeros_like(rho)], axis=1)
    u = y - core
    return c + core + r * u / _norm_rows(u)[:, None]


def _union_candidates(cs, rs, y):
    """Candidate nearest boundary points of a union of balls for query points y (m, d).

    Returns a list of (points (m, d), owning-ball tuple).  The candidates are the critical
    points of the distance to y restricted to each boundary stratum: on each sphere the
    nearest and farthest points; on each pairwise intersection circle (2D: the two
    intersection points) the nearest and farthest points; in 3D each triple point."""
    m, d = y.shape
    S = len(rs)
    cand = []
    for i in range(S):
        u = y - cs[i]
        nu = np.sqrt(np.sum(u * u, axis=1))
        zero = nu == 0.0
        u[zero] = 0.0
        u[zero, 0] = 1.0
        nu[zero] = 1.0
        cand.append((cs[i] + rs[i] * u / nu[:, None], (i,)))
        cand.append((cs[i] - rs[i] * u / nu[:, None], (i,)))
    for i in range(S):
        for j in range(i + 1, S):
            e = cs[j] - cs[i]
            D = np.sqrt(np.sum(e * e))
            if not (abs(rs[i] - rs[j]) < D < rs[i] + rs[j]):
                continue
            e = e / D
            t = (D * D + rs[i] ** 2 - rs[j] ** 2) / (2.0 * D)
            rho = np.sqrt(rs[i] ** 2 - t * t)
            mc = cs[i] + t * e
            if d == 2:
                perp = np.array([-e[1], e[0]])
                cand.append((np.broadcast_to(mc + rho * perp, (m, d)).copy(), (i, j)))
                cand.append((np.broadcast_to(mc - rho * perp, (m, d)).copy(), (i, j)))
            else:
                w = (y - mc) - ((y - mc) @ e)[:, None] * e[None, :]
                nw = np.sqrt(np.sum(w * w, axis=1))
                zero = nw == 0.0
                if np.any(zero):
                    # y on the circle's axis: every circle point is equidistant; fix one
                    a = np.zeros(3)
                    a[int(np.argmin(np.abs(e)))] = 1.0
                    w0 = a - np.dot(a, e) * e
                    w[zero] = w0
                    nw[zero] = np.sqrt(np.sum(w0 * w0))
                cand.append((mc + rho * w / nw[:, None], (i, j)))
                cand.append((mc - rho * w / nw[:, None], (i, j)))
    if d == 3:
        for i in range(S):
            for j in range(i + 1, S):
                for k in range(j + 1, S):
                    for pt in _three_sphere_points(cs[i], rs[i], cs[j], rs[j], cs[k], rs[k]):
                        cand.append((np.broadcast_to(pt, (m, d)).copy(), (i, j, k)))
    return cand


def _three_sphere_points(c1, r1, c2, r2, c3, r3):
    """The 0 or 2 common points of three spheres (trilateration in a local frame)."""
    ex = c2 - c1
    dd = np.sqrt(np.sum(ex * ex))
    if dd == 0.0:
        return []
    ex = ex / dd
    i = np.dot(ex, c3 - c1)
    ey = c3 - c1 - i * ex
    ney = np.sqrt(np.sum(ey * ey))
    if ney == 0.0:
        return []
    ey = ey / ney
    ez = np.cross(ex, ey)
    j = np.dot(ey, c3 - c1)
    x = (r1 * r1 - r2 * r2 + dd * dd) / (2.0 * dd)
    yv = (r1 * r1 - r3 * r3 + i * i + j * j) / (2.0 * j) - (i / j) * x
    z2 = r1 * r1 - x * x - yv * yv
    if z2 <= 0.0:
        return []
    z = np.sqrt(z2)
    base = c1 + x * ex + yv * ey
    return [base + z * ez, base - z * ez]


def _closest_union(cs, rs, y):
    """Nearest valid candidate: a candidate is valid unless it lies strictly inside a ball
    other than its own; ties go to the lowest candidate index."""
    best = np.full(y.shape[0], np.inf)
    out = np.full(y.shape, np.nan)
    for pts, own in _union_candidates(cs, rs, y):
        ok = np.ones(y.shape[0], dtype=bool)
        for l in range(len(rs)):
            if l in own:
                continue
            ok &= np.sqrt(np.sum((pts - cs[l]) ** 2, axis=1)) >= rs[l]
        dist = np.sqrt(np.sum((pts - y) ** 2, axis=1))
        take = ok & (dist < best)
        best[take] = dist[take]
        out[take] = pts[take]
    return out


def closest_point(ls: dict, x: np.ndarray) -> np.ndarray:
    """Exact closest point on the zero level set for each row of x (reading R7)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    d = x.shape[1]
    kind = ls["kind"]
    if kind == "sphere":
        return _closest_sphere(np.asarray(ls["centre"], dtype=np.float64)[:d], ls["radius"], x)
    if kind == "ellipsoid":
        return _closest_ellipsoid(np.asarray(ls["centre"], dtype=np.float64)[:d],
                                  np.asarray(ls["semi_axes"], dtype=np.float64)[:d], x)
    if kind == "torus":
        return _closest_torus(np.asarray(ls["centre"], dtype=np.float64), ls["R"], ls["r"], x)
    if kind == "halfspace":
        nrm = np.asarray(ls["normal"], dtype=np.float64)[:d]
        return x - (phi(ls, x))[:, None] * nrm[None, :]
    if kind == "sphere_union":
        return _closest_union(np.asarray(ls["centres"], dtype=np.float64)[:, :d],
                              np.asarray(ls["radii"], dtype=np.float64), x)
    if kind == "callback":
        return _closest_newton(ls, x)
    raise ValueError(f"unknown level-set kind {kind!r}")


def _closest_newton(ls: dict, x: np.ndarray) -> np.ndarray:
    """Level-set Newton projection (Sec. 4.4: the projection is a Newton solve on the level
    set): per point, y <- y - phi(y) grad phi(y) / |grad phi(y)|^2 from y = x.  The paper does
    not fix a stopping rule; the one used here is scale-aware: stop when the Newton step
    |phi(y)| / |grad phi(y)| is at most 8 eps max(1, max_k |y_k|) (eps = 2^-52), i.e. when the
    point is within a few units in the last place of the zero set, whatever the scaling of phi.
    A point that needs more than 50 steps is an error.  This reaches a point of the boundary;
    it is the closest one for a distance function or, more generally, when the gradient lines
    are straight (spheres, tori given by their distance)."""
    eps = np.finfo(np.float64).eps
    y = np.array(x, dtype=np.float64)
    todo = np.ones(y.shape[0], dtype=bool)
    for it in range(51):
        idx = np.flatnonzero(todo)
        yt = y[idx]
        ph = np.asarray(ls["phi"](yt), dtype=np.float64)
        g = np.asarray(ls["grad"](yt), dtype=np.float64)
        g2 = np.sum(g * g, axis=1)
        scale = np.maximum(1.0, np.max(np.abs(yt), axis=1))
        done = np.isfinite(ph) & (np.abs(ph) <= 8.0 * eps * np.sqrt(g2) * scale)
        todo[idx[done]] = False
        if not todo.any():
            return y
        if it == 50:
            break
        step = ~done
        y[idx[step]] -= ph[step][:, None] * g[step] / g2[step][:, None]
    raise ValueError("level-set Newton projection did not converge in 50 steps")


# ----------------------------------------------------------------------------------------
# Surrogate domain: active cells, faces, DoF numbering  (Sec. 2, Sec. 3.4; readings R2, R6)
# ----------------------------------------------------------------------------------------


@dataclass
class Problem:
    d: int
    p: int
    n: tuple
    lo: np.ndarray
    hi: np.ndarray
    h: float
    levelset: dict
    disc: str  # "cg" or "dg"
    gamma: float
    gamma_dg: float
    shift_scale: float
    nodes: np.ndarray = field(repr=False)
    cells: np.ndarray = field(repr=False)  # (nc, d) multi-indices of active cells, lexicographic
    cell_dofs: np.ndarray = field(repr=False)  # (nc, n1^d) global DoF ids
    n_dofs: int = 0
    sbm_faces: np.ndarray = field(default=None, repr=False)  # (nf, 3): cell rank, axis, side
    interior_faces: np.ndarray = field(default=None, repr=False)  # (ni, 3): rank K1, rank K2, axis
    face_xi_tilde: np.ndarray = field(default=None, repr=False)  # (nf, nq, d)
    face_x_tilde: np.ndarray = field(default=None, repr=False)  # (nf, nq, d)
    face_x_true: np.ndarray = field(default=None, repr=False)  # (nf, nq, d)
    face_xi: np.ndarray = field(default=None, repr=False)  # (nf, nq, d) shifted reference coords
    face_w: np.ndarray = field(default=None, repr=False)  # (nq,) reference tangential weights
    taylor_order: int | None = None  # None: full extension (R1); m >= 0: truncated E_m (R8)

    @property
    def n1(self):
        return self.p + 1

    @property
    def sigma_gamma(self):
        return self.gamma * self.p * self.p / self.h

    @property
    def sigma_f(self):
        return self.gamma_dg * self.p * self.p / self.h


def cell_is_active(d, n, lo, h, ls):
    """Boolean array of shape n (axis 0 = first coordinate): phi < 0 at all 2^d vertices."""
    axes = [lo[k] + h * np.arange(n[k] + 1) for k in range(d)]
    grids = np.meshgrid(*axes, indexing="ij")
    pts = np.stack([g.ravel() for g in grids], axis=1)
    val = phi(ls, pts).reshape([n[k] + 1 for k in range(d)])
    act = np.ones(tuple(n), dtype=bool)
    for off in itertools.product((0, 1), repeat=d):
        sl = tuple(slice(off[k], off[k] + n[k]) for k in range(d))
        act &= val[sl] < 0.0
    return act


def face_reference_points(d: int, p: int, axis: int, side: int):
    """Gauss points of face (axis, side) of [0,1]^d: xi_axis = side, tangential Gauss points
    in increasing axis order with the lower tangential axis fastest.  Returns (pts, weights)."""
    g, w = gauss_rule(p + 1)
    tang = [k for k in range(d) if k != axis]
    mi = np.array(list(itertools.product(range(p + 1), repeat=d - 1)))[:, ::-1]
    pts = np.empty((mi.shape[0], d))
    pts[:, axis] = float(side)
    wts = np.ones(mi.shape[0])
    for t, k in enumerate(tang):
        pts[:, k] = g[mi[:, t]]
        wts *= w[mi[:, t]]
    return pts, wts


def setup(d, n, lo, hi, levelset, p, disc="cg", gamma=10.0, gamma_dg=10.0, shift_scale=1.0,
          taylor_order=None):
    """Build the surrogate domain, face data and DoF numbering for one problem.
    taylor_order: None for the full extension E (R1), m >= 0 for the truncated E_m (R8)."""
    n = tuple(int(v) for v in (n if np.ndim(n) else [n] * d))[:d]
    lo = np.asarray(lo if np.ndim(lo) else [lo] * d, dtype=np.float64)[:d]
    hi = np.asarray(hi if np.ndim(hi) else [hi] * d, dtype=np.float64)[:d]
    hs = (hi - lo) / np.asarray(n, dtype=np.float64)
    if np.max(np.abs(hs - hs[0])) > 1e-12 * hs[0]:
        raise ValueError("the oracle handles isotropic cells only")
    h = float(hs[0])
    n1 = p + 1
    act = cell_is_active(d, n, lo, h, levelset)
    # lexicographic order with the first coordinate fastest: transpose before argwhere
    cells = np.argwhere(act.transpose())[:, ::-1]
    nc = cells.shape[0]
    rank = -np.ones(tuple(n), dtype=np.int64)
    if nc:
        rank[tuple(cells.T)] = np.arange(nc)
    mi = local_multi_indices(d, p)
    if disc == "cg":
        lat = tuple(p * n[k] + 1 for k in range(d))
        touched = np.zeros(lat, dtype=bool)
        for loc in mi:
            touched[tuple(cells[:, k] * p + loc[k] for k in range(d))] = True
        # ranks in lexicographic order, first coordinate fastest
        flat = touched.transpose().ravel()
        ids_t = np.cumsum(flat) - 1
        ids = ids_t.reshape(tuple(reversed(lat))).transpose()
        cell_dofs = np.empty((nc, mi.shape[0]), dtype=np.int64)
        for li, loc in enumerate(mi):
            cell_dofs[:, li] = ids[tuple(cells[:, k] * p + loc[k] for k in range(d))]
        n_dofs = int(flat.sum())
    elif disc == "dg":
        cell_dofs = np.arange(nc * n1 ** d, dtype=np.int64).reshape(nc, n1 ** d)
        n_dofs = nc * n1 ** d
    else:
        raise ValueError("disc must be 'cg' or 'dg'")

    # faces
    sbm, inter = [], []
    for r in range(nc):
        c = cells[r]
        for a in range(d):
            for s in (0, 1):
                nb = c.copy()
                nb[a] += 1 if s == 1 else -1
                inside = 0 <= nb[a] < n[a]
                nb_rank = rank[tuple(nb)] if inside else -1
                if nb_rank < 0:
                    sbm.append((r, a, s))
                elif s == 1:
                    inter.append((r, nb_rank, a))
    sbm = np.array(sbm, dtype=np.int64).reshape(-1, 3)
    inter = np.array(inter, dtype=np.int64).reshape(-1, 3)

    nodes = gll_nodes(p)
    prob = Problem(d=d, p=p, n=n, lo=lo, hi=hi, h=h, levelset=levelset, disc=disc, gamma=gamma,
                   gamma_dg=gamma_dg, shift_scale=shift_scale, nodes=nodes, cells=cells,
                   cell_dofs=cell_dofs, n_dofs=n_dofs, sbm_faces=sbm, interior_faces=inter)
    nf = sbm.shape[0]
    nq = n1 ** (d - 1)
    xi_t = np.empty((nf, nq, d))
    w_face = None
    for f in range(nf):
        pts, w_face = face_reference_points(d, p, int(sbm[f, 1]), int(sbm[f, 2]))
        xi_t[f] = pts
    if w_face is None:
        _, w_face = face_reference_points(d, p, 0, 0)
    if nf:
        cpos = cells[sbm[:, 0]].astype(np.float64)  # (nf, d)
        x_t = lo[None, None, :] + h * (cpos[:, None, :] + xi_t)
        x_true = closest_point(levelset, x_t.reshape(-1, d)).reshape(nf, nq, d)
        dvec = shift_scale * (x_true - x_t)
        xi = xi_t + dvec / h
    else:
        x_t = x_true = xi = np.empty((0, nq, d))
    prob.face_xi_tilde = xi_t
    prob.face_x_tilde = x_t
    prob.face_x_true = x_true
    prob.face_xi = xi
    prob.face_w = w_face
    if taylor_order is not None and int(taylor_order) < 0:
        raise ValueError("taylor_order must be None or >= 0")
    prob.taylor_order = None if taylor_order is None else int(taylor_order)
    return prob


# ----------------------------------------------------------------------------------------
# Local matrices by brute-force quadrature
# ----------------------------------------------------------------------------------------


def cell_matrix(prob: Problem) -> np.ndarray:
    """A^K_ij = sum_q W_q h^(d-2) grad_xi psi_i(g_q) . grad_xi psi_j(g_q)  (Alg. 1; all active
    cells are translates of one reference cell with Jacobian h I, Sec. 3.4)."""
    d, p, h = prob.d, prob.p, prob.h
    pts, wts = tensor_gauss(d, p + 1)
    G = basis_gradients(prob.nodes, pts)  # (nq, nb, d)
    A = np.zeros((G.shape[1], G.shape[1]))
    for q in range(pts.shape[0]):
        A += wts[q] * (G[q] @ G[q].T)
    return A * h ** (d - 2)


def sbm_face_matrix(prob: Problem, f: int) -> np.ndarray:
    """Local SBM face matrix B (rows = test i, columns = trial j) for surrogate face f:

        B_ij = sum_q w_q [ -(dn psi_j)(xi~_q) psi_i(xi~_q)
                           -(dn psi_i)(xi~_q) psi_j(xi_q)
                           + sigma_Gam psi_j(xi_q) psi_i(xi~_q) ]

    with w_q = h^(d-1) * tangential Gauss weights, dn = (2 side - 1)/h d/dxi_axis the
    physical derivative along the outward surrogate normal, and xi_q the shifted
    reference point (Eq. (1) bilinear form; Alg. 3).  With a truncated extension (R8)
    psi_j(xi_q) is replaced by E_m psi_j, the Taylor expansion about xi~_q of order m."""
    d, h = prob.d, prob.h
    _, a, s = (int(v) for v in prob.sbm_faces[f])
    xt = prob.face_xi_tilde[f]
    xs = prob.face_xi[f]
    om = prob.face_w * h ** (d - 1)
    sgn = 2.0 * s - 1.0
    V_t = basis_values(prob.nodes, xt)  # psi_i(xi~_q)
    D_t = basis_gradients(prob.nodes, xt)[:, :, a] * (sgn / h)  # dn psi_i(xi~_q)
    if prob.taylor_order is None:
        V_s = basis_values(prob.nodes, xs)  # psi_j(xi_q)
    else:
        V_s = basis_taylor_values(prob.nodes, xt, xs, prob.taylor_order)  # E_m psi_j
    sig = prob.sigma_gamma
    nb = V_t.shape[1]
    B = np.zeros((nb, nb))
    for q in range(xt.shape[0]):
        B += om[q] * (-np.outer(V_t[q], D_t[q]) - np.outer(D_t[q], V_s[q]) + sig * np.outer(V_t[q], V_s[q]))
    return B


def dg_face_blocks(prob: Problem, fi: int):
    """SIPG interior-face blocks for face fi between K1 (lower) and K2 = K1 + e_axis:

        a_F(u,v) = sum_q w_q ( sigma_F [u][v] - {dn u}[v] - [u]{dn v} ),
        [w] = w_K1 - w_K2, {dn w} = (dn w_K1 + dn w_K2)/2, n = +e_axis  (Sec. 3.2, Alg. 2).

    Returns {(0,0): B11, (0,1): B12, (1,0): B21, (1,1): B22} with (test cell, trial cell)."""
    d, h = prob.d, prob.h
    a = int(prob.interior_faces[fi, 2])
    p1, w = face_reference_points(d, prob.p, a, 1)
    p2, _ = face_reference_points(d, prob.p, a, 0)
    om = w * h ** (d - 1)
    V = [basis_values(prob.nodes, p1), basis_values(prob.nodes, p2)]
    Dn = [basis_gradients(prob.nodes, p1)[:, :, a] / h, basis_gradients(prob.nodes, p2)[:, :, a] / h]
    J = [V[0], -V[1]]  # jump contribution of each side's basis
    Av = [0.5 * Dn[0], 0.5 * Dn[1]]  # average-normal-derivative contribution
    sig = prob.sigma_f
    nb = V[0].shape[1]
    out = {}
    for ti in range(2):
        for tj in range(2):
            B = np.zeros((nb, nb))
            for q in range(p1.shape[0]):
                B += om[q] * (sig * np.outer(J[ti][q], J[tj][q])
                              - np.outer(J[ti][q], Av[tj][q])
                              - np.outer(Av[ti][q], J[tj][q]))
            out[(ti, tj)] = B
    return out


# ----------------------------------------------------------------------------------------
# Assembly, apply, right-hand side, solve, error
# ----------------------------------------------------------------------------------------


def assemble(prob: Problem, parts=("cell", "sbm", "dg")) -> sp.csr_matrix:
    """Global sparse matrix: plain sum of local blocks scattered through the DoF maps (Sec. 3.5)."""
    rows, cols, vals = [], [], []
    cd = prob.cell_dofs
    nb = cd.shape[1]
    if "cell" in parts and cd.shape[0]:
        A = cell_matrix(prob)
        rows.append(np.repeat(cd, nb, axis=1).ravel())
        cols.append(np.tile(cd, (1, nb)).ravel())
        vals.append(np.broadcast_to(A.ravel(), (cd.shape[0], nb * nb)).ravel())
    if "sbm" in parts:
        for f in range(prob.sbm_faces.shape[0]):
            dofs = cd[prob.sbm_faces[f, 0]]
            B = sbm_face_matrix(prob, f)
            rows.append(np.repeat(dofs, nb))
            cols.append(np.tile(dofs, nb))
            vals.append(B.ravel())
    if "dg" in parts and prob.disc == "dg":
        for fi in range(prob.interior_faces.shape[0]):
            ks = (prob.interior_faces[fi, 0], prob.interior_faces[fi, 1])
            blocks = dg_face_blocks(prob, fi)
            for (ti, tj), B in blocks.items():
                rows.append(np.repeat(cd[ks[ti]], nb))
                cols.append(np.tile(cd[ks[tj]], nb))
                vals.append(B.ravel())
    if not rows:
        return sp.csr_matrix((prob.n_dofs, prob.n_dofs))
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(prob.n_dofs, prob.n_dofs))
    return M.tocsr()


def apply(prob: Problem, u: np.ndarray, A: sp.csr_matrix | None = None) -> np.ndarray:
    """v = A u with the assembled matrix (the definition the matrix-free path reproduces)."""
    if A is None:
        A = assemble(prob)
    return A @ np.asarray(u, dtype=np.float64)


def dof_points(prob: Problem) -> np.ndarray:
    """Physical coordinates of every DoF (GLL node of its cell), shape (n_dofs, d)."""
    mi = local_multi_indices(prob.d, prob.p)
    out = np.empty((prob.n_dofs, prob.d))
    for li, loc in enumerate(mi):
        pos = prob.lo[None, :] + prob.h * (prob.cells + prob.nodes[loc][None, :])
        out[prob.cell_dofs[:, li]] = pos
    return out


def interpolate(prob: Problem, fn) -> np.ndarray:
    """Nodal interpolant I_h u: the DoF vector of fn at the GLL nodes."""
    return fn(dof_points(prob))


def rhs(prob: Problem, f_fn, g_fn) -> np.ndarray:
    """Right-hand side of Eq. (1):
        b_i = int f psi_i - int_{Gam~} (dn psi_i) g + int_{Gam~} sigma_Gam g psi_i,
    with g evaluated at the true-boundary point x_q of each surrogate-face quadrature point."""
    d, h = prob.d, prob.h
    b = np.zeros(prob.n_dofs)
    pts, wts = tensor_gauss(d, prob.p + 1)
    V = basis_values(prob.nodes, pts)  # (nq, nb)
    for r in range(prob.cells.shape[0]):
        x = prob.lo[None, :] + h * (prob.cells[r][None, :] + pts)
        fv = f_fn(x) * wts * h ** d
        np.add.at(b, prob.cell_dofs[r], V.T @ fv)
    om = prob.face_w * h ** (d - 1)
    for f in range(prob.sbm_faces.shape[0]):
        r, a, s = (int(v) for v in prob.sbm_faces[f])
        xt = prob.face_xi_tilde[f]
        g = g_fn(prob.face_x_true[f])
        V_t = basis_values(prob.nodes, xt)
        D_t = basis_gradients(prob.nodes, xt)[:, :, a] * ((2.0 * s - 1.0) / h)
        loc = (-D_t.T @ (om * g)) + prob.sigma_gamma * (V_t.T @ (om * g))
        np.add.at(b, prob.cell_dofs[r], loc)
    return b


def l2_error(prob: Problem, uh: np.ndarray, u_fn) -> float:
    """L2 error on the surrogate domain with (p+3)^d Gauss points per cell (App. A)."""
    d, h = prob.d, prob.h
    pts, wts = tensor_gauss(d, prob.p + 3)
    V = basis_values(prob.nodes, pts)
    err = 0.0
    for r in range(prob.cells.shape[0]):
        x = prob.lo[None, :] + h * (prob.cells[r][None, :] + pts)
        diff = V @ uh[prob.cell_dofs[r]] - u_fn(x)
        err += np.sum(wts * diff * diff) * h ** d
    return float(np.sqrt(err))


def solve_direct(A: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    """Sparse direct solve (tiny meshes only)."""
    import scipy.sparse.linalg as spla
    return spla.spsolve(A.tocsc(), b)
