"""Seeded synthetic inputs for the SBM Poisson workloads.

This module holds no part of the method's arithmetic: it only draws random vectors and
geometry parameters and names the workloads (mesh, degree, discretisation, level set,
manufactured solution).  Both the HIP library's harness and the CPU oracle consume what
it returns, so neither side ever generates an input for the other.

Random numbers come from torch's CPU generator (Philox-free Mersenne twister behind
``torch.Generator(device="cpu").manual_seed(s)``), so a seed gives the same arrays on
every machine.  Seeds: 0 for apply vectors (uniform on [-1, 1]); 1 for the random sphere
union (radii first, then centres).
"""

from __future__ import annotations

import math

import numpy as np
import torch


def _gen(seed: int) -> torch.Generator:
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    return g


def uniform_vector(n: int, seed: int = 0, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """n FP64 values uniform on [lo, hi) from the given seed."""
    t = torch.rand(int(n), generator=_gen(seed), dtype=torch.float64)
    return (lo + (hi - lo) * t).numpy()


def sphere_union(seed: int = 1, n: int = 8, r_range=(0.15, 0.35), c_range=(-0.6, 0.6), d: int = 3):
    """Level-set descriptor of a union of n balls: radii U[r_range] drawn first, then
    centres U[c_range]^d (row-major n x d)."""
    g = _gen(seed)
    r = torch.rand(n, generator=g, dtype=torch.float64)
    c = torch.rand(n, d, generator=g, dtype=torch.float64)
    radii = r_range[0] + (r_range[1] - r_range[0]) * r
    centres = c_range[0] + (c_range[1] - c_range[0]) * c
    return {"kind": "sphere_union", "centres": centres.numpy().copy(), "radii": radii.numpy().copy()}


def callback(phi, grad, dim):
    """Level set given by functions of an (N, dim) array of points: phi(X) -> (N,) values and
    grad(X) -> (N, dim) gradients (the library calls them one point at a time)."""
    return {"kind": "callback", "phi": phi, "grad": grad, "dim": int(dim)}


def sphere(centre, radius):
    return {"kind": "sphere", "centre": list(map(float, centre)), "radius": float(radius)}


def ellipsoid(centre, semi_axes):
    return {"kind": "ellipsoid", "centre": list(map(float, centre)),
            "semi_axes": list(map(float, semi_axes))}


def torus(R, r, centre=(0.0, 0.0, 0.0)):
    return {"kind": "torus", "centre": list(map(float, centre)), "R": float(R), "r": float(r)}


def halfspace(normal, offset):
    return {"kind": "halfspace", "normal": list(map(float, normal)), "offset": float(offset)}


# ---- manufactured solutions (problem data: u*, f = -Laplace u*, g = u* on the boundary) ----

# The data are evaluated with torch's CPU kernels (vectorised and multithreaded; numpy's
# are single-threaded, and a 64^3 Q6 request has 45 M quadrature points): FP64 arrays in, FP64
# numpy arrays out.
def _trig(fn, a):
    return fn(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)) * math.pi)


def manufactured_2d():
    """u* = sin(pi x) cos(pi y); f = 2 pi^2 u*."""
    u = lambda x: (_trig(torch.sin, x[:, 0]) * _trig(torch.cos, x[:, 1])).numpy()
    f = lambda x: (2.0 * math.pi ** 2 * (_trig(torch.sin, x[:, 0]) * _trig(torch.cos, x[:, 1]))).numpy()
    return u, f


def manufactured_3d():
    """u* = sin(pi x) sin(pi y) sin(pi z); f = 3 pi^2 u*."""
    u = lambda x: (_trig(torch.sin, x[:, 0]) * _trig(torch.sin, x[:, 1]) * _trig(torch.sin, x[:, 2])).numpy()
    f = lambda x: 3.0 * math.pi ** 2 * u(x)
    return u, f


def manufactured(d: int):
    return manufactured_2d() if d == 2 else manufactured_3d()


def manufactured_cell_f(d: int, cells: np.ndarray, lo: float, h: float, p: int) -> np.ndarray:
    """f of the manufactured solution at the (p+1)^d Gauss points of every cell (cells: n x d
    integer corners; points lexicographic, first coordinate fastest; shape n x (p+1)^d), by the
    product structure of u*: per cell and axis the p+1 one-dimensional factors, then their
    outer product (the same values as f at the points, to rounding; d(p+1) sines per cell
    instead of d(p+1)^d)."""
    g = (np.polynomial.legendre.leggauss(p + 1)[0] + 1.0) / 2.0
    c = np.asarray(cells, dtype=np.float64)
    x = [lo + h * (c[:, m:m + 1] + g[None, :]) for m in range(d)]  # n x (p+1) per axis
    if d == 2:
        a, b = np.sin(np.pi * x[0]), np.cos(np.pi * x[1])
        f = 2.0 * math.pi ** 2 * (b[:, :, None] * a[:, None, :])
    else:
        a, b, e = (np.sin(np.pi * x[m]) for m in range(3))
        f = 3.0 * math.pi ** 2 * (e[:, :, None, None] * (b[:, None, :, None] * a[:, None, None, :]))
    return np.ascontiguousarray(f.reshape(len(c), (p + 1) ** d))


# ---- named workloads ----

def workload(name: str, **over):
    """Mesh/degree/discretisation/level-set description of a named workload.

    disk2d_q2:        2D CG Q2, 16^2 cells on [-1,1]^2, disk r=0.7 centred (0.05,-0.03)
    sphere3d_q4:      3D CG Q4, 64^3 cells on [-1,1]^3, sphere r=0.75 at the origin
    torus3d_dg:       3D SIPG DG, 32^3 cells, torus R=0.6 r=0.25 (axis z), p=3 or 5
    torus3d_dg80:     the same DG Q3 torus on 80^3 cells (fills the device)
    spheres3d_q6:     3D CG Q6, 48^3 cells, union of 8 seeded balls
    """
    if name == "disk2d_q2":
        w = dict(d=2, n=16, lo=-1.0, hi=1.0, p=2, disc="cg", levelset=sphere((0.05, -0.03), 0.7))
    elif name == "sphere3d_q4":
        w = dict(d=3, n=64, lo=-1.0, hi=1.0, p=4, disc="cg", levelset=sphere((0, 0, 0), 0.75))
    elif name == "torus3d_dg":
        w = dict(d=3, n=32, lo=-1.0, hi=1.0, p=3, disc="dg", levelset=torus(0.6, 0.25))
    elif name == "torus3d_dg80":
        w = dict(d=3, n=80, lo=-1.0, hi=1.0, p=3, disc="dg", levelset=torus(0.6, 0.25))
    elif name == "spheres3d_q6":
        w = dict(d=3, n=48, lo=-1.0, hi=1.0, p=6, disc="cg", levelset=sphere_union(1))
    else:
        raise KeyError(name)
    w.update(over)
    return w


def serving_requests(n: int = 512, seed: int = 2, rate: float = 1.0, n_range=(16, 64),
                     p_range=(2, 6)):
    """Stream of solve requests: Poisson arrival times (exponential gaps of mean 1/rate),
    p uniform in p_range, cells per direction uniform in n_range, half ellipsoids
    (semi-axes U[0.4, 0.8]) and half 8-ball unions, half CG and half SIPG."""
    g = _gen(seed)
    out = []
    t = 0.0
    for i in range(n):
        u = torch.rand(8, generator=g, dtype=torch.float64).numpy()
        t += -math.log(max(1e-300, 1.0 - u[0])) / rate
        p = p_range[0] + int(u[1] * (p_range[1] - p_range[0] + 1))
        nc = n_range[0] + int(u[2] * (n_range[1] - n_range[0] + 1))
        if u[3] < 0.5:
            ax = 0.4 + 0.4 * torch.rand(3, generator=g, dtype=torch.float64).numpy()
            ls = ellipsoid((0.0, 0.0, 0.0), ax)
        else:
            ls = sphere_union(seed=int(1000 + i))
        disc = "cg" if u[4] < 0.5 else "dg"
        out.append(dict(id=i, arrival=t, d=3, n=nc, lo=-1.0, hi=1.0, p=p, disc=disc, levelset=ls,
                        rhs_seed=int(10000 + i)))
    return out
