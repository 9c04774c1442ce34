// Analytic level sets: value phi and exact closest point on {phi = 0} (Sec. 2: the true
// domain is {phi < 0}; Sec. 4.4: every surrogate-face quadrature point is mapped to its closest
// point on the true boundary).  Host and device share this one implementation, so the setup
// built on the device and the one built on the host see the same geometry operation by
// operation (the device setup is compiled without floating-point contraction).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>

#include "../../include/sbm.h"

namespace sbm {

struct LsParams {
  int kind = SBM_LS_SPHERE;
  int dim = 3;
  double centre[3] = {0, 0, 0};
  double radius = 0, R = 0, r = 0, offset = 0;
  double semi[3] = {1, 1, 1};
  double normal[3] = {1, 0, 0};
  int n_spheres = 0;
  const double *cs = nullptr;  // n_spheres x 3 (host or device memory, as the caller runs)
  const double *rs = nullptr;  // n_spheres
};

__host__ __device__ inline double ls_norm(const double *v, int d) {
  double s = 0;
  for (int k = 0; k < d; ++k) s += v[k] * v[k];
  return std::sqrt(s);
}

// phi for the analytic kinds (SBM_LS_CALLBACK is evaluated by the caller's function).
__host__ __device__ inline double ls_phi(const LsParams &L, const double *x) {
  const int d = L.dim;
  switch (L.kind) {
    case SBM_LS_SPHERE: {
      double s = 0;
      for (int k = 0; k < d; ++k) s += (x[k] - L.centre[k]) * (x[k] - L.centre[k]);
      return std::sqrt(s) - L.radius;
    }
    case SBM_LS_ELLIPSOID: {
      double s = 0;
      for (int k = 0; k < d; ++k) {
        const double t = (x[k] - L.centre[k]) / L.semi[k];
        s += t * t;
      }
      return s - 1.0;
    }
    case SBM_LS_TORUS: {
      const double y0 = x[0] - L.centre[0], y1 = x[1] - L.centre[1], y2 = x[2] - L.centre[2];
      const double rho = std::sqrt(y0 * y0 + y1 * y1);
      return std::sqrt((rho - L.R) * (rho - L.R) + y2 * y2) - L.r;
    }
    case SBM_LS_HALFSPACE: {
      double s = 0;
      for (int k = 0; k < d; ++k) s += L.normal[k] * x[k];
      return s - L.offset;
    }
    case SBM_LS_SPHERE_UNION: {
      double best = std::numeric_limits<double>::infinity();
      for (int i = 0; i < L.n_spheres; ++i) {
        double s = 0;
        for (int k = 0; k < d; ++k) s += (x[k] - L.cs[3 * i + k]) * (x[k] - L.cs[3 * i + k]);
        best = std::min(best, std::sqrt(s) - L.rs[i]);
      }
      return best;
    }
  }
  return 0.0;
}

// Ellipsoid: x_k = a_k^2 y_k / (a_k^2 + t) with t the largest root of
// F(t) = sum (a_k y_k / (a_k^2 + t))^2 - 1, found by Newton from the left end of a bracket
// (bisection if that fails).
__host__ __device__ inline void ls_closest_ellipsoid(const double *a, const double *c, int d, const double *x,
                                                     double *out) {
  double y[3] = {0, 0, 0}, a2[3] = {1, 1, 1};
  double amin2 = std::numeric_limits<double>::infinity();
  int kmin = 0;
  for (int k = 0; k < d; ++k) {
    y[k] = x[k] - c[k];
    a2[k] = a[k] * a[k];
    if (a2[k] < amin2) {
      amin2 = a2[k];
      kmin = k;
    }
  }
  auto F = [&](double t) {
    double s = 0;
    for (int k = 0; k < d; ++k)
      if (y[k] != 0.0) {
        const double q = a[k] * y[k] / (a2[k] + t);
        s += q * q;
      }
    return s - 1.0;
  };
  double lo = -amin2;
  for (int k = 0; k < d; ++k)
    if (y[k] != 0.0) lo = std::max(lo, -a2[k] + a[k] * std::fabs(y[k]));
  double hs = 0;
  for (int k = 0; k < d; ++k) hs += a2[k] * y[k] * y[k];
  double hi = std::max(0.0, std::sqrt(hs));
  if (lo == -amin2 && y[kmin] == 0.0 && F(lo) <= 0.0) {
    double s = 0;
    for (int k = 0; k < d; ++k) {
      if (k == kmin) continue;
      out[k] = a2[k] * y[k] / (a2[k] - amin2);
      s += (out[k] / a[k]) * (out[k] / a[k]);
    }
    out[kmin] = a[kmin] * std::sqrt(std::max(0.0, 1.0 - s));
    for (int k = 0; k < d; ++k) out[k] += c[k];
    return;
  }
  // F is convex and decreasing on (-amin2, inf), and F(lo) >= 0 (a term with y_k != 0 is
  // at least 1 at -a_k^2 + a_k |y_k|): a tangent lies below F, so Newton's method from lo
  // moves right monotonically and never passes the root.  It stops when F reaches 0 or the
  // step no longer moves t; bisection on [lo, hi] is the fallback.
  double t = lo;
  bool done = false;
  for (int it = 0; it < 100; ++it) {
    double f = -1.0, df = 0.0;
    for (int k = 0; k < d; ++k)
      if (y[k] != 0.0) {
        const double den = a2[k] + t, q = a[k] * y[k] / den;
        f += q * q;
        df -= 2.0 * q * q / den;
      }
    if (!(f > 0.0)) {
      done = f == 0.0 || it > 0;  // at or (by rounding) just past the root
      break;
    }
    if (!(df < 0.0)) break;
    const double tn = t - f / df;
    if (!(tn > t) || !(tn <= hi)) {
      done = !(tn > t);
      break;
    }
    t = tn;
  }
  if (!done) {
    for (int it = 0; it < 400; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (F(mid) > 0.0)
        lo = mid;
      else
        hi = mid;
    }
    t = 0.5 * (lo + hi);
  }
  for (int k = 0; k < d; ++k) out[k] = c[k] + a2[k] * y[k] / (a2[k] + t);
}

// Union of balls: nearest among the critical points of the distance on every boundary
// stratum (each sphere: nearest/farthest point; each pairwise circle: nearest/farthest
// point, or the two intersection points in 2D; each triple point in 3D) that is not
// strictly inside another ball.  Candidates are visited in a fixed order and the first
// strict minimum wins.  Returns false (out = NaN) if no candidate survives.
__host__ __device__ inline bool ls_closest_union(const double *cs, const double *rs, int S, int d, const double *x,
                                                 double *out) {
  double best = std::numeric_limits<double>::infinity();
  bool found = false;
  auto consider = [&](const double *pt, int o0, int o1, int o2) {
    for (int l = 0; l < S; ++l) {
      if (l == o0 || l == o1 || l == o2) continue;
      double s = 0;
      for (int k = 0; k < d; ++k) s += (pt[k] - cs[3 * l + k]) * (pt[k] - cs[3 * l + k]);
      if (std::sqrt(s) < rs[l]) return;
    }
    double s = 0;
    for (int k = 0; k < d; ++k) s += (pt[k] - x[k]) * (pt[k] - x[k]);
    const double dist = std::sqrt(s);
    if (dist < best) {
      best = dist;
      found = true;
      for (int k = 0; k < d; ++k) out[k] = pt[k];
    }
  };
  // Every point of sphere i is at least lb(i) = | |x - c_i| - r_i | from x, so a seam or triple
  // point of spheres whose bounds exceed the best distance so far (with a margin far above
  // rounding) cannot be selected and is skipped: the result is that of the full enumeration.
  auto lb = [&](int i) {
    double u[3];
    for (int k = 0; k < d; ++k) u[k] = x[k] - cs[3 * i + k];
    return std::fabs(ls_norm(u, d) - rs[i]);
  };
  auto hopeless = [&](double bound) { return bound > best * (1.0 + 1e-12) + 1e-300; };
  double pt[3] = {0, 0, 0};
  for (int i = 0; i < S; ++i) {
    double u[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) u[k] = x[k] - cs[3 * i + k];
    double nu = ls_norm(u, d);
    if (nu == 0.0) {
      for (int k = 0; k < d; ++k) u[k] = 0.0;
      u[0] = 1.0;
      nu = 1.0;
    }
    for (int k = 0; k < d; ++k) pt[k] = cs[3 * i + k] + rs[i] * u[k] / nu;
    consider(pt, i, -1, -1);
    for (int k = 0; k < d; ++k) pt[k] = cs[3 * i + k] - rs[i] * u[k] / nu;
    consider(pt, i, -1, -1);
  }
  for (int i = 0; i < S; ++i)
    for (int j = i + 1; j < S; ++j) {
      if (hopeless(std::max(lb(i), lb(j)))) continue;
      double e[3] = {0, 0, 0};
      for (int k = 0; k < d; ++k) e[k] = cs[3 * j + k] - cs[3 * i + k];
      const double D = ls_norm(e, d);
      if (!(std::fabs(rs[i] - rs[j]) < D && D < rs[i] + rs[j])) continue;
      for (int k = 0; k < d; ++k) e[k] /= D;
      const double t = (D * D + rs[i] * rs[i] - rs[j] * rs[j]) / (2.0 * D);
      const double rho = std::sqrt(rs[i] * rs[i] - t * t);
      double m[3] = {0, 0, 0};
      for (int k = 0; k < d; ++k) m[k] = cs[3 * i + k] + t * e[k];
      if (d == 2) {
        const double perp[2] = {-e[1], e[0]};
        for (int k = 0; k < 2; ++k) pt[k] = m[k] + rho * perp[k];
        consider(pt, i, j, -1);
        for (int k = 0; k < 2; ++k) pt[k] = m[k] - rho * perp[k];
        consider(pt, i, j, -1);
      } else {
        double w[3], ym[3];
        for (int k = 0; k < 3; ++k) ym[k] = x[k] - m[k];
        const double pr = ym[0] * e[0] + ym[1] * e[1] + ym[2] * e[2];
        for (int k = 0; k < 3; ++k) w[k] = ym[k] - pr * e[k];
        double nw = ls_norm(w, 3);
        if (nw == 0.0) {
          double a3[3] = {0, 0, 0};
          int km = 0;
          for (int k = 1; k < 3; ++k)
            if (std::fabs(e[k]) < std::fabs(e[km])) km = k;
          a3[km] = 1.0;
          const double ad = a3[0] * e[0] + a3[1] * e[1] + a3[2] * e[2];
          for (int k = 0; k < 3; ++k) w[k] = a3[k] - ad * e[k];
          nw = ls_norm(w, 3);
        }
        for (int k = 0; k < 3; ++k) pt[k] = m[k] + rho * w[k] / nw;
        consider(pt, i, j, -1);
        for (int k = 0; k < 3; ++k) pt[k] = m[k] - rho * w[k] / nw;
        consider(pt, i, j, -1);
      }
    }
  if (d == 3) {
    for (int i = 0; i < S; ++i)
      for (int j = i + 1; j < S; ++j)
        for (int l = j + 1; l < S; ++l) {
          if (hopeless(std::max(std::max(lb(i), lb(j)), lb(l)))) continue;
          // three-sphere intersection in the frame (ex, ey, ez) anchored at c_i
          const double *c1 = &cs[3 * i], *c2 = &cs[3 * j], *c3 = &cs[3 * l];
          double ex[3], ey[3], ez[3];
          for (int k = 0; k < 3; ++k) ex[k] = c2[k] - c1[k];
          const double dd = ls_norm(ex, 3);
          if (dd == 0.0) continue;
          for (int k = 0; k < 3; ++k) ex[k] /= dd;
          double c31[3];
          for (int k = 0; k < 3; ++k) c31[k] = c3[k] - c1[k];
          const double ii = ex[0] * c31[0] + ex[1] * c31[1] + ex[2] * c31[2];
          for (int k = 0; k < 3; ++k) ey[k] = c31[k] - ii * ex[k];
          const double ney = ls_norm(ey, 3);
          if (ney == 0.0) continue;
          for (int k = 0; k < 3; ++k) ey[k] /= ney;
          ez[0] = ex[1] * ey[2] - ex[2] * ey[1];
          ez[1] = ex[2] * ey[0] - ex[0] * ey[2];
          ez[2] = ex[0] * ey[1] - ex[1] * ey[0];
          const double jj = ey[0] * c31[0] + ey[1] * c31[1] + ey[2] * c31[2];
          const double r1 = rs[i], r2 = rs[j], r3 = rs[l];
          const double xx = (r1 * r1 - r2 * r2 + dd * dd) / (2.0 * dd);
          const double yy = (r1 * r1 - r3 * r3 + ii * ii + jj * jj) / (2.0 * jj) - (ii / jj) * xx;
          const double z2 = r1 * r1 - xx * xx - yy * yy;
          if (z2 <= 0.0) continue;
          const double zz = std::sqrt(z2);
          for (int sgn = 1; sgn >= -1; sgn -= 2) {
            for (int k = 0; k < 3; ++k) pt[k] = c1[k] + xx * ex[k] + yy * ey[k] + sgn * zz * ez[k];
            consider(pt, i, j, l);
          }
        }
  }
  if (!found)
    for (int k = 0; k < d; ++k) out[k] = std::numeric_limits<double>::quiet_NaN();
  return found;
}

// Closest point on {phi = 0} for the analytic kinds.
__host__ __device__ inline void ls_closest(const LsParams &L, const double *x, double *out) {
  const int d = L.dim;
  switch (L.kind) {
    case SBM_LS_SPHERE: {
      double u[3] = {0, 0, 0};
      for (int k = 0; k < d; ++k) u[k] = x[k] - L.centre[k];
      const double nu = ls_norm(u, d);
      for (int k = 0; k < d; ++k) out[k] = L.centre[k] + L.radius * u[k] / nu;
      return;
    }
    case SBM_LS_ELLIPSOID:
      ls_closest_ellipsoid(L.semi, L.centre, d, x, out);
      return;
    case SBM_LS_TORUS: {
      const double y0 = x[0] - L.centre[0], y1 = x[1] - L.centre[1], y2 = x[2] - L.centre[2];
      const double rho = std::sqrt(y0 * y0 + y1 * y1);
      const double core[3] = {L.R * y0 / rho, L.R * y1 / rho, 0.0};
      const double u[3] = {y0 - core[0], y1 - core[1], y2 - core[2]};
      const double nu = ls_norm(u, 3);
      for (int k = 0; k < 3; ++k) out[k] = L.centre[k] + core[k] + L.r * u[k] / nu;
      return;
    }
    case SBM_LS_HALFSPACE: {
      const double ph = ls_phi(L, x);
      for (int k = 0; k < d; ++k) out[k] = x[k] - ph * L.normal[k];
      return;
    }
    case SBM_LS_SPHERE_UNION:
      ls_closest_union(L.cs, L.rs, L.n_spheres, d, x, out);
      return;
  }
  for (int k = 0; k < d; ++k) out[k] = std::numeric_limits<double>::quiet_NaN();
}

}  // namespace sbm
