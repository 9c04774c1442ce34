/*
 * Brute-force FP64 apply of the shifted-boundary Poisson operator, plain C + OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY: this is the oracle's timed CPU baseline.  It is built next to
 * the oracle and called only by the tests, the smoke check and the benchmark's
 * CPU-baseline leg.  It shares no code with the HIP library.
 *
 * It computes v = A u as the plain sum of local contributions, one quadrature point at
 * a time, without sum factorisation:
 *   - cell term: w_K = A_K u_K with the dense reference-cell matrix A_K (all active cells
 *     are translates of one cell, Sec. 3.4), formed by the Python oracle by quadrature;
 *   - surrogate (SBM) faces (Sec. 3.3, Alg. 3; weak form Eq. (1)): at each face Gauss
 *     point, E u = u_K(xi_q) at the shifted reference point and dn u at the surrogate
 *     point, both by summing all (p+1)^d basis functions; then
 *       w_i += w_q [ (sigma E u - dn u) psi_i(xi~_q) - E u dn psi_i(xi~_q) ];
 *   - SIPG interior faces (Sec. 3.2, Alg. 2), with [u] = u_K1 - u_K2,
 *     {dn u} = (dn u_K1 + dn u_K2)/2 and n pointing from K1 to K2:
 *       T = sigma_F [u] - {dn u};  K1: +T v, -[u]/2 dn v;  K2: -T v, -[u]/2 dn v.
 * Lagrange values use the product form on GLL nodes, so extrapolated points are safe.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXN1 12

static void lag_vals(int n1, const double *z, double x, double *out) {
  for (int j = 0; j < n1; ++j) {
    double v = 1.0;
    for (int m = 0; m < n1; ++m)
      if (m != j) v *= (x - z[m]) / (z[j] - z[m]);
    out[j] = v;
  }
}

static void lag_ders(int n1, const double *z, double x, double *out) {
  for (int j = 0; j < n1; ++j) {
    double s = 0.0;
    for (int k = 0; k < n1; ++k) {
      if (k == j) continue;
      double t = 1.0 / (z[j] - z[k]);
      for (int m = 0; m < n1; ++m)
        if (m != j && m != k) t *= (x - z[m]) / (z[j] - z[m]);
      s += t;
    }
    out[j] = s;
  }
}

/* psi_i(xi) for all local i, and optionally d psi_i / d xi_axis; lexicographic i. */
static void basis_at(int d, int n1, const double *z, const double *xi, int axis, double *val,
                     double *der) {
  double lv[3][MAXN1], ld[3][MAXN1];
  for (int k = 0; k < d; ++k) {
    lag_vals(n1, z, xi[k], lv[k]);
    if (der) lag_ders(n1, z, xi[k], ld[k]);
  }
  int nb = 1;
  for (int k = 0; k < d; ++k) nb *= n1;
  for (int i = 0; i < nb; ++i) {
    int ik[3] = {i % n1, (i / n1) % n1, (i / n1 / n1) % n1};
    double v = 1.0, g = 1.0;
    for (int k = 0; k < d; ++k) {
      v *= lv[k][ik[k]];
      if (der) g *= (k == axis) ? ld[k][ik[k]] : lv[k][ik[k]];
    }
    val[i] = v;
    if (der) der[i] = g;
  }
}

/* Face point q of face (axis, side): xi_axis = side, tangential Gauss points, lower
 * tangential axis fastest; returns the tangential weight product. */
static double face_point(int d, int n1, const double *g, const double *w, int axis, int side,
                         int q, double *xi) {
  double wt = 1.0;
  int t = 0, qq = q;
  for (int k = 0; k < d; ++k) {
    if (k == axis) {
      xi[k] = (double)side;
      continue;
    }
    int iq = qq % n1;
    qq /= n1;
    xi[k] = g[iq];
    wt *= w[iq];
    ++t;
  }
  return wt;
}

int oracle_apply(int d, int p, int64_t n_dofs, int64_t n_cells, const int64_t *cell_dofs,
                 const double *cell_matrix, int64_t n_sbm, const int64_t *sbm_cell,
                 const int32_t *sbm_axis, const int32_t *sbm_side, const double *sbm_xi,
                 int64_t n_int, const int64_t *int_k1, const int64_t *int_k2,
                 const int32_t *int_axis, const double *gll, const double *gauss_x,
                 const double *gauss_w, double h, double sigma_gamma, double sigma_f,
                 const double *u, double *v, int n_threads) {
  if (d < 2 || d > 3 || p < 1 || p + 1 > MAXN1) return 1;
  const int n1 = p + 1;
  int nb = 1, nq = 1;
  for (int k = 0; k < d; ++k) nb *= n1;
  for (int k = 0; k < d - 1; ++k) nq *= n1;
  const double hf = (d == 3) ? h * h : h; /* h^(d-1): face measure */
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
  memset(v, 0, sizeof(double) * (size_t)n_dofs);

  /* ---- cell term ---- */
  double *wc = (double *)malloc(sizeof(double) * (size_t)(n_cells > 0 ? n_cells : 1) * nb);
  if (!wc) return 2;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < n_cells; ++c) {
    double uk[MAXN1 * MAXN1 * MAXN1];
    const int64_t *dofs = cell_dofs + c * nb;
    for (int j = 0; j < nb; ++j) uk[j] = u[dofs[j]];
    for (int i = 0; i < nb; ++i) {
      double s = 0.0;
      const double *row = cell_matrix + (size_t)i * nb;
      for (int j = 0; j < nb; ++j) s += row[j] * uk[j];
      wc[c * nb + i] = s;
    }
  }
  for (int64_t c = 0; c < n_cells; ++c)
    for (int i = 0; i < nb; ++i) v[cell_dofs[c * nb + i]] += wc[c * nb + i];
  free(wc);

  /* ---- surrogate-boundary faces ---- */
  double *wf = (double *)malloc(sizeof(double) * (size_t)(n_sbm > 0 ? n_sbm : 1) * nb);
  if (!wf) return 2;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t f = 0; f < n_sbm; ++f) {
    double uk[MAXN1 * MAXN1 * MAXN1], vt[MAXN1 * MAXN1 * MAXN1], dt[MAXN1 * MAXN1 * MAXN1],
        vs[MAXN1 * MAXN1 * MAXN1];
    const int64_t *dofs = cell_dofs + sbm_cell[f] * nb;
    const int a = sbm_axis[f], s = sbm_side[f];
    const double sgn = 2.0 * s - 1.0;
    double *out = wf + f * nb;
    for (int j = 0; j < nb; ++j) {
      uk[j] = u[dofs[j]];
      out[j] = 0.0;
    }
    for (int q = 0; q < nq; ++q) {
      double xt[3];
      double om = face_point(d, n1, gauss_x, gauss_w, a, s, q, xt) * hf;
      basis_at(d, n1, gll, xt, a, vt, dt);
      basis_at(d, n1, gll, sbm_xi + ((size_t)f * nq + q) * d, -1, vs, NULL);
      double eu = 0.0, dn = 0.0;
      for (int j = 0; j < nb; ++j) {
        eu += vs[j] * uk[j];
        dn += dt[j] * uk[j];
      }
      dn *= sgn / h;
      const double iv = om * (sigma_gamma * eu - dn);
      const double ig = -om * eu * sgn / h;
      for (int i = 0; i < nb; ++i) out[i] += iv * vt[i] + ig * dt[i];
    }
  }
  for (int64_t f = 0; f < n_sbm; ++f) {
    const int64_t *dofs = cell_dofs + sbm_cell[f] * nb;
    for (int i = 0; i < nb; ++i) v[dofs[i]] += wf[f * nb + i];
  }
  free(wf);

  /* ---- SIPG interior faces ---- */
  double *wi = (double *)malloc(sizeof(double) * (size_t)(n_int > 0 ? n_int : 1) * 2 * nb);
  if (!wi) return 2;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t f = 0; f < n_int; ++f) {
    double u1[MAXN1 * MAXN1 * MAXN1], u2[MAXN1 * MAXN1 * MAXN1];
    double v1[MAXN1 * MAXN1 * MAXN1], d1[MAXN1 * MAXN1 * MAXN1];
    double v2[MAXN1 * MAXN1 * MAXN1], d2[MAXN1 * MAXN1 * MAXN1];
    const int64_t *dof1 = cell_dofs + int_k1[f] * nb, *dof2 = cell_dofs + int_k2[f] * nb;
    const int a = int_axis[f];
    double *o1 = wi + f * 2 * nb, *o2 = o1 + nb;
    for (int j = 0; j < nb; ++j) {
      u1[j] = u[dof1[j]];
      u2[j] = u[dof2[j]];
      o1[j] = o2[j] = 0.0;
    }
    for (int q = 0; q < nq; ++q) {
      double x1[3], x2[3];
      double om = face_point(d, n1, gauss_x, gauss_w, a, 1, q, x1) * hf;
      face_point(d, n1, gauss_x, gauss_w, a, 0, q, x2);
      basis_at(d, n1, gll, x1, a, v1, d1);
      basis_at(d, n1, gll, x2, a, v2, d2);
      double a1 = 0, a2 = 0, g1 = 0, g2 = 0;
      for (int j = 0; j < nb; ++j) {
        a1 += v1[j] * u1[j];
        a2 += v2[j] * u2[j];
        g1 += d1[j] * u1[j];
        g2 += d2[j] * u2[j];
      }
      const double jump = a1 - a2;
      const double avg = 0.5 * (g1 + g2) / h;
      const double T = sigma_f * jump - avg;
      for (int i = 0; i < nb; ++i) {
        o1[i] += om * (T * v1[i] - 0.5 * jump * d1[i] / h);
        o2[i] += om * (-T * v2[i] - 0.5 * jump * d2[i] / h);
      }
    }
  }
  for (int64_t f = 0; f < n_int; ++f) {
    const int64_t *dof1 = cell_dofs + int_k1[f] * nb, *dof2 = cell_dofs + int_k2[f] * nb;
    for (int i = 0; i < nb; ++i) {
      v[dof1[i]] += wi[f * 2 * nb + i];
      v[dof2[i]] += wi[f * 2 * nb + nb + i];
    }
  }
  free(wi);
  return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
