// Right-hand side, batched applies and (later) Krylov solvers.
#include <cmath>
#include <cstring>

#include "sbm_internal.h"

namespace sbm {

struct Workspace {
  int dummy = 0;
};

void free_workspace(sbm_ctx *c) {
  delete c->ws;
  c->ws = nullptr;
}

}  // namespace sbm

using namespace sbm;

extern "C" {

sbm_status sbm_rhs(sbm_handle h, const double *f_qp, const double *g_bp, double *b, void *stream) {
  if (!h || !f_qp || !b || (h->n_sbm > 0 && !g_bp)) {
    set_error("sbm_rhs: NULL argument");
    return SBM_EINVAL;
  }
  const int d = h->dim, n1 = h->n1, nb = h->nb, np = h->nq_face, P = h->p;
  const Rules1D &R = h->rules;
  std::vector<double> bh(h->n_dofs, 0.0);
  // psi_i(g_q) on the reference cell and the cell weights W_q h^d
  std::vector<double> psi((size_t)nb * nb), wq(nb);
  for (int q = 0; q < nb; ++q) {
    int qk[3] = {q % n1, (q / n1) % n1, q / (n1 * n1)};
    double w = 1.0;
    for (int m = 0; m < d; ++m) w *= R.w[qk[m]] * h->h;
    wq[q] = w;
    for (int i = 0; i < nb; ++i) {
      int ik[3] = {i % n1, (i / n1) % n1, i / (n1 * n1)};
      double v = 1.0;
      for (int m = 0; m < d; ++m) v *= R.N[qk[m] * n1 + ik[m]];
      psi[(size_t)q * nb + i] = v;
    }
  }
  auto dof_of = [&](int64_t r, int i) -> int64_t {
    return (h->disc == SBM_CG) ? (int64_t)h->runs[r * np + i / n1] + i % n1 : r * nb + i;
  };
  std::vector<double> loc(nb);
  for (int64_t r = 0; r < h->n_cells; ++r) {
    std::fill(loc.begin(), loc.end(), 0.0);
    for (int q = 0; q < nb; ++q) {
      const double fw = f_qp[r * nb + q] * wq[q];
      for (int i = 0; i < nb; ++i) loc[i] += psi[(size_t)q * nb + i] * fw;
    }
    for (int i = 0; i < nb; ++i) bh[dof_of(r, i)] += loc[i];
  }
  // surrogate faces: int sigma g psi_i - int (dpsi_i/dn~) g, g at the true-boundary points
  for (int64_t f = 0; f < h->n_sbm; ++f) {
    const int32_t r = h->faces[3 * f], a = h->faces[3 * f + 1], s = h->faces[3 * f + 2];
    const double sgn = s ? 1.0 : -1.0;
    const double *Ds = s ? R.D1.data() : R.D0.data();
    std::fill(loc.begin(), loc.end(), 0.0);
    for (int q = 0; q < np; ++q) {
      int qt[2] = {q % n1, q / n1};
      double om = 1.0;
      for (int t = 0; t < d - 1; ++t) om *= R.w[qt[t]] * h->h;
      const double g = g_bp[f * np + q];
      for (int i = 0; i < nb; ++i) {
        int ik[3] = {i % n1, (i / n1) % n1, i / (n1 * n1)};
        double tang = 1.0;
        int t = 0;
        for (int m = 0; m < d; ++m) {
          if (m == a) continue;
          tang *= R.N[qt[t] * n1 + ik[m]];
          ++t;
        }
        const double val = (ik[a] == s * P) ? tang : 0.0;
        const double dn = sgn / h->h * Ds[ik[a]] * tang;
        loc[i] += om * (h->sigma_gamma * g * val - g * dn);
      }
    }
    for (int i = 0; i < nb; ++i) bh[dof_of(r, i)] += loc[i];
  }
  SBM_HIP_CHECK(hipMemcpyAsync(b, bh.data(), bh.size() * sizeof(double), hipMemcpyHostToDevice,
                               (hipStream_t)stream));
  SBM_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
  return SBM_OK;
}

sbm_status sbm_apply_batch(int n, const sbm_handle *hs, const void *const *u, void *const *v, int prec,
                           void *stream) {
  if (n < 0 || (n > 0 && (!hs || !u || !v))) {
    set_error("sbm_apply_batch: bad arguments");
    return SBM_EINVAL;
  }
  for (int i = 0; i < n; ++i) {
    sbm_status st = sbm_apply(hs[i], u[i], v[i], prec, stream);
    if (st != SBM_OK) return st;
  }
  return SBM_OK;
}

sbm_status sbm_diagonal(sbm_handle h, void *diag, int prec, void *stream) {
  (void)h;
  (void)diag;
  (void)prec;
  (void)stream;
  set_error("sbm_diagonal: not available in this build");
  return SBM_EUNSUPPORTED;
}

sbm_status sbm_solve(sbm_handle h, const double *b, double *x, double rel_tol, int max_it, int mode,
                     int restart, int jacobi, void *stream, sbm_solve_info *info) {
  (void)h;
  (void)b;
  (void)x;
  (void)rel_tol;
  (void)max_it;
  (void)mode;
  (void)restart;
  (void)jacobi;
  (void)stream;
  (void)info;
  set_error("sbm_solve: not available in this build");
  return SBM_EUNSUPPORTED;
}

}  // extern "C"
