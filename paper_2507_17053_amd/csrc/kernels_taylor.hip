// Truncated-Taylor extension of the shifted boundary operator.
//
// Sec. 2.1 transfers the boundary value from the true boundary to the surrogate one by a Taylor
// expansion of the solution about the surrogate point x~ along the shift d = x - x~.  The
// default operator evaluates the face's cell polynomial at the shifted point, which is that
// expansion to all orders (it terminates for a polynomial).  This file provides the expansion
// kept to total order m:
//     E_m u(x~) = sum over |alpha| <= m of D^alpha u_K(x~) d^alpha / alpha!,
// in reference coordinates of the face's own cell (D_x^alpha d^alpha = D_xi^alpha delta^alpha,
// delta = xi - xi~).  m = 1 is the value-plus-gradient form; m >= d p is the full extension.
//
// Only the surrogate-face term changes: with an order set on a handle, the apply runs the cell
// term (and the DG interior faces) through the default kernels with the surrogate faces left
// out, then adds the faces' rows from sbm_face_taylor_kernel.  The diagonal is the default one
// plus a correction of its surrogate-face term.
#include <algorithm>

#include "sbm_internal.h"

namespace sbm {
namespace {

constexpr int kTaylorThreads = 256;

// FP64 1D data on [0,1] for the face kernels (kernel argument, by value).
struct TaylorTab {
  double z[kMaxN1], cinv[kMaxN1];  // GLL nodes, 1 / prod_{l != j} (z_j - z_l)
  double g[kMaxN1], w[kMaxN1];     // Gauss points and weights of the face rule
  double N[kMaxN1 * kMaxN1];       // N[q N1 + j] = l_j(g_q)
  double D0[kMaxN1], D1[kMaxN1];   // l'_j(0), l'_j(1)
};

TaylorTab make_taylor_tab(const Rules1D &r) {
  TaylorTab t{};
  const int n1 = r.p + 1;
  for (int j = 0; j < n1; ++j) {
    t.z[j] = r.z[j];
    t.cinv[j] = r.cinv[j];
    t.g[j] = r.g[j];
    t.w[j] = r.w[j];
    t.D0[j] = r.D0[j];
    t.D1[j] = r.D1[j];
  }
  for (int i = 0; i < n1 * n1; ++i) t.N[i] = r.N[i];
  return t;
}

// Taylor terms of the 1D basis function j about x0: c[k] = l_j^(k)(x0) dlt^k / k!, k = 0..p.
// They are the coefficients of t^k in l_j(x0 + t dlt) = cinv_j prod_{l != j} (x0 - z_l + t dlt),
// formed by multiplying out the p linear factors.
template <int N1>
__device__ __forceinline__ void taylor_terms(const TaylorTab &tt, int j, double x0, double dlt, double (&c)[N1]) {
  double poly[N1];
#pragma unroll
  for (int k = 0; k < N1; ++k) poly[k] = k == 0 ? 1.0 : 0.0;
#pragma unroll
  for (int l = 0; l < N1; ++l) {
    if (l == j) continue;
    const double a = x0 - tt.z[l];
#pragma unroll
    for (int k = N1 - 1; k >= 1; --k) poly[k] = a * poly[k] + dlt * poly[k - 1];
    poly[0] *= a;
  }
#pragma unroll
  for (int k = 0; k < N1; ++k) c[k] = tt.cinv[j] * poly[k];
}

// Reference coordinates of the surrogate point of face point q on face (a, s): xi~_a = s, the
// tangential axes (lower one fastest) at the Gauss points.
template <int D, int N1>
__device__ __forceinline__ void surrogate_point(const TaylorTab &tt, int a, int s, int q, double (&x0)[D]) {
  int qq = q;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    if (k == a) {
      x0[k] = (double)s;
    } else {
      x0[k] = tt.g[qq % N1];
      qq /= N1;
    }
  }
}

// Local DoF i of the face's cell -> global DoF (CG through the cell's x-run bases).
template <int D, int N1>
__device__ __forceinline__ int64_t local_dof(int disc_dg, const int32_t *__restrict__ runs, int cell, int i) {
  constexpr int NP = D == 3 ? N1 * N1 : N1, NB = NP * N1;
  return disc_dg ? (int64_t)cell * NB + i : (int64_t)runs[(int64_t)cell * NP + i / N1] + i % N1;
}

// One workgroup per surrogate face (Eq. (1) face terms with E replaced by E_m):
//   row_i = sum_q w_q [ -(dn u)(x~_q) psi_i(x~_q) - (dn psi_i)(x~_q) E_m u(x~_q)
//                       + sigma_Gam E_m u(x~_q) psi_i(x~_q) ],
// added into v.  Phase 1, one thread per face point: the Taylor terms of the three axes,
// E_m u by contracting the cell values axis by axis with the order sum kept <= m, the normal
// derivative at x~_q and the face weight.  Phase 2, one thread per local row.  FP64 inside.
template <typename T, int D, int N1>
__global__ __launch_bounds__(kTaylorThreads) void sbm_face_taylor_kernel(
    int n_faces, int disc_dg, int m, const int32_t *__restrict__ face_cell, const int32_t *__restrict__ face_code,
    const double *__restrict__ face_xi, const int32_t *__restrict__ runs, const T *__restrict__ u, T *__restrict__ v,
    TaylorTab tt, double h, double sigma) {
  constexpr int NP = D == 3 ? N1 * N1 : N1, NB = NP * N1, P = N1 - 1;
  __shared__ double su[NB];
  __shared__ double s_eu[NP], s_dnu[NP], s_om[NP];
  const int f = blockIdx.x;
  if (f >= n_faces) return;
  const int cell = face_cell[f], code = face_code[f], a = code >> 1, s = code & 1;
  const double sgn = s ? 1.0 : -1.0;
  for (int i = threadIdx.x; i < NB; i += blockDim.x) su[i] = (double)u[local_dof<D, N1>(disc_dg, runs, cell, i)];
  __syncthreads();
  for (int q = threadIdx.x; q < NP; q += blockDim.x) {
    double x0[D], dl[D];
    surrogate_point<D, N1>(tt, a, s, q, x0);
#pragma unroll
    for (int k = 0; k < D; ++k) dl[k] = face_xi[((int64_t)f * NP + q) * D + k] - x0[k];
    // c[k][i][j]: order-j Taylor term of basis function i along axis k
    double c[D][N1][N1];
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
      for (int i = 0; i < N1; ++i) taylor_terms<N1>(tt, i, x0[k], dl[k], c[k][i]);
    double eu = 0.0;
    if constexpr (D == 3) {
#pragma unroll
      for (int i2 = 0; i2 < N1; ++i2) {
        double b[N1][N1];  // b[j0][j1] = sum_{i0,i1} c0[i0][j0] c1[i1][j1] u[i0,i1,i2]
#pragma unroll
        for (int j0 = 0; j0 < N1; ++j0)
#pragma unroll
          for (int j1 = 0; j1 < N1; ++j1) b[j0][j1] = 0.0;
#pragma unroll
        for (int i1 = 0; i1 < N1; ++i1) {
          double r[N1];
#pragma unroll
          for (int j0 = 0; j0 < N1; ++j0) {
            double acc = 0.0;
#pragma unroll
            for (int i0 = 0; i0 < N1; ++i0) acc += c[0][i0][j0] * su[i0 + N1 * i1 + NP * i2];
            r[j0] = acc;
          }
#pragma unroll
          for (int j0 = 0; j0 < N1; ++j0)
#pragma unroll
            for (int j1 = 0; j1 < N1; ++j1) b[j0][j1] += c[1][i1][j1] * r[j0];
        }
#pragma unroll
        for (int j0 = 0; j0 < N1; ++j0)
#pragma unroll
          for (int j1 = 0; j1 < N1; ++j1)
#pragma unroll
            for (int j2 = 0; j2 < N1; ++j2)
              if (j0 + j1 + j2 <= m) eu += c[2][i2][j2] * b[j0][j1];
      }
    } else {
#pragma unroll
      for (int i1 = 0; i1 < N1; ++i1) {
#pragma unroll
        for (int j0 = 0; j0 < N1; ++j0) {
          double acc = 0.0;
#pragma unroll
          for (int i0 = 0; i0 < N1; ++i0) acc += c[0][i0][j0] * su[i0 + N1 * i1];
#pragma unroll
          for (int j1 = 0; j1 < N1; ++j1)
            if (j0 + j1 <= m) eu += c[1][i1][j1] * acc;
        }
      }
    }
    // normal derivative at x~_q: (2s-1)/h l'_{i_a}(s) times the tangential interpolation
    double dnu = 0.0;
    for (int i = 0; i < NB; ++i) {
      const int ik[3] = {i % N1, (i / N1) % N1, D == 3 ? i / (N1 * N1) : 0};
      double tang = 1.0;
      int qq = q;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        if (k == a) continue;
        tang *= tt.N[(qq % N1) * N1 + ik[k]];
        qq /= N1;
      }
      dnu += (s ? tt.D1[ik[a]] : tt.D0[ik[a]]) * tang * su[i];
    }
    double om = 1.0;
    int qq = q;
#pragma unroll
    for (int k = 0; k < D - 1; ++k) {
      om *= tt.w[qq % N1] * h;
      qq /= N1;
    }
    s_eu[q] = eu;
    s_dnu[q] = sgn / h * dnu;
    s_om[q] = om;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NB; i += blockDim.x) {
    const int ik[3] = {i % N1, (i / N1) % N1, D == 3 ? i / (N1 * N1) : 0};
    const double ds = s ? tt.D1[ik[a]] : tt.D0[ik[a]];
    const bool on_face = ik[a] == s * P;
    double row = 0.0;
    for (int q = 0; q < NP; ++q) {
      double tang = 1.0;
      int qq = q;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        if (k == a) continue;
        tang *= tt.N[(qq % N1) * N1 + ik[k]];
        qq /= N1;
      }
      const double vt = on_face ? tang : 0.0;  // psi_i(x~_q)
      const double dn = sgn / h * ds * tang;   // d psi_i / dn~ (x~_q)
      row += s_om[q] * (-s_dnu[q] * vt - dn * s_eu[q] + sigma * s_eu[q] * vt);
    }
    unsafeAtomicAdd(v + local_dof<D, N1>(disc_dg, runs, cell, i), (T)row);
  }
}

// Diagonal correction, one thread per (face, local DoF): the default diagonal holds the
// surrogate-face term with psi_i(xi_q) (full extension); add
//   sum_q w_q (E_m psi_i - psi_i(xi_q)) (sigma_Gam psi_i(x~_q) - dn psi_i(x~_q)).
template <typename T, int D, int N1>
__global__ __launch_bounds__(kTaylorThreads) void diag_taylor_kernel(
    int n_faces, int disc_dg, int m, const int32_t *__restrict__ face_cell, const int32_t *__restrict__ face_code,
    const double *__restrict__ face_xi, const int32_t *__restrict__ runs, T *__restrict__ diag, TaylorTab tt,
    double h, double sigma) {
  constexpr int NP = D == 3 ? N1 * N1 : N1, NB = NP * N1, P = N1 - 1;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= (int64_t)n_faces * NB) return;
  const int f = (int)(gid / NB), i = (int)(gid % NB);
  const int cell = face_cell[f], code = face_code[f], a = code >> 1, s = code & 1;
  const int ik[3] = {i % N1, (i / N1) % N1, D == 3 ? i / (N1 * N1) : 0};
  const double sgn = s ? 1.0 : -1.0, ds = s ? tt.D1[ik[a]] : tt.D0[ik[a]];
  double val = 0.0;
  for (int q = 0; q < NP; ++q) {
    double x0[D];
    surrogate_point<D, N1>(tt, a, s, q, x0);
    double c[D][N1];
    double full = 1.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double xq = face_xi[((int64_t)f * NP + q) * D + k];
      taylor_terms<N1>(tt, ik[k], x0[k], xq - x0[k], c[k]);
      // psi_i(xi_q) in product form, as the default diagonal forms it
      double l = tt.cinv[ik[k]];
#pragma unroll
      for (int j = 0; j < N1; ++j)
        if (j != ik[k]) l *= xq - tt.z[j];
      full *= l;
    }
    double em = 0.0;
#pragma unroll
    for (int j0 = 0; j0 < N1; ++j0)
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) {
        if constexpr (D == 3) {
#pragma unroll
          for (int j2 = 0; j2 < N1; ++j2)
            if (j0 + j1 + j2 <= m) em += c[0][j0] * c[1][j1] * c[2][j2];
        } else {
          if (j0 + j1 <= m) em += c[0][j0] * c[1][j1];
        }
      }
    double tang = 1.0, om = 1.0;
    int qq = q;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      if (k == a) continue;
      tang *= tt.N[(qq % N1) * N1 + ik[k]];
      om *= tt.w[qq % N1] * h;
      qq /= N1;
    }
    const double vt = (ik[a] == s * P) ? tang : 0.0;
    const double dn = sgn / h * ds * tang;
    val += om * (em - full) * (sigma * vt - dn);
  }
  unsafeAtomicAdd(diag + local_dof<D, N1>(disc_dg, runs, cell, i), (T)val);
}

template <typename T, int D, int N1>
hipError_t taylor_faces(const sbm_ctx *c, const T *u, T *v, hipStream_t s) {
  const int nf = (int)c->n_sbm;
  if (nf == 0) return hipSuccess;
  // one thread per local row in the second phase (at least one wavefront)
  constexpr int NB = (D == 3 ? N1 * N1 : N1) * N1;
  constexpr int NT = NB < 64 ? 64 : (NB > kTaylorThreads ? kTaylorThreads : (NB + 63) / 64 * 64);
  hipLaunchKernelGGL((sbm_face_taylor_kernel<T, D, N1>), dim3(nf), dim3(NT), 0, s, nf,
                     c->disc == SBM_DG, c->taylor_m, c->d_face_cell, c->d_face_code, c->d_face_xi, c->d_runs, u, v,
                     make_taylor_tab(c->rules), c->h, c->sigma_gamma);
  return hipGetLastError();
}

template <typename T, int D, int N1>
hipError_t taylor_diag(const sbm_ctx *c, T *diag, hipStream_t s) {
  constexpr int NB = (D == 3 ? N1 * N1 : N1) * N1;
  const int64_t nt = c->n_sbm * (int64_t)NB;
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL((diag_taylor_kernel<T, D, N1>), dim3((unsigned)((nt + kTaylorThreads - 1) / kTaylorThreads)),
                     dim3(kTaylorThreads), 0, s, (int)c->n_sbm, c->disc == SBM_DG, c->taylor_m, c->d_face_cell,
                     c->d_face_code, c->d_face_xi, c->d_runs, diag, make_taylor_tab(c->rules), c->h, c->sigma_gamma);
  return hipGetLastError();
}

template <typename T, int D>
hipError_t taylor_dispatch(const sbm_ctx *c, const T *u, T *v, T *diag, hipStream_t s) {
  switch (c->p) {
#define SBM_TAYLOR_CASE(P)                                                                   \
  case P:                                                                                    \
    return diag ? taylor_diag<T, D, P + 1>(c, diag, s) : taylor_faces<T, D, P + 1>(c, u, v, s);
    SBM_TAYLOR_CASE(1)
    SBM_TAYLOR_CASE(2)
    SBM_TAYLOR_CASE(3)
    SBM_TAYLOR_CASE(4)
    SBM_TAYLOR_CASE(5)
    SBM_TAYLOR_CASE(6)
    SBM_TAYLOR_CASE(7)
    SBM_TAYLOR_CASE(8)
#undef SBM_TAYLOR_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t taylor_run(const sbm_ctx *c, const void *u, void *v, void *diag, hipStream_t s) {
  return c->dim == 3 ? taylor_dispatch<T, 3>(c, (const T *)u, (T *)v, (T *)diag, s)
                     : taylor_dispatch<T, 2>(c, (const T *)u, (T *)v, (T *)diag, s);
}

}  // namespace

hipError_t launch_operator(const sbm_ctx *c, const void *u, void *v, int prec, int parts, hipStream_t s) {
  if (c->taylor_m < 0 || !(parts & SBM_PART_SBM_FACES)) return launch_apply(c, u, v, prec, parts, s);
  // the cell term (DG: with the interior faces) overwrites v; the surrogate faces add into it
  const int rest = parts & ~(SBM_PART_SBM_FACES | SBM_PART_REUSE_FACES);
  if (rest & SBM_PART_CELLS) {
    hipError_t e = launch_apply(c, u, v, prec, rest, s);
    if (e != hipSuccess) return e;
  }
  return prec == SBM_F64 ? taylor_run<double>(c, u, v, nullptr, s) : taylor_run<float>(c, u, v, nullptr, s);
}

hipError_t launch_operator_diagonal(const sbm_ctx *c, void *diag, int prec, hipStream_t s) {
  hipError_t e = launch_diagonal(c, diag, prec, s);
  if (e != hipSuccess || c->taylor_m < 0) return e;
  return prec == SBM_F64 ? taylor_run<double>(c, nullptr, nullptr, diag, s)
                         : taylor_run<float>(c, nullptr, nullptr, diag, s);
}

}  // namespace sbm
