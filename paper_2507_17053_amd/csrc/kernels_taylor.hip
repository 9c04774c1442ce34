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
// Only the surrogate-face term changes: with an order set on a handle, sbm_face_taylor_kernel
// leaves each face's (Rv, Rg) per face node in the handle's face buffer, and the default cell
// kernels (brick kernel for CG, cell kernel for DG) then expand and merge them in face order,
// exactly as for the full extension.  The diagonal is the default one plus a correction of its
// surrogate-face term.
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

// Taylor terms of the 1D basis function j about x0: c[k] = l_j^(k)(x0) dlt^k / k!, k < JN
// (JN <= p+1 orders kept).  They are the coefficients of t^k in
// l_j(x0 + t dlt) = cinv_j prod_{l != j} (x0 - z_l + t dlt): the p linear factors (x0 - z_l) + s
// are multiplied out in s = t dlt (one multiply-add per coefficient and factor; coefficient k
// depends on coefficients <= k only, so dropping the higher ones is exact), and coefficient k is
// then scaled by cinv_j dlt^k.
template <int N1, int JN = N1>
__device__ __forceinline__ void taylor_terms(const TaylorTab &tt, int j, double x0, double dlt, double (&c)[JN]) {
  double poly[JN];
#pragma unroll
  for (int k = 0; k < JN; ++k) poly[k] = k == 0 ? 1.0 : 0.0;
#pragma unroll
  for (int l = 0; l < N1; ++l) {
    if (l == j) continue;
    const double a = x0 - tt.z[l];
#pragma unroll
    for (int k = JN - 1; k >= 1; --k) poly[k] = a * poly[k] + poly[k - 1];
    poly[0] *= a;
  }
  double scale = tt.cinv[j];
#pragma unroll
  for (int k = 0; k < JN; ++k) {
    c[k] = scale * poly[k];
    scale *= dlt;
  }
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

// Slabs of the cell that split a face point's evaluation of E_m u over threads: p+1 where
// (p+1)^d threads fit in a workgroup, else 1 (one thread takes every slab).
template <int D, int N1>
constexpr int taylor_slabs() {
  return (D == 3 ? N1 * N1 * N1 : N1 * N1) <= kTaylorThreads ? N1 : 1;
}

// One workgroup per surrogate face (Eq. (1) face terms with E replaced by E_m):
//   row_i = sum_q w_q [ -(dn u)(x~_q) psi_i(x~_q) - (dn psi_i)(x~_q) E_m u(x~_q)
//                       + sigma_Gam E_m u(x~_q) psi_i(x~_q) ],
// added into v.  Phase 1, thread (q, slab): the Taylor terms of face point q along the d axes,
// then its slab's share of E_m u (the cell values contracted axis by axis with the order sum
// kept <= m) and of the normal derivative at x~_q; the slab shares are added in slab order.
// Phase 2, one thread per face node: Rv = sum_q psi(x~_q) w_q (sigma E_m u - dn u) and
// Rg = -sum_q psi(x~_q) w_q E_m u (2s-1)/h over the tangential basis, stored per face node in
// fbuf (fbuf[f][0][t], fbuf[f][1][t]); the cell kernels add the face's rows (Rv on the face's
// own nodes plus Rg times the normal derivative of the row's 1D function) in a fixed order, as
// for the full extension.  FP64 inside; the 1D tables are staged in LDS.  JN: Taylor orders
// carried per axis (p+1, or 2 for a launch with m <= 1).
template <typename T, int D, int N1, int JN>
__global__ __launch_bounds__(kTaylorThreads) void sbm_face_taylor_kernel(
    int n_faces, int disc_dg, int m, const int32_t *__restrict__ face_cell, const int32_t *__restrict__ face_code,
    const double *__restrict__ face_xi, const int32_t *__restrict__ runs, const T *__restrict__ u,
    T *__restrict__ fbuf, TaylorTab tt, double h, double sigma) {
  constexpr int NP = D == 3 ? N1 * N1 : N1, NB = NP * N1, S = taylor_slabs<D, N1>();
  __shared__ double su[NB];
  __shared__ double sN[N1 * N1], sDs[N1], sw[N1];
  __shared__ double pe[S][NP], pd[S][NP];  // slab shares of E_m u and of the normal derivative
  __shared__ double sA[NP], sB[NP];
  const int f = blockIdx.x;
  if (f >= n_faces) return;
  const int cell = face_cell[f], code = face_code[f], a = code >> 1, s = code & 1;
  const double sgn = s ? 1.0 : -1.0;
  for (int i = threadIdx.x; i < NB; i += blockDim.x) su[i] = (double)u[local_dof<D, N1>(disc_dg, runs, cell, i)];
  for (int i = threadIdx.x; i < N1 * N1; i += blockDim.x) sN[i] = tt.N[i];
  if (threadIdx.x < N1) {
    sDs[threadIdx.x] = s ? tt.D1[threadIdx.x] : tt.D0[threadIdx.x];
    sw[threadIdx.x] = tt.w[threadIdx.x];
  }
  __syncthreads();
  // tangential axes of the face, lower one first (face point q = qb + N1 qc)
  const int tb = a == 0 ? 1 : 0;  // (the upper tangential axis is the remaining one)
  for (int t = threadIdx.x; t < NP * S; t += blockDim.x) {
    const int q = t % NP, slab = t / NP;
    const int qb = q % N1, qc = D == 3 ? q / N1 : 0;
    double x0[D], dl[D];
    surrogate_point<D, N1>(tt, a, s, q, x0);
#pragma unroll
    for (int k = 0; k < D; ++k) dl[k] = face_xi[((int64_t)f * NP + q) * D + k] - x0[k];
    // c[k][i][j]: order-j Taylor term of basis function i along axis k < d-1 (the last axis
    // is the slab axis: only the slab's own function is needed, cl below)
    double c[D - 1][N1][JN];
#pragma unroll
    for (int k = 0; k < D - 1; ++k)
#pragma unroll
      for (int i = 0; i < N1; ++i) taylor_terms<N1, JN>(tt, i, x0[k], dl[k], c[k][i]);
    // factor of local index i along axis k in the normal derivative at x~_q
    auto dfac = [&](int k, int i) {
      return k == a ? sDs[i] : sN[(k == tb ? qb : qc) * N1 + i];
    };
    double eu = 0.0, dn = 0.0;
    for (int il = slab; il < N1; il += S) {  // slab il: last local index (i2 in 3D, i1 in 2D)
      double cl[JN];
      taylor_terms<N1, JN>(tt, il, x0[D - 1], dl[D - 1], cl);
      if constexpr (D == 3) {
        double b[JN][JN];  // b[j0][j1] = sum_{i0,i1} c0[i0][j0] c1[i1][j1] u[i0,i1,il]
#pragma unroll
        for (int j0 = 0; j0 < JN; ++j0)
#pragma unroll
          for (int j1 = 0; j1 < JN; ++j1) b[j0][j1] = 0.0;
        const double f2 = dfac(2, il);
#pragma unroll
        for (int i1 = 0; i1 < N1; ++i1) {
          double r[JN];
          double g = 0.0;
          const double f1 = dfac(1, i1);
#pragma unroll
          for (int j0 = 0; j0 < JN; ++j0) r[j0] = 0.0;
#pragma unroll
          for (int i0 = 0; i0 < N1; ++i0) {
            const double uv = su[i0 + N1 * i1 + NP * il];
            g += dfac(0, i0) * uv;
#pragma unroll
            for (int j0 = 0; j0 < JN; ++j0) r[j0] += c[0][i0][j0] * uv;
          }
          dn += f2 * f1 * g;
#pragma unroll
          for (int j0 = 0; j0 < JN; ++j0)
#pragma unroll
            for (int j1 = 0; j1 < JN; ++j1) b[j0][j1] += c[1][i1][j1] * r[j0];
        }
        // sum over j0 + j1 + j2 <= m of cl[j2] b[j0][j1]: b summed along its anti-diagonals
        // (j0 + j1 = k) first, then each order j2 takes the diagonals k <= m - j2
        double bd[2 * JN - 1];
#pragma unroll
        for (int k = 0; k < 2 * JN - 1; ++k) bd[k] = 0.0;
#pragma unroll
        for (int j0 = 0; j0 < JN; ++j0)
#pragma unroll
          for (int j1 = 0; j1 < JN; ++j1) bd[j0 + j1] += b[j0][j1];
#pragma unroll
        for (int j2 = 0; j2 < JN; ++j2) {
          double t = 0.0;
#pragma unroll
          for (int k = 0; k < 2 * JN - 1; ++k)
            if (k + j2 <= m) t += bd[k];
          eu += cl[j2] * t;
        }
      } else {
        double g = 0.0;
        const double f1 = dfac(1, il);
#pragma unroll
        for (int j0 = 0; j0 < JN; ++j0) {
          double acc = 0.0;
#pragma unroll
          for (int i0 = 0; i0 < N1; ++i0) acc += c[0][i0][j0] * su[i0 + N1 * il];
#pragma unroll
          for (int j1 = 0; j1 < JN; ++j1)
            if (j0 + j1 <= m) eu += cl[j1] * acc;
        }
#pragma unroll
        for (int i0 = 0; i0 < N1; ++i0) g += dfac(0, i0) * su[i0 + N1 * il];
        dn += f1 * g;
      }
    }
    pe[slab][q] = eu;
    pd[slab][q] = dn;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NP; q += blockDim.x) {
    double eu = 0.0, dn = 0.0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
      eu += pe[k][q];
      dn += pd[k][q];
    }
    dn *= sgn / h;
    double om = sw[q % N1] * h;
    if constexpr (D == 3) om *= sw[q / N1] * h;
    sA[q] = om * (sigma * eu - dn);  // tested against psi(x~_q)
    sB[q] = -om * eu * sgn / h;      // tested against the normal derivative's 1D factor
  }
  __syncthreads();
  for (int t = threadIdx.x; t < NP; t += blockDim.x) {
    const int jb = t % N1, jc = D == 3 ? t / N1 : 0;
    double rv = 0.0, rg = 0.0;
    for (int q = 0; q < NP; ++q) {
      const double tang = sN[(q % N1) * N1 + jb] * (D == 3 ? sN[(q / N1) * N1 + jc] : 1.0);
      rv += tang * sA[q];
      rg += tang * sB[q];
    }
    fbuf[(int64_t)f * 2 * NP + t] = (T)rv;
    fbuf[(int64_t)f * 2 * NP + NP + t] = (T)rg;
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
hipError_t taylor_faces(const sbm_ctx *c, const T *u, T *fbuf, hipStream_t s) {
  const int nf = (int)c->n_sbm;
  if (nf == 0) return hipSuccess;
  // one thread per (face point, slab) in the first phase (at least one wavefront)
  constexpr int NW = (D == 3 ? N1 * N1 : N1) * taylor_slabs<D, N1>();
  constexpr int NT = NW < 64 ? 64 : (NW > kTaylorThreads ? kTaylorThreads : (NW + 63) / 64 * 64);
  // orders 0 and 1 only for m <= 1 (the first-order extension), all p+1 otherwise
  if (c->taylor_m <= 1)
    hipLaunchKernelGGL((sbm_face_taylor_kernel<T, D, N1, 2>), dim3(nf), dim3(NT), 0, s, nf, c->disc == SBM_DG,
                       c->taylor_m, c->d_face_cell, c->d_face_code, c->d_face_xi, c->d_runs, u, fbuf,
                       make_taylor_tab(c->rules), c->h, c->sigma_gamma);
  else
    hipLaunchKernelGGL((sbm_face_taylor_kernel<T, D, N1, N1>), dim3(nf), dim3(NT), 0, s, nf, c->disc == SBM_DG,
                       c->taylor_m, c->d_face_cell, c->d_face_code, c->d_face_xi, c->d_runs, u, fbuf,
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

hipError_t launch_operator(const sbm_ctx *c, const void *u, void *v, int prec, int parts, hipStream_t s,
                           const Scratch *scr) {
  if (c->taylor_m < 0 || !(parts & SBM_PART_SBM_FACES)) return launch_apply(c, u, v, prec, parts, s, scr);
  // the truncated surrogate-face term leaves (Rv, Rg) per face node in the face-result scratch;
  // the cell launches then take them as computed face results (SBM_PART_REUSE_FACES) and add the
  // rows in their fixed order
  void *fbuf = (scr && scr->fbuf) ? scr->fbuf : c->d_fbuf;
  if (c->n_sbm > 0) {
    const hipError_t e = prec == SBM_F64 ? taylor_run<double>(c, u, fbuf, nullptr, s)
                                         : taylor_run<float>(c, u, fbuf, nullptr, s);
    if (e != hipSuccess) return e;
  }
  return launch_apply(c, u, v, prec, parts | SBM_PART_REUSE_FACES, s, scr);
}

hipError_t launch_taylor_faces(const sbm_ctx *c, const void *u, void *fbuf, int prec, hipStream_t s) {
  if (c->n_sbm == 0) return hipSuccess;
  return prec == SBM_F64 ? taylor_run<double>(c, u, fbuf, nullptr, s) : taylor_run<float>(c, u, fbuf, nullptr, s);
}

hipError_t launch_operator_diagonal(const sbm_ctx *c, void *diag, int prec, hipStream_t s) {
  hipError_t e = launch_diagonal(c, diag, prec, s);
  if (e != hipSuccess || c->taylor_m < 0) return e;
  return prec == SBM_F64 ? taylor_run<double>(c, nullptr, nullptr, diag, s)
                         : taylor_run<float>(c, nullptr, nullptr, diag, s);
}

}  // namespace sbm
