// Matrix-free SBM operator kernels for gfx950 (CDNA4, wave64).
//
//   brick_kernel    CG: one workgroup per brick of BX x BY x BZ background cells.  The
//                   brick's active cells (Alg. 1) are evaluated into an LDS copy of the
//                   brick's DoF lattice (a brick whose cells are all active by 1D line
//                   sweeps over the whole lattice, others cell by cell), then its
//                   surrogate-boundary faces (Alg. 3); points strictly inside the brick are
//                   then stored to v directly, points on the brick's boundary (shared with
//                   neighbouring bricks) go to halo slots that halo_reduce_kernel sums.
//   sbm_face_cg_kernel  CG surrogate-boundary faces (Alg. 3), before the bricks: (Rv, Rg)
//                   per face node, which the brick holding the face's cell expands and merges.
//   sbm_face_kernel DG surrogate-boundary faces (Alg. 3): (Rv, Rg) per face node.
//   dg_cell_kernel  DG: Laplace cell term plus the SIPG terms of the cell's interior faces,
//                   evaluated cell by cell (Alg. 2 split per side), plus the rows of the
//                   cell's surrogate faces; every cell writes only its own block.
//
// Every sum (cells into the brick lattice, face rows, brick-boundary planes, DG face rows) is
// taken in an order fixed by the setup, with no atomics: applies are bitwise reproducible.
//
// Work layout: an "entity" (cell or face) is handled by NP = (p+1)^(d-1) consecutive threads,
// EPB entities at a time per workgroup.  Thread t of an entity owns one pencil of p+1
// values along a coordinate axis; the (p+1)^d tile of the cell lives in LDS.  Within a
// cell, the p+1 DoFs along the first axis (an "x-run") are consecutive in both
// numberings, so gathers read p+1 consecutive entries from a per-run base index.
//
// Cell term in Kronecker-sum form: all active cells are translates of one reference cell
// with Jacobian h I (Sec. 3.4), so the Gauss-point loop of Alg. 1 is a fixed diagonal
// scaling and evaluate / quadrature / integrate collapse per axis into the 1D matrices
//   M_ij = sum_q w_q l_i(g_q) l_j(g_q),   K_ij = sum_q w_q l'_i(g_q) l'_j(g_q)
// (exact with p+1 Gauss points), A_K = h^(d-2) sum_k M x .. K(axis k) .. x M.  In 3D this
// is 7 one-dimensional sweeps instead of the 12 of the gradient form.
#include <algorithm>
#include <climits>
#include <cstring>

#include "sbm_internal.h"

namespace sbm {
namespace {

template <int D, int N1>
struct Shape {
  static constexpr int NP = (D == 3) ? N1 * N1 : N1;
  static constexpr int NB = NP * N1;
};

// Entities per workgroup: fill up to 256 threads, keep the static LDS below ~60 KB.
template <typename T, int D, int N1, int NBUF, int EXTRA>
constexpr int epb() {
  constexpr int NP = Shape<D, N1>::NP, NB = Shape<D, N1>::NB;
  int e = 256 / NP;
  if (e < 1) e = 1;
  while (e > 1 && (e * NBUF * NB + 4 * e * NP + EXTRA) * (int)sizeof(T) > 60000) --e;
  return e;
}

// Entities per workgroup when there are few entities: one wavefront (at least one entity),
// so that small operators still spread over every CU.
template <typename T, int D, int N1, int NBUF>
constexpr int epb_one_wave() {
  constexpr int NP = Shape<D, N1>::NP, E = 64 / NP, F = epb<T, D, N1, NBUF, 0>();
  return E < 1 ? 1 : (E > F ? F : E);
}

// Workgroups that fill the device twice (two per compute unit).
inline int two_per_cu() {
  static const int n = [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                hipSuccess)
      return 512;
    return 2 * cus;
  }();
  return n;
}

// Brick of background cells per CG workgroup, chosen per degree so that the LDS lattice
// ((BX p + 1)(BY p + 1)(BZ p + 1) values) stays near 20 KB in FP64.
template <int D, int P>
struct BrickDims {
  // 3D: p=1 8x8x8, p=2 8x4x4, p=3 4x4x4, p=4,5 4x2x2, p=6 2x2x1, p=7 2x2x2, p=8 2x2x1 (at
  // p=4, 4x2x2 measured faster than 4x4x2, whose LDS allowed 3 workgroups per CU, and than
  // 2x2x2; at p=6, 2x2x1 faster than 2x2x2 on a 48^3 mesh, which has too few 2x2x2 bricks to
  // fill the device)
  // 2D: 8x8 up to p=2, 4x4 up to p=7, 3x3 for p=8 (a lattice row must fit 32 points)
  static constexpr int BX = (D == 2) ? (P <= 2 ? 8 : (P <= 7 ? 4 : 3))
                                     : (P <= 2 ? 8 : (P <= 5 ? 4 : 2));
  static constexpr int BY = (D == 2) ? BX : (P == 1 ? 8 : (P <= 3 ? 4 : 2));
  static constexpr int BZ = (D == 2) ? 1 : (P == 1 ? 8 : (P <= 3 ? 4 : (P <= 5 || P == 7 ? 2 : 1)));
};

// XCD-aware block order: the dispatcher hands block b to XCD (b mod 8), so give every XCD
// one contiguous range of logical blocks; neighbouring cells then share that XCD's L2.
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int x = b & 7, k = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return (x < rem) ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }

template <int N1>
__device__ __forceinline__ void lagrange_at(const double (&z)[N1], const double (&cinv)[N1], double x,
                                            double (&out)[N1]) {
  // l_j(x) = cinv_j prod_{m != j} (x - z_m), product form (stable when extrapolating)
  double dlt[N1], pre[N1], suf[N1];
#pragma unroll
  for (int m = 0; m < N1; ++m) dlt[m] = x - z[m];
  pre[0] = 1.0;
#pragma unroll
  for (int m = 1; m < N1; ++m) pre[m] = pre[m - 1] * dlt[m - 1];
  suf[N1 - 1] = 1.0;
#pragma unroll
  for (int m = N1 - 2; m >= 0; --m) suf[m] = suf[m + 1] * dlt[m + 1];
#pragma unroll
  for (int j = 0; j < N1; ++j) out[j] = cinv[j] * pre[j] * suf[j];
}

// ------------------------------------------------------------------------------------
// Cell term for one entity.  x: thread t's input pencil along the last axis (3D: t =
// i0 + N1 i1 holds u(i0, i1, k), k = 0..p; 2D: t = i0 holds u(i0, k)).  Returns in out
// the p+1 outputs of x-run t (3D: t = i1 + N1 i2; 2D: t = i1).  A, B: this entity's
// two (p+1)^d LDS tiles.  Contains barriers: every thread of the block must call it.
// ------------------------------------------------------------------------------------
// Even/odd pieces of a pencil: e_k = x_k + x_{p-k}, o_k = x_k - x_{p-k} (k < p+1 div 2),
// plus the middle value when p+1 is odd.
template <typename T, int N1>
struct EvenOdd {
  static constexpr int HC = (N1 + 1) / 2, HF = N1 / 2;
  T e[HC], o[HF > 0 ? HF : 1];
  __device__ __forceinline__ explicit EvenOdd(const T (&x)[N1]) {
#pragma unroll
    for (int k = 0; k < HF; ++k) {
      e[k] = x[k] + x[N1 - 1 - k];
      o[k] = x[k] - x[N1 - 1 - k];
    }
    if constexpr (N1 % 2 == 1) e[HF] = x[HF];
  }
};

// ye += E e, yo += O o for one centrosymmetric matrix given by its even/odd parts.
template <typename T, int N1>
__device__ __forceinline__ void eo_acc(const T *E, const T *O, const EvenOdd<T, N1> &v, T (&ye)[(N1 + 1) / 2],
                                       T (&yo)[N1 / 2 > 0 ? N1 / 2 : 1]) {
  constexpr int HC = (N1 + 1) / 2, HF = N1 / 2;
#pragma unroll
  for (int i = 0; i < HC; ++i)
#pragma unroll
    for (int k = 0; k < HC; ++k) ye[i] += E[i * HC + k] * v.e[k];
#pragma unroll
  for (int i = 0; i < HF; ++i)
#pragma unroll
    for (int k = 0; k < HF; ++k) yo[i] += O[i * HF + k] * v.o[k];
}

// y_i = ye_i + yo_i, y_{p-i} = ye_i - yo_i (and the middle row), times s.
template <typename T, int N1>
__device__ __forceinline__ void eo_combine(const T (&ye)[(N1 + 1) / 2], const T (&yo)[N1 / 2 > 0 ? N1 / 2 : 1],
                                           T s, T (&y)[N1]) {
  constexpr int HF = N1 / 2;
#pragma unroll
  for (int i = 0; i < HF; ++i) {
    y[i] = s * (ye[i] + yo[i]);
    y[N1 - 1 - i] = s * (ye[i] - yo[i]);
  }
  if constexpr (N1 % 2 == 1) y[HF] = s * ye[HF];
}

template <typename T, int N1>
struct EOAcc {
  T ye[(N1 + 1) / 2], yo[N1 / 2 > 0 ? N1 / 2 : 1];
  __device__ __forceinline__ EOAcc() {
#pragma unroll
    for (int i = 0; i < (N1 + 1) / 2; ++i) ye[i] = T(0);
#pragma unroll
    for (int i = 0; i < (N1 / 2 > 0 ? N1 / 2 : 1); ++i) yo[i] = T(0);
  }
};

template <typename T, int D, int N1>
__device__ __forceinline__ void kron_cell(const KTab<T, N1> &tab, int t, const T (&x)[N1], T *A, T *B, T scale,
                                          T (&out)[N1], bool on = true, bool work = true) {
  // on = false: compute but store nothing; work = false: only take part in the barriers (out
  // is left as it was)
  constexpr int NP = Shape<D, N1>::NP;
  if (work) {
    // last axis: a = M x, b = K x
    const EvenOdd<T, N1> ex(x);
    EOAcc<T, N1> ya, yb;
    eo_acc<T, N1>(tab.EM, tab.OM, ex, ya.ye, ya.yo);
    eo_acc<T, N1>(tab.EK, tab.OK, ex, yb.ye, yb.yo);
    T a[N1], b[N1];
    eo_combine<T, N1>(ya.ye, ya.yo, T(1), a);
    eo_combine<T, N1>(yb.ye, yb.yo, T(1), b);
    if (on) {
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        A[t + NP * i] = a[i];
        B[t + NP * i] = b[i];
      }
    }
  }
  __syncthreads();
  if constexpr (D == 3) {
    // pencils along axis 1; c = M a, e = K a + M b
    const int ix = t % N1, iz = t / N1;
    T a[N1], b[N1];
    if (work) {
#pragma unroll
      for (int j = 0; j < N1; ++j) {
        a[j] = A[ix + N1 * j + NP * iz];
        b[j] = B[ix + N1 * j + NP * iz];
      }
    }
    __syncthreads();
    if (work) {
      const EvenOdd<T, N1> ea(a), eb(b);
      EOAcc<T, N1> yc, ye;
      eo_acc<T, N1>(tab.EM, tab.OM, ea, yc.ye, yc.yo);
      eo_acc<T, N1>(tab.EK, tab.OK, ea, ye.ye, ye.yo);
      eo_acc<T, N1>(tab.EM, tab.OM, eb, ye.ye, ye.yo);
      T c[N1], e[N1];
      eo_combine<T, N1>(yc.ye, yc.yo, T(1), c);
      eo_combine<T, N1>(ye.ye, ye.yo, T(1), e);
      if (on) {
#pragma unroll
        for (int i = 0; i < N1; ++i) {
          A[ix + N1 * i + NP * iz] = c[i];
          B[ix + N1 * i + NP * iz] = e[i];
        }
      }
    }
    __syncthreads();
  }
  if (work) {
    // pencils along axis 0 (thread t = run index); out = K c + M e
    T c[N1], e[N1];
#pragma unroll
    for (int j = 0; j < N1; ++j) {
      c[j] = A[j + N1 * t];
      e[j] = B[j + N1 * t];
    }
    const EvenOdd<T, N1> ec(c), ee(e);
    EOAcc<T, N1> yo;
    eo_acc<T, N1>(tab.EK, tab.OK, ec, yo.ye, yo.yo);
    eo_acc<T, N1>(tab.EM, tab.OM, ee, yo.ye, yo.yo);
    eo_combine<T, N1>(yo.ye, yo.yo, scale, out);
  }
}

// Thread t's input pencil (see kron_cell) gathered through the x-run bases of a CG cell
// (cell_runs: the cell's (p+1)^(d-1) run bases, in LDS or in global memory).
template <typename T, int D, int N1>
__device__ __forceinline__ void gather_pencil(const int32_t *cell_runs, const T *__restrict__ u, int t, bool act,
                                              T (&x)[N1]) {
  const int i0 = (D == 3) ? t % N1 : t;
  const int r0 = (D == 3) ? t / N1 : 0;
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    const int run = (D == 3) ? r0 + N1 * k : k;
    x[k] = act ? u[cell_runs[run] + i0] : T(0);
  }
}

// ------------------------------------------------------------------------------------
// Face helpers (3D: tangential axes b < c; 2D: one tangential axis b)
// ------------------------------------------------------------------------------------
template <int D, int N1>
struct FaceAxes {
  int a, s, Sa, Sb, Sc;
  __device__ __forceinline__ FaceAxes(int code) {
    a = code >> 1;
    s = code & 1;
    Sa = (a == 0) ? 1 : (a == 1 ? N1 : N1 * N1);
    if (D == 3) {
      Sb = (a == 0) ? N1 : 1;        // lower tangential axis
      Sc = (a == 2) ? N1 : N1 * N1;  // upper tangential axis
    } else {
      Sb = (a == 0) ? N1 : 1;
      Sc = 0;
    }
  }
};

// Gauss -> GLL transposed interpolation of two face arrays f3, f4 (Gauss-point order
// qb + N1 qc), results at face node t = jb + N1 jc.  Uses f1, f2 as scratch.
template <typename T, int D, int N1>
__device__ __forceinline__ void face_integrate(const KTab<T, N1> &tab, int t, T *f1, T *f2, const T *f3,
                                               const T *f4, T &Rv, T &Rg) {
  if constexpr (D == 3) {
    const int qb = t % N1, jc = t / N1;
    T r1 = 0, r2 = 0;
#pragma unroll
    for (int qc = 0; qc < N1; ++qc) {
      r1 += tab.N[qc * N1 + jc] * f3[qb + N1 * qc];
      r2 += tab.N[qc * N1 + jc] * f4[qb + N1 * qc];
    }
    f1[t] = r1;
    f2[t] = r2;
    __syncthreads();
    const int jb = t % N1;
    T a1 = 0, a2 = 0;
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      a1 += tab.N[q * N1 + jb] * f1[q + N1 * jc];
      a2 += tab.N[q * N1 + jb] * f2[q + N1 * jc];
    }
    Rv = a1;
    Rg = a2;
  } else {
    T a1 = 0, a2 = 0;
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      a1 += tab.N[q * N1 + t] * f3[q];
      a2 += tab.N[q * N1 + t] * f4[q];
    }
    Rv = a1;
    Rg = a2;
  }
}

// GLL -> Gauss interpolation on the face of two node arrays f1, f2 (node order jb + N1 jc);
// returns the values at Gauss point t = qb + N1 qc.  Uses f3, f4 as scratch.
template <typename T, int D, int N1>
__device__ __forceinline__ void face_interpolate(const KTab<T, N1> &tab, int t, const T *f1, const T *f2,
                                                 T *f3, T *f4, T &o1, T &o2) {
  if constexpr (D == 3) {
    const int qb = t % N1, jc = t / N1;
    T r1 = 0, r2 = 0;
#pragma unroll
    for (int jb = 0; jb < N1; ++jb) {
      r1 += tab.N[qb * N1 + jb] * f1[jb + N1 * jc];
      r2 += tab.N[qb * N1 + jb] * f2[jb + N1 * jc];
    }
    f3[t] = r1;
    f4[t] = r2;
    __syncthreads();
    const int qc = t / N1;
    T a1 = 0, a2 = 0;
#pragma unroll
    for (int j = 0; j < N1; ++j) {
      a1 += tab.N[qc * N1 + j] * f3[qb + N1 * j];
      a2 += tab.N[qc * N1 + j] * f4[qb + N1 * j];
    }
    o1 = a1;
    o2 = a2;
  } else {
    T a1 = 0, a2 = 0;
#pragma unroll
    for (int j = 0; j < N1; ++j) {
      a1 += tab.N[t * N1 + j] * f1[j];
      a2 += tab.N[t * N1 + j] * f2[j];
    }
    o1 = a1;
    o2 = a2;
  }
}

// ------------------------------------------------------------------------------------
// One surrogate-boundary face (Alg. 3).  su: u_K in LDS (lexicographic), already synced.
// Returns Rv, Rg at this thread's face node t (face_row turns them into the (p+1)^d local
// rows).  xp: the shifted reference point of face Gauss point t, used only when act.
// f1..f4: NP values each of scratch.  Contains barriers.
//   dn u   = (2s-1)/h d/dxi_a u at the face Gauss points (sum factorisation),
//   E u    = u_K(xi_q), point evaluation with (p+1)^d terms per point,
//   tested:  w_q (sigma E u - dn u) against v, -w_q E u against dn v.
// ------------------------------------------------------------------------------------
template <typename T, int D, int N1>
__device__ __forceinline__ void sbm_face_eval(const KTab<T, N1> &tab, const KScal &sc, int t, bool act,
                                              const FaceAxes<D, N1> &fa, const double (&xp)[D], const T *su,
                                              T *f1, T *f2, T *f3, T *f4, T &Rv, T &Rg) {
  constexpr int NP = Shape<D, N1>::NP;
  const T h = T(sc.h), sig = T(sc.sigma_gamma);
  const T sh = (fa.s ? T(1) : T(-1)) / h;  // normal sign over h
  const int jb = (D == 3) ? t % N1 : t, jc = (D == 3) ? t / N1 : 0;
  const int node_off = jb * fa.Sb + jc * fa.Sc;
  {
    T g = 0;
#pragma unroll
    for (int ia = 0; ia < N1; ++ia) g += (fa.s ? tab.D1[ia] : tab.D0[ia]) * su[ia * fa.Sa + node_off];
    f1[t] = g;
    f2[t] = g;
  }
  __syncthreads();
  T dn, dn2;
  face_interpolate<T, D, N1>(tab, t, f1, f2, f3, f4, dn, dn2);
  dn *= sh;

  T eu = 0, om = 0;
  if (act) {
    double l[D][N1];
#pragma unroll
    for (int k = 0; k < D; ++k) lagrange_at<N1>(tab.z, tab.cinv, xp[k], l[k]);
    T l0[N1], l1[N1];
#pragma unroll
    for (int j = 0; j < N1; ++j) {
      l0[j] = T(l[0][j]);
      l1[j] = T(l[1][j]);
    }
    if constexpr (D == 3) {
#pragma unroll
      for (int i2 = 0; i2 < N1; ++i2) {
        T s1 = 0;
#pragma unroll
        for (int i1 = 0; i1 < N1; ++i1) {
          T s0 = 0;
#pragma unroll
          for (int i0 = 0; i0 < N1; ++i0) s0 += l0[i0] * su[i0 + N1 * i1 + NP * i2];
          s1 += l1[i1] * s0;
        }
        eu += T(l[2][i2]) * s1;
      }
      om = h * h * tab.w[t % N1] * tab.w[t / N1];
    } else {
#pragma unroll
      for (int i1 = 0; i1 < N1; ++i1) {
        T s0 = 0;
#pragma unroll
        for (int i0 = 0; i0 < N1; ++i0) s0 += l0[i0] * su[i0 + N1 * i1];
        eu += l1[i1] * s0;
      }
      om = h * tab.w[t];
    }
  }
  __syncthreads();  // f3/f4 reads of face_interpolate are done
  f3[t] = om * (sig * eu - dn);  // tested against v
  f4[t] = -om * eu * sh;         // tested against the reference derivative along a
  __syncthreads();
  face_integrate<T, D, N1>(tab, t, f1, f2, f3, f4, Rv, Rg);
}

// The face's result for the local row at position ia along the face normal, at this
// thread's face node: Rv on the face itself (ia = s p), plus Rg times the normal derivative
// of the 1D basis function ia at the face.
template <typename T, int D, int N1>
__device__ __forceinline__ T face_row(const KTab<T, N1> &tab, const FaceAxes<D, N1> &fa, int ia, T Rv, T Rg) {
  return ((ia == fa.s * (N1 - 1)) ? Rv : T(0)) + (fa.s ? tab.D1[ia] : tab.D0[ia]) * Rg;
}

// Brick description handed to the CG kernel.
struct BrickArgs {
  const int32_t *cell_off;   // n_bricks + 1
  const int32_t *runs;       // run bases of the active cells ((p+1)^(d-1) each), grouped by brick
  const int32_t *cell_loc;   // lattice offset of each cell's corner inside its brick
  // surrogate faces, numbered in brick order (a brick's faces are face_off[b] .. face_off[b+1])
  const int32_t *face_off;   // n_bricks + 1
  const int32_t *face_loc;   // lattice offset of each face's cell inside its brick
  const int32_t *face_code;  // per face: 2 axis + side
  const int32_t *row_base;   // n_bricks x rows: DoF id of the first globally present point
  const uint32_t *row_gmask; // bit x: lattice point x of the row is a DoF
  const uint32_t *row_bmask; // bit x: ... and is touched by an active cell of this brick
  const int32_t *row_hbase;  // first halo slot of the row's brick-boundary points
};

// One operator of a batch of applies (see the batched kernels after apply_impl): its arrays,
// vectors, scalars and its first workgroup in each stage's launch.
struct BatchItem {
  BrickArgs br;  // CG bricks
  const int32_t *face_code, *face_runs, *face_cell, *nbr, *halo_dof;
  const uint8_t *halo_mask;
  const double *face_xi;
  const void *u;
  void *v, *fbuf, *halo;
  KScal sc;
  int nf, nc, nh;
  int blk0[3];  // first workgroup of the item in each stage's launch
};

// ------------------------------------------------------------------------------------
// CG brick kernel
// ------------------------------------------------------------------------------------
// Geometry of the CG brick kernel for (D, P): lattice extents, block size (enough threads
// for the longest set of lattice lines, at most 256 so that several workgroups share a CU),
// cells per batch on the per-cell path, and the LDS size (the larger of the two paths,
// which share one buffer).
template <typename T, int D, int N1>
struct BrickCfg {
  static constexpr int P = N1 - 1, NP = Shape<D, N1>::NP, NB = Shape<D, N1>::NB;
  static constexpr int BX = BrickDims<D, P>::BX, BY = BrickDims<D, P>::BY, BZ = BrickDims<D, P>::BZ;
  static constexpr int LX = BX * P + 1, LY = BY * P + 1, LZ = (D == 3) ? BZ * P + 1 : 1;
  static constexpr int NL = LX * LY * LZ, NROWS = LY * LZ;
  static constexpr int LINES = (D == 3) ? ((LX * LY > LX * LZ ? LX * LY : LX * LZ) > LY * LZ
                                               ? (LX * LY > LX * LZ ? LX * LY : LX * LZ)
                                               : LY * LZ)
                                        : (LX > LY ? LX : LY);
  static constexpr int NT0 = ((LINES + 63) / 64) * 64;
  // (3D p=4: 192 threads measured faster than 256 and 320 in both precisions: FP32 brick kernel
  // 21.1 / 21.9 / 25.9 us, FP64 28.5 / 29.8 / 36.0 us)
  static constexpr int NT = NT0 < 128 ? 128 : (NT0 > 256 ? 256 : NT0);
  static constexpr int EPB0 = NT / NP;
  static constexpr int EPB = EPB0 < 1 ? 1 : EPB0;   // faces per batch (and thread groups with NP threads)
  static constexpr int NG = (NT + NP - 1) / NP;      // thread groups (the last may be partial)
  // cells per batch of the per-cell path: each has two tiles of NB values; the groups beyond
  // only take part in the barriers.  At 3D p=4 the batch is cut to 4 cells so that the tiles
  // and the staged run bases fit in the sweep arrays' space.
  static constexpr int EPC0 = (D == 3 && P == 4) ? 4 : EPB;  // (FP32 too: 20.3 against 20.9 us)
  static constexpr int EPC = EPC0 < EPB ? EPC0 : EPB;
  static constexpr int NTILE = EPC;  // tile pairs (the other groups store nothing)
  // LDS in elements of T: the lattice accumulator (the cell and face rows are summed into it in
  // the apply's precision, in a fixed order), then either the second sweep array of the full
  // path (the first one is the accumulator itself) or the per-cell tiles.
  static constexpr int MAXC = BX * BY * BZ;  // cells of a full brick
  static constexpr int TAIL_SWEEP = NL;
  // per-cell path: the tiles, then (where they are small: p >= 4 in 3D) the brick's run
  // bases and cell offsets (int32), staged in one round trip instead of read per batch
  static constexpr int RUNS_B = (MAXC * NP + MAXC) * 4;
  static constexpr bool STAGE_RUNS = RUNS_B <= 2560;
  static constexpr int RUNS_T = STAGE_RUNS ? (RUNS_B + (int)sizeof(T) - 1) / (int)sizeof(T) : 0;
  // ... then the partial brick's row masks (a full brick's are all ones)
  static constexpr int MASK_T = (2 * NROWS * 4 + (int)sizeof(T) - 1) / (int)sizeof(T);
  static constexpr int TAIL_CELLS = 2 * NTILE * NB + RUNS_T + MASK_T;
  static constexpr int SMEM = NL + (TAIL_SWEEP > TAIL_CELLS ? TAIL_SWEEP : TAIL_CELLS);
};

// Lattice-line segments of a full brick.  A line of B cells has B p + 1 nodes; the segment of
// cell j is nodes j p .. j p + p, and neighbouring segments share one node.  One lane per
// segment, the B lanes of a line side by side in a group of G = pow2 >= B lanes of one
// wavefront: each lane forms its cell's p + 1 outputs, takes the previous lane's last output
// for its first node (the sum of both cells' rows there), and stores nodes j p .. j p + p - 1
// (the last lane also node B p).  Every input is read before any lane of the line stores.
template <int G, typename T>
__device__ __forceinline__ T from_prev_lane(T y, int j) {
  if constexpr (G == 1) {
    return T(0);
  } else {
    const T w = __shfl_up(y, 1, G);
    return j > 0 ? w : T(0);
  }
}

template <int B>
struct LaneGroup {
  static constexpr int G = B <= 1 ? 1 : (B <= 2 ? 2 : (B <= 4 ? 4 : (B <= 8 ? 8 : 16)));
  static_assert(B <= 16 && 64 % G == 0, "segment groups must tile a wavefront");
};

template <typename T, int D, int N1>
__device__ __forceinline__ void brick_body(const int blk, BrickArgs br, const T *__restrict__ fbuf,
                                           const T *__restrict__ u, T *__restrict__ v, T *__restrict__ halo,
                                           int nhalo, KTab<T, N1> tab, T scale, int parts) {
  using C = BrickCfg<T, D, N1>;
  constexpr int P = C::P, NP = C::NP, NB = C::NB, EPB = C::EPB;
  constexpr int BX = C::BX, BY = C::BY, BZ = C::BZ, LX = C::LX, LY = C::LY, LZ = C::LZ;
  constexpr int NL = C::NL, NROWS = C::NROWS;
  static_assert(LX <= 32, "row masks hold 32 points");
  __shared__ T smem[C::SMEM];
  T *const acc = smem;             // the brick lattice (both paths)
  T *const tail = smem + NL;       // per-cell tiles, or the second sweep array
  const int brick = blk;
  const int tid = threadIdx.x;
  constexpr int nthr = C::NT;  // the launch uses exactly NT threads
  const int le = tid / NP, t = tid - le * NP;
  const int64_t rb = (int64_t)brick * NROWS;
  // lattice offset of thread t's x-run inside a cell tile
  const int run_off = (D == 3) ? (t % N1) * LX + (t / N1) * LX * LY : t * LX;
  const int c0 = br.cell_off[brick], c1 = br.cell_off[brick + 1];
  const int f0 = br.face_off[brick], f1e = br.face_off[brick + 1];
  const bool full = (c1 - c0) == C::MAXC;
  // Everything that does not depend on u is fetched in one round trip at the start: the
  // brick's row descriptors (every later lattice access indexes them), for a partial brick
  // its cells' run bases and lattice offsets, and the first batch of surrogate-face results
  // (held in registers through the cell phase).
  __shared__ int32_t s_base[NROWS], s_hbase[NROWS];
  // (the partial brick's run bases, cell offsets and row masks sit behind the per-cell tiles;
  // a full brick's rows are all DoFs, all touched by its cells: masks of all ones, not stored,
  // which keeps the static LDS small enough for one more workgroup per CU)
  int32_t *const s_runs = reinterpret_cast<int32_t *>(tail + 2 * C::NTILE * NB);
  int32_t *const s_loc = s_runs + C::MAXC * NP;
  uint32_t *const s_gmask = reinterpret_cast<uint32_t *>(tail + 2 * C::NTILE * NB + C::RUNS_T);
  uint32_t *const s_bmask = s_gmask + NROWS;
  for (int r = tid; r < NROWS; r += nthr) {
    s_base[r] = br.row_base[rb + r];
    s_hbase[r] = br.row_hbase[rb + r];
    if (!full) {
      s_gmask[r] = br.row_gmask[rb + r];
      s_bmask[r] = br.row_bmask[rb + r];
    }
  }
  if (C::STAGE_RUNS && !full && (parts & SBM_PART_CELLS)) {
    for (int i = tid; i < (c1 - c0) * NP; i += nthr) s_runs[i] = br.runs[(int64_t)c0 * NP + i];
    for (int i = tid; i < c1 - c0; i += nthr) s_loc[i] = br.cell_loc[c0 + i];
  }
  // a cell's run bases and lattice offset (by the cell's rank inside the brick)
  const int32_t *const runs_of = C::STAGE_RUNS ? s_runs : br.runs + (int64_t)c0 * NP;
  const int32_t *const loc_of = C::STAGE_RUNS ? s_loc : br.cell_loc + c0;
  const bool do_faces = (parts & SBM_PART_SBM_FACES) != 0;
  int fcode = 0, floc = 0;
  T fRv = T(0), fRg = T(0);
  if (do_faces && le < EPB && f0 + le < f1e) {
    const int f = f0 + le;
    fcode = br.face_code[f];
    floc = br.face_loc[f];
    fRv = fbuf[(int64_t)f * 2 * NP + t];
    fRg = fbuf[(int64_t)f * 2 * NP + NP + t];
  }
  __syncthreads();

  if (full && (parts & SBM_PART_CELLS)) {
    // ---- full brick: the sum of the cell operators over a tensor-product block of cells is
    // the Kronecker sum of the 1D operators assembled along each direction; sweep the
    // brick lattice line by line (a = M u, b = K u along the last axis, then c = M a,
    // e = K a + M b, then h (K c + M e)), in place in LDS. ----
    // sweep arrays: a/c in the accumulator itself (the last sweep writes in place), b/e in the
    // tail
    T *const LA = acc;
    T *const LB = tail;
    // last axis (z in 3D, y in 2D): a = M u, b = K u, gathered from u (every point of a full
    // brick is a DoF: id = row base + x)
    {
      constexpr int NC = (D == 3) ? BZ : BY, G = LaneGroup<NC>::G;
      constexpr int NLINE = (D == 3) ? LX * LY : LX;
      // every thread's segments are loaded before any is swept: one round trip to memory
      constexpr int NQ = (NLINE * G + nthr - 1) / nthr;
      T xus[NQ][N1];
#pragma unroll
      for (int r = 0; r < NQ; ++r) {
        const int q = tid + r * nthr;
        const int j = q % G, line = q / G;
        const int x = line % LX, y = (D == 3) ? line / LX : 0;
        const bool live = q < NLINE * G && j < NC;
#pragma unroll
        for (int i = 0; i < N1; ++i) {
          const int row = (D == 3) ? y + LY * (j * P + i) : (j * P + i);
          xus[r][i] = live ? u[s_base[live ? row : 0] + x] : T(0);
        }
      }
#pragma unroll
      for (int r = 0; r < NQ; ++r) {
        const int q = tid + r * nthr;
        const int j = q % G, line = q / G;
        const int x = line % LX, y = (D == 3) ? line / LX : 0;
        const bool live = q < NLINE * G && j < NC;
        T ya[N1], yb[N1];
        {
          const EvenOdd<T, N1> ex(xus[r]);
          EOAcc<T, N1> aa, ab;
          eo_acc<T, N1>(tab.EM, tab.OM, ex, aa.ye, aa.yo);
          eo_acc<T, N1>(tab.EK, tab.OK, ex, ab.ye, ab.yo);
          eo_combine<T, N1>(aa.ye, aa.yo, T(1), ya);
          eo_combine<T, N1>(ab.ye, ab.yo, T(1), yb);
        }
        ya[0] += from_prev_lane<G>(ya[P], j);
        yb[0] += from_prev_lane<G>(yb[P], j);
        if (live) {
          const int pt0 = (D == 3) ? x + LX * (y + LY * (j * P)) : x + LX * (j * P);
          constexpr int SL = (D == 3) ? LX * LY : LX;
#pragma unroll
          for (int i = 0; i < P; ++i) {
            LA[pt0 + i * SL] = ya[i];
            LB[pt0 + i * SL] = yb[i];
          }
          if (j == NC - 1) {
            LA[pt0 + P * SL] = ya[P];
            LB[pt0 + P * SL] = yb[P];
          }
        }
      }
    }
    __syncthreads();
    if constexpr (D == 3) {
      // y: c = M a, e = K a + M b, in place
      constexpr int G = LaneGroup<BY>::G;
      for (int q = tid; q < LX * LZ * G; q += nthr) {
        const int j = q % G, line = q / G;
        const int x = line % LX, z = line / LX;
        const bool live = j < BY;
        const int o = x + LX * LY * z + j * P * LX;
        T xa[N1], xb[N1], yc[N1], ye[N1];
#pragma unroll
        for (int i = 0; i < N1; ++i) {
          xa[i] = live ? LA[o + i * LX] : T(0);
          xb[i] = live ? LB[o + i * LX] : T(0);
        }
        {
          const EvenOdd<T, N1> ea(xa), eb(xb);
          EOAcc<T, N1> ac, ae;
          eo_acc<T, N1>(tab.EM, tab.OM, ea, ac.ye, ac.yo);
          eo_acc<T, N1>(tab.EK, tab.OK, ea, ae.ye, ae.yo);
          eo_acc<T, N1>(tab.EM, tab.OM, eb, ae.ye, ae.yo);
          eo_combine<T, N1>(ac.ye, ac.yo, T(1), yc);
          eo_combine<T, N1>(ae.ye, ae.yo, T(1), ye);
        }
        yc[0] += from_prev_lane<G>(yc[P], j);
        ye[0] += from_prev_lane<G>(ye[P], j);
        if (live) {
#pragma unroll
          for (int i = 0; i < P; ++i) {
            LA[o + i * LX] = yc[i];
            LB[o + i * LX] = ye[i];
          }
          if (j == BY - 1) {
            LA[o + P * LX] = yc[P];
            LB[o + P * LX] = ye[P];
          }
        }
      }
      __syncthreads();
    }
    // x: out = h (K c + M e), written over c
    {
      constexpr int G = LaneGroup<BX>::G;
      for (int q = tid; q < NROWS * G; q += nthr) {
        const int j = q % G, row = q / G;
        const bool live = j < BX;
        const int o = LX * row + j * P;
        T xc[N1], xe[N1], yo[N1];
#pragma unroll
        for (int i = 0; i < N1; ++i) {
          xc[i] = live ? LA[o + i] : T(0);
          xe[i] = live ? LB[o + i] : T(0);
        }
        {
          const EvenOdd<T, N1> ec(xc), ee(xe);
          EOAcc<T, N1> ao;
          eo_acc<T, N1>(tab.EK, tab.OK, ec, ao.ye, ao.yo);
          eo_acc<T, N1>(tab.EM, tab.OM, ee, ao.ye, ao.yo);
          eo_combine<T, N1>(ao.ye, ao.yo, scale, yo);
        }
        yo[0] += from_prev_lane<G>(yo[P], j);
        if (live) {
#pragma unroll
          for (int i = 0; i < P; ++i) acc[o + i] = yo[i];
          if (j == BX - 1) acc[o + P] = yo[P];
        }
      }
    }
    __syncthreads();
  } else {
    for (int i = tid; i < NL; i += nthr) acc[i] = T(0);
    __syncthreads();
  }

  if (!full && (parts & SBM_PART_CELLS)) {
    // ---- partial brick: cell by cell (EPC cells per batch; the other thread groups only
    // take part in the barriers) ----
    constexpr int EPC = C::EPC, NTILE = C::NTILE;
    const bool grp = le < EPC;
    const int tl = grp ? le : 0;  // groups beyond EPC only take part in the barriers
    T *A = tail + tl * NB, *B = tail + NTILE * NB + tl * NB;
    // software pipeline: the pencils of batch b+1 are in flight while batch b computes
    T x[N1];
    {
      const bool act = grp && c0 + le < c1;
      gather_pencil<T, D, N1>(runs_of + (act ? le : 0) * NP, u, t, act, x);
    }
    for (int b = c0; b < c1; b += EPC) {
      const int idx = b + le;
      const bool act = grp && idx < c1;
      const int loc = act ? loc_of[idx - c0] : 0;
      const int idn = idx + EPC;
      const bool actn = grp && idn < c1;
      T xn[N1], out[N1];
      gather_pencil<T, D, N1>(runs_of + (actn ? idn - c0 : 0) * NP, u, t, actn, xn);
      kron_cell<T, D, N1>(tab, t, x, A, B, scale, out, grp, grp);
#pragma unroll
      for (int i = 0; i < N1; ++i) x[i] = xn[i];
      // the batch's cells add their rows in slot order (a cell's runs are disjoint), so every
      // lattice point sums its cells in the same order on every launch: bitwise reproducible
      const int nslot = (c1 - b) < EPC ? (c1 - b) : EPC;
      for (int k = 0; k < nslot; ++k) {
        if (le == k) {
#pragma unroll
          for (int i = 0; i < N1; ++i) acc[loc + run_off + i] += out[i];
        }
        __syncthreads();
      }
    }
  }
  if (do_faces) {
    // ---- the brick's surrogate faces: sbm_face_cg_kernel left (Rv, Rg) per face node in
    // fbuf; expand them into the (p+1)^d local rows and add those into the lattice.  The
    // batch's data is in registers (the first batch since the start); the next batch's is
    // fetched while this one merges. ----
    constexpr int SL1 = LX, SL2 = LX * LY;  // lattice strides of axes 1 and 2
    for (int b = f0; b < f1e; b += EPB) {
      const int f = b + le;
      const bool fact = le < EPB && f < f1e;
      const int fn = f + EPB;
      int ncode = 0, nloc = 0;
      T nRv = T(0), nRg = T(0);
      if (le < EPB && fn < f1e) {
        ncode = br.face_code[fn];
        nloc = br.face_loc[fn];
        nRv = fbuf[(int64_t)fn * 2 * NP + t];
        nRg = fbuf[(int64_t)fn * 2 * NP + NP + t];
      }
      int node = 0, Sa = 0;
      T row[N1];
      if (fact) {
        const FaceAxes<D, N1> fa(fcode);
        const int loc = floc;
        const T Rv = fRv, Rg = fRg;
        const int a = fa.a;
        const int jb = (D == 3) ? t % N1 : t, jc = (D == 3) ? t / N1 : 0;
        // normal axis a; tangential axes in increasing order (b < c), as in FaceAxes
        Sa = (a == 0) ? 1 : (a == 1 ? SL1 : SL2);
        const int Sb = (a == 0) ? SL1 : 1;
        const int Sc = (D == 3) ? ((a == 2) ? SL1 : SL2) : 0;
        node = loc + jb * Sb + jc * Sc;
#pragma unroll
        for (int ia = 0; ia < N1; ++ia) row[ia] = face_row<T, D, N1>(tab, fa, ia, Rv, Rg);
      }
      // faces add in slot order (one face's node lines are disjoint): reproducible sums
      const int nslot = (f1e - b) < EPB ? (f1e - b) : EPB;
      for (int k = 0; k < nslot; ++k) {
        if (fact && le == k) {
#pragma unroll
          for (int ia = 0; ia < N1; ++ia) acc[node + ia * Sa] += row[ia];
        }
        __syncthreads();
      }
      fcode = ncode;
      floc = nloc;
      fRv = nRv;
      fRg = nRg;
    }
  }
  __syncthreads();
  // write-out: lanes walk the lattice with x fastest, so stores are row-contiguous.
  // Points strictly inside the brick box belong to this brick alone: final value.  Points
  // on the box boundary go to plane k = [x == 0] + 2 [y == 0] + 4 [z == 0] of the halo (the
  // brick's side of the point; bricks sharing the point differ in k), at the point's halo
  // index (consecutive along the row's boundary DoFs); halo_reduce_kernel sums the planes.
  // Lane layout: each wavefront takes RPW whole rows per pass (lane = row slot * LX + x), so a
  // lane's x and everything that depends on it only (masks below x, x on the box boundary)
  // are fixed, and a pass only advances the row; (y, z) of the row advance by a constant.
  // The passes are unrolled, every LDS read first, so that one wait covers them all.
  {
    constexpr int RPW = 64 / LX, NW = C::NT / 64, STEP = NW * RPW;
    constexpr int NPASS = (NROWS + STEP - 1) / STEP;
    constexpr int QY = STEP % LY, QZ = STEP / LY;
    constexpr uint32_t ALL = (LX == 32) ? 0xffffffffu : ((1u << LX) - 1u);
    static_assert(RPW >= 1 && C::NT % 64 == 0, "a wavefront holds at least one lattice row");
    const int lane = tid & 63, rl = lane / LX, x = lane - rl * LX;
    const bool xl = rl < RPW;
    const uint32_t below = (1u << x) - 1u;
    const bool xin = (unsigned)(x - 1) < (unsigned)(LX - 2);  // 0 < x < LX - 1
    const int xplane = x == 0 ? 1 : 0;
    const int row0 = (tid >> 6) * RPW + rl;
    int y = row0 % LY, z = row0 / LY;
    constexpr int CH = NPASS < 9 ? NPASS : 9;  // passes per group (bounds the registers held)
#pragma unroll
    for (int k0 = 0; k0 < NPASS; k0 += CH) {
      T val[CH];
      int base[CH], hb[CH];
      uint32_t gmk[CH], bmk[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int row = row0 + (k0 + k) * STEP;
        const bool on = xl && k0 + k < NPASS && row < NROWS;
        const int rc = on ? row : 0;
        val[k] = acc[rc * LX + x];
        base[k] = s_base[rc];
        hb[k] = s_hbase[rc];
        gmk[k] = full ? ALL : s_gmask[rc];
        bmk[k] = (full || !on) ? (on ? ALL : 0u) : s_bmask[rc];
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const uint32_t gm = gmk[k];
        const bool brow = ((unsigned)(y - 1) >= (unsigned)(LY - 2)) |
                          ((D == 3) & ((unsigned)(z - 1) >= (unsigned)(LZ - 2)));
        const bool inner = !brow & xin;
        const uint32_t hgm = brow ? gm : (gm & (1u | (1u << (LX - 1))));
        const int plane = xplane | (y == 0 ? 2 : 0) | ((D == 3 && z == 0) ? 4 : 0);
        T *dst = inner ? v + base[k] + __popc(gm & below)
                       : halo + (int64_t)plane * nhalo + hb[k] + __popc(hgm & below);
        if ((bmk[k] >> x) & 1u) *dst = val[k];
        y += QY;
        z += QZ;
        if (y >= LY) {
          y -= LY;
          ++z;
        }
      }
    }
  }
}

template <typename T, int D, int N1>
__global__ __launch_bounds__((BrickCfg<T, D, N1>::NT)) void brick_kernel(
    BrickArgs br, const T *__restrict__ fbuf, const T *__restrict__ u, T *__restrict__ v, T *__restrict__ halo,
    int nhalo, KTab<T, N1> tab, T scale, int parts) {
  brick_body<T, D, N1>(xcd_block(), br, fbuf, u, v, halo, nhalo, tab, scale, parts);
}

// v[dof] = sum over the planes k present in the DoF's mask, in increasing k (deterministic).
// Two DoFs per thread (a block's 2 * 256 consecutive ones), so that each thread has twice the
// loads in flight (FP64 apply at 64^3 Q4: 50.2 against 51.2 us).
constexpr int kHaloPerThread = 2;
template <typename T, int D>
__device__ __forceinline__ void halo_reduce_body(const int blk, int n, const int32_t *__restrict__ dof,
                                                          const uint8_t *__restrict__ mask,
                                                          const T *__restrict__ halo, T *__restrict__ v) {
  const int i0 = blk * (kHaloPerThread * 256) + threadIdx.x;
  uint32_t m[kHaloPerThread];
  int dd[kHaloPerThread];
#pragma unroll
  for (int r = 0; r < kHaloPerThread; ++r) {
    const int i = i0 + r * 256;
    m[r] = i < n ? mask[i] : 0u;
    dd[r] = i < n ? dof[i] : 0;
  }
  T s[kHaloPerThread];
#pragma unroll
  for (int r = 0; r < kHaloPerThread; ++r) s[r] = T(0);
#pragma unroll
  for (int k = 0; k < (1 << D); ++k)
#pragma unroll
    for (int r = 0; r < kHaloPerThread; ++r)
      s[r] += ((m[r] >> k) & 1u) ? halo[(int64_t)k * n + i0 + r * 256] : T(0);
#pragma unroll
  for (int r = 0; r < kHaloPerThread; ++r)
    if (i0 + r * 256 < n) v[dd[r]] = s[r];
}

template <typename T, int D>
__global__ __launch_bounds__(256) void halo_reduce_kernel(int n, const int32_t *__restrict__ dof,
                                                          const uint8_t *__restrict__ mask,
                                                          const T *__restrict__ halo, T *__restrict__ v) {
  halo_reduce_body<T, D>(blockIdx.x, n, dof, mask, halo, v);
}

// ------------------------------------------------------------------------------------
// CG surrogate-boundary faces (Alg. 3), EPB faces per workgroup, faces in brick order.
// Output per face: Rv and Rg at its NP face nodes (fbuf[f][0][t], fbuf[f][1][t]);
// brick_kernel expands them into the (p+1)^d local rows (face_row).
// Two thread layouts: "node" (le = tid / NP, t = tid % NP: one face node or Gauss point
// each) for the sum-factorised face sweeps, and "pair" (HP = ceil(NP / 2) threads per face,
// Gauss points 2k and 2k + 1 each) for the point evaluation E u, which reads the cell's
// (p+1)^d values once for both points.
// ------------------------------------------------------------------------------------
template <typename T, int D, int N1, int EPB>
__device__ __forceinline__ void sbm_face_cg_body(const int blk, int n_faces, const int32_t *__restrict__ face_code,
                                                          const int32_t *__restrict__ face_runs,
                                                          const double *__restrict__ face_xi,
                                                          const T *__restrict__ u, T *__restrict__ fbuf,
                                                          KTab<T, N1> tab, KScal sc) {
  constexpr int NP = Shape<D, N1>::NP, NB = Shape<D, N1>::NB, HP = (NP + 1) / 2;
  __shared__ T su_all[EPB * NB];
  __shared__ T fw_all[6 * EPB * NP];  // per face: g, sweep, E u, integrands v / dn v, scratch
  const int tid = threadIdx.x;
  const int f0 = blk * EPB;
  // node layout
  const int le = tid / NP, t = tid - le * NP;
  const int f = f0 + le;
  const bool act = le < EPB && f < n_faces;
  T *su = su_all + (le < EPB ? le : 0) * NB;
  T *fw = fw_all + (le < EPB ? le : 0) * 6 * NP;
  T *fg = fw, *fs = fw + NP, *fe = fw + 2 * NP, *f5 = fw + 3 * NP, *f6 = fw + 4 * NP, *fx = fw + 5 * NP;
  // pair layout
  const int pf = tid / HP, pk = tid - pf * HP;
  const int q0 = 2 * pk, q1 = 2 * pk + 1;
  const bool pact = pf < EPB && f0 + pf < n_faces;
  const bool has1 = pact && q1 < NP;
  // loads first: face code, the cell's u (one x-run per node thread), the pair's points
  const int code = act ? face_code[f] : 0;
  if (act) {
    const int64_t base = face_runs[(int64_t)f * NP + t];
#pragma unroll
    for (int i = 0; i < N1; ++i) su[N1 * t + i] = u[base + i];
  }
  double xa[D], xb[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    xa[k] = pact ? face_xi[((int64_t)(f0 + pf) * NP + q0) * D + k] : 0.0;
    xb[k] = has1 ? face_xi[((int64_t)(f0 + pf) * NP + q1) * D + k] : 0.0;
  }
  __syncthreads();
  const FaceAxes<D, N1> fa(code);
  const int jb = (D == 3) ? t % N1 : t, jc = (D == 3) ? t / N1 : 0;
  // normal derivative (reference, times the outward sign / h below) at face node t
  {
    T g = 0;
    const int node_off = jb * fa.Sb + jc * fa.Sc;
#pragma unroll
    for (int ia = 0; ia < N1; ++ia) g += (fa.s ? tab.D1[ia] : tab.D0[ia]) * su[ia * fa.Sa + node_off];
    if (le < EPB) fg[t] = g;
  }
  // E u at the pair's two shifted points
  if (pact) {
    const T *sp = su_all + pf * NB;
    double la[D][N1], lb[D][N1];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      lagrange_at<N1>(tab.z, tab.cinv, xa[k], la[k]);
      lagrange_at<N1>(tab.z, tab.cinv, xb[k], lb[k]);
    }
    T a0[N1], a1[N1], b0[N1], b1[N1];
#pragma unroll
    for (int j = 0; j < N1; ++j) {
      a0[j] = T(la[0][j]);
      a1[j] = T(la[1][j]);
      b0[j] = T(lb[0][j]);
      b1[j] = T(lb[1][j]);
    }
    T ea = 0, eb = 0;
    if constexpr (D == 3) {
      T a2[N1], b2[N1];
#pragma unroll
      for (int j = 0; j < N1; ++j) {
        a2[j] = T(la[2][j]);
        b2[j] = T(lb[2][j]);
      }
      // one (p+1)^2 slab per iteration, so that at most one slab of loads is in flight
#pragma unroll 1
      for (int i2 = 0; i2 < N1; ++i2) {
        const T *sl = sp + NP * i2;
        T ra = 0, rb = 0;
#pragma unroll
        for (int i1 = 0; i1 < N1; ++i1) {
          T sa = 0, sb = 0;
#pragma unroll
          for (int i0 = 0; i0 < N1; ++i0) {
            const T w = sl[i0 + N1 * i1];
            sa += a0[i0] * w;
            sb += b0[i0] * w;
          }
          ra += a1[i1] * sa;
          rb += b1[i1] * sb;
        }
        T wa = 0, wb = 0;
#pragma unroll
        for (int j = 0; j < N1; ++j) {
          wa = (j == i2) ? a2[j] : wa;
          wb = (j == i2) ? b2[j] : wb;
        }
        ea += wa * ra;
        eb += wb * rb;
      }
    } else {
#pragma unroll
      for (int i1 = 0; i1 < N1; ++i1) {
        T sa = 0, sb = 0;
#pragma unroll
        for (int i0 = 0; i0 < N1; ++i0) {
          const T w = sp[i0 + N1 * i1];
          sa += a0[i0] * w;
          sb += b0[i0] * w;
        }
        ea += a1[i1] * sa;
        eb += b1[i1] * sb;
      }
    }
    T *pe = fw_all + pf * 6 * NP + 2 * NP;
    pe[q0] = ea;
    if (has1) pe[q1] = eb;
  }
  __syncthreads();
  // GLL -> Gauss interpolation of the normal derivative on the face
  T dn;
  if constexpr (D == 3) {
    const int qb = t % N1;
    T r = 0;
#pragma unroll
    for (int j = 0; j < N1; ++j) r += tab.N[qb * N1 + j] * fg[j + N1 * jc];
    if (le < EPB) fs[t] = r;  // (qb, jc)
    __syncthreads();
    const int qc = t / N1;
    dn = 0;
#pragma unroll
    for (int j = 0; j < N1; ++j) dn += tab.N[qc * N1 + j] * fs[qb + N1 * j];
  } else {
    dn = 0;
#pragma unroll
    for (int j = 0; j < N1; ++j) dn += tab.N[t * N1 + j] * fg[j];
  }
  // integrands at Gauss point t
  {
    const T h = T(sc.h), sig = T(sc.sigma_gamma);
    const T sh = (fa.s ? T(1) : T(-1)) / h;
    const T om = act ? ((D == 3) ? h * h * tab.w[t % N1] * tab.w[t / N1] : h * tab.w[t]) : T(0);
    const T eu = fe[t];
    dn *= sh;
    if (le < EPB) {
      f5[t] = om * (sig * eu - dn);  // tested against v
      f6[t] = -om * eu * sh;         // tested against the reference derivative along a
    }
  }
  __syncthreads();
  T Rv, Rg;
  face_integrate<T, D, N1>(tab, t, fg, fx, f5, f6, Rv, Rg);
  if (act) {
    fbuf[(int64_t)f * 2 * NP + t] = Rv;
    fbuf[(int64_t)f * 2 * NP + NP + t] = Rg;
  }
}

// (at least 4 waves per SIMD: keeps the scheduler from holding the whole tile in registers)
template <typename T, int D, int N1, int EPB>
__global__ __launch_bounds__(256, 4) void sbm_face_cg_kernel(int n_faces, const int32_t *__restrict__ face_code,
                                                          const int32_t *__restrict__ face_runs,
                                                          const double *__restrict__ face_xi,
                                                          const T *__restrict__ u, T *__restrict__ fbuf,
                                                          KTab<T, N1> tab, KScal sc) {
  sbm_face_cg_body<T, D, N1, EPB>(xcd_block(), n_faces, face_code, face_runs, face_xi, u, fbuf, tab, sc);
}

// DG surrogate-boundary faces: one entity = one face.  Output per face: Rv and Rg at its NP
// face nodes (fbuf[f][0][t], fbuf[f][1][t]); the DG cell kernels add the face's rows into the
// cell's block in face order, so the apply has no atomics and is bitwise reproducible.
// ------------------------------------------------------------------------------------
template <typename T, int D, int N1, int EPB>
__device__ __forceinline__ void sbm_face_body(const int blk, int n_faces, const int32_t *__restrict__ face_cell,
                                                       const int32_t *__restrict__ face_code,
                                                       const double *__restrict__ face_xi, const T *__restrict__ u,
                                                       T *__restrict__ fbuf, KTab<T, N1> tab, KScal sc) {
  constexpr int NP = Shape<D, N1>::NP, NB = Shape<D, N1>::NB;
  __shared__ T su_all[EPB * NB];
  __shared__ T f_all[4 * EPB * NP];
  const int le = threadIdx.x / NP, t = threadIdx.x - le * NP;
  const int f = blk * EPB + le;
  const bool act = f < n_faces;
  T *su = su_all + le * NB;
  T *f1 = f_all + le * NP, *f2 = f1 + EPB * NP, *f3 = f2 + EPB * NP, *f4 = f3 + EPB * NP;
  double xp[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xp[k] = act ? face_xi[((int64_t)f * NP + t) * D + k] : 0.0;
  const FaceAxes<D, N1> fa(act ? face_code[f] : 0);
  const int64_t base = (int64_t)(act ? face_cell[f] : 0) * NB + N1 * t;
  if (act) {
#pragma unroll
    for (int i = 0; i < N1; ++i) su[N1 * t + i] = u[base + i];
  }
  __syncthreads();
  T Rv, Rg;
  sbm_face_eval<T, D, N1>(tab, sc, t, act, fa, xp, su, f1, f2, f3, f4, Rv, Rg);
  if (act) {
    fbuf[(int64_t)f * 2 * NP + t] = Rv;
    fbuf[(int64_t)f * 2 * NP + NP + t] = Rg;
  }
}

template <typename T, int D, int N1, int EPB>
__global__ __launch_bounds__(256) void sbm_face_kernel(int n_faces, const int32_t *__restrict__ face_cell,
                                                       const int32_t *__restrict__ face_code,
                                                       const double *__restrict__ face_xi, const T *__restrict__ u,
                                                       T *__restrict__ fbuf, KTab<T, N1> tab, KScal sc) {
  sbm_face_body<T, D, N1, EPB>(xcd_block(), n_faces, face_cell, face_code, face_xi, u, fbuf, tab, sc);
}

// DG surrogate-boundary faces in 3D with (p+1)^3 threads per face: thread (t, i2) takes face
// point t and slab i2 of the cell.  The cell's values are loaded one per thread; E u at each
// shifted point is split over the slabs (each thread one slab's (p+1)^2 terms) and the slab
// sums are added in slab order, as in sbm_face_eval; the face-node phases (normal
// derivative, Gauss interpolation, integration) run in every slab with identical results;
// slab 0 stores the face's (Rv, Rg) as sbm_face_kernel does.  For p <= 5 ((p+1)^3 <= 256).
// face_runs != nullptr (CG): the cell's values are gathered through its x-run bases
// (face_runs[f][t] is the first DoF of run t); otherwise (DG) the cell block is contiguous.
template <typename T, int N1, int EPB>
__device__ __forceinline__ void sbm_face_slab_body(const int blk, int n_faces, const int32_t *__restrict__ face_cell,
                                                            const int32_t *__restrict__ face_code,
                                                            const double *__restrict__ face_xi,
                                                            const int32_t *__restrict__ face_runs,
                                                            const T *__restrict__ u, T *__restrict__ fbuf,
                                                            KTab<T, N1> tab, KScal sc) {
  constexpr int D = 3, NP = N1 * N1, NB = NP * N1;
  __shared__ T su_all[EPB * NB];
  __shared__ T sp_all[EPB * NB];  // slab partial sums of E u
  __shared__ T f_all[4 * EPB * NP];
  const int le = threadIdx.x / NB, r = threadIdx.x - le * NB;
  const int t = r % NP, i2 = r / NP;
  const int f = blk * EPB + le;
  const bool act = f < n_faces;
  T *su = su_all + le * NB, *sp = sp_all + le * NB;
  T *f1 = f_all + le * NP, *f2 = f1 + EPB * NP, *f3 = f2 + EPB * NP, *f4 = f3 + EPB * NP;
  double xp[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xp[k] = act ? face_xi[((int64_t)f * NP + t) * D + k] : 0.0;
  const FaceAxes<D, N1> fa(act ? face_code[f] : 0);
  if (act) {
    const int64_t at = face_runs ? (int64_t)face_runs[(int64_t)f * NP + r / N1] + r % N1
                                 : (int64_t)face_cell[f] * NB + r;
    su[r] = u[at];
  }
  __syncthreads();
  const T h = T(sc.h), sig = T(sc.sigma_gamma);
  const T sh = (fa.s ? T(1) : T(-1)) / h;
  const int jb = t % N1, jc = t / N1;
  const int node_off = jb * fa.Sb + jc * fa.Sc;
  {
    T g = 0;
#pragma unroll
    for (int ia = 0; ia < N1; ++ia) g += (fa.s ? tab.D1[ia] : tab.D0[ia]) * su[ia * fa.Sa + node_off];
    f1[t] = g;
    f2[t] = g;
  }
  __syncthreads();
  T dn, dn2;
  face_interpolate<T, D, N1>(tab, t, f1, f2, f3, f4, dn, dn2);
  dn *= sh;
  // slab i2 of E u at point t
  T part = 0;
  if (act) {
    double l[D][N1];
#pragma unroll
    for (int k = 0; k < D; ++k) lagrange_at<N1>(tab.z, tab.cinv, xp[k], l[k]);
    T s1 = 0;
#pragma unroll
    for (int i1 = 0; i1 < N1; ++i1) {
      T s0 = 0;
#pragma unroll
      for (int i0 = 0; i0 < N1; ++i0) s0 += T(l[0][i0]) * su[i0 + N1 * i1 + NP * i2];
      s1 += T(l[1][i1]) * s0;
    }
    T l2 = 0;
#pragma unroll
    for (int j = 0; j < N1; ++j) l2 = (j == i2) ? T(l[2][j]) : l2;
    part = l2 * s1;
  }
  sp[i2 * NP + t] = part;
  __syncthreads();  // slab sums written; face_interpolate's reads of f3/f4 are done
  T eu = 0;
#pragma unroll
  for (int j = 0; j < N1; ++j) eu += sp[j * NP + t];
  const T om = act ? h * h * tab.w[t % N1] * tab.w[t / N1] : T(0);
  f3[t] = om * (sig * eu - dn);  // tested against v
  f4[t] = -om * eu * sh;         // tested against the reference derivative along a
  __syncthreads();
  T Rv, Rg;
  face_integrate<T, D, N1>(tab, t, f1, f2, f3, f4, Rv, Rg);
  if (act && i2 == 0) {
    fbuf[(int64_t)f * 2 * NP + t] = Rv;
    fbuf[(int64_t)f * 2 * NP + NP + t] = Rg;
  }
}

template <typename T, int N1, int EPB>
__global__ __launch_bounds__(256) void sbm_face_slab_kernel(int n_faces, const int32_t *__restrict__ face_cell,
                                                            const int32_t *__restrict__ face_code,
                                                            const double *__restrict__ face_xi,
                                                            const int32_t *__restrict__ face_runs,
                                                            const T *__restrict__ u, T *__restrict__ fbuf,
                                                            KTab<T, N1> tab, KScal sc) {
  sbm_face_slab_body<T, N1, EPB>(xcd_block(), n_faces, face_cell, face_code, face_xi, face_runs, u, fbuf, tab, sc);
}

// ------------------------------------------------------------------------------------
// DG cell kernel: Laplace cell term + SIPG terms of the cell's interior faces, computed
// from the cell's side only (each interior face is evaluated twice, once per cell), so
// every cell writes only its own block: no atomics, deterministic.
// For the face (a, s) of K with neighbour N and outward normal n_K = (2s-1) e_a:
//   [u]_K = u_K - u_N,  {du/dn_K} = (du_K/dn_K + du_N/dn_K)/2,
//   K's rows += int (sigma_F [u]_K - {du/dn_K}) v - 1/2 [u]_K dv/dn_K   (Alg. 2, per side)
// ------------------------------------------------------------------------------------
// Face-by-face form (one group of NP threads per cell walks the 2d faces in turn), for the
// degrees with more than 128 threads per cell in the parallel form below.
// BATCH: the kernel serves a batch of applies (items, blk_item as in the batched kernels after
// apply_impl; the pointer and size arguments are then taken from the workgroup's item).  This
// form is kept as one kernel rather than a body called by two (as the other kernels are): as
// an inlined body it compiled to about 6 % more instructions (DG Q5 apply 24.9 against 23.6 us).
template <typename T, int D, int N1, int EPB, bool BATCH>
__global__ __launch_bounds__(256) void dg_cell_seq_kernel(int n_cells, const int32_t *__restrict__ nbr,
                                                      const T *__restrict__ u, const T *__restrict__ fbuf,
                                                      T *__restrict__ v, KTab<T, N1> tab, KScal sc, T scale,
                                                      int parts, const BatchItem *__restrict__ items,
                                                      const int32_t *__restrict__ blk_item) {
  int blk = xcd_block();
  if constexpr (BATCH) {
    const BatchItem *it = items + blk_item[blk];
    blk -= it->blk0[1];
    n_cells = it->nc;
    nbr = it->nbr;
    u = (const T *)it->u;
    fbuf = (const T *)it->fbuf;
    v = (T *)it->v;
    sc = it->sc;
    scale = T(D == 3 ? it->sc.h : 1.0);
  }
  constexpr int NP = Shape<D, N1>::NP, NB = Shape<D, N1>::NB, P = N1 - 1;
  __shared__ T su_all[EPB * NB];
  __shared__ T sa_all[EPB * NB];
  __shared__ T sb_all[EPB * NB];
  __shared__ T sw_all[EPB * NB];
  __shared__ T f_all[4 * EPB * NP];
  const int le = threadIdx.x / NP, t = threadIdx.x - le * NP;
  const int cell = blk * EPB + le;
  const bool act = cell < n_cells;
  T *su = su_all + le * NB, *A = sa_all + le * NB, *B = sb_all + le * NB, *sw = sw_all + le * NB;
  T *f1 = f_all + le * NP, *f2 = f1 + EPB * NP, *f3 = f2 + EPB * NP, *f4 = f3 + EPB * NP;
  const T h = T(sc.h), sigf = T(sc.sigma_f);
  const bool use_int = (parts & SBM_PART_CELLS) != 0, use_sbm = (parts & SBM_PART_SBM_FACES) != 0;

  // neighbours of the 2d faces, and the first neighbour's run for this thread: every
  // neighbour's values are loaded one face ahead, so the loads overlap the previous face
  int nbs[2 * D];
#pragma unroll
  for (int k = 0; k < 2 * D; ++k) nbs[k] = act ? nbr[(int64_t)cell * 2 * D + k] : -1;
  T nx[N1];
  if (nbs[0] >= 0) {
    const T *up = u + (int64_t)nbs[0] * NB + N1 * t;
#pragma unroll
    for (int i = 0; i < N1; ++i) nx[i] = up[i];
  }
  // own block (contiguous), thread t = run
  if (act) {
    const T *up = u + (int64_t)cell * NB + N1 * t;
#pragma unroll
    for (int i = 0; i < N1; ++i) su[N1 * t + i] = up[i];
  }
  __syncthreads();
  {
    T x[N1], out[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) x[k] = su[t + NP * k];
    kron_cell<T, D, N1>(tab, t, x, A, B, scale, out);
#pragma unroll
    for (int i = 0; i < N1; ++i) sw[N1 * t + i] = use_int ? out[i] : T(0);
  }
  // ---- interior faces, and the surrogate faces' rows (results of sbm_face_kernel) ----
  const int jb = (D == 3) ? t % N1 : t, jc = (D == 3) ? t / N1 : 0;
#pragma unroll
  for (int code = 0; code < 2 * D; ++code) {
    const FaceAxes<D, N1> fa(code);
    const bool has = nbs[code] >= 0;
    __syncthreads();  // previous users of A (neighbour tile) and f1..f4 are done
    if (has) {
#pragma unroll
      for (int i = 0; i < N1; ++i) A[N1 * t + i] = nx[i];
    }
    if (code + 1 < 2 * D && nbs[code + 1] >= 0) {
      const T *up = u + (int64_t)nbs[code + 1] * NB + N1 * t;
#pragma unroll
      for (int i = 0; i < N1; ++i) nx[i] = up[i];
    }
    __syncthreads();
    const T sgn = fa.s ? T(1) : T(-1);
    const int node_off = jb * fa.Sb + jc * fa.Sc;
    {
      T dK = 0, dN = 0;
#pragma unroll
      for (int ia = 0; ia < N1; ++ia) {
        dK += (fa.s ? tab.D1[ia] : tab.D0[ia]) * su[ia * fa.Sa + node_off];
        dN += (fa.s ? tab.D0[ia] : tab.D1[ia]) * A[ia * fa.Sa + node_off];
      }
      const T uK = su[fa.s * P * fa.Sa + node_off];
      const T uN = A[(1 - fa.s) * P * fa.Sa + node_off];
      f1[t] = uK - uN;                       // [u]_K at the face nodes
      f2[t] = T(0.5) * sgn * (dK + dN) / h;  // {du/dn_K} at the face nodes
    }
    __syncthreads();
    T jq, aq;
    face_interpolate<T, D, N1>(tab, t, f1, f2, f3, f4, jq, aq);
    T om;
    if constexpr (D == 3)
      om = h * h * tab.w[t % N1] * tab.w[t / N1];
    else
      om = h * tab.w[t];
    __syncthreads();
    f3[t] = om * (sigf * jq - aq);
    f4[t] = T(-0.5) * om * jq * sgn / h;
    __syncthreads();
    T Rv, Rg;
    face_integrate<T, D, N1>(tab, t, f1, f2, f3, f4, Rv, Rg);
    const bool sbmf = nbs[code] < -1 && use_sbm;  // surrogate face -2 - nbs[code]
    if (sbmf) {
      const int64_t fo = (int64_t)(-2 - nbs[code]) * 2 * NP;
      Rv = fbuf[fo + t];
      Rg = fbuf[fo + NP + t];
    }
    if ((has && use_int) || sbmf) {
#pragma unroll
      for (int ia = 0; ia < N1; ++ia)
        sw[ia * fa.Sa + node_off] += ((ia == fa.s * P) ? Rv : T(0)) + (fa.s ? tab.D1[ia] : tab.D0[ia]) * Rg;
    }
  }
  __syncthreads();
  if (act) {
    T *vp = v + (int64_t)cell * NB + N1 * t;
#pragma unroll
    for (int i = 0; i < N1; ++i) vp[i] = sw[N1 * t + i];
  }
}

// Thread layout: 2d groups of NP threads per cell, group g evaluates interior face g (code
// 2 axis + side) with its own neighbour tile and scratch, all faces at once; then the block's
// first EPB NP threads form the cells' terms (NP per cell; the rest only pass the barriers).
// Then every row of the cell adds the cell term and the faces' rows in face order (the order
// of a face-by-face loop); a face without a neighbour contributes the surrogate face's rows.
template <typename T, int D, int N1>
constexpr int dg_cells_per_block(bool one_wave) {
  constexpr int NP = Shape<D, N1>::NP, NB = Shape<D, N1>::NB, TPC = 2 * D * NP;
  // LDS per cell: own tile, 2d neighbour tiles (two of them reused for the cell term), cell
  // result (NB each); per face 6 NP of scratch and results
  constexpr int per_cell = ((2 + 2 * D) * NB + 2 * D * 6 * NP) * (int)sizeof(T);
  int e = (one_wave ? 64 : 256) / TPC;
  if (e < 1) e = 1;
  while (e > 1 && e * per_cell > 60000) --e;
  return e;
}

template <typename T, int D, int N1, int EPB>
__device__ __forceinline__ void dg_cell_body(const int blk, int n_cells, const int32_t *__restrict__ nbr,
                                                      const T *__restrict__ u, const T *__restrict__ fbuf,
                                                      T *__restrict__ v, KTab<T, N1> tab, KScal sc, T scale,
                                                      int parts) {
  constexpr int NP = Shape<D, N1>::NP, NB = Shape<D, N1>::NB, P = N1 - 1, NF = 2 * D, TPC = NF * NP;
  __shared__ T su_all[EPB * NB];           // own tile
  __shared__ T sn_all[EPB * NF * NB];      // neighbour tiles, one per face (then the cell-term tiles)
  __shared__ T sw_all[EPB * NB];           // cell term
  __shared__ T f_all[EPB * NF * 6 * NP];   // per face: f1..f4 scratch, Rv, Rg
  const int le = threadIdx.x / TPC, r = threadIdx.x - le * TPC;  // cell in block, thread in cell
  const int g = r / NP, t = r - g * NP;                            // face group, node / run
  const int cell = blk * EPB + le;
  const bool act = cell < n_cells;
  T *su = su_all + le * NB, *sw = sw_all + le * NB;
  T *An = sn_all + (le * NF + g) * NB;
  T *fw = f_all + (le * NF + g) * 6 * NP;
  T *f1 = fw, *f2 = fw + NP, *f3 = fw + 2 * NP, *f4 = fw + 3 * NP, *fRv = fw + 4 * NP, *fRg = fw + 5 * NP;
  const T h = T(sc.h), sigf = T(sc.sigma_f);
  const bool use_int = (parts & SBM_PART_CELLS) != 0, use_sbm = (parts & SBM_PART_SBM_FACES) != 0;

  // loads: group 0 the cell's own block (thread t = run), group g the neighbour across face g
  const int nb = act ? nbr[(int64_t)cell * NF + g] : -1;
  const bool has = nb >= 0;
  if (g == 0 && act) {
    const T *up = u + (int64_t)cell * NB + N1 * t;
#pragma unroll
    for (int i = 0; i < N1; ++i) su[N1 * t + i] = up[i];
  }
  if (has) {
    const T *up = u + (int64_t)nb * NB + N1 * t;
#pragma unroll
    for (int i = 0; i < N1; ++i) An[N1 * t + i] = up[i];
  }
  __syncthreads();
  // ---- interior face g: traces, Gauss-point integrands, transposed integration ----
  {
    const FaceAxes<D, N1> fa(g);
    const int jb = (D == 3) ? t % N1 : t, jc = (D == 3) ? t / N1 : 0;
    const T sgn = fa.s ? T(1) : T(-1);
    const int node_off = jb * fa.Sb + jc * fa.Sc;
    T dK = 0, dN = 0;
#pragma unroll
    for (int ia = 0; ia < N1; ++ia) {
      dK += (fa.s ? tab.D1[ia] : tab.D0[ia]) * su[ia * fa.Sa + node_off];
      dN += (fa.s ? tab.D0[ia] : tab.D1[ia]) * An[ia * fa.Sa + node_off];
    }
    const T uK = su[fa.s * P * fa.Sa + node_off];
    const T uN = An[(1 - fa.s) * P * fa.Sa + node_off];
    f1[t] = uK - uN;                       // [u]_K at the face nodes
    f2[t] = T(0.5) * sgn * (dK + dN) / h;  // {du/dn_K} at the face nodes
    __syncthreads();
    T jq, aq;
    face_interpolate<T, D, N1>(tab, t, f1, f2, f3, f4, jq, aq);
    T om;
    if constexpr (D == 3)
      om = h * h * tab.w[t % N1] * tab.w[t / N1];
    else
      om = h * tab.w[t];
    __syncthreads();
    f3[t] = om * (sigf * jq - aq);
    f4[t] = T(-0.5) * om * jq * sgn / h;
    __syncthreads();
    T Rv, Rg;
    face_integrate<T, D, N1>(tab, t, f1, f2, f3, f4, Rv, Rg);
    if (has) {
      fRv[t] = use_int ? Rv : T(0);
      fRg[t] = use_int ? Rg : T(0);
    } else if (nb < -1 && use_sbm) {
      // surrogate face -2 - nb: its (Rv, Rg) from sbm_face_kernel, rows formed as for the others
      const int64_t fo = (int64_t)(-2 - nb) * 2 * NP;
      fRv[t] = fbuf[fo + t];
      fRg[t] = fbuf[fo + NP + t];
    } else {
      fRv[t] = T(0);
      fRg[t] = T(0);
    }
  }
  // ---- cell term: the block's first EPB * NP threads, NP per cell (whole wavefronts beyond
  // them only take part in the barriers).  Its two sweep tiles are the cell's first two
  // neighbour tiles: every neighbour value was read before the face phase's first barrier ----
  {
    const int lc = threadIdx.x / NP, tc = threadIdx.x - lc * NP;
    const bool work = lc < EPB;
    const int lw = work ? lc : 0;
    T *A = sn_all + lw * NF * NB, *B = A + NB;
    T x[N1], out[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) x[k] = work ? su_all[lw * NB + tc + NP * k] : T(0);
    kron_cell<T, D, N1>(tab, tc, x, A, B, scale, out, true, work);
    if (work) {
#pragma unroll
      for (int i = 0; i < N1; ++i) sw_all[lw * NB + N1 * tc + i] = use_int ? out[i] : T(0);
    }
  }
  __syncthreads();
  // ---- rows: cell term, then each face's rows in face order ----
  if (act) {
    for (int i = r; i < NB; i += TPC) {
      const int ik[3] = {i % N1, (i / N1) % N1, i / (N1 * N1)};
      T val = sw[i];
#pragma unroll
      for (int code = 0; code < NF; ++code) {
        const int a = code >> 1, s = code & 1;
        // node index on face `code`: lower tangential coordinate + N1 * upper one
        const int lo = (a == 0) ? 1 : 0, hi = (a == 2) ? 1 : 2;
        const int node = (D == 3) ? ik[lo] + N1 * ik[hi] : ik[lo];
        const int ia = ik[a];
        const T *fc = f_all + (le * NF + code) * 6 * NP;
        val += ((ia == s * P) ? fc[4 * NP + node] : T(0)) + (s ? tab.D1[ia] : tab.D0[ia]) * fc[5 * NP + node];
      }
      v[(int64_t)cell * NB + i] = val;
    }
  }
}

template <typename T, int D, int N1, int EPB>
__global__ __launch_bounds__(256) void dg_cell_kernel(int n_cells, const int32_t *__restrict__ nbr,
                                                      const T *__restrict__ u, const T *__restrict__ fbuf,
                                                      T *__restrict__ v, KTab<T, N1> tab, KScal sc, T scale,
                                                      int parts) {
  dg_cell_body<T, D, N1, EPB>(xcd_block(), n_cells, nbr, u, fbuf, v, tab, sc, scale, parts);
}

template <typename T, int N1>
KTab<T, N1> make_ktab(const Rules1D &r) {
  KTab<T, N1> k;
  constexpr int HC = (N1 + 1) / 2, HF = N1 / 2, P = N1 - 1;
  const std::vector<double> *mats[2] = {&r.M, &r.K};
  T *E[2] = {k.EM, k.EK}, *O[2] = {k.OM, k.OK};
  for (int m = 0; m < 2; ++m) {
    const std::vector<double> &A = *mats[m];
    for (int i = 0; i < HC; ++i)
      for (int c = 0; c < HC; ++c)
        E[m][i * HC + c] = T(c < HF ? 0.5 * (A[i * N1 + c] + A[i * N1 + (P - c)]) : A[i * N1 + c]);
    for (int i = 0; i < HF; ++i)
      for (int c = 0; c < HF; ++c) O[m][i * HF + c] = T(0.5 * (A[i * N1 + c] - A[i * N1 + (P - c)]));
  }
  for (int i = 0; i < N1 * N1; ++i) {
    k.M[i] = T(r.M[i]);
    k.K[i] = T(r.K[i]);
    k.N[i] = T(r.N[i]);
  }
  for (int j = 0; j < N1; ++j) {
    k.D0[j] = T(r.D0[j]);
    k.D1[j] = T(r.D1[j]);
    k.w[j] = T(r.w[j]);
    k.z[j] = r.z[j];
    k.cinv[j] = r.cinv[j];
  }
  return k;
}

template <typename T, int D, int N1>
hipError_t apply_impl(const sbm_ctx *c, const T *u, T *v, int parts, hipStream_t s, const Scratch &scr) {
  constexpr int NP = Shape<D, N1>::NP;
  const KTab<T, N1> tab = make_ktab<T, N1>(c->rules);
  const KScal sc{c->h, c->sigma_gamma, c->sigma_f};
  const T scale = T(D == 3 ? c->h : 1.0);
  const int nc = (int)c->n_cells, nf = (int)c->n_sbm;
  if (c->disc == SBM_CG) {
    if (c->n_bricks > 0 && (parts & (SBM_PART_CELLS | SBM_PART_SBM_FACES))) {
      constexpr int NT = BrickCfg<T, D, N1>::NT;
      const BrickArgs br{c->d_brick_cell_off, c->d_brick_runs, c->d_brick_cell_loc, c->d_brick_face_off,
                         c->d_brick_face_loc, c->d_face_code,  c->d_row_base,       c->d_row_gmask,
                         c->d_row_bmask,      c->d_row_hbase};
      T *halo = (T *)scr.halo;
      T *fbuf = (T *)scr.fbuf;
      if (nf > 0 && (parts & SBM_PART_SBM_FACES) && !(parts & SBM_PART_REUSE_FACES)) {
        // (the one-thread-per-(point, slab) layout of the DG faces measured 21.7 against
        // 11.6 us here at 3D p = 4: the pair layout reads each cell value once for two points)
        constexpr int EF = epb<T, D, N1, 2, 0>();
        hipLaunchKernelGGL((sbm_face_cg_kernel<T, D, N1, EF>), dim3((nf + EF - 1) / EF), dim3(EF * NP), 0, s, nf,
                           c->d_face_code, c->d_face_runs, c->d_face_xi, u, fbuf, tab, sc);
      }
      const int nh = (int)c->n_halo_dofs;
      hipLaunchKernelGGL((brick_kernel<T, D, N1>), dim3((unsigned)c->n_bricks), dim3(NT), 0, s, br,
                         (const T *)fbuf, u, v, halo, nh, tab, scale, parts);
      if (nh > 0 && !(parts & SBM_PART_NO_ASSEMBLY)) {
        constexpr int HB = kHaloPerThread * 256;  // DoFs per block
        hipLaunchKernelGGL((halo_reduce_kernel<T, D>), dim3((nh + HB - 1) / HB), dim3(256), 0, s, nh, c->d_halo_dof,
                           (const uint8_t *)c->d_halo_mask, (const T *)halo, v);
      }
    }
  } else {
    // surrogate faces first (their (Rv, Rg) go to fbuf), then the cell kernel writes every
    // cell's block once: cell term, interior faces and the surrogate faces' rows in face order
    T *fbuf = (T *)scr.fbuf;
    if (nf > 0 && (parts & SBM_PART_SBM_FACES) && !(parts & SBM_PART_REUSE_FACES)) {
      if constexpr (D == 3 && Shape<D, N1>::NB <= 256) {
        constexpr int NB = Shape<D, N1>::NB, E = 256 / NB, E1 = (64 / NB < 1) ? 1 : 64 / NB;
        if ((nf + E - 1) / E >= two_per_cu())
          hipLaunchKernelGGL((sbm_face_slab_kernel<T, N1, E>), dim3((nf + E - 1) / E), dim3(E * NB), 0, s, nf,
                             c->d_face_cell, c->d_face_code, c->d_face_xi, (const int32_t *)nullptr, u, fbuf, tab, sc);
        else
          hipLaunchKernelGGL((sbm_face_slab_kernel<T, N1, E1>), dim3((nf + E1 - 1) / E1), dim3(E1 * NB), 0, s,
                             nf, c->d_face_cell, c->d_face_code, c->d_face_xi, (const int32_t *)nullptr, u, fbuf, tab,
                             sc);
      } else {
        constexpr int E = epb<T, D, N1, 1, 0>(), E1 = epb_one_wave<T, D, N1, 1>();
        if ((nf + E - 1) / E >= two_per_cu())
          hipLaunchKernelGGL((sbm_face_kernel<T, D, N1, E>), dim3((nf + E - 1) / E), dim3(E * NP), 0, s, nf,
                             c->d_face_cell, c->d_face_code, c->d_face_xi, u, fbuf, tab, sc);
        else
          hipLaunchKernelGGL((sbm_face_kernel<T, D, N1, E1>), dim3((nf + E1 - 1) / E1), dim3(E1 * NP), 0, s, nf,
                             c->d_face_cell, c->d_face_code, c->d_face_xi, u, fbuf, tab, sc);
      }
    }
    // entities per workgroup: as many as fit, unless that leaves fewer than two workgroups
    // per compute unit; then one wavefront's worth
    if (nc > 0 && (parts & (SBM_PART_CELLS | SBM_PART_SBM_FACES))) {
      // faces in parallel where a cell needs at most 128 threads (3D p <= 3, 2D): measured 7 %
      // (FP64) to 20 % (FP32) faster at 3D p=3; at 3D p=5 its 216-thread, 31 KB cells leave the
      // grid in more than one round and the face-by-face form is faster
      constexpr int TPC = 2 * D * NP, NBC = Shape<D, N1>::NB;
      constexpr bool PAR = TPC <= 128 && ((4 + 2 * D) * NBC + 2 * D * 6 * NP + 2 * NBC) * (int)sizeof(T) <= 60000;
      if constexpr (PAR) {
        constexpr int E = dg_cells_per_block<T, D, N1>(false), E1 = dg_cells_per_block<T, D, N1>(true);
        if ((nc + E - 1) / E >= two_per_cu())
          hipLaunchKernelGGL((dg_cell_kernel<T, D, N1, E>), dim3((nc + E - 1) / E), dim3(E * TPC), 0, s, nc,
                             c->d_nbr, u, (const T *)fbuf, v, tab, sc, scale, parts);
        else
          hipLaunchKernelGGL((dg_cell_kernel<T, D, N1, E1>), dim3((nc + E1 - 1) / E1), dim3(E1 * TPC), 0, s, nc,
                             c->d_nbr, u, (const T *)fbuf, v, tab, sc, scale, parts);
      } else {
        constexpr int E = epb<T, D, N1, 4, 0>(), E1 = epb_one_wave<T, D, N1, 4>();
        if ((nc + E - 1) / E >= two_per_cu())
          hipLaunchKernelGGL((dg_cell_seq_kernel<T, D, N1, E, false>), dim3((nc + E - 1) / E), dim3(E * NP), 0, s,
                             nc, c->d_nbr, u, (const T *)fbuf, v, tab, sc, scale, parts, (const BatchItem *)nullptr,
                             (const int32_t *)nullptr);
        else
          hipLaunchKernelGGL((dg_cell_seq_kernel<T, D, N1, E1, false>), dim3((nc + E1 - 1) / E1), dim3(E1 * NP), 0,
                             s, nc, c->d_nbr, u, (const T *)fbuf, v, tab, sc, scale, parts,
                             (const BatchItem *)nullptr, (const int32_t *)nullptr);
      }
    }
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Batched applies: the applies of several operators that share a kernel instantiation
// (discretisation, dimension, degree, precision) run as one launch per stage over all of
// them (surrogate faces, cells or bricks, brick-boundary sums).  Workgroup g of a stage finds
// its item through blk_item[g] and runs the body of the single apply with that item's arrays
// and its block index inside the item, so every item's result is bitwise the one of its own
// apply.  The DG stages use the many-entities-per-workgroup variants (a batch fills the device).
// ------------------------------------------------------------------------------------

template <typename T, int D, int N1>
struct BatchShape {
  static constexpr int NP = Shape<D, N1>::NP, NB = Shape<D, N1>::NB;
  static constexpr int EF = epb<T, D, N1, 2, 0>();  // CG faces per workgroup (as the single apply)
  // DG faces: the slab layout in 3D where a cell fits one workgroup, else one group per face
  static constexpr bool SLAB = D == 3 && NB <= 256;
  static constexpr int EFD = SLAB ? 256 / NB : epb<T, D, N1, 1, 0>();
  static constexpr int TFD = SLAB ? EFD * NB : EFD * NP;
  // DG cells: the parallel-face form where a cell needs at most 128 threads
  static constexpr int TPC = 2 * D * NP;
  static constexpr bool PAR = TPC <= 128 && ((4 + 2 * D) * NB + 2 * D * 6 * NP + 2 * NB) * (int)sizeof(T) <= 60000;
  static constexpr int EC = PAR ? dg_cells_per_block<T, D, N1>(false) : epb<T, D, N1, 4, 0>();
  static constexpr int TC = PAR ? EC * TPC : EC * NP;
};

template <typename T, int D, int N1>
__global__ __launch_bounds__((BrickCfg<T, D, N1>::NT)) void brick_batch_kernel(const BatchItem *__restrict__ items,
                                                                              const int32_t *__restrict__ blk_item,
                                                                              KTab<T, N1> tab) {
  const int g = xcd_block();
  const BatchItem *it = items + blk_item[g];
  brick_body<T, D, N1>(g - it->blk0[1], it->br, (const T *)it->fbuf, (const T *)it->u, (T *)it->v, (T *)it->halo,
                       it->nh, tab, T(D == 3 ? it->sc.h : 1.0), SBM_PART_ALL);
}

template <typename T, int D>
__global__ __launch_bounds__(256) void halo_reduce_batch_kernel(const BatchItem *__restrict__ items,
                                                                const int32_t *__restrict__ blk_item) {
  const int g = blockIdx.x;
  const BatchItem *it = items + blk_item[g];
  halo_reduce_body<T, D>(g - it->blk0[2], it->nh, it->halo_dof, it->halo_mask, (const T *)it->halo, (T *)it->v);
}

template <typename T, int D, int N1, int EPB>
__global__ __launch_bounds__(256, 4) void sbm_face_cg_batch_kernel(const BatchItem *__restrict__ items,
                                                                   const int32_t *__restrict__ blk_item,
                                                                   KTab<T, N1> tab) {
  const int g = xcd_block();
  const BatchItem *it = items + blk_item[g];
  sbm_face_cg_body<T, D, N1, EPB>(g - it->blk0[0], it->nf, it->face_code, it->face_runs, it->face_xi,
                                  (const T *)it->u, (T *)it->fbuf, tab, it->sc);
}

template <typename T, int D, int N1>
__global__ __launch_bounds__(256) void sbm_face_dg_batch_kernel(const BatchItem *__restrict__ items,
                                                                const int32_t *__restrict__ blk_item,
                                                                KTab<T, N1> tab) {
  using S = BatchShape<T, D, N1>;
  const int g = xcd_block();
  const BatchItem *it = items + blk_item[g];
  const int b = g - it->blk0[0];
  if constexpr (S::SLAB)
    sbm_face_slab_body<T, N1, S::EFD>(b, it->nf, it->face_cell, it->face_code, it->face_xi, (const int32_t *)nullptr,
                                      (const T *)it->u, (T *)it->fbuf, tab, it->sc);
  else
    sbm_face_body<T, D, N1, S::EFD>(b, it->nf, it->face_cell, it->face_code, it->face_xi, (const T *)it->u,
                                    (T *)it->fbuf, tab, it->sc);
}

template <typename T, int D, int N1>
__global__ __launch_bounds__(256) void dg_cell_batch_kernel(const BatchItem *__restrict__ items,
                                                            const int32_t *__restrict__ blk_item, KTab<T, N1> tab) {
  using S = BatchShape<T, D, N1>;
  const int g = xcd_block();
  const BatchItem *it = items + blk_item[g];
  const int b = g - it->blk0[1];
  const T scale = T(D == 3 ? it->sc.h : 1.0);
  dg_cell_body<T, D, N1, S::EC>(b, it->nc, it->nbr, (const T *)it->u, (const T *)it->fbuf, (T *)it->v, tab, it->sc,
                                scale, SBM_PART_ALL);
}

// Workgroups of each stage for one item (faces: 0 when the item's surrogate faces are computed
// elsewhere, i.e. by a truncated extension).
template <typename T, int D, int N1>
void batch_blocks_impl(const sbm_ctx *c, bool own_faces, int32_t nb[3]) {
  using S = BatchShape<T, D, N1>;
  const int64_t nf = own_faces ? c->n_sbm : 0;
  if (c->disc == SBM_CG) {
    nb[0] = (int32_t)((nf + S::EF - 1) / S::EF);
    nb[1] = (int32_t)c->n_bricks;
    nb[2] = (int32_t)((c->n_halo_dofs + kHaloPerThread * 256 - 1) / (kHaloPerThread * 256));
  } else {
    nb[0] = (int32_t)((nf + S::EFD - 1) / S::EFD);
    nb[1] = (int32_t)((c->n_cells + S::EC - 1) / S::EC);
    nb[2] = 0;
  }
}

template <typename T, int D, int N1>
hipError_t batch_launch_impl(const BatchGroup &g, const unsigned char *base, hipStream_t s) {
  using S = BatchShape<T, D, N1>;
  const KTab<T, N1> tab = make_ktab<T, N1>(g.first->rules);
  const BatchItem *items = reinterpret_cast<const BatchItem *>(base + g.off_items);
  const int32_t *bi[3];
  for (int k = 0; k < 3; ++k) bi[k] = reinterpret_cast<const int32_t *>(base + g.off_blk[k]);
  if (g.first->disc == SBM_CG) {
    if (g.nblk[0] > 0)
      hipLaunchKernelGGL((sbm_face_cg_batch_kernel<T, D, N1, S::EF>), dim3(g.nblk[0]), dim3(S::EF * S::NP), 0, s,
                         items, bi[0], tab);
    if (g.nblk[1] > 0)
      hipLaunchKernelGGL((brick_batch_kernel<T, D, N1>), dim3(g.nblk[1]), dim3(BrickCfg<T, D, N1>::NT), 0, s, items,
                         bi[1], tab);
    if (g.nblk[2] > 0)
      hipLaunchKernelGGL((halo_reduce_batch_kernel<T, D>), dim3(g.nblk[2]), dim3(256), 0, s, items, bi[2]);
  } else {
    if (g.nblk[0] > 0)
      hipLaunchKernelGGL((sbm_face_dg_batch_kernel<T, D, N1>), dim3(g.nblk[0]), dim3(S::TFD), 0, s, items, bi[0], tab);
    if (g.nblk[1] > 0) {
      if constexpr (S::PAR)
        hipLaunchKernelGGL((dg_cell_batch_kernel<T, D, N1>), dim3(g.nblk[1]), dim3(S::TC), 0, s, items, bi[1], tab);
      else
        hipLaunchKernelGGL((dg_cell_seq_kernel<T, D, N1, S::EC, true>), dim3(g.nblk[1]), dim3(S::TC), 0, s, 0,
                           (const int32_t *)nullptr, (const T *)nullptr, (const T *)nullptr, (T *)nullptr, tab, KScal{},
                           T(0), (int)SBM_PART_ALL, items, bi[1]);
    }
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Diagonal of A (for Jacobi preconditioning), one thread per (entity, local DoF):
//   cell:  h^(d-2) sum_k K_ii(axis k) prod_{m != k} M_ii(axis m)            (same every cell)
//   DG interior face (a, s) of K:  sum_q w_q (sigma_F psi_i^2 - psi_i dpsi_i/dn_K)
//   surrogate face:  sum_q w_q [ -dn psi_i psi_i(x~) - dn psi_i psi_i(x) + sigma psi_i(x) psi_i(x~) ]
// with psi_i(x~) on the face Gauss points and psi_i(x) at the shifted points.  Computed
// once per solve, so it uses plain loops and global atomics.
// ------------------------------------------------------------------------------------
template <typename T, int D, int N1>
__global__ void diag_cell_kernel(int n_cells, int disc_dg, const int32_t *__restrict__ runs,
                                 const int32_t *__restrict__ nbr, T *__restrict__ diag, KTab<T, N1> tab, KScal sc,
                                 T scale) {
  constexpr int NP = Shape<D, N1>::NP, NB = Shape<D, N1>::NB, P = N1 - 1;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= (int64_t)n_cells * NB) return;
  const int cell = (int)(gid / NB), i = (int)(gid % NB);
  const int ik[3] = {i % N1, (i / N1) % N1, (D == 3) ? i / (N1 * N1) : 0};
  double val = 0.0;
  for (int k = 0; k < D; ++k) {
    double t = tab.K[ik[k] * N1 + ik[k]];
    for (int m = 0; m < D; ++m)
      if (m != k) t *= tab.M[ik[m] * N1 + ik[m]];
    val += t;
  }
  val *= (double)scale;
  if (disc_dg) {
    const double h = sc.h;
    for (int code = 0; code < 2 * D; ++code) {
      if (nbr[(int64_t)cell * 2 * D + code] < 0) continue;
      const int a = code >> 1, s = code & 1;
      if (ik[a] != s * P) {
        // psi_i vanishes on this face: only the derivative term times psi_i = 0
        continue;
      }
      const double sgn = s ? 1.0 : -1.0;
      const double ds = s ? (double)tab.D1[ik[a]] : (double)tab.D0[ik[a]];
      for (int q = 0; q < NP; ++q) {
        const int qt[2] = {q % N1, (D == 3) ? q / N1 : 0};
        double tang = 1.0, om = 1.0;
        int t = 0;
        for (int m = 0; m < D; ++m) {
          if (m == a) continue;
          tang *= (double)tab.N[qt[t] * N1 + ik[m]];
          om *= (double)tab.w[qt[t]] * h;
          ++t;
        }
        val += om * (sc.sigma_f * tang * tang - tang * sgn / h * ds * tang);
      }
    }
    diag[(int64_t)cell * NB + i] = (T)val;
  } else {
    atomic_add(diag + runs[(int64_t)cell * NP + i / N1] + i % N1, (T)val);
  }
}

template <typename T, int D, int N1>
__global__ void diag_face_kernel(int n_faces, int disc_dg, const int32_t *__restrict__ face_cell,
                                 const int32_t *__restrict__ face_code, const double *__restrict__ face_xi,
                                 const int32_t *__restrict__ runs, T *__restrict__ diag, KTab<T, N1> tab, KScal sc) {
  constexpr int NP = Shape<D, N1>::NP, NB = Shape<D, N1>::NB, P = N1 - 1;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= (int64_t)n_faces * NB) return;
  const int f = (int)(gid / NB), i = (int)(gid % NB);
  const int cell = face_cell[f], code = face_code[f], a = code >> 1, s = code & 1;
  const int ik[3] = {i % N1, (i / N1) % N1, (D == 3) ? i / (N1 * N1) : 0};
  const double h = sc.h, sgn = s ? 1.0 : -1.0;
  const double ds = s ? (double)tab.D1[ik[a]] : (double)tab.D0[ik[a]];
  double val = 0.0;
  for (int q = 0; q < NP; ++q) {
    const int qt[2] = {q % N1, (D == 3) ? q / N1 : 0};
    double tang = 1.0, om = 1.0;
    int t = 0;
    for (int m = 0; m < D; ++m) {
      if (m == a) continue;
      tang *= (double)tab.N[qt[t] * N1 + ik[m]];
      om *= (double)tab.w[qt[t]] * h;
      ++t;
    }
    const double vt = (ik[a] == s * P) ? tang : 0.0;  // psi_i(x~_q)
    const double dn = sgn / h * ds * tang;            // d psi_i / dn~ (x~_q)
    double vs = 1.0;                                  // psi_i(x_q), shifted point
    const double *xq = face_xi + ((int64_t)f * NP + q) * D;
    for (int m = 0; m < D; ++m) {
      double l[N1];
      lagrange_at<N1>(tab.z, tab.cinv, xq[m], l);
      vs *= l[ik[m]];
    }
    val += om * (-dn * vt - dn * vs + sc.sigma_gamma * vs * vt);
  }
  const int64_t dof = disc_dg ? (int64_t)cell * NB + i : (int64_t)runs[(int64_t)cell * NP + i / N1] + i % N1;
  atomic_add(diag + dof, (T)val);
}

template <typename T, int D, int N1>
hipError_t diag_impl(const sbm_ctx *c, T *diag, hipStream_t s) {
  constexpr int NB = Shape<D, N1>::NB;
  const KTab<T, N1> tab = make_ktab<T, N1>(c->rules);
  const KScal sc{c->h, c->sigma_gamma, c->sigma_f};
  const T scale = T(D == 3 ? c->h : 1.0);
  const int dg = c->disc == SBM_DG;
  hipError_t e = vec_fill(diag, c->n_dofs, 0.0, sizeof(T) == 8 ? SBM_F64 : SBM_F32, s);
  if (e != hipSuccess) return e;
  const int64_t nc = c->n_cells * NB, nf = c->n_sbm * NB;
  if (nc > 0)
    hipLaunchKernelGGL((diag_cell_kernel<T, D, N1>), dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s,
                       (int)c->n_cells, dg, c->d_runs, c->d_nbr, diag, tab, sc, scale);
  if (nf > 0)
    hipLaunchKernelGGL((diag_face_kernel<T, D, N1>), dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s,
                       (int)c->n_sbm, dg, c->d_face_cell, c->d_face_code, c->d_face_xi, c->d_runs, diag, tab, sc);
  return hipGetLastError();
}

template <typename T, int D>
hipError_t diag_dim(const sbm_ctx *c, T *diag, hipStream_t s) {
  switch (c->p) {
    case 1: return diag_impl<T, D, 2>(c, diag, s);
    case 2: return diag_impl<T, D, 3>(c, diag, s);
    case 3: return diag_impl<T, D, 4>(c, diag, s);
    case 4: return diag_impl<T, D, 5>(c, diag, s);
    case 5: return diag_impl<T, D, 6>(c, diag, s);
    case 6: return diag_impl<T, D, 7>(c, diag, s);
    case 7: return diag_impl<T, D, 8>(c, diag, s);
    case 8: return diag_impl<T, D, 9>(c, diag, s);
  }
  return hipErrorInvalidValue;
}

#define SBM_P_SWITCH(P_, CALL)     \
  switch (P_) {                    \
    case 1: return CALL(2);        \
    case 2: return CALL(3);        \
    case 3: return CALL(4);        \
    case 4: return CALL(5);        \
    case 5: return CALL(6);        \
    case 6: return CALL(7);        \
    case 7: return CALL(8);        \
    case 8: return CALL(9);        \
  }

template <typename T, int D>
bool batch_blocks_dim(const sbm_ctx *c, bool own_faces, int32_t nb[3]) {
#define SBM_BB(N1_) (batch_blocks_impl<T, D, N1_>(c, own_faces, nb), true)
  SBM_P_SWITCH(c->p, SBM_BB)
#undef SBM_BB
  return false;
}

template <typename T, int D>
hipError_t batch_launch_dim(const BatchGroup &g, const unsigned char *base, hipStream_t s) {
#define SBM_BL(N1_) batch_launch_impl<T, D, N1_>(g, base, s)
  SBM_P_SWITCH(g.first->p, SBM_BL)
#undef SBM_BL
  return hipErrorInvalidValue;
}
#undef SBM_P_SWITCH

template <typename T, int D>
hipError_t apply_dim(const sbm_ctx *c, const T *u, T *v, int parts, hipStream_t s, const Scratch &scr) {
  switch (c->p) {
    case 1: return apply_impl<T, D, 2>(c, u, v, parts, s, scr);
    case 2: return apply_impl<T, D, 3>(c, u, v, parts, s, scr);
    case 3: return apply_impl<T, D, 4>(c, u, v, parts, s, scr);
    case 4: return apply_impl<T, D, 5>(c, u, v, parts, s, scr);
    case 5: return apply_impl<T, D, 6>(c, u, v, parts, s, scr);
    case 6: return apply_impl<T, D, 7>(c, u, v, parts, s, scr);
    case 7: return apply_impl<T, D, 8>(c, u, v, parts, s, scr);
    case 8: return apply_impl<T, D, 9>(c, u, v, parts, s, scr);
  }
  return hipErrorInvalidValue;
}

}  // namespace

void brick_dims(int dim, int p, int *bx, int *by, int *bz) {
#define SBM_BD(D_, P_)                  \
  if (dim == D_ && p == P_) {           \
    *bx = BrickDims<D_, P_>::BX;        \
    *by = BrickDims<D_, P_>::BY;        \
    *bz = BrickDims<D_, P_>::BZ;        \
    return;                             \
  }
  SBM_BD(2, 1) SBM_BD(2, 2) SBM_BD(2, 3) SBM_BD(2, 4) SBM_BD(2, 5) SBM_BD(2, 6) SBM_BD(2, 7) SBM_BD(2, 8)
  SBM_BD(3, 1) SBM_BD(3, 2) SBM_BD(3, 3) SBM_BD(3, 4) SBM_BD(3, 5) SBM_BD(3, 6) SBM_BD(3, 7) SBM_BD(3, 8)
#undef SBM_BD
  *bx = *by = *bz = 1;
}

hipError_t launch_diagonal(const sbm_ctx *c, void *diag, int prec, hipStream_t s) {
  if (prec == SBM_F64)
    return c->dim == 3 ? diag_dim<double, 3>(c, (double *)diag, s) : diag_dim<double, 2>(c, (double *)diag, s);
  return c->dim == 3 ? diag_dim<float, 3>(c, (float *)diag, s) : diag_dim<float, 2>(c, (float *)diag, s);
}

size_t apply_scratch_bytes(const sbm_ctx *c, int prec) {
  const size_t s = prec == SBM_F64 ? sizeof(double) : sizeof(float);
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t halo = c->disc == SBM_CG ? ((size_t)1 << c->dim) * (size_t)c->n_halo_dofs * s : 0;
  const size_t fbuf = (size_t)c->n_sbm * 2 * (size_t)c->nq_face * s;
  return up(halo) + up(fbuf);
}

hipError_t batch_group_build(BatchGroup &g, const std::vector<const sbm_ctx *> &cs,
                             const std::vector<const void *> &u, const std::vector<void *> &v,
                             const std::vector<int> &own_faces, std::vector<unsigned char> &image) {
  const sbm_ctx *c0 = cs.empty() ? nullptr : cs[0];
  if (!c0 || u.size() != cs.size() || v.size() != cs.size() || own_faces.size() != cs.size())
    return hipErrorInvalidValue;
  g.first = c0;
  g.n_items = (int)cs.size();
  std::vector<BatchItem> items(cs.size());
  std::vector<int32_t> blk[3];
  int64_t tot[3] = {0, 0, 0};
  for (size_t i = 0; i < cs.size(); ++i) {
    const sbm_ctx *c = cs[i];
    if (c->disc != c0->disc || c->dim != c0->dim || c->p != c0->p) return hipErrorInvalidValue;
    int32_t nb[3] = {0, 0, 0};
    const bool ok = g.prec == SBM_F64 ? (c->dim == 3 ? batch_blocks_dim<double, 3>(c, own_faces[i] != 0, nb)
                                                     : batch_blocks_dim<double, 2>(c, own_faces[i] != 0, nb))
                                      : (c->dim == 3 ? batch_blocks_dim<float, 3>(c, own_faces[i] != 0, nb)
                                                     : batch_blocks_dim<float, 2>(c, own_faces[i] != 0, nb));
    if (!ok) return hipErrorInvalidValue;
    BatchItem &it = items[i];
    it.br = BrickArgs{c->d_brick_cell_off, c->d_brick_runs, c->d_brick_cell_loc, c->d_brick_face_off,
                      c->d_brick_face_loc, c->d_face_code,  c->d_row_base,       c->d_row_gmask,
                      c->d_row_bmask,      c->d_row_hbase};
    it.face_code = c->d_face_code;
    it.face_runs = c->d_face_runs;
    it.face_cell = c->d_face_cell;
    it.nbr = c->d_nbr;
    it.halo_dof = c->d_halo_dof;
    it.halo_mask = c->d_halo_mask;
    it.face_xi = c->d_face_xi;
    it.u = u[i];
    it.v = v[i];
    it.fbuf = c->d_fbuf;
    it.halo = c->d_halo;
    it.sc = KScal{c->h, c->sigma_gamma, c->sigma_f};
    it.nf = (int)c->n_sbm;
    it.nc = (int)c->n_cells;
    it.nh = (int)c->n_halo_dofs;
    for (int k = 0; k < 3; ++k) {
      it.blk0[k] = (int)tot[k];
      blk[k].insert(blk[k].end(), (size_t)nb[k], (int32_t)i);
      tot[k] += nb[k];
      if (tot[k] > INT32_MAX / 2) return hipErrorInvalidValue;
    }
  }
  auto put = [&image](const void *src, size_t bytes) {
    const size_t off = (image.size() + 255) / 256 * 256;
    image.resize(off + std::max<size_t>(bytes, 4));
    if (bytes) std::memcpy(image.data() + off, src, bytes);
    return off;
  };
  g.off_items = put(items.data(), items.size() * sizeof(BatchItem));
  for (int k = 0; k < 3; ++k) {
    g.nblk[k] = (int)tot[k];
    g.off_blk[k] = put(blk[k].data(), blk[k].size() * sizeof(int32_t));
  }
  return hipSuccess;
}

hipError_t launch_batch_group(const BatchGroup &g, const void *base, hipStream_t s) {
  const unsigned char *b = static_cast<const unsigned char *>(base);
  if (g.prec == SBM_F64)
    return g.first->dim == 3 ? batch_launch_dim<double, 3>(g, b, s) : batch_launch_dim<double, 2>(g, b, s);
  return g.first->dim == 3 ? batch_launch_dim<float, 3>(g, b, s) : batch_launch_dim<float, 2>(g, b, s);
}

hipError_t launch_apply(const sbm_ctx *c, const void *u, void *v, int prec, int parts, hipStream_t s,
                        const Scratch *scr) {
  Scratch use;
  use.halo = (scr && scr->halo) ? scr->halo : c->d_halo;
  use.fbuf = (scr && scr->fbuf) ? scr->fbuf : c->d_fbuf;
  if (prec == SBM_F64) {
    return c->dim == 3 ? apply_dim<double, 3>(c, (const double *)u, (double *)v, parts, s, use)
                       : apply_dim<double, 2>(c, (const double *)u, (double *)v, parts, s, use);
  }
  return c->dim == 3 ? apply_dim<float, 3>(c, (const float *)u, (float *)v, parts, s, use)
                     : apply_dim<float, 2>(c, (const float *)u, (float *)v, parts, s, use);
}

}  // namespace sbm
