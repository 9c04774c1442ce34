// Right-hand side, batched applies and the Krylov solvers around the operator.
//
// The SBM operator of Eq. (1) is nonsymmetric (the extension E acts on the trial side
// only) and, with full polynomial extrapolation, indefinite, so the default solver is
// restarted GMRES(m) with classical Gram-Schmidt and one re-orthogonalisation pass
// (CGS2).  A step is the operator apply and three Gram-Schmidt kernels, each one pass over
// the row-tiled basis (products; update fused with the next products; update fused with the
// norm and the Givens rotation update), so the host reads back only a residual estimate every
// few steps.  The mixed-precision mode runs GMRES on the FP32 operator inside FP64 iterative
// refinement: the outer residual r = b - A x, its norm and the update x += c are FP64 on the
// device.  Reductions are block partial sums added in a fixed order, so a solve is
// deterministic given a deterministic apply.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <thread>
#include <type_traits>
#include <vector>

#include "sbm_internal.h"

namespace sbm {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 1024;
constexpr int kMaxRestart = 256;  // longest GMRES restart (basis columns)
// The GMRES basis is stored in row tiles: the m1 columns of rows [128 t, 128 t + 128) are one
// contiguous block (column i at offset 128 i), so a sweep over a range of rows and all columns
// streams contiguous memory.
constexpr int kTile = 128;
__host__ __device__ __forceinline__ int64_t tile_ix(int64_t k, int i, int m1) {
  return ((k / kTile) * m1 + i) * kTile + (k % kTile);
}

inline int nblocks(int64_t n) {
  int64_t b = (n + kThreads * 8 - 1) / (kThreads * 8);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMaxBlocks));
}

// partial[blk * ncol + i] = sum over this block's entries of V_i . w  (i < ncol)
template <typename T, int NCOL_MAX>
__global__ __launch_bounds__(kThreads) void multidot_kernel(const T *__restrict__ V, int64_t ld, int ncol,
                                                            const T *__restrict__ w, int64_t n,
                                                            double *__restrict__ partial) {
  __shared__ double red[kThreads / 64][NCOL_MAX];
  double acc[NCOL_MAX];
#pragma unroll
  for (int i = 0; i < NCOL_MAX; ++i) acc[i] = 0.0;
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads) {
    const double wk = (double)w[k];
#pragma unroll
    for (int i = 0; i < NCOL_MAX; ++i)
      if (i < ncol) acc[i] += (double)V[i * ld + k] * wk;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NCOL_MAX; ++i) {
    if (i >= ncol) break;
    double s = acc[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) red[wave][i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ncol; i += kThreads) {
    double s = 0.0;
    for (int wv = 0; wv < kThreads / 64; ++wv) s += red[wv][i];
    partial[(int64_t)blockIdx.x * ncol + i] = s;
  }
}

// out[i] = sum_b partial[b * ncol + i], fixed order
__global__ void reduce_partials_kernel(const double *__restrict__ partial, int nblk, int ncol,
                                       double *__restrict__ out) {
  const int i = threadIdx.x;
  if (i >= ncol) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * ncol + i];
  out[i] = s;
}

// x += sum_i y[i] Z_i  (Z_i = V_i of the tiled basis with m1 columns, optionally scaled by
// dinv), y on the device
template <typename T>
__global__ void update_kernel(const T *__restrict__ V, int m1, int ncol, const double *__restrict__ y,
                              const T *__restrict__ dinv, T *__restrict__ x, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads) {
    double s = 0.0;
    const int64_t base = tile_ix(k, 0, m1);
#pragma unroll 8
    for (int i = 0; i < ncol; ++i) s += y[i] * (double)V[base + (int64_t)i * kTile];
    if (dinv) s *= (double)dinv[k];
    x[k] = (T)((double)x[k] + s);
  }
}

// r = b - v
template <typename T>
__global__ void residual_kernel(const T *__restrict__ b, const T *__restrict__ v, T *__restrict__ r, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads)
    r[k] = b[k] - v[k];
}

// z = dinv .* v
template <typename T>
__global__ void diag_scale_kernel(const T *__restrict__ dinv, const T *__restrict__ v, T *__restrict__ z, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads)
    z[k] = dinv[k] * v[k];
}

// r32 = (float)(r64 / nrm)
__global__ void to_f32_kernel(const double *__restrict__ r, const double *__restrict__ nrm2, float *__restrict__ o,
                              int64_t n) {
  const double inv = 1.0 / sqrt(*nrm2);
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads)
    o[k] = (float)(r[k] * inv);
}

// x64 += sqrt(nrm2) * c32
__global__ void add_f32_kernel(const float *__restrict__ c, const double *__restrict__ nrm2, double *__restrict__ x,
                               int64_t n) {
  const double s = sqrt(*nrm2);
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads)
    x[k] += s * (double)c[k];
}

__global__ void invert_kernel(double *__restrict__ d, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads)
    d[k] = d[k] != 0.0 ? 1.0 / d[k] : 0.0;
}

__global__ void cast_f64_f32_kernel(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads)
    b[k] = (float)a[k];
}

__global__ void fill_f32_kernel(float *__restrict__ a, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads)
    a[k] = 0.0f;
}

template <typename T>
__global__ void copy_kernel(const T *__restrict__ a, T *__restrict__ b, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads)
    b[k] = a[k];
}

// ---- conjugate gradients: three fused kernels per iteration besides the apply, scalars in
// FP64 on the device, reductions as block partials summed in a fixed order ----

// Sum of the nblk block partials in a fixed order; every thread (and every block, since all
// blocks run the same code on the same data) gets the identical value.
__device__ __forceinline__ double block_sum(const double *__restrict__ part, int nblk) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) s += part[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double tot = red[0];
  __syncthreads();
  return tot;
}

// part[blockIdx.x] = sum of acc over the block (fixed order)
__device__ __forceinline__ void block_partial(double acc, double *__restrict__ part) {
  __shared__ double red[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
    part[blockIdx.x] = s;
  }
}

// r = rhs - q, p = r; partials of |r|^2
template <typename T>
__global__ __launch_bounds__(kThreads) void cg_init_kernel(const T *__restrict__ rhs, const T *__restrict__ q,
                                                           T *__restrict__ r, T *__restrict__ p,
                                                           double *__restrict__ part, int64_t n) {
  double acc = 0.0;
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads) {
    const T rk = rhs[k] - q[k];
    r[k] = rk;
    p[k] = rk;
    acc += (double)rk * (double)rk;
  }
  block_partial(acc, part);
}

// partials of p . q
template <typename T>
__global__ __launch_bounds__(kThreads) void cg_dot_kernel(const T *__restrict__ p, const T *__restrict__ q,
                                                          double *__restrict__ part, int64_t n) {
  double acc = 0.0;
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads)
    acc += (double)p[k] * (double)q[k];
  block_partial(acc, part);
}

// alpha = |r|^2 / (p . q); x += alpha p; r -= alpha q; partials of the new |r|^2 (x may be
// kept in a wider type than the other vectors)
template <typename T, typename TX = T>
__global__ __launch_bounds__(kThreads) void cg_update_kernel(TX *__restrict__ x, T *__restrict__ r,
                                                             const T *__restrict__ p, const T *__restrict__ q,
                                                             const double *__restrict__ rr,
                                                             const double *__restrict__ part_pq, int nblk,
                                                             double *__restrict__ part_rr, int64_t n) {
  const double alpha = *rr / block_sum(part_pq, nblk);
  double acc = 0.0;
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads) {
    x[k] = (TX)((double)x[k] + alpha * (double)p[k]);
    const T rk = (T)((double)r[k] - alpha * (double)q[k]);
    r[k] = rk;
    acc += (double)rk * (double)rk;
  }
  block_partial(acc, part_rr);
}

// beta = |r_new|^2 / |r|^2; p = r + beta p; |r_new|^2 stored for the next iteration
template <typename T>
__global__ __launch_bounds__(kThreads) void cg_dir_kernel(T *__restrict__ p, const T *__restrict__ r,
                                                          const double *__restrict__ rr,
                                                          const double *__restrict__ part_rr, int nblk,
                                                          double *__restrict__ rr_new, int64_t n) {
  const double rn = block_sum(part_rr, nblk);
  const double beta = rn / *rr;
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads)
    p[k] = (T)((double)r[k] + beta * (double)p[k]);
  if (blockIdx.x == 0 && threadIdx.x == 0) *rr_new = rn;
}

// Arnoldi step j of restarted GMRES, done by one thread: column j of the Hessenberg matrix
// (H, (m+1) x m, row-major with row stride m) from the two projection passes h1, h2 and the
// squared norm nrm2 of the orthogonalised vector, the rotations of steps < j applied to it, the
// new Givens rotation (cs, sn), the rotated right-hand side g, the residual estimate
// |g_(j+1)| in res[j] (-1 on breakdown), and the factor 1 / h_(j+1,j) (0 on breakdown) that
// normalises the next basis vector.
struct ArnoldiArgs {
  int j, m;
  const double *h1, *h2;
  double *H, *cs, *sn, *g, *res, *fac;
};

__device__ void arnoldi_step(const ArnoldiArgs &a, double nrm2) {
  const int j = a.j, m = a.m;
  double *H = a.H;
  for (int i = 0; i <= j; ++i) H[(int64_t)i * m + j] = a.h1[i] + a.h2[i];
  const double hn = sqrt(nrm2);
  *a.fac = hn > 0.0 ? 1.0 / hn : 0.0;
  for (int i = 0; i < j; ++i) {
    const double x = H[(int64_t)i * m + j], y = H[(int64_t)(i + 1) * m + j];
    H[(int64_t)i * m + j] = a.cs[i] * x + a.sn[i] * y;
    H[(int64_t)(i + 1) * m + j] = -a.sn[i] * x + a.cs[i] * y;
  }
  const double x = H[(int64_t)j * m + j], y = hn;
  const double rr = hypot(x, y);
  a.cs[j] = rr > 0.0 ? x / rr : 1.0;
  a.sn[j] = rr > 0.0 ? y / rr : 0.0;
  H[(int64_t)j * m + j] = rr;
  a.g[j + 1] = -a.sn[j] * a.g[j];
  a.g[j] = a.cs[j] * a.g[j];
  a.res[j] = rr > 0.0 ? fabs(a.g[j + 1]) : -1.0;
}

// Sum of p[0 .. nblk) (nblk <= kMaxBlocks) by the 64 lanes of one wave in a fixed order:
// lane l adds p[l + 64 j] over j (all loads issued at once, from clamped indices), then a
// shuffle tree; the result is valid in lane 0.
__device__ __forceinline__ double wave_sum(const double *__restrict__ p, int nblk, int lane) {
  constexpr int NJ = kMaxBlocks / 64;
  double v[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) v[j] = p[lane + 64 * j < nblk ? lane + 64 * j : 0];
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < NJ; ++j) s += lane + 64 * j < nblk ? v[j] : 0.0;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  return s;
}

// One Gram-Schmidt kernel of a GMRES step, in a single launch:
//   MODE 0: out = V^T w                                  (ncol columns of V)
//   MODE 1: w -= V coef, then out = V^T w
//   MODE 2: w -= V coef, then out[0] = w . w and the Arnoldi step (arnoldi_step)
// V is the tiled basis (tile_ix, m1 columns).
// Layout: lane l of a wave takes rows l, l + 64, ..., l + 64 (R - 1) of each 64 R-row block
// (coalesced column reads, R CPW loads in flight per lane); wave q of the 4 owns columns
// q, q + 4, ... (at most CPW each).  The update sums the four waves' partial products in wave
// order through LDS; the values of V read for it are reused from registers for the products
// that follow, so V is read once per launch.  Every block writes its partial sums (column i of
// block b at partial[i kMaxBlocks + b]); the last block to finish (ticket on *counter, which it
// resets to 0 for the next launch) adds them in a fixed order, so the result is independent of
// the block schedule.
template <typename T, int CPW, int MODE, bool TICKET = true>
__device__ __forceinline__ void gs_body(const int blk, const int nblk, const T *__restrict__ V, int m1, int ncol,
                                        const double *__restrict__ coef, T *__restrict__ w, int64_t n,
                                        double *__restrict__ partial, unsigned *__restrict__ counter,
                                        double *__restrict__ out, const ArnoldiArgs &aa) {
  constexpr int NW = kThreads / 64, R = 32 / CPW;
  __shared__ double red[MODE == 0 ? 1 : NW][64 * R];
  __shared__ bool last;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[CPW], cf[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int i = wave + NW * c;
    acc[c] = 0.0;
    cf[c] = (MODE != 0 && i < ncol) ? coef[i] : 0.0;
  }
  for (int64_t r0 = (int64_t)blk * 64 * R; r0 < n; r0 += (int64_t)nblk * 64 * R) {
    // unconditional loads from a clamped index (entry 0 outside the range), masked after the
    // conversion: no branch separates a load from the next, so all of them are in flight at once
    T tv[R][CPW], tw[R];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int64_t k = r0 + rr * 64 + lane;
      const bool ok = k < n;
      const int64_t base = tile_ix(ok ? k : 0, 0, m1);
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int i = wave + NW * c;
        tv[rr][c] = V[(ok && i < ncol) ? base + (int64_t)i * kTile : 0];
      }
      tw[rr] = w[ok ? k : 0];
    }
    double v[R][CPW], wv[R];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const bool ok = r0 + rr * 64 + lane < n;
#pragma unroll
      for (int c = 0; c < CPW; ++c) v[rr][c] = (ok && wave + NW * c < ncol) ? (double)tv[rr][c] : 0.0;
      wv[rr] = ok ? (double)tw[rr] : 0.0;
    }
    if constexpr (MODE != 0) {
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        double sp = 0.0;
#pragma unroll
        for (int c = 0; c < CPW; ++c) sp += cf[c] * v[rr][c];
        red[wave][rr * 64 + lane] = sp;
      }
      __syncthreads();
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int64_t k = r0 + rr * 64 + lane;
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) sum += red[q][rr * 64 + lane];
        const T t = (T)(wv[rr] - sum);
        if (wave == 0 && k < n) w[k] = t;
        wv[rr] = k < n ? (double)t : 0.0;
      }
      __syncthreads();  // red is rewritten by the next row block
    }
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      if constexpr (MODE == 2) {
        acc[0] += wv[rr] * wv[rr];
      } else {
#pragma unroll
        for (int c = 0; c < CPW; ++c) acc[c] += v[rr][c] * wv[rr];
      }
    }
  }
  // block partials: column i = wave + NW c (MODE 2: wave 0's sum as column 0)
  const int nout = MODE == 2 ? 1 : ncol;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int i = wave + NW * c;
    double sacc = acc[c];
    for (int off = 32; off > 0; off >>= 1) sacc += __shfl_down(sacc, off, 64);
    const bool mine = MODE == 2 ? (c == 0 && wave == 0) : i < ncol;
    if (lane == 0 && mine) partial[(int64_t)i * kMaxBlocks + blk] = sacc;
  }
  if constexpr (!TICKET) return;  // the partials are summed by a later launch (gs_reduce_batch_kernel)
  __syncthreads();  // the block's partials are written (each wave waited for its stores)
  if (threadIdx.x == 0) {
    __threadfence();  // release: the partials before the ticket
    last = atomicAdd(counter, 1u) == (unsigned)(nblk - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();  // acquire: the other blocks' partials
    if constexpr (MODE == 2) {
    if (wave == 0) {
      const double sum = wave_sum(partial, nblk, lane);
      if (lane == 0) {
        *out = sum;
        arnoldi_step(aa, sum);
        *counter = 0u;
      }
    }
  } else {
    for (int i = wave; i < nout; i += NW) {
      const double sum = wave_sum(partial + (int64_t)i * kMaxBlocks, nblk, lane);
      if (lane == 0) out[i] = sum;
    }
    if (threadIdx.x == 0) *counter = 0u;
  }
}

template <typename T, int CPW, int MODE>
__global__ __launch_bounds__(kThreads) void gs_kernel(const T *__restrict__ V, int m1, int ncol,
                                                      const double *__restrict__ coef, T *__restrict__ w, int64_t n,
                                                      double *__restrict__ partial, unsigned *__restrict__ counter,
                                                      double *__restrict__ out, ArnoldiArgs aa) {
  gs_body<T, CPW, MODE>(blockIdx.x, gridDim.x, V, m1, ncol, coef, w, n, partial, counter, out, aa);
}

// The Gram-Schmidt kernels for more than 64 columns: the columns are taken in chunks of 64
// (wave q of the 4 owns chunk columns q, q + 4, ...), with the same row layout, partial
// layout and last-block reduction as gs_kernel.  MODE 0: one sweep per chunk.  MODE 1: a
// sweep for w -= V coef over all chunks (the block's new w values are its own rows, read back
// after a barrier), then one sweep per chunk for the products: V is read twice.  MODE 2: one
// sweep (update and norm).
template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void gs_wide_kernel(const T *__restrict__ V, int m1, int ncol,
                                                           const double *__restrict__ coef, T *__restrict__ w,
                                                           int64_t n, double *__restrict__ partial,
                                                           unsigned *__restrict__ counter, double *__restrict__ out,
                                                           ArnoldiArgs aa) {
  constexpr int NW = kThreads / 64, CPW = 16, R = 2, CH = NW * CPW;
  __shared__ double red[NW][64 * R];
  __shared__ bool last;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nch = (ncol + CH - 1) / CH;
  const int64_t stride = (int64_t)gridDim.x * 64 * R;
  // products of the chunk columns with the current w over this block's rows -> partials
  auto products = [&](int ch) {
    double acc[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) acc[c] = 0.0;
    for (int64_t r0 = (int64_t)blockIdx.x * 64 * R; r0 < n; r0 += stride) {
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int64_t k = r0 + rr * 64 + lane;
        const bool ok = k < n;
        const int64_t base = tile_ix(ok ? k : 0, 0, m1);
        const double wk = ok ? (double)w[k] : 0.0;
        T tv[CPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          const int i = ch * CH + wave + NW * c;
          tv[c] = V[(ok && i < ncol) ? base + (int64_t)i * kTile : 0];
        }
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          const int i = ch * CH + wave + NW * c;
          acc[c] += (ok && i < ncol) ? (double)tv[c] * wk : 0.0;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int i = ch * CH + wave + NW * c;
      double sacc = acc[c];
      for (int off = 32; off > 0; off >>= 1) sacc += __shfl_down(sacc, off, 64);
      if (lane == 0 && i < ncol) partial[(int64_t)i * kMaxBlocks + blockIdx.x] = sacc;
    }
  };
  if constexpr (MODE == 0) {
    for (int ch = 0; ch < nch; ++ch) products(ch);
  } else {
    double nrm = 0.0;
    for (int64_t r0 = (int64_t)blockIdx.x * 64 * R; r0 < n; r0 += stride) {
      double sp[R];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) sp[rr] = 0.0;
      for (int ch = 0; ch < nch; ++ch) {
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          const int64_t k = r0 + rr * 64 + lane;
          const bool ok = k < n;
          const int64_t base = tile_ix(ok ? k : 0, 0, m1);
          T tv[CPW];
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            const int i = ch * CH + wave + NW * c;
            tv[c] = V[(ok && i < ncol) ? base + (int64_t)i * kTile : 0];
          }
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            const int i = ch * CH + wave + NW * c;
            sp[rr] += (ok && i < ncol) ? coef[i] * (double)tv[c] : 0.0;
          }
        }
      }
#pragma unroll
      for (int rr = 0; rr < R; ++rr) red[wave][rr * 64 + lane] = sp[rr];
      __syncthreads();
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int64_t k = r0 + rr * 64 + lane;
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) sum += red[q][rr * 64 + lane];
        if (wave == 0 && k < n) {  // wave 0 alone reads and writes w here
          const T t = (T)((double)w[k] - sum);
          w[k] = t;
          nrm += (double)t * (double)t;
        }
      }
      __syncthreads();  // red is rewritten by the next row block; the block's new w rows are written
    }
    if constexpr (MODE == 1) {
      for (int ch = 0; ch < nch; ++ch) products(ch);
    } else {
      for (int off = 32; off > 0; off >>= 1) nrm += __shfl_down(nrm, off, 64);
      if (lane == 0 && wave == 0) partial[blockIdx.x] = nrm;
    }
  }
  __syncthreads();  // the block's partials are written (each wave waited for its stores)
  if (threadIdx.x == 0) {
    __threadfence();  // release: the partials before the ticket
    last = atomicAdd(counter, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();  // acquire: the other blocks' partials
  const int nblk = gridDim.x;
  if constexpr (MODE == 2) {
    if (wave == 0) {
      const double sum = wave_sum(partial, nblk, lane);
      if (lane == 0) {
        *out = sum;
        arnoldi_step(aa, sum);
        *counter = 0u;
      }
    }
  } else {
    for (int i = wave; i < ncol; i += NW) {
      const double sum = wave_sum(partial + (int64_t)i * kMaxBlocks, nblk, lane);
      if (lane == 0) out[i] = sum;
    }
    if (threadIdx.x == 0) *counter = 0u;
  }
}

// g = (sqrt(*nrm2), 0, ..., 0), m + 1 entries
__global__ void gmres_init_kernel(const double *__restrict__ nrm2, double *__restrict__ g, int m) {
  for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = i == 0 ? sqrt(*nrm2) : 0.0;
}

// y = R^-1 g for the leading j x j upper triangle R of H, by one thread; for j <= 64 the
// triangle and g are first staged in LDS by the whole block (the same operations in the same
// order, without a global-memory round trip per term)
constexpr int kBacksubLds = 64;
__device__ void backsub_body(int j, int m, const double *__restrict__ H, const double *__restrict__ g,
                             double *__restrict__ y) {
  __shared__ double sH[kBacksubLds * kBacksubLds], sg[kBacksubLds], sy[kBacksubLds];
  if (j <= kBacksubLds) {
    for (int t = threadIdx.x; t < j * j; t += blockDim.x) sH[t] = H[(int64_t)(t / j) * m + t % j];
    for (int t = threadIdx.x; t < j; t += blockDim.x) sg[t] = g[t];
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int i = j - 1; i >= 0; --i) {
        double s = sg[i];
        for (int k = i + 1; k < j; ++k) s -= sH[i * j + k] * sy[k];
        const double d = sH[i * j + i];
        sy[i] = d != 0.0 ? s / d : 0.0;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < j; t += blockDim.x) y[t] = sy[t];
    return;
  }
  if (threadIdx.x != 0) return;
  for (int i = j - 1; i >= 0; --i) {
    double s = g[i];
    for (int k = i + 1; k < j; ++k) s -= H[(int64_t)i * m + k] * y[k];
    const double d = H[(int64_t)i * m + i];
    y[i] = d != 0.0 ? s / d : 0.0;
  }
}

__global__ void backsub_kernel(int j, int m, const double *__restrict__ H, const double *__restrict__ g,
                               double *__restrict__ y) {
  backsub_body(j, m, H, g, y);
}

// Basis vector col = x * f, stored in column col of the tiled basis V (m1 columns) and in the
// contiguous vector vc (the next operator input); f = *fac, or 1 / sqrt(*fac) if inv_sqrt.
template <typename T>
__global__ void basis_store_kernel(const T *__restrict__ x, const double *__restrict__ fac, int inv_sqrt,
                                   T *__restrict__ V, int col, int m1, T *__restrict__ vc, int64_t n) {
  const double f = inv_sqrt ? 1.0 / sqrt(*fac) : *fac;
  for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads) {
    const T y = (T)((double)x[k] * f);
    V[tile_ix(k, col, m1)] = y;
    vc[k] = y;
  }
}

// ---- the orthogonalisation of a step for several GMRES runs at once (lockstep batches):
// workgroup g of a launch serves the run blk_item[g] with its own block index and its own
// block count, the ones the run's single launch would have, so every run's reductions are
// summed exactly as in its own solve ----
constexpr int kOrthoKinds = 13;  // 4 column classes (2, 4, 8, 16 columns per wave) x 3 modes, basis store
struct OrthoItem {
  void *V, *w, *vc, *x;
  int64_t n;
  int m1, m;
  double *partial;
  unsigned *counter;
  double *h1, *h2, *hn, *y;
  double *H, *cs, *sn, *g, *res, *fac;
  int blk0[kOrthoKinds], nblk[kOrthoKinds];
};

template <typename T, int CPW, int MODE>
__global__ __launch_bounds__(kThreads) void gs_batch_kernel(const OrthoItem *__restrict__ items,
                                                            const int32_t *__restrict__ blk_item, int ncol, int k) {
  constexpr int L = CPW == 2 ? 0 : (CPW == 4 ? 1 : (CPW == 8 ? 2 : 3)), KIND = 3 * L + MODE;
  const int g = blockIdx.x;
  const OrthoItem *it = items + blk_item[g];
  const ArnoldiArgs aa{k, it->m, it->h1, it->h2, it->H, it->cs, it->sn, it->g, it->res, it->fac};
  const double *coef = MODE == 0 ? nullptr : (MODE == 1 ? it->h1 : it->h2);
  double *out = MODE == 0 ? it->h1 : (MODE == 1 ? it->h2 : it->hn);
  gs_body<T, CPW, MODE, false>(g - it->blk0[KIND], it->nblk[KIND], (const T *)it->V, it->m1, ncol, coef, (T *)it->w,
                               it->n, it->partial, it->counter, out, aa);
}

// The sums of the block partials of a batched Gram-Schmidt launch, one workgroup per run:
// exactly the last-block sums of gs_body (same partials, same order); MODE 2 also does the
// run's Arnoldi step.
template <int CPW, int MODE>
__global__ __launch_bounds__(kThreads) void gs_reduce_batch_kernel(const OrthoItem *__restrict__ items, int ncol,
                                                                   int k) {
  constexpr int L = CPW == 2 ? 0 : (CPW == 4 ? 1 : (CPW == 8 ? 2 : 3)), KIND = 3 * L + MODE, NW = kThreads / 64;
  const OrthoItem *it = items + blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nblk = it->nblk[KIND];
  if constexpr (MODE == 2) {
    if (wave == 0) {
      const double sum = wave_sum(it->partial, nblk, lane);
      if (lane == 0) {
        *it->hn = sum;
        const ArnoldiArgs aa{k, it->m, it->h1, it->h2, it->H, it->cs, it->sn, it->g, it->res, it->fac};
        arnoldi_step(aa, sum);
      }
    }
  } else {
    double *out = MODE == 0 ? it->h1 : it->h2;
    for (int i = wave; i < ncol; i += NW) {
      const double sum = wave_sum(it->partial + (int64_t)i * kMaxBlocks, nblk, lane);
      if (lane == 0) out[i] = sum;
    }
  }
}

// The end of a restart cycle for several runs: y = R^-1 g (one workgroup per run, ncol[i]
// columns), then x += V y (workgroups of the basis-store table); and the residual estimates
// res[j0 .. j0 + cnt) of every run gathered into out (run i at out[i * cnt]).
__global__ __launch_bounds__(kThreads) void backsub_batch_kernel(const OrthoItem *__restrict__ items,
                                                                 const int *__restrict__ ncol) {
  const OrthoItem *it = items + blockIdx.x;
  backsub_body(ncol[blockIdx.x], it->m, it->H, it->g, it->y);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void update_batch_kernel(const OrthoItem *__restrict__ items,
                                                                const int32_t *__restrict__ blk_item,
                                                                const int *__restrict__ ncols) {
  const int gi = blk_item[blockIdx.x];
  const OrthoItem *it = items + gi;
  const int b = blockIdx.x - it->blk0[kOrthoKinds - 1], nb = it->nblk[kOrthoKinds - 1], ncol = ncols[gi];
  const T *V = (const T *)it->V;
  T *x = (T *)it->x;
  const double *y = it->y;
  for (int64_t k = b * (int64_t)kThreads + threadIdx.x; k < it->n; k += (int64_t)nb * kThreads) {
    double s = 0.0;
    const int64_t base = tile_ix(k, 0, it->m1);
#pragma unroll 8
    for (int i = 0; i < ncol; ++i) s += y[i] * (double)V[base + (int64_t)i * kTile];
    x[k] = (T)((double)x[k] + s);
  }
}

__global__ void gather_res_batch_kernel(const OrthoItem *__restrict__ items, int n_items, int j0, int cnt,
                                        double *__restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_items * cnt) return;
  out[t] = items[t / cnt].res[j0 + t % cnt];
}

__global__ void gather_norm_batch_kernel(const OrthoItem *__restrict__ items, int n_items, double *__restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_items) out[t] = *items[t].hn;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void basis_store_batch_kernel(const OrthoItem *__restrict__ items,
                                                                     const int32_t *__restrict__ blk_item, int col) {
  const int g = blockIdx.x;
  const OrthoItem *it = items + blk_item[g];
  const int b = g - it->blk0[kOrthoKinds - 1], nb = it->nblk[kOrthoKinds - 1];
  const double f = *it->fac;
  const T *x = (const T *)it->w;
  T *V = (T *)it->V, *vc = (T *)it->vc;
  for (int64_t k = b * (int64_t)kThreads + threadIdx.x; k < it->n; k += (int64_t)nb * kThreads) {
    const T y = (T)((double)x[k] * f);
    V[tile_ix(k, col, it->m1)] = y;
    vc[k] = y;
  }
}

}  // namespace

struct Workspace {
  int64_t n = 0;
  int m = 0;
  // FP64
  double *V = nullptr;   // (m+1) columns of the GMRES basis in row tiles (tile_ix), rows padded to kTile
  double *vc = nullptr;  // newest basis vector, contiguous
  double *w = nullptr, *r = nullptr, *t = nullptr, *z = nullptr;
  double *dinv = nullptr;
  // FP32
  float *V32 = nullptr;  // as V
  float *vc32 = nullptr;
  float *w32 = nullptr, *c32 = nullptr, *z32 = nullptr, *r32 = nullptr, *dinv32 = nullptr;
  // reductions
  double *partial = nullptr;  // kMaxBlocks x (m+2)
  double *h = nullptr;        // 3 (m+2) device scalars: two projection passes and a norm (also scratch)
  double *y = nullptr;        // m+2 coefficients for the update (slot m+1: scratch of the refinement)
  double *gm = nullptr;       // GMRES state: H ((m+1) x m), cs, sn (m), g (m+1), res (m), factor
  unsigned *ticket = nullptr; // block counter of the single-pass reductions (0 between launches)
  void *arena = nullptr;      // the allocation holding all of the above
  size_t bytes = 0;           // device bytes held: the arena plus the Jacobi diagonals
  // the solver runs on a stream of its own (after the caller's stream, by an event), so that
  // its Arnoldi steps can be captured into graphs and replayed; one graph per run of steps
  // j..j1 of a restart cycle (key: precision, j, j1, preconditioner, extension order), made in
  // the second cycle of a solve and replayed in every later one
  hipStream_t stream = nullptr;
  hipEvent_t ready = nullptr;
  std::map<uint64_t, hipGraphExec_t> graphs;
  bool graphs_off = false;    // a capture failed: steps are launched one by one
  bool have_diag = false;
  // grid of each Gram-Schmidt kernel: as many blocks as fit on the device at once (no partial
  // last round), index [FP32][log2(CPW) - 1, 4 for the kernel of more than 64 columns][MODE]
  int gs_grid[2][5][3] = {};
};

size_t workspace_bytes(const sbm_ctx *c) { return c->ws ? c->ws->bytes : 0; }

void free_workspace(sbm_ctx *c) {
  Workspace *ws = c->ws;
  if (!ws) return;
  // one allocation for the vectors and scalars; the Jacobi diagonals are allocated on their
  // first use; all from the device pool, released stream-ordered
  if (ws->stream) (void)hipStreamSynchronize(ws->stream);
  for (auto &g : ws->graphs) (void)hipGraphExecDestroy(g.second);
  ws->graphs.clear();
  for (void *p : {ws->arena, (void *)ws->dinv, (void *)ws->dinv32}) dev_free(p);
  if (ws->ready) (void)hipEventDestroy(ws->ready);
  if (ws->stream) (void)hipStreamDestroy(ws->stream);
  delete ws;
  c->ws = nullptr;
}

static hipError_t ensure_workspace(sbm_ctx *c, int m, bool need32) {
  Workspace *ws = c->ws;
  if (ws && ws->m >= m && (!need32 || ws->V32)) return hipSuccess;
  free_workspace(c);
  ws = new Workspace();
  c->ws = ws;
  ws->n = c->n_dofs;
  ws->m = m;
  const size_t n = (size_t)std::max<int64_t>(1, c->n_dofs);
  const size_t npad = (n + kTile - 1) / kTile * kTile;
  // carve the arena: every piece starts on a 256-byte boundary
  size_t off = 0;
  std::vector<std::function<void(char *)>> parts;
  auto piece = [&](auto *&ptr, size_t bytes) {
    using P = std::remove_reference_t<decltype(*ptr)>;
    const size_t at = off;
    parts.push_back([&ptr, at](char *base) { ptr = reinterpret_cast<P *>(base + at); });
    off += (bytes + 255) / 256 * 256;
  };
  piece(ws->V, sizeof(double) * npad * (m + 1));
  piece(ws->vc, sizeof(double) * n);
  piece(ws->w, sizeof(double) * n);
  piece(ws->r, sizeof(double) * n);
  piece(ws->t, sizeof(double) * n);
  piece(ws->z, sizeof(double) * n);
  piece(ws->partial, sizeof(double) * kMaxBlocks * (m + 2));
  piece(ws->h, sizeof(double) * 3 * (m + 2));
  piece(ws->y, sizeof(double) * (m + 2));
  piece(ws->gm, sizeof(double) * ((size_t)(m + 1) * m + 4 * m + 2));
  piece(ws->ticket, sizeof(unsigned));
  if (need32) {
    piece(ws->V32, sizeof(float) * npad * (m + 1));
    piece(ws->vc32, sizeof(float) * n);
    piece(ws->w32, sizeof(float) * n);
    piece(ws->c32, sizeof(float) * n);
    piece(ws->z32, sizeof(float) * n);
    piece(ws->r32, sizeof(float) * n);
  }
  hipError_t e = dev_alloc(&ws->arena, off);
  if (e != hipSuccess) return e;
  ws->bytes = off;
  e = hipStreamCreateWithFlags(&ws->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ws->ready, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  for (auto &set : parts) set(static_cast<char *>(ws->arena));
  e = hipMemsetAsync(ws->ticket, 0, sizeof(unsigned), lib_stream());
  return e == hipSuccess ? hipStreamSynchronize(lib_stream()) : e;
}

// device dot products: out[i] = V_i . w for i < ncol (out on the device)
template <typename T>
static hipError_t multidot(const T *V, int64_t ld, int ncol, const T *w, int64_t n, double *partial, double *out,
                           hipStream_t s) {
  const int nb = nblocks(n);
  if (ncol <= 8)
    hipLaunchKernelGGL((multidot_kernel<T, 8>), dim3(nb), dim3(kThreads), 0, s, V, ld, ncol, w, n, partial);
  else if (ncol <= 16)
    hipLaunchKernelGGL((multidot_kernel<T, 16>), dim3(nb), dim3(kThreads), 0, s, V, ld, ncol, w, n, partial);
  else if (ncol <= 32)
    hipLaunchKernelGGL((multidot_kernel<T, 32>), dim3(nb), dim3(kThreads), 0, s, V, ld, ncol, w, n, partial);
  else
    hipLaunchKernelGGL((multidot_kernel<T, 64>), dim3(nb), dim3(kThreads), 0, s, V, ld, ncol, w, n, partial);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(64), 0, s, partial, nb, ncol, out);
  return hipGetLastError();
}

template <typename K>
static int grid_cap(K kernel) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess)
    return kMaxBlocks;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess) return kMaxBlocks;
  return std::max(1, std::min(kMaxBlocks, per_cu * cus));
}

template <typename T, int L>
static void gs_grid_caps1(int *g) {
  constexpr int CPW = 2 << L;
  if constexpr (L == 4) {
    g[0] = grid_cap(gs_wide_kernel<T, 0>), g[1] = grid_cap(gs_wide_kernel<T, 1>), g[2] = grid_cap(gs_wide_kernel<T, 2>);
  } else {
    g[0] = grid_cap(gs_kernel<T, CPW, 0>), g[1] = grid_cap(gs_kernel<T, CPW, 1>), g[2] = grid_cap(gs_kernel<T, CPW, 2>);
  }
}

template <typename T>
static void gs_grid_caps(int (*g)[3]) {
  gs_grid_caps1<T, 0>(g[0]), gs_grid_caps1<T, 1>(g[1]), gs_grid_caps1<T, 2>(g[2]), gs_grid_caps1<T, 3>(g[3]);
  gs_grid_caps1<T, 4>(g[4]);
}

template <typename T, int CPW, int MODE>
static void gs_launch1(const Workspace *ws, const T *V, int m1, int ncol, const double *coef, T *w, int64_t n,
                       double *partial, unsigned *ticket, double *out, const ArnoldiArgs &aa, hipStream_t s) {
  constexpr int L = CPW == 2 ? 0 : (CPW == 4 ? 1 : (CPW == 8 ? 2 : 3));
  const int64_t rows = 64 * (32 / CPW);  // rows per block and step
  const int cap = ws->gs_grid[sizeof(T) == 4 ? 1 : 0][L][MODE];
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((n + rows - 1) / rows, cap));
  hipLaunchKernelGGL((gs_kernel<T, CPW, MODE>), dim3(nb), dim3(kThreads), 0, s, V, m1, ncol, coef, w, n, partial,
                     ticket, out, aa);
}

template <typename T, int MODE>
static void gs_launch(const Workspace *ws, const T *V, int m1, int ncol, const double *coef, T *w, int64_t n,
                      double *partial, unsigned *ticket, double *out, const ArnoldiArgs &aa, hipStream_t s) {
  if (ncol <= 8)
    gs_launch1<T, 2, MODE>(ws, V, m1, ncol, coef, w, n, partial, ticket, out, aa, s);
  else if (ncol <= 16)
    gs_launch1<T, 4, MODE>(ws, V, m1, ncol, coef, w, n, partial, ticket, out, aa, s);
  else if (ncol <= 32)
    gs_launch1<T, 8, MODE>(ws, V, m1, ncol, coef, w, n, partial, ticket, out, aa, s);
  else if (ncol <= 64)
    gs_launch1<T, 16, MODE>(ws, V, m1, ncol, coef, w, n, partial, ticket, out, aa, s);
  else {
    const int64_t rows = 128;  // rows per block and step of gs_wide_kernel
    const int cap = ws->gs_grid[sizeof(T) == 4 ? 1 : 0][4][MODE];
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((n + rows - 1) / rows, cap));
    hipLaunchKernelGGL((gs_wide_kernel<T, MODE>), dim3(nb), dim3(kThreads), 0, s, V, m1, ncol, coef, w, n, partial,
                       ticket, out, aa);
  }
}

// Arnoldi steps j <= k < j1 of restarted GMRES(m) on the basis V (column k + 1 is formed from
// column k): w = A M^-1 v_k, two classical Gram-Schmidt passes (CGS2), the norm, the device
// rotation update (arnoldi_step) and v_(k+1) = w / h_(k+1,k).  Launches only (no host
// synchronisation).
// Step k of an Arnoldi run after the apply w = A M^-1 v_k: two classical Gram-Schmidt passes
// (CGS2: h1 = V^T w; w -= V h1, h2 = V^T w; w -= V h2), |w|^2 and the rotation update, and
// v_(k+1) = w / h_(k+1,k) into V and vc.
template <typename T>
static void arnoldi_orthogonalise(sbm_ctx *c, T *V, T *vc, T *w, int m, int k, hipStream_t s) {
  Workspace *ws = c->ws;
  const int64_t n = c->n_dofs;
  const int nb = nblocks(n);
  const int m1 = ws->m + 1;
  double *h1 = ws->h, *h2 = ws->h + (m + 2), *hn = ws->h + 2 * (m + 2);
  double *H = ws->gm, *cs = H + (size_t)(m + 1) * m, *sn = cs + m, *g = sn + m, *dres = g + (m + 1);
  double *fac = dres + m;
  const ArnoldiArgs aa{k, m, h1, h2, H, cs, sn, g, dres, fac};
  gs_launch<T, 0>(ws, V, m1, k + 1, nullptr, w, n, ws->partial, ws->ticket, h1, aa, s);
  gs_launch<T, 1>(ws, V, m1, k + 1, h1, w, n, ws->partial, ws->ticket, h2, aa, s);
  gs_launch<T, 2>(ws, V, m1, k + 1, h2, w, n, ws->partial, ws->ticket, hn, aa, s);
  hipLaunchKernelGGL(basis_store_kernel<T>, dim3(nb), dim3(kThreads), 0, s, w, fac, 0, V, k + 1, m1, vc, n);
}

template <typename T>
static sbm_status arnoldi_steps(sbm_ctx *c, int prec, T *V, T *vc, T *w, T *z, const T *dinv, int m, int j,
                                int j1, hipStream_t s) {
  const int64_t n = c->n_dofs;
  const int nb = nblocks(n);
  for (int k = j; k < j1; ++k) {
    // vc holds v_k contiguously
    const T *src = vc;
    if (dinv) {
      hipLaunchKernelGGL(diag_scale_kernel<T>, dim3(nb), dim3(kThreads), 0, s, dinv, vc, z, n);
      src = z;
    }
    SBM_HIP_CHECK(launch_operator(c, src, w, prec, SBM_PART_ALL, s));
    arnoldi_orthogonalise<T>(c, V, vc, w, m, k, s);
  }
  SBM_HIP_CHECK(hipGetLastError());
  return SBM_OK;
}

// One restarted-GMRES run in precision T on A_T (prec) with optional right Jacobi
// preconditioning.  Solves A c = rhs to ||rhs - A c|| <= tol_abs starting from c (device),
// at most max_it iterations.  Returns the final true residual norm in *res (FP64, device
// computed) and the iteration count in *its.
//
// The Arnoldi steps, the Givens rotations and the back substitution run on the device; the
// host reads the residual estimates back every few steps (the steps launched past the first
// one that met the tolerance are discarded: only the leading columns enter the update, so the
// result and the iteration count are those of a check after every step).
template <typename T>
static sbm_status gmres_run(sbm_ctx *c, int prec, const T *rhs, T *x, T *V, T *vc, T *w, T *z, const T *dinv,
                            int m, double tol_abs, int max_it, hipStream_t s, int *its, int *applies,
                            double *res) {
  Workspace *ws = c->ws;
  const int64_t n = c->n_dofs;
  const int nb = nblocks(n);
  const int check = n > (1 << 20) ? 4 : 8;  // steps between residual read-backs
  double *hn = ws->h + 2 * (m + 2);
  double *H = ws->gm, *g = H + (size_t)(m + 1) * m + 2 * m, *dres = g + (m + 1);
  std::vector<double> rh(m);
  int(*grid)[3] = ws->gs_grid[sizeof(T) == 4 ? 1 : 0];
  if (grid[0][0] == 0) gs_grid_caps<T>(grid);
  *its = 0;
  double beta = 0.0;
  for (int cycle = 0;; ++cycle) {
    // r = rhs - A x  -> V_0
    SBM_HIP_CHECK(launch_operator(c, x, w, prec, SBM_PART_ALL, s));
    ++*applies;
    hipLaunchKernelGGL(residual_kernel<T>, dim3(nb), dim3(kThreads), 0, s, rhs, w, vc, n);
    SBM_HIP_CHECK(multidot<T>(vc, n, 1, vc, n, ws->partial, hn, s));
    SBM_HIP_CHECK(hipMemcpyAsync(&beta, hn, sizeof(double), hipMemcpyDeviceToHost, s));
    SBM_HIP_CHECK(hipStreamSynchronize(s));
    beta = std::sqrt(beta);
    *res = beta;
    if (!(beta > tol_abs) || *its >= max_it) return std::isfinite(beta) ? SBM_OK : SBM_ENOCONV;
    hipLaunchKernelGGL(basis_store_kernel<T>, dim3(nb), dim3(kThreads), 0, s, vc, hn, 1, V, 0, ws->m + 1, vc, n);
    hipLaunchKernelGGL(gmres_init_kernel, dim3(1), dim3(64), 0, s, hn, g, m);
    int j = 0;
    bool stop = false;
    while (j < m && *its < max_it && !stop) {
      const int j1 = std::min({m, j + check, j + (max_it - *its)});
      // a run of steps of the regular length, from the second cycle on: its graph (captured at
      // its first use, then replayed); otherwise the steps are launched one by one
      const bool use_graph = cycle > 0 && c->solver_graphs && !ws->graphs_off && j1 == std::min(m, j + check);
      sbm_status st = SBM_OK;
      if (use_graph) {
        const uint64_t key = ((uint64_t)(sizeof(T) == 4) << 62) | ((uint64_t)(dinv != nullptr) << 61) |
                             ((uint64_t)(c->taylor_m + 1) << 40) | ((uint64_t)m << 20) | ((uint64_t)j << 10) |
                             (uint64_t)j1;
        auto it = ws->graphs.find(key);
        if (it == ws->graphs.end()) {
          hipGraph_t g = nullptr;
          hipGraphExec_t ge = nullptr;
          bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
          if (ok) {
            st = arnoldi_steps<T>(c, prec, V, vc, w, z, dinv, m, j, j1, s);
            ok = hipStreamEndCapture(s, &g) == hipSuccess && st == SBM_OK && g;
            if (ok) ok = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
          }
          if (!ok) {
            (void)hipGetLastError();
            ws->graphs_off = true;  // launch one by one from now on
            st = arnoldi_steps<T>(c, prec, V, vc, w, z, dinv, m, j, j1, s);
          } else {
            it = ws->graphs.emplace(key, ge).first;
          }
        }
        if (it != ws->graphs.end()) SBM_HIP_CHECK(hipGraphLaunch(it->second, s));
      } else {
        st = arnoldi_steps<T>(c, prec, V, vc, w, z, dinv, m, j, j1, s);
      }
      if (st != SBM_OK) return st;
      *applies += j1 - j;
      SBM_HIP_CHECK(hipMemcpyAsync(rh.data(), dres + j, sizeof(double) * (j1 - j), hipMemcpyDeviceToHost, s));
      SBM_HIP_CHECK(hipStreamSynchronize(s));
      int k = j;
      while (k < j1 && rh[k - j] > tol_abs) ++k;  // stops at convergence, breakdown (-1) or NaN
      if (k < j1) {
        *its += k + 1 - j;
        j = k + 1;
        stop = true;
      } else {
        *its += j1 - j;
        j = j1;
      }
    }
    // back substitution and update x += M^-1 V y, from the leading j columns
    if (j > 0) {
      hipLaunchKernelGGL(backsub_kernel, dim3(1), dim3(64), 0, s, j, m, H, g, ws->y);
      hipLaunchKernelGGL(update_kernel<T>, dim3(nb), dim3(kThreads), 0, s, V, ws->m + 1, j, ws->y, dinv, x, n);
    }
  }
}

// Conjugate gradients in precision T on A_T (prec), for symmetric positive definite
// operators: solves A c = rhs from the initial c to a recursive residual norm <= tol_abs, at
// most max_it iterations (r, p, q: work vectors).  The residual norm is read back every 10
// iterations.  Uses ws->partial (2 kMaxBlocks) and ws->y[0..1] (|r|^2, alternating).
template <typename T>
static sbm_status cg_run(sbm_ctx *c, int prec, const T *rhs, T *x, T *r, T *p, T *q, double tol_abs, int max_it,
                         hipStream_t s, int *its_out, int *applies, double *res_out) {
  Workspace *ws = c->ws;
  const int64_t n = c->n_dofs;
  const int nb = nblocks(n);
  double *part_pq = ws->partial, *part_rr = ws->partial + kMaxBlocks;
  double *rr = ws->y;
  SBM_HIP_CHECK(launch_operator(c, x, q, prec, SBM_PART_ALL, s));
  ++*applies;
  hipLaunchKernelGGL(cg_init_kernel<T>, dim3(nb), dim3(kThreads), 0, s, rhs, q, r, p, part_rr, n);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(64), 0, s, part_rr, nb, 1, rr);
  int it = 0;
  double res = 0.0;
  for (;; ++it) {
    const int cur = it & 1;
    if (it % 10 == 0 || it >= max_it) {
      double v = 0.0;
      SBM_HIP_CHECK(hipMemcpyAsync(&v, rr + cur, sizeof(double), hipMemcpyDeviceToHost, s));
      SBM_HIP_CHECK(hipStreamSynchronize(s));
      res = std::sqrt(v);
      if (!(res > tol_abs) || !std::isfinite(res) || it >= max_it) break;
    }
    SBM_HIP_CHECK(launch_operator(c, p, q, prec, SBM_PART_ALL, s));
    ++*applies;
    hipLaunchKernelGGL(cg_dot_kernel<T>, dim3(nb), dim3(kThreads), 0, s, p, q, part_pq, n);
    hipLaunchKernelGGL(cg_update_kernel<T>, dim3(nb), dim3(kThreads), 0, s, x, r, p, q, rr + cur, part_pq, nb,
                       part_rr, n);
    hipLaunchKernelGGL(cg_dir_kernel<T>, dim3(nb), dim3(kThreads), 0, s, p, r, rr + cur, part_rr, nb, rr + (1 - cur),
                       n);
  }
  *its_out = it;
  *res_out = res;
  return SBM_OK;
}

// CG on the FP32 operator with FP64 residual replacement (van der Vorst and Ye, "Residual
// replacement strategies for Krylov subspace iterative methods", SIAM J. Sci. Comput. 22,
// 2000), for symmetric positive definite operators: x is accumulated in FP64, r, p, q are FP32.
// Whenever the recursive residual has dropped by 1e3 since the last replacement (or claims
// convergence), r is replaced by the true residual b - A x computed with the FP64 operator
// (the search direction is kept), so the FP32 recursion never drifts far from it.  The
// iteration stops on the true residual.  Uses ws->r, t (FP64), r32, z32, w32 (FP32),
// ws->partial and ws->y[0..1].
static sbm_status cg_rr_run(sbm_ctx *c, const double *b, double *x, double tol_abs, int max_it, hipStream_t s,
                            int *its_out, int *replacements, int *applies64, int *applies32, double *res_out) {
  Workspace *ws = c->ws;
  const int64_t n = c->n_dofs;
  const int nb = nblocks(n);
  float *r = ws->r32, *p = ws->z32, *q = ws->w32;
  double *part_pq = ws->partial, *part_rr = ws->partial + kMaxBlocks;
  double *rr = ws->y;
  // r = b - A64 x in FP64, its square norm into rr[slot] (read back), r32 = (float) r
  auto replace = [&](int slot, double *rn2) -> sbm_status {
    SBM_HIP_CHECK(launch_operator(c, x, ws->t, SBM_F64, SBM_PART_ALL, s));
    ++*applies64;
    hipLaunchKernelGGL(residual_kernel<double>, dim3(nb), dim3(kThreads), 0, s, b, ws->t, ws->r, n);
    SBM_HIP_CHECK(multidot<double>(ws->r, n, 1, ws->r, n, ws->partial, rr + slot, s));
    hipLaunchKernelGGL(cast_f64_f32_kernel, dim3(nb), dim3(kThreads), 0, s, ws->r, r, n);
    SBM_HIP_CHECK(hipMemcpyAsync(rn2, rr + slot, sizeof(double), hipMemcpyDeviceToHost, s));
    SBM_HIP_CHECK(hipStreamSynchronize(s));
    return SBM_OK;
  };
  double seg = 0.0;
  sbm_status st = replace(0, &seg);
  if (st != SBM_OK) return st;
  hipLaunchKernelGGL(copy_kernel<float>, dim3(nb), dim3(kThreads), 0, s, r, p, n);
  double res = std::sqrt(seg);
  int it = 0;
  for (;; ++it) {
    const int cur = it & 1;
    if (!(res > tol_abs) || !std::isfinite(res)) break;
    if (it > 0 && (it % 10 == 0 || it >= max_it)) {
      double v = 0.0;
      SBM_HIP_CHECK(hipMemcpyAsync(&v, rr + cur, sizeof(double), hipMemcpyDeviceToHost, s));
      SBM_HIP_CHECK(hipStreamSynchronize(s));
      if (!(std::sqrt(v) > tol_abs) || !(v > 1e-6 * seg) || it >= max_it) {
        st = replace(cur, &seg);
        if (st != SBM_OK) return st;
        ++*replacements;
        res = std::sqrt(seg);
        if (!(res > tol_abs) || it >= max_it) break;
      }
    }
    SBM_HIP_CHECK(launch_operator(c, p, q, SBM_F32, SBM_PART_ALL, s));
    ++*applies32;
    hipLaunchKernelGGL(cg_dot_kernel<float>, dim3(nb), dim3(kThreads), 0, s, p, q, part_pq, n);
    hipLaunchKernelGGL((cg_update_kernel<float, double>), dim3(nb), dim3(kThreads), 0, s, x, r, p, q, rr + cur,
                       part_pq, nb, part_rr, n);
    hipLaunchKernelGGL(cg_dir_kernel<float>, dim3(nb), dim3(kThreads), 0, s, p, r, rr + cur, part_rr, nb,
                       rr + (1 - cur), n);
  }
  *its_out = it;
  *res_out = res;
  return SBM_OK;
}

}  // namespace sbm

using namespace sbm;

static sbm_status solve_on(sbm_handle h, const double *b, double *x, double rel_tol, int max_it, int mode, int m,
                           int jacobi, hipStream_t s, sbm_solve_info *info,
                           std::chrono::steady_clock::time_point t0) {
  Workspace *ws = h->ws;
  const int64_t n = h->n_dofs;
  const int nb = nblocks(n);
  // Jacobi: inverse diagonal
  const double *dinv = nullptr;
  const float *dinv32 = nullptr;
  if (jacobi) {
    if (!ws->dinv) {
      if (dev_alloc((void **)&ws->dinv, sizeof(double) * n) != hipSuccess) {
        set_error("sbm_solve: out of device memory");
        return SBM_ENOMEM;
      }
      ws->bytes += sizeof(double) * n;
    }
    sbm_status st = sbm_diagonal(h, ws->dinv, SBM_F64, s);
    if (st != SBM_OK) {
      info->status = st;
      return st;
    }
    hipLaunchKernelGGL(invert_kernel, dim3(nb), dim3(kThreads), 0, s, ws->dinv, n);
    dinv = ws->dinv;
    if (mode == SBM_SOLVE_GMRES_IR) {
      if (!ws->dinv32) {
        if (dev_alloc((void **)&ws->dinv32, sizeof(float) * n) != hipSuccess) {
          set_error("sbm_solve: out of device memory");
          return SBM_ENOMEM;
        }
        ws->bytes += sizeof(float) * n;
      }
      hipLaunchKernelGGL(cast_f64_f32_kernel, dim3(nb), dim3(kThreads), 0, s, ws->dinv, ws->dinv32, n);
      dinv32 = ws->dinv32;
    }
  }
  // ||b||
  SBM_HIP_CHECK(multidot<double>(b, n, 1, b, n, ws->partial, ws->h, s));
  double bn2 = 0.0;
  SBM_HIP_CHECK(hipMemcpyAsync(&bn2, ws->h, sizeof(double), hipMemcpyDeviceToHost, s));
  SBM_HIP_CHECK(hipStreamSynchronize(s));
  const double bnorm = std::sqrt(bn2);
  const double tol_abs = rel_tol * (bnorm > 0 ? bnorm : 1.0);
  sbm_status st = SBM_OK;
  double res = 0.0;
  if (mode == SBM_SOLVE_GMRES_F64) {
    int its = 0, applies = 0;
    st = gmres_run<double>(h, SBM_F64, b, x, ws->V, ws->vc, ws->w, ws->z, dinv, m, tol_abs, max_it, s, &its,
                           &applies, &res);
    info->inner_its = its;
    info->outer_its = (its + m - 1) / m;
    info->applies_f64 = applies;
  } else if (mode == SBM_SOLVE_GMRES_IR) {
    // FP64 refinement: r = b - A x (FP64), c ~= A32^-1 (r / |r|) by FP32 GMRES, x += |r| c
    int total_its = 0;
    for (int outer = 0;; ++outer) {
      SBM_HIP_CHECK(launch_operator(h, x, ws->t, SBM_F64, SBM_PART_ALL, s));
      ++info->applies_f64;
      hipLaunchKernelGGL(residual_kernel<double>, dim3(nb), dim3(kThreads), 0, s, b, ws->t, ws->r, n);
      SBM_HIP_CHECK(multidot<double>(ws->r, n, 1, ws->r, n, ws->partial, ws->h, s));
      double rn2 = 0.0;
      SBM_HIP_CHECK(hipMemcpyAsync(&rn2, ws->h, sizeof(double), hipMemcpyDeviceToHost, s));
      SBM_HIP_CHECK(hipStreamSynchronize(s));
      res = std::sqrt(rn2);
      info->outer_its = outer;
      if (!(res > tol_abs) || total_its >= max_it || !std::isfinite(res)) break;
      // keep |r|^2 on the device for the scaling kernels (slot m+1 of h is GMRES scratch)
      SBM_HIP_CHECK(hipMemcpyAsync(ws->y + (m + 1), ws->h, sizeof(double), hipMemcpyDeviceToDevice, s));
      hipLaunchKernelGGL(to_f32_kernel, dim3(nb), dim3(kThreads), 0, s, ws->r, ws->y + (m + 1), ws->r32, n);
      hipLaunchKernelGGL(fill_f32_kernel, dim3(nb), dim3(kThreads), 0, s, ws->c32, n);
      int its = 0, applies = 0;
      double inner_res = 0.0;
      // inner solve of A32 c = r / |r| (unit right-hand side) to what the remaining reduction
      // needs, max(1e-6, tol / (2 |r|)) (FP32 reaches about 1e-6), at most 4 restart cycles
      const double inner_tol = std::max(1e-6, 0.5 * tol_abs / res);
      (void)gmres_run<float>(h, SBM_F32, ws->r32, ws->c32, ws->V32, ws->vc32, ws->w32, ws->z32, dinv32, m,
                             inner_tol, std::min(4 * m, max_it - total_its), s, &its, &applies, &inner_res);
      total_its += its;
      info->applies_f32 += applies;
      hipLaunchKernelGGL(add_f32_kernel, dim3(nb), dim3(kThreads), 0, s, ws->c32, ws->y + (m + 1), x, n);
      if (its == 0) break;
    }
    info->inner_its = total_its;
  } else if (mode == SBM_SOLVE_CG_F64) {
    // CG (symmetric operators only)
    int its = 0, applies = 0;
    st = cg_run<double>(h, SBM_F64, b, x, ws->r, ws->z, ws->t, tol_abs, max_it, s, &its, &applies, &res);
    info->inner_its = its;
    info->outer_its = 1;
    info->applies_f64 = applies;
  } else if (mode == SBM_SOLVE_CG_RR) {
    int its = 0, reps = 0, a64 = 0, a32 = 0;
    st = cg_rr_run(h, b, x, tol_abs, max_it, s, &its, &reps, &a64, &a32, &res);
    info->inner_its = its;
    info->outer_its = reps;
    info->applies_f64 = a64;
    info->applies_f32 = a32;
  } else {
    // FP64 refinement around FP32 CG: r = b - A x and |r| in FP64, c ~= A32^-1 (r / |r|) by
    // FP32 CG, x += |r| c in FP64.  The inner tolerance is what the remaining reduction needs
    // (half of tol / |r|), but not below 1e-6 (FP32): every restart of CG discards its Krylov
    // space, so each inner solve should do as much of the work as FP32 allows.
    int total_its = 0;
    for (int outer = 0;; ++outer) {
      SBM_HIP_CHECK(launch_operator(h, x, ws->t, SBM_F64, SBM_PART_ALL, s));
      ++info->applies_f64;
      hipLaunchKernelGGL(residual_kernel<double>, dim3(nb), dim3(kThreads), 0, s, b, ws->t, ws->r, n);
      SBM_HIP_CHECK(multidot<double>(ws->r, n, 1, ws->r, n, ws->partial, ws->h, s));  // |r|^2 stays in h[0]
      double rn2 = 0.0;
      SBM_HIP_CHECK(hipMemcpyAsync(&rn2, ws->h, sizeof(double), hipMemcpyDeviceToHost, s));
      SBM_HIP_CHECK(hipStreamSynchronize(s));
      res = std::sqrt(rn2);
      info->outer_its = outer;
      if (!(res > tol_abs) || total_its >= max_it || !std::isfinite(res)) break;
      hipLaunchKernelGGL(to_f32_kernel, dim3(nb), dim3(kThreads), 0, s, ws->r, ws->h, ws->r32, n);
      hipLaunchKernelGGL(fill_f32_kernel, dim3(nb), dim3(kThreads), 0, s, ws->c32, n);
      int its = 0, applies = 0;
      double inner_res = 0.0;
      const double inner_tol = std::max(1e-6, 0.5 * tol_abs / res);
      const sbm_status ist = cg_run<float>(h, SBM_F32, ws->r32, ws->c32, ws->w32, ws->z32, ws->V32, inner_tol,
                                           max_it - total_its, s, &its, &applies, &inner_res);
      if (ist != SBM_OK) {
        info->status = ist;
        return ist;
      }
      total_its += its;
      info->applies_f32 += applies;
      hipLaunchKernelGGL(add_f32_kernel, dim3(nb), dim3(kThreads), 0, s, ws->c32, ws->h, x, n);
      if (its == 0) break;
    }
    info->inner_its = total_its;
  }
  // final true residual in FP64
  SBM_HIP_CHECK(launch_operator(h, x, ws->t, SBM_F64, SBM_PART_ALL, s));
  ++info->applies_f64;
  hipLaunchKernelGGL(residual_kernel<double>, dim3(nb), dim3(kThreads), 0, s, b, ws->t, ws->r, n);
  SBM_HIP_CHECK(multidot<double>(ws->r, n, 1, ws->r, n, ws->partial, ws->h, s));
  double rn2 = 0.0;
  SBM_HIP_CHECK(hipMemcpyAsync(&rn2, ws->h, sizeof(double), hipMemcpyDeviceToHost, s));
  SBM_HIP_CHECK(hipStreamSynchronize(s));
  info->rel_residual = std::sqrt(rn2) / (bnorm > 0 ? bnorm : 1.0);
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st == SBM_OK && !(info->rel_residual <= rel_tol)) st = SBM_ENOCONV;
  if (st == SBM_ENOCONV) set_error("sbm_solve: tolerance not reached within max_it");
  info->status = st;
  return st;
}

// ---- batched solves: restarted GMRES (FP64, or FP32 inside FP64 refinement) of several
// operators in lockstep.  Every operator apply of a step runs for all operators at once
// through a batch of applies (sbm_batch_*: one launch per stage per group of operators of one
// kernel instantiation); everything else is launched per operator exactly as a single solve
// launches it, in the same order on its own data, so each result is bitwise that operator's
// sbm_solve (the residual checks are only read back at other points of the run) ----

namespace {

// One operator's restarted-GMRES run inside a lockstep batch (the state gmres_run keeps in
// locals).
template <typename T>
struct GItem {
  sbm_ctx *c = nullptr;
  const T *rhs = nullptr;
  T *x = nullptr, *V = nullptr, *vc = nullptr, *w = nullptr;
  double tol_abs = 0.0;
  int max_it = 0;
  int its = 0, applies = 0;
  double res = 0.0;
  bool done = false;   // the run has ended (tolerance, iteration bound or breakdown)
  int j = 0, j1 = 0;   // Arnoldi steps of the current cycle: done so far, and this chunk's end
  bool stop = false;
  sbm_status st = SBM_OK;
};

// A batch of applies kept while its membership does not change.
struct PlanCache {
  sbm_batch b = nullptr;
  std::vector<const void *> key;
  ~PlanCache() { (void)sbm_batch_destroy(b); }
  sbm_status run(const std::vector<sbm_ctx *> &cs, const std::vector<const void *> &u, const std::vector<void *> &v,
                 int prec, hipStream_t s) {
    std::vector<const void *> k;
    for (size_t i = 0; i < cs.size(); ++i) {
      k.push_back(cs[i]);
      k.push_back(u[i]);
      k.push_back(v[i]);
    }
    if (!b || k != key) {
      (void)sbm_batch_destroy(b);
      b = nullptr;
      std::vector<sbm_handle> hs(cs.begin(), cs.end());
      std::vector<void *> vv(v.begin(), v.end());
      const sbm_status st =
          sbm_batch_create((int)cs.size(), hs.data(), u.data(), vv.data(), prec, 0, 4, &b);
      if (st != SBM_OK) return st;
      key = k;
    }
    return sbm_batch_run(b, s);
  }
};

// The orthogonalisation of step k for a set of runs (all at the same step, so with the same
// number of columns): one launch per Gram-Schmidt kernel and one for the basis store, with the
// tables of the set (every column class and mode) built once per set.  Past 64 columns
// (restart > 63) the runs are launched one by one.
template <typename T>
struct OrthoPlan {
  void *d = nullptr;
  std::vector<const void *> key;
  size_t off_items = 0, off_tab[kOrthoKinds] = {}, off_ncol = 0, off_out = 0;
  int total[kOrthoKinds] = {};
  std::vector<GItem<T> *> set;
  std::vector<int> ncol_h;  // host copy of the column counts being uploaded (kept until the next sync)
  hipStream_t stream = nullptr;  // where the tables are read (waited for before they are released)
  ~OrthoPlan() {
    if (!d) return;
    (void)hipStreamSynchronize(stream);
    dev_free(d);
  }

  sbm_status prepare(const std::vector<GItem<T> *> &sub, int m, hipStream_t s) {
    stream = s;
    std::vector<const void *> k(sub.begin(), sub.end());
    if (d && k == key) return SBM_OK;
    if (d) {
      SBM_HIP_CHECK(hipStreamSynchronize(s));  // the old tables may still be read
      dev_free(d);
      d = nullptr;
    }
    std::vector<OrthoItem> items(sub.size());
    std::vector<int32_t> tab[kOrthoKinds];
    int tot[kOrthoKinds] = {};
    for (size_t i = 0; i < sub.size(); ++i) {
      GItem<T> *a = sub[i];
      Workspace *ws = a->c->ws;
      const int64_t n = a->c->n_dofs;
      OrthoItem &o = items[i];
      o.V = a->V;
      o.w = a->w;
      o.vc = a->vc;
      o.x = a->x;
      o.y = ws->y;
      o.n = n;
      o.m1 = ws->m + 1;
      o.m = m;
      o.partial = ws->partial;
      o.counter = ws->ticket;
      o.h1 = ws->h;
      o.h2 = ws->h + (m + 2);
      o.hn = ws->h + 2 * (m + 2);
      o.H = ws->gm;
      o.cs = o.H + (size_t)(m + 1) * m;
      o.sn = o.cs + m;
      o.g = o.sn + m;
      o.res = o.g + (m + 1);
      o.fac = o.res + m;
      const int(*caps)[3] = ws->gs_grid[sizeof(T) == 4 ? 1 : 0];
      for (int kind = 0; kind < kOrthoKinds; ++kind) {
        int nb;
        if (kind < kOrthoKinds - 1) {
          const int L = kind / 3, mode = kind % 3;
          const int64_t rows = 64 * (32 / (2 << L));  // as gs_launch1
          nb = (int)std::max<int64_t>(1, std::min<int64_t>((n + rows - 1) / rows, caps[L][mode]));
        } else {
          nb = nblocks(n);
        }
        o.blk0[kind] = tot[kind];
        o.nblk[kind] = nb;
        tab[kind].insert(tab[kind].end(), (size_t)nb, (int32_t)i);
        tot[kind] += nb;
      }
    }
    std::vector<unsigned char> image;
    auto put = [&image](const void *src, size_t bytes) {
      const size_t off = (image.size() + 255) / 256 * 256;
      image.resize(off + std::max<size_t>(bytes, 4));
      if (bytes) std::memcpy(image.data() + off, src, bytes);
      return off;
    };
    off_items = put(items.data(), items.size() * sizeof(OrthoItem));
    for (int kind = 0; kind < kOrthoKinds; ++kind) {
      off_tab[kind] = put(tab[kind].data(), tab[kind].size() * sizeof(int32_t));
      total[kind] = tot[kind];
    }
    off_ncol = put(nullptr, 0);
    image.resize(off_ncol + sizeof(int) * sub.size());
    off_out = put(nullptr, 0);
    image.resize(off_out + sizeof(double) * sub.size() * (size_t)(m + 1));
    SBM_HIP_CHECK(dev_alloc(&d, image.size()));
    SBM_HIP_CHECK(hipMemcpyAsync(d, image.data(), image.size(), hipMemcpyHostToDevice, lib_stream()));
    SBM_HIP_CHECK(hipStreamSynchronize(lib_stream()));
    key = k;
    set = sub;
    return SBM_OK;
  }

  template <int CPW>
  void launch_modes(int ncol, int k, hipStream_t s) {
    constexpr int L = CPW == 2 ? 0 : (CPW == 4 ? 1 : (CPW == 8 ? 2 : 3));
    const unsigned char *b = static_cast<const unsigned char *>(d);
    const OrthoItem *items = reinterpret_cast<const OrthoItem *>(b + off_items);
    auto tab = [&](int kind) { return reinterpret_cast<const int32_t *>(b + off_tab[kind]); };
    const int ni = (int)set.size();
    hipLaunchKernelGGL((gs_batch_kernel<T, CPW, 0>), dim3(total[3 * L]), dim3(kThreads), 0, s, items, tab(3 * L),
                       ncol, k);
    hipLaunchKernelGGL((gs_reduce_batch_kernel<CPW, 0>), dim3(ni), dim3(kThreads), 0, s, items, ncol, k);
    hipLaunchKernelGGL((gs_batch_kernel<T, CPW, 1>), dim3(total[3 * L + 1]), dim3(kThreads), 0, s, items,
                       tab(3 * L + 1), ncol, k);
    hipLaunchKernelGGL((gs_reduce_batch_kernel<CPW, 1>), dim3(ni), dim3(kThreads), 0, s, items, ncol, k);
    hipLaunchKernelGGL((gs_batch_kernel<T, CPW, 2>), dim3(total[3 * L + 2]), dim3(kThreads), 0, s, items,
                       tab(3 * L + 2), ncol, k);
    hipLaunchKernelGGL((gs_reduce_batch_kernel<CPW, 2>), dim3(ni), dim3(kThreads), 0, s, items, ncol, k);
    hipLaunchKernelGGL((basis_store_batch_kernel<T>), dim3(total[kOrthoKinds - 1]), dim3(kThreads), 0, s, items,
                       tab(kOrthoKinds - 1), k + 1);
  }

  const OrthoItem *items_dev() const {
    return reinterpret_cast<const OrthoItem *>(static_cast<const unsigned char *>(d) + off_items);
  }
  double *out_dev() const { return reinterpret_cast<double *>(static_cast<unsigned char *>(d) + off_out); }

  // res[j0 .. j0 + cnt) of every run of the set, run i at out[i cnt] (one copy, one sync)
  sbm_status gather_res(int j0, int cnt, std::vector<double> &out, hipStream_t s) {
    const int ni = (int)set.size(), tot = ni * cnt;
    out.assign((size_t)tot, 0.0);
    if (tot == 0) return SBM_OK;
    hipLaunchKernelGGL(gather_res_batch_kernel, dim3((tot + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                       items_dev(), ni, j0, cnt, out_dev());
    SBM_HIP_CHECK(hipMemcpyAsync(out.data(), out_dev(), sizeof(double) * tot, hipMemcpyDeviceToHost, s));
    SBM_HIP_CHECK(hipStreamSynchronize(s));
    return SBM_OK;
  }

  // the squared norms *hn of every run of the set
  sbm_status gather_norms(std::vector<double> &out, hipStream_t s) {
    const int ni = (int)set.size();
    out.assign((size_t)ni, 0.0);
    hipLaunchKernelGGL(gather_norm_batch_kernel, dim3((ni + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                       items_dev(), ni, out_dev());
    SBM_HIP_CHECK(hipMemcpyAsync(out.data(), out_dev(), sizeof(double) * ni, hipMemcpyDeviceToHost, s));
    SBM_HIP_CHECK(hipStreamSynchronize(s));
    return SBM_OK;
  }

  // y = R^-1 g and x += V y with ncol[i] columns for run i of the set
  sbm_status finish(const std::vector<int> &ncol, hipStream_t s) {
    ncol_h = ncol;
    int *dn = reinterpret_cast<int *>(static_cast<unsigned char *>(d) + off_ncol);
    SBM_HIP_CHECK(hipMemcpyAsync(dn, ncol_h.data(), sizeof(int) * ncol_h.size(), hipMemcpyHostToDevice, s));
    const unsigned char *b = static_cast<const unsigned char *>(d);
    hipLaunchKernelGGL(backsub_batch_kernel, dim3((unsigned)set.size()), dim3(kThreads), 0, s, items_dev(),
                       (const int *)dn);
    hipLaunchKernelGGL((update_batch_kernel<T>), dim3(total[kOrthoKinds - 1]), dim3(kThreads), 0, s, items_dev(),
                       reinterpret_cast<const int32_t *>(b + off_tab[kOrthoKinds - 1]), (const int *)dn);
    SBM_HIP_CHECK(hipGetLastError());
    return SBM_OK;
  }

  // step k (column k + 1 formed) for the prepared set
  void launch(int m, int k, hipStream_t s) {
    const int ncol = k + 1;
    if (ncol <= 8) {
      launch_modes<2>(ncol, k, s);
    } else if (ncol <= 16) {
      launch_modes<4>(ncol, k, s);
    } else if (ncol <= 32) {
      launch_modes<8>(ncol, k, s);
    } else if (ncol <= 64) {
      launch_modes<16>(ncol, k, s);
    } else {
      for (GItem<T> *a : set) arnoldi_orthogonalise<T>(a->c, a->V, a->vc, a->w, m, k, s);
    }
  }
};

// Reads one device double per entry of src into out (one synchronisation).
static hipError_t read_scalars(const std::vector<const double *> &src, std::vector<double> &out, hipStream_t s) {
  out.assign(src.size(), 0.0);
  for (size_t i = 0; i < src.size(); ++i) {
    hipError_t e = hipMemcpyAsync(&out[i], src[i], sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
  }
  return hipStreamSynchronize(s);
}

template <typename T>
static sbm_status gmres_batch(std::vector<GItem<T>> &items, int prec, int m, hipStream_t s) {
  const int check = 8;  // steps between residual read-backs
  PlanCache px, pv;
  OrthoPlan<T> ortho, pact, prun;
  for (auto &it : items) {
    int(*grid)[3] = it.c->ws->gs_grid[sizeof(T) == 4 ? 1 : 0];
    if (grid[0][0] == 0) gs_grid_caps<T>(grid);
    it.its = 0;
    it.done = false;
  }
  for (;;) {  // restart cycles
    std::vector<GItem<T> *> act;
    for (auto &it : items)
      if (!it.done) act.push_back(&it);
    if (act.empty()) return SBM_OK;
    // r = rhs - A x -> V_0, for every run still going
    {
      std::vector<sbm_ctx *> cs;
      std::vector<const void *> us;
      std::vector<void *> vs;
      for (auto *a : act) {
        cs.push_back(a->c);
        us.push_back(a->x);
        vs.push_back(a->w);
      }
      const sbm_status st = px.run(cs, us, vs, prec, s);
      if (st != SBM_OK) return st;
    }
    for (auto *a : act) {
      Workspace *ws = a->c->ws;
      const int64_t n = a->c->n_dofs;
      ++a->applies;
      hipLaunchKernelGGL(residual_kernel<T>, dim3(nblocks(n)), dim3(kThreads), 0, s, a->rhs, a->w, a->vc, n);
      SBM_HIP_CHECK(multidot<T>(a->vc, n, 1, a->vc, n, ws->partial, ws->h + 2 * (m + 2), s));
    }
    std::vector<double> b2;
    {
      sbm_status st = pact.prepare(act, m, s);
      if (st == SBM_OK) st = pact.gather_norms(b2, s);
      if (st != SBM_OK) return st;
    }
    std::vector<GItem<T> *> run;
    for (size_t i = 0; i < act.size(); ++i) {
      GItem<T> *a = act[i];
      const double beta = std::sqrt(b2[i]);
      a->res = beta;
      if (!(beta > a->tol_abs) || a->its >= a->max_it) {
        a->done = true;
        a->st = std::isfinite(beta) ? SBM_OK : SBM_ENOCONV;
        continue;
      }
      Workspace *ws = a->c->ws;
      const int64_t n = a->c->n_dofs;
      double *hn = ws->h + 2 * (m + 2);
      double *g = ws->gm + (size_t)(m + 1) * m + 2 * m;
      hipLaunchKernelGGL(basis_store_kernel<T>, dim3(nblocks(n)), dim3(kThreads), 0, s, a->vc, hn, 1, a->V, 0,
                         ws->m + 1, a->vc, n);
      hipLaunchKernelGGL(gmres_init_kernel, dim3(1), dim3(64), 0, s, hn, g, m);
      a->j = 0;
      a->stop = false;
      run.push_back(a);
    }
    // Arnoldi steps in chunks of `check`, the applies of each step batched over the runs
    // taking it
    for (;;) {
      std::vector<GItem<T> *> in;
      for (auto *a : run)
        if (a->j < m && a->its < a->max_it && !a->stop) in.push_back(a);
      if (in.empty()) break;
      int k0 = m, k1 = 0;
      for (auto *a : in) {
        a->j1 = std::min({m, a->j + check, a->j + (a->max_it - a->its)});
        k0 = std::min(k0, a->j);
        k1 = std::max(k1, a->j1);
      }
      for (int k = k0; k < k1; ++k) {
        std::vector<sbm_ctx *> cs;
        std::vector<const void *> us;
        std::vector<void *> vs;
        std::vector<GItem<T> *> sub;
        for (auto *a : in)
          if (a->j <= k && k < a->j1) {
            cs.push_back(a->c);
            us.push_back(a->vc);
            vs.push_back(a->w);
            sub.push_back(a);
          }
        sbm_status st = pv.run(cs, us, vs, prec, s);
        if (st == SBM_OK) st = ortho.prepare(sub, m, s);
        if (st != SBM_OK) return st;
        ortho.launch(m, k, s);
      }
      SBM_HIP_CHECK(hipGetLastError());
      // residual estimates of the chunk (gathered into one copy when every run took the same
      // steps), then the same stopping rule as a check after every step
      std::vector<std::vector<double>> rh(in.size());
      bool same = true;
      for (auto *a : in) same = same && a->j == in[0]->j && a->j1 == in[0]->j1;
      if (same && ortho.set == in) {
        const int cnt = in[0]->j1 - in[0]->j;
        std::vector<double> all;
        const sbm_status st = ortho.gather_res(in[0]->j, cnt, all, s);
        if (st != SBM_OK) return st;
        for (size_t i = 0; i < in.size(); ++i) rh[i].assign(all.begin() + i * cnt, all.begin() + (i + 1) * cnt);
      } else {
        for (size_t i = 0; i < in.size(); ++i) {
          GItem<T> *a = in[i];
          const double *dres = a->c->ws->gm + (size_t)(m + 1) * m + 2 * m + (m + 1);
          rh[i].resize(a->j1 - a->j);
          SBM_HIP_CHECK(hipMemcpyAsync(rh[i].data(), dres + a->j, sizeof(double) * (a->j1 - a->j),
                                       hipMemcpyDeviceToHost, s));
        }
        SBM_HIP_CHECK(hipStreamSynchronize(s));
      }
      for (size_t i = 0; i < in.size(); ++i) {
        GItem<T> *a = in[i];
        a->applies += a->j1 - a->j;
        int k = a->j;
        while (k < a->j1 && rh[i][k - a->j] > a->tol_abs) ++k;
        if (k < a->j1) {
          a->its += k + 1 - a->j;
          a->j = k + 1;
          a->stop = true;
        } else {
          a->its += a->j1 - a->j;
          a->j = a->j1;
        }
      }
    }
    // back substitution and update x += V y, from the leading j columns
    std::vector<GItem<T> *> fin;
    std::vector<int> ncol;
    for (auto *a : run)
      if (a->j > 0) {
        fin.push_back(a);
        ncol.push_back(a->j);
      }
    if (!fin.empty()) {
      sbm_status st = prun.prepare(fin, m, s);
      if (st == SBM_OK) st = prun.finish(ncol, s);
      if (st != SBM_OK) return st;
    }
  }
}

// FP64 applies of x for every operator listed (t = A x), then r = b - t and |r|^2 read back.
static sbm_status batch_residuals(const std::vector<sbm_ctx *> &cs, const std::vector<const double *> &b,
                                  const std::vector<double *> &x, PlanCache &plan, hipStream_t s,
                                  std::vector<double> &rn2) {
  std::vector<const void *> us(x.begin(), x.end());
  std::vector<void *> vs;
  for (sbm_ctx *c : cs) vs.push_back(c->ws->t);
  sbm_status st = plan.run(cs, us, vs, SBM_F64, s);
  if (st != SBM_OK) return st;
  std::vector<const double *> src;
  for (size_t i = 0; i < cs.size(); ++i) {
    Workspace *ws = cs[i]->ws;
    const int64_t n = cs[i]->n_dofs;
    hipLaunchKernelGGL(residual_kernel<double>, dim3(nblocks(n)), dim3(kThreads), 0, s, b[i], ws->t, ws->r, n);
    SBM_HIP_CHECK(multidot<double>(ws->r, n, 1, ws->r, n, ws->partial, ws->h, s));
    src.push_back(ws->h);
  }
  SBM_HIP_CHECK(read_scalars(src, rn2, s));
  return SBM_OK;
}

}  // namespace

static sbm_status solve_batch_on(int n, sbm_handle *hs, const double *const *b, double *const *x, double rel_tol,
                                 int max_it, int mode, int m, hipStream_t s, sbm_solve_info *infos,
                                 std::chrono::steady_clock::time_point t0) {
  std::vector<int> idx;  // operators with unknowns
  for (int i = 0; i < n; ++i) {
    if (hs[i]->n_dofs > 0) {
      idx.push_back(i);
    } else {
      infos[i].status = SBM_OK;
    }
  }
  const int q = (int)idx.size();
  if (q == 0) return SBM_OK;
  std::vector<sbm_ctx *> cs;
  std::vector<const double *> bs;
  std::vector<double *> xs;
  for (int i : idx) {
    cs.push_back(hs[i]);
    bs.push_back(b[i]);
    xs.push_back(x[i]);
  }
  // ||b|| and the absolute tolerances
  std::vector<const double *> src;
  for (int k = 0; k < q; ++k) {
    SBM_HIP_CHECK(multidot<double>(bs[k], cs[k]->n_dofs, 1, bs[k], cs[k]->n_dofs, cs[k]->ws->partial, cs[k]->ws->h, s));
    src.push_back(cs[k]->ws->h);
  }
  std::vector<double> bn2;
  SBM_HIP_CHECK(read_scalars(src, bn2, s));
  std::vector<double> bnorm(q), tol_abs(q);
  for (int k = 0; k < q; ++k) {
    bnorm[k] = std::sqrt(bn2[k]);
    tol_abs[k] = rel_tol * (bnorm[k] > 0 ? bnorm[k] : 1.0);
  }
  std::vector<sbm_status> st(q, SBM_OK);
  PlanCache p64;
  if (mode == SBM_SOLVE_GMRES_F64) {
    std::vector<GItem<double>> items(q);
    for (int k = 0; k < q; ++k) {
      Workspace *ws = cs[k]->ws;
      GItem<double> &it = items[k];
      it.c = cs[k];
      it.rhs = bs[k];
      it.x = xs[k];
      it.V = ws->V;
      it.vc = ws->vc;
      it.w = ws->w;
      it.tol_abs = tol_abs[k];
      it.max_it = max_it;
    }
    const sbm_status e = gmres_batch<double>(items, SBM_F64, m, s);
    if (e != SBM_OK) return e;
    for (int k = 0; k < q; ++k) {
      sbm_solve_info &inf = infos[idx[k]];
      inf.inner_its = items[k].its;
      inf.outer_its = (items[k].its + m - 1) / m;
      inf.applies_f64 = items[k].applies;
      st[k] = items[k].st;
    }
  } else {
    // FP64 refinement around FP32 GMRES, in lockstep: r = b - A x (FP64), c ~= A32^-1 (r / |r|)
    // by FP32 GMRES to max(1e-6, tol / (2 |r|)) in at most 4 restart cycles, x += |r| c
    std::vector<int> total(q, 0);
    std::vector<bool> live(q, true);
    for (int outer = 0;; ++outer) {
      std::vector<int> on;
      for (int k = 0; k < q; ++k)
        if (live[k]) on.push_back(k);
      if (on.empty()) break;
      std::vector<sbm_ctx *> c_on;
      std::vector<const double *> b_on;
      std::vector<double *> x_on;
      for (int k : on) {
        c_on.push_back(cs[k]);
        b_on.push_back(bs[k]);
        x_on.push_back(xs[k]);
      }
      std::vector<double> rn2;
      const sbm_status e = batch_residuals(c_on, b_on, x_on, p64, s, rn2);
      if (e != SBM_OK) return e;
      std::vector<GItem<float>> items;
      std::vector<int> of;
      std::vector<double> res_on;
      for (size_t i = 0; i < on.size(); ++i) {
        const int k = on[i];
        sbm_solve_info &inf = infos[idx[k]];
        ++inf.applies_f64;
        const double res = std::sqrt(rn2[i]);
        inf.outer_its = outer;
        if (!(res > tol_abs[k]) || total[k] >= max_it || !std::isfinite(res)) {
          live[k] = false;
          continue;
        }
        Workspace *ws = cs[k]->ws;
        const int64_t nk = cs[k]->n_dofs;
        SBM_HIP_CHECK(hipMemcpyAsync(ws->y + (m + 1), ws->h, sizeof(double), hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(to_f32_kernel, dim3(nblocks(nk)), dim3(kThreads), 0, s, ws->r, ws->y + (m + 1), ws->r32,
                           nk);
        hipLaunchKernelGGL(fill_f32_kernel, dim3(nblocks(nk)), dim3(kThreads), 0, s, ws->c32, nk);
        GItem<float> it;
        it.c = cs[k];
        it.rhs = ws->r32;
        it.x = ws->c32;
        it.V = ws->V32;
        it.vc = ws->vc32;
        it.w = ws->w32;
        it.tol_abs = std::max(1e-6, 0.5 * tol_abs[k] / res);
        it.max_it = std::min(4 * m, max_it - total[k]);
        items.push_back(it);
        of.push_back(k);
      }
      if (items.empty()) continue;
      const sbm_status ge = gmres_batch<float>(items, SBM_F32, m, s);
      if (ge != SBM_OK) return ge;
      for (size_t i = 0; i < items.size(); ++i) {
        const int k = of[i];
        sbm_solve_info &inf = infos[idx[k]];
        total[k] += items[i].its;
        inf.applies_f32 += items[i].applies;
        Workspace *ws = cs[k]->ws;
        hipLaunchKernelGGL(add_f32_kernel, dim3(nblocks(cs[k]->n_dofs)), dim3(kThreads), 0, s, ws->c32,
                           ws->y + (m + 1), xs[k], cs[k]->n_dofs);
        if (items[i].its == 0) live[k] = false;
      }
    }
    for (int k = 0; k < q; ++k) infos[idx[k]].inner_its = total[k];
  }
  // final true residuals in FP64
  std::vector<double> rn2;
  const sbm_status e = batch_residuals(cs, bs, xs, p64, s, rn2);
  if (e != SBM_OK) return e;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  sbm_status worst = SBM_OK;
  for (int k = 0; k < q; ++k) {
    sbm_solve_info &inf = infos[idx[k]];
    ++inf.applies_f64;
    inf.rel_residual = std::sqrt(rn2[k]) / (bnorm[k] > 0 ? bnorm[k] : 1.0);
    inf.seconds = secs;
    sbm_status sk = st[k];
    if (sk == SBM_OK && !(inf.rel_residual <= rel_tol)) sk = SBM_ENOCONV;
    inf.status = sk;
    if (sk != SBM_OK && worst == SBM_OK) worst = sk;
  }
  if (worst == SBM_ENOCONV) set_error("sbm_solve_batch: tolerance not reached within max_it by some systems");
  return worst;
}

extern "C" {

sbm_status sbm_l2_error(sbm_handle h, const double *x, const double *ustar_qp, double *err) {
  if (!h || !ustar_qp || !err || (h->n_dofs > 0 && !x) || h->host_only) {
    set_error("sbm_l2_error: NULL argument or host-only handle");
    return SBM_EINVAL;
  }
  *err = 0.0;
  const int d = h->dim, n1 = h->n1, nb = h->nb, np = h->nq_face;
  const Rules1D &R = h->rules;
  const int64_t nc = h->n_cells;
  if (nc == 0) return SBM_OK;
  std::vector<double> xh(h->n_dofs);
  SBM_HIP_CHECK(hipMemcpy(xh.data(), x, sizeof(double) * h->n_dofs, hipMemcpyDeviceToHost));
  // per cell: u_K at the GLL nodes -> values at the (p+1)^d Gauss points (N along each axis),
  // then sum_q W_q h^d (u_h - u*)^2; partial sums per cell, added in cell order
  std::vector<double> part(nc);
  auto cells = [&](int64_t r0, int64_t r1) {
    std::vector<double> A(nb), B(nb);
    for (int64_t r = r0; r < r1; ++r) {
      for (int i = 0; i < nb; ++i)
        A[i] = xh[(h->disc == SBM_CG) ? (int64_t)h->runs[r * np + i / n1] + i % n1 : r * nb + i];
      double *src = A.data(), *dst = B.data();
      int st = 1;
      for (int m = 0; m < d; ++m) {
        for (int idx = 0; idx < nb; ++idx) {
          const int q = (idx / st) % n1, base = idx - q * st;
          double acc = 0.0;
          for (int j = 0; j < n1; ++j) acc += R.N[q * n1 + j] * src[base + j * st];
          dst[idx] = acc;
        }
        std::swap(src, dst);
        st *= n1;
      }
      double s = 0.0;
      for (int q = 0; q < nb; ++q) {
        const int qk[3] = {q % n1, (q / n1) % n1, q / (n1 * n1)};
        double w = 1.0;
        for (int m = 0; m < d; ++m) w *= R.w[qk[m]] * h->h;
        const double e = src[q] - ustar_qp[r * nb + q];
        s += w * e * e;
      }
      part[r] = s;
    }
  };
  const int64_t nt = std::max<int64_t>(1, std::min<int64_t>({(int64_t)std::thread::hardware_concurrency(), 16, nc / 1024}));
  if (nt <= 1) {
    cells(0, nc);
  } else {
    std::vector<std::thread> pool;
    for (int64_t t = 0; t < nt; ++t) pool.emplace_back([&, t] { cells(nc * t / nt, nc * (t + 1) / nt); });
    for (auto &th : pool) th.join();
  }
  double tot = 0.0;
  for (int64_t r = 0; r < nc; ++r) tot += part[r];
  *err = std::sqrt(tot);
  return SBM_OK;
}

sbm_status sbm_rhs(sbm_handle h, const double *f_qp, const double *g_bp, double *b, void *stream) {
  if (!h || !f_qp || !b || (h->n_sbm > 0 && !g_bp) || h->host_only) {
    set_error("sbm_rhs: NULL argument or host-only handle");
    return SBM_EINVAL;
  }
  const int d = h->dim, n1 = h->n1, nb = h->nb, np = h->nq_face, P = h->p;
  const Rules1D &R = h->rules;
  const int64_t nc = h->n_cells, nf = h->n_sbm;
  // Every integral is a tensor-product quadrature, so the transposed interpolation to the
  // basis is done axis by axis (N^T along each axis in turn):
  //   cell r:  loc_i = sum_q psi_i(g_q) W_q h^d f(x_q)
  //   face:    loc_i = c(i_a) T(i_t), T = sum_q psi_t(g_q) omega_q g(x_q) (tangential axes),
  //            c(i_a) = sigma [i_a = s p] - sgn / h l'_{i_a}(s)   (sigma g v - g dv/dn~)
  // Each DoF sums its contributions in entity order: all cells in rank order, then all faces
  // in face order.  The work is split over host threads without changing that order: DG
  // cells own disjoint blocks (each face adds to its cell's block, the faces of a cell in face
  // order); CG cells are split into chunks that accumulate into private DoF ranges, which are
  // then added in chunk order (a chunk's zero entries add exactly nothing).
  auto contract = [&](const double *in, double *out, int dims, int axis) {
    // out = contraction of in (n1 points per axis, `dims` axes, first fastest) with N^T along axis
    int st = 1;
    for (int m = 0; m < axis; ++m) st *= n1;
    int outer = 1;
    for (int m = axis + 1; m < dims; ++m) outer *= n1;
    const double *N = R.N.data();
    for (int o = 0; o < outer; ++o) {
      const double *src = in + (size_t)o * n1 * st;
      double *dst = out + (size_t)o * n1 * st;
      for (int i = 0; i < n1; ++i)
        for (int l = 0; l < st; ++l) {
          double acc = 0.0;
          for (int q = 0; q < n1; ++q) acc += N[q * n1 + i] * src[q * st + l];
          dst[i * st + l] = acc;
        }
    }
  };
  // cell r's local vector into out (A, B: scratch of nb)
  auto cell_local = [&](int64_t r, double *A, double *B, double *out) {
    for (int q = 0; q < nb; ++q) {
      const int qk[3] = {q % n1, (q / n1) % n1, q / (n1 * n1)};
      double w = 1.0;
      for (int m = 0; m < d; ++m) w *= R.w[qk[m]] * h->h;
      A[q] = f_qp[r * nb + q] * w;
    }
    double *src = A, *dst = B;
    for (int m = 0; m < d; ++m) {
      contract(src, dst, d, m);
      std::swap(src, dst);
    }
    std::copy(src, src + nb, out);
  };
  // face f's local vector into out (A, B: scratch of np)
  auto face_local = [&](int64_t f, double *A, double *B, double *out) {
    const int32_t a = h->faces[3 * f + 1], s = h->faces[3 * f + 2];
    const double sgn = s ? 1.0 : -1.0;
    const double *Ds = s ? R.D1.data() : R.D0.data();
    for (int q = 0; q < np; ++q) {
      const int qt[2] = {q % n1, q / n1};
      double om = 1.0;
      for (int t = 0; t < d - 1; ++t) om *= R.w[qt[t]] * h->h;
      A[q] = om * g_bp[f * np + q];
    }
    double *src = A, *dst = B;
    for (int m = 0; m < d - 1; ++m) {
      contract(src, dst, d - 1, m);
      std::swap(src, dst);
    }
    double cn[kMaxN1];
    for (int ia = 0; ia < n1; ++ia) cn[ia] = (ia == s * P ? h->sigma_gamma : 0.0) - sgn / h->h * Ds[ia];
    for (int i = 0; i < nb; ++i) {
      const int ik[3] = {i % n1, (i / n1) % n1, i / (n1 * n1)};
      int jt = 0, sc = 1;
      for (int m = 0; m < d; ++m)
        if (m != a) {
          jt += ik[m] * sc;
          sc *= n1;
        }
      out[i] = cn[ik[a]] * src[jt];
    }
  };
  auto run = [](int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)> &fn) {
    const int64_t nt = std::max<int64_t>(
        1, std::min<int64_t>({(int64_t)std::thread::hardware_concurrency(), 16, n / grain}));
    if (nt <= 1) {
      fn(0, n);
      return;
    }
    std::vector<std::thread> pool;
    for (int64_t t = 0; t < nt; ++t) pool.emplace_back([&, t] { fn(n * t / nt, n * (t + 1) / nt); });
    for (auto &th : pool) th.join();
  };
  auto dof_of = [&](int64_t r, int i) -> int64_t {
    return (h->disc == SBM_CG) ? (int64_t)h->runs[r * np + i / n1] + i % n1 : r * nb + i;
  };
  std::unique_ptr<double[]> bh(new double[(size_t)std::max<int64_t>(1, h->n_dofs)]);
  if (h->disc == SBM_DG) {
    // faces of each cell, in face order (the faces are listed by cell rank, but this does not
    // rely on it)
    std::vector<int64_t> fstart(nc + 1, 0), flist(nf);
    for (int64_t f = 0; f < nf; ++f) ++fstart[h->faces[3 * f] + 1];
    for (int64_t r = 0; r < nc; ++r) fstart[r + 1] += fstart[r];
    {
      std::vector<int64_t> pos(fstart.begin(), fstart.end() - 1);
      for (int64_t f = 0; f < nf; ++f) flist[pos[h->faces[3 * f]]++] = f;
    }
    run(nc, 256, [&](int64_t r0, int64_t r1) {
      std::vector<double> A(std::max(nb, np)), B(std::max(nb, np)), L(nb);
      for (int64_t r = r0; r < r1; ++r) {
        double *blk = bh.get() + r * nb;
        cell_local(r, A.data(), B.data(), L.data());
        for (int i = 0; i < nb; ++i) blk[i] = 0.0 + L[i];
        for (int64_t k = fstart[r]; k < fstart[r + 1]; ++k) {
          face_local(flist[k], A.data(), B.data(), L.data());
          for (int i = 0; i < nb; ++i) blk[i] += L[i];
        }
      }
    });
  } else {
    // CG: chunks of cells in rank order, each into a private copy of the DoF range it touches
    const int64_t nt = std::max<int64_t>(
        1, std::min<int64_t>({(int64_t)std::thread::hardware_concurrency(), 16, nc / 64}));
    std::vector<int64_t> lo(nt), hi(nt);
    std::vector<std::vector<double>> priv(nt);
    run(nt, 1, [&](int64_t t0, int64_t t1) {
      std::vector<double> A(nb), B(nb), L(nb);
      for (int64_t t = t0; t < t1; ++t) {
        const int64_t r0 = nc * t / nt, r1 = nc * (t + 1) / nt;
        int64_t mn = INT64_MAX, mx = -1;
        for (int64_t r = r0; r < r1; ++r)
          for (int j = 0; j < np; ++j) {
            mn = std::min<int64_t>(mn, h->runs[r * np + j]);
            mx = std::max<int64_t>(mx, (int64_t)h->runs[r * np + j] + n1 - 1);
          }
        if (mx < 0) mn = mx = 0;
        lo[t] = mn;
        hi[t] = mx;
        std::vector<double> &pv = priv[t];
        pv.assign((size_t)(mx - mn + 1), 0.0);
        for (int64_t r = r0; r < r1; ++r) {
          cell_local(r, A.data(), B.data(), L.data());
          for (int i = 0; i < nb; ++i) pv[dof_of(r, i) - mn] += L[i];
        }
      }
    });
    run(h->n_dofs, 1 << 16, [&](int64_t d0, int64_t d1) {
      for (int64_t k = d0; k < d1; ++k) {
        double v = 0.0;
        for (int64_t t = 0; t < nt; ++t)
          if (lo[t] <= k && k <= hi[t]) v += priv[t][k - lo[t]];
        bh[k] = v;
      }
    });
    // the faces' local vectors in parallel, then added in face order
    std::vector<double> fl((size_t)nf * nb);
    run(nf, 64, [&](int64_t f0, int64_t f1) {
      std::vector<double> A(std::max(nb, np)), B(std::max(nb, np));
      for (int64_t f = f0; f < f1; ++f) face_local(f, A.data(), B.data(), fl.data() + (size_t)f * nb);
    });
    for (int64_t f = 0; f < nf; ++f) {
      const int32_t r = h->faces[3 * f];
      const double *L = fl.data() + (size_t)f * nb;
      for (int i = 0; i < nb; ++i) bh[dof_of(r, i)] += L[i];
    }
  }
  SBM_HIP_CHECK(hipMemcpyAsync(b, bh.get(), (size_t)h->n_dofs * sizeof(double), hipMemcpyHostToDevice,
                               (hipStream_t)stream));
  SBM_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
  return SBM_OK;
}

sbm_status sbm_solve_batch(int n, const sbm_handle *hs, const double *const *b, double *const *x, double rel_tol,
                           int max_it, int mode, int restart, void *stream, sbm_solve_info *infos) {
  const auto t0 = std::chrono::steady_clock::now();
  if (n < 0 || (n > 0 && (!hs || !b || !x || !infos)) || !(rel_tol > 0) || max_it < 1) {
    set_error("sbm_solve_batch: invalid argument");
    return SBM_EINVAL;
  }
  for (int i = 0; i < n; ++i) std::memset(&infos[i], 0, sizeof(sbm_solve_info));
  if (mode != SBM_SOLVE_GMRES_F64 && mode != SBM_SOLVE_GMRES_IR) {
    set_error("sbm_solve_batch: only SBM_SOLVE_GMRES_F64 and SBM_SOLVE_GMRES_IR are batched");
    for (int i = 0; i < n; ++i) infos[i].status = SBM_EUNSUPPORTED;
    return SBM_EUNSUPPORTED;
  }
  std::vector<const sbm_ctx *> seen;
  for (int i = 0; i < n; ++i) {
    const sbm_ctx *c = hs[i];
    const bool bad = !c || c->host_only || (c->n_dofs > 0 && (!b[i] || !x[i] || (const void *)b[i] == x[i])) ||
                     std::find(seen.begin(), seen.end(), c) != seen.end();
    if (bad) {
      set_error("sbm_solve_batch: NULL, host-only or repeated handle, or NULL or aliased vectors");
      for (int k = 0; k < n; ++k) infos[k].status = SBM_EINVAL;
      return SBM_EINVAL;
    }
    seen.push_back(c);
  }
  const int m = restart > 0 ? std::min(restart, kMaxRestart) : 50;
  for (int i = 0; i < n; ++i) {
    if (hs[i]->n_dofs == 0) continue;
    const hipError_t e = ensure_workspace(hs[i], m, mode == SBM_SOLVE_GMRES_IR);
    if (e != hipSuccess) {
      set_error(std::string("sbm_solve_batch: workspace allocation failed: ") + hipGetErrorString(e));
      for (int k = 0; k < n; ++k) infos[k].status = SBM_ENOMEM;
      return SBM_ENOMEM;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<sbm_handle> hv(hs, hs + n);
  sbm_status st = solve_batch_on(n, hv.data(), b, x, rel_tol, max_it, mode, m, s, infos, t0);
  const hipError_t se = hipStreamSynchronize(s);
  if (st == SBM_OK && se != hipSuccess) {
    set_error(std::string("sbm_solve_batch: ") + hipGetErrorString(se));
    st = SBM_EHIP;
  }
  if (st == SBM_EHIP || st == SBM_ENOMEM || st == SBM_EINVAL)
    for (int k = 0; k < n; ++k)
      if (infos[k].status == SBM_OK) infos[k].status = st;
  return st;
}

sbm_status sbm_diagonal(sbm_handle h, void *diag, int prec, void *stream) {
  if (!h || (!diag && h->n_dofs > 0) || h->host_only || (prec != SBM_F64 && prec != SBM_F32)) {
    set_error("sbm_diagonal: invalid argument");
    return SBM_EINVAL;
  }
  if (h->n_dofs == 0) return SBM_OK;
  hipError_t e = launch_operator_diagonal(h, diag, prec, (hipStream_t)stream);
  if (e == hipErrorNotSupported) {
    set_error("sbm_diagonal: not available for this discretisation");
    return SBM_EUNSUPPORTED;
  }
  SBM_HIP_CHECK(e);
  note_work(h, (hipStream_t)stream);
  return SBM_OK;
}

sbm_status sbm_solve(sbm_handle h, const double *b, double *x, double rel_tol, int max_it, int mode,
                     int restart, int jacobi, void *stream, sbm_solve_info *info) {
  const auto t0 = std::chrono::steady_clock::now();
  sbm_solve_info loc{};
  if (!info) info = &loc;
  std::memset(info, 0, sizeof(*info));
  if (!h || h->host_only || (h->n_dofs > 0 && (!b || !x)) || !(rel_tol > 0) || max_it < 1 ||
      (mode != SBM_SOLVE_GMRES_F64 && mode != SBM_SOLVE_GMRES_IR && mode != SBM_SOLVE_CG_F64 &&
       mode != SBM_SOLVE_CG_IR && mode != SBM_SOLVE_CG_RR)) {
    set_error("sbm_solve: invalid argument");
    info->status = SBM_EINVAL;
    return SBM_EINVAL;
  }
  if (h->n_dofs == 0) {
    info->status = SBM_OK;
    return SBM_OK;
  }
  const bool cg = mode == SBM_SOLVE_CG_F64 || mode == SBM_SOLVE_CG_IR || mode == SBM_SOLVE_CG_RR;
  // CG needs no Krylov basis: one spare column of it serves as a work vector
  const int m = cg ? 1 : (restart > 0 ? std::min(restart, kMaxRestart) : 50);
  hipError_t e =
      ensure_workspace(h, m, mode == SBM_SOLVE_GMRES_IR || mode == SBM_SOLVE_CG_IR || mode == SBM_SOLVE_CG_RR);
  if (e != hipSuccess) {
    set_error(std::string("sbm_solve: workspace allocation failed: ") + hipGetErrorString(e));
    info->status = SBM_ENOMEM;
    return SBM_ENOMEM;
  }
  Workspace *ws = h->ws;
  // everything below runs on the workspace's stream, after the work already on the caller's
  // stream; the call returns when it has finished (so later work on the caller's stream sees x)
  SBM_HIP_CHECK(hipEventRecord(ws->ready, (hipStream_t)stream));
  SBM_HIP_CHECK(hipStreamWaitEvent(ws->stream, ws->ready, 0));
  hipStream_t s = ws->stream;
  const sbm_status st = solve_on(h, b, x, rel_tol, max_it, mode, m, jacobi, s, info, t0);
  const hipError_t se = hipStreamSynchronize(s);
  if (st == SBM_OK && se != hipSuccess) {
    set_error(std::string("sbm_solve: ") + hipGetErrorString(se));
    info->status = SBM_EHIP;
    return SBM_EHIP;
  }
  return st;
}

}  // extern "C"
