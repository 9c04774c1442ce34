// Operator setup on the device for the analytic level-set kinds (Sec. 4.4: the SBM data --
// active cells, surrogate faces, closest points -- are computed once per geometry; Sec. 3.4:
// the precomputed per-face data and the DoF maps).  The same results as the host build in
// setup.cpp, produced by kernels and prefix sums:
//
//   vertices -> phi < 0 flags -> active cells (all 2^d vertices inside) -> scan -> cell ranks
//   cells x 2d faces -> surrogate/interior flags -> scan -> surrogate-face list (cell, axis, side)
//   face points -> closest point (levelset.h, shared with the host) -> shifted points xi
//   CG: touched lattice points -> scan -> DoF ids; x-run bases; bricks (counts on the device,
//       their order from order_bricks on the host: a few thousand integers), each brick's cells
//       and faces, lattice-row descriptors, brick-boundary (halo) numbering
//
// Orders are those of the host build: cells lexicographic (first coordinate fastest), faces by
// (cell, axis, side), DoFs by lattice rank, a brick's cells and faces by cell rank.  Every value
// is an integer or comes from the same floating-point operations as on the host (this file is
// compiled without contraction of multiply-adds), so the two builds agree bit for bit.  Each
// write goes to a slot of its own, or writes the same value (flags), so the result does not
// depend on thread order.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <vector>

#include "sbm_internal.h"

namespace sbm {
namespace {

constexpr int kT = 256;

inline int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kT - 1) / kT, 65536)); }

#define GRID_LOOP(i, n) for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); \
                             i += (int64_t)gridDim.x * blockDim.x)

struct Geo {
  int d, p, n1, np, nb;
  int64_t nx, ny, nz;        // cells per direction (nz = 1 in 2D)
  double lo[3], h;
  double shift;
};

// ---- cells and faces ----
__global__ void vertex_kernel(Geo g, LsParams L, unsigned char *vin) {
  const int64_t vx = g.nx + 1, vy = g.ny + 1, vz = g.d == 3 ? g.nz + 1 : 1;
  GRID_LOOP(v, vx * vy * vz) {
    const int64_t i = v % vx, j = (v / vx) % vy, k = v / (vx * vy);
    double x[3] = {g.lo[0] + g.h * i, g.lo[1] + g.h * j, g.d == 3 ? g.lo[2] + g.h * k : 0.0};
    vin[v] = ls_phi(L, x) < 0.0;
  }
}

__global__ void cell_flag_kernel(Geo g, const unsigned char *vin, int32_t *act) {
  const int64_t vx = g.nx + 1, vy = g.ny + 1;
  GRID_LOOP(ci, g.nx * g.ny * g.nz) {
    const int64_t i = ci % g.nx, j = (ci / g.nx) % g.ny, k = ci / (g.nx * g.ny);
    bool in = true;
    for (int o = 0; o < (1 << g.d) && in; ++o) {
      const int64_t ii = i + (o & 1), jj = j + ((o >> 1) & 1), kk = k + ((o >> 2) & 1);
      in = vin[(kk * vy + jj) * vx + ii] != 0;
    }
    act[ci] = in ? 1 : 0;
  }
}

// cells[r] = multi-index of the r-th active cell; rank_grid[ci] = r or -1
__global__ void cell_list_kernel(Geo g, const int32_t *act, const int32_t *pre, int32_t *cells, int32_t *rank_grid) {
  GRID_LOOP(ci, g.nx * g.ny * g.nz) {
    if (act[ci]) {
      const int32_t r = pre[ci];
      cells[(int64_t)r * g.d + 0] = (int32_t)(ci % g.nx);
      cells[(int64_t)r * g.d + 1] = (int32_t)((ci / g.nx) % g.ny);
      if (g.d == 3) cells[(int64_t)r * g.d + 2] = (int32_t)(ci / (g.nx * g.ny));
      rank_grid[ci] = r;
    } else {
      rank_grid[ci] = -1;
    }
  }
}

__device__ __forceinline__ int32_t neighbour(const Geo &g, const int32_t *cells, const int32_t *rank_grid, int64_t r,
                                             int a, int s) {
  int64_t c[3] = {cells[r * g.d], cells[r * g.d + 1], g.d == 3 ? cells[r * g.d + 2] : 0};
  c[a] += s ? 1 : -1;
  const int64_t n[3] = {g.nx, g.ny, g.nz};
  if (c[a] < 0 || c[a] >= n[a]) return -1;
  return rank_grid[(c[2] * g.ny + c[1]) * g.nx + c[0]];
}

// per (cell, code = 2 axis + side): surrogate flag and interior-face flag (side 1 only)
__global__ void face_flag_kernel(Geo g, int64_t nc, const int32_t *cells, const int32_t *rank_grid, int32_t *sflag,
                                 int32_t *iflag) {
  const int nf = 2 * g.d;
  GRID_LOOP(e, nc * nf) {
    const int64_t r = e / nf;
    const int code = (int)(e % nf);
    const int32_t nr = neighbour(g, cells, rank_grid, r, code >> 1, code & 1);
    sflag[e] = nr < 0 ? 1 : 0;
    iflag[e] = (nr >= 0 && (code & 1)) ? 1 : 0;
  }
}

__global__ void face_list_kernel(Geo g, int64_t nc, const int32_t *cells, const int32_t *rank_grid,
                                 const int32_t *sflag, const int32_t *fidx, int32_t *faces, int32_t *nbr) {
  const int nf = 2 * g.d;
  GRID_LOOP(e, nc * nf) {
    const int64_t r = e / nf;
    const int code = (int)(e % nf);
    const int32_t f = fidx[e];
    if (sflag[e]) {
      faces[3 * (int64_t)f] = (int32_t)r;
      faces[3 * (int64_t)f + 1] = code >> 1;
      faces[3 * (int64_t)f + 2] = code & 1;
    }
    if (nbr) nbr[e] = sflag[e] ? -2 - f : neighbour(g, cells, rank_grid, r, code >> 1, code & 1);
  }
}

struct Gauss {
  double g[kMaxN1];
};

// xi = xi~ + shift (x - x~) / h at every face Gauss point (host order of the points)
__global__ void project_kernel(Geo g, int64_t nfaces, LsParams L, Gauss gq, const int32_t *faces,
                               const int32_t *cells, double *xi, double *xtrue, int *bad) {
  const int d = g.d;
  GRID_LOOP(e, nfaces * g.np) {
    const int64_t f = e / g.np;
    const int q = (int)(e % g.np);
    const int32_t r = faces[3 * f], a = faces[3 * f + 1], s = faces[3 * f + 2];
    double xt[3] = {0, 0, 0}, xx[3] = {0, 0, 0}, cp[3] = {0, 0, 0};
    int qq = q;
    for (int k = 0; k < d; ++k) {
      if (k == a) {
        xt[k] = (double)s;
      } else {
        xt[k] = gq.g[qq % g.n1];
        qq /= g.n1;
      }
      xx[k] = g.lo[k] + g.h * ((double)cells[(int64_t)r * d + k] + xt[k]);
    }
    ls_closest(L, xx, cp);
    bool ok = true;
    for (int k = 0; k < d; ++k) {
      const double xs = xt[k] + g.shift * (cp[k] - xx[k]) / g.h;
      xi[e * d + k] = xs;
      xtrue[e * d + k] = cp[k];
      ok = ok && isfinite(xs);
    }
    if (!ok) atomicOr(bad, 1);
  }
}

// ---- CG: DoF numbering ----
struct Lat {
  int64_t lx, ly, lz;
};

__global__ void touch_kernel(Geo g, Lat lt, int64_t nc, const int32_t *cells, int32_t *lflag) {
  const int64_t per = g.nb;
  GRID_LOOP(e, nc * per) {
    const int64_t r = e / per;
    const int loc = (int)(e % per);
    const int i = loc % g.n1, j = (loc / g.n1) % g.n1, k = g.d == 3 ? loc / (g.n1 * g.n1) : 0;
    const int64_t m0 = (int64_t)g.p * cells[r * g.d] + i, m1 = (int64_t)g.p * cells[r * g.d + 1] + j;
    const int64_t m2 = g.d == 3 ? (int64_t)g.p * cells[r * g.d + 2] + k : 0;
    lflag[(m2 * lt.ly + m1) * lt.lx + m0] = 1;
  }
}

__device__ __forceinline__ int32_t lat_id(const Lat &lt, const int32_t *lflag, const int32_t *lpre, int64_t X,
                                          int64_t Y, int64_t Z) {
  const int64_t m = (Z * lt.ly + Y) * lt.lx + X;
  return lflag[m] ? lpre[m] : -1;
}

__global__ void runs_kernel(Geo g, Lat lt, int64_t nc, const int32_t *cells, const int32_t *lflag,
                            const int32_t *lpre, int32_t *runs) {
  GRID_LOOP(e, nc * g.np) {
    const int64_t r = e / g.np;
    const int t = (int)(e % g.np);
    const int j = t % g.n1, k = g.d == 3 ? t / g.n1 : 0;
    const int64_t m0 = (int64_t)g.p * cells[r * g.d], m1 = (int64_t)g.p * cells[r * g.d + 1] + j;
    const int64_t m2 = g.d == 3 ? (int64_t)g.p * cells[r * g.d + 2] + k : 0;
    runs[e] = lat_id(lt, lflag, lpre, m0, m1, m2);
  }
}

// ---- CG: bricks ----
struct Bricks {
  int BX, BY, BZ, LX, LY, LZ, nrows;
  int64_t nbx, nby, nbz;
};

__device__ __forceinline__ int64_t brick_key(const Geo &g, const Bricks &bk, const int32_t *cc) {
  const int64_t bz = g.d == 3 ? cc[2] / bk.BZ : 0;
  return (bz * bk.nby + cc[1] / bk.BY) * bk.nbx + cc[0] / bk.BX;
}

__device__ __forceinline__ int32_t cell_loc(const Geo &g, const Bricks &bk, const int32_t *cc) {
  const int64_t ox = cc[0] % bk.BX, oy = cc[1] % bk.BY, oz = g.d == 3 ? cc[2] % bk.BZ : 0;
  return (int32_t)(ox * g.p + oy * g.p * bk.LX + oz * g.p * bk.LX * bk.LY);
}

__device__ __forceinline__ bool cell_active(const Geo &g, const int32_t *rank_grid, int64_t i, int64_t j, int64_t k) {
  if (i < 0 || j < 0 || k < 0 || i >= g.nx || j >= g.ny || k >= g.nz) return false;
  return rank_grid[(k * g.ny + j) * g.nx + i] >= 0;
}

__global__ void brick_count_kernel(Geo g, Bricks bk, int64_t nc, int64_t nf, const int32_t *cells, const int32_t *faces,
                                   int32_t *count, int32_t *fcount) {
  GRID_LOOP(e, nc + nf) {
    if (e < nc) {
      atomicAdd(&count[brick_key(g, bk, cells + e * g.d)], 1);
    } else {
      const int64_t r = faces[3 * (e - nc)];
      atomicAdd(&fcount[brick_key(g, bk, cells + r * g.d)], 1);
    }
  }
}

// A brick's cells in rank order: the position of a cell is the number of active cells of its
// brick that come before it (z, then y, then x, as the ranks).
__global__ void brick_cells_kernel(Geo g, Bricks bk, int64_t nc, const int32_t *cells, const int32_t *rank_grid,
                                   const int32_t *bid, const int32_t *cell_off, const int32_t *runs,
                                   int32_t *brick_cell_loc, int32_t *brick_runs) {
  GRID_LOOP(r, nc) {
    const int32_t *cc = cells + r * g.d;
    const int64_t key = brick_key(g, bk, cc);
    const int64_t x0 = cc[0] - cc[0] % bk.BX, y0 = cc[1] - cc[1] % bk.BY;
    const int64_t z0 = g.d == 3 ? cc[2] - cc[2] % bk.BZ : 0;
    const int64_t me = ((g.d == 3 ? cc[2] : 0) - z0) * bk.BY * bk.BX + (cc[1] - y0) * bk.BX + (cc[0] - x0);
    int pos = 0;
    for (int64_t q = 0; q < me; ++q) {
      const int64_t ox = q % bk.BX, oy = (q / bk.BX) % bk.BY, oz = q / (bk.BX * bk.BY);
      pos += cell_active(g, rank_grid, x0 + ox, y0 + oy, z0 + oz) ? 1 : 0;
    }
    const int64_t i = cell_off[bid[key]] + pos;
    brick_cell_loc[i] = cell_loc(g, bk, cc);
    for (int t = 0; t < g.np; ++t) brick_runs[i * g.np + t] = runs[r * g.np + t];
  }
}

// A brick's faces in host face order: after the faces of the brick's earlier cells, and after
// the earlier faces of the same cell.
__global__ void brick_faces_kernel(Geo g, Bricks bk, int64_t nf, const int32_t *cells, const int32_t *rank_grid,
                                   const int32_t *faces, const int32_t *sflag, const int32_t *fidx,
                                   const int32_t *bid, const int32_t *face_off, const int32_t *runs,
                                   const double *xi_host, int32_t *face_loc, int32_t *dface_cell,
                                   int32_t *dface_code, double *dface_xi, int32_t *face_runs) {
  const int ncode = 2 * g.d;
  GRID_LOOP(f, nf) {
    const int32_t r = faces[3 * f];
    const int32_t *cc = cells + (int64_t)r * g.d;
    const int64_t key = brick_key(g, bk, cc);
    const int64_t x0 = cc[0] - cc[0] % bk.BX, y0 = cc[1] - cc[1] % bk.BY;
    const int64_t z0 = g.d == 3 ? cc[2] - cc[2] % bk.BZ : 0;
    const int64_t me = ((g.d == 3 ? cc[2] : 0) - z0) * bk.BY * bk.BX + (cc[1] - y0) * bk.BX + (cc[0] - x0);
    int64_t pos = f - fidx[(int64_t)r * ncode];  // earlier faces of the same cell
    for (int64_t q = 0; q < me; ++q) {
      const int64_t ox = x0 + q % bk.BX, oy = y0 + (q / bk.BX) % bk.BY, oz = z0 + q / (bk.BX * bk.BY);
      if (!cell_active(g, rank_grid, ox, oy, oz)) continue;
      const int64_t rr = rank_grid[(oz * g.ny + oy) * g.nx + ox];
      for (int c2 = 0; c2 < ncode; ++c2) pos += sflag[rr * ncode + c2];
    }
    const int64_t i = face_off[bid[key]] + pos;
    face_loc[i] = cell_loc(g, bk, cc);
    dface_cell[i] = r;
    dface_code[i] = 2 * faces[3 * f + 1] + faces[3 * f + 2];
    for (int e = 0; e < g.np * g.d; ++e) dface_xi[i * g.np * g.d + e] = xi_host[f * g.np * g.d + e];
    for (int t = 0; t < g.np; ++t) face_runs[i * g.np + t] = runs[(int64_t)r * g.np + t];
  }
}

// Lattice point (x, y, z) of brick b is touched by the brick's own active cells.
__device__ __forceinline__ bool brick_touched(const Geo &g, const Bricks &bk, const int32_t *rank_grid, int64_t cx0,
                                              int64_t cy0, int64_t cz0, int x, int y, int z) {
  const int p = g.p;
  int ox[2], oy[2], oz[2], nxo = 0, nyo = 0, nzo = 0;
  if (x / p < bk.BX) ox[nxo++] = x / p;
  if (x % p == 0 && x / p - 1 >= 0) ox[nxo++] = x / p - 1;
  if (y / p < bk.BY) oy[nyo++] = y / p;
  if (y % p == 0 && y / p - 1 >= 0) oy[nyo++] = y / p - 1;
  if (g.d == 3) {
    if (z / p < bk.BZ) oz[nzo++] = z / p;
    if (z % p == 0 && z / p - 1 >= 0) oz[nzo++] = z / p - 1;
  } else {
    oz[nzo++] = 0;
  }
  for (int a = 0; a < nxo; ++a)
    for (int b = 0; b < nyo; ++b)
      for (int c = 0; c < nzo; ++c)
        if (cell_active(g, rank_grid, cx0 + ox[a], cy0 + oy[b], cz0 + oz[c])) return true;
  return false;
}

__device__ __forceinline__ uint32_t boundary_mask(const Geo &g, const Bricks &bk, int y, int z, uint32_t m) {
  const uint32_t edge = 1u | (1u << (bk.LX - 1));
  const bool brow = (y == 0 || y == bk.LY - 1 || (g.d == 3 && (z == 0 || z == bk.LZ - 1)));
  return brow ? m : (m & edge);
}

__global__ void rows_kernel(Geo g, Bricks bk, Lat lt, int64_t nbricks, const int64_t *key_of,
                            const int32_t *rank_grid, const int32_t *lflag, const int32_t *lpre, int32_t *row_base,
                            uint32_t *row_gmask, uint32_t *row_bmask, int32_t *hflag) {
  GRID_LOOP(e, nbricks * bk.nrows) {
    const int64_t b = e / bk.nrows;
    const int row = (int)(e % bk.nrows);
    const int y = row % bk.LY, z = row / bk.LY;
    const int64_t key = key_of[b];
    const int64_t bx = key % bk.nbx, by = (key / bk.nbx) % bk.nby, bz = key / (bk.nbx * bk.nby);
    const int64_t X0 = bx * bk.BX * g.p, Y = by * bk.BY * g.p + y, Z = g.d == 3 ? bz * bk.BZ * g.p + z : 0;
    uint32_t gm = 0, bm = 0;
    int32_t base = 0;
    bool first = true;
    if (Y < lt.ly && Z < lt.lz) {
      for (int x = 0; x < bk.LX; ++x) {
        const int64_t X = X0 + x;
        if (X >= lt.lx) break;
        const int32_t id = lat_id(lt, lflag, lpre, X, Y, Z);
        if (id < 0) continue;
        gm |= 1u << x;
        if (first) {
          base = id;
          first = false;
        }
        if (brick_touched(g, bk, rank_grid, bx * bk.BX, by * bk.BY, g.d == 3 ? bz * bk.BZ : 0, x, y, z)) bm |= 1u << x;
      }
    }
    row_base[e] = base;
    row_gmask[e] = gm;
    row_bmask[e] = bm;
    const uint32_t hm = boundary_mask(g, bk, y, z, bm);
    for (int x = 0; x < bk.LX; ++x)
      if ((hm >> x) & 1u) hflag[base + __popc(gm & ((1u << x) - 1u))] = 1;
  }
}

__global__ void halo_dof_kernel(int64_t n, const int32_t *hflag, const int32_t *hpre, int32_t *halo_dof) {
  GRID_LOOP(g, n) {
    if (hflag[g]) halo_dof[hpre[g]] = (int32_t)g;
  }
}

__global__ void halo_rows_kernel(Geo g, Bricks bk, int64_t nbricks, const int32_t *row_base, const uint32_t *row_gmask,
                                 const uint32_t *row_bmask, const int32_t *hflag, const int32_t *hpre,
                                 int32_t *row_hbase, uint32_t *hmask32, unsigned long long *slots, int *bad) {
  GRID_LOOP(e, nbricks * bk.nrows) {
    const int row = (int)(e % bk.nrows);
    const int y = row % bk.LY, z = row / bk.LY;
    const uint32_t gm = row_gmask[e];
    const uint32_t hgm = boundary_mask(g, bk, y, z, gm), hm = boundary_mask(g, bk, y, z, row_bmask[e]);
    const int32_t base = row_base[e];
    auto hidx = [&](int x) {
      const int32_t dof = base + __popc(gm & ((1u << x) - 1u));
      return hflag[dof] ? hpre[dof] : -1;
    };
    int32_t hb = 0;
    if (hgm) hb = hidx(__ffs(hgm) - 1);
    row_hbase[e] = hb;
    int cnt = 0;
    for (int x = 0; x < bk.LX; ++x) {
      if (!((hgm >> x) & 1u)) continue;
      const int32_t h = hidx(x);
      // every boundary DoF of the row is a halo DoF, numbered consecutively along the row
      if (h < 0 || h != hb + (int32_t)__popc(hgm & ((1u << x) - 1u))) atomicOr(bad, 2);
      if ((hm >> x) & 1u) {
        const int k = (x == 0 ? 1 : 0) | (y == 0 ? 2 : 0) | ((g.d == 3 && z == 0) ? 4 : 0);
        if (h >= 0) atomicOr(&hmask32[h], 1u << k);
        ++cnt;
      }
    }
    if (cnt) atomicAdd(slots, (unsigned long long)cnt);
  }
}

__global__ void to_u8_kernel(int64_t n, const uint32_t *in, uint8_t *out) {
  GRID_LOOP(i, n) { out[i] = (uint8_t)in[i]; }
}

__global__ void fill_i32_kernel(int64_t n, int32_t v, int32_t *out) {
  GRID_LOOP(i, n) { out[i] = v; }
}

// ---- helpers ----
struct Temps {
  hipStream_t s;
  std::vector<void *> ptrs;
  hipError_t err = hipSuccess;
  template <typename T>
  T *get(int64_t n) {
    void *p = nullptr;
    if (err != hipSuccess) return nullptr;
    err = hipMallocAsync(&p, (size_t)std::max<int64_t>(1, n) * sizeof(T), s);
    if (err != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return (T *)p;
  }
  ~Temps() {
    for (void *p : ptrs) (void)hipFreeAsync(p, s);
  }
};

// exclusive prefix sum of n int32 (in place allowed); returns the total through *total (host)
hipError_t exclusive_scan(Temps &tmp, const int32_t *in, int32_t *out, int64_t n, int64_t *total) {
  *total = 0;
  if (n == 0) return hipSuccess;
  size_t bytes = 0;
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, (int)n, tmp.s);
  if (e != hipSuccess) return e;
  void *ws = tmp.get<char>((int64_t)bytes);
  if (!ws) return tmp.err;
  e = hipcub::DeviceScan::ExclusiveSum(ws, bytes, in, out, (int)n, tmp.s);
  if (e != hipSuccess) return e;
  int32_t last_in = 0, last_out = 0;
  e = hipMemcpyAsync(&last_in, in + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, tmp.s);
  if (e == hipSuccess) e = hipMemcpyAsync(&last_out, out + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, tmp.s);
  if (e == hipSuccess) e = hipStreamSynchronize(tmp.s);
  *total = (int64_t)last_in + last_out;
  return e;
}

// The handle's arena: every array on a 256-byte boundary, one allocation.
struct Carve {
  size_t off = 0;
  std::vector<std::pair<void **, size_t>> items;
  template <typename T>
  void add(T *&ptr, int64_t n) {
    ptr = nullptr;
    if (n <= 0) return;
    items.push_back({(void **)&ptr, off});
    off += ((size_t)n * sizeof(T) + 255) / 256 * 256;
  }
  void add_bytes(void *&ptr, size_t bytes) {
    ptr = nullptr;
    if (bytes == 0) return;
    items.push_back({&ptr, off});
    off += (bytes + 255) / 256 * 256;
  }
  hipError_t commit(void **arena) {
    *arena = nullptr;
    if (off == 0) return hipSuccess;
    hipError_t e = dev_alloc(arena, off);
    if (e != hipSuccess) return e;
    for (auto &it : items) *it.first = (char *)*arena + it.second;
    return hipSuccess;
  }
};

sbm_status fail(const char *what, hipError_t e) {
  set_error(std::string("sbm_setup (device build): ") + what + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? SBM_ENOMEM : SBM_EHIP;
}

#define DS_CHECK(expr, what)                 \
  do {                                       \
    hipError_t _e = (expr);                  \
    if (_e != hipSuccess) return fail(what, _e); \
  } while (0)

sbm_status device_setup_impl(sbm_ctx *c, Temps &tmp) {
  const hipStream_t s = tmp.s;
  Geo g{};
  g.d = c->dim;
  g.p = c->p;
  g.n1 = c->p + 1;
  g.np = c->nq_face;
  g.nb = c->nb;
  g.nx = c->n[0];
  g.ny = c->n[1];
  g.nz = g.d == 3 ? c->n[2] : 1;
  for (int k = 0; k < 3; ++k) g.lo[k] = c->lo[k];
  g.h = c->h;
  g.shift = c->shift_scale;
  const int d = g.d;
  const int64_t ncell_grid = g.nx * g.ny * g.nz;
  const int64_t nvert = (g.nx + 1) * (g.ny + 1) * (d == 3 ? g.nz + 1 : 1);
  if (nvert >= (int64_t)INT32_MAX / (2 * 3)) {
    set_error("sbm_setup: background mesh too large for the device build");
    return SBM_EUNSUPPORTED;
  }

  // level set on the device (sphere-union arrays copied)
  LsParams L = c->ls.params();
  if (L.kind == SBM_LS_SPHERE_UNION) {
    double *dcs = tmp.get<double>(3 * (int64_t)L.n_spheres), *drs = tmp.get<double>(L.n_spheres);
    DS_CHECK(tmp.err, "allocation");
    DS_CHECK(hipMemcpyAsync(dcs, L.cs, sizeof(double) * 3 * L.n_spheres, hipMemcpyHostToDevice, s), "upload");
    DS_CHECK(hipMemcpyAsync(drs, L.rs, sizeof(double) * L.n_spheres, hipMemcpyHostToDevice, s), "upload");
    L.cs = dcs;
    L.rs = drs;
  }

  // ---- active cells ----
  unsigned char *vin = tmp.get<unsigned char>(nvert);
  int32_t *act = tmp.get<int32_t>(ncell_grid), *pre = tmp.get<int32_t>(ncell_grid);
  int32_t *rank_grid = tmp.get<int32_t>(ncell_grid);
  DS_CHECK(tmp.err, "allocation");
  hipLaunchKernelGGL(vertex_kernel, dim3(grid_for(nvert)), dim3(kT), 0, s, g, L, vin);
  hipLaunchKernelGGL(cell_flag_kernel, dim3(grid_for(ncell_grid)), dim3(kT), 0, s, g, vin, act);
  int64_t nc = 0;
  DS_CHECK(exclusive_scan(tmp, act, pre, ncell_grid, &nc), "cell scan");
  c->n_cells = nc;
  int32_t *cells = tmp.get<int32_t>(nc * d);
  DS_CHECK(tmp.err, "allocation");
  hipLaunchKernelGGL(cell_list_kernel, dim3(grid_for(ncell_grid)), dim3(kT), 0, s, g, act, pre, cells, rank_grid);

  // ---- faces ----
  const int64_t ne = nc * 2 * d;
  int32_t *sflag = tmp.get<int32_t>(ne), *iflag = tmp.get<int32_t>(ne), *fidx = tmp.get<int32_t>(ne);
  int32_t *ipre = tmp.get<int32_t>(ne);
  DS_CHECK(tmp.err, "allocation");
  int64_t nf = 0, nint = 0;
  if (nc > 0) {
    hipLaunchKernelGGL(face_flag_kernel, dim3(grid_for(ne)), dim3(kT), 0, s, g, nc, cells, rank_grid, sflag, iflag);
    DS_CHECK(exclusive_scan(tmp, sflag, fidx, ne, &nf), "face scan");
    DS_CHECK(exclusive_scan(tmp, iflag, ipre, ne, &nint), "interior-face scan");
  }
  c->n_sbm = nf;
  c->n_int = nint;
  int32_t *faces = tmp.get<int32_t>(3 * nf);
  double *xi_h = tmp.get<double>(nf * g.np * d), *xtrue = tmp.get<double>(nf * g.np * d);
  int *bad = tmp.get<int>(1);
  DS_CHECK(tmp.err, "allocation");
  DS_CHECK(hipMemsetAsync(bad, 0, sizeof(int), s), "memset");

  const bool cg = c->disc == SBM_CG;
  // DG neighbour table is written straight into its arena slot below; first the CG layout
  int32_t *runs = nullptr, *lflag = nullptr, *lpre = nullptr;
  Lat lt{0, 0, 0};
  Bricks bk{};
  std::vector<int64_t> key_of;
  std::vector<int32_t> bid, cell_off, face_off;
  int64_t n_dofs = 0, n_halo = 0;
  if (cg) {
    lt.lx = (int64_t)g.p * g.nx + 1;
    lt.ly = (int64_t)g.p * g.ny + 1;
    lt.lz = d == 3 ? (int64_t)g.p * g.nz + 1 : 1;
    const int64_t nl = lt.lx * lt.ly * lt.lz;
    if (nl >= (int64_t)INT32_MAX) {
      set_error("sbm_setup: the DoF lattice has more than 2^31-1 points");
      return SBM_EUNSUPPORTED;
    }
    lflag = tmp.get<int32_t>(nl);
    lpre = tmp.get<int32_t>(nl);
    runs = tmp.get<int32_t>(nc * g.np);
    DS_CHECK(tmp.err, "allocation");
    DS_CHECK(hipMemsetAsync(lflag, 0, sizeof(int32_t) * nl, s), "memset");
    if (nc > 0)
      hipLaunchKernelGGL(touch_kernel, dim3(grid_for(nc * g.nb)), dim3(kT), 0, s, g, lt, nc, cells, lflag);
    DS_CHECK(exclusive_scan(tmp, lflag, lpre, nl, &n_dofs), "DoF scan");
    if (nc > 0)
      hipLaunchKernelGGL(runs_kernel, dim3(grid_for(nc * g.np)), dim3(kT), 0, s, g, lt, nc, cells, lflag, lpre, runs);
  } else {
    if (nc * (int64_t)c->nb >= (int64_t)INT32_MAX) {
      set_error("sbm_setup: more than 2^31-1 DoFs");
      return SBM_EUNSUPPORTED;
    }
    n_dofs = nc * c->nb;
  }
  c->n_dofs = n_dofs;

  // face list (and, for DG, the neighbour table in a temporary) and the closest points
  int32_t *nbr_t = cg ? nullptr : tmp.get<int32_t>(ne);
  DS_CHECK(tmp.err, "allocation");
  if (nc > 0)
    hipLaunchKernelGGL(face_list_kernel, dim3(grid_for(ne)), dim3(kT), 0, s, g, nc, cells, rank_grid, sflag, fidx, faces,
                       nbr_t);
  Gauss gq{};
  for (int q = 0; q < g.n1; ++q) gq.g[q] = c->rules.g[q];
  if (nf > 0)
    hipLaunchKernelGGL(project_kernel, dim3(grid_for(nf * g.np)), dim3(kT), 0, s, g, nf, L, gq, faces, cells, xi_h,
                       xtrue, bad);

  // ---- CG bricks ----
  int32_t *d_bid = nullptr;
  int64_t *d_key_of = nullptr;
  int32_t *hflag = nullptr, *hpre = nullptr;
  if (cg) {
    int BX, BY, BZ;
    brick_dims(d, g.p, &BX, &BY, &BZ);
    if (d == 2) BZ = 1;
    c->brick[0] = BX;
    c->brick[1] = BY;
    c->brick[2] = BZ;
    bk.BX = BX;
    bk.BY = BY;
    bk.BZ = BZ;
    bk.LX = BX * g.p + 1;
    bk.LY = BY * g.p + 1;
    bk.LZ = d == 3 ? BZ * g.p + 1 : 1;
    bk.nrows = bk.LY * bk.LZ;
    bk.nbx = (g.nx + BX - 1) / BX;
    bk.nby = (g.ny + BY - 1) / BY;
    bk.nbz = d == 3 ? (g.nz + BZ - 1) / BZ : 1;
    const int64_t nslot = bk.nbx * bk.nby * bk.nbz;
    int32_t *cnt = tmp.get<int32_t>(2 * nslot);
    DS_CHECK(tmp.err, "allocation");
    DS_CHECK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * 2 * nslot, s), "memset");
    if (nc + nf > 0)
      hipLaunchKernelGGL(brick_count_kernel, dim3(grid_for(nc + nf)), dim3(kT), 0, s, g, bk, nc, nf, cells, faces, cnt,
                         cnt + nslot);
    std::vector<int32_t> hc(2 * nslot);
    DS_CHECK(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * 2 * nslot, hipMemcpyDeviceToHost, s), "download");
    DS_CHECK(hipStreamSynchronize(s), "synchronise");
    std::vector<int32_t> count(hc.begin(), hc.begin() + nslot), fcount(hc.begin() + nslot, hc.end());
    c->n_bricks_faces = order_bricks(count, fcount, key_of, bid);
    const int64_t nbk = (int64_t)key_of.size();
    c->n_bricks = nbk;
    cell_off.assign(nbk + 1, 0);
    face_off.assign(nbk + 1, 0);
    for (int64_t b = 0; b < nbk; ++b) {
      cell_off[b + 1] = cell_off[b] + count[key_of[b]];
      face_off[b + 1] = face_off[b] + fcount[key_of[b]];
    }
    d_bid = tmp.get<int32_t>(nslot);
    d_key_of = tmp.get<int64_t>(nbk);
    DS_CHECK(tmp.err, "allocation");
    DS_CHECK(hipMemcpyAsync(d_bid, bid.data(), sizeof(int32_t) * nslot, hipMemcpyHostToDevice, s), "upload");
    if (nbk)
      DS_CHECK(hipMemcpyAsync(d_key_of, key_of.data(), sizeof(int64_t) * nbk, hipMemcpyHostToDevice, s), "upload");
    hflag = tmp.get<int32_t>(n_dofs);
    hpre = tmp.get<int32_t>(n_dofs);
    DS_CHECK(tmp.err, "allocation");
    DS_CHECK(hipMemsetAsync(hflag, 0, sizeof(int32_t) * std::max<int64_t>(1, n_dofs), s), "memset");  // >= 1 slot
  }

  // ---- the arena: the arrays the kernels and the host build upload, same order ----
  Carve cv;
  const int64_t nbk = c->n_bricks;
  const int64_t nrow_all = cg ? nbk * bk.nrows : 0;
  if (cg) {
    cv.add(c->d_runs, nc * g.np);
    cv.add(c->d_brick_cell_off, nbk + 1);
    cv.add(c->d_brick_runs, nc * g.np);
    cv.add(c->d_face_runs, nf * g.np);
    cv.add(c->d_brick_cell_loc, nc);
    cv.add(c->d_brick_face_off, nbk + 1);
    cv.add(c->d_brick_face_loc, nf);
    cv.add(c->d_row_base, nrow_all);
    cv.add(c->d_row_gmask, nrow_all);
    cv.add(c->d_row_bmask, nrow_all);
    cv.add(c->d_row_hbase, nrow_all);
  } else {
    cv.add(c->d_nbr, ne);
  }
  cv.add(c->d_face_cell, nf);
  cv.add(c->d_face_code, nf);
  cv.add(c->d_face_xi, nf * g.np * d);
  // row descriptors and the halo flags (into temporaries: the halo arrays of the arena are
  // sized by the halo count, known only after the flags' scan)
  int32_t *t_row_base = nullptr;
  uint32_t *t_row_gmask = nullptr, *t_row_bmask = nullptr;
  if (cg) {
    t_row_base = tmp.get<int32_t>(nrow_all);
    t_row_gmask = tmp.get<uint32_t>(nrow_all);
    t_row_bmask = tmp.get<uint32_t>(nrow_all);
    DS_CHECK(tmp.err, "allocation");
    if (nrow_all > 0)
      hipLaunchKernelGGL(rows_kernel, dim3(grid_for(nrow_all)), dim3(kT), 0, s, g, bk, lt, nbk, d_key_of, rank_grid,
                         lflag, lpre, t_row_base, t_row_gmask, t_row_bmask, hflag);
    DS_CHECK(exclusive_scan(tmp, hflag, hpre, n_dofs, &n_halo), "halo scan");
    c->n_halo_dofs = n_halo;
    cv.add(c->d_halo_dof, n_halo);
    cv.add(c->d_halo_mask, n_halo);
    cv.add_bytes(c->d_halo, ((size_t)1 << d) * (size_t)n_halo * sizeof(double));  // per-handle scratch
  }
  cv.add_bytes(c->d_fbuf, (size_t)nf * 2 * g.np * sizeof(double));                 // per-handle scratch
  void *arena = nullptr;
  DS_CHECK(cv.commit(&arena), "arena allocation");
  c->d_arena = arena;
  c->device_bytes = cv.off;

  if (cg) {
    DS_CHECK(hipMemcpyAsync(c->d_brick_cell_off, cell_off.data(), sizeof(int32_t) * (nbk + 1), hipMemcpyHostToDevice, s),
             "upload");
    DS_CHECK(hipMemcpyAsync(c->d_brick_face_off, face_off.data(), sizeof(int32_t) * (nbk + 1), hipMemcpyHostToDevice, s),
             "upload");
    if (nc > 0) {
      DS_CHECK(hipMemcpyAsync(c->d_runs, runs, sizeof(int32_t) * nc * g.np, hipMemcpyDeviceToDevice, s), "copy");
      hipLaunchKernelGGL(brick_cells_kernel, dim3(grid_for(nc)), dim3(kT), 0, s, g, bk, nc, cells, rank_grid, d_bid,
                         c->d_brick_cell_off, runs, c->d_brick_cell_loc, c->d_brick_runs);
    }
    if (nf > 0)
      hipLaunchKernelGGL(brick_faces_kernel, dim3(grid_for(nf)), dim3(kT), 0, s, g, bk, nf, cells, rank_grid, faces,
                         sflag, fidx, d_bid, c->d_brick_face_off, runs, xi_h, c->d_brick_face_loc, c->d_face_cell,
                         c->d_face_code, c->d_face_xi, c->d_face_runs);
    if (nrow_all > 0) {
      DS_CHECK(hipMemcpyAsync(c->d_row_base, t_row_base, sizeof(int32_t) * nrow_all, hipMemcpyDeviceToDevice, s), "copy");
      DS_CHECK(hipMemcpyAsync(c->d_row_gmask, t_row_gmask, sizeof(uint32_t) * nrow_all, hipMemcpyDeviceToDevice, s),
               "copy");
      DS_CHECK(hipMemcpyAsync(c->d_row_bmask, t_row_bmask, sizeof(uint32_t) * nrow_all, hipMemcpyDeviceToDevice, s),
               "copy");
    }
    uint32_t *hmask32 = tmp.get<uint32_t>(n_halo);
    unsigned long long *slots = tmp.get<unsigned long long>(1);
    DS_CHECK(tmp.err, "allocation");
    DS_CHECK(hipMemsetAsync(hmask32, 0, sizeof(uint32_t) * std::max<int64_t>(1, n_halo), s), "memset");
    DS_CHECK(hipMemsetAsync(slots, 0, sizeof(unsigned long long), s), "memset");
    if (n_dofs > 0)
      hipLaunchKernelGGL(halo_dof_kernel, dim3(grid_for(n_dofs)), dim3(kT), 0, s, n_dofs, hflag, hpre, c->d_halo_dof);
    if (nrow_all > 0)
      hipLaunchKernelGGL(halo_rows_kernel, dim3(grid_for(nrow_all)), dim3(kT), 0, s, g, bk, nbk, c->d_row_base,
                         c->d_row_gmask, c->d_row_bmask, hflag, hpre, c->d_row_hbase, hmask32, slots, bad);
    if (n_halo > 0)
      hipLaunchKernelGGL(to_u8_kernel, dim3(grid_for(n_halo)), dim3(kT), 0, s, n_halo, hmask32, c->d_halo_mask);
    unsigned long long hs = 0;
    DS_CHECK(hipMemcpyAsync(&hs, slots, sizeof(hs), hipMemcpyDeviceToHost, s), "download");
    DS_CHECK(hipStreamSynchronize(s), "synchronise");
    c->n_halo_slots = (int64_t)hs;
  } else {
    if (ne > 0) DS_CHECK(hipMemcpyAsync(c->d_nbr, nbr_t, sizeof(int32_t) * ne, hipMemcpyDeviceToDevice, s), "copy");
    if (nf > 0) {
      // DG face arrays in host order: cell rank and code from the face list, xi as projected
      // (the host vectors are read by the copies before the synchronisation below)
      std::vector<int32_t> hf(3 * nf);
      DS_CHECK(hipMemcpyAsync(hf.data(), faces, sizeof(int32_t) * 3 * nf, hipMemcpyDeviceToHost, s), "download");
      DS_CHECK(hipStreamSynchronize(s), "synchronise");
      std::vector<int32_t> fcell(nf), fcode(nf);
      for (int64_t f = 0; f < nf; ++f) {
        fcell[f] = hf[3 * f];
        fcode[f] = 2 * hf[3 * f + 1] + hf[3 * f + 2];
      }
      DS_CHECK(hipMemcpyAsync(c->d_face_cell, fcell.data(), sizeof(int32_t) * nf, hipMemcpyHostToDevice, s), "upload");
      DS_CHECK(hipMemcpyAsync(c->d_face_code, fcode.data(), sizeof(int32_t) * nf, hipMemcpyHostToDevice, s), "upload");
      DS_CHECK(hipMemcpyAsync(c->d_face_xi, xi_h, sizeof(double) * nf * g.np * d, hipMemcpyDeviceToDevice, s), "copy");
      DS_CHECK(hipStreamSynchronize(s), "synchronise");
    }
  }

  // ---- host copies (exports, right-hand side points, the host-side right-hand side) ----
  c->cells.resize(nc * d);
  c->faces.resize(3 * nf);
  c->face_xi.resize(nf * g.np * d);
  c->face_xtrue.resize(nf * g.np * d);
  c->runs.resize(cg ? nc * g.np : 0);
  if (nc) DS_CHECK(hipMemcpyAsync(c->cells.data(), cells, sizeof(int32_t) * nc * d, hipMemcpyDeviceToHost, s), "download");
  if (nf) {
    DS_CHECK(hipMemcpyAsync(c->faces.data(), faces, sizeof(int32_t) * 3 * nf, hipMemcpyDeviceToHost, s), "download");
    DS_CHECK(hipMemcpyAsync(c->face_xi.data(), xi_h, sizeof(double) * nf * g.np * d, hipMemcpyDeviceToHost, s),
             "download");
    DS_CHECK(hipMemcpyAsync(c->face_xtrue.data(), xtrue, sizeof(double) * nf * g.np * d, hipMemcpyDeviceToHost, s),
             "download");
  }
  if (cg && nc) DS_CHECK(hipMemcpyAsync(c->runs.data(), runs, sizeof(int32_t) * nc * g.np, hipMemcpyDeviceToHost, s),
                         "download");
  int hbad = 0;
  DS_CHECK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s), "download");
  DS_CHECK(hipStreamSynchronize(s), "synchronise");
  if (hbad & 1) {
    set_error("sbm_setup: closest-point projection failed (degenerate level set?)");
    return SBM_EINVAL;
  }
  if (hbad & 2) {
    set_error("sbm_setup: internal error: brick-boundary DoFs are not numbered consecutively along a row");
    return SBM_EUNSUPPORTED;
  }
  return SBM_OK;
}

}  // namespace

sbm_status device_setup(sbm_ctx *c) {
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return fail("stream", e);
  sbm_status st;
  {
    Temps tmp;
    tmp.s = s;
    st = device_setup_impl(c, tmp);
  }  // temporaries released (stream-ordered)
  e = hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  if (st == SBM_OK && e != hipSuccess) return fail("synchronise", e);
  return st;
}

}  // namespace sbm
