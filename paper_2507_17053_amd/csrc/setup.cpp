// Host-side setup of the SBM operator (Sec. 2 surrogate domain, Sec. 2.1 closest-point
// shifts, Sec. 3.4 per-face data) and the C-ABI entry points that do not launch kernels.
#include <algorithm>
#include <utility>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <functional>
#include <new>
#include <map>
#include <mutex>
#include <thread>

#include "sbm_internal.h"

namespace sbm {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

namespace {
constexpr int kMaxDev = 64;
std::mutex g_lib_mu;
hipStream_t g_lib_stream[kMaxDev] = {};
// Released device blocks kept for reuse, per device: (bytes, pointer), at most kCacheBytes in
// total per device; a request takes the smallest cached block that fits and is at most twice
// its size.
constexpr size_t kCacheBytes = (size_t)16 << 30;
std::mutex g_cache_mu;
std::multimap<size_t, void *> g_cache[kMaxDev];
size_t g_cached[kMaxDev] = {};
std::map<void *, std::pair<int, size_t>> g_live;  // block -> (device, bytes)
}  // namespace

hipStream_t lib_stream() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return nullptr;
  std::lock_guard<std::mutex> lock(g_lib_mu);
  if (!g_lib_stream[dev]) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    g_lib_stream[dev] = s;
  }
  return g_lib_stream[dev];
}

hipError_t dev_alloc(void **p, size_t bytes) {
  *p = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto it = g_cache[dev].lower_bound(bytes);
    if (it != g_cache[dev].end() && it->first <= 2 * bytes) {
      *p = it->second;
      g_cached[dev] -= it->first;
      g_live[*p] = {dev, it->first};
      g_cache[dev].erase(it);
      return hipSuccess;
    }
  }
  e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    // release the cache of this device and try once more
    std::vector<void *> drop;
    {
      std::lock_guard<std::mutex> lock(g_cache_mu);
      for (auto &kv : g_cache[dev]) drop.push_back(kv.second);
      g_cache[dev].clear();
      g_cached[dev] = 0;
    }
    if (drop.empty()) return e;
    for (void *q : drop) (void)hipFree(q);
    (void)hipGetLastError();
    e = hipMalloc(p, bytes);
    if (e != hipSuccess) return e;
  }
  std::lock_guard<std::mutex> lock(g_cache_mu);
  g_live[*p] = {dev, bytes};
  return hipSuccess;
}

void dev_free(void *p) {
  if (!p) return;
  std::pair<int, size_t> info{-1, 0};
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto it = g_live.find(p);
    if (it != g_live.end()) {
      info = it->second;
      g_live.erase(it);
      if (g_cached[info.first] + info.second <= kCacheBytes) {
        g_cache[info.first].emplace(info.second, p);
        g_cached[info.first] += info.second;
        return;
      }
    }
  }
  (void)hipFree(p);  // beyond the cache (this synchronises the device)
}

void note_work(sbm_ctx *c, hipStream_t stream) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  if (!c->last_work && hipEventCreateWithFlags(&c->last_work, hipEventDisableTiming) != hipSuccess) {
    c->last_work = nullptr;
    return;
  }
  (void)hipEventRecord(c->last_work, stream);
}

// ---------------------------------------------------------------------------------------
// 1D rules on [0,1] (Sec. 3.1): GLL nodes for the basis, Gauss points for quadrature.
// ---------------------------------------------------------------------------------------
static void legendre(int n, double x, double &pn, double &dpn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    pn = 1.0;
    dpn = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  dpn = n * (x * p1 - p0) / (x * x - 1.0);
}

Rules1D make_rules(int p) {
  Rules1D r;
  r.p = p;
  const int n1 = p + 1;
  // Gauss-Legendre: roots of P_{p+1} by Newton
  std::vector<double> gx(n1), gw(n1);
  if (n1 == 1) {
    gx[0] = 0.0;
    gw[0] = 2.0;
  } else {
    for (int i = 0; i < n1; ++i) {
      double x = -std::cos(M_PI * (i + 0.75) / (n1 + 0.5));
      for (int it = 0; it < 100; ++it) {
        double pn, dp;
        legendre(n1, x, pn, dp);
        const double dx = pn / dp;
        x -= dx;
        if (std::fabs(dx) < 1e-16) break;
      }
      double pn, dp;
      legendre(n1, x, pn, dp);
      gx[i] = x;
      gw[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
  }
  std::vector<int> ord(n1);
  for (int i = 0; i < n1; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return gx[a] < gx[b]; });
  r.g.resize(n1);
  r.w.resize(n1);
  for (int i = 0; i < n1; ++i) {
    r.g[i] = 0.5 * (gx[ord[i]] + 1.0);
    r.w[i] = 0.5 * gw[ord[i]];
  }
  // GLL: -1, roots of P'_p, 1
  std::vector<double> zz(n1);
  zz[0] = -1.0;
  zz[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double x = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double pn, dp;
      legendre(p, x, pn, dp);
      const double d2 = (2.0 * x * dp - p * (p + 1.0) * pn) / (1.0 - x * x);
      const double dx = dp / d2;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    zz[i] = x;
  }
  std::sort(zz.begin(), zz.end());
  r.z.resize(n1);
  for (int i = 0; i < n1; ++i) r.z[i] = 0.5 * (zz[i] + 1.0);
  r.cinv.resize(n1);
  for (int j = 0; j < n1; ++j) {
    double d = 1.0;
    for (int m = 0; m < n1; ++m)
      if (m != j) d *= (r.z[j] - r.z[m]);
    r.cinv[j] = 1.0 / d;
  }
  r.N.assign(n1 * n1, 0.0);
  r.M.assign(n1 * n1, 0.0);
  r.K.assign(n1 * n1, 0.0);
  r.D0.resize(n1);
  r.D1.resize(n1);
  std::vector<double> lv(n1 * n1), ld(n1 * n1);
  for (int q = 0; q < n1; ++q)
    for (int j = 0; j < n1; ++j) {
      lv[q * n1 + j] = lagrange_value(r, j, r.g[q]);
      ld[q * n1 + j] = lagrange_derivative(r, j, r.g[q]);
      r.N[q * n1 + j] = lv[q * n1 + j];
    }
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      double m = 0, k = 0;
      for (int q = 0; q < n1; ++q) {
        m += r.w[q] * lv[q * n1 + i] * lv[q * n1 + j];
        k += r.w[q] * ld[q * n1 + i] * ld[q * n1 + j];
      }
      r.M[i * n1 + j] = m;
      r.K[i * n1 + j] = k;
    }
  for (int j = 0; j < n1; ++j) {
    r.D0[j] = lagrange_derivative(r, j, 0.0);
    r.D1[j] = lagrange_derivative(r, j, 1.0);
  }
  return r;
}

double lagrange_value(const Rules1D &r, int j, double x) {
  double v = r.cinv[j];
  for (int m = 0; m <= r.p; ++m)
    if (m != j) v *= (x - r.z[m]);
  return v;
}

double lagrange_derivative(const Rules1D &r, int j, double x) {
  double s = 0.0;
  for (int k = 0; k <= r.p; ++k) {
    if (k == j) continue;
    double t = r.cinv[j];
    for (int m = 0; m <= r.p; ++m)
      if (m != j && m != k) t *= (x - r.z[m]);
    s += t;
  }
  return s;
}

// ---------------------------------------------------------------------------------------
// Level sets and exact closest points
// ---------------------------------------------------------------------------------------
static double norm_d(const double *v, int d) {
  double s = 0;
  for (int k = 0; k < d; ++k) s += v[k] * v[k];
  return std::sqrt(s);
}

LsParams LevelSet::params() const {
  LsParams P;
  P.kind = kind;
  P.dim = dim;
  for (int k = 0; k < 3; ++k) {
    P.centre[k] = centre[k];
    P.semi[k] = semi[k];
    P.normal[k] = normal[k];
  }
  P.radius = radius;
  P.R = R;
  P.r = r;
  P.offset = offset;
  P.n_spheres = (int)rs.size();
  P.cs = cs.data();
  P.rs = rs.data();
  return P;
}

double LevelSet::phi(const double *x) const {
  if (kind == SBM_LS_CALLBACK) {
    double xx[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) xx[k] = x[k];
    return cb_phi(xx, cb_user);
  }
  return ls_phi(params(), x);
}

// Level-set Newton projection onto {phi = 0} (the projection of Sec. 4.4): from x, repeat
// x <- x - phi(x) grad phi(x) / |grad phi(x)|^2 until the Newton step |phi| / |grad phi| is at
// most 8 eps max(1, max_k |x_k|) (a few units in the last place of the point, whatever the
// scaling of phi), at most 50 steps.  Returns false if that was not met or the gradient
// vanished.
static bool closest_newton(const LevelSet &L, const double *x, double *out) {
  const int d = L.dim;
  const double eps = std::numeric_limits<double>::epsilon();
  double y[3] = {0.0, 0.0, 0.0}, g[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < d; ++k) y[k] = x[k];
  for (int it = 0; it <= 50; ++it) {
    const double ph = L.cb_phi(y, L.cb_user);
    if (!std::isfinite(ph)) break;
    L.cb_grad(y, g, L.cb_user);
    double g2 = 0.0, ymax = 1.0;
    for (int k = 0; k < d; ++k) {
      g2 += g[k] * g[k];
      ymax = std::max(ymax, std::fabs(y[k]));
    }
    if (std::fabs(ph) <= 8.0 * eps * std::sqrt(g2) * ymax) {
      for (int k = 0; k < d; ++k) out[k] = y[k];
      return true;
    }
    if (it == 50 || !(g2 > 0.0) || !std::isfinite(g2)) break;
    for (int k = 0; k < d; ++k) y[k] -= ph * g[k] / g2;
  }
  for (int k = 0; k < d; ++k) out[k] = std::numeric_limits<double>::quiet_NaN();
  return false;
}

void LevelSet::closest(const double *x, double *out) const {
  if (kind == SBM_LS_CALLBACK) {
    closest_newton(*this, x, out);
    return;
  }
  ls_closest(params(), x, out);
}

}  // namespace sbm

using namespace sbm;

// ---------------------------------------------------------------------------------------
// Setup
// ---------------------------------------------------------------------------------------
// All device arrays of a handle live in one allocation (the arena): one hipMalloc at setup
// and one hipFree at destroy (hipFree synchronises the device, which would otherwise stall
// every other stream once per array).  Each array starts on a 256-byte boundary.
struct ArenaPlan {
  struct Item {
    std::function<void(char *)> set;
    const void *src;  // host data to copy, or nullptr for scratch
    size_t bytes;
  };
  std::vector<Item> items;
  template <typename P, typename V>
  void add(P *&ptr, const std::vector<V> &src) {
    ptr = nullptr;
    if (!src.empty())
      items.push_back({[&ptr](char *a) { ptr = reinterpret_cast<P *>(a); }, src.data(), src.size() * sizeof(V)});
  }
  void scratch(void *&ptr, size_t bytes) {
    ptr = nullptr;
    if (bytes) items.push_back({[&ptr](char *a) { ptr = a; }, nullptr, bytes});
  }
  static size_t aligned(size_t b) { return (b + 255) / 256 * 256; }
  hipError_t commit(void **arena, size_t *total) {
    *total = 0;
    for (const Item &it : items) *total += aligned(it.bytes);
    *arena = nullptr;
    if (*total == 0) return hipSuccess;
    hipError_t e = dev_alloc(arena, *total);
    if (e != hipSuccess) return e;
    size_t off = 0;
    for (const Item &it : items) {
      char *p = static_cast<char *>(*arena) + off;
      it.set(p);
      if (it.src) {
        e = hipMemcpyAsync(p, it.src, it.bytes, hipMemcpyHostToDevice, lib_stream());
        if (e != hipSuccess) return e;
      }
      off += aligned(it.bytes);
    }
    return hipStreamSynchronize(lib_stream());
  }
};

static void free_device(sbm_ctx *c) {
  if (c->d_arena) dev_free(c->d_arena);
  c->d_arena = nullptr;
  c->d_runs = c->d_nbr = c->d_face_cell = c->d_face_code = nullptr;
  c->d_face_xi = nullptr;
  c->d_brick_cell_off = c->d_brick_runs = c->d_face_runs = c->d_brick_cell_loc = nullptr;
  c->d_brick_face_off = c->d_brick_face_loc = c->d_row_base = c->d_row_hbase = c->d_halo_dof = nullptr;
  c->d_row_gmask = c->d_row_bmask = nullptr;
  c->d_halo_mask = nullptr;
  c->d_halo = c->d_fbuf = nullptr;
}

// CG bricks: group the active cells into blocks of BX x BY x BZ background cells (one
// workgroup each), list each brick's cells and surrogate faces, and describe every
// lattice row of the brick box by (id of its first DoF, mask of points that are DoFs,
// mask of points touched by the brick's own cells).  id: global lattice -> DoF id or -1.
namespace sbm {
int64_t order_bricks(const std::vector<int32_t> &count, const std::vector<int32_t> &fcount,
                     std::vector<int64_t> &key_of, std::vector<int32_t> &bid) {
  std::vector<int64_t> with_f, without_f;
  for (size_t k = 0; k < count.size(); ++k)
    if (count[k] > 0) (fcount[k] > 0 ? with_f : without_f).push_back((int64_t)k);
  const int64_t nbt = (int64_t)(with_f.size() + without_f.size());
  const int64_t nwf = (int64_t)with_f.size();
  bid.assign(count.size(), -1);
  key_of.clear();
  key_of.reserve(nbt);
  const int64_t per = nbt / 8, rem = nbt % 8;
  int64_t fi = 0, gi = 0;
  for (int x = 0; x < 8; ++x) {
    const int64_t size = per + (x < rem ? 1 : 0);
    const int64_t fend = std::min<int64_t>(nwf * (x + 1) / 8, fi + size);
    int64_t k = 0;
    for (; fi < fend; ++fi, ++k) key_of.push_back(with_f[fi]);
    for (; k < size && gi < (int64_t)without_f.size(); ++gi, ++k) key_of.push_back(without_f[gi]);
    for (; k < size; ++fi, ++k) key_of.push_back(with_f[fi]);  // only if the others ran out
  }
  for (size_t b = 0; b < key_of.size(); ++b) bid[key_of[b]] = (int32_t)b;
  return nwf;
}
}  // namespace sbm

static void build_bricks(sbm_ctx *c, const std::vector<int32_t> &id, int64_t lx, int64_t ly, int64_t lz) {
  const int d = c->dim, p = c->p;
  int BX, BY, BZ;
  brick_dims(d, p, &BX, &BY, &BZ);
  if (d == 2) BZ = 1;
  c->brick[0] = BX;
  c->brick[1] = BY;
  c->brick[2] = BZ;
  const int LX = BX * p + 1, LY = BY * p + 1, LZ = (d == 3) ? BZ * p + 1 : 1;
  const int nrows = LY * LZ;
  const int64_t nbx = (c->n[0] + BX - 1) / BX, nby = (c->n[1] + BY - 1) / BY;
  const int64_t nbz = (d == 3) ? (c->n[2] + BZ - 1) / BZ : 1;
  const int64_t nc = c->n_cells;
  std::vector<int64_t> bkey(nc);
  std::vector<int32_t> count(nbx * nby * nbz, 0);
  for (int64_t r = 0; r < nc; ++r) {
    const int32_t *cc = &c->cells[r * d];
    const int64_t bz = (d == 3) ? cc[2] / BZ : 0;
    bkey[r] = (bz * nby + cc[1] / BY) * nbx + cc[0] / BX;
    ++count[bkey[r]];
  }
  // Brick numbering.  The kernel gives each of the 8 XCDs one contiguous range of bricks (see
  // xcd_block); the face-carrying bricks (partial, cell by cell, plus their faces) are the
  // slow ones.  So every XCD range gets an equal share of the face-carrying bricks, numbered
  // first within the range (the dispatcher starts workgroups in order: the slow ones start
  // early), then its share of the others; each share is a contiguous run of the lexicographic
  // order (neighbouring bricks share an L2).
  std::vector<int32_t> fcount(count.size(), 0);
  for (int64_t f = 0; f < c->n_sbm; ++f) ++fcount[bkey[c->faces[3 * f]]];
  std::vector<int32_t> bid;
  std::vector<int64_t> key_of;
  c->n_bricks_faces = order_bricks(count, fcount, key_of, bid);
  const int32_t nb = (int32_t)key_of.size();
  c->n_bricks = nb;
  auto cell_loc = [&](int64_t r, int64_t key) {
    const int32_t *cc = &c->cells[r * d];
    const int64_t bx = key % nbx, by = (key / nbx) % nby, bz = key / (nbx * nby);
    const int64_t ox = cc[0] - bx * BX, oy = cc[1] - by * BY, oz = (d == 3) ? cc[2] - bz * BZ : 0;
    return (int32_t)(ox * p + oy * p * LX + oz * p * LX * LY);
  };
  c->brick_cell_off.assign(nb + 1, 0);
  for (int64_t r = 0; r < nc; ++r) ++c->brick_cell_off[bid[bkey[r]] + 1];
  for (int32_t b = 0; b < nb; ++b) c->brick_cell_off[b + 1] += c->brick_cell_off[b];
  c->brick_cells.assign(nc, 0);
  c->brick_cell_loc.assign(nc, 0);
  {
    std::vector<int32_t> fill(c->brick_cell_off.begin(), c->brick_cell_off.end() - 1);
    for (int64_t r = 0; r < nc; ++r) {
      const int32_t b = bid[bkey[r]];
      c->brick_cells[fill[b]] = (int32_t)r;
      c->brick_cell_loc[fill[b]] = cell_loc(r, bkey[r]);
      ++fill[b];
    }
  }
  // run bases of the cells in brick order (the kernel reads them without the cell rank)
  const int npr = (d == 3) ? (p + 1) * (p + 1) : (p + 1);
  c->brick_runs.resize((size_t)nc * npr);
  for (int64_t i = 0; i < nc; ++i)
    std::copy(c->runs.begin() + (size_t)c->brick_cells[i] * npr, c->runs.begin() + (size_t)(c->brick_cells[i] + 1) * npr,
              c->brick_runs.begin() + (size_t)i * npr);
  const int64_t nf = c->n_sbm;
  c->brick_face_off.assign(nb + 1, 0);
  for (int64_t f = 0; f < nf; ++f) ++c->brick_face_off[bid[bkey[c->faces[3 * f]]] + 1];
  for (int32_t b = 0; b < nb; ++b) c->brick_face_off[b + 1] += c->brick_face_off[b];
  c->brick_faces.assign(nf, 0);
  c->brick_face_loc.assign(nf, 0);
  {
    std::vector<int32_t> fill(c->brick_face_off.begin(), c->brick_face_off.end() - 1);
    for (int64_t f = 0; f < nf; ++f) {
      const int64_t r = c->faces[3 * f];
      const int32_t b = bid[bkey[r]];
      c->brick_faces[fill[b]] = (int32_t)f;
      c->brick_face_loc[fill[b]] = cell_loc(r, bkey[r]);
      ++fill[b];
    }
  }
  // run bases of each surrogate face's cell, faces in brick order (the device copies of the
  // face arrays of a CG operator are stored in brick order, see the upload)
  c->face_runs.resize((size_t)nf * npr);
  for (int64_t i = 0; i < nf; ++i) {
    const int64_t r = c->faces[3 * (int64_t)c->brick_faces[i]];
    std::copy(c->runs.begin() + (size_t)r * npr, c->runs.begin() + (size_t)(r + 1) * npr,
              c->face_runs.begin() + (size_t)i * npr);
  }
  c->row_base.assign((size_t)nb * nrows, 0);
  c->row_gmask.assign((size_t)nb * nrows, 0u);
  c->row_bmask.assign((size_t)nb * nrows, 0u);
  std::vector<unsigned char> touched(LX * LY * LZ);
  const int n1 = p + 1;
  for (int32_t b = 0; b < nb; ++b) {
    const int64_t key = key_of[b];
    const int64_t bx = key % nbx, by = (key / nbx) % nby, bz = key / (nbx * nby);
    std::fill(touched.begin(), touched.end(), 0);
    for (int32_t i = c->brick_cell_off[b]; i < c->brick_cell_off[b + 1]; ++i) {
      const int32_t loc = c->brick_cell_loc[i];
      for (int k = 0; k < ((d == 3) ? n1 : 1); ++k)
        for (int j = 0; j < n1; ++j)
          for (int ii = 0; ii < n1; ++ii) touched[loc + ii + j * LX + k * LX * LY] = 1;
    }
    for (int z = 0; z < LZ; ++z)
      for (int y = 0; y < LY; ++y) {
        const int row = y + LY * z;
        const int64_t X0 = bx * BX * p, Y = by * BY * p + y, Z = (d == 3) ? bz * BZ * p + z : 0;
        uint32_t gm = 0, bm = 0;
        int32_t base = 0;
        bool first = true;
        if (Y < ly && Z < lz) {
          for (int x = 0; x < LX; ++x) {
            const int64_t X = X0 + x;
            if (X >= lx) break;
            const int32_t g = id[(Z * ly + Y) * lx + X];
            if (g < 0) continue;
            gm |= 1u << x;
            if (first) {
              base = g;
              first = false;
            }
            if (touched[x + LX * (y + LY * z)]) bm |= 1u << x;
          }
        }
        c->row_base[(size_t)b * nrows + row] = base;
        c->row_gmask[(size_t)b * nrows + row] = gm;
        c->row_bmask[(size_t)b * nrows + row] = bm;
      }
  }
  // Halo: the DoFs on brick-box boundaries (bricks are aligned, so such a point lies on the
  // boundary of every brick that contains it).  They are numbered in DoF order (halo index);
  // along a brick row the boundary DoFs have consecutive halo indices.  A brick writes its
  // value for such a point into plane k = [x == 0] + 2 [y == 0] + 4 [z == 0] (its brick-
  // lattice coordinates: the side of the point the brick lies on), at the point's halo index;
  // bricks sharing a point have distinct k.  The reduction sums, per halo DoF, the planes
  // present in its mask in increasing k (a fixed order).  row_hbase: halo index of the row's
  // first boundary DoF.
  const uint32_t edge = 1u | (1u << (LX - 1));
  auto boundary_mask = [&](int y, int z, uint32_t gm) {
    const bool brow = (y == 0 || y == LY - 1 || (d == 3 && (z == 0 || z == LZ - 1)));
    return brow ? gm : (gm & edge);
  };
  std::vector<int32_t> hidx(c->n_dofs, -1);
  for (int32_t b = 0; b < nb; ++b)
    for (int z = 0; z < LZ; ++z)
      for (int y = 0; y < LY; ++y) {
        const size_t ri = (size_t)b * nrows + y + LY * z;
        const uint32_t hm = boundary_mask(y, z, c->row_bmask[ri]);
        for (int x = 0; x < LX; ++x)
          if ((hm >> x) & 1u)
            hidx[c->row_base[ri] + __builtin_popcount(c->row_gmask[ri] & ((1u << x) - 1u))] = 0;
      }
  c->halo_dof.clear();
  for (int64_t g = 0; g < c->n_dofs; ++g)
    if (hidx[g] == 0) {
      hidx[g] = (int32_t)c->halo_dof.size();
      c->halo_dof.push_back((int32_t)g);
    }
  c->n_halo_dofs = (int64_t)c->halo_dof.size();
  c->halo_mask.assign(c->n_halo_dofs, 0);
  c->row_hbase.assign((size_t)nb * nrows, 0);
  int64_t slots = 0;
  c->halo_ok = true;
  for (int32_t b = 0; b < nb; ++b)
    for (int z = 0; z < LZ; ++z)
      for (int y = 0; y < LY; ++y) {
        const size_t ri = (size_t)b * nrows + y + LY * z;
        const uint32_t gm = c->row_gmask[ri];
        const uint32_t hgm = boundary_mask(y, z, gm), hm = boundary_mask(y, z, c->row_bmask[ri]);
        if (hgm) {
          const int x0 = __builtin_ctz(hgm);
          c->row_hbase[ri] = hidx[c->row_base[ri] + __builtin_popcount(gm & ((1u << x0) - 1u))];
        }
        for (int x = 0; x < LX; ++x) {
          if (!((hgm >> x) & 1u)) continue;
          const int32_t h = hidx[c->row_base[ri] + __builtin_popcount(gm & ((1u << x) - 1u))];
          // every boundary DoF of the row is a halo DoF, numbered consecutively along the row
          if (h < 0 || h != c->row_hbase[ri] + __builtin_popcount(hgm & ((1u << x) - 1u))) c->halo_ok = false;
          if ((hm >> x) & 1u) {
            const int k = (x == 0 ? 1 : 0) | (y == 0 ? 2 : 0) | ((d == 3 && z == 0) ? 4 : 0);
            if (h >= 0) c->halo_mask[h] |= (uint8_t)(1u << k);
            ++slots;
          }
        }
      }
  c->n_halo_slots = slots;
}

namespace sbm {
void free_workspace(sbm_ctx *c);  // solver.hip
}

// Host part of the setup; separate so that tests can exercise it without a device.
// Validation and the per-operator parameters (mesh, penalties, level set, 1D rules).
static sbm_status prepare(sbm_ctx *c, const sbm_mesh *mesh, const sbm_levelset *ls, int p, int disc,
                          const sbm_options *opts) {
  if (!mesh || !ls) {
    set_error("sbm_setup: NULL mesh or level set");
    return SBM_EINVAL;
  }
  const int d = mesh->dim;
  if (d != 2 && d != 3) {
    set_error("sbm_setup: dim must be 2 or 3");
    return SBM_EUNSUPPORTED;
  }
  if (p < 1 || p > kMaxP) {
    set_error("sbm_setup: p must be in 1..8");
    return SBM_EUNSUPPORTED;
  }
  if (disc != SBM_CG && disc != SBM_DG) {
    set_error("sbm_setup: disc must be SBM_CG or SBM_DG");
    return SBM_EINVAL;
  }
  for (int k = 0; k < d; ++k) {
    if (mesh->n[k] < 1 || !(mesh->hi[k] > mesh->lo[k])) {
      set_error("sbm_setup: mesh needs n >= 1 and hi > lo in every direction");
      return SBM_EINVAL;
    }
  }
  c->dim = d;
  c->p = p;
  c->n1 = p + 1;
  c->disc = disc;
  for (int k = 0; k < 3; ++k) {
    c->n[k] = k < d ? mesh->n[k] : 1;
    c->lo[k] = k < d ? mesh->lo[k] : 0.0;
    c->hi[k] = k < d ? mesh->hi[k] : 1.0;
  }
  c->h = (c->hi[0] - c->lo[0]) / c->n[0];
  for (int k = 1; k < d; ++k) {
    const double hk = (c->hi[k] - c->lo[k]) / c->n[k];
    if (std::fabs(hk - c->h) > 1e-12 * c->h) {
      set_error("sbm_setup: cells must be isotropic (equal h in every direction)");
      return SBM_EUNSUPPORTED;
    }
  }
  c->gamma = (opts && opts->penalty_gamma > 0) ? opts->penalty_gamma : 10.0;
  c->gamma_dg = (opts && opts->dg_penalty_gamma > 0) ? opts->dg_penalty_gamma : 10.0;
  c->shift_scale = opts ? opts->shift_scale : 1.0;
  c->solver_graphs = !(opts && (opts->flags & SBM_SETUP_NO_GRAPHS));
  c->sigma_gamma = c->gamma * p * p / c->h;
  c->sigma_f = c->gamma_dg * p * p / c->h;

  // level set
  LevelSet &L = c->ls;
  L.kind = ls->kind;
  L.dim = d;
  for (int k = 0; k < 3; ++k) {
    L.centre[k] = ls->centre[k];
    L.semi[k] = ls->semi_axes[k];
    L.normal[k] = ls->normal[k];
  }
  L.radius = ls->radius;
  L.R = ls->R;
  L.r = ls->r;
  L.offset = ls->offset;
  switch (ls->kind) {
    case SBM_LS_SPHERE:
      if (!(ls->radius > 0)) {
        set_error("sbm_setup: sphere radius must be > 0");
        return SBM_EINVAL;
      }
      break;
    case SBM_LS_ELLIPSOID:
      for (int k = 0; k < d; ++k)
        if (!(ls->semi_axes[k] > 0)) {
          set_error("sbm_setup: ellipsoid semi-axes must be > 0");
          return SBM_EINVAL;
        }
      break;
    case SBM_LS_TORUS:
      if (d != 3 || !(ls->r > 0) || !(ls->R > ls->r)) {
        set_error("sbm_setup: torus needs dim 3 and R > r > 0");
        return SBM_EINVAL;
      }
      break;
    case SBM_LS_HALFSPACE: {
      const double nn = norm_d(ls->normal, d);
      if (!(std::fabs(nn - 1.0) < 1e-12)) {
        set_error("sbm_setup: half-space normal must have unit length");
        return SBM_EINVAL;
      }
      break;
    }
    case SBM_LS_SPHERE_UNION:
      if (ls->n_spheres < 1 || !ls->centres || !ls->radii) {
        set_error("sbm_setup: sphere union needs n_spheres >= 1 and centre/radius arrays");
        return SBM_EINVAL;
      }
      L.cs.assign(3 * ls->n_spheres, 0.0);
      L.rs.assign(ls->n_spheres, 0.0);
      for (int i = 0; i < ls->n_spheres; ++i) {
        for (int k = 0; k < d; ++k) L.cs[3 * i + k] = ls->centres[3 * i + k];
        L.rs[i] = ls->radii[i];
        if (!(L.rs[i] > 0)) {
          set_error("sbm_setup: sphere radii must be > 0");
          return SBM_EINVAL;
        }
      }
      break;
    case SBM_LS_CALLBACK:
      if (!ls->phi || !ls->grad) {
        set_error("sbm_setup: callback level set needs phi and grad");
        return SBM_EINVAL;
      }
      L.cb_phi = ls->phi;
      L.cb_grad = ls->grad;
      L.cb_user = ls->user;
      break;
    default:
      set_error("sbm_setup: unknown level-set kind");
      return SBM_EINVAL;
  }
  c->rules = make_rules(p);
  const int n1 = p + 1;
  c->nb = (d == 3) ? n1 * n1 * n1 : n1 * n1;
  c->nq_face = (d == 3) ? n1 * n1 : n1;
  return SBM_OK;
}

// Geometry and numbering on the host: active cells, faces, closest points, DoF numbering and
// (CG) the brick layout.  Used for user level sets (SBM_LS_CALLBACK), for host-only handles and
// when SBM_SETUP_HOST_BUILD asks for it; the analytic kinds are built on the device otherwise
// (setup_gpu.hip), with identical results.
static sbm_status host_geometry(sbm_ctx *c) {
  const int d = c->dim, p = c->p, disc = c->disc;
  const LevelSet &L = c->ls;
  const Rules1D &R = c->rules;
  const int n1 = p + 1;
  const int np = c->nq_face;  // runs per cell = face points

  // ---- vertex values and active cells (phi < 0 at all 2^d vertices) ----
  const int64_t nx = c->n[0], ny = c->n[1], nz = (d == 3) ? c->n[2] : 1;
  const int64_t vx = nx + 1, vy = ny + 1, vz = (d == 3) ? nz + 1 : 1;
  std::vector<unsigned char> vin(vx * vy * vz);
  for (int64_t k = 0; k < vz; ++k)
    for (int64_t j = 0; j < vy; ++j)
      for (int64_t i = 0; i < vx; ++i) {
        double x[3] = {c->lo[0] + c->h * i, c->lo[1] + c->h * j, d == 3 ? c->lo[2] + c->h * k : 0.0};
        vin[(k * vy + j) * vx + i] = L.phi(x) < 0.0;
      }
  std::vector<int32_t> rank(nx * ny * nz, -1);
  c->cells.clear();
  int64_t nc = 0;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        bool in = true;
        for (int o = 0; o < (1 << d) && in; ++o) {
          const int64_t ii = i + (o & 1), jj = j + ((o >> 1) & 1), kk = k + ((o >> 2) & 1);
          in = vin[(kk * vy + jj) * vx + ii];
        }
        if (in) {
          rank[(k * ny + j) * nx + i] = (int32_t)nc++;
          c->cells.push_back((int32_t)i);
          c->cells.push_back((int32_t)j);
          if (d == 3) c->cells.push_back((int32_t)k);
        }
      }
  c->n_cells = nc;

  // ---- faces: neighbours, surrogate faces, interior-face count ----
  c->nbr.assign(nc * 2 * d, -1);
  c->faces.clear();
  int64_t n_int = 0;
  for (int64_t r = 0; r < nc; ++r) {
    const int32_t *cc = &c->cells[r * d];
    for (int a = 0; a < d; ++a)
      for (int s = 0; s < 2; ++s) {
        int64_t nbv[3] = {cc[0], cc[1], d == 3 ? cc[2] : 0};
        nbv[a] += s ? 1 : -1;
        int32_t nr = -1;
        if (nbv[a] >= 0 && nbv[a] < c->n[a]) nr = rank[(nbv[2] * ny + nbv[1]) * nx + nbv[0]];
        // a missing neighbour is a surrogate face f, stored as -2 - f (every reader tests < 0)
        c->nbr[r * 2 * d + 2 * a + s] = nr >= 0 ? nr : (int32_t)(-2 - (int64_t)c->faces.size() / 3);
        if (nr < 0) {
          c->faces.push_back((int32_t)r);
          c->faces.push_back(a);
          c->faces.push_back(s);
        } else if (s == 1) {
          ++n_int;
        }
      }
  }
  c->n_sbm = (int64_t)c->faces.size() / 3;
  c->n_int = n_int;

  // ---- face points: xi~ (face Gauss points), closest points, shifted xi ----
  // (the projections are independent per face: faces are split over host threads, every
  // face's results go to its own slots, so the outcome does not depend on the split)
  const int64_t nf = c->n_sbm;
  c->face_xi.assign(nf * np * d, 0.0);
  c->face_xtrue.assign(nf * np * d, 0.0);
  auto project = [&](int64_t f0, int64_t f1) -> bool {
    bool ok = true;
    for (int64_t f = f0; f < f1; ++f) {
      const int32_t r = c->faces[3 * f], a = c->faces[3 * f + 1], s = c->faces[3 * f + 2];
      const int32_t *cc = &c->cells[(int64_t)r * d];
      for (int q = 0; q < np; ++q) {
        double xt[3], xs[3], xx[3], cp[3];
        int qq = q;
        for (int k = 0; k < d; ++k) {
          if (k == a) {
            xt[k] = (double)s;
          } else {
            xt[k] = R.g[qq % n1];
            qq /= n1;
          }
          xx[k] = c->lo[k] + c->h * ((double)cc[k] + xt[k]);
        }
        L.closest(xx, cp);
        for (int k = 0; k < d; ++k) {
          xs[k] = xt[k] + c->shift_scale * (cp[k] - xx[k]) / c->h;
          c->face_xi[(f * np + q) * d + k] = xs[k];
          c->face_xtrue[(f * np + q) * d + k] = cp[k];
          ok = ok && std::isfinite(xs[k]);
        }
      }
    }
    return ok;
  };
  // user callbacks are called from this thread only
  const int64_t nthr = L.kind == SBM_LS_CALLBACK ? 1 : std::max<int64_t>(
      1, std::min<int64_t>({(int64_t)std::thread::hardware_concurrency(), 16, (nf * np) / 4096}));
  bool proj_ok = true;
  if (nthr <= 1) {
    proj_ok = project(0, nf);
  } else {
    std::vector<std::thread> pool;
    std::vector<char> oks((size_t)nthr, 1);
    for (int64_t t = 0; t < nthr; ++t)
      pool.emplace_back([&, t] { oks[t] = project(nf * t / nthr, nf * (t + 1) / nthr) ? 1 : 0; });
    for (auto &th : pool) th.join();
    for (char o : oks) proj_ok = proj_ok && o;
  }
  if (!proj_ok) {
    set_error("sbm_setup: closest-point projection failed (degenerate level set?)");
    return SBM_EINVAL;
  }

  // ---- DoF numbering ----
  if (disc == SBM_CG) {
    const int64_t lx = p * nx + 1, ly = p * ny + 1, lz = (d == 3) ? p * nz + 1 : 1;
    std::vector<int32_t> id(lx * ly * lz, 0);
    for (int64_t r = 0; r < nc; ++r) {
      const int32_t *cc = &c->cells[r * d];
      const int kz = (d == 3) ? n1 : 1;
      for (int k = 0; k < kz; ++k)
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i) {
            const int64_t m0 = (int64_t)p * cc[0] + i, m1 = (int64_t)p * cc[1] + j;
            const int64_t m2 = (d == 3) ? (int64_t)p * cc[2] + k : 0;
            id[(m2 * ly + m1) * lx + m0] = 1;
          }
    }
    int64_t cnt = 0;
    for (size_t m = 0; m < id.size(); ++m) {
      if (id[m]) {
        if (cnt >= (int64_t)std::numeric_limits<int32_t>::max()) {
          set_error("sbm_setup: more than 2^31-1 DoFs");
          return SBM_EUNSUPPORTED;
        }
        id[m] = (int32_t)cnt++;
      } else {
        id[m] = -1;
      }
    }
    c->n_dofs = cnt;
    c->runs.assign(nc * np, 0);
    for (int64_t r = 0; r < nc; ++r) {
      const int32_t *cc = &c->cells[r * d];
      for (int t = 0; t < np; ++t) {
        const int j = t % n1, k = (d == 3) ? t / n1 : 0;
        const int64_t m0 = (int64_t)p * cc[0], m1 = (int64_t)p * cc[1] + j;
        const int64_t m2 = (d == 3) ? (int64_t)p * cc[2] + k : 0;
        c->runs[r * np + t] = id[(m2 * ly + m1) * lx + m0];
      }
    }
    build_bricks(c, id, lx, ly, lz);
  } else {
    if (nc * (int64_t)c->nb >= (int64_t)std::numeric_limits<int32_t>::max()) {
      set_error("sbm_setup: more than 2^31-1 DoFs");
      return SBM_EUNSUPPORTED;
    }
    c->n_dofs = nc * c->nb;
    c->runs.clear();
  }
  return SBM_OK;
}

extern "C" {

const char *sbm_last_error(void) { return g_last_error.c_str(); }

sbm_status sbm_setup(const sbm_mesh *mesh, const sbm_levelset *ls, int p, int disc,
                     const sbm_options *opts, sbm_handle *out) {
  if (!out) {
    set_error("sbm_setup: NULL output handle");
    return SBM_EINVAL;
  }
  *out = nullptr;
  sbm_ctx *c = new (std::nothrow) sbm_ctx();
  if (!c) {
    set_error("sbm_setup: out of host memory");
    return SBM_ENOMEM;
  }
  sbm_status st;
  const int flags = opts ? opts->flags : 0;
  const bool on_device = !(flags & (SBM_SETUP_HOST_ONLY | SBM_SETUP_HOST_BUILD)) && ls &&
                         ls->kind != SBM_LS_CALLBACK;
  try {
    st = prepare(c, mesh, ls, p, disc, opts);
    if (st == SBM_OK && on_device) {
      st = sbm::device_setup(c);
      if (st == SBM_OK) {
        *out = c;
        return SBM_OK;
      }
      free_device(c);
      delete c;
      return st;
    }
    if (st == SBM_OK) st = host_geometry(c);
  } catch (const std::bad_alloc &) {
    set_error("sbm_setup: out of host memory");
    st = SBM_ENOMEM;
  }
  if (st == SBM_OK && !c->halo_ok) {
    set_error("sbm_setup: internal error: brick-boundary DoFs are not numbered consecutively along a row");
    st = SBM_EUNSUPPORTED;
  }
  if (st != SBM_OK) {
    delete c;
    return st;
  }
  if (flags & SBM_SETUP_HOST_ONLY) {
    c->host_only = true;
    *out = c;
    return SBM_OK;
  }
  // ---- upload ----
  // Device face arrays: CG in brick order (face i of the device arrays is host face
  // brick_faces[i], so a brick's faces are contiguous), DG in host order.  Host arrays and
  // the exports keep the host order.
  const bool cg = c->disc == SBM_CG;
  std::vector<int32_t> fcell(c->n_sbm), fcode(c->n_sbm);
  std::vector<double> fxi(c->face_xi.size());
  const size_t xq = (size_t)c->nq_face * c->dim;
  for (int64_t i = 0; i < c->n_sbm; ++i) {
    const int64_t f = cg ? c->brick_faces[i] : i;
    fcell[i] = c->faces[3 * f];
    fcode[i] = 2 * c->faces[3 * f + 1] + c->faces[3 * f + 2];
    std::copy(c->face_xi.begin() + f * xq, c->face_xi.begin() + (f + 1) * xq, fxi.begin() + i * xq);
  }
  ArenaPlan plan;
  if (c->disc == SBM_CG) {
    plan.add(c->d_runs, c->runs);
    plan.add(c->d_brick_cell_off, c->brick_cell_off);
    plan.add(c->d_brick_runs, c->brick_runs);
    plan.add(c->d_face_runs, c->face_runs);
    plan.add(c->d_brick_cell_loc, c->brick_cell_loc);
    plan.add(c->d_brick_face_off, c->brick_face_off);
    plan.add(c->d_brick_face_loc, c->brick_face_loc);
    plan.add(c->d_row_base, c->row_base);
    plan.add(c->d_row_gmask, c->row_gmask);
    plan.add(c->d_row_bmask, c->row_bmask);
    plan.add(c->d_row_hbase, c->row_hbase);
    plan.add(c->d_halo_dof, c->halo_dof);
    plan.add(c->d_halo_mask, c->halo_mask);
    plan.scratch(c->d_halo, ((size_t)1 << c->dim) * (size_t)c->n_halo_dofs * sizeof(double));
    plan.scratch(c->d_fbuf, (size_t)c->n_sbm * 2 * c->nq_face * sizeof(double));
  } else {
    plan.add(c->d_nbr, c->nbr);
    plan.scratch(c->d_fbuf, (size_t)c->n_sbm * 2 * c->nq_face * sizeof(double));
  }
  plan.add(c->d_face_cell, fcell);
  plan.add(c->d_face_code, fcode);
  plan.add(c->d_face_xi, fxi);
  size_t bytes = 0;
  const hipError_t e = plan.commit(&c->d_arena, &bytes);
  if (e != hipSuccess) {
    set_error(std::string("sbm_setup: device upload failed: ") + hipGetErrorString(e));
    free_device(c);
    delete c;
    return e == hipErrorOutOfMemory ? SBM_ENOMEM : SBM_EHIP;
  }
  c->device_bytes = bytes;
  *out = c;
  return SBM_OK;
}

sbm_status sbm_info(sbm_handle h, int64_t *n_dofs, int64_t *n_cells, int64_t *n_sbm_faces,
                    int64_t *n_interior_faces, size_t *device_bytes) {
  if (!h) {
    set_error("sbm_info: NULL handle");
    return SBM_EINVAL;
  }
  if (n_dofs) *n_dofs = h->n_dofs;
  if (n_cells) *n_cells = h->n_cells;
  if (n_sbm_faces) *n_sbm_faces = h->n_sbm;
  if (n_interior_faces) *n_interior_faces = h->n_int;
  if (device_bytes) *device_bytes = h->device_bytes + sbm::workspace_bytes(h);
  return SBM_OK;
}

void sbm_destroy(sbm_handle h) {
  if (!h) return;
  // wait for the handle's last asynchronous work only (its memory returns to the pool
  // stream-ordered; nothing else on the device is waited for)
  if (h->last_work) {
    (void)hipEventSynchronize(h->last_work);
    (void)hipEventDestroy(h->last_work);
    h->last_work = nullptr;
  }
  sbm::wait_batches();  // batches that include h record their completion, not h's
  sbm::free_workspace(h);
  free_device(h);
  delete h;
}

sbm_status sbm_apply(sbm_handle h, const void *u, void *v, int prec, void *stream) {
  if (!h) {
    set_error("sbm_apply: NULL handle");
    return SBM_EINVAL;
  }
  if (h->n_dofs == 0 && !h->host_only && (prec == SBM_F64 || prec == SBM_F32)) return SBM_OK;
  if (!u || !v) {
    set_error("sbm_apply: NULL vector");
    return SBM_EINVAL;
  }
  if (h->host_only) {
    set_error("sbm_apply: handle was set up with SBM_SETUP_HOST_ONLY");
    return SBM_EINVAL;
  }
  if (u == v) {
    set_error("sbm_apply: u and v must not alias");
    return SBM_EINVAL;
  }
  if (prec != SBM_F64 && prec != SBM_F32) {
    set_error("sbm_apply: prec must be SBM_F64 or SBM_F32");
    return SBM_EINVAL;
  }
  SBM_HIP_CHECK(launch_operator(h, u, v, prec, SBM_PART_ALL, (hipStream_t)stream));
  note_work(h, (hipStream_t)stream);
  return SBM_OK;
}

sbm_status sbm_apply_parts(sbm_handle h, const void *u, void *v, int prec, int parts, void *stream) {
  if (!h || h->host_only || (h->n_dofs > 0 && (!u || !v)) || (u == v && h->n_dofs > 0) ||
      (prec != SBM_F64 && prec != SBM_F32) ||
      (parts & ~(SBM_PART_ALL | SBM_PART_NO_ASSEMBLY | SBM_PART_REUSE_FACES))) {
    set_error("sbm_apply_parts: invalid argument");
    return SBM_EINVAL;
  }
  if (h->taylor_m >= 0) {
    set_error("sbm_apply_parts: the diagnostic split is for the full extension only");
    return SBM_EUNSUPPORTED;
  }
  if (h->n_dofs == 0) return SBM_OK;
  SBM_HIP_CHECK(launch_apply(h, u, v, prec, parts, (hipStream_t)stream));
  note_work(h, (hipStream_t)stream);
  return SBM_OK;
}

sbm_status sbm_set_extension_order(sbm_handle h, int m) {
  if (!h) {
    set_error("sbm_set_extension_order: NULL handle");
    return SBM_EINVAL;
  }
  h->taylor_m = m < 0 ? -1 : m;
  return SBM_OK;
}

sbm_status sbm_layout_stats(sbm_handle h, int64_t *n_bricks, int64_t *n_boundary_dofs,
                            int64_t *n_boundary_slots) {
  if (!h) {
    set_error("sbm_layout_stats: NULL handle");
    return SBM_EINVAL;
  }
  if (n_bricks) *n_bricks = h->n_bricks;
  if (n_boundary_dofs) *n_boundary_dofs = h->n_halo_dofs;
  if (n_boundary_slots) *n_boundary_slots = h->n_halo_slots;
  return SBM_OK;
}

sbm_status sbm_dof_points(sbm_handle h, double *xyz) {
  if (!h || !xyz) {
    set_error("sbm_dof_points: NULL argument");
    return SBM_EINVAL;
  }
  const int d = h->dim, n1 = h->n1, np = h->nq_face;
  for (int64_t r = 0; r < h->n_cells; ++r) {
    const int32_t *cc = &h->cells[r * d];
    for (int t = 0; t < np; ++t) {
      const int j = t % n1, k = (d == 3) ? t / n1 : 0;
      for (int i = 0; i < n1; ++i) {
        const int64_t dof = (h->disc == SBM_CG) ? (int64_t)h->runs[r * np + t] + i
                                                : r * h->nb + (int64_t)n1 * t + i;
        const int loc[3] = {i, j, k};
        for (int m = 0; m < d; ++m) xyz[dof * d + m] = h->lo[m] + h->h * (cc[m] + h->rules.z[loc[m]]);
      }
    }
  }
  return SBM_OK;
}

sbm_status sbm_rhs_points(sbm_handle h, double *cell_qp, double *bdry_pts) {
  if (!h) {
    set_error("sbm_rhs_points: NULL handle");
    return SBM_EINVAL;
  }
  const int d = h->dim, n1 = h->n1;
  if (cell_qp) {
    const int nq = h->nb;
    auto fill = [&](int64_t r0, int64_t r1) {
      for (int64_t r = r0; r < r1; ++r) {
        const int32_t *cc = &h->cells[r * d];
        for (int q = 0; q < nq; ++q) {
          int qq = q;
          for (int m = 0; m < d; ++m) {
            cell_qp[(r * nq + q) * d + m] = h->lo[m] + h->h * (cc[m] + h->rules.g[qq % n1]);
            qq /= n1;
          }
        }
      }
    };
    // every point on its own (host threads over cell ranges for large meshes)
    const int64_t nt = std::max<int64_t>(
        1, std::min<int64_t>({(int64_t)std::thread::hardware_concurrency(), 16, h->n_cells / 2048}));
    if (nt <= 1) {
      fill(0, h->n_cells);
    } else {
      std::vector<std::thread> pool;
      for (int64_t t = 0; t < nt; ++t)
        pool.emplace_back([&, t] { fill(h->n_cells * t / nt, h->n_cells * (t + 1) / nt); });
      for (auto &th : pool) th.join();
    }
  }
  if (bdry_pts) std::memcpy(bdry_pts, h->face_xtrue.data(), h->face_xtrue.size() * sizeof(double));
  return SBM_OK;
}

sbm_status sbm_export_cells(sbm_handle h, int32_t *cells) {
  if (!h || !cells) {
    set_error("sbm_export_cells: NULL argument");
    return SBM_EINVAL;
  }
  std::memcpy(cells, h->cells.data(), h->cells.size() * sizeof(int32_t));
  return SBM_OK;
}

sbm_status sbm_export_sbm_faces(sbm_handle h, int32_t *faces) {
  if (!h || !faces) {
    set_error("sbm_export_sbm_faces: NULL argument");
    return SBM_EINVAL;
  }
  std::memcpy(faces, h->faces.data(), h->faces.size() * sizeof(int32_t));
  return SBM_OK;
}

sbm_status sbm_export_face_xi(sbm_handle h, double *xi) {
  if (!h || !xi) {
    set_error("sbm_export_face_xi: NULL argument");
    return SBM_EINVAL;
  }
  std::memcpy(xi, h->face_xi.data(), h->face_xi.size() * sizeof(double));
  return SBM_OK;
}

sbm_status sbm_export_cell_dofs(sbm_handle h, int64_t *dofs) {
  if (!h || !dofs) {
    set_error("sbm_export_cell_dofs: NULL argument");
    return SBM_EINVAL;
  }
  const int n1 = h->n1, np = h->nq_face, nb = h->nb;
  for (int64_t r = 0; r < h->n_cells; ++r)
    for (int t = 0; t < np; ++t)
      for (int i = 0; i < n1; ++i)
        dofs[r * nb + (int64_t)n1 * t + i] = (h->disc == SBM_CG) ? (int64_t)h->runs[r * np + t] + i
                                                                  : r * nb + (int64_t)n1 * t + i;
  return SBM_OK;
}

size_t sbm_footprint_estimate(const sbm_mesh *mesh, int p, int disc, int64_t n_cells_hint,
                              int64_t n_faces_hint) {
  // An upper bound of what sbm_setup allocates for at most n_cells_hint active cells and
  // n_faces_hint surrogate faces: every array of the handle's arena (one hipMalloc), sized by
  // bounds that hold for any geometry, each rounded up to 256 bytes as the arena does.
  if (!mesh || p < 1 || p > kMaxP || (mesh->dim != 2 && mesh->dim != 3) || n_cells_hint < 0 ||
      n_faces_hint < 0)
    return 0;
  const int d = mesh->dim;
  const int64_t n1 = p + 1;
  const int64_t nb = (d == 3) ? n1 * n1 * n1 : n1 * n1;
  const int64_t np = (d == 3) ? n1 * n1 : n1;
  const int64_t nc = n_cells_hint, nf = n_faces_hint;
  auto up = [](int64_t b) { return (size_t)((b + 255) / 256 * 256); };
  size_t b = 0;
  if (disc == SBM_CG) {
    const int64_t ndofs = nc * nb;  // every active cell touches (p+1)^d lattice points
    int bx = 1, by = 1, bz = 1;
    brick_dims(d, p, &bx, &by, &bz);
    const int64_t B[3] = {bx, by, d == 3 ? bz : 1};
    // brick-boundary points of one cell: on each axis it meets both brick planes if the brick
    // is one cell wide there, else at most one
    int64_t inner = 1;
    for (int k = 0; k < d; ++k) inner *= (n1 - (B[k] == 1 ? 2 : 1));
    const int64_t halo = std::min<int64_t>(ndofs, nc * (nb - inner));
    const int64_t rows = (B[1] * p + 1) * (d == 3 ? B[2] * p + 1 : 1);  // lattice rows per brick
    const int64_t nbricks = nc;                                        // every brick has a cell
    b += up(4 * nc * np) * 2;                                          // runs, brick_runs
    b += up(4 * (nbricks + 1)) * 2 + up(4 * nc) + up(4 * nf);          // offsets, cell/face locations
    b += up(4 * nf * np);                                              // face_runs
    b += 4 * up(4 * nbricks * rows);                                   // row descriptors
    b += up(4 * halo) + up(halo);                                      // halo DoF ids and masks
    b += up(((int64_t)1 << d) * 8 * halo);                             // halo planes (FP64)
  } else {
    b += up(4 * nc * 2 * d);  // neighbour table
  }
  b += up(8 * nf * 2 * np);                              // surrogate-face results (FP64)
  b += up(4 * nf) * 2 + up(8 * nf * np * d);             // face cell, code, shifted points
  return b;
}

}  // extern "C"
