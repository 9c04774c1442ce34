// Internal declarations of the SBM library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sbm.h"
#include "levelset.h"

namespace sbm {

constexpr int kMaxP = 8;
constexpr int kMaxN1 = kMaxP + 1;

// 1D reference data on [0,1] for one degree p (always computed in FP64 on the host).
struct Rules1D {
  int p = 0;
  std::vector<double> z;      // GLL nodes (p+1)
  std::vector<double> g, w;   // Gauss points and weights (p+1), weights sum to 1
  std::vector<double> cinv;   // 1 / prod_{m != j} (z_j - z_m)
  std::vector<double> M, K;   // 1D mass / stiffness on [0,1]: sum_q w_q l_i(g_q) l_j(g_q), ... l'_i l'_j
  std::vector<double> N;      // N[q*(p+1)+j] = l_j(g_q): GLL -> Gauss interpolation
  std::vector<double> D0, D1; // l'_j(0), l'_j(1)
};
Rules1D make_rules(int p);
double lagrange_value(const Rules1D &r, int j, double x);
double lagrange_derivative(const Rules1D &r, int j, double x);

// Level set held by a context (arrays copied from the caller).
struct LevelSet {
  int kind = 0;
  int dim = 3;
  double centre[3] = {0, 0, 0};
  double radius = 0, R = 0, r = 0, offset = 0;
  double semi[3] = {1, 1, 1};
  double normal[3] = {1, 0, 0};
  std::vector<double> cs;  // n x 3
  std::vector<double> rs;
  double (*cb_phi)(const double *, void *) = nullptr;  // SBM_LS_CALLBACK
  void (*cb_grad)(const double *, double *, void *) = nullptr;
  void *cb_user = nullptr;
  double phi(const double *x) const;
  void closest(const double *x, double *out) const;  // exact closest point on {phi = 0}
  LsParams params() const;                            // analytic kinds (host pointers)
};

// Kernel-side tables, passed by value (kernel arguments live in the constant kernarg
// segment; all table indices in the kernels are compile-time constants after unrolling).
template <typename T, int N1>
struct KTab {
  // M and K are centrosymmetric (symmetric node set), so y = A x splits into an even part
  // (E, on e_k = x_k + x_{p-k} and the middle value) and an odd part (O, on
  // o_k = x_k - x_{p-k}): y_i = ye_i + yo_i, y_{p-i} = ye_i - yo_i.
  static constexpr int HC = (N1 + 1) / 2, HF = N1 / 2;
  T EM[HC * HC], OM[HF * HF];
  T EK[HC * HC], OK[HF * HF];
  T M[N1 * N1];
  T K[N1 * N1];
  T N[N1 * N1];
  T D0[N1];
  T D1[N1];
  T w[N1];
  double z[N1];
  double cinv[N1];
};

// Per-operator scalars passed to the kernels.
struct KScal {
  double h;
  double sigma_gamma;
  double sigma_f;
};

struct Workspace;  // solver vectors (allocated on first solve)

}  // namespace sbm

struct sbm_ctx {
  int dim = 3, p = 1, n1 = 2, disc = SBM_CG;
  int n[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  double h = 1.0;
  double gamma = 10.0, gamma_dg = 10.0, shift_scale = 1.0;
  int taylor_m = -1;  // surrogate-face extension: < 0 full (point value at the shifted point), else E_m
  bool solver_graphs = true;  // the solver replays its Arnoldi steps from captured graphs
  double sigma_gamma = 0.0, sigma_f = 0.0;
  int64_t n_cells = 0, n_dofs = 0, n_sbm = 0, n_int = 0;
  int nq_face = 1;   // (p+1)^(d-1)
  int nb = 1;        // (p+1)^d
  sbm::Rules1D rules;
  sbm::LevelSet ls;
  // host copies (setup results)
  std::vector<int32_t> cells;      // n_cells x dim
  std::vector<int32_t> faces;      // n_sbm x 3 (cell rank, axis, side)
  std::vector<double> face_xi;     // n_sbm x nq x dim
  std::vector<double> face_xtrue;  // n_sbm x nq x dim
  std::vector<int32_t> runs;       // CG: n_cells x (p+1)^(d-1) first DoF of each x-run
  std::vector<int32_t> nbr;        // n_cells x 2d: neighbour rank, or -2 - f for surrogate face f
  // CG bricks: BX x BY x BZ blocks of background cells, one workgroup each
  int brick[3] = {1, 1, 1};
  int64_t n_bricks = 0;
  int64_t n_bricks_faces = 0;  // number of bricks that carry surrogate faces
  std::vector<int32_t> brick_cell_off, brick_cells, brick_cell_loc;
  std::vector<int32_t> brick_runs;  // run bases of the cells in brick order (n_cells x (p+1)^(d-1))
  std::vector<int32_t> face_runs;   // run bases of each surrogate face's cell, faces in brick order
  std::vector<int32_t> brick_face_off, brick_faces, brick_face_loc;
  std::vector<int32_t> row_base, row_hbase;
  std::vector<uint32_t> row_gmask, row_bmask;
  // halo assembly: a DoF on brick boundaries collects one value per touching brick, in plane
  // k (2^d planes of n_halo_dofs values) given by the brick's side of the point
  int64_t n_halo_slots = 0, n_halo_dofs = 0;
  std::vector<int32_t> halo_dof;   // halo index -> DoF
  std::vector<uint8_t> halo_mask;  // halo index -> planes written
  bool halo_ok = true;             // consistency of the halo numbering (checked at setup)
  int32_t *d_row_hbase = nullptr, *d_halo_dof = nullptr;
  uint8_t *d_halo_mask = nullptr;
  void *d_halo = nullptr;  // 2^d x n_halo_dofs doubles (also used as floats); per-handle scratch
  void *d_fbuf = nullptr;  // n_sbm x 2 x (p+1)^(d-1) doubles, surrogate-face results; per-handle scratch
  int32_t *d_brick_cell_off = nullptr, *d_brick_runs = nullptr, *d_brick_cell_loc = nullptr;
  int32_t *d_face_runs = nullptr;
  int32_t *d_brick_face_off = nullptr, *d_brick_face_loc = nullptr;
  int32_t *d_row_base = nullptr;
  uint32_t *d_row_gmask = nullptr, *d_row_bmask = nullptr;
  // device copies (all inside one allocation, d_arena)
  void *d_arena = nullptr;
  int32_t *d_runs = nullptr;       // CG
  int32_t *d_nbr = nullptr;        // DG
  int32_t *d_face_cell = nullptr;  // n_sbm
  int32_t *d_face_code = nullptr;  // n_sbm: 2*axis + side
  double *d_face_xi = nullptr;     // n_sbm x nq x dim
  size_t device_bytes = 0;
  bool host_only = false;
  sbm::Workspace *ws = nullptr;
  // completion of the handle's last stream-ordered work (recorded by the asynchronous entry
  // points); sbm_destroy waits for it instead of for the whole device
  hipEvent_t last_work = nullptr;
};

namespace sbm {
// Thread-local last error.
void set_error(const std::string &msg);
// Scratch of one apply: the CG halo planes and the surrogate-face results.  NULL members (or
// a NULL Scratch) select the handle's own buffers (d_halo, d_fbuf).
struct Scratch {
  void *halo = nullptr;
  void *fbuf = nullptr;
};
// Bytes of scratch one apply of c needs in precision prec (elements of the apply's type):
// halo planes and face results, each rounded up to 256 bytes.
size_t apply_scratch_bytes(const sbm_ctx *c, int prec);
// Launchers (kernels.hip).  All asynchronous on stream.
hipError_t launch_apply(const sbm_ctx *c, const void *u, void *v, int prec, int parts, hipStream_t s,
                        const Scratch *scr = nullptr);
hipError_t launch_diagonal(const sbm_ctx *c, void *diag, int prec, hipStream_t s);
// The operator of the handle's extension (kernels_taylor.hip): launch_apply / launch_diagonal
// when the extension is the full one, else the cell term by launch_apply plus the truncated
// surrogate-face term.  Every apply and diagonal of the library goes through these.
hipError_t launch_operator(const sbm_ctx *c, const void *u, void *v, int prec, int parts, hipStream_t s,
                           const Scratch *scr = nullptr);
hipError_t launch_operator_diagonal(const sbm_ctx *c, void *diag, int prec, hipStream_t s);
// Batched applies (kernels_apply.hip).  A group holds operators of one kernel instantiation
// (discretisation, dimension, degree; prec); its applies run as one launch per stage.  The
// group's device tables (per item: its arrays and vectors and its first workgroup in every
// stage; per stage: the item of every workgroup) are appended to image, the host copy of the
// plan's device memory, at 256-byte aligned offsets recorded in the group.  own_faces[i] = 0:
// item i's surrogate-face results are computed elsewhere (truncated extension) before the group.
struct BatchGroup {
  const sbm_ctx *first = nullptr;
  int prec = SBM_F64;
  int n_items = 0;
  int nblk[3] = {0, 0, 0};  // workgroups per stage: surrogate faces, cells or bricks, brick-boundary sums
  size_t off_items = 0, off_blk[3] = {0, 0, 0};
};
hipError_t batch_group_build(BatchGroup &g, const std::vector<const sbm_ctx *> &cs,
                             const std::vector<const void *> &u, const std::vector<void *> &v,
                             const std::vector<int> &own_faces, std::vector<unsigned char> &image);
// Launches a group's stages; base = device address of the plan's tables (the uploaded image).
hipError_t launch_batch_group(const BatchGroup &g, const void *base, hipStream_t s);
// The truncated extension's surrogate-face results (Rv, Rg per face node) of u into fbuf
// (kernels_taylor.hip); nothing to do for an operator without surrogate faces.
hipError_t launch_taylor_faces(const sbm_ctx *c, const void *u, void *fbuf, int prec, hipStream_t s);
// Brick shape (cells per direction) used by the CG kernel for (dim, p).
void brick_dims(int dim, int p, int *bx, int *by, int *bz);
// Brick numbering from the per-slot cell and face counts of the brick grid: key_of[b] is the
// grid slot of brick b, bid[slot] its brick number (-1 if empty).  Every one of the 8 XCD
// ranges gets an equal share of the face-carrying bricks, first, then of the others (see
// xcd_block).  Returns the number of face-carrying bricks.
int64_t order_bricks(const std::vector<int32_t> &count, const std::vector<int32_t> &fcount,
                     std::vector<int64_t> &key_of, std::vector<int32_t> &bid);
// Setup on the device (setup_gpu.hip) for the analytic level-set kinds: after prepare(), builds
// the geometry, the DoF numbering and the brick layout with kernels, fills the handle's arena
// and the host copies (cells, faces, shifted and true points, runs).
sbm_status device_setup(sbm_ctx *c);
// Device memory of handles and workspaces: a released block goes to a per-device cache
// (bounded, 16 GB) and is handed to the next allocation that fits, so releasing memory does not
// synchronise the device (hipFree does); only what exceeds the cache is freed.  The caller of
// dev_free must have finished all device work on the block.  lib_stream: a library stream of
// the current device (default priority) for the library's own uploads.
hipStream_t lib_stream();
hipError_t dev_alloc(void **p, size_t bytes);
void dev_free(void *p);
// Record the completion of the work just enqueued on stream for handle c (skipped while the
// stream is being captured into a graph).
void note_work(sbm_ctx *c, hipStream_t stream);
// Wait for the last run of every batch of applies still pending or alive (batch.cpp; batches
// record their completion once per run, not per handle).
void wait_batches();
// Device bytes of the handle's solver workspace (0 before the first solve).
size_t workspace_bytes(const sbm_ctx *c);
// Vector kernels (vec.hip)
hipError_t vec_fill(void *x, int64_t n, double val, int prec, hipStream_t s);
}  // namespace sbm

#define SBM_HIP_CHECK(expr)                                                      \
  do {                                                                           \
    hipError_t _e = (expr);                                                      \
    if (_e != hipSuccess) {                                                      \
      sbm::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));         \
      return SBM_EHIP;                                                           \
    }                                                                            \
  } while (0)
