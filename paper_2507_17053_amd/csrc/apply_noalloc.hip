// sbm_apply_noalloc: the operator apply with its scratch (CG halo planes, surrogate-face
// results) taken from one file-scope device array instead of the handle's own buffers, for
// callers that cannot allocate.  The call itself allocates nothing: no hipMalloc, no hipFree,
// no allocating library routine.
//
// The array `scratch` exists once per device (every device the library runs on holds its own
// copy until the process ends).  In host code its name is only a host-side stand-in, so the
// device address is looked up once per device with hipGetSymbolAddress, with that device
// current, and kept in scratch_ptr[]; every kernel argument uses that address.  Nothing in the
// scratch has to start at zero: the surrogate-face kernel writes every face result before the
// cell kernels read it, and the halo pass reads only the planes the brick kernel wrote in the
// same apply.  All calls on one device share the array, so calls that overlap on one device
// (different streams, or other threads) race; calls ordered on one stream do not.
#include <mutex>

#include "sbm_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)96 << 20;  // 96 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on the first call on the
// device, which is then current).  Returns hipSuccess and sets *out, or the HIP error.
hipError_t scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" sbm_status sbm_apply_noalloc(sbm_handle h, const void *u, void *v, int prec, void *stream) {
  using sbm::set_error;
  if (!h) {
    set_error("sbm_apply_noalloc: NULL handle");
    return SBM_EINVAL;
  }
  if (h->host_only) {
    set_error("sbm_apply_noalloc: handle was set up with SBM_SETUP_HOST_ONLY");
    return SBM_EINVAL;
  }
  if (prec != SBM_F64 && prec != SBM_F32) {
    set_error("sbm_apply_noalloc: prec must be SBM_F64 or SBM_F32");
    return SBM_EINVAL;
  }
  if (h->n_dofs == 0) return SBM_OK;
  if (!u || !v) {
    set_error("sbm_apply_noalloc: NULL vector");
    return SBM_EINVAL;
  }
  if (u == v) {
    set_error("sbm_apply_noalloc: u and v must not alias");
    return SBM_EINVAL;
  }
  const size_t need = sbm::apply_scratch_bytes(h, prec);
  if (need > kScratchBytes) {
    set_error("sbm_apply_noalloc: the operator needs " + std::to_string(need) +
              " bytes of scratch, more than the " + std::to_string(kScratchBytes) +
              " bytes of the static device scratch; use sbm_apply");
    return SBM_EINVAL;
  }
  void *base = nullptr;
  SBM_HIP_CHECK(scratch_address(&base));
  const size_t s = prec == SBM_F64 ? sizeof(double) : sizeof(float);
  const size_t halo_bytes = h->disc == SBM_CG ? ((size_t)1 << h->dim) * (size_t)h->n_halo_dofs * s : 0;
  sbm::Scratch scr;
  scr.halo = base;
  scr.fbuf = (unsigned char *)base + (halo_bytes + 255) / 256 * 256;
  SBM_HIP_CHECK(sbm::launch_operator(h, u, v, prec, SBM_PART_ALL, (hipStream_t)stream, &scr));
  sbm::note_work(h, (hipStream_t)stream);
  return SBM_OK;
}
