// Vector fill (x = val in FP64 or FP32), used by the solver to clear its vectors.  The other
// vector operations of the solvers (casts, fused updates, reductions) live in solver.hip,
// fused into the kernels that need them.
#include "sbm_internal.h"

namespace sbm {
namespace {

constexpr int kVecThreads = 256;

inline int vec_blocks(int64_t n) {
  int64_t b = (n + kVecThreads * 4 - 1) / (kVecThreads * 4);
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (int)b;
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void fill_kernel(T *x, int64_t n, T val) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = val;
}

}  // namespace

hipError_t vec_fill(void *x, int64_t n, double val, int prec, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (prec == SBM_F64)
    hipLaunchKernelGGL(fill_kernel<double>, dim3(vec_blocks(n)), dim3(kVecThreads), 0, s, (double *)x, n, val);
  else
    hipLaunchKernelGGL(fill_kernel<float>, dim3(vec_blocks(n)), dim3(kVecThreads), 0, s, (float *)x, n,
                       (float)val);
  return hipGetLastError();
}

}  // namespace sbm
