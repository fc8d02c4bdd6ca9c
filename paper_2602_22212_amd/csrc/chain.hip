// Chain-rule product for reverse-mode callers (torch.autograd Functions over
// the stage entry points): a stage's gradient times the upstream gradient of
// the scalar it feeds, x[k] *= c * s[0], with the factor formed in float64 on
// the device so the host never reads the upstream gradient.
#include <algorithm>

#include "internal.h"

namespace {

constexpr int kB = 256;

template <typename F>
__global__ __launch_bounds__(kB) void k_scale(const double* __restrict__ s, double c, F* __restrict__ x, int64_t n) {
  const double f = c * s[0];
  const int64_t stride = (int64_t)gridDim.x * kB;
  for (int64_t k = blockIdx.x * (int64_t)kB + threadIdx.x; k < n; k += stride) x[k] = (F)((double)x[k] * f);
}

__global__ void k_scaled_copy(const double* __restrict__ w, const double* __restrict__ g, double* __restrict__ out,
                              int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = w[k] * g[0];
}

}  // namespace

hipError_t npg_launch_scaled_copy(const npg_plan* P, const double* w, const double* g, double* out, int n) {
  hipLaunchKernelGGL(k_scaled_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, P->stream, w, g, out, n);
  return hipGetLastError();
}

extern "C" npg_status npg_scale(npg_plan* P, const double* s, double c, void* x, int32_t is_f64, int64_t n) {
  if (!P || !s || (!x && n > 0) || n < 0) return npg_fail(NPG_EINVAL, "npg_scale: NULL plan/factor/vector or n < 0");
  if (n == 0) return NPG_OK;
  const unsigned grid = (unsigned)std::min<int64_t>((n + kB - 1) / kB, 4096);
  if (is_f64)
    hipLaunchKernelGGL(k_scale<double>, dim3(grid), dim3(kB), 0, P->stream, s, c, (double*)x, n);
  else
    hipLaunchKernelGGL(k_scale<float>, dim3(grid), dim3(kB), 0, P->stream, s, c, (float*)x, n);
  NPG_HIP(hipGetLastError());
  return NPG_OK;
}
