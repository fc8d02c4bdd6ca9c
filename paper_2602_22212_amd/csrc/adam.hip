// Adam (Sec. 3.5, "Implementation Details": default constants, bias
// corrected) over the flat parameter vector, with one learning rate per grid
// level, one for the normal grid and one for the MLP.
#include "internal.h"

namespace {

struct Segs {
  int n;
  int64_t start[NPG_MAX_SYS + 2];
  float lr[NPG_MAX_SYS + 1];
};

__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, Segs sg, float b1, float b2, float eps, float inv_bc1,
                       float inv_sqrt_bc2, const NpgStepScal* __restrict__ sc, int* __restrict__ flag) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (sc) {
    if (sc->cg_state & 3) return;  // a recorded CG solve stopped short: the step is redone
    inv_bc1 = sc->inv_bc1;
    inv_sqrt_bc2 = sc->inv_sqrt_bc2;
  }
  int s = 0;
  while (s + 1 < sg.n && i >= sg.start[s + 1]) ++s;
  const float gi = g[i];
  const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
  const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
  m[i] = mi;
  v[i] = vi;
  const float denom = sqrtf(vi) * inv_sqrt_bc2 + eps;
  const float t = th[i] - sg.lr[s] * (mi * inv_bc1) / denom;
  th[i] = t;
  if (!isfinite(t)) atomicOr(flag, 1);
}

}  // namespace

void npg_adam_scalars(const npg_plan* P, int64_t k, float* inv_bc1, float* inv_sqrt_bc2) {
  const double bc1 = 1.0 - pow((double)P->cfg.beta1, (double)k);
  const double bc2 = 1.0 - pow((double)P->cfg.beta2, (double)k);
  *inv_bc1 = (float)(1.0 / bc1);
  *inv_sqrt_bc2 = (float)(1.0 / sqrt(bc2));
}

hipError_t npg_launch_adam(const npg_plan* P, float* params, const float* grad, float* m, float* v, int64_t k,
                           int* flag, const NpgStepScal* sc) {
  Segs sg;
  sg.n = P->n_sys + 1;
  for (int s = 0; s < P->n_sys; ++s) {
    sg.start[s] = P->g[s].poff;
    sg.lr[s] = P->g[s].lr;
  }
  sg.start[P->n_sys] = P->mlp_off;
  sg.lr[P->n_sys] = P->cfg.lr_mlp;
  sg.start[P->n_sys + 1] = P->n_params;
  float ib1 = 1.f, ib2 = 1.f;
  if (!sc) npg_adam_scalars(P, k, &ib1, &ib2);
  const int64_t n = P->n_params;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, P->stream, params, grad, m, v, n, sg,
                     P->cfg.beta1, P->cfg.beta2, P->cfg.eps, ib1, ib2, sc, flag);
  return hipGetLastError();
}
