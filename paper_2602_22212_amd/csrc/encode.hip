// Multi-resolution latent-grid lookup (Sec. 3.2) and its backward.
//
// Forward: one thread per reference vertex gathers the 8 cell corners of
// every position level and of the normal grid; the position result is the
// mean over levels. In the BF16 form each gathered feature is rounded to
// bfloat16 first (the float32 master grid is unchanged).
// Backward: the vertex -> node scatter is replaced by a gather over a
// node-sorted table built once per plan (setup.hip): chunks of at most 32
// entries are summed in order, then each touched node adds its chunks in
// order. No atomics, so the result is bitwise reproducible.
#include "internal.h"

namespace {

__global__ void k_encode_fwd(const float4* __restrict__ xyz, const float4* __restrict__ nrm,
                             const NpgGrid* __restrict__ g, int L, const float* __restrict__ params,
                             int64_t V, int Fp, int Fn, int bf16, float* __restrict__ z) {
  int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int Fz = Fn + Fp;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  float4 x = xyz[v];
  for (int s = 0; s < L; ++s) {
    const int R = g[s].R;
    const float* G = params + g[s].poff;
    int ix, iy, iz;
    float fx, fy, fz;
    npg_cell(x.x, R, ix, fx);
    npg_cell(x.y, R, iy, fy);
    npg_cell(x.z, R, iz, fz);
    float lv[4] = {0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < 8; ++c) {
      int64_t node = ((int64_t)(iz + (c >> 2)) * R + (iy + ((c >> 1) & 1))) * R + (ix + (c & 1));
      float w = npg_corner_w(c, fx, fy, fz);
      for (int f = 0; f < Fp; ++f) {
        const float gv = G[node * Fp + f];
        lv[f] = fmaf(w, bf16 ? npg_bf16_round(gv) : gv, lv[f]);
      }
    }
    for (int f = 0; f < Fp; ++f) acc[f] += lv[f];
  }
  const float invL = g[0].scale;
  for (int f = 0; f < Fp; ++f) z[v * Fz + Fn + f] = acc[f] * invL;

  float4 n = nrm[v];
  const int R = g[L].R;
  const float* G = params + g[L].poff;
  int ix, iy, iz;
  float fx, fy, fz;
  npg_cell(n.x, R, ix, fx);
  npg_cell(n.y, R, iy, fy);
  npg_cell(n.z, R, iz, fz);
  float zn[4] = {0.f, 0.f, 0.f, 0.f};
  for (int c = 0; c < 8; ++c) {
    int64_t node = ((int64_t)(iz + (c >> 2)) * R + (iy + ((c >> 1) & 1))) * R + (ix + (c & 1));
    float w = npg_corner_w(c, fx, fy, fz);
    for (int f = 0; f < Fn; ++f) {
      const float gv = G[node * Fn + f];
      zn[f] = fmaf(w, bf16 ? npg_bf16_round(gv) : gv, zn[f]);
    }
  }
  for (int f = 0; f < Fn; ++f) z[v * Fz + f] = zn[f];
}

__global__ void k_fill_zero(float* __restrict__ p, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// Pass 1: one thread per chunk of consecutive (same-node) entries.
__global__ void k_encode_bwd_chunks(const int32_t* __restrict__ chunk_start, const int8_t* __restrict__ chunk_sys,
                                    int64_t n_chunk, const int32_t* __restrict__ e_vert,
                                    const float* __restrict__ e_w, const NpgGrid* __restrict__ g, int L,
                                    int Fz, int Fn, const float* __restrict__ gz,
                                    float* __restrict__ chunk_sum) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= n_chunk) return;
  const int s = chunk_sys[c];
  const int F = g[s].F;
  const int col = s < L ? Fn : 0;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int e = chunk_start[c]; e < chunk_start[c + 1]; ++e) {
    const float* src = gz + (int64_t)e_vert[e] * Fz + col;
    const float w = e_w[e];
    for (int f = 0; f < F; ++f) acc[f] = fmaf(w, src[f], acc[f]);
  }
  for (int f = 0; f < 4; ++f) chunk_sum[c * 4 + f] = acc[f];
}

// Pass 2: one thread per touched node adds its chunks in order.
__global__ void k_encode_bwd_nodes(const int32_t* __restrict__ seg_key, const int32_t* __restrict__ seg_chunk0,
                                   int64_t n_seg, const float* __restrict__ chunk_sum,
                                   const NpgGrid* __restrict__ g, int n_sys, float* __restrict__ grad) {
  int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (u >= n_seg) return;
  const int64_t key = seg_key[u];
  int s = 0;
  while (s + 1 < n_sys && key >= g[s + 1].noff) ++s;
  const int F = g[s].F;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int c = seg_chunk0[u]; c < seg_chunk0[u + 1]; ++c)
    for (int f = 0; f < F; ++f) acc[f] += chunk_sum[(int64_t)c * 4 + f];
  float* dst = grad + g[s].poff + (key - g[s].noff) * F;
  const float sc = g[s].scale;
  for (int f = 0; f < F; ++f) dst[f] = acc[f] * sc;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t npg_launch_encode_fwd(const npg_plan* P, const float* params, float* z) {
  hipLaunchKernelGGL(k_encode_fwd, dim3(nblk(P->V, 128)), dim3(128), 0, P->stream, P->xyz, P->nrm, P->d_g,
                     P->L, params, P->V, P->cfg.feat_p, P->cfg.feat_n, (int)(P->cfg.precision == NPG_PREC_BF16), z);
  return hipGetLastError();
}

hipError_t npg_launch_encode_bwd(const npg_plan* P, const float* gz, float* grad) {
  hipLaunchKernelGGL(k_fill_zero, dim3(nblk(P->n_grid_params, 256)), dim3(256), 0, P->stream, grad,
                     P->n_grid_params);
  hipLaunchKernelGGL(k_encode_bwd_chunks, dim3(nblk(P->n_chunk, 256)), dim3(256), 0, P->stream,
                     P->chunk_start, P->chunk_sys, P->n_chunk, P->e_vert, P->e_w, P->d_g, P->L, P->Fz,
                     P->cfg.feat_n, gz, P->chunk_sum);
  hipLaunchKernelGGL(k_encode_bwd_nodes, dim3(nblk(P->n_seg, 256)), dim3(256), 0, P->stream, P->seg_key,
                     P->seg_chunk0, P->n_seg, P->chunk_sum, P->d_g, P->n_sys, grad);
  return hipGetLastError();
}
