// Multi-resolution latent-grid lookup (Sec. 3.2) and its backward.
//
// Forward: the 8 cell corners of every position level and of the normal grid
// at each reference vertex, the position result the mean over levels;
// vertices in Morton order, each grid's box of a 64-vertex patch staged in
// LDS (k_encode_fwd). In the BF16 form each gathered feature is rounded to
// bfloat16 first (the float32 master grid is unchanged).
// Backward: the vertex -> node scatter is replaced by a gather over a
// node-sorted table built once per plan (setup.hip): chunks of at most 32
// entries are summed in order, then each touched node adds its chunks in
// order. No atomics, so the result is bitwise reproducible.
#include "internal.h"

namespace {

constexpr int kEV = 64;       // vertices per work-group (the lanes of a wave)
constexpr int kEW = 4;        // waves per work-group: the grids are dealt to them in turn
constexpr int kETile = 512;   // nodes of one grid a wave stages in LDS (float4 each)

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v = min(v, __shfl_xor(v, m));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v = max(v, __shfl_xor(v, m));
  return v;
}

// One work-group: 64 vertices consecutive in the plan's Morton order (a
// compact patch of the surface), every grid (the L position levels, then the
// normal grid) dealt to its four waves in turn. Per grid the wave takes the
// bounding box of the 64 vertices' cells (corner nodes included); when it
// holds at most kETile nodes of 4 features (every grid at the benchmark
// sizes), the wave copies it from HBM into LDS with coalesced loads (rows of
// consecutive x) and gathers the 8 corners of each vertex there, otherwise
// it gathers from global memory. The per-grid sums (corners in order) meet
// in LDS and the first wave adds the levels in order, so the result is
// bitwise that of a corner-by-corner, level-by-level evaluation. In the BF16
// form each gathered feature is rounded to bfloat16 first.
__global__ __launch_bounds__(kEV * kEW) void k_encode_fwd(const float4* __restrict__ xyz,
                                                          const float4* __restrict__ nrm,
                                                          const int32_t* __restrict__ perm,
                                                          const NpgGrid* __restrict__ g, int L,
                                                          const float* __restrict__ params, int64_t V, int Fp,
                                                          int Fn, int bf16, float* __restrict__ z) {
  __shared__ float4 tile[kEW][kETile];
  __shared__ float4 lvs[NPG_MAX_SYS][kEV];
  const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
  const int64_t k = (int64_t)blockIdx.x * kEV + lane;
  const bool valid = k < V;
  const int64_t v = perm[valid ? k : V - 1];
  const float4 xv = xyz[v], nv = nrm[v];
  for (int s = w; s <= L; s += kEW) {
    const NpgGrid gs = g[s];
    const float4 q = s < L ? xv : nv;
    const float* G = params + gs.poff;
    const int R = gs.R, F = gs.F;
    int ix, iy, iz;
    float fx, fy, fz;
    npg_cell(q.x, R, ix, fx);
    npg_cell(q.y, R, iy, fy);
    npg_cell(q.z, R, iz, fz);
    // lanes past V repeat the last vertex, so every lane's cell is in the box
    const int lx = wave_min_i(ix), ly = wave_min_i(iy), lz = wave_min_i(iz);
    const int nx = wave_max_i(ix) + 2 - lx, ny = wave_max_i(iy) + 2 - ly, nz = wave_max_i(iz) + 2 - lz;
    const bool staged = F == 4 && (gs.poff % 4) == 0 && (int64_t)nx * ny * nz <= kETile;
    float lv[4] = {0.f, 0.f, 0.f, 0.f};
    if (staged) {
      const float4* G4 = reinterpret_cast<const float4*>(G);
      const int nxy = nx * ny, nn = nxy * nz;
      for (int e = lane; e < nn; e += 64) {
        const int ez = e / nxy, rem = e - ez * nxy, ey = rem / nx, ex = rem - ey * nx;
        tile[w][e] = G4[((int64_t)(lz + ez) * R + (ly + ey)) * R + (lx + ex)];
      }
      // only this wave reads its buffer (LDS operations of a wave complete in order)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int base = ((iz - lz) * ny + (iy - ly)) * nx + (ix - lx);
      for (int c = 0; c < 8; ++c) {
        const float4 gv = tile[w][base + ((c >> 2) * ny + ((c >> 1) & 1)) * nx + (c & 1)];
        const float wc = npg_corner_w(c, fx, fy, fz);
        lv[0] = fmaf(wc, bf16 ? npg_bf16_round(gv.x) : gv.x, lv[0]);
        lv[1] = fmaf(wc, bf16 ? npg_bf16_round(gv.y) : gv.y, lv[1]);
        lv[2] = fmaf(wc, bf16 ? npg_bf16_round(gv.z) : gv.z, lv[2]);
        lv[3] = fmaf(wc, bf16 ? npg_bf16_round(gv.w) : gv.w, lv[3]);
      }
      // the buffer is refilled by this wave's next grid only after every lane's reads
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      for (int c = 0; c < 8; ++c) {
        const int64_t node = ((int64_t)(iz + (c >> 2)) * R + (iy + ((c >> 1) & 1))) * R + (ix + (c & 1));
        const float wc = npg_corner_w(c, fx, fy, fz);
        for (int f = 0; f < F; ++f) {
          const float gv = G[node * F + f];
          lv[f] = fmaf(wc, bf16 ? npg_bf16_round(gv) : gv, lv[f]);
        }
      }
    }
    lvs[s][lane] = make_float4(lv[0], lv[1], lv[2], lv[3]);
  }
  __syncthreads();
  if (w != 0 || !valid) return;
  const int Fz = Fn + Fp;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int s = 0; s < L; ++s) {
    const float4 lv = lvs[s][lane];
    acc[0] += lv.x;
    acc[1] += lv.y;
    acc[2] += lv.z;
    acc[3] += lv.w;
  }
  const float invL = g[0].scale;
  for (int f = 0; f < Fp; ++f) z[v * Fz + Fn + f] = acc[f] * invL;
  const float4 zn = lvs[L][lane];
  const float znv[4] = {zn.x, zn.y, zn.z, zn.w};
  for (int f = 0; f < Fn; ++f) z[v * Fz + f] = znv[f];
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
  // the systems' node offsets, read at the same addresses by every thread
  // (one scalar batch) before the search, which then runs in registers
  int64_t noff[NPG_MAX_SYS];
#pragma unroll
  for (int k = 0; k < NPG_MAX_SYS; ++k) noff[k] = k < n_sys ? g[k].noff : INT64_MAX;
  int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (u >= n_seg) return;
  const int64_t key = seg_key[u];
  int s = 0;
#pragma unroll
  for (int k = 1; k < NPG_MAX_SYS; ++k) s += key >= noff[k];
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
  hipLaunchKernelGGL(k_encode_fwd, dim3(nblk(P->V, kEV)), dim3(kEV * kEW), 0, P->stream, P->xyz, P->nrm, P->vperm,
                     P->d_g, P->L, params, P->V, P->cfg.feat_p, P->cfg.feat_n,
                     (int)(P->cfg.precision == NPG_PREC_BF16), z);
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
