// Plan-time kernels: input packing and validation, and the node-sorted
// scatter table used by the encode backward (built once per plan, because the
// reference positions and normals never change during the optimization).
#include "internal.h"

namespace {

__global__ void k_pack(const float* __restrict__ src, float4* __restrict__ dst, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = make_float4(src[3 * i], src[3 * i + 1], src[3 * i + 2], 0.0f);
}

__global__ void k_point_frames(const int64_t* __restrict__ off, int T, int* __restrict__ pf, int64_t N) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  int lo = 0, hi = T - 1;  // last t with off[t] <= j
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= j) lo = mid; else hi = mid - 1;
  }
  pf[j] = lo;
}

__global__ void k_check_finite(const float* __restrict__ p, int64_t n, int* flag) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && !isfinite(p[i])) atomicOr(flag, 1);
}

// Entry e = (s*V + v)*8 + corner: key = global node touched, val = e.
__global__ void k_gen_entries(const float4* __restrict__ xyz, const float4* __restrict__ nrm,
                              const NpgGrid* __restrict__ g, int n_sys, int L, int64_t V,
                              uint32_t* __restrict__ key, int32_t* __restrict__ val) {
  int64_t tv = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (tv >= V * n_sys) return;
  int s = (int)(tv / V);
  int64_t v = tv - (int64_t)s * V;
  float4 x = (s < L) ? xyz[v] : nrm[v];
  int R = g[s].R;
  int ix, iy, iz;
  float fx, fy, fz;
  npg_cell(x.x, R, ix, fx);
  npg_cell(x.y, R, iy, fy);
  npg_cell(x.z, R, iz, fz);
  for (int c = 0; c < 8; ++c) {
    int64_t node = ((int64_t)(iz + (c >> 2)) * R + (iy + ((c >> 1) & 1))) * R + (ix + (c & 1));
    key[tv * 8 + c] = (uint32_t)(g[s].noff + node);
    val[tv * 8 + c] = (int32_t)(tv * 8 + c);
  }
}

constexpr int kTile = 2048;

__global__ void k_radix_hist(const uint32_t* __restrict__ key, int64_t n, int shift, int nb,
                             int* __restrict__ counts) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kTile;
  for (int i = threadIdx.x; i < kTile; i += 256) {
    int64_t e = base + i;
    if (e < n) atomicAdd(&cnt[(key[e] >> shift) & 255], 1);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: thread d walks the tile in order and moves the items whose
// digit is d, so equal keys keep their input order.
__global__ void k_radix_scatter(const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                int64_t n, int shift, int nb, const int* __restrict__ offs,
                                uint32_t* __restrict__ kout, int32_t* __restrict__ vout) {
  __shared__ uint32_t sk[kTile];
  __shared__ int32_t sv[kTile];
  int64_t base = (int64_t)blockIdx.x * kTile;
  int cntn = (int)((n - base) < kTile ? (n - base) : kTile);
  for (int i = threadIdx.x; i < cntn; i += 256) {
    sk[i] = kin[base + i];
    sv[i] = vin[base + i];
  }
  __syncthreads();
  int d = threadIdx.x;
  int pos = offs[(int64_t)d * nb + blockIdx.x];
  for (int i = 0; i < cntn; ++i) {
    uint32_t k = sk[i];
    if (((k >> shift) & 255) == (uint32_t)d) {
      kout[pos] = k;
      vout[pos] = sv[i];
      ++pos;
    }
  }
}

// Single-block scan of n int32 values (inclusive or exclusive). Plan-time only.
__global__ void k_scan1(const int* __restrict__ in, int* __restrict__ out, int64_t n, int exclusive) {
  __shared__ int64_t part[1024];
  int tid = threadIdx.x;
  int64_t per = (n + 1023) / 1024;
  int64_t lo = tid * per, hi = lo + per < n ? lo + per : n;
  int64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += in[i];
  part[tid] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int64_t add = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  int64_t run = part[tid] - s;  // exclusive prefix of this thread's range
  for (int64_t i = lo; i < hi; ++i) {
    int x = in[i];
    if (exclusive) { out[i] = (int)run; run += x; }
    else { run += x; out[i] = (int)run; }
  }
}

__global__ void k_heads(const uint32_t* __restrict__ key, int64_t n, int* __restrict__ head) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) head[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

__global__ void k_seg_fill(const uint32_t* __restrict__ key, const int* __restrict__ head,
                           const int* __restrict__ seg_incl, int64_t n, int* __restrict__ seg_start,
                           int32_t* __restrict__ seg_key) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && head[i]) {
    int s = seg_incl[i] - 1;
    seg_start[s] = (int)i;
    seg_key[s] = (int32_t)key[i];
  }
}

__global__ void k_chunk_heads(const int* __restrict__ seg_incl, const int* __restrict__ seg_start,
                              int64_t n, int chunk, int* __restrict__ ch) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    int s = seg_incl[i] - 1;
    ch[i] = ((i - seg_start[s]) % chunk == 0) ? 1 : 0;
  }
}

__global__ void k_chunk_fill(const uint32_t* __restrict__ key, const int* __restrict__ head,
                             const int* __restrict__ seg_incl, const int* __restrict__ ch,
                             const int* __restrict__ ch_incl, int64_t n, const NpgGrid* __restrict__ g,
                             int n_sys, int32_t* __restrict__ chunk_start, int32_t* __restrict__ seg_chunk0,
                             int8_t* __restrict__ chunk_sys) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && ch[i]) {
    int c = ch_incl[i] - 1;
    chunk_start[c] = (int32_t)i;
    int s = 0;
    while (s + 1 < n_sys && (int64_t)key[i] >= g[s + 1].noff) ++s;
    chunk_sys[c] = (int8_t)s;
    if (head[i]) seg_chunk0[seg_incl[i] - 1] = c;
  }
}

// Sorted entry -> (vertex, trilinear weight), with the forward's cell routine.
__global__ void k_entry_weights(const int32_t* __restrict__ val, int64_t n, const float4* __restrict__ xyz,
                                const float4* __restrict__ nrm, const NpgGrid* __restrict__ g, int L,
                                int64_t V, int32_t* __restrict__ e_vert, float* __restrict__ e_w) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t e = val[i];
  int c = (int)(e & 7);
  int64_t tv = e >> 3;
  int s = (int)(tv / V);
  int64_t v = tv - (int64_t)s * V;
  float4 x = (s < L) ? xyz[v] : nrm[v];
  int R = g[s].R, ix, iy, iz;
  float fx, fy, fz;
  npg_cell(x.x, R, ix, fx);
  npg_cell(x.y, R, iy, fy);
  npg_cell(x.z, R, iz, fz);
  e_vert[i] = (int32_t)v;
  e_w[i] = npg_corner_w(c, fx, fy, fz);
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t npg_launch_pack(const float* src, float4* dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack, dim3(nblk(n, 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t npg_launch_point_frames(const int64_t* off, int T, int* pf, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_point_frames, dim3(nblk(N, 256)), dim3(256), 0, s, off, T, pf, N);
  return hipGetLastError();
}

hipError_t npg_launch_check_finite(const float* p, int64_t n, int* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_finite, dim3(nblk(n, 256)), dim3(256), 0, s, p, n, flag);
  return hipGetLastError();
}

npg_status npg_build_scatter_table(npg_plan* P) {
  const int64_t V = P->V;
  const int64_t E = V * 8 * P->n_sys;
  hipStream_t s = P->stream;
  if (E >= (int64_t)1 << 31) return npg_fail(NPG_EINVAL, "scatter table too large (V too big)");
  P->n_entries = E;
  uint32_t *k0, *k1;
  int32_t *v0, *v1;
  int *counts, *head, *seg_incl, *seg_start, *ch, *ch_incl;
  const int nb = (int)nblk(E, kTile);
  NPG_HIP(hipMalloc(&k0, E * 4));
  NPG_HIP(hipMalloc(&k1, E * 4));
  NPG_HIP(hipMalloc(&v0, E * 4));
  NPG_HIP(hipMalloc(&v1, E * 4));
  NPG_HIP(hipMalloc(&counts, (int64_t)256 * nb * 4));
  hipLaunchKernelGGL(k_gen_entries, dim3(nblk(V * P->n_sys, 256)), dim3(256), 0, s, P->xyz, P->nrm,
                     P->d_g, P->n_sys, P->L, V, k0, v0);
  NPG_HIP(hipGetLastError());
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) <= P->n_nodes) ++bits;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(256), 0, s, k0, E, shift, nb, counts);
    hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, s, counts, counts, (int64_t)256 * nb, 1);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(256), 0, s, k0, v0, E, shift, nb, counts, k1, v1);
    NPG_HIP(hipGetLastError());
    std::swap(k0, k1);
    std::swap(v0, v1);
  }
  NPG_HIP(hipMalloc(&head, E * 4));
  NPG_HIP(hipMalloc(&seg_incl, E * 4));
  NPG_HIP(hipMalloc(&ch, E * 4));
  NPG_HIP(hipMalloc(&ch_incl, E * 4));
  hipLaunchKernelGGL(k_heads, dim3(nblk(E, 256)), dim3(256), 0, s, k0, E, head);
  hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, s, head, seg_incl, E, 0);
  NPG_HIP(hipGetLastError());
  int U = 0;
  NPG_HIP(hipMemcpyAsync(&U, seg_incl + E - 1, 4, hipMemcpyDeviceToHost, s));
  NPG_HIP(hipStreamSynchronize(s));
  P->n_seg = U;
  NPG_HIP(hipMalloc(&seg_start, (int64_t)U * 4));
  NPG_HIP(hipMalloc(&P->seg_key, (int64_t)U * 4));
  hipLaunchKernelGGL(k_seg_fill, dim3(nblk(E, 256)), dim3(256), 0, s, k0, head, seg_incl, E, seg_start,
                     P->seg_key);
  const int kChunk = 32;
  hipLaunchKernelGGL(k_chunk_heads, dim3(nblk(E, 256)), dim3(256), 0, s, seg_incl, seg_start, E, kChunk, ch);
  hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, s, ch, ch_incl, E, 0);
  NPG_HIP(hipGetLastError());
  int C = 0;
  NPG_HIP(hipMemcpyAsync(&C, ch_incl + E - 1, 4, hipMemcpyDeviceToHost, s));
  NPG_HIP(hipStreamSynchronize(s));
  P->n_chunk = C;
  NPG_HIP(hipMalloc(&P->chunk_start, ((int64_t)C + 1) * 4));
  NPG_HIP(hipMalloc(&P->seg_chunk0, ((int64_t)U + 1) * 4));
  NPG_HIP(hipMalloc(&P->chunk_sum, (int64_t)C * 4 * 4));
  NPG_HIP(hipMalloc(&P->chunk_sys, (int64_t)C));
  hipLaunchKernelGGL(k_chunk_fill, dim3(nblk(E, 256)), dim3(256), 0, s, k0, head, seg_incl, ch, ch_incl, E,
                     P->d_g, P->n_sys, P->chunk_start, P->seg_chunk0, P->chunk_sys);
  int32_t tailC = (int32_t)C, tailE = (int32_t)E;
  NPG_HIP(hipMemcpyAsync(P->seg_chunk0 + U, &tailC, 4, hipMemcpyHostToDevice, s));
  NPG_HIP(hipMemcpyAsync(P->chunk_start + C, &tailE, 4, hipMemcpyHostToDevice, s));
  NPG_HIP(hipMalloc(&P->e_vert, E * 4));
  NPG_HIP(hipMalloc(&P->e_w, E * 4));
  hipLaunchKernelGGL(k_entry_weights, dim3(nblk(E, 256)), dim3(256), 0, s, v0, E, P->xyz, P->nrm, P->d_g,
                     P->L, V, P->e_vert, P->e_w);
  NPG_HIP(hipGetLastError());
  NPG_HIP(hipStreamSynchronize(s));
  hipFree(k0); hipFree(k1); hipFree(v0); hipFree(v1); hipFree(counts);
  hipFree(head); hipFree(seg_incl); hipFree(ch); hipFree(ch_incl); hipFree(seg_start);
  return NPG_OK;
}
