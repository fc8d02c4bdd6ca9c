// Isometry loss of Sec. 3.5: L_iso = mean over frames t and mesh edges (i, j)
// of | |x^_i,t - x^_j,t| - sg(|x^_i,key - x^_j,key|) |, the key-frame lengths
// taken from the current deformed key frame under a stop-gradient, and its
// gradient w_iso dL_iso/dx^ added into the loss gradient.
//
// One thread per (frame, vertex) walks the vertex's incident edges (a
// vertex -> edge table built once from the edge list), so the gradient is a
// gather: no atomics, bitwise reproducible. Each edge's loss term and
// subgradient decision is taken by its lower-indexed endpoint only.
// Lengths and decisions are computed in float64 from the float32 vertices;
// sign(0) = 0 (the key frame's own terms, exactly equal lengths) and a
// zero-length edge contributes no gradient.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace {

constexpr int kB = 256;
constexpr int kR = 1024;
constexpr uint32_t kOwn = 0x80000000u;

// Length of a - b in float64 and the difference vector. The difference of
// the swapped pair is the exact negation, so both endpoints of an edge get
// the same length and the same decision.
__device__ __forceinline__ double len64(const float4& a, const float4& b, double& dx, double& dy, double& dz) {
  dx = (double)a.x - (double)b.x;
  dy = (double)a.y - (double)b.y;
  dz = (double)a.z - (double)b.z;
  return sqrt(dx * dx + dy * dy + dz * dz);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__global__ __launch_bounds__(kB) void k_iso(const float4* __restrict__ xhat, int64_t V, int T, int t_key,
                                            const int* __restrict__ row, const int* __restrict__ nbr,
                                            const uint32_t* __restrict__ eid, int64_t E, double scale,
                                            const double* __restrict__ gs, float4* __restrict__ gxhat,
                                            int8_t* __restrict__ sign, double* __restrict__ part) {
  if (gs) scale *= gs[0];  // upstream factor of a reverse-mode caller
  __shared__ double ws[kB / 64];
  const int64_t s = blockIdx.x * (int64_t)kB + threadIdx.x;
  double acc = 0.0;
  if (s < (int64_t)T * V) {
    const int64_t t = s / V, i = s - t * V;
    const float4* Xt = xhat + t * V;
    const float4* Xk = xhat + (int64_t)t_key * V;
    const float4 xi = Xt[i], ki = Xk[i];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    const int k1 = row[i + 1];
    for (int k = row[i]; k < k1; ++k) {
      const int64_t j = nbr[k];
      const uint32_t ek = eid[k];
      double dx, dy, dz, kx, ky, kz;
      const double l = len64(xi, Xt[j], dx, dy, dz);
      const double lb = len64(ki, Xk[j], kx, ky, kz);
      const double diff = l - lb;
      const int sg = (diff > 0.0) - (diff < 0.0);
      if (ek & kOwn) {
        acc += fabs(diff);
        if (sign) sign[t * E + (ek & ~kOwn)] = (int8_t)sg;
      }
      if (sg != 0 && l > 0.0) {
        const double c = (double)sg / l;
        gx += c * dx;
        gy += c * dy;
        gz += c * dz;
      }
    }
    if (gxhat) {
      float4 g = gxhat[s];
      g.x += (float)(scale * gx);
      g.y += (float)(scale * gy);
      g.z += (float)(scale * gz);
      gxhat[s] = g;
    }
  }
  const double w = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// L_iso = (sum of the block partials in order) / (T E); optionally
// loss += w_iso L_iso.
__global__ __launch_bounds__(kR) void k_iso_finish(const double* __restrict__ part, int nblk, double inv_te,
                                                   double w_iso, double* __restrict__ iso,
                                                   double* __restrict__ loss) {
  __shared__ double red[kR / 64];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kR) acc += part[b];
  const double w = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double v = 0.0;
  for (int k = 0; k < kR / 64; ++k) v += red[k];
  v *= inv_te;
  if (iso) iso[0] = v;
  if (loss) loss[0] += w_iso * v;
}

}  // namespace

npg_status npg_iso_set_edges(npg_plan* P, int64_t E, const int32_t* edges) {
  const int64_t V = P->V;
  std::vector<int> deg(V + 1, 0);
  for (int64_t e = 0; e < E; ++e) {
    const int32_t i = edges[2 * e], j = edges[2 * e + 1];
    if (i < 0 || j < 0 || i >= V || j >= V || i == j)
      return npg_fail(NPG_EINVAL, "edge " + std::to_string(e) + " has an endpoint outside [0, V) or i == j");
    ++deg[i + 1];
    ++deg[j + 1];
  }
  for (int64_t v = 0; v < V; ++v) deg[v + 1] += deg[v];
  std::vector<int> nbr(2 * E), fill(deg.begin(), deg.end() - 1);
  std::vector<uint32_t> eid(2 * E);
  for (int64_t e = 0; e < E; ++e) {  // edge order within each vertex: deterministic
    const int32_t i = edges[2 * e], j = edges[2 * e + 1];
    const int ki = fill[i]++, kj = fill[j]++;
    nbr[ki] = j;
    eid[ki] = (uint32_t)e | (i < j ? kOwn : 0u);
    nbr[kj] = i;
    eid[kj] = (uint32_t)e | (j < i ? kOwn : 0u);
  }
  NPG_HIP(hipStreamSynchronize(P->stream));  // earlier steps may still read the old table
  hipFree(P->iso_row);
  hipFree(P->iso_nbr);
  hipFree(P->iso_eid);
  P->iso_row = nullptr;
  P->iso_nbr = nullptr;
  P->iso_eid = nullptr;
  P->n_edges = 0;
  NPG_HIP(hipMalloc(&P->iso_row, (V + 1) * sizeof(int)));
  NPG_HIP(hipMalloc(&P->iso_nbr, std::max<int64_t>(1, 2 * E) * sizeof(int)));
  NPG_HIP(hipMalloc(&P->iso_eid, std::max<int64_t>(1, 2 * E) * sizeof(uint32_t)));
  NPG_HIP(hipMemcpy(P->iso_row, deg.data(), (V + 1) * sizeof(int), hipMemcpyHostToDevice));
  NPG_HIP(hipMemcpy(P->iso_nbr, nbr.data(), 2 * E * sizeof(int), hipMemcpyHostToDevice));
  NPG_HIP(hipMemcpy(P->iso_eid, eid.data(), 2 * E * sizeof(uint32_t), hipMemcpyHostToDevice));
  if (!P->iso_part) {
    P->n_iso_blk = (int)(((int64_t)P->T * V + kB - 1) / kB);
    NPG_HIP(hipMalloc(&P->iso_part, (size_t)P->n_iso_blk * sizeof(double)));
    NPG_HIP(hipMalloc(&P->iso_val, sizeof(double)));
  }
  P->n_edges = E;
  return NPG_OK;
}

void npg_iso_free(npg_plan* P) {
  hipFree(P->iso_row);
  hipFree(P->iso_nbr);
  hipFree(P->iso_eid);
  hipFree(P->iso_part);
  hipFree(P->iso_val);
}

hipError_t npg_launch_iso(const npg_plan* P, const float4* xhat, float4* gxhat, double* iso, int8_t* sign,
                          double* loss, const double* gs) {
  const double inv_te = 1.0 / ((double)P->T * (double)P->n_edges);
  const double scale = (double)P->cfg.w_iso * inv_te;
  hipLaunchKernelGGL(k_iso, dim3(P->n_iso_blk), dim3(kB), 0, P->stream, xhat, P->V, P->T, P->t_key, P->iso_row,
                     P->iso_nbr, P->iso_eid, P->n_edges, scale, gs, gxhat, sign, P->iso_part);
  hipLaunchKernelGGL(k_iso_finish, dim3(1), dim3(kR), 0, P->stream, P->iso_part, P->n_iso_blk, inv_te,
                     (double)P->cfg.w_iso, iso, loss);
  return hipGetLastError();
}
