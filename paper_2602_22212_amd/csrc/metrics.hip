// Evaluation metrics of Sec. 4 on ground truth (the paper names CD, NC,
// F-score and correspondence error; the per-frame definitions below are the
// readings this library takes). Per frame t, with nearest neighbours between
// the predicted vertices x^ and the true vertices g (a: prediction -> truth,
// b: truth -> prediction, lowest index on exact ties):
//   CD   = mean_i |x^_i - g_a(i)|^2 + mean_j |g_j - x^_b(j)|^2
//   NC   = (mean_i |n^_i . m_a(i)| + mean_j |m_j . n^_b(j)|) / 2
//   F    = 2 P R / (P + R), P and R the shares of squared NN distances
//          below tau^2 in each direction (0 when P + R = 0)
//   Corr = mean_i |x^_i - g_i|
// The nearest-neighbour search is the Chamfer kernel pair with the true
// vertices as the point set; one work-group per frame reduces the sums in
// float64 in a fixed order.
#include "internal.h"

namespace {

constexpr int kB = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ double absdot(const float4& p, const float4& q) {
  return fabs((double)p.x * q.x + (double)p.y * q.y + (double)p.z * q.z);
}

__global__ void k_frame_index(int64_t V, int T, int64_t* __restrict__ off, int* __restrict__ pt_frame) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e <= T) off[e] = e * V;
  if (e < (int64_t)T * V) pt_frame[e] = (int)(e / V);
}

__global__ __launch_bounds__(kB) void k_metrics(const float4* __restrict__ xhat, const float4* __restrict__ nhat,
                                                const float4* __restrict__ gt, const float4* __restrict__ gtn,
                                                const int32_t* __restrict__ a, const float* __restrict__ da,
                                                const int32_t* __restrict__ b, const float* __restrict__ db,
                                                int64_t V, float tau2, double* __restrict__ out) {
  constexpr int kN = 7;  // cd_a, cd_b, nc_a, nc_b, P count, R count, corr
  __shared__ double ws[kB / 64][kN];
  const int t = blockIdx.x;
  const int64_t base = (int64_t)t * V;
  double s[kN] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = threadIdx.x; i < V; i += kB) {
    const int64_t e = base + i;
    const float dai = da[e], dbi = db[e];
    s[0] += dai;
    s[1] += dbi;
    s[2] += absdot(nhat[e], gtn[base + a[e]]);
    s[3] += absdot(gtn[e], nhat[base + b[e]]);
    s[4] += dai < tau2 ? 1.0 : 0.0;
    s[5] += dbi < tau2 ? 1.0 : 0.0;
    const float4 x = xhat[e], g = gt[e];
    const double dx = (double)x.x - g.x, dy = (double)x.y - g.y, dz = (double)x.z - g.z;
    s[6] += sqrt(dx * dx + dy * dy + dz * dz);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kN; ++k) {
    const double v = wave_sum(s[k]);
    if (lane == 0) ws[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double r[kN];
  for (int k = 0; k < kN; ++k) r[k] = ((ws[0][k] + ws[1][k]) + ws[2][k]) + ws[3][k];
  const double inv = 1.0 / (double)V;
  const double P = r[4] * inv, R = r[5] * inv;
  out[4 * t + 0] = r[0] * inv + r[1] * inv;
  out[4 * t + 1] = 0.5 * (r[2] * inv + r[3] * inv);
  out[4 * t + 2] = P + R > 0.0 ? 2.0 * P * R / (P + R) : 0.0;
  out[4 * t + 3] = r[6] * inv;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

npg_status npg_run_metrics(npg_plan* P, const float4* xhat, const float4* nhat, const float4* gt, const float4* gtn,
                           float tau, double* out) {
  const int64_t V = P->V, T = P->T, n = T * V;
  int64_t* off = nullptr;
  int* pt_frame = nullptr;
  void* colpart = nullptr;
  int32_t *a = nullptr, *b = nullptr;
  float *da = nullptr, *db = nullptr;
  npg_status st = NPG_OK;
  auto alloc = [&](void** p, size_t bytes) {
    if (st == NPG_OK && hipMalloc(p, bytes) != hipSuccess) st = npg_fail(NPG_ENOMEM, "metrics workspace allocation failed");
  };
  alloc((void**)&off, (T + 1) * sizeof(int64_t));
  alloc((void**)&pt_frame, n * sizeof(int));
  alloc(&colpart, (size_t)T * P->nvb * V * sizeof(unsigned long long));
  alloc((void**)&a, n * sizeof(int32_t));
  alloc((void**)&b, n * sizeof(int32_t));
  alloc((void**)&da, n * sizeof(float));
  alloc((void**)&db, n * sizeof(float));
  if (st == NPG_OK) {
    hipLaunchKernelGGL(k_frame_index, dim3(nblk(n + 1, 256)), dim3(256), 0, P->stream, V, (int)T, off, pt_frame);
    hipError_t e = npg_launch_nn(P, xhat, gt, off, pt_frame, n, V, colpart, a, da, b, db);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_metrics, dim3((unsigned)T), dim3(kB), 0, P->stream, xhat, nhat, gt, gtn, a, da, b, db, V,
                         tau * tau, out);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) st = npg_fail(NPG_EHIP, std::string("metrics: ") + hipGetErrorString(e));
  } else {
    hipStreamSynchronize(P->stream);
  }
  hipFree(off);
  hipFree(pt_frame);
  hipFree(colpart);
  hipFree(a);
  hipFree(b);
  hipFree(da);
  hipFree(db);
  return st;
}
