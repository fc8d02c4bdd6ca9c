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
#include <mutex>

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

// Fixed workspace of npg_metrics_noalloc: one copy per GPU, created when the
// library's code object is loaded on that GPU and held until the process
// ends. In host code `scratch` names a host-side stand-in; kernels receive
// the device address found by hipGetSymbolAddress (npg_scratch_setup).
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
unsigned char* g_scratch_addr[kMaxDevices] = {};

inline size_t a256(size_t n) { return (n + 255) & ~(size_t)255; }

// Workspace of nT frames: frame offsets, frame of every true vertex, column
// records, both directions' indices and distances (256-byte aligned parts).
size_t metrics_bytes(const npg_plan* P, int64_t nT) {
  const int64_t n = nT * P->V;
  return a256((size_t)(nT + 1) * 8) + a256((size_t)n * 4) + a256((size_t)nT * P->nvb * P->V * 8) +
         4 * a256((size_t)n * 4);
}

}  // namespace

npg_status npg_scratch_setup(npg_plan* P) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (P->device < 0 || P->device >= kMaxDevices) return npg_fail(NPG_EINVAL, "device ordinal beyond 63");
  if (!g_scratch_addr[P->device]) {
    void* ptr = nullptr;
    NPG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));  // with the plan's device current
    g_scratch_addr[P->device] = static_cast<unsigned char*>(ptr);
  }
  P->scratch = g_scratch_addr[P->device];
  return NPG_OK;
}

// The metrics of npg_run_metrics with their workspace in the fixed array:
// frames are processed in chunks that fit it, one chunk after the other on the
// plan's stream (frames are independent, so results are bitwise those of
// npg_run_metrics). Every workspace entry a kernel reads was written earlier
// in the same chunk, so nothing needs clearing. No allocation, no
// synchronisation.
npg_status npg_run_metrics_noalloc(npg_plan* P, const float4* xhat, const float4* nhat, const float4* gt,
                                   const float4* gtn, float tau, double* out) {
  if (!P->scratch) return npg_fail(NPG_EHIP, "the scratch array has no device address on this GPU");
  const int64_t V = P->V, T = P->T;
  if (metrics_bytes(P, 1) > kScratchBytes)
    return npg_fail(NPG_EINVAL, "one frame's metrics workspace (" + std::to_string(metrics_bytes(P, 1)) +
                                    " bytes) exceeds the fixed scratch array (" + std::to_string(kScratchBytes) +
                                    " bytes)");
  // the most frames whose workspace fits (the size grows with the frame count)
  int64_t lo = 1, hi = T;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (metrics_bytes(P, mid) <= kScratchBytes) lo = mid;
    else hi = mid - 1;
  }
  const int64_t nT = lo;
  for (int64_t t0 = 0; t0 < T; t0 += nT) {
    const int64_t nt = std::min(nT, T - t0), n = nt * V;
    unsigned char* w = P->scratch;
    int64_t* off = reinterpret_cast<int64_t*>(w);
    w += a256((size_t)(nt + 1) * 8);
    int* pt_frame = reinterpret_cast<int*>(w);
    w += a256((size_t)n * 4);
    void* colpart = w;
    w += a256((size_t)nt * P->nvb * V * 8);
    int32_t* a = reinterpret_cast<int32_t*>(w);
    w += a256((size_t)n * 4);
    int32_t* b = reinterpret_cast<int32_t*>(w);
    w += a256((size_t)n * 4);
    float* da = reinterpret_cast<float*>(w);
    w += a256((size_t)n * 4);
    float* db = reinterpret_cast<float*>(w);
    const int64_t e0 = t0 * V;
    hipLaunchKernelGGL(k_frame_index, dim3(nblk(n + 1, 256)), dim3(256), 0, P->stream, V, (int)nt, off, pt_frame);
    NPG_HIP(npg_launch_nn(P, xhat + e0, gt + e0, off, pt_frame, n, V, colpart, a, da, b, db, (int)nt));
    hipLaunchKernelGGL(k_metrics, dim3((unsigned)nt), dim3(kB), 0, P->stream, xhat + e0, nhat + e0, gt + e0,
                       gtn + e0, a, da, b, db, V, tau * tau, out + 4 * t0);
    NPG_HIP(hipGetLastError());
  }
  return NPG_OK;
}

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
