// Bidirectional nearest-neighbour Chamfer distance per frame, the confidence
// weighted deformation loss (Sec. 3.5), and the loss gradient w.r.t. the
// deformed vertices.
//
// Distances are float32 in the direct form (x-p).(x-p) with one fixed
// operation order (dist2 below), used everywhere a distance is compared, so
// the argmin recovered in a second pass is the one the first pass saw.
// Ties resolve to the lowest index in both directions.
//
// Main pass, per (frame, block of KT*kK vertices): each thread keeps kK
// vertices in registers and streams the frame's points through LDS tiles, two
// points per iteration. The inner loop tracks values only (min3 updates): the
// running row minimum per vertex and, per point, the minimum over the
// thread's vertices. That column value is reduced across the wave with DPP,
// the lowest lane attaining it is found with a ballot, and an LDS 64-bit
// atomic min over (distance bits, first vertex of that lane) combines the
// waves (exact and order independent). The best tile of each vertex is
// re-scanned afterwards to recover its lowest row index; a second pass takes
// the smallest column record over vertex blocks and re-scans its kK
// vertices.
#include "internal.h"

namespace {

constexpr int kK = 16;     // vertices per thread
constexpr int kPT = 256;   // points per LDS tile
// work-group size KT of the main pass: 64, 128 (default) or 256 threads, the
// plan's choice (npg_tune_nn); results do not depend on it

__device__ __forceinline__ float dist2(float4 x, float4 p) {
  float dx = x.x - p.x, dy = x.y - p.y, dz = x.z - p.z;
  return __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmul_rn(dx, dx)));
}

__device__ __forceinline__ float min3f(float a, float b, float c) { return fminf(fminf(a, b), c); }

// Minimum over the 64 lanes with DPP moves; lane 63 ends with the result.
// Distances are non-negative finite floats (+0 included, never -0), whose
// bit patterns order like unsigned integers, so the reduction runs on the
// bits (an integer minimum folds into the DPP move; identity 0xffffffff).
// Within rows of 16: quad xor 1, quad xor 2, half-row mirror, row mirror;
// then row 15 -> rows 1, 3 and row 31 -> rows 2, 3 broadcasts.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t umin_dpp(uint32_t v) {
  return min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0xffffffffu, (int)v, CTRL, ROWS, 0xF, false));
}
// two independent reductions stage by stage (no wait between dependent DPP steps)
__device__ __forceinline__ void wave_min2_to_lane63(uint32_t& a, uint32_t& b) {
  a = umin_dpp<0xB1, 0xF>(a);
  b = umin_dpp<0xB1, 0xF>(b);
  a = umin_dpp<0x4E, 0xF>(a);
  b = umin_dpp<0x4E, 0xF>(b);
  a = umin_dpp<0x141, 0xF>(a);
  b = umin_dpp<0x141, 0xF>(b);
  a = umin_dpp<0x140, 0xF>(a);
  b = umin_dpp<0x140, 0xF>(b);
  a = umin_dpp<0x142, 0xA>(a);
  b = umin_dpp<0x142, 0xA>(b);
  a = umin_dpp<0x143, 0xC>(a);
  b = umin_dpp<0x143, 0xC>(b);
}

// Column records of two points (the second only when has1): per point
// (distance bits << 32) | first vertex of the lowest lane attaining the wave
// minimum; an LDS 64-bit atomic min keeps the smallest distance and, among
// equal ones, the lowest vertex range.
__device__ __forceinline__ void column_record2(float m0, float m1, unsigned long long* slot, bool has1,
                                               uint32_t lane_v0) {
  const uint32_t b0 = __float_as_uint(m0), b1 = __float_as_uint(m1);
  uint32_t r0 = b0, r1 = b1;
  wave_min2_to_lane63(r0, r1);
  const uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane((int)r0, 63);
  const uint32_t w1 = (uint32_t)__builtin_amdgcn_readlane((int)r1, 63);
  const int lane = (int)(threadIdx.x & 63);
  const int f0 = __builtin_ctzll(__ballot(b0 == w0));
  const int f1 = __builtin_ctzll(__ballot(b1 == w1));
  if (lane == f0) atomicMin(slot, ((unsigned long long)w0 << 32) | (unsigned long long)lane_v0);
  if (has1 && lane == f1) atomicMin(slot + 1, ((unsigned long long)w1 << 32) | (unsigned long long)lane_v0);
}

// Vertices of a lane are contiguous: thread th of block vb owns
// vb*KT*kK + th*kK + k, k < kK, so the lowest lane attaining a column minimum
// holds the lowest vertex index attaining it.
template <int KT>
__global__ __launch_bounds__(KT) void k_chamfer_main(const float4* __restrict__ xhat, const float4* __restrict__ pts,
                                                     const int64_t* __restrict__ off, int64_t V, int nvb,
                                                     int64_t Nmax, int32_t* __restrict__ a, float* __restrict__ da,
                                                     unsigned long long* __restrict__ colpart) {
  __shared__ float4 sp[kPT + 2];
  __shared__ unsigned long long cm[kPT];
  const int t = blockIdx.y, vb = blockIdx.x;
  const int64_t p0 = off[t];
  const int Nt = (int)(off[t + 1] - p0);
  const int64_t vbase = (int64_t)vb * (KT * kK) + (int64_t)threadIdx.x * kK;
  float4 x[kK];
  float best[kK];
  int btile[kK];
#pragma unroll
  for (int k = 0; k < kK; ++k) {
    const int64_t i = vbase + k;
    x[k] = i < V ? xhat[(int64_t)t * V + i] : make_float4(1e18f, 1e18f, 1e18f, 0.f);
    best[k] = INFINITY;
    btile[k] = 0;
  }
  const uint32_t lane_v0 = (uint32_t)vbase;
  const int ntile = (Nt + kPT - 1) / kPT;
  for (int tile = 0; tile < ntile; ++tile) {
    const int cnt = min(kPT, Nt - tile * kPT);
    for (int j = threadIdx.x; j < kPT + 2; j += KT) {
      // padding points sit far away: they never win a row minimum
      sp[j] = j < cnt ? pts[p0 + (int64_t)tile * kPT + j] : make_float4(3e18f, 3e18f, 3e18f, 0.f);
      if (j < kPT) cm[j] = ~0ull;
    }
    __syncthreads();
    float tmin[kK];
#pragma unroll
    for (int k = 0; k < kK; ++k) tmin[k] = INFINITY;
    for (int j = 0; j < cnt; j += 2) {
      const float4 q0 = sp[j], q1 = sp[j + 1];
      float m0 = INFINITY, m1 = INFINITY;
#pragma unroll
      for (int k = 0; k < kK; k += 2) {
        const float d00 = dist2(x[k], q0), d01 = dist2(x[k], q1);
        const float d10 = dist2(x[k + 1], q0), d11 = dist2(x[k + 1], q1);
        tmin[k] = min3f(tmin[k], d00, d01);
        tmin[k + 1] = min3f(tmin[k + 1], d10, d11);
        m0 = min3f(m0, d00, d10);
        m1 = min3f(m1, d01, d11);
      }
      column_record2(m0, m1, &cm[j], j + 1 < cnt, lane_v0);
    }
#pragma unroll
    for (int k = 0; k < kK; ++k)
      if (tmin[k] < best[k]) {
        best[k] = tmin[k];
        btile[k] = tile;
      }
    __syncthreads();
    unsigned long long* dst = colpart + ((int64_t)t * nvb + vb) * Nmax + (int64_t)tile * kPT;
    for (int j = threadIdx.x; j < cnt; j += KT) dst[j] = cm[j];
    __syncthreads();
  }
  // recover the lowest index attaining the row minimum inside its best tile
#pragma unroll
  for (int k = 0; k < kK; ++k) {
    const int64_t i = vbase + k;
    if (i >= V) continue;
    const int j0 = btile[k] * kPT;
    const int cnt = min(kPT, Nt - j0);
    int arg = j0;
    for (int j = 0; j < cnt; ++j)
      if (dist2(x[k], pts[p0 + j0 + j]) == best[k]) {
        arg = j0 + j;
        break;
      }
    a[(int64_t)t * V + i] = arg;
    da[(int64_t)t * V + i] = best[k];
  }
}

// One thread per point: the smallest record over the vertex blocks names the
// lowest lane range attaining the minimum; its kK vertices are re-scanned.
__global__ void k_chamfer_cols(const float4* __restrict__ xhat, const float4* __restrict__ pts,
                               const int64_t* __restrict__ off, const int* __restrict__ pt_frame, int64_t Ntot,
                               int64_t V, int nvb, int64_t Nmax, const unsigned long long* __restrict__ colpart,
                               int32_t* __restrict__ b, float* __restrict__ db) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= Ntot) return;
  const int t = pt_frame[g];
  const int64_t j = g - off[t];
  unsigned long long m = ~0ull;
  for (int vb = 0; vb < nvb; ++vb) {
    const unsigned long long u = colpart[((int64_t)t * nvb + vb) * Nmax + j];
    m = u < m ? u : m;
  }
  const float dm = __uint_as_float((uint32_t)(m >> 32));
  const int64_t i0 = (int64_t)(uint32_t)(m & 0xffffffffu);
  const float4 p = pts[g];
  int64_t arg = i0;
  for (int k = 0; k < kK && i0 + k < V; ++k)
    if (dist2(xhat[(int64_t)t * V + i0 + k], p) == dm) {
      arg = i0 + k;
      break;
    }
  // only reachable with non-finite vertices (flagged by the step): keep the
  // index inside [0, V) so no later pass can address past the vertex arrays
  if (arg >= V) arg = V - 1;
  b[g] = (int32_t)arg;
  db[g] = dm;
}

// cd_t = mean_i da + mean_j db in float64, fixed-order block reduction.
__global__ void k_frame_sums(const float* __restrict__ da, const float* __restrict__ db,
                             const int64_t* __restrict__ off, int64_t V, double* __restrict__ cd) {
  __shared__ double red[2][256];
  const int t = blockIdx.x;
  double sa = 0.0, sb = 0.0;
  for (int64_t i = threadIdx.x; i < V; i += 256) sa += (double)da[(int64_t)t * V + i];
  const int64_t p0 = off[t], p1 = off[t + 1];
  for (int64_t j = p0 + threadIdx.x; j < p1; j += 256) sb += (double)db[j];
  red[0][threadIdx.x] = sa;
  red[1][threadIdx.x] = sb;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      red[0][threadIdx.x] += red[0][threadIdx.x + st];
      red[1][threadIdx.x] += red[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) cd[t] = red[0][0] / (double)V + red[1][0] / (double)(p1 - p0);
}

// Sec. 3.5: omega(tau) = 1/(1 + max(0, cd_tau - cd_key)), w_t = product of
// omega^delta over the frames between t_key and t (inclusive), delta =
// 1 - sqrt(e/e_max); L_def = (1/T) sum_t w_t cd_t.
__global__ void k_loss(const double* __restrict__ cd, int T, int t_key, int conf, double delta,
                       const NpgStepScal* __restrict__ sc, double* __restrict__ w, double* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (sc) delta = sc->delta;
  const double ck = cd[t_key];
  if (!conf) {
    for (int t = 0; t < T; ++t) w[t] = 1.0;
  } else {
    w[t_key] = 1.0;
    double run = 1.0;
    for (int t = t_key + 1; t < T; ++t) {
      run *= pow(1.0 / (1.0 + fmax(0.0, cd[t] - ck)), delta);
      w[t] = run;
    }
    run = 1.0;
    for (int t = t_key - 1; t >= 0; --t) {
      run *= pow(1.0 / (1.0 + fmax(0.0, cd[t] - ck)), delta);
      w[t] = run;
    }
  }
  double s = 0.0;
  for (int t = 0; t < T; ++t) s += w[t] * cd[t];
  loss[0] = s / (double)T;
}

__global__ void k_zero_ll(long long* __restrict__ p, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Point -> its nearest vertex: accumulate x^_b - p in 2^-32 fixed point with
// 64-bit integer atomics (exact, hence order independent).
__global__ void k_chamfer_bwd_points(const float4* __restrict__ xhat, const float4* __restrict__ pts,
                                     const int* __restrict__ pt_frame, const int32_t* __restrict__ b, int64_t Ntot,
                                     int64_t V, long long* __restrict__ acc, int* __restrict__ flag) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= Ntot) return;
  const int t = pt_frame[g];
  const int64_t i = b[g];
  const float4 x = xhat[(int64_t)t * V + i];
  const float4 p = pts[g];
  float d[3] = {x.x - p.x, x.y - p.y, x.z - p.z};
  long long* dst = acc + ((int64_t)t * V + i) * 3;
  for (int k = 0; k < 3; ++k) {
    double v = (double)d[k] * 4294967296.0;
    if (!(fabs(v) < 9.0e15)) {
      atomicOr(flag, 1);
      v = 0.0;
    }
    atomicAdd(reinterpret_cast<unsigned long long*>(dst + k), (unsigned long long)__double2ll_rn(v));
  }
}

__global__ void k_chamfer_bwd_verts(const float4* __restrict__ xhat, const float4* __restrict__ pts,
                                    const int64_t* __restrict__ off, const int32_t* __restrict__ a,
                                    const double* __restrict__ w, const long long* __restrict__ acc, int64_t V,
                                    int T, float4* __restrict__ gx) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)T * V) return;
  const int t = (int)(e / V);
  const float4 x = xhat[e];
  const float4 p = pts[off[t] + a[e]];
  const float s = (float)(w[t] / (double)T);
  const float cv = 2.0f / (float)V;
  const float cn = (float)(2.0 / (double)(off[t + 1] - off[t]));
  const long long* ac = acc + e * 3;
  const float inv = 1.0f / 4294967296.0f;
  float4 r;
  r.x = s * (cv * (x.x - p.x) + cn * ((float)ac[0] * inv));
  r.y = s * (cv * (x.y - p.y) + cn * ((float)ac[1] * inv));
  r.z = s * (cv * (x.z - p.z) + cn * ((float)ac[2] * inv));
  r.w = 0.f;
  gx[e] = r;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int npg_chamfer_vblock(int threads) { return threads * kK; }

// Both nearest-neighbour directions between the plan's per-frame vertices and
// any per-frame point set (frame t owns points off[t] .. off[t+1]-1, at most
// Nmax; colpart holds T * nvb * Nmax 64-bit column records).
hipError_t npg_launch_nn(const npg_plan* P, const float4* xhat, const float4* pts, const int64_t* off,
                         const int* pt_frame, int64_t Ntot, int64_t Nmax, void* colpart, int32_t* a, float* da,
                         int32_t* b, float* db, int nT) {
  unsigned long long* cp = reinterpret_cast<unsigned long long*>(colpart);
  const unsigned frames = (unsigned)(nT > 0 ? nT : P->T);
  switch (P->nn_threads) {
    case 64:
      hipLaunchKernelGGL(k_chamfer_main<64>, dim3(P->nvb, frames), dim3(64), 0, P->stream, xhat, pts, off, P->V,
                         P->nvb, Nmax, a, da, cp);
      break;
    case 256:
      hipLaunchKernelGGL(k_chamfer_main<256>, dim3(P->nvb, frames), dim3(256), 0, P->stream, xhat, pts, off, P->V,
                         P->nvb, Nmax, a, da, cp);
      break;
    default:
      hipLaunchKernelGGL(k_chamfer_main<128>, dim3(P->nvb, frames), dim3(128), 0, P->stream, xhat, pts, off, P->V,
                         P->nvb, Nmax, a, da, cp);
  }
  hipLaunchKernelGGL(k_chamfer_cols, dim3(nblk(Ntot, 256)), dim3(256), 0, P->stream, xhat, pts, off, pt_frame, Ntot,
                     P->V, P->nvb, Nmax, reinterpret_cast<const unsigned long long*>(colpart), b, db);
  return hipGetLastError();
}

// Both directions for the plan's own points, by the search the config names.
hipError_t npg_launch_nn_step(const npg_plan* P, const float4* xhat, int32_t* a, float* da, int32_t* b, float* db) {
  if (P->cfg.nn_search == NPG_NN_PRUNED && P->nn) return npg_launch_nn_pruned(P, xhat, a, da, b, db);
  return npg_launch_nn(P, xhat, P->pts, P->d_off, P->pt_frame, P->Ntot, P->Nmax, P->colpart, a, da, b, db);
}

hipError_t npg_launch_chamfer_fwd(const npg_plan* P, const float4* xhat, int32_t* a, float* da, int32_t* b,
                                  float* db, double* cd) {
  hipError_t e = npg_launch_nn_step(P, xhat, a, da, b, db);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_frame_sums, dim3(P->T), dim3(256), 0, P->stream, da, db, P->d_off, P->V, cd);
  return hipGetLastError();
}

double npg_loss_delta(int epoch, int n_epochs) { return 1.0 - sqrt((double)epoch / (double)n_epochs); }

hipError_t npg_launch_loss(const npg_plan* P, const double* cd, int epoch, int n_epochs, double* w,
                           double* loss, const NpgStepScal* sc) {
  const double delta = npg_loss_delta(epoch, n_epochs);
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(64), 0, P->stream, cd, P->T, P->t_key, P->cfg.conf_weight, delta, sc,
                     w, loss);
  return hipGetLastError();
}

hipError_t npg_launch_chamfer_bwd(const npg_plan* P, const float4* xhat, const int32_t* a, const int32_t* b,
                                  const double* w, float4* gxhat) {
  const int64_t n = (int64_t)P->T * P->V;
  hipLaunchKernelGGL(k_zero_ll, dim3(nblk(3 * n, 256)), dim3(256), 0, P->stream, P->acc, 3 * n);
  hipLaunchKernelGGL(k_chamfer_bwd_points, dim3(nblk(P->Ntot, 256)), dim3(256), 0, P->stream, xhat, P->pts,
                     P->pt_frame, b, P->Ntot, P->V, P->acc, P->d_flag);
  hipLaunchKernelGGL(k_chamfer_bwd_verts, dim3(nblk(n, 256)), dim3(256), 0, P->stream, xhat, P->pts, P->d_off, a,
                     w, P->acc, P->V, P->T, gxhat);
  return hipGetLastError();
}
