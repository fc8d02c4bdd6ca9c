// Sobolev preconditioning of the grid gradients (Sec. 3.5): g~ = (I+lam L)^-2 g
// per grid and feature channel, L the 6-neighbour lattice Laplacian with free
// boundary, as two conjugate-gradient solves from a zero start.
//
// All grids (every position level and the normal grid) iterate together:
// each launch covers the blocks of every system still active, through a
// block -> (system, first node) table. Vectors are float32 in the parameter
// layout ([node][F] per grid); inner products are float64, reduced per wave
// and then per system in a fixed order (bitwise reproducible).
//
// One CG iteration is two streaming kernels:
//   k_cg_dir_ap:  p = r + beta p, and p.(A p) with A p formed on the fly from
//                 r and the old p at the 6 neighbours (p is written, A p is not)
//   k_cg_update:  x += alpha p, r -= alpha A p (A p recomputed from p),
//                 and r.r
// i.e. 8 vector passes (r, p, p | p, x, r, x, r) instead of storing A p.
// A p = p + lam * sum over existing neighbours of (p_n - p_nb): sums of
// differences keep the float32 rounding proportional to |A p|, not to
// (1 + 12 lam)|p|.
//
// Work-groups are mapped XCD-aware: consecutive work-group ids go round-robin
// to the 8 XCDs, so the logical chunk of id b is (b % 8) * per_xcd + b / 8
// and each XCD streams one contiguous slab of nodes; the +-R^2 neighbour
// planes are then read from the same XCD's L2.
#include "internal.h"

namespace {

constexpr int kB = 256;       // threads per work-group
constexpr int kPer = 8;       // nodes per thread
constexpr int kChunk = kB * kPer;
constexpr int kXcd = 8;

// per (system, channel) scalars: 0 rr, 1 bb, 2 pq, 3 alpha, 4 beta, 5 active, 6 iterations
constexpr int kS = 8;

// Loads/stores of one node's F channels: vector instructions when the grid's
// offset keeps every node 4F-byte aligned (always for F = 1 and 3, which use
// scalars), otherwise scalar fallbacks (FF = -F below).
template <int F>
struct Vec {
  static constexpr int N = F < 0 ? -F : F;
  static __device__ __forceinline__ void load(const float* p, float (&v)[N]) {
#pragma unroll
    for (int c = 0; c < N; ++c) v[c] = p[c];
  }
  static __device__ __forceinline__ void store(float* p, const float (&v)[N]) {
#pragma unroll
    for (int c = 0; c < N; ++c) p[c] = v[c];
  }
};
template <>
struct Vec<4> {
  static __device__ __forceinline__ void load(const float* p, float (&v)[4]) {
    float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  }
  static __device__ __forceinline__ void store(float* p, const float (&v)[4]) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  }
};
template <>
struct Vec<2> {
  static __device__ __forceinline__ void load(const float* p, float (&v)[2]) {
    float2 t = *reinterpret_cast<const float2*>(p);
    v[0] = t.x; v[1] = t.y;
  }
  static __device__ __forceinline__ void store(float* p, const float (&v)[2]) {
    *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
  }
};
template <>
struct Vec<1> {
  static __device__ __forceinline__ void load(const float* p, float (&v)[1]) { v[0] = p[0]; }
  static __device__ __forceinline__ void store(float* p, const float (&v)[1]) { p[0] = v[0]; }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Logical work-group of this launch (XCD-aware), or -1 past the end.
__device__ __forceinline__ int logical_block(int nb) {
  const int per = (nb + kXcd - 1) / kXcd;
  const int lb = (int)(blockIdx.x % kXcd) * per + (int)(blockIdx.x / kXcd);
  return lb < nb ? lb : -1;
}

// Block partials of F channels, part[blk*4 + c]: wave sums, then the 4
// waves in order.
template <int F>
__device__ __forceinline__ void store_partials(double (&acc)[4], double* part, int blk) {
  __shared__ double ws[4][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < F; ++c) {
    double s = wave_sum(acc[c]);
    if (lane == 0) ws[wave][c] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < F) {
    const int c = threadIdx.x;
    part[(int64_t)blk * 4 + c] = ((ws[0][c] + ws[1][c]) + ws[2][c]) + ws[3][c];
  }
}

// Division of a node index n < 2^31 by the lattice size, as a multiply-high
// with a per-divisor magic number (Granlund-Montgomery round-up method):
// q = (umulhi(n, m) + n) >> s with s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1.
struct FastDiv {
  uint32_t m;
  int s;
  uint32_t d;
};
inline FastDiv make_fastdiv(uint32_t d) {
  int s = 0;
  while ((1ull << s) < d) ++s;
  const uint64_t m = ((1ull << 32) * ((1ull << s) - d)) / d + 1;
  return FastDiv{(uint32_t)m, s, d};
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) { return (__umulhi(n, f.m) + n) >> f.s; }

struct Nb {
  int o[6];
  int mask;
};
// Neighbour offsets of node n and a mask of the neighbours that exist.
__device__ __forceinline__ Nb neighbours(uint32_t n, int R, const FastDiv& fR, const FastDiv& fR2) {
  const uint32_t iz = fdiv(n, fR2);
  const uint32_t rem = n - iz * fR2.d;
  const uint32_t iy = fdiv(rem, fR);
  const uint32_t ix = rem - iy * (uint32_t)R;
  const int R2 = (int)fR2.d;
  Nb b;
  b.o[0] = -1; b.o[1] = 1; b.o[2] = -R; b.o[3] = R; b.o[4] = -R2; b.o[5] = R2;
  b.mask = (ix > 0) | ((ix < (uint32_t)R - 1) << 1) | ((iy > 0) << 2) | ((iy < (uint32_t)R - 1) << 3) |
           ((iz > 0) << 4) | ((iz < (uint32_t)R - 1) << 5);
  return b;
}

template <int FV, int F = (FV < 0 ? -FV : FV)>
__device__ void init_body(const NpgGrid& g, int64_t n0, const float* b, float* x, float* r, float* p, double* part,
                          int blk) {
  double acc[4] = {0, 0, 0, 0};
  for (int k = 0; k < kPer; ++k) {
    const int64_t n = n0 + k * kB + threadIdx.x;
    if (n >= g.nodes) break;
    const int64_t e = g.poff + n * F;
    float v[F], z[F];
    Vec<FV>::load(b + e, v);
#pragma unroll
    for (int c = 0; c < F; ++c) {
      z[c] = 0.f;
      acc[c] += (double)v[c] * (double)v[c];
    }
    Vec<FV>::store(x + e, z);
    Vec<FV>::store(r + e, v);
    Vec<FV>::store(p + e, v);
  }
  store_partials<F>(acc, part, blk);
}

// p_new = r + beta p_old; pq partial with A p_new formed from r and p_old at
// the neighbours. p_old and p_new are different buffers (ping-pong), so no
// work-group ever reads a value another one has already overwritten.
template <int FV, int F = (FV < 0 ? -FV : FV)>
__device__ void dir_ap_body(const NpgGrid& g, const FastDiv& fR, const FastDiv& fR2, int64_t n0, const double* st,
                            int s, const float* r, const float* p_old, float* p_new, double* part, int blk) {
  float be[F];
#pragma unroll
  for (int c = 0; c < F; ++c) be[c] = (float)st[(s * 4 + c) * kS + 4];
  const float lam = g.lam;
  const float* rb = r + g.poff;
  const float* pb = p_old + g.poff;
  float* qb = p_new + g.poff;
  double acc[4] = {0, 0, 0, 0};
  for (int k = 0; k < kPer; ++k) {
    const int64_t n = n0 + k * kB + threadIdx.x;
    if (n >= g.nodes) break;
    const Nb nb = neighbours((uint32_t)n, g.R, fR, fR2);
    float rc[F], pc[F], pn[F], lap[F];
    Vec<FV>::load(rb + n * F, rc);
    Vec<FV>::load(pb + n * F, pc);
#pragma unroll
    for (int c = 0; c < F; ++c) {
      pn[c] = fmaf(be[c], pc[c], rc[c]);
      lap[c] = 0.f;
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (nb.mask & (1 << d)) {
        const int64_t m = n + nb.o[d];
        float rm[F], pm[F];
        Vec<FV>::load(rb + m * F, rm);
        Vec<FV>::load(pb + m * F, pm);
#pragma unroll
        for (int c = 0; c < F; ++c) lap[c] += pn[c] - fmaf(be[c], pm[c], rm[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < F; ++c) acc[c] += (double)pn[c] * (double)fmaf(lam, lap[c], pn[c]);
    Vec<FV>::store(qb + n * F, pn);
  }
  store_partials<F>(acc, part, blk);
}

// x += alpha p, r -= alpha A p; rr partial.
template <int FV, int F = (FV < 0 ? -FV : FV)>
__device__ void update_body(const NpgGrid& g, const FastDiv& fR, const FastDiv& fR2, int64_t n0, const double* st,
                            int s, float* x, float* r, const float* p, double* part, int blk) {
  float al[F];
#pragma unroll
  for (int c = 0; c < F; ++c) al[c] = (float)st[(s * 4 + c) * kS + 3];
  const float lam = g.lam;
  const float* pb = p + g.poff;
  double acc[4] = {0, 0, 0, 0};
  for (int k = 0; k < kPer; ++k) {
    const int64_t n = n0 + k * kB + threadIdx.x;
    if (n >= g.nodes) break;
    const Nb nb = neighbours((uint32_t)n, g.R, fR, fR2);
    const int64_t e = g.poff + n * F;
    float pc[F], lap[F], xc[F], rc[F];
    Vec<FV>::load(pb + n * F, pc);
#pragma unroll
    for (int c = 0; c < F; ++c) lap[c] = 0.f;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (nb.mask & (1 << d)) {
        float pm[F];
        Vec<FV>::load(pb + (n + nb.o[d]) * F, pm);
#pragma unroll
        for (int c = 0; c < F; ++c) lap[c] += pc[c] - pm[c];
      }
    }
    Vec<FV>::load(x + e, xc);
    Vec<FV>::load(r + e, rc);
#pragma unroll
    for (int c = 0; c < F; ++c) {
      xc[c] = fmaf(al[c], pc[c], xc[c]);
      rc[c] = fmaf(-al[c], fmaf(lam, lap[c], pc[c]), rc[c]);
      acc[c] += (double)rc[c] * (double)rc[c];
    }
    Vec<FV>::store(x + e, xc);
    Vec<FV>::store(r + e, rc);
  }
  store_partials<F>(acc, part, blk);
}

#define NPG_F_SWITCH(g, CALL)                                               \
  switch ((g).F * 2 + (int)(((g).poff % (g).F) == 0)) {                     \
    case 9: { constexpr int FF = 4; CALL; } break;                          \
    case 8: { constexpr int FF = -4; CALL; } break;                         \
    case 5: { constexpr int FF = 2; CALL; } break;                          \
    case 4: { constexpr int FF = -2; CALL; } break;                         \
    case 7: case 6: { constexpr int FF = -3; CALL; } break;                 \
    default: { constexpr int FF = 1; CALL; } break;                         \
  }

// b may alias x (second solve): no __restrict__ on either.
__global__ __launch_bounds__(kB) void k_cg_init(const NpgGrid* __restrict__ G, int nb, const int* __restrict__ blk_sys,
                                                const int64_t* __restrict__ blk_start, const float* b, float* x,
                                                float* __restrict__ r, float* __restrict__ p,
                                                double* __restrict__ part) {
  const int blk = logical_block(nb);
  if (blk < 0) return;
  const int s = blk_sys[blk];
  const NpgGrid g = G[s];
  NPG_F_SWITCH(g, (init_body<FF>(g, blk_start[blk], b, x, r, p, part, blk)));
}

struct Divs {
  FastDiv r[NPG_MAX_SYS], r2[NPG_MAX_SYS];
};

__global__ __launch_bounds__(kB) void k_cg_dir_ap(const NpgGrid* __restrict__ G, Divs dv, int nb, const int* __restrict__ blk_sys,
                                                  const int64_t* __restrict__ blk_start,
                                                  const int* __restrict__ active, const double* __restrict__ st,
                                                  const float* __restrict__ r, const float* __restrict__ p_old,
                                                  float* __restrict__ p_new, double* __restrict__ part) {
  const int blk = logical_block(nb);
  if (blk < 0) return;
  const int s = blk_sys[blk];
  if (!active[s]) return;
  const NpgGrid g = G[s];
  NPG_F_SWITCH(g, (dir_ap_body<FF>(g, dv.r[s], dv.r2[s], blk_start[blk], st, s, r, p_old, p_new, part, blk)));
}

__global__ __launch_bounds__(kB) void k_cg_update(const NpgGrid* __restrict__ G, Divs dv, int nb, const int* __restrict__ blk_sys,
                                                  const int64_t* __restrict__ blk_start,
                                                  const int* __restrict__ active, const double* __restrict__ st,
                                                  float* __restrict__ x, float* __restrict__ r,
                                                  const float* __restrict__ p, double* __restrict__ part) {
  const int blk = logical_block(nb);
  if (blk < 0) return;
  const int s = blk_sys[blk];
  if (!active[s]) return;
  const NpgGrid g = G[s];
  NPG_F_SWITCH(g, (update_body<FF>(g, dv.r[s], dv.r2[s], blk_start[blk], st, s, x, r, p, part, blk)));
}

// Per system (one work-group each): reduce the block partials in order and
// update the scalars. mode 0: after init (rr, bb); 1: alpha = rr / pq;
// 2: beta = rr_new / rr and the convergence test.
constexpr int kR = 1024;
__global__ __launch_bounds__(kR) void k_cg_reduce(const NpgGrid* __restrict__ G, const int* __restrict__ sys_blk0,
                                                  int* __restrict__ active, const double* __restrict__ part,
                                                  double* __restrict__ st, int mode, double rtol) {
  const int s = blockIdx.x;
  if (mode != 0 && !active[s]) return;
  __shared__ double red[4][kR / 64];
  const int F = G[s].F;
  const int b0 = sys_blk0[s], b1 = sys_blk0[s + 1];
  double acc[4] = {0, 0, 0, 0};
  for (int b = b0 + threadIdx.x; b < b1; b += kR) {
    const double4 v = *reinterpret_cast<const double4*>(part + (int64_t)b * 4);
    acc[0] += v.x;
    acc[1] += v.y;
    acc[2] += v.z;
    acc[3] += v.w;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = 0; c < 4; ++c) {
    double v = wave_sum(acc[c]);
    if (lane == 0) red[c][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  int any = 0;
  for (int c = 0; c < F; ++c) {
    double v = 0.0;
    for (int w = 0; w < kR / 64; ++w) v += red[c][w];
    double* S = st + (s * 4 + c) * kS;
    if (mode == 0) {
      S[0] = v;
      S[1] = v;
      S[3] = 0.0;
      S[4] = 0.0;
      S[6] = 0.0;
      S[5] = v > 0.0 ? 1.0 : 0.0;
    } else if (mode == 1) {
      S[3] = (S[5] != 0.0 && v > 0.0) ? S[0] / v : 0.0;
    } else if (S[5] != 0.0) {
      S[4] = S[0] > 0.0 ? v / S[0] : 0.0;
      S[0] = v;
      S[6] += 1.0;
      if (!(sqrt(v) > rtol * sqrt(S[1]))) {
        S[5] = 0.0;
        S[3] = 0.0;
        S[4] = 0.0;
      }
    } else {
      S[3] = 0.0;
      S[4] = 0.0;
    }
    any |= S[5] != 0.0;
  }
  active[s] = any;
}

__global__ void k_copy(const float* __restrict__ src, float* __restrict__ dst, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
inline unsigned xcd_grid(int nb) { return (unsigned)(((nb + kXcd - 1) / kXcd) * kXcd); }

}  // namespace

npg_status npg_cg_setup(npg_plan* P) {
  NpgCG& C = P->cg;
  std::vector<int> bsys;
  std::vector<int64_t> bstart;
  std::vector<int> s0(P->n_sys + 1);
  for (int s = 0; s < P->n_sys; ++s) {
    s0[s] = (int)bsys.size();
    for (int64_t n = 0; n < P->g[s].nodes; n += kChunk) {
      bsys.push_back(s);
      bstart.push_back(n);
    }
  }
  s0[P->n_sys] = (int)bsys.size();
  C.n_blocks = (int)bsys.size();
  const int64_t n = P->n_grid_params;
  NPG_HIP(hipMalloc(&C.x, n * 4));
  NPG_HIP(hipMalloc(&C.r, n * 4));
  NPG_HIP(hipMalloc(&C.p, n * 4));
  NPG_HIP(hipMalloc(&C.q, n * 4));
  NPG_HIP(hipMalloc(&C.part, (int64_t)C.n_blocks * 4 * 8));
  NPG_HIP(hipMalloc(&C.st, (int64_t)P->n_sys * 4 * kS * 8));
  NPG_HIP(hipMalloc(&C.active, P->n_sys * 4));
  NPG_HIP(hipMalloc(&C.blk_sys, C.n_blocks * 4));
  NPG_HIP(hipMalloc(&C.blk_start, C.n_blocks * 8));
  NPG_HIP(hipMalloc(&C.sys_blk0, (P->n_sys + 1) * 4));
  NPG_HIP(hipMemcpy(C.blk_sys, bsys.data(), C.n_blocks * 4, hipMemcpyHostToDevice));
  NPG_HIP(hipMemcpy(C.blk_start, bstart.data(), C.n_blocks * 8, hipMemcpyHostToDevice));
  NPG_HIP(hipMemcpy(C.sys_blk0, s0.data(), (P->n_sys + 1) * 4, hipMemcpyHostToDevice));
  return NPG_OK;
}

void npg_cg_free(npg_plan* P) {
  NpgCG& C = P->cg;
  hipFree(C.x); hipFree(C.r); hipFree(C.p); hipFree(C.q); hipFree(C.part); hipFree(C.st);
  hipFree(C.active); hipFree(C.blk_sys); hipFree(C.blk_start); hipFree(C.sys_blk0);
}

// Solve (I + lam L) x = b for every system; the solution is left in C.x
// (b may alias C.x: each node of b is read before its x is cleared).
// The iteration count of each system goes to iters (if not NULL).
static npg_status cg_solve(npg_plan* P, const float* b, int32_t* iters, bool* capped) {
  NpgCG& C = P->cg;
  hipStream_t s = P->stream;
  const int nb = C.n_blocks;
  const dim3 grid(xcd_grid(nb)), blk(kB);
  Divs dv;
  for (int sy = 0; sy < P->n_sys; ++sy) {
    dv.r[sy] = make_fastdiv((uint32_t)P->g[sy].R);
    dv.r2[sy] = make_fastdiv((uint32_t)P->g[sy].R * (uint32_t)P->g[sy].R);
  }
  hipLaunchKernelGGL(k_cg_init, grid, blk, 0, s, P->d_g, nb, C.blk_sys, C.blk_start, b, C.x, C.r, C.p, C.part);
  hipLaunchKernelGGL(k_cg_reduce, dim3(P->n_sys), dim3(kR), 0, s, P->d_g, C.sys_blk0, C.active, C.part, C.st, 0,
                     P->cfg.cg_rtol);
  NPG_HIP(hipGetLastError());
  std::vector<int> act(P->n_sys);
  float* pa = C.p;  // current direction
  float* pb = C.q;  // next direction
  int it = 0;
  bool done = false;
  const int maxit = P->cfg.cg_maxit;
  while (it < maxit) {
    const int chunk = 16 < maxit - it ? 16 : maxit - it;
    for (int k = 0; k < chunk; ++k) {
      // optional profiling: event pairs around both streaming kernels,
      // resolved after the step (no synchronisation here)
      const bool prof = P->prof_cg && P->prof_n + 4 <= (int)P->prof_ev.size();
      if (prof) NPG_HIP(hipEventRecord(P->prof_ev[P->prof_n], s));
      hipLaunchKernelGGL(k_cg_dir_ap, grid, blk, 0, s, P->d_g, dv, nb, C.blk_sys, C.blk_start, C.active, C.st, C.r,
                         pa, pb, C.part);
      if (prof) NPG_HIP(hipEventRecord(P->prof_ev[P->prof_n + 1], s));
      std::swap(pa, pb);
      hipLaunchKernelGGL(k_cg_reduce, dim3(P->n_sys), dim3(kR), 0, s, P->d_g, C.sys_blk0, C.active, C.part, C.st, 1,
                         P->cfg.cg_rtol);
      if (prof) NPG_HIP(hipEventRecord(P->prof_ev[P->prof_n + 2], s));
      hipLaunchKernelGGL(k_cg_update, grid, blk, 0, s, P->d_g, dv, nb, C.blk_sys, C.blk_start, C.active, C.st, C.x,
                         C.r, pa, C.part);
      if (prof) {
        NPG_HIP(hipEventRecord(P->prof_ev[P->prof_n + 3], s));
        P->prof_n += 4;
      }
      hipLaunchKernelGGL(k_cg_reduce, dim3(P->n_sys), dim3(kR), 0, s, P->d_g, C.sys_blk0, C.active, C.part, C.st, 2,
                         P->cfg.cg_rtol);
    }
    NPG_HIP(hipGetLastError());
    it += chunk;
    NPG_HIP(hipMemcpyAsync(act.data(), C.active, P->n_sys * 4, hipMemcpyDeviceToHost, s));
    NPG_HIP(hipStreamSynchronize(s));
    done = true;
    for (int v : act) done &= (v == 0);
    if (done) break;
  }
  if (!done) *capped = true;
  std::vector<double> stv((size_t)P->n_sys * 4 * kS);
  NPG_HIP(hipMemcpyAsync(stv.data(), C.st, stv.size() * 8, hipMemcpyDeviceToHost, s));
  NPG_HIP(hipStreamSynchronize(s));
  for (int sy = 0; sy < P->n_sys; ++sy) {
    double m = 0;
    for (int c = 0; c < P->g[sy].F; ++c) m = stv[(sy * 4 + c) * kS + 6] > m ? stv[(sy * 4 + c) * kS + 6] : m;
    if (iters) iters[sy] = (int32_t)m;
    // algorithmic traffic of this solve: 6 vector passes (x, r, p read and
    // written) per iteration over the grid's R^3 F float32 unknowns
    P->cg_alg_bytes += m * 6.0 * (double)P->g[sy].nodes * P->g[sy].F * 4.0;
    P->cg_iters_sum += (int64_t)m;
  }
  return NPG_OK;
}

npg_status npg_run_precond_cg(npg_plan* P, float* grad, int32_t* iters) {
  bool capped = false;
  P->cg_alg_bytes = 0.0;
  P->cg_iters_sum = 0;
  npg_status st = cg_solve(P, grad, iters, &capped);
  if (st != NPG_OK) return st;
  st = cg_solve(P, P->cg.x, iters ? iters + P->n_sys : nullptr, &capped);
  if (st != NPG_OK) return st;
  hipLaunchKernelGGL(k_copy, dim3(nblk(P->n_grid_params, 256)), dim3(256), 0, P->stream, P->cg.x, grad,
                     P->n_grid_params);
  NPG_HIP(hipGetLastError());
  return capped ? NPG_ENOTCONV : NPG_OK;
}
