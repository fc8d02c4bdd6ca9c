// Sobolev preconditioning of the grid gradients (Sec. 3.5): g~ = (I+lam L)^-2 g
// per grid and feature channel, L the 6-neighbour lattice Laplacian with free
// boundary, as two conjugate-gradient solves from a zero start.
//
// All grids (every position level and the normal grid) iterate together:
// each launch covers the blocks of every system that is still active, with a
// block -> (system, first node) table. Vectors are float32 in the parameter
// layout ([node][F] per grid); inner products are accumulated in float64,
// per block, and reduced per system in a fixed order (deterministic).
// The operator is applied as p + lam * sum over existing neighbours of
// (p_n - p_nb), i.e. sums of differences, which keeps float32 rounding
// proportional to |A p| rather than to (1 + 12 lam)|p|.
#include "internal.h"

namespace {

constexpr int kB = 256;

struct Sys {
  int R, F;
  int64_t poff;
  float lam;
};

// scalars per (system, channel): 0 rr, 1 bb, 2 pq, 3 alpha, 4 beta, 5 active, 6 iterations
__device__ __forceinline__ double* scal(double* st, int s, int c) { return st + (s * 4 + c) * 8; }

__device__ __forceinline__ void block_dot_store(double (&v)[4], int F, double* part, int blk) {
  __shared__ double red[4][kB];
  for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = c < F ? v[c] : 0.0;
  __syncthreads();
  for (int st = kB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[(int64_t)blk * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kB) void k_cg_init(const NpgGrid* __restrict__ g, const int* __restrict__ blk_sys,
                                                const int64_t* __restrict__ blk_start, const float* __restrict__ b,
                                                float* __restrict__ x, float* __restrict__ r, float* __restrict__ p,
                                                double* __restrict__ part) {
  const int blk = blockIdx.x;
  const int s = blk_sys[blk];
  const int F = g[s].F;
  const int64_t node = blk_start[blk] + threadIdx.x;
  double acc[4] = {0, 0, 0, 0};
  if (node < g[s].nodes) {
    const int64_t base = g[s].poff + node * F;
    for (int c = 0; c < F; ++c) {
      float v = b[base + c];
      x[base + c] = 0.f;
      r[base + c] = v;
      p[base + c] = v;
      acc[c] = (double)v * (double)v;
    }
  }
  block_dot_store(acc, F, part, blk);
}

// q = A p and per-block partial p.q
__global__ __launch_bounds__(kB) void k_cg_ap(const NpgGrid* __restrict__ g, const int* __restrict__ blk_sys,
                                              const int64_t* __restrict__ blk_start, const int* __restrict__ active,
                                              const float* __restrict__ p, float* __restrict__ q,
                                              double* __restrict__ part) {
  const int blk = blockIdx.x;
  const int s = blk_sys[blk];
  if (!active[s]) return;
  const int F = g[s].F, R = g[s].R;
  const float lam = g[s].lam;
  const int64_t node = blk_start[blk] + threadIdx.x;
  double acc[4] = {0, 0, 0, 0};
  if (node < g[s].nodes) {
    const int64_t R2 = (int64_t)R * R;
    const int ix = (int)(node % R), iy = (int)((node / R) % R), iz = (int)(node / R2);
    const float* P0 = p + g[s].poff;
    const int64_t nb[6] = {ix > 0 ? node - 1 : -1,     ix < R - 1 ? node + 1 : -1,
                           iy > 0 ? node - R : -1,     iy < R - 1 ? node + R : -1,
                           iz > 0 ? node - R2 : -1,    iz < R - 1 ? node + R2 : -1};
    for (int c = 0; c < F; ++c) {
      const float pc = P0[node * F + c];
      float lap = 0.f;
      for (int k = 0; k < 6; ++k)
        if (nb[k] >= 0) lap += pc - P0[nb[k] * F + c];
      const float qc = fmaf(lam, lap, pc);
      q[g[s].poff + node * F + c] = qc;
      acc[c] = (double)pc * (double)qc;
    }
  }
  block_dot_store(acc, F, part, blk);
}

// x += alpha p, r -= alpha q, per-block partial r.r
__global__ __launch_bounds__(kB) void k_cg_update(const NpgGrid* __restrict__ g, const int* __restrict__ blk_sys,
                                                  const int64_t* __restrict__ blk_start, const int* __restrict__ active,
                                                  const double* __restrict__ st, float* __restrict__ x,
                                                  float* __restrict__ r, const float* __restrict__ p,
                                                  const float* __restrict__ q, double* __restrict__ part) {
  const int blk = blockIdx.x;
  const int s = blk_sys[blk];
  if (!active[s]) return;
  const int F = g[s].F;
  const int64_t node = blk_start[blk] + threadIdx.x;
  double acc[4] = {0, 0, 0, 0};
  if (node < g[s].nodes) {
    const int64_t base = g[s].poff + node * F;
    for (int c = 0; c < F; ++c) {
      const float al = (float)st[(s * 4 + c) * 8 + 3];
      x[base + c] = fmaf(al, p[base + c], x[base + c]);
      const float rv = fmaf(-al, q[base + c], r[base + c]);
      r[base + c] = rv;
      acc[c] = (double)rv * (double)rv;
    }
  }
  block_dot_store(acc, F, part, blk);
}

// p = r + beta p
__global__ __launch_bounds__(kB) void k_cg_dir(const NpgGrid* __restrict__ g, const int* __restrict__ blk_sys,
                                               const int64_t* __restrict__ blk_start, const int* __restrict__ active,
                                               const double* __restrict__ st, const float* __restrict__ r,
                                               float* __restrict__ p) {
  const int blk = blockIdx.x;
  const int s = blk_sys[blk];
  if (!active[s]) return;
  const int F = g[s].F;
  const int64_t node = blk_start[blk] + threadIdx.x;
  if (node < g[s].nodes) {
    const int64_t base = g[s].poff + node * F;
    for (int c = 0; c < F; ++c) {
      const float be = (float)st[(s * 4 + c) * 8 + 4];
      p[base + c] = fmaf(be, p[base + c], r[base + c]);
    }
  }
}

// Per system (one block each): reduce the block partials in order and update
// the scalars. mode 0: after init (rr, bb); 1: alpha = rr / pq;
// 2: beta = rr_new / rr and the convergence test.
__global__ __launch_bounds__(kB) void k_cg_reduce(const NpgGrid* __restrict__ g, const int* __restrict__ sys_blk0,
                                                  int* __restrict__ active, const double* __restrict__ part,
                                                  double* __restrict__ st, int mode, double rtol) {
  const int s = blockIdx.x;
  if (mode != 0 && !active[s]) return;
  __shared__ double red[4][kB];
  const int F = g[s].F;
  const int b0 = sys_blk0[s], b1 = sys_blk0[s + 1];
  double acc[4] = {0, 0, 0, 0};
  for (int b = b0 + threadIdx.x; b < b1; b += kB)
    for (int c = 0; c < 4; ++c) acc[c] += part[(int64_t)b * 4 + c];
  for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = kB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  int any = 0;
  for (int c = 0; c < F; ++c) {
    double* S = st + (s * 4 + c) * 8;
    const double v = red[c][0];
    if (mode == 0) {
      S[0] = v;
      S[1] = v;
      S[3] = 0.0;
      S[4] = 0.0;
      S[6] = 0.0;
      S[5] = v > 0.0 ? 1.0 : 0.0;
    } else if (mode == 1) {
      S[3] = (S[5] != 0.0 && v > 0.0) ? S[0] / v : 0.0;
    } else {
      if (S[5] != 0.0) {
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

}  // namespace

npg_status npg_cg_setup(npg_plan* P) {
  NpgCG& C = P->cg;
  std::vector<int> bsys;
  std::vector<int64_t> bstart;
  std::vector<int> s0(P->n_sys + 1);
  for (int s = 0; s < P->n_sys; ++s) {
    s0[s] = (int)bsys.size();
    for (int64_t n = 0; n < P->g[s].nodes; n += kB) {
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
  NPG_HIP(hipMalloc(&C.st, (int64_t)P->n_sys * 4 * 8 * 8));
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

// Solve (I + lam L) x = b for every system; b and the result live in grad.
static npg_status cg_solve(npg_plan* P, float* grad, int32_t* iters, bool* capped) {
  NpgCG& C = P->cg;
  hipStream_t s = P->stream;
  const int nb = C.n_blocks;
  hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(kB), 0, s, P->d_g, C.blk_sys, C.blk_start, grad, C.x, C.r, C.p,
                     C.part);
  hipLaunchKernelGGL(k_cg_reduce, dim3(P->n_sys), dim3(kB), 0, s, P->d_g, C.sys_blk0, C.active, C.part, C.st, 0,
                     P->cfg.cg_rtol);
  NPG_HIP(hipGetLastError());
  std::vector<int> act(P->n_sys);
  int it = 0;
  bool done = false;
  const int maxit = P->cfg.cg_maxit;
  while (it < maxit) {
    const int chunk = 16 < maxit - it ? 16 : maxit - it;
    for (int k = 0; k < chunk; ++k) {
      hipLaunchKernelGGL(k_cg_ap, dim3(nb), dim3(kB), 0, s, P->d_g, C.blk_sys, C.blk_start, C.active, C.p, C.q,
                         C.part);
      hipLaunchKernelGGL(k_cg_reduce, dim3(P->n_sys), dim3(kB), 0, s, P->d_g, C.sys_blk0, C.active, C.part, C.st,
                         1, P->cfg.cg_rtol);
      hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(kB), 0, s, P->d_g, C.blk_sys, C.blk_start, C.active, C.st,
                         C.x, C.r, C.p, C.q, C.part);
      hipLaunchKernelGGL(k_cg_reduce, dim3(P->n_sys), dim3(kB), 0, s, P->d_g, C.sys_blk0, C.active, C.part, C.st,
                         2, P->cfg.cg_rtol);
      hipLaunchKernelGGL(k_cg_dir, dim3(nb), dim3(kB), 0, s, P->d_g, C.blk_sys, C.blk_start, C.active, C.st, C.r,
                         C.p);
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
  if (iters) {
    std::vector<double> st((size_t)P->n_sys * 32);
    NPG_HIP(hipMemcpyAsync(st.data(), C.st, st.size() * 8, hipMemcpyDeviceToHost, s));
    NPG_HIP(hipStreamSynchronize(s));
    for (int sy = 0; sy < P->n_sys; ++sy) {
      double m = 0;
      for (int c = 0; c < P->g[sy].F; ++c) m = st[(sy * 4 + c) * 8 + 6] > m ? st[(sy * 4 + c) * 8 + 6] : m;
      iters[sy] = (int32_t)m;
    }
  }
  hipLaunchKernelGGL(k_copy, dim3(nblk(P->n_grid_params, 256)), dim3(256), 0, s, C.x, grad, P->n_grid_params);
  NPG_HIP(hipGetLastError());
  return NPG_OK;
}

npg_status npg_run_precond_cg(npg_plan* P, float* grad, int32_t* iters) {
  bool capped = false;
  npg_status st = cg_solve(P, grad, iters, &capped);
  if (st != NPG_OK) return st;
  st = cg_solve(P, grad, iters ? iters + P->n_sys : nullptr, &capped);
  if (st != NPG_OK) return st;
  return capped ? NPG_ENOTCONV : NPG_OK;
}
