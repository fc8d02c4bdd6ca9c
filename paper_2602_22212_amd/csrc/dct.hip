// Exact Sobolev preconditioner (Sec. 3.5): (I + lam L)^-2 g through the
// orthonormal 3-D DCT-II, which diagonalises the free-boundary lattice
// Laplacian: the path-graph Laplacian of R nodes has the DCT-II vectors
// C[k][n] = s_k cos(pi k (2n+1) / (2R)) as eigenvectors with eigenvalues
// mu_k = 2 - 2 cos(pi k / R), and the lattice Laplacian is their Kronecker
// sum. So g~ = C3^T diag(1 / (1 + lam (mu_kx + mu_ky + mu_kz))^2) C3 g per
// feature channel, C3 = C (x) C (x) C.
//
// Five in-place passes over each grid ([z][y][x][f] layout):
//   x forward, y forward, z forward + scale + z inverse (fused), y inverse,
//   x inverse.
// Each pass is a batched R x R matrix product along one axis: a work-group
// stages a tile of 64 lines (K = R samples each) in LDS, multiplies it by C
// (or C^T, read as float4 rows from a padded table in global memory) with
// v_mfma_f32_16x16x4_f32, and writes the tile back in place. Work-groups of
// every grid share one launch per pass.
#include <algorithm>
#include <vector>

#include "internal.h"

typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

constexpr int kJ = 64;  // lines per tile

enum Pass { kX = 0, kY = 1, kZ = 2 };

struct DctSys {
  int64_t poff;       // offset of the grid in the flat gradient vector
  const float* C;     // [Rp][Rp] C[k][n], zero padded
  const float* CT;    // [Rp][Rp] CT[n][k] = C[k][n]
  const float* mu;    // [Rp] eigenvalues 2 - 2 cos(pi k / R), zero padded
  int R, Rp, F;
  float lam;
  int64_t lines;      // number of lines of the pass
};

__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ float comp(const float4& v, int r) {
  return r == 0 ? v.x : (r == 1 ? v.y : (r == 2 ? v.z : v.w));
}

// Float offset of sample 0 of line j for a pass (layout [z][y][x][f]);
// sample n of the line sits n * stride further.
__device__ __forceinline__ int64_t line_base(int pass, int R, int F, int64_t j) {
  if (pass == kX) {  // j = (z*R + y)*F + f, n = x
    const int64_t zy = j / F, f = j - zy * F;
    return zy * R * F + f;
  }
  const int64_t RF = (int64_t)R * F;
  if (pass == kY) {  // j = z*R*F + (x*F + f), n = y
    const int64_t z = j / RF, xf = j - z * RF;
    return z * R * RF + xf;
  }
  return j;  // z: j = (y*R + x)*F + f, n = z
}
__device__ __forceinline__ int64_t line_stride(int pass, int R, int F) {
  return pass == kX ? F : (pass == kY ? (int64_t)R * F : (int64_t)R * R * F);
}

// D[k][j] = sum_n A[k][n] T[n][j] for this wave's k-tiles (kt = wave,
// wave+4, ...) and all 4 j-tiles. T is in LDS as T[n][j] (row stride kLD);
// A rows come from a padded [Rp][Rp] table as float4, fetched one k-group
// ahead of the matrix instructions that use them.
constexpr int kLD = kJ + 4;

template <int NKT>
__device__ __forceinline__ void tile_gemm(const float* __restrict__ A, int Rp, const float* T, int wave, int q,
                                          int c, v4f (&acc)[NKT][4]) {
#pragma unroll
  for (int i = 0; i < NKT; ++i)
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) acc[i][jt] = v4f{0.f, 0.f, 0.f, 0.f};
  const int nkt = Rp / 16;
  const int ng = Rp / 16;
  // the operands of the current and of the next k-group, in registers (fixed
  // names, so no dynamically indexed buffer)
  float4 cur[NKT], nxt[NKT];
#pragma unroll
  for (int i = 0; i < NKT; ++i) {
    const int kt = wave + 4 * i;
    cur[i] = kt < nkt ? *reinterpret_cast<const float4*>(A + (int64_t)(16 * kt + c) * Rp + 4 * q)
                      : make_float4(0.f, 0.f, 0.f, 0.f);
    nxt[i] = cur[i];
  }
  for (int g = 0; g < ng; ++g) {
    if (g + 1 < ng) {
#pragma unroll
      for (int i = 0; i < NKT; ++i) {
        const int kt = wave + 4 * i;
        if (kt < nkt) nxt[i] = *reinterpret_cast<const float4*>(A + (int64_t)(16 * kt + c) * Rp + 16 * (g + 1) + 4 * q);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float b[4];
#pragma unroll
      for (int jt = 0; jt < 4; ++jt) b[jt] = T[(16 * g + 4 * q + r) * kLD + 16 * jt + c];
#pragma unroll
      for (int i = 0; i < NKT; ++i) {
        if (wave + 4 * i >= nkt) break;
#pragma unroll
        for (int jt = 0; jt < 4; ++jt) acc[i][jt] = mfma(comp(cur[i], r), b[jt], acc[i][jt]);
      }
    }
#pragma unroll
    for (int i = 0; i < NKT; ++i) cur[i] = nxt[i];
  }
}

// Tile fill / write-back. x pass: lines j = (zy, f) -> 64 / F rows zy of F
// channels, stored as T[x][zl*F + f] (float4 when F = 4); y and z passes:
// 64 lines contiguous in memory per sample n, T[n][jj].
__device__ __forceinline__ void tile_io(float* base, float* T, int pass, int R, int Rp, int F, int64_t j0, int njl,
                                        const int64_t* lb, int64_t stride, bool store) {
  if (pass == 0 && F == 4 && (j0 & 3) == 0) {
    const int nzl = njl / 4;  // full rows of 4 channels (the tile never splits a row)
    for (int e = threadIdx.x; e < 16 * Rp; e += 256) {
      const int zl = e / Rp, n = e - zl * Rp;
      float4* tp = reinterpret_cast<float4*>(T + n * kLD + 4 * zl);
      if (store) {
        if (zl < nzl && n < R) *reinterpret_cast<float4*>(base + lb[4 * zl] + (int64_t)n * 4) = *tp;
      } else {
        *tp = (zl < nzl && n < R) ? *reinterpret_cast<const float4*>(base + lb[4 * zl] + (int64_t)n * 4)
                                  : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    return;
  }
  for (int e = threadIdx.x; e < kJ * Rp; e += 256) {
    int jj, n;
    if (pass == 0) {
      n = e % Rp;
      jj = e / Rp;
    } else {
      jj = e % kJ;
      n = e / kJ;
    }
    float* tp = T + n * kLD + jj;
    const bool in = n < R && jj < njl;
    if (store) {
      if (in) base[lb[jj] + n * stride] = *tp;
    } else {
      *tp = in ? base[lb[jj] + n * stride] : 0.f;
    }
  }
}

// One pass over one tile of kJ lines. mode: 0 = multiply by C (forward),
// 1 = multiply by C^T (inverse), 2 = forward, scale, inverse (z only).
template <int NKT>
__global__ __launch_bounds__(256) void k_dct_pass(float* __restrict__ grad, const DctSys* __restrict__ sys,
                                                  const int* __restrict__ blk_sys,
                                                  const int64_t* __restrict__ blk_j0, int pass, int mode) {
  extern __shared__ float T[];  // [Rp][kLD]
  __shared__ int64_t lb[kJ];
  const int s = blk_sys[blockIdx.x];
  const DctSys S = sys[s];
  float* base = grad + S.poff;
  const int64_t j0 = blk_j0[blockIdx.x];
  const int R = S.R, Rp = S.Rp, F = S.F;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar branches on k-tiles
  const int q = lane >> 4, c = lane & 15;
  const int njl = (int)min((int64_t)kJ, S.lines - j0);
  const int64_t stride = line_stride(pass, R, F);
  if ((int)threadIdx.x < kJ) lb[threadIdx.x] = line_base(pass, R, F, j0 + threadIdx.x);
  __syncthreads();
  tile_io(base, T, pass, R, Rp, F, j0, njl, lb, stride, false);
  __syncthreads();

  v4f acc[NKT][4];
  const int nkt = Rp / 16;
  tile_gemm<NKT>(mode == 1 ? S.CT : S.C, Rp, T, wave, q, c, acc);
  if (mode == 2) {
    // scale by 1 / (1 + lam (mu_kz + mu_ky + mu_kx))^2; the line index
    // j = (y*R + x)*F + f names the (ky, kx) of the two earlier passes
    float mj[4];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {
      const int64_t j = j0 + 16 * jt + c;
      const int64_t yx = j / F;
      const int ky = (int)(yx / R), kx = (int)(yx - (int64_t)(yx / R) * R);
      mj[jt] = j < S.lines ? S.mu[ky] + S.mu[kx] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < NKT; ++i) {
      const int kt = wave + 4 * i;
      if (kt >= nkt) break;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float mk = S.mu[16 * kt + 4 * q + r];
#pragma unroll
        for (int jt = 0; jt < 4; ++jt) {
          const float d = 1.f + S.lam * (mk + mj[jt]);
          acc[i][jt][r] = acc[i][jt][r] / (d * d);
        }
      }
    }
    __syncthreads();  // every wave has finished reading T
#pragma unroll
    for (int i = 0; i < NKT; ++i) {
      const int kt = wave + 4 * i;
      if (kt >= nkt) break;
#pragma unroll
      for (int jt = 0; jt < 4; ++jt)
#pragma unroll
        for (int r = 0; r < 4; ++r) T[(16 * kt + 4 * q + r) * kLD + 16 * jt + c] = acc[i][jt][r];
    }
    __syncthreads();
    tile_gemm<NKT>(S.CT, Rp, T, wave, q, c, acc);
  }
  __syncthreads();  // every wave has finished reading T
#pragma unroll
  for (int i = 0; i < NKT; ++i) {
    const int kt = wave + 4 * i;
    if (kt >= nkt) break;
#pragma unroll
    for (int jt = 0; jt < 4; ++jt)
#pragma unroll
      for (int r = 0; r < 4; ++r) T[(16 * kt + 4 * q + r) * kLD + 16 * jt + c] = acc[i][jt][r];
  }
  __syncthreads();
  tile_io(base, T, pass, R, Rp, F, j0, njl, lb, stride, true);
}

__global__ void k_dct_tables(int R, int Rp, float* __restrict__ C, float* __restrict__ CT, float* __restrict__ mu) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < (int64_t)Rp * Rp) {
    const int k = (int)(e / Rp), n = (int)(e % Rp);
    double v = 0.0;
    if (k < R && n < R) v = sqrt((k == 0 ? 1.0 : 2.0) / R) * cos(M_PI * k * (2.0 * n + 1.0) / (2.0 * R));
    C[e] = (float)v;
    CT[(int64_t)n * Rp + k] = (float)v;
  }
  if (e < Rp) mu[e] = e < R ? (float)(2.0 - 2.0 * cos(M_PI * (double)e / R)) : 0.f;
}

}  // namespace

struct NpgDct {
  std::vector<float*> tables;
  DctSys* d_sys[3] = {nullptr, nullptr, nullptr};
  int* blk_sys[3] = {nullptr, nullptr, nullptr};
  int64_t* blk_j0[3] = {nullptr, nullptr, nullptr};
  int nblk[3] = {0, 0, 0};
  int max_rp = 16;
};

npg_status npg_dct_setup(npg_plan* P) {
  NpgDct* D = new NpgDct();
  P->dct = D;
  std::vector<DctSys> sys(P->n_sys);
  for (int s = 0; s < P->n_sys; ++s) {
    const NpgGrid& g = P->g[s];
    const int Rp = (g.R + 15) / 16 * 16;
    if (Rp > 256) return npg_fail(NPG_EINVAL, "the DCT preconditioner supports up to 256 nodes per axis");
    float *C, *CT, *mu;
    NPG_HIP(hipMalloc(&C, (size_t)Rp * Rp * 4));
    NPG_HIP(hipMalloc(&CT, (size_t)Rp * Rp * 4));
    NPG_HIP(hipMalloc(&mu, (size_t)Rp * 4));
    D->tables.push_back(C);
    D->tables.push_back(CT);
    D->tables.push_back(mu);
    hipLaunchKernelGGL(k_dct_tables, dim3((Rp * Rp + 255) / 256), dim3(256), 0, P->stream, g.R, Rp, C, CT, mu);
    NPG_HIP(hipGetLastError());
    sys[s] = DctSys{g.poff, C, CT, mu, g.R, Rp, g.F, g.lam, 0};
    D->max_rp = std::max(D->max_rp, Rp);
  }
  for (int pass = 0; pass < 3; ++pass) {
    std::vector<int> bs;
    std::vector<int64_t> bj;
    std::vector<DctSys> ps = sys;
    for (int s = 0; s < P->n_sys; ++s) {
      const int64_t lines = (int64_t)P->g[s].R * P->g[s].R * P->g[s].F;
      ps[s].lines = lines;
      for (int64_t j = 0; j < lines; j += kJ) {
        bs.push_back(s);
        bj.push_back(j);
      }
    }
    // largest grids first
    std::vector<int> order(bs.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ps[bs[a]].Rp > ps[bs[b]].Rp; });
    std::vector<int> bs2(bs.size());
    std::vector<int64_t> bj2(bj.size());
    for (size_t i = 0; i < order.size(); ++i) {
      bs2[i] = bs[order[i]];
      bj2[i] = bj[order[i]];
    }
    D->nblk[pass] = (int)bs2.size();
    NPG_HIP(hipMalloc(&D->d_sys[pass], sizeof(DctSys) * P->n_sys));
    NPG_HIP(hipMalloc(&D->blk_sys[pass], bs2.size() * 4));
    NPG_HIP(hipMalloc(&D->blk_j0[pass], bj2.size() * 8));
    NPG_HIP(hipMemcpy(D->d_sys[pass], ps.data(), sizeof(DctSys) * P->n_sys, hipMemcpyHostToDevice));
    NPG_HIP(hipMemcpy(D->blk_sys[pass], bs2.data(), bs2.size() * 4, hipMemcpyHostToDevice));
    NPG_HIP(hipMemcpy(D->blk_j0[pass], bj2.data(), bj2.size() * 8, hipMemcpyHostToDevice));
  }
  return NPG_OK;
}

void npg_dct_free(npg_plan* P) {
  NpgDct* D = P->dct;
  if (!D) return;
  for (float* t : D->tables) hipFree(t);
  for (int p = 0; p < 3; ++p) {
    hipFree(D->d_sys[p]);
    hipFree(D->blk_sys[p]);
    hipFree(D->blk_j0[p]);
  }
  delete D;
  P->dct = nullptr;
}

template <int NKT>
static hipError_t launch_pass(const npg_plan* P, float* grad, int pass, int mode) {
  NpgDct* D = P->dct;
  const size_t lds = (size_t)D->max_rp * kLD * sizeof(float);
  hipError_t e = hipFuncSetAttribute((const void*)k_dct_pass<NKT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_dct_pass<NKT>), dim3(D->nblk[pass]), dim3(256), lds, P->stream, grad, D->d_sys[pass],
                     D->blk_sys[pass], D->blk_j0[pass], pass, mode);
  return hipGetLastError();
}

// Applies the preconditioner in place to every grid block of grad.
npg_status npg_run_precond_dct(npg_plan* P, float* grad) {
  NpgDct* D = P->dct;
  const int nkt = D->max_rp / 16;
  auto run = [&](int pass, int mode) -> hipError_t {
    if (nkt <= 4) return launch_pass<1>(P, grad, pass, mode);
    if (nkt <= 8) return launch_pass<2>(P, grad, pass, mode);
    if (nkt <= 12) return launch_pass<3>(P, grad, pass, mode);
    return launch_pass<4>(P, grad, pass, mode);
  };
  NPG_HIP(run(kX, 0));
  NPG_HIP(run(kY, 0));
  NPG_HIP(run(kZ, 2));
  NPG_HIP(run(kY, 1));
  NPG_HIP(run(kX, 1));
  return NPG_OK;
}
