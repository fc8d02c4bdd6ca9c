// Pruned nearest-neighbour search for the Chamfer distance of Sec. 3.5: per
// frame, every vertex's nearest point (a, da) and every point's nearest
// vertex (b, db), with the same results as the exhaustive pass of
// chamfer.hip: float32 distances in the direct form (x-p).(x-p) (the same
// operation order, which is symmetric in its operands bit for bit), and on
// equal distances the lowest original index.
//
// Both directions run the same kernel: one wave takes 64 x NQ queries of one
// frame and scans the frame's targets in tiles of kNT. Queries and targets
// are in Morton order (vertices by their rest position, points per frame by
// position), so a wave's queries and a tile's targets each occupy a compact
// region. A tile is skipped when, for every query of the wave, the squared
// distance from the query to the tile's bounding box exceeds the query's best
// distance so far: every target in the tile is then strictly farther than the
// best, so neither the minimum nor any tie can be lost. The comparison keeps a
// margin above the float32 rounding of both the box distance and the direct
// form (see lb_skip). Tiles overlapping the wave's own query box are scanned
// first, the others afterwards, both in tile order.
//
// The scan tracks values only (running minima); afterwards each query
// re-scans the tile that first reached its minimum and takes the lowest
// original index among the targets at exactly that distance. A later tile
// that reached the same minimum marks a tie across tiles, and that query then
// re-scans every target of the frame.
#include "internal.h"

#include <algorithm>
#include <cstring>
#include <numeric>

namespace {

constexpr int kNQV = 2;         // queries per lane, vertex queries (over point tiles)
constexpr int kNQP = 2;         // queries per lane, point queries (over vertex tiles)
constexpr int kNT = 128;        // targets per tile
constexpr int kMaxTL = 16;      // tiles per lane of the ordered walk: at most 64 kMaxTL tiles per frame

__device__ __forceinline__ float dist2(float4 x, float4 p) {
  float dx = x.x - p.x, dy = x.y - p.y, dz = x.z - p.z;
  return __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmul_rn(dx, dx)));
}
__device__ __forceinline__ float min3f(float a, float b, float c) { return fminf(fminf(a, b), c); }
// lane `src` of a float (its bits, not a conversion)
__device__ __forceinline__ float rdl(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}

// Squared distance from q to the box [lo, hi] (0 inside).
__device__ __forceinline__ float box_d2(float4 q, float4 lo, float4 hi) {
  const float gx = fmaxf(fmaxf(lo.x - q.x, q.x - hi.x), 0.f);
  const float gy = fmaxf(fmaxf(lo.y - q.y, q.y - hi.y), 0.f);
  const float gz = fmaxf(fmaxf(lo.z - q.z, q.z - hi.z), 0.f);
  return __fmaf_rn(gz, gz, __fmaf_rn(gy, gy, __fmul_rn(gx, gx)));
}

// True when every target in a box at computed squared distance lb from the
// query is strictly farther than `best`. The exact box distance bounds the
// exact distance of every target from below; each float32 result carries a
// relative error of at most a few units of 2^-24 (a difference, three
// products and two sums), so a computed distance is at least lb (1 - 2^-20).
// lb is scaled by 1 - 2^-18 before the comparison, and lb below 2^-100 (where
// underflow breaks the relative bound) never skips. NaN never skips.
__device__ __forceinline__ bool lb_skip(float lb, float best) {
  return lb > 0x1p-100f && lb * (1.0f - 0x1p-18f) > best;
}

struct NnArgs {
  const int2* grp;          // [ngroups] (frame, first sorted query of the wave)
  int ngroups;
  const float4* q;          // sorted queries, frame after frame
  const int64_t* qoff;      // [T+1] frame offsets into q (and into the outputs)
  const int32_t* qperm;     // sorted query -> original index within its frame
  int qperm_global;         // 1: qperm indexed like q; 0: one table for every frame
  const float4* tg;         // sorted targets, frame after frame
  const int64_t* toff;      // [T+1] frame offsets into tg
  const int32_t* tperm;     // sorted target -> original index within its frame
  int tperm_global;
  const float4* box;        // [tiles][2] lo, hi of each target tile
  const int* tboff;         // [T+1] first tile of each frame
  int32_t* idx;             // outputs at qoff[t] + original query index
  float* dist;
};

// Squared distance between two boxes (0 when they overlap).
__device__ __forceinline__ float boxbox_d2(float4 alo, float4 ahi, float4 blo, float4 bhi) {
  const float gx = fmaxf(fmaxf(blo.x - ahi.x, alo.x - bhi.x), 0.f);
  const float gy = fmaxf(fmaxf(blo.y - ahi.y, alo.y - bhi.y), 0.f);
  const float gz = fmaxf(fmaxf(blo.z - ahi.z, alo.z - bhi.z), 0.f);
  return __fmaf_rn(gz, gz, __fmaf_rn(gy, gy, __fmul_rn(gx, gx)));
}

// Wave minimum of (v, k) pairs, smaller v first and then smaller k (all lanes
// receive it). NaN never wins.
__device__ __forceinline__ void wave_argmin(float& v, int& k) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const float ov = __shfl_xor(v, m);
    const int ok = __shfl_xor(k, m);
    if (ov < v || (ov == v && ok < k)) {
      v = ov;
      k = ok;
    }
  }
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v = fmaxf(v, __shfl_xor(v, m));
  return v;
}

// One wave: NQ queries per lane against the frame's target tiles (at most
// 64 TL tiles), nearest tile first. Every lane holds the distances from the
// wave's query box to tiles lane, lane + 64, ...; each round selects the
// nearest tile not yet taken (lowest index on equal distances). The walk ends
// when that distance exceeds the largest current minimum of the wave's
// queries: every remaining tile is then farther than every query's minimum.
// A selected tile is scanned when at least one query's own box distance does
// not exceed its minimum. The waves of a work-group are independent (no
// work-group barrier: their walks differ in length).
template <int WG, int NQ, int TL>
__global__ __launch_bounds__(WG) void k_nn_pruned(NnArgs A) {
  const int g = (int)blockIdx.x * (WG / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (g >= A.ngroups) return;
  const int lane = (int)(threadIdx.x & 63);
  const int2 gr = A.grp[g];
  const int t = gr.x, q0 = gr.y;
  const int64_t qb = A.qoff[t];
  const int nq = (int)(A.qoff[t + 1] - qb);
  const int64_t tb = A.toff[t];
  const int nt = (int)(A.toff[t + 1] - tb);
  const int b0 = A.tboff[t], nb = A.tboff[t + 1] - b0;

  float4 q[NQ];
  float best[NQ];
  int btile[NQ];
  bool tie[NQ];
  float4 wlo = make_float4(INFINITY, INFINITY, INFINITY, 0.f), whi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int qi = q0 + k * 64 + lane;
    const bool valid = qi < nq;
    q[k] = A.q[qb + (valid ? qi : nq - 1)];
    // a padding query never asks for a tile and never improves
    best[k] = valid ? INFINITY : -1.0f;
    btile[k] = -1;
    tie[k] = false;
    if (valid) {
      wlo.x = fminf(wlo.x, q[k].x), wlo.y = fminf(wlo.y, q[k].y), wlo.z = fminf(wlo.z, q[k].z);
      whi.x = fmaxf(whi.x, q[k].x), whi.y = fmaxf(whi.y, q[k].y), whi.z = fmaxf(whi.z, q[k].z);
    }
  }
  // the wave's query box
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    wlo.x = fminf(wlo.x, __shfl_xor(wlo.x, m)), wlo.y = fminf(wlo.y, __shfl_xor(wlo.y, m));
    wlo.z = fminf(wlo.z, __shfl_xor(wlo.z, m));
    whi.x = fmaxf(whi.x, __shfl_xor(whi.x, m)), whi.y = fmaxf(whi.y, __shfl_xor(whi.y, m));
    whi.z = fmaxf(whi.z, __shfl_xor(whi.z, m));
  }
  // box distances of this lane's tiles (infinite once taken or absent); with
  // at most 256 tiles the boxes themselves stay in the lanes' registers
  constexpr bool kBoxReg = TL <= 4;
  float tlb[TL];
  float4 rlo[kBoxReg ? TL : 1], rhi[kBoxReg ? TL : 1];
#pragma unroll
  for (int m = 0; m < TL; ++m) {
    const int k = lane + 64 * m;
    float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
    if (k < nb) {
      lo = A.box[2 * (int64_t)(b0 + k)];
      hi = A.box[2 * (int64_t)(b0 + k) + 1];
    }
    tlb[m] = k < nb ? boxbox_d2(wlo, whi, lo, hi) : INFINITY;
    if constexpr (kBoxReg) {
      rlo[m] = lo;
      rhi[m] = hi;
    }
  }
  auto tile_box = [&](int k, float4& lo, float4& hi) {  // k wave-uniform
    if constexpr (kBoxReg) {
      const int src = k & 63;
#pragma unroll
      for (int m = 0; m < TL; ++m)
        if (m == (k >> 6)) {
          lo = make_float4(rdl(rlo[m].x, src), rdl(rlo[m].y, src), rdl(rlo[m].z, src), 0.f);
          hi = make_float4(rdl(rhi[m].x, src), rdl(rhi[m].y, src), rdl(rhi[m].z, src), 0.f);
        }
    } else {
      lo = A.box[2 * (int64_t)(b0 + k)];
      hi = A.box[2 * (int64_t)(b0 + k) + 1];
    }
  };

  // The next needed tile's targets are loaded into registers while the
  // current one is scanned from LDS (two buffers per wave; the wave's lanes
  // write a tile and then all read it, LDS operations of one wave completing
  // in order).
  __shared__ float4 sT[WG / 64][2][kNT];
  const int w = (int)(threadIdx.x >> 6);
  auto select = [&](float& mv) -> int {  // nearest remaining tile, taken; -1 if none
    mv = INFINITY;
    int mk = INT_MAX;
#pragma unroll
    for (int m = 0; m < TL; ++m)
      if (tlb[m] < mv) {
        mv = tlb[m];
        mk = lane + 64 * m;
      }
    wave_argmin(mv, mk);
    if (mk == INT_MAX) return -1;
    const int k = __builtin_amdgcn_readfirstlane(mk);
#pragma unroll
    for (int m = 0; m < TL; ++m)
      if (m == (k >> 6) && lane == (k & 63)) tlb[m] = INFINITY;
    return k;
  };
  auto max_best = [&]() {
    float mb = best[0];
#pragma unroll
    for (int kk = 1; kk < NQ; ++kk) mb = fmaxf(mb, best[kk]);
    return wave_max(mb);
  };
  auto needed = [&](int k) {  // some query's box distance does not exceed its minimum
    float4 lo, hi;
    tile_box(k, lo, hi);
    bool need = false;
#pragma unroll
    for (int kk = 0; kk < NQ; ++kk) need |= best[kk] >= 0.f && !lb_skip(box_d2(q[kk], lo, hi), best[kk]);
    return __any(need) != 0;
  };
  // The nearest remaining tile some query needs, or -1 when none is left or
  // every remaining tile is farther than every minimum (minima only shrink,
  // so a tile found unneeded here stays unneeded).
  auto next = [&]() -> int {
    for (;;) {
      float mv;
      const int k = select(mv);
      if (k < 0 || lb_skip(mv, max_best())) return -1;
      if (needed(k)) return k;
    }
  };
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0;
  auto fetch = [&](int k) {
    const int j0 = k * kNT, cnt = min(kNT, nt - j0);
    if (lane < cnt) r0 = A.tg[tb + j0 + lane];
    if (lane + 64 < cnt) r1 = A.tg[tb + j0 + lane + 64];
  };
  auto stash = [&](int buf) {
    sT[w][buf][lane] = r0;
    sT[w][buf][lane + 64] = r1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  int k = next();
  if (k >= 0) {
    fetch(k);
    stash(0);
    int buf = 0;
    bool fresh = true;  // k was found needed with the current minima
    for (;;) {
      const int kn = next();
      if (kn >= 0) fetch(kn);  // in flight during the scan of tile k
      if (fresh || needed(k)) {
        const int cnt = min(kNT, nt - k * kNT);
        const float4* tp = sT[w][buf];
        float tmin[NQ];
#pragma unroll
        for (int kk = 0; kk < NQ; ++kk) tmin[kk] = INFINITY;
        int j = 0;
        for (; j + 3 < cnt; j += 4) {
          const float4 p0 = tp[j], p1 = tp[j + 1], p2 = tp[j + 2], p3 = tp[j + 3];
#pragma unroll
          for (int kk = 0; kk < NQ; ++kk) {
            tmin[kk] = min3f(tmin[kk], dist2(q[kk], p0), dist2(q[kk], p1));
            tmin[kk] = min3f(tmin[kk], dist2(q[kk], p2), dist2(q[kk], p3));
          }
        }
        for (; j < cnt; ++j) {
          const float4 p0 = tp[j];
#pragma unroll
          for (int kk = 0; kk < NQ; ++kk) tmin[kk] = fminf(tmin[kk], dist2(q[kk], p0));
        }
#pragma unroll
        for (int kk = 0; kk < NQ; ++kk) {
          if (tmin[kk] < best[kk]) {
            best[kk] = tmin[kk];
            btile[kk] = k;
            tie[kk] = false;
          } else if (tmin[kk] == best[kk] && btile[kk] >= 0) {
            tie[kk] = true;
          }
        }
      }
      if (kn < 0) break;
      buf ^= 1;
      stash(buf);
      k = kn;
      fresh = false;
    }
  }

  // lowest original target index at the minimum: among the targets of the
  // tile that first reached it, or, after a tie across tiles, of every tile
  // whose box is not strictly farther than the minimum (eight loads at a time)
  const int64_t tpb = A.tperm_global ? tb : 0;
  auto lowest_in = [&](int kk, int j0, int j1, int& o) {
    for (int j = j0; j < j1; j += 8) {
      float4 p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) p[u] = A.tg[tb + min(j + u, j1 - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j + u < j1 && dist2(q[kk], p[u]) == best[kk]) o = min(o, A.tperm[tpb + j + u]);
    }
  };
#pragma unroll
  for (int kk = 0; kk < NQ; ++kk) {
    const int qi = q0 + kk * 64 + lane;
    if (qi >= nq) continue;
    int o = INT_MAX;
    if (btile[kk] >= 0 && !tie[kk]) {
      lowest_in(kk, btile[kk] * kNT, min(nt, (btile[kk] + 1) * kNT), o);
    } else if (btile[kk] >= 0) {
      for (int kt = 0; kt < nb; ++kt) {
        const float4 lo = A.box[2 * (int64_t)(b0 + kt)], hi = A.box[2 * (int64_t)(b0 + kt) + 1];
        if (!lb_skip(box_d2(q[kk], lo, hi), best[kk])) lowest_in(kk, kt * kNT, min(nt, (kt + 1) * kNT), o);
      }
    }
    const int iq = A.qperm[(A.qperm_global ? qb : 0) + qi];
    A.idx[qb + iq] = o == INT_MAX ? 0 : o;
    A.dist[qb + iq] = best[kk];
  }
}

// Sorted copy of the deformed vertices (x^_s[t][k] = x^[t][perm[k]]) and the
// bounding box of each tile of kNT sorted vertices; one wave per (frame, tile).
__global__ __launch_bounds__(256) void k_nn_gather(const float4* __restrict__ xhat, const int32_t* __restrict__ perm,
                                                   int64_t V, int T, int ntv, float4* __restrict__ xs,
                                                   float4* __restrict__ vbox) {
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= (int64_t)T * ntv) return;
  const int lane = (int)(threadIdx.x & 63);
  const int t = (int)(w / ntv), tile = (int)(w - (int64_t)t * ntv);
  float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f), hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
  for (int h = 0; h < kNT; h += 64) {
    const int64_t k = (int64_t)tile * kNT + h + lane;
    if (k < V) {
      const float4 v = xhat[(int64_t)t * V + perm[k]];
      xs[(int64_t)t * V + k] = v;
      lo.x = fminf(lo.x, v.x), lo.y = fminf(lo.y, v.y), lo.z = fminf(lo.z, v.z);
      hi.x = fmaxf(hi.x, v.x), hi.y = fmaxf(hi.y, v.y), hi.z = fmaxf(hi.z, v.z);
    }
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    lo.x = fminf(lo.x, __shfl_xor(lo.x, m)), lo.y = fminf(lo.y, __shfl_xor(lo.y, m));
    lo.z = fminf(lo.z, __shfl_xor(lo.z, m));
    hi.x = fmaxf(hi.x, __shfl_xor(hi.x, m)), hi.y = fmaxf(hi.y, __shfl_xor(hi.y, m));
    hi.z = fmaxf(hi.z, __shfl_xor(hi.z, m));
  }
  if (lane == 0) {
    vbox[2 * w] = lo;
    vbox[2 * w + 1] = hi;
  }
}

// ---- host side: Morton order and the static tables ---------------------------
// 30-bit Morton code of a position quantised to 10 bits per axis inside [lo, hi].
uint32_t spread10(uint32_t v) {
  v &= 0x3ff;
  v = (v | (v << 16)) & 0x030000ff;
  v = (v | (v << 8)) & 0x0300f00f;
  v = (v | (v << 4)) & 0x030c30c3;
  v = (v | (v << 2)) & 0x09249249;
  return v;
}
// order[k] = the k-th of n points (xyz, stride 4 floats) in Morton order,
// equal codes by index
void morton_order(const float* p, int64_t n, std::vector<int32_t>& order) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], p[4 * i + a]);
      hi[a] = std::max(hi[a], p[4 * i + a]);
    }
  std::vector<uint64_t> key((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    uint32_t c = 0;
    for (int a = 0; a < 3; ++a) {
      const float span = hi[a] - lo[a];
      const float u = span > 0.f ? (p[4 * i + a] - lo[a]) / span : 0.f;
      const uint32_t qv = (uint32_t)std::min(1023.f, std::max(0.f, u * 1023.f));
      c |= spread10(qv) << a;
    }
    key[(size_t)i] = ((uint64_t)c << 32) | (uint64_t)i;
  }
  std::sort(key.begin(), key.end());
  order.resize((size_t)n);
  for (int64_t k = 0; k < n; ++k) order[(size_t)k] = (int32_t)(key[(size_t)k] & 0xffffffffu);
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

struct NpgNn {
  const int32_t* perm_v = nullptr;  // [V] sorted vertex -> original vertex (the plan's vperm)
  float4* pts_s = nullptr;      // [Ntot] points sorted within each frame
  int32_t* perm_p = nullptr;    // [Ntot] sorted point -> original index within its frame
  float4* pbox = nullptr;       // [point tiles][2]
  int* ptile_off = nullptr;     // [T+1]
  int2* pgrp = nullptr;         // point-query waves
  int n_pgrp = 0;
  float4* xs = nullptr;         // [T][V] sorted deformed vertices (per call)
  float4* vbox = nullptr;       // [T * ntv][2]
  int* vtile_off = nullptr;     // [T+1] = t * ntv
  int64_t* vx_off = nullptr;    // [T+1] = t * V
  int2* vgrp = nullptr;         // vertex-query waves
  int n_vgrp = 0;
  int ntv = 0;
  int tl_rows = 2, tl_cols = 2;  // tiles per lane of the ordered walk (2, 4, 8 or 16)
};

void npg_nn_free(npg_plan* P) {
  NpgNn* N = P->nn;
  if (!N) return;
  void* bufs[] = {N->pts_s, N->perm_p, N->pbox, N->ptile_off, N->pgrp,
                  N->xs, N->vbox, N->vtile_off, N->vx_off, N->vgrp};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete N;
  P->nn = nullptr;
}

// Static tables of the pruned search (synchronizes the plan's stream): Morton
// orders of the reference vertices and of every frame's points, the sorted
// points, their tile boxes and the wave tables of both directions. A plan with
// more than 64 kMaxTL kNT (131072) vertices or points in a frame gets no tables
// (P->nn stays NULL) and uses the exhaustive search.
npg_status npg_nn_setup(npg_plan* P) {
  const int64_t V = P->V, Ntot = P->Ntot;
  const int T = P->T;
  if (V > 64 * kMaxTL * kNT || P->Nmax > 64 * kMaxTL * kNT) return NPG_OK;  // exhaustive search (P->nn stays NULL)
  NpgNn* N = new NpgNn();
  P->nn = N;
  std::vector<float4> pts((size_t)Ntot);
  NPG_HIP(hipMemcpyAsync(pts.data(), P->pts, Ntot * sizeof(float4), hipMemcpyDeviceToHost, P->stream));
  NPG_HIP(hipStreamSynchronize(P->stream));
  N->perm_v = P->vperm;
  N->ntv = (int)((V + kNT - 1) / kNT);

  std::vector<float4> ps((size_t)Ntot), pbox;
  std::vector<int32_t> pp((size_t)Ntot), ord;
  std::vector<int> ptoff(T + 1, 0);
  std::vector<int2> pg, vg;
  for (int t = 0; t < T; ++t) {
    const int64_t o0 = P->off_h[t], n = P->off_h[t + 1] - o0;
    morton_order(reinterpret_cast<const float*>(pts.data() + o0), n, ord);
    for (int64_t k = 0; k < n; ++k) {
      ps[(size_t)(o0 + k)] = pts[(size_t)(o0 + ord[(size_t)k])];
      pp[(size_t)(o0 + k)] = ord[(size_t)k];
    }
    for (int64_t j0 = 0; j0 < n; j0 += kNT) {
      float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f), hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
      for (int64_t j = j0; j < std::min(n, j0 + kNT); ++j) {
        const float4 v = ps[(size_t)(o0 + j)];
        lo.x = std::min(lo.x, v.x), lo.y = std::min(lo.y, v.y), lo.z = std::min(lo.z, v.z);
        hi.x = std::max(hi.x, v.x), hi.y = std::max(hi.y, v.y), hi.z = std::max(hi.z, v.z);
      }
      pbox.push_back(lo);
      pbox.push_back(hi);
    }
    ptoff[t + 1] = ptoff[t] + (int)((n + kNT - 1) / kNT);
    for (int64_t q0 = 0; q0 < n; q0 += 64 * kNQP) pg.push_back(make_int2(t, (int)q0));
    for (int64_t q0 = 0; q0 < V; q0 += 64 * kNQV) vg.push_back(make_int2(t, (int)q0));
  }
  std::vector<int> vtoff(T + 1);
  std::vector<int64_t> vxoff(T + 1);
  for (int t = 0; t <= T; ++t) {
    vtoff[t] = t * N->ntv;
    vxoff[t] = (int64_t)t * V;
  }
  auto tl_of = [](int tiles) { return tiles <= 128 ? 2 : tiles <= 256 ? 4 : tiles <= 512 ? 8 : 16; };
  int max_pt = 0;
  for (int t = 0; t < T; ++t) max_pt = std::max(max_pt, ptoff[t + 1] - ptoff[t]);
  N->tl_rows = tl_of(max_pt);
  N->tl_cols = tl_of(N->ntv);
  N->n_pgrp = (int)pg.size();
  N->n_vgrp = (int)vg.size();
  auto up = [&](auto** dst, const auto& src) -> npg_status {
    const size_t bytes = src.size() * sizeof(src[0]);
    if (hipMalloc((void**)dst, bytes ? bytes : 16) != hipSuccess)
      return npg_fail(NPG_ENOMEM, "hipMalloc of the nearest-neighbour tables failed");
    if (bytes) NPG_HIP(hipMemcpyAsync(*dst, src.data(), bytes, hipMemcpyHostToDevice, P->stream));
    return NPG_OK;
  };
  npg_status st;
  if ((st = up(&N->pts_s, ps)) != NPG_OK) return st;
  if ((st = up(&N->perm_p, pp)) != NPG_OK) return st;
  if ((st = up(&N->pbox, pbox)) != NPG_OK) return st;
  if ((st = up(&N->ptile_off, ptoff)) != NPG_OK) return st;
  if ((st = up(&N->pgrp, pg)) != NPG_OK) return st;
  if ((st = up(&N->vgrp, vg)) != NPG_OK) return st;
  if ((st = up(&N->vtile_off, vtoff)) != NPG_OK) return st;
  if ((st = up(&N->vx_off, vxoff)) != NPG_OK) return st;
  if (hipMalloc((void**)&N->xs, (size_t)T * V * sizeof(float4)) != hipSuccess ||
      hipMalloc((void**)&N->vbox, (size_t)T * N->ntv * 2 * sizeof(float4)) != hipSuccess)
    return npg_fail(NPG_ENOMEM, "hipMalloc of the nearest-neighbour workspace failed");
  NPG_HIP(hipStreamSynchronize(P->stream));
  return NPG_OK;
}

// The plan's vertex order (P->vperm, synchronizes): the reference vertices in
// Morton order of their rest positions, equal codes by index. The encode
// walks vertices in this order and the pruned search builds its query waves
// and target tiles from it.
npg_status npg_vertex_order(npg_plan* P) {
  std::vector<float4> xyz((size_t)P->V);
  NPG_HIP(hipMemcpyAsync(xyz.data(), P->xyz, P->V * sizeof(float4), hipMemcpyDeviceToHost, P->stream));
  NPG_HIP(hipStreamSynchronize(P->stream));
  std::vector<int32_t> pv;
  morton_order(reinterpret_cast<const float*>(xyz.data()), P->V, pv);
  if (hipMalloc((void**)&P->vperm, (size_t)P->V * sizeof(int32_t)) != hipSuccess)
    return npg_fail(NPG_ENOMEM, "hipMalloc of the vertex order failed");
  NPG_HIP(hipMemcpy(P->vperm, pv.data(), (size_t)P->V * sizeof(int32_t), hipMemcpyHostToDevice));
  return NPG_OK;
}

// Both directions of the pruned search for the plan's own points.
hipError_t npg_launch_nn_pruned(const npg_plan* P, const float4* xhat, int32_t* a, float* da, int32_t* b,
                                float* db) {
  const NpgNn* N = P->nn;
  hipLaunchKernelGGL(k_nn_gather, dim3(nblk((int64_t)P->T * N->ntv, 4)), dim3(256), 0, P->stream, xhat, N->perm_v,
                     P->V, P->T, N->ntv, N->xs, N->vbox);
  NnArgs rows{N->vgrp, N->n_vgrp, N->xs, N->vx_off, N->perm_v, 0, N->pts_s, P->d_off, N->perm_p, 1,
              N->pbox, N->ptile_off, a, da};
  NnArgs cols{N->pgrp, N->n_pgrp, N->pts_s, P->d_off, N->perm_p, 1, N->xs, N->vx_off, N->perm_v, 0,
              N->vbox, N->vtile_off, b, db};
  const int wpb = std::max(1, std::min(4, P->nn_threads / 64));
  for (int d = 0; d < 2; ++d) {
    const NnArgs& A = d == 0 ? rows : cols;
    const int tl = d == 0 ? N->tl_rows : N->tl_cols;
    const unsigned grid = nblk(A.ngroups, wpb);
#define NPG_NN_LAUNCH(W, TLV)                                                                                \
  do {                                                                                                       \
    if (d == 0) hipLaunchKernelGGL((k_nn_pruned<W, kNQV, TLV>), dim3(grid), dim3(W), 0, P->stream, A);      \
    else hipLaunchKernelGGL((k_nn_pruned<W, kNQP, TLV>), dim3(grid), dim3(W), 0, P->stream, A);             \
  } while (0)
#define NPG_NN_TL(W)                            \
  switch (tl) {                                 \
    case 2: NPG_NN_LAUNCH(W, 2); break;         \
    case 4: NPG_NN_LAUNCH(W, 4); break;         \
    case 8: NPG_NN_LAUNCH(W, 8); break;         \
    default: NPG_NN_LAUNCH(W, 16); break;       \
  }
    switch (wpb) {
      case 1: NPG_NN_TL(64); break;
      case 2: NPG_NN_TL(128); break;
      default: NPG_NN_TL(256); break;
    }
#undef NPG_NN_TL
#undef NPG_NN_LAUNCH
  }
  return hipGetLastError();
}
