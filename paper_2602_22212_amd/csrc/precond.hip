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
//   k_cg_update:  r -= alpha A p (A p recomputed from p) and r.r; x is
//                 updated every second iteration only, with both pending terms
//                 (x += alpha_{k-1} p_{k-1}, then x += alpha_k p_k: the same
//                 float32 operations in the same order as one update per
//                 iteration), the older direction read from the other
//                 ping-pong buffer
// i.e. 7.5 vector passes per iteration on average (r, p, p | p, r, r, and
// every second iteration p_{k-1}, x, x) instead of 10 with A p stored. A
// term left pending when a system stops is added by a flush pass.
// A p = p + lam * sum over existing neighbours of (p_n - p_nb): sums of
// differences keep the float32 rounding proportional to |A p|, not to
// (1 + 12 lam)|p|.
//
// Large grids (R >= 100) are walked in z-columns (registers carry the z
// neighbours, lane shifts the x neighbours, LDS the y neighbours); small grids
// in contiguous node chunks. Work-groups are dispatched largest grid first.
#include <algorithm>

#include "internal.h"

namespace {

constexpr int kB = 256;       // threads per work-group
constexpr int kPer = 8;       // nodes per thread
constexpr int kChunk = kB * kPer;

// per (system, channel) scalars: 0 rr, 1 bb, 2 pq, 3 alpha, 4 beta, 5 active, 6 iterations,
// 7 alpha of the pending x term (0 when none)
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

// Logical work-group of this launch. Work-groups go to the 8 XCDs in turn
// (launch index mod 8); every XCD takes kXG consecutive logical blocks in a
// row, so tiles that are y-neighbours (and share halo rows) run on the same
// XCD and meet in its L2. The block table is walked in reverse, so the
// largest grids (last in the table) are dispatched first. Launches are padded
// to a multiple of 8 kXG work-groups; the padding returns at once.
constexpr int kXCD = 8, kXG = 16;
__device__ __forceinline__ int logical_block(int nb) {
  const int b = (int)blockIdx.x;
  const int round = b / kXCD;
  const int fwd = (round / kXG) * (kXCD * kXG) + (b % kXCD) * kXG + round % kXG;
  const int lb = nb - 1 - fwd;
  return lb >= 0 ? lb : -1;
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

// r -= alpha A p; rr partial. XM = 1: also x += alpha_prev p_prev, then
// x += alpha p (the term of the previous iteration and this one's).
template <int XM, int FV, int F = (FV < 0 ? -FV : FV)>
__device__ void update_body(const NpgGrid& g, const FastDiv& fR, const FastDiv& fR2, int64_t n0, const double* st,
                            int s, float* x, float* r, const float* p, const float* p_prev, double* part, int blk) {
  float al[F], ap[F];
#pragma unroll
  for (int c = 0; c < F; ++c) {
    al[c] = (float)st[(s * 4 + c) * kS + 3];
    ap[c] = (float)st[(s * 4 + c) * kS + 7];
  }
  const float lam = g.lam;
  const float* pb = p + g.poff;
  double acc[4] = {0, 0, 0, 0};
  for (int k = 0; k < kPer; ++k) {
    const int64_t n = n0 + k * kB + threadIdx.x;
    if (n >= g.nodes) break;
    const Nb nb = neighbours((uint32_t)n, g.R, fR, fR2);
    const int64_t e = g.poff + n * F;
    float pc[F], lap[F], rc[F];
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
    if (XM) {
      float xc[F], pp[F];
      Vec<FV>::load(x + e, xc);
      Vec<FV>::load(p_prev + e, pp);
#pragma unroll
      for (int c = 0; c < F; ++c) xc[c] = fmaf(al[c], pc[c], fmaf(ap[c], pp[c], xc[c]));
      Vec<FV>::store(x + e, xc);
    }
    Vec<FV>::load(r + e, rc);
#pragma unroll
    for (int c = 0; c < F; ++c) {
      rc[c] = fmaf(-al[c], fmaf(lam, lap[c], pc[c]), rc[c]);
      acc[c] += (double)rc[c] * (double)rc[c];
    }
    Vec<FV>::store(r + e, rc);
  }
  store_partials<F>(acc, part, blk);
}

// ---- z-column walks for large grids -----------------------------------------
// A work-group owns a kTX x kTY block of (x, y) columns and the z range
// [z0, z1); wave w walks row y0 + w, one column per lane. Per plane:
//   z neighbours   registers (the previous and next plane's operand)
//   x neighbours   the neighbouring lanes (DPP wave shifts); only lanes 0 and
//                  kTX-1 load the node beyond the tile
//   y neighbours   the other waves' rows through a triple-buffered LDS plane;
//                  the first and last wave also load the halo row beyond the
//                  tile
// Loads run one plane ahead of the arithmetic (the next plane's operand two).
// Missing neighbours (grid boundary) and lanes/rows past the grid edge are
// clamped to the nearest node inside, whose difference then contributes 0.
constexpr int kZmR = 100;  // grids with R >= kZmR, F = 4 and 16-byte alignment
constexpr int kTX = 64, kTY = 4, kZS = 64;
static_assert(kTX * kTY == kB, "one wave per tile row");

__device__ __forceinline__ bool use_zm(const NpgGrid& g) { return g.R >= kZmR && g.F == 4 && (g.poff % 4) == 0; }

struct Tile {
  int x0, y0, z0, z1;
};
__device__ __forceinline__ Tile unpack_tile(int64_t v) {
  return Tile{(int)(v & 0xffff), (int)((v >> 16) & 0xffff), (int)((v >> 32) & 0xffff), (int)((v >> 48) & 0xffff)};
}
inline int64_t pack_tile(int x0, int y0, int z0, int z1) {
  return (int64_t)x0 | ((int64_t)y0 << 16) | ((int64_t)z0 << 32) | ((int64_t)z1 << 48);
}

__device__ __forceinline__ float4 f4fma(float4 a, const float (&s)[4], float4 b) {  // a*s + b per channel
  return make_float4(fmaf(s[0], a.x, b.x), fmaf(s[1], a.y, b.y), fmaf(s[2], a.z, b.z), fmaf(s[3], a.w, b.w));
}
__device__ __forceinline__ void f4lap(float4& acc, const float4& c, const float4& n) {
  acc.x += c.x - n.x;
  acc.y += c.y - n.y;
  acc.z += c.z - n.z;
  acc.w += c.w - n.w;
}

// Wave-wide lane shifts by one (DPP wave_shr:1 / wave_shl:1). The lane
// without a source (0, resp. 63) keeps its own `edge` value.
__device__ __forceinline__ float dpp_from_left(float edge, float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                               __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_from_right(float edge, float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                               __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ float4 from_left(const float4& edge, const float4& v) {
  return make_float4(dpp_from_left(edge.x, v.x), dpp_from_left(edge.y, v.y), dpp_from_left(edge.z, v.z),
                     dpp_from_left(edge.w, v.w));
}
__device__ __forceinline__ float4 from_right(const float4& edge, const float4& v) {
  return make_float4(dpp_from_right(edge.x, v.x), dpp_from_right(edge.y, v.y), dpp_from_right(edge.z, v.z),
                     dpp_from_right(edge.w, v.w));
}

struct Raw1 {
  float4 a;
};
struct Raw2 {
  float4 a, b;
};
struct NoExtra {};

// Raw loads of one plane: the lane's node, the node beyond the tile (lanes 0
// and kTX-1 only), the halo row (first and last wave only) and the extra
// per-node data the body needs.
template <typename RAW, typename EX>
struct ZPlane {
  RAW c, e, h;
  EX ex;
};

// LD(node) loads the raw stencil operand, OP(raw) forms it, LDC(node) loads
// the body's extra data; BODY(node, lap, operand, extra) runs at every node
// of the grid inside the tile. Every thread of the work-group must call this
// (it synchronises the work-group once per plane).
template <typename RAW, typename EX, typename LD, typename LDC, typename OP, typename BODY>
__device__ __forceinline__ void zm_walk(const NpgGrid& g, const Tile& t, LD ld, LDC ldc, OP op, BODY body) {
  __shared__ float4 sh[3][kTY + 2][kTX];
  const int R = g.R;
  const int64_t R2 = (int64_t)R * R;
  const int lane = threadIdx.x & (kTX - 1), w = threadIdx.x / kTX;
  const int x = t.x0 + lane, y = t.y0 + w;
  const int xe = min(x, R - 1), ye = min(y, R - 1);
  const bool inside = x < R && y < R;
  const int oxm = xe > 0 ? -1 : 0, oxp = xe < R - 1 ? 1 : 0;
  const bool edge_lane = lane == 0 || lane == kTX - 1;
  const int64_t de = lane == 0 ? oxm : oxp;
  const bool halo = w == 0 || w == kTY - 1;
  const int hy = w == 0 ? max(t.y0 - 1, 0) : min(t.y0 + kTY, R - 1);
  const int hrow = w == 0 ? 0 : kTY + 1;
  const int64_t dh = (int64_t)(hy - ye) * R;
  auto load_plane = [&](int64_t m, ZPlane<RAW, EX>& P) {
    P.c = ld(m);
    P.ex = ldc(m);
    if (edge_lane) P.e = ld(m + de);
    if (halo) P.h = ld(m + dh);
  };
  int64_t n = (int64_t)t.z0 * R2 + (int64_t)ye * R + xe;
  ZPlane<RAW, EX> A = {}, B = {};
  load_plane(n, A);
  float4 cur = op(A.c), edge = op(A.e);
  EX ex = A.ex;
  sh[t.z0 % 3][w + 1][lane] = cur;
  if (halo) sh[t.z0 % 3][hrow][lane] = op(A.h);
  float4 prev = t.z0 > 0 ? op(ld(n - R2)) : cur;
  load_plane(t.z0 + 1 < R ? n + R2 : n, A);
  for (int z = t.z0; z < t.z1; ++z, n += R2) {
    const int64_t n1 = z + 1 < R ? n + R2 : n;
    load_plane(z + 2 < R ? n1 + R2 : n1, B);
    // plane z+1 (clamped to z at the top face, where it then adds 0)
    const float4 nxt = op(A.c), nedge = op(A.e);
    sh[(z + 1) % 3][w + 1][lane] = nxt;
    if (halo) sh[(z + 1) % 3][hrow][lane] = op(A.h);
    __syncthreads();
    float4 lap = make_float4(0.f, 0.f, 0.f, 0.f);
    f4lap(lap, cur, from_left(edge, cur));
    f4lap(lap, cur, from_right(edge, cur));
    f4lap(lap, cur, sh[z % 3][w][lane]);
    f4lap(lap, cur, sh[z % 3][w + 2][lane]);
    f4lap(lap, cur, prev);
    f4lap(lap, cur, nxt);
    if (inside) body(n, lap, cur, ex);
    prev = cur;
    cur = nxt;
    edge = nedge;
    ex = A.ex;
    A = B;
  }
}

__device__ void zm_init(const NpgGrid& g, const Tile& t, const float* b, float* x, float* r, float* p, double* part,
                        int blk) {
  const int R = g.R;
  const int64_t R2 = (int64_t)R * R;
  const int xx = t.x0 + (int)(threadIdx.x & (kTX - 1));
  const int yy = t.y0 + (int)(threadIdx.x / kTX);
  const float4* B = reinterpret_cast<const float4*>(b + g.poff);
  float4* X = reinterpret_cast<float4*>(x + g.poff);
  float4* Rr = reinterpret_cast<float4*>(r + g.poff);
  float4* Pp = reinterpret_cast<float4*>(p + g.poff);
  double acc[4] = {0, 0, 0, 0};
  if (xx < R && yy < R)
    for (int z = t.z0; z < t.z1; ++z) {
      const int64_t n = (int64_t)z * R2 + (int64_t)yy * R + xx;
      const float4 v = B[n];
      X[n] = make_float4(0.f, 0.f, 0.f, 0.f);
      Rr[n] = v;
      Pp[n] = v;
      acc[0] += (double)v.x * v.x;
      acc[1] += (double)v.y * v.y;
      acc[2] += (double)v.z * v.z;
      acc[3] += (double)v.w * v.w;
    }
  store_partials<4>(acc, part, blk);
}

__device__ void zm_dir_ap(const NpgGrid& g, const Tile& t, const double* st, int s, const float* r,
                          const float* p_old, float* p_new, double* part, int blk) {
  float be[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) be[c] = (float)st[(s * 4 + c) * kS + 4];
  const float lam = g.lam;
  const float4* Rr = reinterpret_cast<const float4*>(r + g.poff);
  const float4* Po = reinterpret_cast<const float4*>(p_old + g.poff);
  float4* Pn = reinterpret_cast<float4*>(p_new + g.poff);
  double acc[4] = {0, 0, 0, 0};
  zm_walk<Raw2, NoExtra>(
      g, t, [&](int64_t n) { return Raw2{Po[n], Rr[n]}; }, [&](int64_t) { return NoExtra{}; },
      [&](const Raw2& v) { return f4fma(v.a, be, v.b); },
      [&](int64_t n, const float4& lap, const float4& pn, const NoExtra&) {
        acc[0] += (double)pn.x * (double)fmaf(lam, lap.x, pn.x);
        acc[1] += (double)pn.y * (double)fmaf(lam, lap.y, pn.y);
        acc[2] += (double)pn.z * (double)fmaf(lam, lap.z, pn.z);
        acc[3] += (double)pn.w * (double)fmaf(lam, lap.w, pn.w);
        Pn[n] = pn;
      });
  store_partials<4>(acc, part, blk);
}

struct Raw3 {
  float4 a, b, c;
};

template <int XM>
__device__ void zm_update(const NpgGrid& g, const Tile& t, const double* st, int s, float* x, float* r,
                          const float* p, const float* p_prev, double* part, int blk) {
  float al[4], ap[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    al[c] = (float)st[(s * 4 + c) * kS + 3];
    ap[c] = (float)st[(s * 4 + c) * kS + 7];
  }
  const float lam = g.lam;
  const float4* Pp = reinterpret_cast<const float4*>(p + g.poff);
  const float4* Pq = reinterpret_cast<const float4*>(p_prev + g.poff);
  float4* X = reinterpret_cast<float4*>(x + g.poff);
  float4* Rr = reinterpret_cast<float4*>(r + g.poff);
  double acc[4] = {0, 0, 0, 0};
  auto r_update = [&](int64_t n, const float4& lap, const float4& pc, float4 rv) {
    rv.x = fmaf(-al[0], fmaf(lam, lap.x, pc.x), rv.x);
    rv.y = fmaf(-al[1], fmaf(lam, lap.y, pc.y), rv.y);
    rv.z = fmaf(-al[2], fmaf(lam, lap.z, pc.z), rv.z);
    rv.w = fmaf(-al[3], fmaf(lam, lap.w, pc.w), rv.w);
    Rr[n] = rv;
    acc[0] += (double)rv.x * rv.x;
    acc[1] += (double)rv.y * rv.y;
    acc[2] += (double)rv.z * rv.z;
    acc[3] += (double)rv.w * rv.w;
  };
  if (XM) {
    zm_walk<Raw1, Raw3>(
        g, t, [&](int64_t n) { return Raw1{Pp[n]}; }, [&](int64_t n) { return Raw3{X[n], Rr[n], Pq[n]}; },
        [&](const Raw1& v) { return v.a; },
        [&](int64_t n, const float4& lap, const float4& pc, const Raw3& e) {
          float4 xv = e.a;
          const float4 pq = e.c;
          xv.x = fmaf(al[0], pc.x, fmaf(ap[0], pq.x, xv.x));
          xv.y = fmaf(al[1], pc.y, fmaf(ap[1], pq.y, xv.y));
          xv.z = fmaf(al[2], pc.z, fmaf(ap[2], pq.z, xv.z));
          xv.w = fmaf(al[3], pc.w, fmaf(ap[3], pq.w, xv.w));
          X[n] = xv;
          r_update(n, lap, pc, e.b);
        });
  } else {
    zm_walk<Raw1, Raw1>(
        g, t, [&](int64_t n) { return Raw1{Pp[n]}; }, [&](int64_t n) { return Raw1{Rr[n]}; },
        [&](const Raw1& v) { return v.a; },
        [&](int64_t n, const float4& lap, const float4& pc, const Raw1& e) { r_update(n, lap, pc, e.a); });
  }
  store_partials<4>(acc, part, blk);
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

__global__ __launch_bounds__(kB) void k_cg_init(const NpgGrid* __restrict__ G, int nb, const int* __restrict__ blk_sys,
                                                const int64_t* __restrict__ blk_start, const float* b, float* x,
                                                float* __restrict__ r, float* __restrict__ p,
                                                double* __restrict__ part) {
  const int blk = logical_block(nb);
  if (blk < 0) return;
  const int s = blk_sys[blk];
  const NpgGrid g = G[s];
  if (use_zm(g)) {
    zm_init(g, unpack_tile(blk_start[blk]), b, x, r, p, part, blk);
    return;
  }
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
  if (use_zm(g)) {
    zm_dir_ap(g, unpack_tile(blk_start[blk]), st, s, r, p_old, p_new, part, blk);
    return;
  }
  NPG_F_SWITCH(g, (dir_ap_body<FF>(g, dv.r[s], dv.r2[s], blk_start[blk], st, s, r, p_old, p_new, part, blk)));
}

template <int XM>
__global__ __launch_bounds__(kB) void k_cg_update(const NpgGrid* __restrict__ G, Divs dv, int nb, const int* __restrict__ blk_sys,
                                                  const int64_t* __restrict__ blk_start,
                                                  const int* __restrict__ active, const double* __restrict__ st,
                                                  float* __restrict__ x, float* __restrict__ r,
                                                  const float* __restrict__ p, const float* __restrict__ p_prev,
                                                  double* __restrict__ part) {
  const int blk = logical_block(nb);
  if (blk < 0) return;
  const int s = blk_sys[blk];
  if (!active[s]) return;
  const NpgGrid g = G[s];
  if (use_zm(g)) {
    zm_update<XM>(g, unpack_tile(blk_start[blk]), st, s, x, r, p, p_prev, part, blk);
    return;
  }
  NPG_F_SWITCH(g, (update_body<XM, FF>(g, dv.r[s], dv.r2[s], blk_start[blk], st, s, x, r, p, p_prev, part, blk)));
}

// The pending x term of one system: x += alpha_pending p (flat, F channels).
__global__ void k_cg_flush(float* __restrict__ x, const float* __restrict__ p, int64_t n, int F, float a0, float a1,
                           float a2, float a3) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e % F);
  const float a = c == 0 ? a0 : (c == 1 ? a1 : (c == 2 ? a2 : a3));
  x[e] = fmaf(a, p[e], x[e]);
}
// Per system (one work-group each): reduce the block partials in order and
// update the scalars. mode 0: after init (rr, bb); 1: alpha = rr / pq;
// 2: beta = rr_new / rr and the convergence test (defer: the update left
// this iteration's x term pending).
constexpr int kR = 1024;
__global__ __launch_bounds__(kR) void k_cg_reduce(const NpgGrid* __restrict__ G, const int* __restrict__ sys_blk0,
                                                  int* __restrict__ active, const double* __restrict__ part,
                                                  double* __restrict__ st, int mode, double rtol, int defer) {
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
      S[7] = 0.0;
      S[5] = v > 0.0 ? 1.0 : 0.0;
    } else if (mode == 1) {
      S[3] = (S[5] != 0.0 && v > 0.0) ? S[0] / v : 0.0;
    } else {
      S[7] = defer ? S[3] : 0.0;  // this iteration's x term, when the update left it pending
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

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
inline unsigned xcd_grid(int nb) { return (unsigned)((nb + kXCD * kXG - 1) / (kXCD * kXG) * (kXCD * kXG)); }

}  // namespace

npg_status npg_cg_setup(npg_plan* P) {
  NpgCG& C = P->cg;
  std::vector<int> bsys;
  std::vector<int64_t> bstart;
  std::vector<int> s0(P->n_sys + 1);
  for (int s = 0; s < P->n_sys; ++s) {
    s0[s] = (int)bsys.size();
    const NpgGrid& g = P->g[s];
    if (g.R >= kZmR && g.F == 4 && g.poff % 4 == 0) {
      // z-marching tiles, z ranges interleaved so concurrently running
      // work-groups share planes
      for (int z0 = 0; z0 < g.R; z0 += kZS)
        for (int y0 = 0; y0 < g.R; y0 += kTY)
          for (int x0 = 0; x0 < g.R; x0 += kTX) {
            bsys.push_back(s);
            bstart.push_back(pack_tile(x0, y0, z0, std::min(g.R, z0 + kZS)));
          }
    } else {
      for (int64_t n = 0; n < g.nodes; n += kChunk) {
        bsys.push_back(s);
        bstart.push_back(n);
      }
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

// Solve (I + lam L) x = b for every system (b and x distinct buffers in the
// grid-block layout). The iteration count of each system goes to iters (if
// not NULL). Iteration k writes p_k into C.q for even k and into C.p for odd
// k; the update of an even iteration leaves its x term pending (p_k stays in
// C.q: later iterations write only the blocks of systems still active), the
// next odd one adds both terms, and a term still pending when a system stops
// is added at the end.
static npg_status cg_solve(npg_plan* P, const float* b, float* x, int32_t* iters, bool* capped, double* relres) {
  NpgCG& C = P->cg;
  hipStream_t s = P->stream;
  const int nb = C.n_blocks;
  const dim3 grid(xcd_grid(nb)), blk(kB);
  Divs dv;
  for (int sy = 0; sy < P->n_sys; ++sy) {
    dv.r[sy] = make_fastdiv((uint32_t)P->g[sy].R);
    dv.r2[sy] = make_fastdiv((uint32_t)P->g[sy].R * (uint32_t)P->g[sy].R);
  }
  hipLaunchKernelGGL(k_cg_init, grid, blk, 0, s, P->d_g, nb, C.blk_sys, C.blk_start, b, x, C.r, C.p, C.part);
  hipLaunchKernelGGL(k_cg_reduce, dim3(P->n_sys), dim3(kR), 0, s, P->d_g, C.sys_blk0, C.active, C.part, C.st, 0,
                     P->cfg.cg_rtol, 0);
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
      const bool odd = ((it + k) & 1) != 0;
      // optional profiling: event pairs around both streaming kernels,
      // resolved after the step (no synchronisation here)
      const bool prof = P->prof_cg && P->prof_n + 4 <= (int)P->prof_ev.size();
      if (prof) NPG_HIP(hipEventRecord(P->prof_ev[P->prof_n], s));
      hipLaunchKernelGGL(k_cg_dir_ap, grid, blk, 0, s, P->d_g, dv, nb, C.blk_sys, C.blk_start, C.active, C.st, C.r,
                         pa, pb, C.part);
      if (prof) NPG_HIP(hipEventRecord(P->prof_ev[P->prof_n + 1], s));
      std::swap(pa, pb);  // pa = p_k, pb = p_{k-1}
      hipLaunchKernelGGL(k_cg_reduce, dim3(P->n_sys), dim3(kR), 0, s, P->d_g, C.sys_blk0, C.active, C.part, C.st, 1,
                         P->cfg.cg_rtol, 0);
      if (prof) NPG_HIP(hipEventRecord(P->prof_ev[P->prof_n + 2], s));
      if (odd)
        hipLaunchKernelGGL(k_cg_update<1>, grid, blk, 0, s, P->d_g, dv, nb, C.blk_sys, C.blk_start, C.active, C.st,
                           x, C.r, pa, pb, C.part);
      else
        hipLaunchKernelGGL(k_cg_update<0>, grid, blk, 0, s, P->d_g, dv, nb, C.blk_sys, C.blk_start, C.active, C.st,
                           x, C.r, pa, pb, C.part);
      if (prof) {
        NPG_HIP(hipEventRecord(P->prof_ev[P->prof_n + 3], s));
        P->prof_n += 4;
      }
      hipLaunchKernelGGL(k_cg_reduce, dim3(P->n_sys), dim3(kR), 0, s, P->d_g, C.sys_blk0, C.active, C.part, C.st, 2,
                         P->cfg.cg_rtol, (int)!odd);
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
    const NpgGrid& g = P->g[sy];
    double m = 0;
    for (int c = 0; c < g.F; ++c) m = stv[(sy * 4 + c) * kS + 6] > m ? stv[(sy * 4 + c) * kS + 6] : m;
    if (iters) iters[sy] = (int32_t)m;
    // final relative residual ||r|| / ||b|| in float64, the largest over the channels
    double rel = 0.0;
    float pend[4] = {0.f, 0.f, 0.f, 0.f};
    bool any = false;
    for (int c = 0; c < g.F; ++c) {
      const double* S = stv.data() + (sy * 4 + c) * kS;
      const double v = S[1] > 0.0 ? sqrt(S[0] / S[1]) : 0.0;
      rel = v > rel ? v : rel;
      pend[c] = (float)S[7];
      any |= S[7] != 0.0;
    }
    relres[sy] = rel;
    if (any) {
      const int64_t n = g.nodes * g.F;
      hipLaunchKernelGGL(k_cg_flush, dim3(nblk(n, 256)), dim3(256), 0, s, x + g.poff, C.q + g.poff, n, g.F, pend[0],
                         pend[1], pend[2], pend[3]);
    }
    // algorithmic traffic of this solve: 6 vector passes (x, r, p read and
    // written) per iteration over the grid's R^3 F float32 unknowns
    P->cg_alg_bytes += m * 6.0 * (double)g.nodes * g.F * 4.0;
    P->cg_iters_sum += (int64_t)m;
  }
  NPG_HIP(hipGetLastError());
  return NPG_OK;
}

npg_status npg_run_precond_cg(npg_plan* P, float* grad, int32_t* iters) {
  bool capped = false;
  P->cg_alg_bytes = 0.0;
  P->cg_iters_sum = 0;
  // y = A^-1 g into the workspace, then A^-1 y back into the gradient
  npg_status st = cg_solve(P, grad, P->cg.x, iters, &capped, P->cg_relres);
  if (st != NPG_OK) return st;
  st = cg_solve(P, P->cg.x, grad, iters ? iters + P->n_sys : nullptr, &capped, P->cg_relres + P->n_sys);
  if (st != NPG_OK) return st;
  return capped ? NPG_ENOTCONV : NPG_OK;
}
