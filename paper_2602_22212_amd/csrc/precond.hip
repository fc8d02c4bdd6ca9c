// Sobolev preconditioning of the grid gradients (Sec. 3.5): g~ = (I+lam L)^-2 g
// per grid and feature channel, L the 6-neighbour lattice Laplacian with free
// boundary, as two conjugate-gradient solves from a zero start, each stopped
// at ||r|| <= rtol ||b||. With cg_mg = 1 every solve is preconditioned by one
// multigrid V-cycle per iteration (z = M^-1 r; p = z + beta p, rho = r.z; see
// "multigrid V-cycle preconditioner" below), otherwise plain CG (z = r).
//
// All grids (every position level and the normal grid) iterate together:
// each launch covers the blocks of every system still active, through a
// block -> (system, first node) table. Vectors are float32 in the parameter
// layout ([node][F] per grid); inner products are float64, reduced per wave
// and then per system in a fixed order (bitwise reproducible).
//
// One CG iteration is two streaming kernels (plus the V-cycle):
//   k_cg_dir_ap:  p = z + beta p, and p.(A p) with A p formed on the fly from
//                 z and the old p at the 6 neighbours (p is written, A p is not)
//   k_cg_update:  r -= alpha A p (A p recomputed from p) and r.r
// and every kCgDirs iterations one pass (k_cg_xacc) adds the window's x
// terms, x += alpha_j p_j in iteration order (the same float32 operations in
// the same order as one update per iteration), the directions kept in a ring
// of kCgDirs buffers: 6 + (kCgDirs + 2) / kCgDirs vector passes per iteration
// (z, p, p | p, r, r, and the x pass) instead of 10 with A p stored and x
// updated every iteration. The terms left when a system stops are added by
// a flush pass.
// A p = p + lam * sum over existing neighbours of (p_n - p_nb): sums of
// differences keep the float32 rounding proportional to |A p|, not to
// (1 + 12 lam)|p|.
//
// Large grids (R >= 100) are walked in z-columns (registers carry the z
// neighbours, lane shifts the x neighbours, LDS the y neighbours); small grids
// in contiguous node chunks. Work-groups are dispatched largest grid first.
#include <algorithm>
#include <climits>
#include <functional>
#include <thread>

#include "internal.h"

#define NPG_TRY_ST(call)                  \
  do {                                    \
    const npg_status st_ = (call);        \
    if (st_ != NPG_OK) return st_;        \
  } while (0)

namespace {

constexpr int kB = 256;       // threads per work-group
constexpr int kPer = 8;       // nodes per thread
constexpr int kChunk = kB * kPer;

// per (system, channel) scalars: 0 rho (r.z with the V-cycle, else r.r), 1 bb, 2 rr, 3 alpha,
// 4 beta, 5 active, 6 iterations, 7 unused
constexpr int kS = 8;
constexpr float kMgOmegaW = 0.85f;  // Jacobi damping of the V-cycle (kMgOmega below)
constexpr int kR_THREADS = 1024, kR_WAVES = kR_THREADS / 64;  // reduction work-group

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
// to a multiple of 8 kXG work-groups; the padding returns at once. A launch
// may cover the range [lo, nb) of the table (one group of grids).
constexpr int kXCD = 8, kXG = 16;
__device__ __forceinline__ int logical_block(int nb, int lo = 0) {
  const int b = (int)blockIdx.x;
  const int round = b / kXCD;
  const int fwd = (round / kXG) * (kXCD * kXG) + (b % kXCD) * kXG + round % kXG;
  const int lb = nb - 1 - fwd;
  return lb >= lo ? lb : -1;
}

// Block partials of F channels, part[blk*4 + c]: wave sums, then the
// waves in order (NT threads per work-group).
template <int F, int NT = kB>
__device__ __forceinline__ void store_partials(double (&acc)[4], double* part, int blk) {
  constexpr int NW = NT / 64;
  __shared__ double ws[NW][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < F; ++c) {
    double s = wave_sum(acc[c]);
    if (lane == 0) ws[wave][c] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < F) {
    const int c = threadIdx.x;
    double v = ws[0][c];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += ws[w][c];
    part[(int64_t)blk * 4 + c] = v;
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

// r = p = b and the b.b partials. x is not written: the first window's x
// pass writes it without reading it, or k_cg_flush when a solve stops before
// the first window ends.
template <int FV, int F = (FV < 0 ? -FV : FV)>
__device__ void init_body(const NpgGrid& g, int64_t n0, const float* b, float* r, float* p, double* part, int blk) {
  double acc[4] = {0, 0, 0, 0};
  for (int k = 0; k < kPer; ++k) {
    const int64_t n = n0 + k * kB + threadIdx.x;
    if (n >= g.nodes) break;
    const int64_t e = g.poff + n * F;
    float v[F];
    Vec<FV>::load(b + e, v);
#pragma unroll
    for (int c = 0; c < F; ++c) acc[c] += (double)v[c] * (double)v[c];
    Vec<FV>::store(r + e, v);
    Vec<FV>::store(p + e, v);
  }
  store_partials<F>(acc, part, blk);
}

// p_new = r + beta p_old; pq partial with A p_new formed from r and p_old at
// the neighbours. p_old and p_new are different ring slots, so no
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

// r = r_in - alpha A p (r_in: r, or b in the first iteration); rr partial.
// x is not touched: k_cg_xacc adds the terms of kCgDirs iterations at once.
template <int FV, int F = (FV < 0 ? -FV : FV)>
__device__ void update_body(const NpgGrid& g, const FastDiv& fR, const FastDiv& fR2, int64_t n0, const double* st,
                            int s, const float* r_in, float* r, const float* p, double* part, int blk) {
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
    Vec<FV>::load(r_in + e, rc);
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
constexpr int kTX = 64, kTY = 4;  // tile columns; the z planes per tile are the plan's cg_zs (even)
static_assert(kTX * kTY == kB, "one wave per tile row");

__host__ __device__ __forceinline__ bool use_zm(const NpgGrid& g) { return g.R >= kZmR && g.F == 4 && (g.poff % 4) == 0; }

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

// Streaming float4 access with the nontemporal hint, for the streams of a
// grid's vectors that no other work-group reads back soon (every grid vector
// of the large grids far exceeds the caches).
typedef float npg_nt4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ldnt(const float4* p) {
  const npg_nt4 v = __builtin_nontemporal_load(reinterpret_cast<const npg_nt4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void stnt(float4* p, float4 v) {
  __builtin_nontemporal_store(npg_nt4{v.x, v.y, v.z, v.w}, reinterpret_cast<npg_nt4*>(p));
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

// LD(node, column, plane) loads the raw stencil operand, OP(raw, column,
// plane) forms it, LDC(node) loads the body's extra data; BODY(node, lap,
// operand, extra, plane) runs at every node of the grid inside the tile.
// The column argument says which of the thread's three columns is meant (0
// its own, 1 the x neighbour beyond the tile, 2 the halo row), so callers can
// precompute per-column data. Every thread of the work-group must call this
// (it synchronises the work-group once per plane). POST(z) runs in every
// thread after the plane's BODY (it may synchronise the work-group).
//
// The raw loads run DEPTH-1 planes ahead of the arithmetic (DEPTH = 2 to 4
// plane buffers whose roles rotate; the loop is unrolled by DEPTH so no buffer
// is copied) and are formed by OP only when their plane is reached, so they stay
// in flight across the work-group barriers of DEPTH-1 planes.
template <typename RAW, typename EX, int DEPTH = 2, typename LD, typename LDC, typename OP, typename BODY,
          typename POST>
__device__ __forceinline__ void zm_walk_post(const NpgGrid& g, const Tile& t, LD ld, LDC ldc, OP op, BODY body,
                                             POST post) {
  static_assert(DEPTH >= 2 && DEPTH <= 4, "planes loaded ahead of the arithmetic: 2 to 4");
  __shared__ float4 sh[3][kTY + 2][kTX];
  const int R = g.R;
  const int64_t R2 = (int64_t)R * R;
  const int lane = threadIdx.x & (kTX - 1), w = threadIdx.x / kTX;
  const int x = t.x0 + lane, y = t.y0 + w;
  const int xe = min(x, R - 1), ye = min(y, R - 1);
  const bool inside = x < R && y < R;
  const int oxm = xe > 0 ? -1 : 0, oxp = xe < R - 1 ? 1 : 0;
  const bool edge_lane = lane == 0 || lane == kTX - 1;
  const bool halo = w == 0 || w == kTY - 1;
  const int hy = w == 0 ? max(t.y0 - 1, 0) : min(t.y0 + kTY, R - 1);
  const int hrow = w == 0 ? 0 : kTY + 1;
  // every thread issues all three loads (threads without an x neighbour or
  // halo row beyond the tile reload their own node), so no load sits behind a
  // branch and the wait for a plane never has to cover later planes' loads
  const int64_t nxy = (int64_t)ye * R + xe;
  const int64_t de = edge_lane ? (lane == 0 ? oxm : oxp) : 0;
  const int64_t dh = halo ? (int64_t)(hy - ye) * R : 0;
  auto load_plane = [&](int zz, ZPlane<RAW, EX>& P) {  // zz already clamped to [0, R)
    const int64_t m = (int64_t)zz * R2 + nxy;
    P.c = ld(m, 0, zz);
    P.ex = ldc(m);
    P.e = ld(m + de, 1, zz);
    P.h = ld(m + dh, 2, zz);
  };
  int64_t n = (int64_t)t.z0 * R2 + nxy;
  ZPlane<RAW, EX> A, B, C, D;
  load_plane(t.z0, A);
  float4 cur = op(A.c, 0, t.z0), edge = op(A.e, 1, t.z0);
  EX ex = A.ex;
  sh[t.z0 % 3][w + 1][lane] = cur;
  if (halo) sh[t.z0 % 3][hrow][lane] = op(A.h, 2, t.z0);
  float4 prev = t.z0 > 0 ? op(ld(n - R2, 0, t.z0 - 1), 0, t.z0 - 1) : cur;
  load_plane(min(t.z0 + 1, R - 1), B);
  if (DEPTH >= 3) load_plane(min(t.z0 + 2, R - 1), C);
  if (DEPTH == 4) load_plane(min(t.z0 + 3, R - 1), D);
  // Pn holds plane z+1 (clamped to z at the top face, where it then adds 0);
  // Pl held plane z and receives plane z+DEPTH.
  auto step = [&](int z, ZPlane<RAW, EX>& Pn, ZPlane<RAW, EX>& Pl) {
    const int z1c = min(z + 1, R - 1);
    load_plane(min(z + DEPTH, R - 1), Pl);
    const float4 nxt = op(Pn.c, 0, z1c), nedge = op(Pn.e, 1, z1c);
    sh[(z + 1) % 3][w + 1][lane] = nxt;
    if (halo) sh[(z + 1) % 3][hrow][lane] = op(Pn.h, 2, z1c);
    __syncthreads();
    float4 lap = make_float4(0.f, 0.f, 0.f, 0.f);
    f4lap(lap, cur, from_left(edge, cur));
    f4lap(lap, cur, from_right(edge, cur));
    f4lap(lap, cur, sh[z % 3][w][lane]);
    f4lap(lap, cur, sh[z % 3][w + 2][lane]);
    f4lap(lap, cur, prev);
    f4lap(lap, cur, nxt);
    if (inside) body(n, lap, cur, ex, z);
    post(z);
    prev = cur;
    cur = nxt;
    edge = nedge;
    ex = Pn.ex;
    n += R2;
  };
  if (DEPTH == 2) {
    for (int z = t.z0; z < t.z1; z += 2) {
      step(z, B, A);
      if (z + 1 >= t.z1) break;
      step(z + 1, A, B);
    }
  } else if (DEPTH == 3) {
    for (int z = t.z0; z < t.z1; z += 3) {
      step(z, B, A);
      if (z + 1 >= t.z1) break;
      step(z + 1, C, B);
      if (z + 2 >= t.z1) break;
      step(z + 2, A, C);
    }
  } else {
    for (int z = t.z0; z < t.z1; z += 4) {
      step(z, B, A);
      if (z + 1 >= t.z1) break;
      step(z + 1, C, B);
      if (z + 2 >= t.z1) break;
      step(z + 2, D, C);
      if (z + 3 >= t.z1) break;
      step(z + 3, A, D);
    }
  }
}
template <typename RAW, typename EX, typename LD, typename LDC, typename OP, typename BODY>
__device__ __forceinline__ void zm_walk(const NpgGrid& g, const Tile& t, LD ld, LDC ldc, OP op, BODY body) {
  zm_walk_post<RAW, EX>(
      g, t, [&](int64_t m, int, int) { return ld(m); }, ldc, [&](const RAW& v, int, int) { return op(v); },
      [&](int64_t n, const float4& lap, const float4& c, const EX& e, int) { body(n, lap, c, e); }, [](int) {});
}

// Per-column data of a z-column walk for the V-cycle's finest level: the
// Jacobi factor w / (1 + lam deg) of the thread's three columns (own, x
// neighbour beyond the tile, halo row) on interior and on boundary planes,
// and the parent row offset (x/2, y/2) on the level below.
struct ZmCols {
  float fin[3], fbd[3];
  int pxy[3];
};
__device__ __forceinline__ ZmCols zm_cols(const Tile& t, int R, float lam, int nh) {
  const int lane = threadIdx.x & (kTX - 1), w = threadIdx.x / kTX;
  const int xe = min(t.x0 + lane, R - 1), ye = min(t.y0 + w, R - 1);
  const int xs[3] = {xe, lane == 0 ? max(xe - 1, 0) : min(xe + 1, R - 1), xe};
  const int ys[3] = {ye, ye, w == 0 ? max(t.y0 - 1, 0) : min(t.y0 + kTY, R - 1)};
  ZmCols c;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int d = ((xs[s] > 0) + (xs[s] < R - 1)) + ((ys[s] > 0) + (ys[s] < R - 1));
    c.fin[s] = kMgOmegaW * __builtin_amdgcn_rcpf(fmaf(lam, (float)(d + 2), 1.f));
    c.fbd[s] = kMgOmegaW * __builtin_amdgcn_rcpf(fmaf(lam, (float)(d + 1), 1.f));
    c.pxy[s] = (ys[s] >> 1) * nh + (xs[s] >> 1);
  }
  return c;
}

// b.b partials and r = p = b (not for a split grid of the V-cycle form: the
// V-cycle reads b itself, the first update reads r from b, the start's
// prolongation writes the first direction and the start's finest restriction
// forms the b.b partials). x is not written (see init_body).
__device__ void zm_init(const NpgGrid& g, const Tile& t, const float* b, float* r, float* p, double* part, int blk) {
  const int R = g.R;
  const int64_t R2 = (int64_t)R * R;
  const int xx = t.x0 + (int)(threadIdx.x & (kTX - 1));
  const int yy = t.y0 + (int)(threadIdx.x / kTX);
  const float4* B = reinterpret_cast<const float4*>(b + g.poff);
  float4* Rr = reinterpret_cast<float4*>(r + g.poff);
  float4* Pp = reinterpret_cast<float4*>(p + g.poff);
  double acc[4] = {0, 0, 0, 0};
  if (xx < R && yy < R)
    for (int z = t.z0; z < t.z1; ++z) {
      const int64_t n = (int64_t)z * R2 + (int64_t)yy * R + xx;
      const float4 v = B[n];
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

// p.(A p) of a direction the V-cycle's finest prolongation already formed
// (the large grids of the multigrid form): p is only read.
__device__ void zm_pap(const NpgGrid& g, const Tile& t, const float* p, double* part, int blk) {
  const float lam = g.lam;
  const float4* Pp = reinterpret_cast<const float4*>(p + g.poff);
  double acc[4] = {0, 0, 0, 0};
  zm_walk<Raw1, NoExtra>(
      g, t, [&](int64_t n) { return Raw1{Pp[n]}; }, [&](int64_t) { return NoExtra{}; },
      [&](const Raw1& v) { return v.a; },
      [&](int64_t, const float4& lap, const float4& pn, const NoExtra&) {
        acc[0] += (double)pn.x * (double)fmaf(lam, lap.x, pn.x);
        acc[1] += (double)pn.y * (double)fmaf(lam, lap.y, pn.y);
        acc[2] += (double)pn.z * (double)fmaf(lam, lap.z, pn.z);
        acc[3] += (double)pn.w * (double)fmaf(lam, lap.w, pn.w);
      });
  store_partials<4>(acc, part, blk);
}


__device__ void zm_update(const NpgGrid& g, const Tile& t, const double* st, int s, const float* r_in, float* r,
                          const float* p, double* part, int blk) {
  float al[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) al[c] = (float)st[(s * 4 + c) * kS + 3];
  const float lam = g.lam;
  const float4* Pp = reinterpret_cast<const float4*>(p + g.poff);
  const float4* Ri = reinterpret_cast<const float4*>(r_in + g.poff);
  float4* Rr = reinterpret_cast<float4*>(r + g.poff);
  double acc[4] = {0, 0, 0, 0};
  zm_walk<Raw1, Raw1>(
      g, t, [&](int64_t n) { return Raw1{Pp[n]}; }, [&](int64_t n) { return Raw1{ldnt(Ri + n)}; },
      [&](const Raw1& v) { return v.a; },
      [&](int64_t n, const float4& lap, const float4& pc, const Raw1& e) {
        float4 rv = e.a;
        rv.x = fmaf(-al[0], fmaf(lam, lap.x, pc.x), rv.x);
        rv.y = fmaf(-al[1], fmaf(lam, lap.y, pc.y), rv.y);
        rv.z = fmaf(-al[2], fmaf(lam, lap.z, pc.z), rv.z);
        rv.w = fmaf(-al[3], fmaf(lam, lap.w, pc.w), rv.w);
        stnt(Rr + n, rv);
        acc[0] += (double)rv.x * rv.x;
        acc[1] += (double)rv.y * rv.y;
        acc[2] += (double)rv.z * rv.z;
        acc[3] += (double)rv.w * rv.w;
      });
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

// sys_split (NULL without the V-cycle): the systems whose direction the
// V-cycle's finest prolongation forms and whose b.b partials the start's
// finest restriction forms (see zm_init); their work-groups return at once.
__global__ __launch_bounds__(kB) void k_cg_init(const NpgGrid* __restrict__ G, int nb, int lo,
                                                const int* __restrict__ blk_sys,
                                                const int64_t* __restrict__ blk_start, const float* __restrict__ b,
                                                float* __restrict__ r, float* __restrict__ p,
                                                const int* __restrict__ sys_split, double* __restrict__ part) {
  const int blk = logical_block(nb, lo);
  if (blk < 0) return;
  const int s = blk_sys[blk];
  const NpgGrid g = G[s];
  if (use_zm(g)) {
    // split: nothing to store, and the start's V-cycle forms the b.b partials
    if (!(sys_split && sys_split[s])) zm_init(g, unpack_tile(blk_start[blk]), b, r, p, part, blk);
    return;
  }
  NPG_F_SWITCH(g, (init_body<FF>(g, blk_start[blk], b, r, p, part, blk)));
}

struct Divs {
  FastDiv r[NPG_MAX_SYS], r2[NPG_MAX_SYS];
};

__global__ __launch_bounds__(kB) void k_cg_dir_ap(const NpgGrid* __restrict__ G, Divs dv, int nb, int lo,
                                                  const int* __restrict__ blk_sys,
                                                  const int64_t* __restrict__ blk_start,
                                                  const int* __restrict__ active, const double* __restrict__ st,
                                                  const float* __restrict__ r, const float* __restrict__ p_old,
                                                  float* __restrict__ p_new, double* __restrict__ part, int mgp) {
  const int blk = logical_block(nb, lo);
  if (blk < 0) return;
  const int s = blk_sys[blk];
  if (!active[s]) return;
  const NpgGrid g = G[s];
  if (use_zm(g)) {
    if (mgp) zm_pap(g, unpack_tile(blk_start[blk]), p_new, part, blk);
    else zm_dir_ap(g, unpack_tile(blk_start[blk]), st, s, r, p_old, p_new, part, blk);
    return;
  }
  NPG_F_SWITCH(g, (dir_ap_body<FF>(g, dv.r[s], dv.r2[s], blk_start[blk], st, s, r, p_old, p_new, part, blk)));
}

// r_b: the right-hand side in the first iteration of a solve (r is read from
// it, r = b not having been stored), NULL later (r updated in place).
__global__ __launch_bounds__(kB) void k_cg_update(const NpgGrid* __restrict__ G, Divs dv, int nb, int lo,
                                                  const int* __restrict__ blk_sys,
                                                  const int64_t* __restrict__ blk_start,
                                                  const int* __restrict__ active, const double* __restrict__ st,
                                                  const float* __restrict__ r_b, float* __restrict__ r,
                                                  const float* __restrict__ p, double* __restrict__ part) {
  const int blk = logical_block(nb, lo);
  if (blk < 0) return;
  const int s = blk_sys[blk];
  if (!active[s]) return;
  const NpgGrid g = G[s];
  const float* r_in = r_b ? r_b : r;
  if (use_zm(g)) {
    zm_update(g, unpack_tile(blk_start[blk]), st, s, r_in, r, p, part, blk);
    return;
  }
  NPG_F_SWITCH(g, (update_body<FF>(g, dv.r[s], dv.r2[s], blk_start[blk], st, s, r_in, r, p, part, blk)));
}

// The ring of directions, by slot (passed by value).
struct Dirs {
  const float* p[kCgDirs];
};

// x of the systems [s_lo, s_hi) still iterating after iteration k (k + 1 a
// multiple of kCgDirs): x = fmaf(alpha_j, p_j, x) for the iterations j of
// the window k + 1 - kCgDirs .. k in order (ring slots 0 .. kCgDirs-1), from
// x = 0 (not read) for the first window: the float32 chain that one update
// per iteration would form.
__global__ __launch_bounds__(256) void k_cg_xacc(const NpgGrid* __restrict__ G, int s_lo, int s_hi,
                                                 const int* __restrict__ active, const double* __restrict__ ah,
                                                 int first, float* __restrict__ x, Dirs d) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int s = s_lo; s < s_hi; ++s) {
    if (!active[s]) continue;
    const NpgGrid g = G[s];
    float a[kCgDirs][4];
#pragma unroll
    for (int j = 0; j < kCgDirs; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) a[j][c] = c < g.F ? (float)ah[(s * 4 + c) * kCgDirs + j] : 0.f;
    if (g.F == 4 && g.poff % 4 == 0) {
      float4* X = reinterpret_cast<float4*>(x + g.poff);
      for (int64_t v = tid; v < g.nodes; v += stride) {
        float4 xv = first ? make_float4(0.f, 0.f, 0.f, 0.f) : ldnt(X + v);
#pragma unroll
        for (int j = 0; j < kCgDirs; ++j) {
          const float4 pv = ldnt(reinterpret_cast<const float4*>(d.p[j] + g.poff) + v);
          xv = make_float4(fmaf(a[j][0], pv.x, xv.x), fmaf(a[j][1], pv.y, xv.y), fmaf(a[j][2], pv.z, xv.z),
                           fmaf(a[j][3], pv.w, xv.w));
        }
        stnt(X + v, xv);
      }
      continue;
    }
    for (int64_t v = tid; v < g.nodes; v += stride)
      for (int c = 0; c < g.F; ++c) {
        const int64_t e = g.poff + v * g.F + c;
        float xv = first ? 0.f : x[e];
#pragma unroll
        for (int j = 0; j < kCgDirs; ++j) xv = fmaf(a[j][c], d.p[j][e], xv);
        x[e] = xv;
      }
  }
}

// The end of a solve, from its scalars on the device: a system that took
// `taken` iterations (scalar 6, the largest over its channels) has had the
// terms of its first floor(taken / kCgDirs) windows added to x by k_cg_xacc;
// the rest, iterations kCgDirs floor(taken / kCgDirs) .. taken-1, are added
// here in order, from x = 0 (not read) when no window was added. One launch
// covers the systems [s_lo, s_hi).
__global__ __launch_bounds__(256) void k_cg_flush(const NpgGrid* __restrict__ G, int s_lo, int s_hi,
                                                  const double* __restrict__ st, const double* __restrict__ ah,
                                                  float* __restrict__ x, Dirs d) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int s = s_lo; s < s_hi; ++s) {
    const NpgGrid g = G[s];
    double tk = 0.0;
    for (int c = 0; c < g.F; ++c) tk = fmax(tk, st[(s * 4 + c) * kS + 6]);
    const int taken = (int)tk;
    const int done = taken / kCgDirs * kCgDirs, pend = taken - done;
    const bool stored = done > 0;
    if (stored && pend == 0) continue;
    float a[kCgDirs][4];
#pragma unroll
    for (int j = 0; j < kCgDirs; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) a[j][c] = c < g.F && j < pend ? (float)ah[(s * 4 + c) * kCgDirs + j] : 0.f;
    if (g.F == 4 && g.poff % 4 == 0) {  // one node (float4) per thread and pass
      float4* X = reinterpret_cast<float4*>(x + g.poff);
      for (int64_t v = tid; v < g.nodes; v += stride) {
        float4 xv = stored ? ldnt(X + v) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int j = 0; j < kCgDirs; ++j) {
          if (j >= pend) break;
          const float4 pv = ldnt(reinterpret_cast<const float4*>(d.p[j] + g.poff) + v);
          xv = make_float4(fmaf(a[j][0], pv.x, xv.x), fmaf(a[j][1], pv.y, xv.y), fmaf(a[j][2], pv.z, xv.z),
                           fmaf(a[j][3], pv.w, xv.w));
        }
        stnt(X + v, xv);
      }
      continue;
    }
    for (int64_t v = tid; v < g.nodes; v += stride)
      for (int c = 0; c < g.F; ++c) {
        const int64_t e = g.poff + v * g.F + c;
        float xv = stored ? x[e] : 0.f;
#pragma unroll
        for (int j = 0; j < kCgDirs; ++j) {
          if (j >= pend) break;
          xv = fmaf(a[j][c], d.p[j][e], xv);
        }
        x[e] = xv;
      }
  }
}

// After a fixed number of launched iterations: sets `bit` in *state when
// one of the systems [s_lo, s_hi) is still iterating (one thread; an atomic
// OR, as the groups of grids check on their own streams).
__global__ void k_cg_done(const int* __restrict__ active, int s_lo, int s_hi, int* __restrict__ state, int bit) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int any = 0;
  for (int s = s_lo; s < s_hi; ++s) any |= active[s];
  if (any) atomicOr(state, bit);
}

// Sum of the block partials [b0, b1) of part per channel, in a fixed order
// (strided per thread, then per wave, then the waves in order); the result
// is valid in thread 0.
__device__ __forceinline__ void reduce_range(const double* part, int b0, int b1, double (*red)[kR_WAVES],
                                             double (&out)[4]) {
  double acc[4] = {0, 0, 0, 0};
  for (int b = b0 + threadIdx.x; b < b1; b += kR_THREADS) {
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
  for (int c = 0; c < 4; ++c) {
    double v = 0.0;
    for (int w = 0; w < kR_WAVES; ++w) v += red[c][w];
    out[c] = v;
  }
}

// Per system (one work-group each): reduce the block partials in order and
// update the scalars (S[0] rho = r.z, or r.r without the V-cycle; S[2] r.r).
// mode 0: after init (bb, rho); 1: alpha = rho / pq, also kept in ring slot
// `slot` of ah (the x terms are added later, see k_cg_xacc); 2: beta =
// rho_new / rho and the convergence test on r.r. part2 (NULL without the V-cycle): the r.z partials, blocks
// [blk0_2[s], blk0_2[s+1]) of system s, plus (part3 not NULL) the blocks
// [r3[s].x, r3[s].y) of part3: for the large grids of the multigrid form, r.z
// is the finest restriction's term plus the level-1 term (see k_mg_up0).
// filter: -1 every system, 0 only systems without that split, 1 only those
// with it (sys_split[s]).
__global__ __launch_bounds__(kR_THREADS) void k_cg_reduce(const NpgGrid* __restrict__ G,
                                                          const int* __restrict__ sys_blk0, int* __restrict__ active,
                                                          const double* __restrict__ part,
                                                          const double* __restrict__ part2,
                                                          const int* __restrict__ blk0_2, double* __restrict__ st,
                                                          int mode, double rtol, double* __restrict__ ah, int slot,
                                                          const double* __restrict__ part3, const int2* __restrict__ r3,
                                                          const int* __restrict__ sys_split, int filter, int s0) {
  const int s = s0 + (int)blockIdx.x;
  if (mode != 0 && !active[s]) return;
  if (filter >= 0 && sys_split && (sys_split[s] != 0) != (filter != 0)) return;
  __shared__ double red[4][kR_WAVES], red2[4][kR_WAVES], red3[4][kR_WAVES];
  const int F = G[s].F;
  double vv[4], rho[4];
  reduce_range(part, sys_blk0[s], sys_blk0[s + 1], red, vv);
  if (part2 && mode != 1) {
    reduce_range(part2, blk0_2[s], blk0_2[s + 1], red2, rho);
    if (part3) {
      double rc[4];
      reduce_range(part3, r3[s].x, r3[s].y, red3, rc);
      for (int c = 0; c < 4; ++c) rho[c] += rc[c];
    }
  } else {
    for (int c = 0; c < 4; ++c) rho[c] = vv[c];
  }
  if (threadIdx.x != 0) return;
  int any = 0;
  for (int c = 0; c < F; ++c) {
    const double v = vv[c];
    double* S = st + (s * 4 + c) * kS;
    if (mode == 0) {
      S[0] = rho[c];
      S[1] = v;
      S[2] = v;
      S[3] = 0.0;
      S[4] = 0.0;
      S[6] = 0.0;
      S[7] = 0.0;
      S[5] = v > 0.0 ? 1.0 : 0.0;
    } else if (mode == 1) {
      S[3] = (S[5] != 0.0 && v > 0.0) ? S[0] / v : 0.0;
      ah[(s * 4 + c) * kCgDirs + slot] = S[3];  // this iteration's x term, added later
    } else {
      if (S[5] != 0.0) {
        S[4] = S[0] > 0.0 ? rho[c] / S[0] : 0.0;
        S[0] = rho[c];
        S[2] = v;
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

// ---- multigrid V-cycle preconditioner ----------------------------------------
// Level l of a system aggregates 2^l x 2^l x 2^l fine nodes (fewer at the far
// faces): n_l = ceil(R / 2^l) nodes per axis, extent e(i) = min(2^l, R - 2^l i)
// fine nodes along an axis. With piecewise-constant prolongation P the
// Galerkin operator P^T A P of A = I + lam L is again "mass + lam weighted
// Laplacian": mass = ex ey ez, the weight of a face = its area in fine nodes
// (ey ez across x, ...). One V-cycle (preconditioner input b, output x):
// x0 = w D^-1 b; restrict b - A x0 to the next level; recurse; x = x0 + P e;
// x += w D^-1 (b - A x). A system coarsens until a level has at most kMgMinN
// nodes per axis or it has kMgMaxLev coarse levels; its coarsest level takes
// the same two damped Jacobi steps from zero with no coarser correction
// (x0 = w D^-1 b, x = x0 + w D^-1 (b - A x0)). The mass term of a level grows
// 8x per level and its Laplacian weights 4x, so D^-1 A is close to the
// identity three levels down (lam / 8 at most 0.85 at the headline's 6.83):
// two sweeps there give the iteration counts of a hierarchy down to 8^3 with
// four sweeps at its bottom, in four fewer launches per cycle. Smoothing before
// and after is the same symmetric Jacobi step and the restriction is P^T, so
// the preconditioner is symmetric and positive definite
// (w < 1 < 2 / rho(D^-1 A)).
constexpr float kMgOmega = kMgOmegaW;
constexpr int kMgMinN = 8;
constexpr int kMgMaxLev = 3;
constexpr int kMgB = 256;

struct MgLvl {
  int64_t off;  // float offset of the level's [node][F] array
  int n, s, R, F;
  float lam;
  FastDiv fn, fn2;  // division by n and n^2
};
struct MgTask {
  int sys, blk0;  // system; first block of the system in its launch
  int64_t nodes;  // threads of the system
  MgLvl lo, hi;   // finer and coarser level (the coarsest launch uses lo)
  // fast path of a level with uniform aggregates (F = 4, 16-byte aligned):
  // mass s^3, lam times the face weight s^2, and the divisions of the
  // prolongation's thread index (one thread per pair of x-adjacent nodes:
  // ceil(n/2) x n x n threads)
  int fast;
  float mass, lw;
  FastDiv fx, fx2;
  int zm0;  // a finest restriction: runs in k_mg_down0 over the CG work-group table
  int rz1;  // prolongation onto level 1 of such a grid: b1 . e1 partials (the coarse r.z term)
};

__device__ __forceinline__ int mg_ext(int i, const MgLvl& L) { return min(L.s, L.R - L.s * i); }

// Mass, face weights and neighbour mask (bit d: neighbour d exists; order
// -x, +x, -y, +y, -z, +z) of node (i, j, k), and its Jacobi diagonal.
struct MgNode {
  float mass, wx, wy, wz, diag;
  int mask;
};
__device__ __forceinline__ MgNode mg_node(int i, int j, int k, const MgLvl& L) {
  const float ex = (float)mg_ext(i, L), ey = (float)mg_ext(j, L), ez = (float)mg_ext(k, L);
  MgNode m;
  m.mass = ex * ey * ez;
  m.wx = ey * ez;
  m.wy = ex * ez;
  m.wz = ex * ey;
  m.mask = (i > 0) | ((i < L.n - 1) << 1) | ((j > 0) << 2) | ((j < L.n - 1) << 3) | ((k > 0) << 4) |
           ((k < L.n - 1) << 5);
  const float nx = (float)((i > 0) + (i < L.n - 1)), ny = (float)((j > 0) + (j < L.n - 1)),
              nz = (float)((k > 0) + (k < L.n - 1));
  m.diag = m.mass + L.lam * (m.wx * nx + m.wy * ny + m.wz * nz);
  return m;
}
__device__ __forceinline__ void mg_load(const float* p, int F, float (&v)[4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) v[c] = c < F ? p[c] : 0.f;
}
__device__ __forceinline__ int64_t mg_idx(int i, int j, int k, int n) { return ((int64_t)k * n + j) * n + i; }

// x0 = w b / d at node (i, j, k) of level L (b: the level's array)
__device__ __forceinline__ void mg_x0(const float* b, const MgLvl& L, int i, int j, int k, float (&x)[4]) {
  const MgNode m = mg_node(i, j, k, L);
  mg_load(b + L.off + mg_idx(i, j, k, L.n) * L.F, L.F, x);
  const float f = kMgOmega * __builtin_amdgcn_rcpf(m.diag);
#pragma unroll
  for (int c = 0; c < 4; ++c) x[c] *= f;
}

// Logical block of a launch of nblk blocks (grid padded to a multiple of 8):
// work-groups go to the 8 XCDs in turn, and XCD x takes the x-th contiguous
// eighth of the logical blocks in order, so the neighbour rows and planes a
// block reads were fetched into the same L2 by the blocks just before it.
// -1 for the padding.
__device__ __forceinline__ int mg_block(int nblk, int lo = 0) {  // blocks [lo, nblk)
  const int n = nblk - lo;
  const int per = (n + kXCD - 1) / kXCD;
  const int b = (int)blockIdx.x;
  const int L = (b % kXCD) * per + b / kXCD;
  return L < n ? lo + L : -1;
}
// The first block of each task of one launch (tasks sorted by blk0, at most
// one per system; unused slots hold INT_MAX), passed by value so the lookup
// of a block's task reads kernel arguments only, all at once.
constexpr int kMgTaskMax = NPG_MAX_SYS;
struct MgBlk0 {
  int b[kMgTaskMax];
};
__device__ __forceinline__ int mg_task_of(const MgBlk0& B, int blk) {
  int t = 0;
#pragma unroll
  for (int q = 1; q < kMgTaskMax; ++q) t += blk >= B.b[q] ? 1 : 0;
  return t;
}

__device__ __forceinline__ void mg_coords(int64_t m, const MgLvl& L, int& i, int& j, int& k) {
  k = (int)fdiv((uint32_t)m, L.fn2);
  const uint32_t rem = (uint32_t)m - (uint32_t)k * L.fn2.d;
  j = (int)fdiv(rem, L.fn);
  i = (int)(rem - (uint32_t)j * (uint32_t)L.n);
}

// ---- levels with uniform aggregates (R a multiple of the extent s) and F = 4:
// float4 loads, 32-bit node indices, mass s^3 and face weight s^2 for every
// node, Jacobi factor w / (s^3 + lam s^2 deg) from the node's degree
__device__ __forceinline__ int mg_deg1(int i, int n) { return (i > 0) + (i < n - 1); }
__device__ __forceinline__ float mg_f(const MgTask* tk, int d) {
  return kMgOmega * __builtin_amdgcn_rcpf(fmaf(tk->lw, (float)d, tk->mass));
}
__device__ __forceinline__ float4 f4sub(float4 a, float4 b) { return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w); }
__device__ __forceinline__ float4 f4add(float4 a, float4 b) { return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
__device__ __forceinline__ float4 f4scale(float s, float4 a) { return make_float4(s * a.x, s * a.y, s * a.z, s * a.w); }
__device__ __forceinline__ float4 f4axpy(float s, float4 a, float4 y) {  // y + s a
  return make_float4(fmaf(s, a.x, y.x), fmaf(s, a.y, y.y), fmaf(s, a.z, y.z), fmaf(s, a.w, y.w));
}

// Restriction, one coarse node: the sum over the block's children of
// b - A x0 equals sum(b - mass x0) minus lam w times the differences across
// the block's outer faces (the inner edges cancel).
__device__ __forceinline__ void mg_down_u4(const MgTask* tk, const float* __restrict__ bl, float* __restrict__ bh,
                                           int m) {
  const MgLvl& lo = tk->lo;
  const MgLvl& hi = tk->hi;
  const int R = lo.n;
  int I, J, K;
  mg_coords(m, hi, I, J, K);
  const float4* B = reinterpret_cast<const float4*>(bl + lo.off);
  const float nlw = -tk->lw, mass = tk->mass;
  const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 acc = zero;
  // all 8 children and their 24 outer neighbours, branch-free: indices
  // clamped into the grid, absent nodes masked to 0; every load is issued
  // before the first is used
  float4 ld[8][4];
#pragma unroll
  for (int c3 = 0; c3 < 8; ++c3) {
    const int cx = c3 & 1, cy = (c3 >> 1) & 1, cz = c3 >> 2;
    const int ic = min(2 * I + cx, R - 1), jc = min(2 * J + cy, R - 1), kc = min(2 * K + cz, R - 1);
    const int n = (kc * R + jc) * R + ic;
    const int ox = cx ? ic + 1 : ic - 1, oy = cy ? jc + 1 : jc - 1, oz = cz ? kc + 1 : kc - 1;
    const int oxc = ox >= 0 && ox < R ? ox : ic, oyc = oy >= 0 && oy < R ? oy : jc, ozc = oz >= 0 && oz < R ? oz : kc;
    ld[c3][0] = B[n];
    ld[c3][1] = B[n + (oxc - ic)];
    ld[c3][2] = B[n + (oyc - jc) * R];
    ld[c3][3] = B[n + (ozc - kc) * R * R];
  }
#pragma unroll
  for (int c3 = 0; c3 < 8; ++c3) {
    const int cx = c3 & 1, cy = (c3 >> 1) & 1, cz = c3 >> 2;
    const int i = 2 * I + cx, j = 2 * J + cy, k = 2 * K + cz;
    const bool valid = i < R && j < R && k < R;
    const int ic = min(i, R - 1), jc = min(j, R - 1), kc = min(k, R - 1);
    const int di = mg_deg1(ic, R), dj = mg_deg1(jc, R), dk = mg_deg1(kc, R);
    const int ox = cx ? ic + 1 : ic - 1, oy = cy ? jc + 1 : jc - 1, oz = cz ? kc + 1 : kc - 1;
    const bool vx = valid && ox >= 0 && ox < R, vy = valid && oy >= 0 && oy < R, vz = valid && oz >= 0 && oz < R;
    const int oxc = vx ? ox : ic, oyc = vy ? oy : jc, ozc = vz ? oz : kc;
    const float4 bc = ld[c3][0], bx = ld[c3][1], by = ld[c3][2], bz = ld[c3][3];
    const float4 xc = f4scale(mg_f(tk, di + dj + dk), bc);
    float4 t = f4axpy(-mass, xc, bc);
    t = f4axpy(vx ? nlw : 0.f, f4sub(xc, f4scale(mg_f(tk, mg_deg1(oxc, R) + dj + dk), bx)), t);
    t = f4axpy(vy ? nlw : 0.f, f4sub(xc, f4scale(mg_f(tk, di + mg_deg1(oyc, R) + dk), by)), t);
    t = f4axpy(vz ? nlw : 0.f, f4sub(xc, f4scale(mg_f(tk, di + dj + mg_deg1(ozc, R)), bz)), t);
    acc = f4add(acc, valid ? t : zero);
  }
  reinterpret_cast<float4*>(bh + hi.off)[m] = acc;
}

// Prolongation and post-smoothing for the x-adjacent node pair (2I, 2I+1)
// of row (j, k), which shares one parent in x; r.z of the pair into acc on
// the finest level.
__device__ __forceinline__ void mg_up_u4(const MgTask* tk, const float* __restrict__ bl,
                                         const float* __restrict__ eh, float* __restrict__ out, int m,
                                         double (&acc)[4]) {
  const MgLvl& lo = tk->lo;
  const MgLvl& hi = tk->hi;
  const int R = lo.n, nh = hi.n;
  const int k = (int)fdiv((uint32_t)m, tk->fx2);
  const uint32_t rem = (uint32_t)m - (uint32_t)k * tk->fx2.d;
  const int j = (int)fdiv(rem, tk->fx);
  const int I = (int)(rem - (uint32_t)j * tk->fx.d);
  const float4* B = reinterpret_cast<const float4*>(bl + lo.off);
  const float4* E = reinterpret_cast<const float4*>(eh + hi.off);
  float4* Z = reinterpret_cast<float4*>(out + lo.off);
  const float lw = tk->lw, mass = tk->mass;
  const bool fine = lo.s == 1, ident = fine && lo.lam == 0.f;
  // x = w D^-1 b + P e at node (a, b2, c2). A neighbour index clamped into the
  // grid lands on the node itself, whose x is bitwise the same, so an absent
  // neighbour adds exactly 0 and every load can be issued unconditionally.
  // The 12 nodes (the pair, its two x neighbours and the y and z neighbours of
  // each of the pair) are loaded before any is used.
  const int i0 = 2 * I, i1 = min(2 * I + 1, R - 1);  // i1 = i0 when the pair has one node
  const int jm = max(j - 1, 0), jp = min(j + 1, R - 1), km = max(k - 1, 0), kp = min(k + 1, R - 1);
  const int na[12] = {i0, i1, max(i0 - 1, 0), min(i1 + 1, R - 1), i0, i0, i0, i0, i1, i1, i1, i1};
  const int nb2[12] = {j, j, j, j, jm, jp, j, j, jm, jp, j, j};
  const int nc2[12] = {k, k, k, k, k, k, km, kp, k, k, km, kp};
  float4 vb[12], ve[12];
  const bool has_e = nh > 0;  // false on a coarsest level: no coarser correction
#pragma unroll
  for (int q = 0; q < 12; ++q) {
    vb[q] = B[(nc2[q] * R + nb2[q]) * R + na[q]];
    ve[q] = has_e ? E[((nc2[q] >> 1) * nh + (nb2[q] >> 1)) * nh + (na[q] >> 1)] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  float4 xv[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) {
    const int d = mg_deg1(na[q], R) + mg_deg1(nb2[q], R) + mg_deg1(nc2[q], R);
    xv[q] = f4add(f4scale(mg_f(tk, d), vb[q]), ve[q]);
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h == 1 && 2 * I + 1 >= R) break;
    const int i = h ? i1 : i0;
    const float4 xc = xv[h];
    // sum over the neighbours of (x_c - x_nb)
    float4 nb = f4add(f4sub(xc, h ? xv[0] : xv[2]), f4sub(xc, h ? xv[3] : xv[1]));
    nb = f4add(nb, f4add(f4sub(xc, xv[4 + 4 * h]), f4sub(xc, xv[5 + 4 * h])));
    nb = f4add(nb, f4add(f4sub(xc, xv[6 + 4 * h]), f4sub(xc, xv[7 + 4 * h])));
    const int n = (k * R + j) * R + i;
    const float4 bc = vb[h];
    const float4 ax = f4axpy(lw, nb, f4scale(mass, xc));
    // lam = 0 (A = I): the identity preconditioner
    const int dc = mg_deg1(i, R) + mg_deg1(j, R) + mg_deg1(k, R);
    const float4 z = ident ? bc : f4axpy(mg_f(tk, dc), f4sub(bc, ax), xc);
    Z[n] = z;
    if (fine || tk->rz1) {
      acc[0] += (double)bc.x * (double)z.x;
      acc[1] += (double)bc.y * (double)z.y;
      acc[2] += (double)bc.z * (double)z.z;
      acc[3] += (double)bc.w * (double)z.w;
    }
  }
}

// Restriction for any level (aggregate extents that differ at the upper
// faces, F < 4, unaligned arrays), in the same form as mg_down_u4: each child
// takes the mass term and the faces to its three outer neighbours (the faces
// between two children cancel in the sum), every load issued first with
// indices clamped into the grid, absent nodes masked to 0.
__device__ __forceinline__ void mg_down_gen(const MgTask* tk, const float* __restrict__ bl, float* __restrict__ bh,
                                            int64_t m) {
  const MgLvl& lo = tk->lo;
  const MgLvl& hi = tk->hi;
  const int R = lo.n;
  int I, J, K;
  mg_coords(m, hi, I, J, K);
  const float* Bb = bl + lo.off;
  float ld[8][4][4];
#pragma unroll
  for (int c3 = 0; c3 < 8; ++c3) {
    const int cx = c3 & 1, cy = (c3 >> 1) & 1, cz = c3 >> 2;
    const int ic = min(2 * I + cx, R - 1), jc = min(2 * J + cy, R - 1), kc = min(2 * K + cz, R - 1);
    const int ox = cx ? ic + 1 : ic - 1, oy = cy ? jc + 1 : jc - 1, oz = cz ? kc + 1 : kc - 1;
    const int oxc = ox >= 0 && ox < R ? ox : ic, oyc = oy >= 0 && oy < R ? oy : jc, ozc = oz >= 0 && oz < R ? oz : kc;
    mg_load(Bb + mg_idx(ic, jc, kc, R) * lo.F, lo.F, ld[c3][0]);
    mg_load(Bb + mg_idx(oxc, jc, kc, R) * lo.F, lo.F, ld[c3][1]);
    mg_load(Bb + mg_idx(ic, oyc, kc, R) * lo.F, lo.F, ld[c3][2]);
    mg_load(Bb + mg_idx(ic, jc, ozc, R) * lo.F, lo.F, ld[c3][3]);
  }
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c3 = 0; c3 < 8; ++c3) {
    const int cx = c3 & 1, cy = (c3 >> 1) & 1, cz = c3 >> 2;
    const int i = 2 * I + cx, j = 2 * J + cy, k = 2 * K + cz;
    const bool valid = i < R && j < R && k < R;
    const int ic = min(i, R - 1), jc = min(j, R - 1), kc = min(k, R - 1);
    const int ox = cx ? ic + 1 : ic - 1, oy = cy ? jc + 1 : jc - 1, oz = cz ? kc + 1 : kc - 1;
    const bool vx = valid && ox >= 0 && ox < R, vy = valid && oy >= 0 && oy < R, vz = valid && oz >= 0 && oz < R;
    const int oxc = vx ? ox : ic, oyc = vy ? oy : jc, ozc = vz ? oz : kc;
    const MgNode nd = mg_node(ic, jc, kc, lo);
    const float f = kMgOmega * __builtin_amdgcn_rcpf(nd.diag);
    const float fx = kMgOmega * __builtin_amdgcn_rcpf(mg_node(oxc, jc, kc, lo).diag);
    const float fy = kMgOmega * __builtin_amdgcn_rcpf(mg_node(ic, oyc, kc, lo).diag);
    const float fz = kMgOmega * __builtin_amdgcn_rcpf(mg_node(ic, jc, ozc, lo).diag);
    const float lx = vx ? lo.lam * nd.wx : 0.f, ly = vy ? lo.lam * nd.wy : 0.f, lz = vz ? lo.lam * nd.wz : 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float bc = ld[c3][0][c], xc = f * bc;
      float t = bc - nd.mass * xc;
      t -= lx * (xc - fx * ld[c3][1][c]);
      t -= ly * (xc - fy * ld[c3][2][c]);
      t -= lz * (xc - fz * ld[c3][3][c]);
      acc[c] += valid ? t : 0.f;
    }
  }
  float* o = bh + hi.off + m * hi.F;
  for (int c = 0; c < hi.F; ++c) o[c] = acc[c];
}

// Restriction of the smoothed residual: thread per coarse node J,
// bh[J] = sum over the children j of (b - A x0)[j], x0 = w D^-1 b.
__global__ __launch_bounds__(kMgB) void k_mg_down(const MgTask* __restrict__ T, MgBlk0 B0, int nblk, int lo,
                                                  const int* __restrict__ active, int check_active,
                                                  const float* __restrict__ bl, float* __restrict__ bh) {
  const int blk = mg_block(nblk, lo);
  if (blk < 0) return;
  const MgTask task = T[mg_task_of(B0, blk)];
  const MgTask* tk = &task;
  if (tk->zm0 || (check_active && !active[tk->sys])) return;
  const int64_t m = (int64_t)(blk - tk->blk0) * kMgB + threadIdx.x;
  if (m >= tk->nodes) return;
  if (tk->fast) {
    mg_down_u4(tk, bl, bh, (int)m);
    return;
  }
  mg_down_gen(tk, bl, bh, m);
}

// Prolongation and post-smoothing: thread per node j of the finer level,
// x = w D^-1 b + P e (at j and its neighbours), out[j] = x + w D^-1 (b - A x).
// On the finest level (out = z, b = r) the block partials of r.z per channel
// go to part. A system with lam = 0 (A = I) gets z = r.
// One node m of the finer level, any F and extents; adds r.z to acc (used
// on the finest level, where b = r and out = z).
__device__ __forceinline__ void mg_up_node(const MgTask* tk, const float* __restrict__ bl,
                                           const float* __restrict__ eh, float* __restrict__ out, int64_t m,
                                           double (&acc)[4]) {
  const MgLvl& lo = tk->lo;
  const MgLvl& hi = tk->hi;
  int i, j, k;
  mg_coords(m, lo, i, j, k);
  const MgNode nd = mg_node(i, j, k, lo);
  auto xat = [&](int a, int b2, int c2, float (&x)[4]) {
    mg_x0(bl, lo, a, b2, c2, x);
    if (hi.n == 0) return;  // a coarsest level: no coarser correction
    float e[4];
    mg_load(eh + hi.off + mg_idx(a >> 1, b2 >> 1, c2 >> 1, hi.n) * hi.F, hi.F, e);
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] += e[c];
  };
  float xc[4], bc[4], ax[4];
  xat(i, j, k, xc);
  mg_load(bl + lo.off + m * lo.F, lo.F, bc);
#pragma unroll
  for (int c = 0; c < 4; ++c) ax[c] = nd.mass * xc[c];
  const int di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
  const float w[6] = {nd.wx, nd.wx, nd.wy, nd.wy, nd.wz, nd.wz};
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    if (!(nd.mask & (1 << d))) continue;
    float xn[4];
    xat(i + di[d], j + dj[d], k + dk[d], xn);
#pragma unroll
    for (int c = 0; c < 4; ++c) ax[c] += lo.lam * w[d] * (xc[c] - xn[c]);
  }
  const float f = kMgOmega * __builtin_amdgcn_rcpf(nd.diag);
  const bool ident = lo.lam == 0.f;  // A = I: the identity preconditioner (CG then solves it in one step)
  float* o = out + lo.off + m * lo.F;
  for (int c = 0; c < lo.F; ++c) {
    const float v = ident ? bc[c] : xc[c] + f * (bc[c] - ax[c]);
    o[c] = v;
    acc[c] += (double)bc[c] * (double)v;
  }
}

// Prolongation and post-smoothing from level l+1 to l >= 1 (l = 0: k_mg_up0).
// part3 (may be NULL): the b . out partials of every block of an rz1 task.
__global__ __launch_bounds__(kMgB) void k_mg_up(const MgTask* __restrict__ T, MgBlk0 B0, int nblk, int lo,
                                                const int* __restrict__ active, int check_active,
                                                const float* __restrict__ bl, const float* __restrict__ eh,
                                                float* __restrict__ out, double* __restrict__ part3) {
  const int blk = mg_block(nblk, lo);
  if (blk < 0) return;
  const MgTask task = T[mg_task_of(B0, blk)];
  const MgTask* tk = &task;
  if (check_active && !active[tk->sys]) return;
  const int64_t m = (int64_t)(blk - tk->blk0) * kMgB + threadIdx.x;
  double acc[4] = {0, 0, 0, 0};
  if (m < tk->nodes) {
    if (tk->fast) mg_up_u4(tk, bl, eh, out, (int)m, acc);
    else mg_up_node(tk, bl, eh, out, m, acc);
  }
  if (part3 && tk->rz1) store_partials<4, kMgB>(acc, part3, blk);
}

// Restriction from the finest level of a large grid over its z-column tiles
// (each row read once): the residual b - A x0 of every node, x0 = w D^-1 b,
// summed over x-adjacent lanes, then y-adjacent waves (through LDS), then
// z-adjacent planes (registers), and written by the even lane of the even
// wave at the odd plane (or at the last plane of an odd-sized grid). Tiles
// start at even x, y and z, so no 2x2x2 block straddles two tiles.
// acc: the fine-level term of r.z, sum of x0 (2 b - A x0) (b . b when lam = 0,
// where the preconditioner is the identity); see k_mg_up0.
template <bool BB>
__device__ void mg_down0_zm(const NpgGrid& g, const Tile& t, const MgTask* tk, const float* __restrict__ r,
                            float* __restrict__ bh, double (&acc)[4], double (&bb)[4]) {
  __shared__ float4 ys[2][kTY / 2][kTX];
  const int R = g.R;
  const int nh = tk->hi.n;
  const float lam = g.lam;
  const float4* B = reinterpret_cast<const float4*>(r + g.poff);
  float4* H = reinterpret_cast<float4*>(bh + tk->hi.off);
  const int lane = threadIdx.x & (kTX - 1), w = threadIdx.x / kTX;
  const int x = t.x0 + lane, y = t.y0 + w;
  const ZmCols cols = zm_cols(t, R, lam, nh);
  float4 rs = make_float4(0.f, 0.f, 0.f, 0.f), zacc = rs;
  zm_walk_post<Raw1, Raw1, 4>(
      g, t,
      [&](int64_t m, int, int) { return Raw1{B[m]}; }, [&](int64_t m) { return Raw1{B[m]}; },
      [&](const Raw1& v, int s, int zz) {
        return f4scale((zz == 0 || zz == R - 1) ? cols.fbd[s] : cols.fin[s], v.a);
      },
      [&](int64_t, const float4& lap, const float4& xc, const Raw1& e, int) {
        rs = f4sub(e.a, f4axpy(lam, lap, xc));
        const float4 u = lam == 0.f ? e.a : xc;
        acc[0] += (double)u.x * ((double)e.a.x + (double)(lam == 0.f ? 0.f : rs.x));
        acc[1] += (double)u.y * ((double)e.a.y + (double)(lam == 0.f ? 0.f : rs.y));
        acc[2] += (double)u.z * ((double)e.a.z + (double)(lam == 0.f ? 0.f : rs.z));
        acc[3] += (double)u.w * ((double)e.a.w + (double)(lam == 0.f ? 0.f : rs.w));
        if (BB) {  // r = b at the start: b.b, in the order of the other grids' k_cg_init
          bb[0] += (double)e.a.x * e.a.x;
          bb[1] += (double)e.a.y * e.a.y;
          bb[2] += (double)e.a.z * e.a.z;
          bb[3] += (double)e.a.w * e.a.w;
        }
      },
      [&](int z) {
        float4 v = f4add(rs, make_float4(__shfl_xor(rs.x, 1), __shfl_xor(rs.y, 1), __shfl_xor(rs.z, 1),
                                         __shfl_xor(rs.w, 1)));
        rs = make_float4(0.f, 0.f, 0.f, 0.f);
        if (w & 1) ys[z & 1][w >> 1][lane] = v;
        __syncthreads();
        if (!(w & 1)) v = f4add(v, ys[z & 1][w >> 1][lane]);
        const bool last = (z & 1) || z + 1 >= R;
        if (z & 1) v = f4add(zacc, v);
        else zacc = v;
        if (last && !(w & 1) && !(lane & 1) && x < R && y < R)
          H[((z >> 1) * nh + (y >> 1)) * nh + (x >> 1)] = v;
      });
}

// The finest restriction of every grid, over the CG work-group table: the
// z-column walk (with the fine r.z term) for the large grids; for the others
// the grid's work-groups take its coarse nodes in turn (one thread per coarse
// node, as in k_mg_down), so the V-cycle needs no separate launch for them.
// BB (the start of a solve, r = b): the large grids' walks also write the
// b.b partials of the work-group into part (k_cg_init leaves them out).
template <bool BB>
__global__ __launch_bounds__(kB) void k_mg_down0(const NpgGrid* __restrict__ G, int nb, int lo,
                                                 const int* __restrict__ blk_sys,
                                                 const int64_t* __restrict__ blk_start,
                                                 const int* __restrict__ sys_blk0,
                                                 const int* __restrict__ active, int check_active,
                                                 const MgTask* __restrict__ T0, const float* __restrict__ r,
                                                 float* __restrict__ bh, double* __restrict__ part2,
                                                 double* __restrict__ part) {
  const int blk = logical_block(nb, lo);
  if (blk < 0) return;
  const int s = blk_sys[blk];
  if (check_active && !active[s]) return;
  const MgTask* tk = T0 + s;
  if (!tk->zm0) return;
  const NpgGrid g = G[s];
  if (!use_zm(g)) {
    const int b0 = sys_blk0[s], nbs = sys_blk0[s + 1] - b0;
    for (int64_t m = (int64_t)(blk - b0) * kB + threadIdx.x; m < tk->nodes; m += (int64_t)nbs * kB) {
      if (tk->fast) mg_down_u4(tk, r, bh, (int)m);
      else mg_down_gen(tk, r, bh, m);
    }
    return;
  }
  double acc[4] = {0, 0, 0, 0}, bb[4] = {0, 0, 0, 0};
  mg_down0_zm<BB>(g, unpack_tile(blk_start[blk]), tk, r, bh, acc, bb);
  store_partials<4>(acc, part2, blk);
  if (BB) store_partials<4>(bb, part, blk);
}

// Prolongation and post-smoothing onto the finest level (z = M^-1 r) over the
// CG work-group table: the z-column walk for the large grids (each row read
// once; x = w D^-1 r + P e formed as it is loaded), node chunks otherwise;
// r.z partials per work-group. T0: the system's task (system order).
//
// On the large grids z is never stored: the kernel writes the next search
// direction p = z + beta p_old itself (beta = 0 on the first call of a
// solve), which needs beta = r.z / rho_old before z exists. With x0 = w D^-1 r,
// the post-smoothed V-cycle is z = x0 + (I - w D^-1 A)(P e) + w D^-1 (r - A x0),
// e = C P^T (r - A x0) for the symmetric coarse-level cycle C, so
//   r.z = x0 . (2 r - A x0) + b1 . e1,   b1 = P^T (r - A x0), e1 = C b1:
// the first sum is formed by the finest restriction (k_mg_down0) and the second
// by the prolongation onto level 1 (k_mg_up, rz1 tasks), both before this
// kernel runs.
template <bool FIRST>
__device__ void mg_up0_zm(const NpgGrid& g, const Tile& t, const MgTask* tk, const float* __restrict__ r,
                          const float* __restrict__ eh, const float* __restrict__ p_old, float* __restrict__ p_new,
                          const float (&be)[4]) {
  const int R = g.R;
  const int nh = tk->hi.n;
  const float lam = g.lam;
  const float4* B = reinterpret_cast<const float4*>(r + g.poff);
  const float4* E = reinterpret_cast<const float4*>(eh + tk->hi.off);
  const float4* Po = reinterpret_cast<const float4*>(p_old + g.poff);
  float4* Pn = reinterpret_cast<float4*>(p_new + g.poff);
  const ZmCols cols = zm_cols(t, R, lam, nh);
  const int nh2 = nh * nh;
  zm_walk_post<Raw2, Raw2>(
      g, t,
      [&](int64_t m, int s, int zz) { return Raw2{B[m], E[(zz >> 1) * nh2 + cols.pxy[s]]}; },
      [&](int64_t m) { return Raw2{B[m], FIRST ? make_float4(0.f, 0.f, 0.f, 0.f) : ldnt(Po + m)}; },
      [&](const Raw2& v, int s, int zz) {
        const float f = (zz == 0 || zz == R - 1) ? cols.fbd[s] : cols.fin[s];
        return f4add(f4scale(f, v.a), v.b);
      },
      [&](int64_t n, const float4& lap, const float4& xc, const Raw2& e, int zz) {
        const float4 bc = e.a;
        const float4 ax = f4axpy(lam, lap, xc);
        const float f = (zz == 0 || zz == R - 1) ? cols.fbd[0] : cols.fin[0];
        const float4 zv = lam == 0.f ? bc : f4axpy(f, f4sub(bc, ax), xc);
        // p = z + beta p_old (p = z first); both directions streamed with the
        // nontemporal hint (the grid's directions far exceed the caches)
        stnt(Pn + n, FIRST ? zv : f4fma(e.b, be, zv));
      },
      [](int) {});
}

// Large grids: p_new = z + beta p_old (first: p_new = z, p_old not read), no
// partials; otherwise z and its r.z partials.
__global__ __launch_bounds__(kB) void k_mg_up0(const NpgGrid* __restrict__ G, int nb, int lo,
                                               const int* __restrict__ blk_sys, const int64_t* __restrict__ blk_start,
                                               const int* __restrict__ active, int check_active,
                                               const MgTask* __restrict__ T0, const float* __restrict__ r,
                                               const float* __restrict__ eh, float* __restrict__ z,
                                               double* __restrict__ part, const double* __restrict__ st,
                                               const float* __restrict__ p_old, float* __restrict__ p_new, int first) {
  const int blk = logical_block(nb, lo);
  if (blk < 0) return;
  const int s = blk_sys[blk];
  if (check_active && !active[s]) return;
  const NpgGrid g = G[s];
  const MgTask* tk = T0 + s;
  double acc[4] = {0, 0, 0, 0};
  if (use_zm(g)) {  // the block table holds z-column tiles for these grids
    float be[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) be[c] = first ? 0.f : (float)st[(s * 4 + c) * kS + 4];
    if (first) mg_up0_zm<true>(g, unpack_tile(blk_start[blk]), tk, r, eh, p_old, p_new, be);
    else mg_up0_zm<false>(g, unpack_tile(blk_start[blk]), tk, r, eh, p_old, p_new, be);
    return;
  } else {
    for (int k = 0; k < kPer; ++k) {
      const int64_t n = blk_start[blk] + k * kB + threadIdx.x;
      if (n >= g.nodes) break;
      mg_up_node(tk, r, eh, z, n, acc);
    }
  }
  store_partials<4>(acc, part, blk);
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
inline unsigned mg_grid(int nb) { return (unsigned)((nb + kXCD - 1) / kXCD * kXCD); }
inline unsigned xcd_grid(int nb) { return (unsigned)((nb + kXCD * kXG - 1) / (kXCD * kXG) * (kXCD * kXG)); }

}  // namespace

// V-cycle hierarchy of every system and its launch table. Launch l (l = 0 ..
// nlev-2) restricts level l to l+1, launch nlev-1+l prolongs level l+1 back
// to l, launch 2(nlev-1) solves every system's coarsest level (the
// prolongation kernel with no coarser level: hi.n = 0). A system has at least
// two levels (the grid and one coarser) and coarsens until a level has at
// most kMgMinN nodes per axis or kMgMaxLev coarse levels exist; it takes part
// in the launches of the levels it has.
static npg_status mg_setup(npg_plan* P) {
  NpgCG& C = P->cg;
  std::vector<std::vector<MgLvl>> lv(P->n_sys);
  int64_t coarse = 0;
  int nlev = 0;
  for (int sy = 0; sy < P->n_sys; ++sy) {
    const NpgGrid& g = P->g[sy];
    MgLvl L{};
    L.off = g.poff;
    L.n = g.R;
    L.s = 1;
    L.R = g.R;
    L.F = g.F;
    L.lam = g.lam;
    C.mg_elems[sy] = 0.0;
    while (true) {
      L.fn = make_fastdiv((uint32_t)L.n);
      L.fn2 = make_fastdiv((uint32_t)L.n * (uint32_t)L.n);
      lv[sy].push_back(L);
      if (lv[sy].size() >= 2 && (L.n <= kMgMinN || (int)lv[sy].size() > kMgMaxLev)) break;
      L.n = (L.n + 1) / 2;
      L.s *= 2;
      L.off = coarse;
      const int64_t e = (int64_t)L.n * L.n * L.n * L.F;
      coarse += (e + 3) / 4 * 4;  // every level 16-byte aligned (the z-column kernels rely on it)
      C.mg_elems[sy] += (double)e;
    }
    nlev = std::max(nlev, (int)lv[sy].size());
  }
  std::vector<MgTask> tasks;
  C.mg_l_task0.assign(2 * nlev - 1, 0);
  C.mg_l_ntask.assign(2 * nlev - 1, 0);
  C.mg_l_nblk.assign(2 * nlev - 1, 0);
  C.mg_split.assign(2 * nlev - 1, 0);
  auto add_launch = [&](int li, int l, bool up) {
    C.mg_l_task0[li] = (int)tasks.size();
    int blk = 0;
    for (int sy = 0; sy < P->n_sys; ++sy) {
      if ((int)lv[sy].size() <= l + 1) continue;
      MgTask t{};
      t.sys = sy;
      t.blk0 = blk;
      t.lo = lv[sy][l];
      t.hi = lv[sy][l + 1];
      const MgLvl& W = up ? t.lo : t.hi;
      t.nodes = (int64_t)W.n * W.n * W.n;
      t.fast = t.lo.F == 4 && t.lo.off % 4 == 0 && t.hi.off % 4 == 0 && t.lo.R % t.lo.s == 0;
      // the z-column tiles of the CG table (same test as use_zm; every coarse
      // level is 16-byte aligned, so the float4 access to level 1 holds too)
      t.zm0 = !up && l == 0;  // every finest restriction runs in k_mg_down0
      if (t.fast) {
        const float sz = (float)t.lo.s;
        t.mass = sz * sz * sz;
        t.lw = t.lo.lam * sz * sz;
        const int nx = (t.lo.n + 1) / 2;
        t.fx = make_fastdiv((uint32_t)nx);
        t.fx2 = make_fastdiv((uint32_t)nx * (uint32_t)t.lo.n);
        if (up) t.nodes = (int64_t)nx * t.lo.n * t.lo.n;  // one thread per x-adjacent pair
      }
      // a task restricted by k_mg_down0 gets no blocks here (it keeps its
      // slot: k_mg_down0 and k_mg_up0 look tasks up by system)
      if (!t.zm0) blk += (int)((t.nodes + kMgB - 1) / kMgB);
      tasks.push_back(t);
    }
    C.mg_l_ntask[li] = (int)tasks.size() - C.mg_l_task0[li];
    C.mg_l_nblk[li] = blk;
    C.mg_split[li] = blk;  // group 1's tasks (systems from grp_sys[1] on) start here
    for (int q = C.mg_l_task0[li]; q < (int)tasks.size(); ++q)
      if (tasks[q].sys >= C.grp_sys[1]) {
        C.mg_split[li] = tasks[q].blk0;
        break;
      }
  };
  for (int l = 0; l + 1 < nlev; ++l) add_launch(l, l, false);
  for (int l = 0; l + 1 < nlev; ++l) add_launch(nlev - 1 + l, l, true);
  {  // coarsest levels: two Jacobi steps, the prolongation kernel without a coarser level
    const int li = 2 * (nlev - 1);
    C.mg_l_task0[li] = (int)tasks.size();
    int blk = 0;
    for (int sy = 0; sy < P->n_sys; ++sy) {
      MgTask t{};
      t.sys = sy;
      t.blk0 = blk;
      t.lo = lv[sy].back();
      t.hi = MgLvl{};  // n = 0: no coarser correction
      t.nodes = (int64_t)t.lo.n * t.lo.n * t.lo.n;
      t.fast = t.lo.F == 4 && t.lo.off % 4 == 0 && t.lo.R % t.lo.s == 0;
      if (t.fast) {
        const float sz = (float)t.lo.s;
        t.mass = sz * sz * sz;
        t.lw = t.lo.lam * sz * sz;
        const int nx = (t.lo.n + 1) / 2;
        t.fx = make_fastdiv((uint32_t)nx);
        t.fx2 = make_fastdiv((uint32_t)nx * (uint32_t)t.lo.n);
        t.nodes = (int64_t)nx * t.lo.n * t.lo.n;
      }
      blk += (int)((t.nodes + kMgB - 1) / kMgB);
      tasks.push_back(t);
    }
    C.mg_l_ntask[li] = P->n_sys;
    C.mg_l_nblk[li] = blk;
    C.mg_split[li] = blk;
    for (int q = C.mg_l_task0[li]; q < (int)tasks.size(); ++q)
      if (tasks[q].sys >= C.grp_sys[1]) {
        C.mg_split[li] = tasks[q].blk0;
        break;
      }
  }
  // the finest prolongation runs over the CG work-group table (its tasks are
  // looked up by system: every system takes part, in order)
  if (C.mg_l_ntask[0] != P->n_sys || C.mg_l_ntask[nlev - 1] != P->n_sys)
    return npg_fail(NPG_EINVAL, "multigrid: finest level table");
  // Large grids (z-column tiles) form r.z from the finest restriction's term
  // and the level-1 term of the launch that produces level 1 (the up launch
  // from level 2, or the coarsest launch of a two-level hierarchy), whose
  // blocks write partials into their own range of part3 (lam = 0: no level-1
  // term, the preconditioner being the identity).
  std::vector<int> split(P->n_sys, 0);
  std::vector<int2> r3(P->n_sys, make_int2(0, 0));
  C.mg_l_p3.assign(2 * nlev - 1, -1);
  int p3 = 0;
  for (int sy = 0; sy < P->n_sys; ++sy) {
    const NpgGrid& g = P->g[sy];
    split[sy] = g.R >= kZmR && g.F == 4 && g.poff % 4 == 0;
    if (!split[sy] || g.lam == 0.f) continue;
    const int li = (int)lv[sy].size() >= 3 ? nlev : 2 * (nlev - 1);
    MgTask* tk = nullptr;
    for (int q = 0; q < C.mg_l_ntask[li]; ++q)
      if (tasks[C.mg_l_task0[li] + q].sys == sy) tk = &tasks[C.mg_l_task0[li] + q];
    if (!tk || tk->lo.s != 2) return npg_fail(NPG_EINVAL, "multigrid: level-1 task");
    tk->rz1 = 1;
    if (C.mg_l_p3[li] < 0) {
      C.mg_l_p3[li] = p3;
      p3 += C.mg_l_nblk[li];
    }
    const int b0 = C.mg_l_p3[li] + tk->blk0;
    r3[sy] = make_int2(b0, b0 + (int)((tk->nodes + kMgB - 1) / kMgB));
  }
  C.n_split = 0;
  for (int v : split) C.n_split += v;
  NPG_HIP(hipMalloc(&C.part3, (int64_t)std::max(p3, 1) * 4 * 8));
  NPG_HIP(hipMalloc(&C.r3, P->n_sys * sizeof(int2)));
  NPG_HIP(hipMalloc(&C.sys_split, P->n_sys * sizeof(int)));
  NPG_HIP(hipMemcpy(C.r3, r3.data(), P->n_sys * sizeof(int2), hipMemcpyHostToDevice));
  NPG_HIP(hipMemcpy(C.sys_split, split.data(), P->n_sys * sizeof(int), hipMemcpyHostToDevice));
  C.mg_nlev = nlev;
  NPG_HIP(hipMalloc(&C.z, P->n_grid_params * 4));
  NPG_HIP(hipMalloc(&C.mgB, std::max<int64_t>(coarse, 1) * 4));
  NPG_HIP(hipMalloc(&C.mgX, std::max<int64_t>(coarse, 1) * 4));
  NPG_HIP(hipMalloc(&C.part2, (int64_t)C.n_blocks * 4 * 8));
  C.mg_l_blk0.assign(2 * nlev - 1, std::vector<int>(kMgTaskMax, INT_MAX));
  for (int li = 0; li < 2 * nlev - 1; ++li) {
    if (C.mg_l_ntask[li] > kMgTaskMax) return npg_fail(NPG_EINVAL, "multigrid: too many tasks in one launch");
    for (int q = 0; q < C.mg_l_ntask[li]; ++q) C.mg_l_blk0[li][q] = tasks[C.mg_l_task0[li] + q].blk0;
  }
  NPG_HIP(hipMalloc(&C.mg_tasks, tasks.size() * sizeof(MgTask)));
  NPG_HIP(hipMemcpy(C.mg_tasks, tasks.data(), tasks.size() * sizeof(MgTask), hipMemcpyHostToDevice));
  return NPG_OK;
}

// z = M^-1 r (one V-cycle for every system; with check_active only the
// systems still iterating). Small grids: z and its r.z partials (part2). Large
// grids (split): the r.z terms (part2 from the finest restriction, part3 from
// level 1), then `beta` (when not NULL) reduces them, updates their scalars
// (k_cg_reduce mode 2 of the split systems: beta, convergence), and the finest
// prolongation writes their next direction p_dst = z + beta p_src (first:
// p_dst = z; p_src is not read).
struct MgDir {
  const float* p_src;
  float* p_dst;
  const double* st;
  int first;
};
// The grids of one V-cycle or CG call: systems [s_lo, s_hi) and CG
// work-groups [b_lo, b_hi) on `stream`; grp is the group (0 or 1) of a
// two-group plan, -1 for every system.
struct CgGrp {
  int grp, s_lo, s_hi, b_lo, b_hi;
  hipStream_t stream;
  bool split;  // a system of the range is split (its r.z taken in the V-cycle)
};

static CgGrp cg_all(const npg_plan* P) {
  return CgGrp{-1, 0, P->n_sys, 0, P->cg.n_blocks, P->stream, P->cg.n_split > 0};
}

static CgGrp cg_grp(const npg_plan* P, int g) {
  const NpgCG& C = P->cg;
  if (C.n_grp == 1) return cg_all(P);
  hipStream_t s = g == 0 && C.stream2 ? C.stream2 : P->stream;
  CgGrp G{g, C.grp_sys[g], C.grp_sys[g + 1], C.grp_blk[g], C.grp_blk[g + 1], s, false};
  for (int sy = G.s_lo; sy < G.s_hi; ++sy) G.split |= use_zm(P->g[sy]);
  return G;
}

static npg_status mg_apply(npg_plan* P, const CgGrp& G, const float* r, float* z, int check_active, const MgDir& d,
                           const std::function<void()>& beta) {
  NpgCG& C = P->cg;
  hipStream_t s = G.stream;
  const int nl = C.mg_nlev;
  const MgTask* T = static_cast<const MgTask*>(C.mg_tasks);
  const unsigned gb = xcd_grid(G.b_hi - G.b_lo);
  if (d.first)  // the start of a solve (r = b): also the large grids' b.b partials
    hipLaunchKernelGGL(k_mg_down0<true>, dim3(gb), dim3(kB), 0, s, P->d_g, G.b_hi, G.b_lo, C.blk_sys, C.blk_start,
                       C.sys_blk0, C.active, check_active, T + C.mg_l_task0[0], r, C.mgB, C.part2, C.part);
  else
    hipLaunchKernelGGL(k_mg_down0<false>, dim3(gb), dim3(kB), 0, s, P->d_g, G.b_hi, G.b_lo, C.blk_sys,
                       C.blk_start, C.sys_blk0, C.active, check_active, T + C.mg_l_task0[0], r, C.mgB, C.part2,
                       nullptr);
  auto blk0 = [&](int li) {
    MgBlk0 b;
    for (int q = 0; q < kMgTaskMax; ++q) b.b[q] = C.mg_l_blk0[li][q];
    return b;
  };
  auto p3 = [&](int li) { return C.mg_l_p3[li] >= 0 ? C.part3 + (int64_t)C.mg_l_p3[li] * 4 : nullptr; };
  // this range's blocks of launch li: [lo, hi)
  auto range = [&](int li, int& lo, int& hi) {
    lo = G.grp == 1 ? C.mg_split[li] : 0;
    hi = G.grp == 0 ? C.mg_split[li] : C.mg_l_nblk[li];
    return hi > lo;
  };
  int lo, hi;
  for (int l = 0; l + 1 < nl; ++l)
    if (range(l, lo, hi))
      hipLaunchKernelGGL(k_mg_down, dim3(mg_grid(hi - lo)), dim3(kMgB), 0, s, T + C.mg_l_task0[l], blk0(l), hi, lo,
                         C.active, check_active, l == 0 ? r : C.mgB, C.mgB);
  for (int l = nl - 1; l >= 1; --l) {
    const int li = l == nl - 1 ? 2 * (nl - 1) : nl - 1 + l;  // the coarsest solve, then the prolongations
    if (range(li, lo, hi))
      hipLaunchKernelGGL(k_mg_up, dim3(mg_grid(hi - lo)), dim3(kMgB), 0, s, T + C.mg_l_task0[li], blk0(li), hi, lo,
                         C.active, check_active, C.mgB, C.mgX, C.mgX, p3(li));
  }
  if (beta) beta();
  hipLaunchKernelGGL(k_mg_up0, dim3(gb), dim3(kB), 0, s, P->d_g, G.b_hi, G.b_lo, C.blk_sys, C.blk_start, C.active,
                     check_active, T + C.mg_l_task0[nl - 1], r, C.mgX, z, C.part2, d.st, d.p_src, d.p_dst, d.first);
  NPG_HIP(hipGetLastError());
  return NPG_OK;
}

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
      for (int z0 = 0; z0 < g.R; z0 += P->cg_zs)
        for (int y0 = 0; y0 < g.R; y0 += kTY)
          for (int x0 = 0; x0 < g.R; x0 += kTX) {
            bsys.push_back(s);
            bstart.push_back(pack_tile(x0, y0, z0, std::min(g.R, z0 + P->cg_zs)));
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
  for (auto& d : C.pd) NPG_HIP(hipMalloc(&d, n * 4));
  NPG_HIP(hipMalloc(&C.ahist, 2 * (int64_t)P->n_sys * 4 * kCgDirs * 8));
  NPG_HIP(hipMalloc(&C.part, (int64_t)C.n_blocks * 4 * 8));
  NPG_HIP(hipMalloc(&C.st, 2 * (int64_t)P->n_sys * 4 * kS * 8));  // one block per solve
  NPG_HIP(hipMalloc(&C.active, P->n_sys * 4));
  NPG_HIP(hipMalloc(&C.blk_sys, C.n_blocks * 4));
  NPG_HIP(hipMalloc(&C.blk_start, C.n_blocks * 8));
  NPG_HIP(hipMalloc(&C.sys_blk0, (P->n_sys + 1) * 4));
  NPG_HIP(hipMemcpy(C.blk_sys, bsys.data(), C.n_blocks * 4, hipMemcpyHostToDevice));
  NPG_HIP(hipMemcpy(C.blk_start, bstart.data(), C.n_blocks * 8, hipMemcpyHostToDevice));
  NPG_HIP(hipMemcpy(C.sys_blk0, s0.data(), (P->n_sys + 1) * 4, hipMemcpyHostToDevice));
  // Two groups when the largest grid is walked in z-column tiles and other
  // grids come before it: the largest and the systems after it (group 1, on
  // the plan's stream) iterate beside the grids before it (group 0, on a
  // second stream unless cfg.cg_one_stream), so the short latency-bound
  // launches of one group overlap the streaming kernels of the other. The
  // systems are independent, so the results do not depend on the grouping.
  {
    int big = 0;
    for (int sy = 1; sy < P->n_sys; ++sy)
      if (P->g[sy].nodes * P->g[sy].F > P->g[big].nodes * P->g[big].F) big = sy;
    const NpgGrid& gb = P->g[big];
    const bool zm = gb.R >= kZmR && gb.F == 4 && gb.poff % 4 == 0;
    C.n_grp = big > 0 && zm ? 2 : 1;
    C.grp_sys[0] = 0;
    C.grp_sys[1] = C.n_grp == 2 ? big : P->n_sys;
    C.grp_sys[2] = P->n_sys;
    C.grp_blk[0] = 0;
    C.grp_blk[1] = s0[C.grp_sys[1]];
    C.grp_blk[2] = C.n_blocks;
    if (C.n_grp == 2 && !P->cfg.cg_one_stream) {
      NPG_HIP(hipStreamCreateWithFlags(&C.stream2, hipStreamNonBlocking));
      NPG_HIP(hipEventCreateWithFlags(&C.ev_fork, hipEventDisableTiming));
      NPG_HIP(hipEventCreateWithFlags(&C.ev_join, hipEventDisableTiming));
    }
    for (auto& e : C.ev_grp) NPG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    NPG_HIP(hipHostMalloc((void**)&C.act_host, P->n_sys * sizeof(int), hipHostMallocDefault));
  }
  C.mg = P->cfg.cg_mg != 0;
  if (C.mg) {
    const npg_status st = mg_setup(P);
    if (st != NPG_OK) return st;
  }
  return NPG_OK;
}

void npg_cg_free(npg_plan* P) {
  NpgCG& C = P->cg;
  for (auto d : C.pd)
    if (d) (void)hipFree(d);
  if (C.ahist) (void)hipFree(C.ahist);
  void* bufs[] = {C.x, C.r, C.part, C.st, C.active, C.blk_sys, C.blk_start, C.sys_blk0,
                  C.z, C.mgB, C.mgX, C.part2, C.mg_tasks, C.part3, C.r3, C.sys_split};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (C.stream2) (void)hipStreamDestroy(C.stream2);
  if (C.ev_fork) (void)hipEventDestroy(C.ev_fork);
  if (C.ev_join) (void)hipEventDestroy(C.ev_join);
  for (auto e : C.ev_grp)
    if (e) (void)hipEventDestroy(e);
  if (C.act_host) (void)hipHostFree(C.act_host);
  const int keep[2] = {C.last_iters[0], C.last_iters[1]};
  int keep_grp[2][2];
  for (int w = 0; w < 2; ++w)
    for (int g = 0; g < 2; ++g) keep_grp[w][g] = C.last_grp[w][g];
  C = NpgCG();
  C.last_iters[0] = keep[0];
  C.last_iters[1] = keep[1];
  for (int w = 0; w < 2; ++w)
    for (int g = 0; g < 2; ++g) C.last_grp[w][g] = keep_grp[w][g];
}

// ---- the two solves ------------------------------------------------------------
// Solve (I + lam L) x = b for every system (b and x distinct buffers in the
// grid-block layout); solve `which` (0 first, 1 second) keeps its scalars in
// its own block of C.st. Iteration k writes p_k into ring slot k mod
// kCgDirs and its alpha into the same slot of the solve's alpha history; the
// updates leave x alone, and after iterations kCgDirs-1, 2 kCgDirs-1, ...
// k_cg_xacc adds the window's kCgDirs terms to x in one pass (p_k is
// overwritten kCgDirs iterations later, after its window was added; later
// iterations write only the blocks of systems still active, so a stopped
// system's last terms stay in the ring), and k_cg_flush adds the terms still
// pending when a system stops. An iteration launched after
// every system of the solve has converged changes nothing (each work-group
// returns on the system's device-side active flag), so the result does not
// depend on how many iterations are launched past convergence: the eager
// form launches them in batches between host tests of the flags, the
// graph-recorded form a fixed count followed by a device-side check.
namespace {

struct CgCtx {
  dim3 grid, blk;
  Divs dv;
  bool mg;
  double* part2;
  const float* dir_src;
  double* st;
  double* ah;  // the solve's alpha of each ring slot
  Dirs dirs;
};

CgCtx cg_ctx(const npg_plan* P, int which) {
  const NpgCG& C = P->cg;
  CgCtx c;
  c.grid = dim3(xcd_grid(C.n_blocks));
  c.blk = dim3(kB);
  for (int sy = 0; sy < P->n_sys; ++sy) {
    c.dv.r[sy] = make_fastdiv((uint32_t)P->g[sy].R);
    c.dv.r2[sy] = make_fastdiv((uint32_t)P->g[sy].R * (uint32_t)P->g[sy].R);
  }
  c.mg = C.mg != 0;
  c.part2 = c.mg ? C.part2 : nullptr;
  c.dir_src = c.mg ? C.z : C.r;  // p = z + beta p (z = r without the V-cycle)
  c.st = C.st + (size_t)which * P->n_sys * 4 * kS;
  c.ah = C.ahist + (size_t)which * P->n_sys * 4 * kCgDirs;
  for (int j = 0; j < kCgDirs; ++j) c.dirs.p[j] = C.pd[j];
  return c;
}

// The scalar update of the range's systems (filter -1), of those whose r.z is
// split over the finest restriction and level 1 (filter 1), or of the others
// (filter 0); see k_cg_reduce.
void cg_reduce(npg_plan* P, const CgCtx& c, const CgGrp& G, int mode, int k, int filter) {
  NpgCG& C = P->cg;
  hipLaunchKernelGGL(k_cg_reduce, dim3(G.s_hi - G.s_lo), dim3(kR_THREADS), 0, G.stream, P->d_g, C.sys_blk0,
                     C.active, C.part, c.part2, C.sys_blk0, c.st, mode, P->cfg.cg_rtol, c.ah, k % kCgDirs,
                     c.mg ? C.part3 : nullptr, c.mg ? C.r3 : nullptr, c.mg ? C.sys_split : nullptr, filter, G.s_lo);
}

// Iteration 0 takes ring slot 0 as its direction: the start writes p_0 = z_0
// there on the large grids of the multigrid form (in the V-cycle's finest
// prolongation); the other grids form it in k_cg_dir_ap from z with beta = 0
// and the old direction in the last slot, which k_cg_init sets to b.
npg_status cg_start(npg_plan* P, const CgCtx& c, const CgGrp& G, const float* b) {
  NpgCG& C = P->cg;
  hipLaunchKernelGGL(k_cg_init, dim3(xcd_grid(G.b_hi - G.b_lo)), c.blk, 0, G.stream, P->d_g, G.b_hi, G.b_lo,
                     C.blk_sys, C.blk_start, b, C.r, C.pd[kCgDirs - 1], c.mg ? C.sys_split : nullptr, C.part);
  // r = b: the first V-cycle reads b (the split grids never store r = b)
  if (c.mg) NPG_TRY_ST(mg_apply(P, G, b, C.z, 0, MgDir{C.pd[kCgDirs - 1], C.pd[0], c.st, 1}, nullptr));
  cg_reduce(P, c, G, 0, 0, -1);
  NPG_HIP(hipGetLastError());
  return NPG_OK;
}

// Iteration k (0-based) of a solve of right-hand side b over the grids of G,
// on G's stream.
npg_status cg_iteration(npg_plan* P, const CgCtx& c, const CgGrp& G, const float* b, float* x, int k) {
  NpgCG& C = P->cg;
  hipStream_t s = G.stream;
  const dim3 grid(xcd_grid(G.b_hi - G.b_lo));
  const int nb = G.b_hi, lo = G.b_lo;
  float* p_old = C.pd[(k + kCgDirs - 1) % kCgDirs];
  float* p_new = C.pd[k % kCgDirs];
  float* p_next = C.pd[(k + 1) % kCgDirs];
  hipLaunchKernelGGL(k_cg_dir_ap, grid, c.blk, 0, s, P->d_g, c.dv, nb, lo, C.blk_sys, C.blk_start, C.active, c.st,
                     c.dir_src, p_old, p_new, C.part, (int)c.mg);
  cg_reduce(P, c, G, 1, k, -1);
  // the first iteration reads r from b
  hipLaunchKernelGGL(k_cg_update, grid, c.blk, 0, s, P->d_g, c.dv, nb, lo, C.blk_sys, C.blk_start, C.active, c.st,
                     k == 0 ? b : nullptr, C.r, p_new, C.part);
  // the last iteration of a window: its kCgDirs x terms (before the
  // convergence test, so a system that stops here has them all in x)
  if (k % kCgDirs == kCgDirs - 1)
    hipLaunchKernelGGL(k_cg_xacc, dim3((unsigned)(4 * P->n_cu)), dim3(256), 0, s, P->d_g, G.s_lo, G.s_hi, C.active,
                       c.ah, (int)(k == kCgDirs - 1), x, c.dirs);
  if (c.mg) {
    // large grids: beta (and the convergence test) before the prolongation,
    // which writes their next direction into the next ring slot (its old
    // direction's x term was added with its window); the other grids after it
    const std::function<void()> beta = [&]() { cg_reduce(P, c, G, 2, k, 1); };
    NPG_TRY_ST(mg_apply(P, G, C.r, C.z, 1, MgDir{p_new, p_next, c.st, 0}, G.split ? beta : nullptr));
    cg_reduce(P, c, G, 2, k, 0);
  } else {
    cg_reduce(P, c, G, 2, k, -1);
  }
  NPG_HIP(hipGetLastError());
  return NPG_OK;
}

// Iterations [k0, k0 + n) of a solve over every system: with two groups on
// two streams, the second stream waits for the plan's stream, each group's
// iterations go to its own stream (interleaved, so that both are fed), and
// the plan's stream waits for the second at the end. With profiling on, HIP events on the
// plan's stream bracket the batch, resolved after the step.
npg_status cg_iterations(npg_plan* P, const CgCtx& c, const float* b, float* x, int k0, int n) {
  NpgCG& C = P->cg;
  const bool prof = P->prof_cg && P->prof_n + 2 <= (int)P->prof_ev.size();
  if (prof) NPG_HIP(hipEventRecord(P->prof_ev[P->prof_n], P->stream));
  if (C.stream2) {
    NPG_HIP(hipEventRecord(C.ev_fork, P->stream));
    NPG_HIP(hipStreamWaitEvent(C.stream2, C.ev_fork, 0));
  }
  const CgGrp G0 = cg_grp(P, 0), G1 = cg_grp(P, 1);
  for (int k = k0; k < k0 + n; ++k) {
    NPG_TRY_ST(cg_iteration(P, c, G0, b, x, k));
    if (C.n_grp == 2) NPG_TRY_ST(cg_iteration(P, c, G1, b, x, k));
  }
  if (C.stream2) {
    NPG_HIP(hipEventRecord(C.ev_join, C.stream2));
    NPG_HIP(hipStreamWaitEvent(P->stream, C.ev_join, 0));
  }
  if (prof) {
    NPG_HIP(hipEventRecord(P->prof_ev[P->prof_n + 1], P->stream));
    P->prof_n += 2;
    P->prof_it += n;
  }
  return NPG_OK;
}

npg_status cg_finish(npg_plan* P, const CgCtx& c, const CgGrp& G, float* x) {
  hipLaunchKernelGGL(k_cg_flush, dim3((unsigned)(4 * P->n_cu)), dim3(256), 0, G.stream, P->d_g, G.s_lo, G.s_hi, c.st,
                     c.ah, x, c.dirs);
  NPG_HIP(hipGetLastError());
  return NPG_OK;
}

// Eager solve over every system, the groups of grids in step (the form
// used with iteration profiling: events bracket each batch of iterations of
// both groups): iterations launched in batches between host tests of the
// active flags. The first batch is what the same solve of the previous call
// took (16 the first time, at most kFirstMax, and not carried over from a
// solve that reached the cap); later batches are 2 iterations long.
constexpr int kFirstMax = 128;

npg_status cg_solve_eager(npg_plan* P, int which, const float* b, float* x, bool* capped) {
  NpgCG& C = P->cg;
  hipStream_t s = P->stream;
  const CgCtx c = cg_ctx(P, which);
  const CgGrp all = cg_all(P);
  NPG_TRY_ST(cg_start(P, c, all, b));
  std::vector<int> act(P->n_sys);
  const int maxit = P->cfg.cg_maxit;
  const int last = C.last_iters[which];
  const int first = last > 0 ? std::min(last, kFirstMax) : 16;
  int it = 0;
  bool done = false;
  while (it < maxit) {
    const int want = it == 0 ? first : (last > 0 ? 2 : 16);
    const int chunk = std::min(want, maxit - it);
    NPG_TRY_ST(cg_iterations(P, c, b, x, it, chunk));
    it += chunk;
    NPG_HIP(hipMemcpyAsync(act.data(), C.active, P->n_sys * 4, hipMemcpyDeviceToHost, s));
    NPG_HIP(hipStreamSynchronize(s));
    done = true;
    for (int v : act) done &= (v == 0);
    if (done) break;
  }
  if (!done) *capped = true;
  return cg_finish(P, c, all, x);
}

// Both eager solves with every group of grids on its own stream and at its
// own pace: a group's second solve starts as soon as its first has stopped
// (the systems are independent: the results are those of cg_solve_eager),
// so one group's start, flush and host tests overlap the other group's
// iterations. Batches as in cg_solve_eager, counted per group (the first
// batch of a solve is what the group's slowest system took in the same
// solve of the previous call). Each batch ends with a copy of the group's
// flags to pinned host memory and an event, which the host polls.
npg_status cg_precond_pipelined(npg_plan* P, float* grad, bool* capped) {
  NpgCG& C = P->cg;
  const float* bs[2] = {grad, C.x};
  float* xs[2] = {C.x, grad};
  const int ng = C.n_grp, maxit = P->cfg.cg_maxit;
  const CgCtx cx[2] = {cg_ctx(P, 0), cg_ctx(P, 1)};
  CgGrp G[2];
  for (int g = 0; g < ng; ++g) G[g] = cg_grp(P, g);
  struct Run {
    int which, it;
    bool done;
  } run[2] = {{0, 0, false}, {0, 0, false}};
  auto batch = [&](int g) -> npg_status {
    Run& R = run[g];
    const int last = C.last_grp[R.which][g];
    const int want = R.it == 0 ? (last > 0 ? std::min(last, kFirstMax) : 16) : (last > 0 ? 2 : 16);
    const int n = std::min(want, maxit - R.it);
    for (int k = R.it; k < R.it + n; ++k) NPG_TRY_ST(cg_iteration(P, cx[R.which], G[g], bs[R.which], xs[R.which], k));
    R.it += n;
    NPG_HIP(hipMemcpyAsync(C.act_host + G[g].s_lo, C.active + G[g].s_lo, (G[g].s_hi - G[g].s_lo) * sizeof(int),
                           hipMemcpyDeviceToHost, G[g].stream));
    NPG_HIP(hipEventRecord(C.ev_grp[g], G[g].stream));
    return NPG_OK;
  };
  if (C.stream2) {
    NPG_HIP(hipEventRecord(C.ev_fork, P->stream));
    NPG_HIP(hipStreamWaitEvent(C.stream2, C.ev_fork, 0));
  }
  for (int g = 0; g < ng; ++g) {
    NPG_TRY_ST(cg_start(P, cx[0], G[g], bs[0]));
    NPG_TRY_ST(batch(g));
  }
  for (int left = ng; left > 0;) {
    bool ready = false;
    for (int g = 0; g < ng; ++g) {
      Run& R = run[g];
      if (R.done) continue;
      const hipError_t e = hipEventQuery(C.ev_grp[g]);
      if (e == hipErrorNotReady) continue;
      NPG_HIP(e);
      ready = true;
      bool active = false;
      for (int sy = G[g].s_lo; sy < G[g].s_hi; ++sy) active |= C.act_host[sy] != 0;
      if (active && R.it < maxit) {
        NPG_TRY_ST(batch(g));
        continue;
      }
      if (active) *capped = true;
      NPG_TRY_ST(cg_finish(P, cx[R.which], G[g], xs[R.which]));
      if (R.which == 0) {
        R.which = 1;
        R.it = 0;
        NPG_TRY_ST(cg_start(P, cx[1], G[g], bs[1]));
        NPG_TRY_ST(batch(g));
      } else {
        R.done = true;
        --left;
      }
    }
    if (!ready) std::this_thread::yield();
  }
  if (C.stream2) {
    NPG_HIP(hipEventRecord(C.ev_join, C.stream2));
    NPG_HIP(hipStreamWaitEvent(P->stream, C.ev_join, 0));
  }
  return NPG_OK;
}

}  // namespace

// Host bookkeeping of the last preconditioning from both solves' scalars
// (synchronizes): iteration counts (iters may be NULL), final relative
// residuals, the algorithmic bytes of the iterations, the first batch of the
// next eager call (not carried over from a solve that reached the cap).
npg_status npg_cg_report(npg_plan* P, int32_t* iters) {
  NpgCG& C = P->cg;
  const bool mg = C.mg != 0;
  std::vector<double> stv((size_t)2 * P->n_sys * 4 * kS);
  NPG_HIP(hipMemcpyAsync(stv.data(), C.st, stv.size() * 8, hipMemcpyDeviceToHost, P->stream));
  NPG_HIP(hipStreamSynchronize(P->stream));
  P->cg_alg_bytes = 0.0;
  P->cg_alg_bytes_mg = 0.0;
  P->cg_iters_sum = 0;
  for (int which = 0; which < 2; ++which) {
    int taken = 0;  // iterations of the slowest system
    int taken_grp[2] = {0, 0};
    for (int sy = 0; sy < P->n_sys; ++sy) {
      const NpgGrid& g = P->g[sy];
      const double* S0 = stv.data() + ((size_t)which * P->n_sys + sy) * 4 * kS;
      double m = 0.0, rel = 0.0;
      for (int ch = 0; ch < g.F; ++ch) {
        const double* S = S0 + ch * kS;
        m = S[6] > m ? S[6] : m;
        // final relative residual ||r|| / ||b|| in float64, the largest over the channels
        const double v = S[1] > 0.0 ? sqrt(S[2] / S[1]) : 0.0;
        rel = v > rel ? v : rel;
      }
      if (iters) iters[which * P->n_sys + sy] = (int32_t)m;
      P->cg_relres[which * P->n_sys + sy] = rel;
      taken = std::max(taken, (int)m);
      const int grp = C.n_grp == 2 && sy >= C.grp_sys[1] ? 1 : 0;
      taken_grp[grp] = std::max(taken_grp[grp], (int)m);
      // algorithmic traffic per iteration: 6 vector passes (x, r, p read and
      // written) over the grid's R^3 F float32 unknowns; the V-cycle form
      // also moves z (written, read) and each coarse level's right-hand side
      // and correction (written, read)
      const double fine = (double)g.nodes * g.F;
      P->cg_alg_bytes += m * 4.0 * 6.0 * fine;
      const bool split = g.R >= kZmR && g.F == 4 && g.poff % 4 == 0;  // no stored z
      P->cg_alg_bytes_mg += m * 4.0 * (mg ? (split ? 6.0 : 8.0) * fine + 4.0 * C.mg_elems[sy] : 6.0 * fine);
      P->cg_iters_sum += (int64_t)m;
    }
    C.last_iters[which] = taken >= P->cfg.cg_maxit ? 0 : taken;
    for (int g = 0; g < 2; ++g) C.last_grp[which][g] = taken_grp[g] >= P->cfg.cg_maxit ? 0 : taken_grp[g];
  }
  return NPG_OK;
}

npg_status npg_run_precond_cg(npg_plan* P, float* grad, int32_t* iters) {
  bool capped = false;
  // y = A^-1 g into the workspace, then A^-1 y back into the gradient; with
  // iteration profiling the groups of grids go in step (each batch bracketed)
  if (P->prof_cg) {
    NPG_TRY_ST(cg_solve_eager(P, 0, grad, P->cg.x, &capped));
    NPG_TRY_ST(cg_solve_eager(P, 1, P->cg.x, grad, &capped));
  } else {
    NPG_TRY_ST(cg_precond_pipelined(P, grad, &capped));
  }
  NPG_TRY_ST(npg_cg_report(P, iters));
  return capped ? NPG_ENOTCONV : NPG_OK;
}

// Graph-recordable form (no host synchronisation): solve `which` launches
// exactly n_iter[which] iterations, then k_cg_done sets bit (1 << which) of
// *state_dev if a system is still iterating, or bit 4 when the count is the
// cap cg_maxit (the eager form's NPG_ENOTCONV case, whose result stands).
// Each group of grids runs both solves on its own stream (a group's second
// solve starts when its own first one ends); the launches of the groups are
// issued interleaved, step by step.
npg_status npg_run_precond_cg_fixed(npg_plan* P, float* grad, const int n_iter[2], int* state_dev) {
  NpgCG& C = P->cg;
  const float* b[2] = {grad, C.x};
  float* x[2] = {C.x, grad};
  const int ng = C.n_grp;
  CgGrp G[2];
  for (int g = 0; g < ng; ++g) G[g] = cg_grp(P, g);
  if (C.stream2) {
    NPG_HIP(hipEventRecord(C.ev_fork, P->stream));
    NPG_HIP(hipStreamWaitEvent(C.stream2, C.ev_fork, 0));
  }
  for (int which = 0; which < 2; ++which) {
    const CgCtx c = cg_ctx(P, which);
    for (int g = 0; g < ng; ++g) NPG_TRY_ST(cg_start(P, c, G[g], b[which]));
    for (int k = 0; k < n_iter[which]; ++k)
      for (int g = 0; g < ng; ++g) NPG_TRY_ST(cg_iteration(P, c, G[g], b[which], x[which], k));
    const int bit = n_iter[which] >= P->cfg.cg_maxit ? 4 : (1 << which);
    for (int g = 0; g < ng; ++g) {
      hipLaunchKernelGGL(k_cg_done, dim3(1), dim3(64), 0, G[g].stream, C.active, G[g].s_lo, G[g].s_hi, state_dev,
                         bit);
      NPG_HIP(hipGetLastError());
      NPG_TRY_ST(cg_finish(P, c, G[g], x[which]));
    }
  }
  if (C.stream2) {
    NPG_HIP(hipEventRecord(C.ev_join, C.stream2));
    NPG_HIP(hipStreamWaitEvent(P->stream, C.ev_join, 0));
  }
  return NPG_OK;
}
