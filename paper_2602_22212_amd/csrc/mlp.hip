// Time-modulated MLP decode (Sec. 3.3), exponential-map transform and apply
// (Sec. 3.4, supplementary rotation study), and their backward.
//
// Layout. A sample is a (frame t, vertex i) pair, s = t*V + i. Activations
// are kept transposed in registers as 16x16 tiles of the MFMA
// v_mfma_f32_16x16x4_f32 result layout: lane (q = lane/16, c = lane%16)
// register r holds feature 16*mt + 4q + r of sample c. That layout is exactly
// the B operand the next layer needs when the K index of k-step r is
// 16*kt + 4q + r, so the chain of layers never leaves registers; the A
// operand of every MFMA is a float4 read of 4 consecutive weights of one row.
//
// First layer. W1 y + b1 with y = (z_i, gamma_t) splits into
// A_i = W1z z_i + b1 ([V][W]) and B_t = W1g gamma_t ([T][W]), computed once
// per call, so the per-sample first layer is one add.
//
// Backward. Activations are recomputed per tile (never stored), so memory is
// O(V + T) per call. Weight gradients contract over samples, which needs the
// sample index in the MFMA K position: each layer's (gradient, input) tiles
// of the work-group's 64 samples are staged through LDS, and each of the 4
// waves accumulates a fixed quarter of the weight-gradient tiles in
// registers over all frames. Per-work-group partials are summed in a fixed
// order afterwards, so every result is bitwise reproducible.
#include <algorithm>
#include <vector>

#include "internal.h"

typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

// Activation: x > 0 ? x : slope x, with slope 0 for ReLU and in (0, 1] for
// LeakyReLU (the host sets it), so that it equals max(x, slope x); the
// maximum is taken as the median of (x, slope x, FLT_MAX) (the same for finite
// values), one instruction without the operand quieting that the IEEE maximum
// adds for matrix-core results.
struct ActP {
  int relu;
  float slope;
};
constexpr float kFltMax = 3.40282347e38f;

__device__ __forceinline__ float actf(float x, ActP a) { return __builtin_amdgcn_fmed3f(x, a.slope * x, kFltMax); }
// derivative from the activation's output (same sign as its input)
__device__ __forceinline__ float actd(float h, ActP a) { return h > 0.f ? 1.f : a.slope; }

__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Sum over the 16 lanes of a row with DPP moves (quad xor 1, quad xor 2,
// half-row mirror, row mirror); every lane of the row ends with the sum.
__device__ __forceinline__ float row16_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
  return v;
}

// row16_sum of the 4 components, one DPP stage for all of them at a time
template <int CTRL>
__device__ __forceinline__ void dpp_add4(v4f& v) {
#pragma unroll
  for (int r = 0; r < 4; ++r)
    v[r] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[r]), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ v4f row16_sum4(v4f v) {
  dpp_add4<0xB1>(v);
  dpp_add4<0x4E>(v);
  dpp_add4<0x141>(v);
  dpp_add4<0x140>(v);
  return v;
}

__device__ __forceinline__ float comp(const float4& v, int r) {
  return r == 0 ? v.x : (r == 1 ? v.y : (r == 2 ? v.z : v.w));
}

// Workspace layout of the repacked weights (floats, every block 16-B aligned):
//   for hidden layer l = 1..H-1:  Wh[l] [W][W] (row = out), WhT[l] [W][W]
//   (row = in), bh[l] [W]; then WoP [16][W] (output rows; rows n_out..15
//   zero), WoT [W][16] (transposed, columns n_out..15 zero), bo [16].
struct WPack {
  int64_t wh, wht, bh, wop, wot, bo, total;
  __host__ __device__ WPack(int W, int H) {
    int64_t hsz = (int64_t)W * W;
    wh = 0;
    wht = wh + (H - 1) * hsz;
    bh = wht + (H - 1) * hsz;
    wop = bh + (int64_t)(H - 1) * W;
    wot = wop + 16 * (int64_t)W;
    bo = wot + 16 * (int64_t)W;
    total = bo + 16;
  }
};

// Offsets (floats) inside the flat MLP block.
__host__ __device__ inline int64_t mlp_layer_off(int l, int W, int Din) {
  if (l == 0) return 0;
  return (int64_t)W * Din + W + (int64_t)(l - 1) * ((int64_t)W * W + W);
}

__global__ void k_prep_weights(const float* __restrict__ mlp, int W, int H, int Din, int n_out,
                               float* __restrict__ wp) {
  WPack P(W, H);
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= P.total) return;
  float val = 0.f;
  if (e < P.wht) {
    int64_t l = e / ((int64_t)W * W) + 1, k = e % ((int64_t)W * W);
    val = mlp[mlp_layer_off((int)l, W, Din) + k];
  } else if (e < P.bh) {
    int64_t k = e - P.wht;
    int64_t l = k / ((int64_t)W * W) + 1, kk = k % ((int64_t)W * W);
    int64_t in = kk / W, out = kk % W;  // WhT[in][out] = Wh[out][in]
    val = mlp[mlp_layer_off((int)l, W, Din) + out * W + in];
  } else if (e < P.wop) {
    int64_t k = e - P.bh;
    int64_t l = k / W + 1, o = k % W;
    val = mlp[mlp_layer_off((int)l, W, Din) + (int64_t)W * W + o];
  } else if (e < P.wot) {
    int64_t k = e - P.wop;
    int64_t row = k / W, col = k % W;
    if (row < n_out) val = mlp[mlp_layer_off(H, W, Din) + row * W + col];
  } else if (e < P.bo) {
    int64_t k = e - P.wot;
    int64_t in = k / 16, o = k % 16;
    if (o < n_out) val = mlp[mlp_layer_off(H, W, Din) + o * W + in];
  } else {
    int64_t o = e - P.bo;
    if (o < n_out) val = mlp[mlp_layer_off(H, W, Din) + n_out * (int64_t)W + o];
  }
  wp[e] = val;
}

__device__ __forceinline__ float rnd(float x, int bf16) { return bf16 ? npg_bf16_round(x) : x; }

// A[i][o] = b1[o] + sum_k W1[o][k] z[i][k] (k < Fz); in the BF16 form W1 and z
// are rounded to bfloat16 first (float32 accumulation)
__global__ void k_prep_A(const float* __restrict__ mlp, const float* __restrict__ z, int64_t V, int W, int Din,
                         int Fz, int bf16, float* __restrict__ A) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= V * W) return;
  int64_t i = e / W;
  int o = (int)(e % W);
  const float* w1 = mlp + (int64_t)o * Din;
  float acc = mlp[(int64_t)W * Din + o];
  for (int k = 0; k < Fz; ++k) acc = fmaf(rnd(w1[k], bf16), rnd(z[i * Fz + k], bf16), acc);
  A[e] = acc;
}

// B[t][o] = sum_k W1[o][Fz + k] gamma_t[k]
__global__ void k_prep_B(const float* __restrict__ mlp, const float* __restrict__ gam, int T, int W, int Din,
                         int Fz, int bf16, float* __restrict__ B) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)T * W) return;
  int64_t t = e / W;
  int o = (int)(e % W);
  const int Dt = Din - Fz;
  const float* w1 = mlp + (int64_t)o * Din + Fz;
  float acc = 0.f;
  for (int k = 0; k < Dt; ++k) acc = fmaf(rnd(w1[k], bf16), rnd(gam[t * Dt + k], bf16), acc);
  B[e] = acc;
}

// ---- exponential map (Rodrigues) in float32 --------------------------------
// A = sin(th)/th, B = (1-cos th)/th^2 = 2 sin^2(th/2)/th^2, C = (th - sin th)/th^3.
// One sine-cosine pair of the half angle h = th/2 gives both A = (sin h / h)
// cos h and B = (sin h / h)^2 / 2 (and sin th = 2 sin h cos h); the
// half-angle form of B and a Taylor series of C below th = 0.5 avoid the
// cancellation of the textbook forms in float32.
__device__ __forceinline__ void rod_coef(float th2, float& A, float& B, float& C) {
  float th = sqrtf(th2);
  float sin_th;
  if (th < 1e-4f) {
    A = 1.f - th2 * (1.f / 6.f);
    B = 0.5f - th2 * (1.f / 24.f);
    sin_th = th;
  } else {
    float h = 0.5f * th;
    float s, c;
    sincosf(h, &s, &c);
    float sh = s / h;
    A = sh * c;
    B = 0.5f * sh * sh;
    sin_th = 2.f * s * c;
  }
  if (th < 0.5f) {
    C = (1.f / 6.f) - th2 * ((1.f / 120.f) - th2 * ((1.f / 5040.f) - th2 * ((1.f / 362880.f) - th2 * (1.f / 39916800.f))));
  } else {
    C = (th - sin_th) / (th2 * th);
  }
}

__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
  return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// R(w) n for a direction n (the rotation part alone)
__device__ __forceinline__ float4 rotate_expmap(const float* o, float4 nr) {
  float3 w = make_float3(o[0], o[1], o[2]);
  float A, B, C;
  rod_coef(w.x * w.x + w.y * w.y + w.z * w.z, A, B, C);
  float3 n = make_float3(nr.x, nr.y, nr.z);
  float3 wn = cross3(w, n);
  float3 wwn = cross3(w, wn);
  return make_float4(n.x + A * wn.x + B * wwn.x, n.y + A * wn.y + B * wwn.y, n.z + A * wn.z + B * wwn.z, 0.f);
}

// x^ = R(w) x + tanh(alpha d)
__device__ __forceinline__ float4 apply_transform(const float* o, float4 xr, float alpha) {
  float3 w = make_float3(o[0], o[1], o[2]);
  float A, B, C;
  rod_coef(w.x * w.x + w.y * w.y + w.z * w.z, A, B, C);
  float3 x = make_float3(xr.x, xr.y, xr.z);
  float3 wx = cross3(w, x);
  float3 wwx = cross3(w, wx);
  return make_float4(x.x + A * wx.x + B * wwx.x + tanhf(alpha * o[3]),
                     x.y + A * wx.y + B * wwx.y + tanhf(alpha * o[4]),
                     x.z + A * wx.z + B * wwx.z + tanhf(alpha * o[5]), 0.f);
}

// Gradient of g . x^ w.r.t. o = (w, d): with u = R^T g and c = x cross u,
// d/dw = J_r(w)^T c = c + B (w x c) + C (w x (w x c)); d/dd = alpha (1 - d^2) g.
__device__ __forceinline__ void transform_grad(const float* o, float4 xr, float4 gr, float alpha, float* go) {
  float3 w = make_float3(o[0], o[1], o[2]);
  float A, B, C;
  rod_coef(w.x * w.x + w.y * w.y + w.z * w.z, A, B, C);
  float3 g = make_float3(gr.x, gr.y, gr.z);
  float3 wg = cross3(w, g);
  float3 wwg = cross3(w, wg);
  float3 u = make_float3(g.x - A * wg.x + B * wwg.x, g.y - A * wg.y + B * wwg.y, g.z - A * wg.z + B * wwg.z);
  float3 c = cross3(make_float3(xr.x, xr.y, xr.z), u);
  float3 wc = cross3(w, c);
  float3 wwc = cross3(w, wc);
  go[0] = c.x + B * wc.x + C * wwc.x;
  go[1] = c.y + B * wc.y + C * wwc.y;
  go[2] = c.z + B * wc.z + C * wwc.z;
  for (int k = 0; k < 3; ++k) {
    float dh = tanhf(alpha * o[3 + k]);
    float gk = k == 0 ? g.x : (k == 1 ? g.y : g.z);
    go[3 + k] = alpha * (1.f - dh * dh) * gk;
  }
}

// ---- quaternion head (Sec. 3.4) ----------------------------------------------
// u = (w, v) = (1 + o0, o1, o2, o3) / norm; for a unit quaternion
// R(u) x = x + 2w (v x x) + 2 v x (v x x); d^ = tanh(alpha o[4..6]).
__device__ __forceinline__ float4 apply_quat(const float* o, float4 xr, float alpha) {
  const float a0 = 1.f + o[0];
  const float inv = 1.f / sqrtf(a0 * a0 + o[1] * o[1] + o[2] * o[2] + o[3] * o[3]);
  const float w = a0 * inv;
  const float3 v = make_float3(o[1] * inv, o[2] * inv, o[3] * inv);
  const float3 x = make_float3(xr.x, xr.y, xr.z);
  const float3 t = cross3(v, x);
  const float3 vt = cross3(v, t);
  return make_float4(x.x + 2.f * (w * t.x + vt.x) + tanhf(alpha * o[4]),
                     x.y + 2.f * (w * t.y + vt.y) + tanhf(alpha * o[5]),
                     x.z + 2.f * (w * t.z + vt.z) + tanhf(alpha * o[6]), 0.f);
}

// R(u) n for a direction n (the rotation part alone)
__device__ __forceinline__ float4 rotate_quat(const float* o, float4 nr) {
  const float a0 = 1.f + o[0];
  const float inv = 1.f / sqrtf(a0 * a0 + o[1] * o[1] + o[2] * o[2] + o[3] * o[3]);
  const float w = a0 * inv;
  const float3 v = make_float3(o[1] * inv, o[2] * inv, o[3] * inv);
  const float3 n = make_float3(nr.x, nr.y, nr.z);
  const float3 t = cross3(v, n);
  const float3 vt = cross3(v, t);
  return make_float4(n.x + 2.f * (w * t.x + vt.x), n.y + 2.f * (w * t.y + vt.y), n.z + 2.f * (w * t.z + vt.z), 0.f);
}

// Gradient of g . x^ w.r.t. the 7 outputs. With the form above,
// d/dw = 2 g.(v x x), d/dv = 2w (x x g) + 2 [g (v.x) + x (g.v) - 2 v (g.x)];
// the normalisation maps a gradient gu on u to (gu - u (u.gu)) / norm.
__device__ __forceinline__ void quat_grad(const float* o, float4 xr, float4 gr, float alpha, float* go) {
  const float a0 = 1.f + o[0];
  const float inv = 1.f / sqrtf(a0 * a0 + o[1] * o[1] + o[2] * o[2] + o[3] * o[3]);
  const float w = a0 * inv;
  const float3 v = make_float3(o[1] * inv, o[2] * inv, o[3] * inv);
  const float3 x = make_float3(xr.x, xr.y, xr.z);
  const float3 g = make_float3(gr.x, gr.y, gr.z);
  const float3 vx = cross3(v, x), xg = cross3(x, g);
  const float vdx = v.x * x.x + v.y * x.y + v.z * x.z;
  const float gdv = g.x * v.x + g.y * v.y + g.z * v.z;
  const float gdx = g.x * x.x + g.y * x.y + g.z * x.z;
  const float gw = 2.f * (g.x * vx.x + g.y * vx.y + g.z * vx.z);
  const float g1 = 2.f * (w * xg.x + g.x * vdx + x.x * gdv - 2.f * v.x * gdx);
  const float g2 = 2.f * (w * xg.y + g.y * vdx + x.y * gdv - 2.f * v.y * gdx);
  const float g3 = 2.f * (w * xg.z + g.z * vdx + x.z * gdv - 2.f * v.z * gdx);
  const float ug = w * gw + v.x * g1 + v.y * g2 + v.z * g3;
  go[0] = (gw - w * ug) * inv;
  go[1] = (g1 - v.x * ug) * inv;
  go[2] = (g2 - v.y * ug) * inv;
  go[3] = (g3 - v.z * ug) * inv;
  for (int k = 0; k < 3; ++k) {
    float dh = tanhf(alpha * o[4 + k]);
    float gk = k == 0 ? g.x : (k == 1 ? g.y : g.z);
    go[4 + k] = alpha * (1.f - dh * dh) * gk;
  }
}

// out[mt] += sum_k Wrow(16mt + c, k) * in[k] over all k tiles; wl(mt, kt)
// returns the float4 of row 16mt + c at columns 16kt + 4q .. +3. The operands
// of k-tile kt+1 are requested before the MFMAs of k-tile kt are issued, so
// their latency hides behind the matrix work.
template <int NT, typename WL>
__device__ __forceinline__ void dense(const v4f (&in)[NT], v4f (&out)[NT], WL wl) {
  float4 w[2][NT];
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) w[0][mt] = wl(mt, 0);
#pragma unroll
  for (int kt = 0; kt < NT; ++kt) {
    const int cb = kt & 1;
    if (kt + 1 < NT) {
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) w[cb ^ 1][mt] = wl(mt, kt + 1);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) out[mt] = mfma(comp(w[cb][mt], r), in[kt][r], out[mt]);
    // keep later k-tiles' loads from being hoisted further up
    __builtin_amdgcn_sched_barrier(0);
  }
}

// 16-row output layer (rows n_out..15 zero): o = Wo h + bo.
template <int NT, typename WL>
__device__ __forceinline__ v4f dense_out(const v4f (&in)[NT], v4f init, WL wl) {
  v4f a0 = init, a1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < NT; ++kt) {
    float4 w = wl(kt);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (kt & 1) a1 = mfma(comp(w, r), in[kt][r], a1);
      else a0 = mfma(comp(w, r), in[kt][r], a0);
    }
  }
  return a0 + a1;
}

// Forward activations of one 16-sample tile: h[l] for the H hidden layers.
template <int W, int H, typename WH, typename BH>
__device__ __forceinline__ void mlp_hidden(v4f (&h)[H][W / 16], const float* __restrict__ A,
                                           const float* __restrict__ B, int64_t i, int64_t t, int q, ActP ap,
                                           WH wh, BH bh) {
  constexpr int NT = W / 16;
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    float4 a = *reinterpret_cast<const float4*>(A + i * W + 16 * mt + 4 * q);
    float4 b = *reinterpret_cast<const float4*>(B + t * W + 16 * mt + 4 * q);
    h[0][mt] = v4f{actf(a.x + b.x, ap), actf(a.y + b.y, ap), actf(a.z + b.z, ap), actf(a.w + b.w, ap)};
  }
#pragma unroll
  for (int l = 1; l < H; ++l) {
    v4f o[NT];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
      float4 b = bh(l, mt);
      o[mt] = v4f{b.x, b.y, b.z, b.w};
    }
    dense<NT>(h[l - 1], o, [&](int mt, int kt) { return wh(l, mt, kt); });
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
      h[l][mt] = v4f{actf(o[mt][0], ap), actf(o[mt][1], ap), actf(o[mt][2], ap), actf(o[mt][3], ap)};
  }
}

// ---------------------------------------------------------------------------
// Forward: 8 waves per work-group share the hidden and output weights in LDS;
// each wave decodes 16-sample tiles in a grid-stride loop. STORE: the hidden
// activations of layers 2..H are also written to act ([T][V][H-1][W], sample
// s = t V + i), for a backward that then does not recompute them.
// ---------------------------------------------------------------------------
template <int W, int H, bool STORE>
__global__ __launch_bounds__(512) void k_decode_fwd(const float* __restrict__ wp, const float* __restrict__ A,
                                                    const float* __restrict__ B, const float4* __restrict__ xyz,
                                                    float4* __restrict__ xhat, int64_t V, int T, ActP ap,
                                                    float alpha, int quat, const float4* __restrict__ nrm,
                                                    float4* __restrict__ nhat, float* __restrict__ act) {
  constexpr int NT = W / 16;
  constexpr int LD = W + 4;  // padded LDS row
  extern __shared__ float lds[];
  float* sW = lds;                           // [H-1][W][LD]
  float* sWo = sW + (H - 1) * W * LD;        // [16][LD]
  float* sB = sWo + 16 * LD;                 // [H-1][W] + [16]
  const WPack P(W, H);
  for (int e = threadIdx.x; e < (H - 1) * W * W; e += blockDim.x) {
    int l = e / (W * W), k = e % (W * W);
    sW[(l * W + k / W) * LD + k % W] = wp[P.wh + e];
  }
  for (int e = threadIdx.x; e < 16 * W; e += blockDim.x) sWo[(e / W) * LD + e % W] = wp[P.wop + e];
  for (int e = threadIdx.x; e < (H - 1) * W; e += blockDim.x) sB[e] = wp[P.bh + e];
  for (int e = threadIdx.x; e < 16; e += blockDim.x) sB[(H - 1) * W + e] = wp[P.bo + e];
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, c = lane & 15;
  const int nw = blockDim.x >> 6;
  const int64_t S = V * (int64_t)T;
  const int64_t ntiles = (S + 15) / 16;
  auto wh = [&](int l, int mt, int kt) {
    return *reinterpret_cast<const float4*>(sW + ((l - 1) * W + 16 * mt + c) * LD + 16 * kt + 4 * q);
  };
  auto bh = [&](int l, int mt) { return *reinterpret_cast<const float4*>(sB + (l - 1) * W + 16 * mt + 4 * q); };
  auto wo = [&](int kt) { return *reinterpret_cast<const float4*>(sWo + c * LD + 16 * kt + 4 * q); };
  float4 bo4 = *reinterpret_cast<const float4*>(sB + (H - 1) * W + 4 * q);
  const v4f boi = v4f{bo4.x, bo4.y, bo4.z, bo4.w};

  for (int64_t tile = (int64_t)blockIdx.x * nw + wave; tile < ntiles; tile += (int64_t)gridDim.x * nw) {
    // opaque zero: keeps the LDS weight reads inside the loop (not hoisted)
    int z0 = 0;
    asm volatile("" : "+s"(z0));
    const float* sWl = sW + z0;
    const float* sWol = sWo + z0;
    auto whl = [&](int l, int mt, int kt) {
      return *reinterpret_cast<const float4*>(sWl + ((l - 1) * W + 16 * mt + c) * LD + 16 * kt + 4 * q);
    };
    auto wol = [&](int kt) { return *reinterpret_cast<const float4*>(sWol + c * LD + 16 * kt + 4 * q); };
    int64_t s = tile * 16 + c;
    const bool valid = s < S;
    if (!valid) s = S - 1;
    const int64_t t = s / V, i = s - t * V;
    v4f h[H][NT];
    mlp_hidden<W, H>(h, A, B, i, t, q, ap, whl, bh);
    if (STORE && valid) {
      float* dst = act + s * (int64_t)((H - 1) * W) + 4 * q;
#pragma unroll
      for (int l = 1; l < H; ++l)
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
          *reinterpret_cast<float4*>(dst + (l - 1) * W + 16 * mt) =
              make_float4(h[l][mt][0], h[l][mt][1], h[l][mt][2], h[l][mt][3]);
    }
    v4f o = dense_out<NT>(h[H - 1], boi, wol);
    float o4 = __shfl(o[0], (lane + 16) & 63);
    float o5 = __shfl(o[1], (lane + 16) & 63);
    float o6 = __shfl(o[2], (lane + 16) & 63);
    if (q == 0 && valid) {
      float ov[7] = {o[0], o[1], o[2], o[3], o4, o5, o6};
      xhat[s] = quat ? apply_quat(ov, xyz[i], alpha) : apply_transform(ov, xyz[i], alpha);
      if (nhat) nhat[s] = quat ? rotate_quat(ov, nrm[i]) : rotate_expmap(ov, nrm[i]);
    }
  }
}

// ---------------------------------------------------------------------------
// Backward: one work-group = 4 waves = 64 vertices, looping over all frames.
// ---------------------------------------------------------------------------
constexpr int kSP = 68;  // staged samples per row (64 + pad)

// LDS of the backward (floats): sH [H][W][kSP] recomputed activations of the
// work-group's 64 samples, sG [W][kSP] staged gradient rows, sGb bias
// gradients [H-1][W] + [16], sGt [4][W] per-wave frame sums.
template <int W, int H>
constexpr size_t bwd_lds_floats() {
  return (size_t)H * W * kSP + (size_t)W * kSP + (H - 1) * W + 16 + 4 * W;
}

// STORED: the hidden activations of layers 2..H are read from act (written
// by the forward of the same parameters, bitwise what the recompute gives)
// instead of recomputed; the first layer's act(A_i + B_t) is always formed.
template <int W, int H, bool STORED>
__global__ __launch_bounds__(256) void k_decode_bwd(const float* __restrict__ wp, const float* __restrict__ A,
                                                    const float* __restrict__ B, const float4* __restrict__ xyz,
                                                    const float4* __restrict__ gxhat, int64_t V, int T, ActP ap,
                                                    float alpha, int quat, int nvb, int nch, float* __restrict__ Gv,
                                                    float* __restrict__ Gt_part, float* __restrict__ gW_part,
                                                    const float* __restrict__ act) {
  constexpr int NT = W / 16;
  constexpr int NTT = (NT * NT + 3) / 4;  // owned hidden weight-gradient tiles per wave
  constexpr int NTO = (NT + 3) / 4;       // owned output weight-gradient tiles per wave
  extern __shared__ float lds[];
  float* sH = lds;                        // [H][W][kSP]
  float* sG = sH + H * W * kSP;           // [W][kSP]
  float* sGb = sG + W * kSP;              // [H-1][W] + [16]
  float* sGt = sGb + (H - 1) * W + 16;    // [4][W]
  const WPack P(W, H);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, c = lane & 15;
  const int sp = wave * 16 + c;

  for (int e = threadIdx.x; e < (H - 1) * W + 16; e += 256) sGb[e] = 0.f;

  float4 bo4 = *reinterpret_cast<const float4*>(wp + P.bo + 4 * q);
  const v4f boi = v4f{bo4.x, bo4.y, bo4.z, bo4.w};

  v4f accW[H > 1 ? H - 1 : 1][NTT];
  v4f accO[NTO];
  v4f gv[NT];
#pragma unroll
  for (int l = 0; l < (H > 1 ? H - 1 : 1); ++l)
#pragma unroll
    for (int k = 0; k < NTT; ++k) accW[l][k] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < NTO; ++k) accO[k] = v4f{0.f, 0.f, 0.f, 0.f};
  __syncthreads();

  // this lane's element (feature 16*mt + 4q + r, own sample) of a staged row block
  auto at = [&](float* base, int mt, int r) -> float& { return base[(16 * mt + 4 * q + r) * kSP + sp]; };
  // acc += sum over the 64 staged samples of sG[16mt + m][s] * hs[16kt + n][s]
  auto wgrad_load = [&](const float* hs, int mt, int kt, float4 (&a)[4], float4 (&b)[4]) {
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      a[jj] = *reinterpret_cast<const float4*>(sG + (16 * mt + c) * kSP + 16 * q + 4 * jj);
      b[jj] = *reinterpret_cast<const float4*>(hs + (16 * kt + c) * kSP + 16 * q + 4 * jj);
    }
  };
  auto wgrad_mma = [&](const float4 (&a)[4], const float4 (&b)[4], v4f acc) {
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mfma(comp(a[jj], r), comp(b[jj], r), acc);
    return acc;
  };
  // all owned tiles of one layer, operands of tile k+1 fetched before tile k's MFMAs
  auto wgrad_layer = [&](const float* hs, auto& accs, int ntiles_total, int ncols) {
    constexpr int NA = sizeof(accs) / sizeof(v4f);
    float4 a[2][4], b[2][4];
    if (wave < ntiles_total) wgrad_load(hs, wave / ncols, wave % ncols, a[0], b[0]);
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const int tau = wave + 4 * k;
      if (tau >= ntiles_total) break;
      const int nx = tau + 4;
      if (k + 1 < NA && nx < ntiles_total) wgrad_load(hs, nx / ncols, nx % ncols, a[(k + 1) & 1], b[(k + 1) & 1]);
      accs[k] = wgrad_mma(a[k & 1], b[k & 1], accs[k]);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  // bias gradient rows: thread tid sums staged gradient row tid over the 64 samples
  auto bias_rows = [&](int rows, float* dst) {
    if ((int)threadIdx.x < rows) {
      const float* src = sG + threadIdx.x * kSP;
      float s0 = 0.f;
      for (int j = 0; j < 64; j += 4) {
        float4 v = *reinterpret_cast<const float4*>(src + j);
        s0 += (v.x + v.y) + (v.z + v.w);
      }
      dst[threadIdx.x] += s0;
    }
  };

  // work items (block of 64 vertices, chunk of frames) in a fixed round-robin
  // order; the weight-gradient accumulators run over all of them
  const int64_t n_items = (int64_t)nvb * nch;
  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int64_t vb = item % nvb;
    const int ch = (int)(item / nvb);
    const int t0 = (int)((int64_t)T * ch / nch), t1 = (int)((int64_t)T * (ch + 1) / nch);
    const int64_t i_raw = vb * 64 + wave * 16 + c;
    const bool vvalid = i_raw < V;
    const int64_t i = vvalid ? i_raw : V - 1;
    const float4 xi = xyz[i];
#pragma unroll
    for (int k = 0; k < NT; ++k) gv[k] = v4f{0.f, 0.f, 0.f, 0.f};
    // the stored activations of the frame to come, loaded one frame ahead
    float4 hn[STORED ? H - 1 : 1][NT];
    auto load_act = [&](int t) {
      const float* src = act + ((int64_t)t * V + i) * ((H - 1) * W) + 4 * q;
#pragma unroll
      for (int l = 1; l < H; ++l)
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) hn[l - 1][mt] = *reinterpret_cast<const float4*>(src + (l - 1) * W + 16 * mt);
    };
    if (STORED) load_act(t0);
    for (int t = t0; t < t1; ++t) {
      // Opaque copies of the weight pointers: keeps the compiler from hoisting
      // every (loop-invariant) weight load of the frame loop into registers.
      const float* wpl = wp;
      asm volatile("" : "+s"(wpl));
      const float* Wh = wpl + P.wh;
      const float* WhT = wpl + P.wht;
      // ---- recompute the forward pass; activations go to LDS ---------------
      v4f h[NT];
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) {
        float4 a = *reinterpret_cast<const float4*>(A + i * W + 16 * mt + 4 * q);
        float4 b = *reinterpret_cast<const float4*>(B + (int64_t)t * W + 16 * mt + 4 * q);
        h[mt] = v4f{actf(a.x + b.x, ap), actf(a.y + b.y, ap), actf(a.z + b.z, ap), actf(a.w + b.w, ap)};
#pragma unroll
        for (int r = 0; r < 4; ++r) at(sH, mt, r) = h[mt][r];
      }
      if (STORED) {
#pragma unroll
        for (int l = 1; l < H; ++l)
#pragma unroll
          for (int mt = 0; mt < NT; ++mt) {
            const float4 v = hn[l - 1][mt];
            h[mt] = v4f{v.x, v.y, v.z, v.w};
#pragma unroll
            for (int r = 0; r < 4; ++r) at(sH + l * W * kSP, mt, r) = h[mt][r];
          }
        if (t + 1 < t1) load_act(t + 1);
      } else {
#pragma unroll
        for (int l = 1; l < H; ++l) {
          v4f o[NT];
#pragma unroll
          for (int mt = 0; mt < NT; ++mt) {
            float4 b = *reinterpret_cast<const float4*>(wpl + P.bh + (l - 1) * W + 16 * mt + 4 * q);
            o[mt] = v4f{b.x, b.y, b.z, b.w};
          }
          dense<NT>(h, o, [&](int mt, int kt) {
            return *reinterpret_cast<const float4*>(Wh + (int64_t)(l - 1) * W * W + (16 * mt + c) * W + 16 * kt +
                                                    4 * q);
          });
#pragma unroll
          for (int mt = 0; mt < NT; ++mt) {
            h[mt] = v4f{actf(o[mt][0], ap), actf(o[mt][1], ap), actf(o[mt][2], ap), actf(o[mt][3], ap)};
#pragma unroll
            for (int r = 0; r < 4; ++r) at(sH + l * W * kSP, mt, r) = h[mt][r];
          }
        }
      }
      v4f o = dense_out<NT>(h, boi, [&](int kt) {
        return *reinterpret_cast<const float4*>(wpl + P.wop + c * W + 16 * kt + 4 * q);
      });

      // ---- transform backward: every lane evaluates its sample c -----------
      float o4 = __shfl(o[0], (lane + 16) & 63);
      float o5 = __shfl(o[1], (lane + 16) & 63);
      float o6 = __shfl(o[2], (lane + 16) & 63);
      float ov[7] = {__shfl(o[0], c), __shfl(o[1], c), __shfl(o[2], c), __shfl(o[3], c), __shfl(o4, c),
                     __shfl(o5, c), __shfl(o6, c)};
      float4 gx = vvalid ? gxhat[(int64_t)t * V + i] : make_float4(0.f, 0.f, 0.f, 0.f);
      float go[7];
      go[6] = 0.f;
      if (quat) quat_grad(ov, xi, gx, alpha, go);
      else transform_grad(ov, xi, gx, alpha, go);
      if (!vvalid)
        for (int k = 0; k < 7; ++k) go[k] = 0.f;
      const v4f got = q == 0 ? v4f{go[0], go[1], go[2], go[3]}
                             : (q == 1 ? v4f{go[4], go[5], go[6], 0.f} : v4f{0.f, 0.f, 0.f, 0.f});

      // ---- output layer: weight gradient and back-propagation ---------------
#pragma unroll
      for (int r = 0; r < 4; ++r) at(sG, 0, r) = got[r];
      __syncthreads();
      wgrad_layer(sH + (H - 1) * W * kSP, accO, NT, NT);
      bias_rows(16, sGb + (H - 1) * W);
      v4f gp[NT];
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) {
        float4 w = *reinterpret_cast<const float4*>(wpl + P.wot + (16 * mt + c) * 16 + 4 * q);
        v4f a = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < 4; ++r) a = mfma(comp(w, r), got[r], a);
#pragma unroll
        for (int r = 0; r < 4; ++r) gp[mt][r] = a[r] * actd(at(sH + (H - 1) * W * kSP, mt, r), ap);
      }
      __syncthreads();

      // ---- hidden layers, last to first --------------------------------------
#pragma unroll
      for (int l = H - 1; l >= 1; --l) {
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) at(sG, mt, r) = gp[mt][r];
        __syncthreads();
        wgrad_layer(sH + (l - 1) * W * kSP, accW[l - 1], NT * NT, NT);
        bias_rows(W, sGb + (l - 1) * W);
        v4f gh[NT];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) gh[mt] = v4f{0.f, 0.f, 0.f, 0.f};
        dense<NT>(gp, gh, [&](int mt, int kt) {
          return *reinterpret_cast<const float4*>(WhT + (int64_t)(l - 1) * W * W + (16 * mt + c) * W + 16 * kt + 4 * q);
        });
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) gp[mt][r] = gh[mt][r] * actd(at(sH + (l - 1) * W * kSP, mt, r), ap);
        __syncthreads();
      }

      // ---- first layer: per-vertex (Gv) and per-frame (Gt) sums -------------
#pragma unroll
      for (int mt = 0; mt < NT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          gv[mt][r] += gp[mt][r];
          const float v = row16_sum(gp[mt][r]);
          if (c == 0) sGt[wave * W + 16 * mt + 4 * q + r] = v;
        }
      __syncthreads();
      if ((int)threadIdx.x < W) {
        float s0 = ((sGt[threadIdx.x] + sGt[W + threadIdx.x]) + sGt[2 * W + threadIdx.x]) + sGt[3 * W + threadIdx.x];
        Gt_part[((int64_t)t * nvb + vb) * W + threadIdx.x] = s0;
      }
    }
    if (vvalid) {  // this chunk's per-vertex sums
      float* dv = Gv + ((int64_t)ch * V + i_raw) * W;
#pragma unroll
      for (int mt = 0; mt < NT; ++mt)
        *reinterpret_cast<float4*>(dv + 16 * mt + 4 * q) = make_float4(gv[mt][0], gv[mt][1], gv[mt][2], gv[mt][3]);
    }
  }
  __syncthreads();

  // per-work-group weight-gradient partials, flat MLP layout of layers 1..H
  const int n_out = quat ? 7 : 6;
  const int64_t len = (int64_t)(H - 1) * ((int64_t)W * W + W) + n_out * (int64_t)W + n_out;
  float* dst = gW_part + (int64_t)blockIdx.x * len;
#pragma unroll
  for (int l = 1; l < H; ++l) {
    float* dl = dst + (int64_t)(l - 1) * ((int64_t)W * W + W);
#pragma unroll
    for (int k = 0; k < NTT; ++k) {
      int tau = wave + 4 * k;
      if (tau < NT * NT) {
        int mt = tau / NT, kt = tau % NT;
#pragma unroll
        for (int r = 0; r < 4; ++r) dl[(16 * mt + 4 * q + r) * W + 16 * kt + c] = accW[l - 1][k][r];
      }
    }
    for (int e = threadIdx.x; e < W; e += 256) dl[(int64_t)W * W + e] = sGb[(l - 1) * W + e];
  }
  float* dout = dst + (int64_t)(H - 1) * ((int64_t)W * W + W);
#pragma unroll
  for (int k = 0; k < NTO; ++k) {
    int kt = wave + 4 * k;
    if (kt < NT) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (4 * q + r < n_out) dout[(4 * q + r) * W + 16 * kt + c] = accO[k][r];
    }
  }
  if ((int)threadIdx.x < n_out) dout[n_out * W + threadIdx.x] = sGb[(H - 1) * W + threadIdx.x];
}

// ===========================================================================
// BF16 form. Every MLP matrix operand (hidden activations, weights,
// back-propagated gradients) is rounded to bfloat16 and multiplied on
// v_mfma_f32_16x16x32_bf16 with float32 accumulation. Lane (q, c) supplies 8
// operand values; its slot j stands for K index 16*(j/4) + 4q + j%4 of the
// 32-wide K block, so the B operand of K block kb is the register pair
// (tile 2kb, tile 2kb+1) of a feature-major activation (rows 4q + r of each
// 16-row tile at lane q) and layers chain without moving data. Weight rows
// are staged once per work-group into LDS with their columns permuted within
// every 32-column block to that slot order (one 16-byte read per operand);
// back-propagation reads the transposed operands from the same rows with the
// LDS transpose load.
// ===========================================================================
typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2b __attribute__((ext_vector_type(2)));
typedef __bf16 v4b __attribute__((ext_vector_type(4)));
typedef __bf16 v8b __attribute__((ext_vector_type(8)));
#define NPG_LDS __attribute__((address_space(3)))

// round to nearest even (the conversion instruction, denormals kept: the same
// result as npg_bf16_bits)
__device__ __forceinline__ v4s pack_bf16(const v4f& v) {
  const v2b lo = __builtin_convertvector((v2f{v[0], v[1]}), v2b);
  const v2b hi = __builtin_convertvector((v2f{v[2], v[3]}), v2b);
  return __builtin_bit_cast(v4s, __builtin_shufflevector(lo, hi, 0, 1, 2, 3));
}
__device__ __forceinline__ float bf16_val(short h) { return __uint_as_float((uint32_t)(uint16_t)h << 16); }
// K = 16 product (lane (q, c) supplies K indices 4q..4q+3)
__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8b, a), __builtin_bit_cast(v8b, b), c, 0, 0, 0);
}
__device__ __forceinline__ v8s cat8(v4s lo, v4s hi) { return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7); }
__device__ __forceinline__ v8s lds8(const uint16_t* p) { return *reinterpret_cast<const v8s*>(p); }
// LDS transpose load: every lane reads 4 consecutive bfloat16 at p; within
// each group of 16 lanes, lane 4a + b receives element b of the reads of
// lanes a, 4 + a, 8 + a, 12 + a (in that order).
__device__ __forceinline__ v4s lds_tr(const uint16_t* p) {
  NPG_LDS uint16_t* l = (NPG_LDS uint16_t*)const_cast<uint16_t*>(p);
  return __builtin_bit_cast(v4s, __builtin_amdgcn_ds_read_tr16_b64_v4bf16(reinterpret_cast<NPG_LDS v4b*>(l)));
}
// LDS position of weight column k within its row (the slot order above)
__device__ __forceinline__ int kpos(int k) {
  return (k & ~31) | (((k >> 2) & 3) << 3) | (((k >> 4) & 1) << 2) | (k & 3);
}

// bfloat16 copy of the float32 weight pack (same layout)
__global__ void k_pack_bf16(const float* __restrict__ src, int64_t n, uint16_t* __restrict__ dst) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n) dst[e] = npg_bf16_bits(src[e]);
}

// LDS rows of staged bfloat16 weights: row stride LD; for W = 32 and 128 the
// 16-byte chunks of a row are XOR-swizzled by a function of the row's low 4
// bits (a bijection whose high 2 bits differ between the 4 rows one 16-lane
// transpose read touches), so the row reads of the forward pass and the
// transpose reads of back-propagation both spread over the LDS banks. All
// row bases passed around are multiples of 16 rows.
template <int W>
struct WLds {
  static constexpr bool kSwz = (W != 64);
  static constexpr int LD = kSwz ? W : W + 8;
  __device__ static int swz(int row) {
    return kSwz ? ((((row & 3) << 2) | ((row >> 2) & 3)) & (W / 8 - 1)) : 0;
  }
  // element offset of permuted position p of row `row`
  __device__ static int at(int row, int p) { return row * LD + ((((p >> 3) ^ swz(row))) << 3) + (p & 7); }
};

// Stage the hidden matrices (H-1 blocks of W rows, row = output unit) and the
// 16 output rows into LDS in permuted column order.
template <int W, int H>
__device__ void stage_w16(const uint16_t* __restrict__ wp16, uint16_t* sW) {
  using L = WLds<W>;
  const WPack P(W, H);
  for (int e = threadIdx.x; e < (H - 1) * W * W; e += blockDim.x) sW[L::at(e / W, kpos(e % W))] = wp16[P.wh + e];
  for (int e = threadIdx.x; e < 16 * W; e += blockDim.x) sW[L::at((H - 1) * W + e / W, kpos(e % W))] = wp16[P.wop + e];
}

// out[mt] += sum_k Wl[16mt + c][k] in[k] over the W inputs (feature-major).
// With PF the next K block's weights are read while the current one
// multiplies (NT more operand registers).
template <int W, bool PF>
__device__ __forceinline__ void dense32(const v4s (&in)[W / 16], v4f (&out)[W / 16], const uint16_t* sWl, int q,
                                        int c) {
  constexpr int NT = W / 16;
  using L = WLds<W>;
  const int sc = L::swz(c);  // rows 16mt + c share their low 4 bits
  auto frag = [&](int mt, int kb) { return lds8(sWl + (16 * mt + c) * L::LD + (((4 * kb + q) ^ sc) << 3)); };
  v8s w[PF ? 2 : 1][NT];
  if (PF) {
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) w[0][mt] = frag(mt, 0);
  }
#pragma unroll
  for (int kb = 0; kb < NT / 2; ++kb) {
    const int cb = PF ? (kb & 1) : 0;
    if (PF && kb + 1 < NT / 2) {
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) w[cb ^ 1][mt] = frag(mt, kb + 1);
    }
    if (!PF) {
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) w[0][mt] = frag(mt, kb);
    }
    const v8s b = cat8(in[2 * kb], in[2 * kb + 1]);
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) out[mt] = mfma32(w[cb][mt], b, out[mt]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// output rows (sWo: the 16 output rows): init + sum_k Wo[c][k] in[k]
template <int W>
__device__ __forceinline__ v4f dense_out32(const v4s (&in)[W / 16], v4f init, const uint16_t* sWo, int q, int c) {
  using L = WLds<W>;
  const int sc = L::swz(c);
  v4f a0 = init, a1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < W / 32; ++kb) {
    const v4f r = mfma32(lds8(sWo + c * L::LD + (((4 * kb + q) ^ sc) << 3)), cat8(in[2 * kb], in[2 * kb + 1]),
                         (kb & 1) ? a1 : a0);
    if (kb & 1) a1 = r;
    else a0 = r;
  }
  return a0 + a1;
}

// Transpose read of 4 weights for back-propagation: lane (q, c) reads row
// `row` (its low 4 bits = 4q + c/4) at the permuted position of columns
// 16mt + 4(c%4) .. +3, i.e. chunk 4(mt/2) + c%4, half mt%2.
template <int W>
__device__ __forceinline__ v4s wtr(const uint16_t* sWl, int row, int mt, int c) {
  using L = WLds<W>;
  return lds_tr(sWl + row * L::LD + (((4 * (mt >> 1) + (c & 3)) ^ L::swz(row)) << 3) + 4 * (mt & 1));
}

// out[mt] += sum_k Wl[k][16mt + c] g[k]: back-propagation through the rows of
// Wl with the transposed operands from the LDS transpose read
template <int W>
__device__ __forceinline__ void dgrad32(const v4s (&g)[W / 16], v4f (&out)[W / 16], const uint16_t* sWl, int q,
                                        int c) {
  constexpr int NT = W / 16;
  const int rl = 4 * q + (c >> 2);
#pragma unroll
  for (int kb = 0; kb < NT / 2; ++kb) {
    const v8s b = cat8(g[2 * kb], g[2 * kb + 1]);
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
      const v4s lo = wtr<W>(sWl, 32 * kb + rl, mt, c);
      const v4s hi = wtr<W>(sWl, 32 * kb + 16 + rl, mt, c);
      out[mt] = mfma32(cat8(lo, hi), b, out[mt]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// out_u[mt] += sum_k Wl[16mt + c][k] in_u[k] for two 16-sample tiles u: each
// weight operand read from LDS feeds both tiles' products.
template <int W>
__device__ __forceinline__ void dense32x2(const v4s (&in0)[W / 16], const v4s (&in1)[W / 16],
                                          v4f (&out0)[W / 16], v4f (&out1)[W / 16], const uint16_t* sWl, int q,
                                          int c) {
  constexpr int NT = W / 16;
  using L = WLds<W>;
  const int sc = L::swz(c);
  auto frag = [&](int mt, int kb) { return lds8(sWl + (16 * mt + c) * L::LD + (((4 * kb + q) ^ sc) << 3)); };
  v8s w[2][NT];
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) w[0][mt] = frag(mt, 0);
#pragma unroll
  for (int kb = 0; kb < NT / 2; ++kb) {
    const int cb = kb & 1;
    if (kb + 1 < NT / 2) {
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) w[cb ^ 1][mt] = frag(mt, kb + 1);
    }
    const v8s b0 = cat8(in0[2 * kb], in0[2 * kb + 1]);
    const v8s b1 = cat8(in1[2 * kb], in1[2 * kb + 1]);
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
      out0[mt] = mfma32(w[cb][mt], b0, out0[mt]);
      out1[mt] = mfma32(w[cb][mt], b1, out1[mt]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// the output rows for two tiles (same summation order as dense_out32)
template <int W>
__device__ __forceinline__ void dense_out32x2(const v4s (&in0)[W / 16], const v4s (&in1)[W / 16], v4f init,
                                              const uint16_t* sWo, int q, int c, v4f& r0, v4f& r1) {
  using L = WLds<W>;
  const int sc = L::swz(c);
  v4f a0 = init, a1 = {0.f, 0.f, 0.f, 0.f}, b0 = init, b1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < W / 32; ++kb) {
    const v8s w = lds8(sWo + c * L::LD + (((4 * kb + q) ^ sc) << 3));
    if (kb & 1) {
      a1 = mfma32(w, cat8(in0[2 * kb], in0[2 * kb + 1]), a1);
      b1 = mfma32(w, cat8(in1[2 * kb], in1[2 * kb + 1]), b1);
    } else {
      a0 = mfma32(w, cat8(in0[2 * kb], in0[2 * kb + 1]), a0);
      b0 = mfma32(w, cat8(in1[2 * kb], in1[2 * kb + 1]), b0);
    }
  }
  r0 = a0 + a1;
  r1 = b0 + b1;
}

// activation of 4 values and bfloat16 packing (RELU: the median with 0)
template <bool RELU>
__device__ __forceinline__ v4s act_pack(v4f x, float s) {
  v4f y;
#pragma unroll
  for (int j = 0; j < 4; ++j) y[j] = __builtin_amdgcn_fmed3f(x[j], RELU ? 0.f : s * x[j], kFltMax);
  return pack_bf16(y);
}

// g * actd(h) for a bfloat16 activation output h (its bits): h > 0 exactly
// when the bits, read as a 16-bit integer, are positive
__device__ __forceinline__ float actd_mul(float g, short h, float s) { return h > 0 ? g : s * g; }

// The forward items of one wave (see k_decode_fwd16).
template <int W, int H, bool RELU>
__device__ __forceinline__ void fwd16_items(const uint16_t* sW, const float* sB, const float* __restrict__ A,
                                            const float* __restrict__ B, const float4* __restrict__ xyz,
                                            float4* __restrict__ xhat, int64_t V, int T, float s, float alpha,
                                            int quat, const float4* __restrict__ nrm, float4* __restrict__ nhat,
                                            int pc, int nch, int64_t it0, int64_t stride) {
  constexpr int NT = W / 16;
  constexpr int LD = WLds<W>::LD;
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, c = lane & 15;
  const int np = (T + 1) / 2;
  const int64_t items = (V + 15) / 16 * nch;
  const float4 bo4 = *reinterpret_cast<const float4*>(sB + (H - 1) * W + 4 * q);
  const v4f boi = v4f{bo4.x, bo4.y, bo4.z, bo4.w};

  for (int64_t it = it0; it < items; it += stride) {
    const int64_t vb = it / nch;
    const int ch = (int)(it - vb * nch);
    const int p0 = ch * pc, p1 = min(np, p0 + pc);
    const int64_t i = vb * 16 + c;
    const bool vvalid = i < V;
    const int64_t ic = vvalid ? i : V - 1;
    float4 av[NT];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) av[mt] = *reinterpret_cast<const float4*>(A + ic * W + 16 * mt + 4 * q);
    const float4 xr = xyz[ic];
    const float4 nr = nhat ? nrm[ic] : make_float4(0.f, 0.f, 0.f, 0.f);
    for (int pp = p0; pp < p1; ++pp) {
      const int t0 = 2 * pp, t1 = min(2 * pp + 1, T - 1);
      // first layer: act(A_i + B_t) of both frames
      v4s h0[NT], h1[NT];
      {
        float4 b0[NT], b1[NT];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
          b0[mt] = *reinterpret_cast<const float4*>(B + (int64_t)t0 * W + 16 * mt + 4 * q);
          b1[mt] = *reinterpret_cast<const float4*>(B + (int64_t)t1 * W + 16 * mt + 4 * q);
        }
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
          const float4 a = av[mt];
          h0[mt] = act_pack<RELU>(v4f{a.x + b0[mt].x, a.y + b0[mt].y, a.z + b0[mt].z, a.w + b0[mt].w}, s);
          h1[mt] = act_pack<RELU>(v4f{a.x + b1[mt].x, a.y + b1[mt].y, a.z + b1[mt].z, a.w + b1[mt].w}, s);
        }
      }
#pragma unroll
      for (int l = 1; l < H; ++l) {
        v4f a[NT], b[NT];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
          const float4 bb = *reinterpret_cast<const float4*>(sB + (l - 1) * W + 16 * mt + 4 * q);
          a[mt] = v4f{bb.x, bb.y, bb.z, bb.w};
          b[mt] = a[mt];
        }
        dense32x2<W>(h0, h1, a, b, sW + (l - 1) * W * LD, q, c);
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
          h0[mt] = act_pack<RELU>(a[mt], s);
          h1[mt] = act_pack<RELU>(b[mt], s);
        }
      }
      v4f o0, o1;
      dense_out32x2<W>(h0, h1, boi, sW + (H - 1) * W * LD, q, c, o0, o1);
      // lanes 0-15 take frame t0's 7 outputs of column c, lanes 16-31 frame t1's
      float ov[7];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float x1 = __shfl(o1[j], c);
        ov[j] = q == 0 ? o0[j] : x1;
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float x0 = __shfl(o0[j], c + 16);
        ov[4 + j] = q == 0 ? x0 : o1[j];
      }
      if (q < 2 && vvalid && (q == 0 || 2 * pp + 1 < T)) {
        const int64_t sidx = (int64_t)(q ? t1 : t0) * V + i;
        xhat[sidx] = quat ? apply_quat(ov, xr, alpha) : apply_transform(ov, xr, alpha);
        if (nhat) nhat[sidx] = quat ? rotate_quat(ov, nr) : rotate_expmap(ov, nr);
      }
    }
  }
}

// Persistent forward pass: the work-group stages the bfloat16 weights once;
// each wave then takes (16-vertex block, chunk of `pc` frame pairs) items
// round-robin (nch chunks per block). The block's first-layer term A_i stays
// in registers over the chunk; per frame pair the two frames run as two
// 16-sample tiles that share every weight operand, and the 6-DoF transform
// of frame 2p runs on lanes 0-15 while that of frame 2p+1 runs on lanes
// 16-31.
template <int W, int H>
__global__ __launch_bounds__(512) void k_decode_fwd16(const uint16_t* __restrict__ wp16,
                                                      const float* __restrict__ wp, const float* __restrict__ A,
                                                      const float* __restrict__ B, const float4* __restrict__ xyz,
                                                      float4* __restrict__ xhat, int64_t V, int T, ActP ap,
                                                      float alpha, int quat, const float4* __restrict__ nrm,
                                                      float4* __restrict__ nhat, int pc, int nch) {
  constexpr int LD = WLds<W>::LD;
  extern __shared__ __attribute__((aligned(16))) float lds[];
  uint16_t* sW = reinterpret_cast<uint16_t*>(lds);                      // [(H-1)W + 16][LD]
  float* sB = reinterpret_cast<float*>(sW + ((H - 1) * W + 16) * LD);   // [H-1][W] + [16]
  const WPack P(W, H);
  stage_w16<W, H>(wp16, sW);
  for (int e = threadIdx.x; e < (H - 1) * W; e += blockDim.x) sB[e] = wp[P.bh + e];
  for (int e = threadIdx.x; e < 16; e += blockDim.x) sB[(H - 1) * W + e] = wp[P.bo + e];
  __syncthreads();
  const int nw = blockDim.x >> 6;
  const int64_t it0 = (int64_t)blockIdx.x * nw + (threadIdx.x >> 6), stride = (int64_t)gridDim.x * nw;
  if (ap.relu)
    fwd16_items<W, H, true>(sW, sB, A, B, xyz, xhat, V, T, 0.f, alpha, quat, nrm, nhat, pc, nch, it0, stride);
  else
    fwd16_items<W, H, false>(sW, sB, A, B, xyz, xhat, V, T, ap.slope, alpha, quat, nrm, nhat, pc, nch, it0,
                             stride);
}

// Backward, BF16 form. A persistent work-group of 4 waves (one per SIMD, so
// each wave has the whole register file) takes work items (block of 64
// vertices, chunk of consecutive frames) in a fixed round-robin order. Per
// frame every wave recomputes the forward pass of its 16 vertices,
// back-propagates in registers, and stages each layer's bfloat16 (gradient,
// input) of the 64 samples in LDS as [sample][feature] rows (one 8-byte store
// per tile), from which every wave accumulates a fixed quarter of the
// weight-gradient tiles (K = samples, operands by the LDS transpose read) in
// registers over all its items. Bias gradients use the float32 gradients (per-wave row sums
// in LDS), as do the first-layer sums: per vertex over the chunk's frames
// (Gv, one slice per chunk) and per frame over the block's vertices
// (Gt_part). Every partial is reduced later in a fixed order. The
// first-layer terms of the item (A_i of its vertices, B_t of its frames) are
// staged in LDS at the start of the item; the next frame's gradient rows are
// read one frame ahead.
constexpr int kB16W = 4;            // waves per work-group
constexpr int kB16S = 16 * kB16W;   // vertices (samples) per frame round
template <int W>
constexpr int b16_ls() { return W + 16; }  // staged [sample][feature] row stride (bfloat16)
constexpr int kB16TC = 16;          // most frames per work item

template <int W, int H>
constexpr size_t bwd16_lds_bytes() {
  return sizeof(uint16_t) * ((size_t)((H - 1) * W + 16) * WLds<W>::LD + 2 * (size_t)kB16S * b16_ls<W>()) +
         sizeof(float) * ((size_t)kB16W * ((H - 1) * W + 16) + (size_t)kB16W * W + (size_t)kB16S * (W + 4) +
                          (size_t)kB16TC * W);
}

template <int W, int H>
__global__ __launch_bounds__(64 * kB16W) void k_decode_bwd16(
    const uint16_t* __restrict__ wp16, const float* __restrict__ wp, const float* __restrict__ A,
    const float* __restrict__ B, const float4* __restrict__ xyz, const float4* __restrict__ gxhat, int64_t V, int T,
    ActP ap, float alpha, int quat, int nvb, int nch, float* __restrict__ Gv, float* __restrict__ Gt_part,
    float* __restrict__ gW_part) {
  constexpr int NT = W / 16;
  constexpr int LD = WLds<W>::LD;
  constexpr int LA = W + 4;                            // A-row stride in LDS (floats)
  constexpr int NTT = (NT * NT + kB16W - 1) / kB16W;   // owned hidden weight-gradient tiles per wave
  constexpr int NTO = (NT + kB16W - 1) / kB16W;        // owned output weight-gradient tiles per wave
  constexpr int NB = (H - 1) * W + 16;                 // bias-gradient entries (hidden, then output rows)
  extern __shared__ __attribute__((aligned(16))) float lds[];
  uint16_t* sW = reinterpret_cast<uint16_t*>(lds);                 // [NB][LD] weights
  constexpr int LS = b16_ls<W>();
  uint16_t* sG = sW + NB * LD;                                     // [kB16S][LS] staged gradients
  uint16_t* sH = sG + kB16S * LS;                                  // [kB16S][LS] staged layer inputs
  float* sGb = reinterpret_cast<float*>(sH + kB16S * LS);          // [kB16W][NB]
  float* sGt = sGb + kB16W * NB;                                   // [kB16W][W]
  float* sA = sGt + kB16W * W;                                     // [kB16S][LA] the item's A rows
  float* sBt = sA + kB16S * LA;                                    // [kB16TC][W] the item's B rows
  const WPack P(W, H);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, c = lane & 15;
  const int sp = wave * 16 + c;

  stage_w16<W, H>(wp16, sW);
  for (int e = threadIdx.x; e < kB16W * NB; e += blockDim.x) sGb[e] = 0.f;
  float4 bo4 = *reinterpret_cast<const float4*>(wp + P.bo + 4 * q);
  const v4f boi = v4f{bo4.x, bo4.y, bo4.z, bo4.w};
  v4f accW[H > 1 ? H - 1 : 1][NTT];
  v4f accO[NTO];
#pragma unroll
  for (int l = 0; l < (H > 1 ? H - 1 : 1); ++l)
#pragma unroll
    for (int k = 0; k < NTT; ++k) accW[l][k] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < NTO; ++k) accO[k] = v4f{0.f, 0.f, 0.f, 0.f};
  __syncthreads();

  // this lane's 4 features 16mt + 4q .. +3 of its sample, one 8-byte store
  auto stage = [&](uint16_t* buf, int mt, v4s v) { *reinterpret_cast<v4s*>(buf + sp * LS + 16 * mt + 4 * q) = v; };
  // operand of K block ks (samples 32ks ..): row tile t of buf, slot 4h + k of
  // lane (q, c) = feature 16t + c of sample 32ks + 16h + 4q + k
  auto kop = [&](const uint16_t* buf, int t, int ks) {
    const uint16_t* p = buf + (32 * ks + 4 * q + (c >> 2)) * LS + 16 * t + 4 * (c & 3);
    return cat8(lds_tr(p), lds_tr(p + 16 * LS));
  };

  const int64_t n_items = (int64_t)nvb * nch;
  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int vb = (int)(item % nvb), ch = (int)(item / nvb);
    const int t0 = (int)((int64_t)T * ch / nch), t1 = (int)((int64_t)T * (ch + 1) / nch);
    const int64_t i_raw = (int64_t)vb * kB16S + sp;
    const bool vvalid = i_raw < V;
    const int64_t i = vvalid ? i_raw : V - 1;
    const float4 xi = xyz[i];
    {  // the item's first-layer rows (the previous item's readers have passed a barrier)
      const int64_t v0 = (int64_t)vb * kB16S;
      for (int e = threadIdx.x; e < kB16S * W / 4; e += blockDim.x) {
        const int64_t v = std::min<int64_t>(v0 + (4 * e) / W, V - 1);
        *reinterpret_cast<float4*>(sA + ((4 * e) / W) * LA + (4 * e) % W) =
            *reinterpret_cast<const float4*>(A + v * W + (4 * e) % W);
      }
      for (int e = threadIdx.x; e < (t1 - t0) * W / 4; e += blockDim.x)
        reinterpret_cast<float4*>(sBt)[e] = *reinterpret_cast<const float4*>(B + (int64_t)t0 * W + 4 * e);
    }
    __syncthreads();
    float4 gxn = vvalid ? gxhat[(int64_t)t0 * V + i] : make_float4(0.f, 0.f, 0.f, 0.f);
    v4f gv[NT];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) gv[mt] = v4f{0.f, 0.f, 0.f, 0.f};

    // first hidden layer's output of this lane's sample at frame t (from LDS)
    auto first_layer = [&](int t, v4s (&h0)[NT]) {
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) {
        const float4 a = *reinterpret_cast<const float4*>(sA + sp * LA + 16 * mt + 4 * q);
        const float4 b = *reinterpret_cast<const float4*>(sBt + (t - t0) * W + 16 * mt + 4 * q);
        h0[mt] = pack_bf16(v4f{actf(a.x + b.x, ap), actf(a.y + b.y, ap), actf(a.z + b.z, ap), actf(a.w + b.w, ap)});
      }
    };

    for (int t = t0; t < t1; ++t) {
      // ---- forward pass, recomputed; bfloat16 inputs of the layers kept
      // (the first one is read again from LDS when it is needed) -----------
      v4s h[H][NT];
      first_layer(t, h[0]);
      const float4 gx = gxn;
      if (t + 1 < t1 && vvalid) gxn = gxhat[(int64_t)(t + 1) * V + i];  // next frame's row
#pragma unroll
      for (int l = 1; l < H; ++l) {
        v4f o[NT];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
          float4 b = *reinterpret_cast<const float4*>(wp + P.bh + (l - 1) * W + 16 * mt + 4 * q);
          o[mt] = v4f{b.x, b.y, b.z, b.w};
        }
        dense32<W, false>(h[l - 1], o, sW + (l - 1) * W * LD, q, c);
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
          h[l][mt] = pack_bf16(v4f{actf(o[mt][0], ap), actf(o[mt][1], ap), actf(o[mt][2], ap), actf(o[mt][3], ap)});
      }
      const v4f o = dense_out32<W>(h[H - 1], boi, sW + (H - 1) * W * LD, q, c);

      // ---- transform backward (float32) -----------------------------------
      float o4 = __shfl(o[0], (lane + 16) & 63);
      float o5 = __shfl(o[1], (lane + 16) & 63);
      float o6 = __shfl(o[2], (lane + 16) & 63);
      float ov[7] = {__shfl(o[0], c), __shfl(o[1], c), __shfl(o[2], c), __shfl(o[3], c), __shfl(o4, c),
                     __shfl(o5, c), __shfl(o6, c)};
      float go[7];
      go[6] = 0.f;
      if (quat) quat_grad(ov, xi, gx, alpha, go);
      else transform_grad(ov, xi, gx, alpha, go);
      if (!vvalid)
        for (int k = 0; k < 7; ++k) go[k] = 0.f;
      const v4f got = q == 0 ? v4f{go[0], go[1], go[2], go[3]}
                             : (q == 1 ? v4f{go[4], go[5], go[6], 0.f} : v4f{0.f, 0.f, 0.f, 0.f});
      const v4s gotb = pack_bf16(got);

      // ---- output layer ---------------------------------------------------
      stage(sG, 0, gotb);
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) stage(sH, mt, h[H - 1][mt]);
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < kB16S / 32; ++ks) {
        const v8s a = kop(sG, 0, ks);
#pragma unroll
        for (int k = 0; k < NTO; ++k) {
          const int kt = wave + kB16W * k;
          if (kt < NT) accO[k] = mfma32(a, kop(sH, kt, ks), accO[k]);
        }
      }
      {
        const v4f v = row16_sum4(got);
        if (c == 0) {
          float4* p = reinterpret_cast<float4*>(sGb + wave * NB + (H - 1) * W + 4 * q);
          const float4 u = *p;
          *p = make_float4(u.x + v[0], u.y + v[1], u.z + v[2], u.w + v[3]);
        }
      }
      v4f gp[NT];
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) {
        const v4f a = mfma16(wtr<W>(sW + (H - 1) * W * LD, 4 * q + (c >> 2), mt, c), gotb, v4f{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int r = 0; r < 4; ++r) gp[mt][r] = actd_mul(a[r], h[H - 1][mt][r], ap.slope);
      }
      __syncthreads();

      // ---- hidden layers, last to first ----------------------------------
#pragma unroll
      for (int l = H - 1; l >= 1; --l) {
        if (l == 1 && H > 2) first_layer(t, h[0]);
        v4s gb[NT];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
          gb[mt] = pack_bf16(gp[mt]);
          stage(sG, mt, gb[mt]);
          stage(sH, mt, h[l - 1][mt]);
        }
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
          const v4f v = row16_sum4(gp[mt]);
          if (c == 0) {
            float4* p = reinterpret_cast<float4*>(sGb + wave * NB + (l - 1) * W + 16 * mt + 4 * q);
            const float4 u = *p;
            *p = make_float4(u.x + v[0], u.y + v[1], u.z + v[2], u.w + v[3]);
          }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kB16S / 32; ++ks) {
          // owned tile k is (row tile (wave + 4k) / NT, column tile (wave + 4k) % NT):
          // every row tile's gradient operand and the wave's NKT column tiles'
          // input operands are read once per K block and reused across tiles
          constexpr int NKT = NT >= 8 ? 2 : 1;
          v8s gk[NT], hk[NKT];
#pragma unroll
          for (int mt = 0; mt < NT; ++mt) gk[mt] = kop(sG, mt, ks);
#pragma unroll
          for (int j = 0; j < NKT; ++j) hk[j] = kop(sH, (wave + kB16W * j) % NT, ks);
#pragma unroll
          for (int k = 0; k < NTT; ++k) {
            const unsigned tau = (unsigned)wave + kB16W * k;
            if (tau < (unsigned)(NT * NT)) {
              // row tile: k / 2 for NT = 8, k for NT = 4, wave / 2 for NT = 2
              const v8s g = NT == 2 ? ((wave >> 1) ? gk[NT - 1] : gk[0]) : gk[(kB16W * k) / NT];
              accW[l - 1][k] = mfma32(g, hk[k % NKT], accW[l - 1][k]);
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        v4f gh[NT];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) gh[mt] = v4f{0.f, 0.f, 0.f, 0.f};
        dgrad32<W>(gb, gh, sW + (l - 1) * W * LD, q, c);
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) gp[mt][r] = actd_mul(gh[mt][r], h[l - 1][mt][r], ap.slope);
        if (l > 1) __syncthreads();
      }

      // ---- first layer: per-vertex and per-frame sums ---------------------
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) {
        gv[mt] += gp[mt];
        const v4f v = row16_sum4(gp[mt]);
        if (c == 0) *reinterpret_cast<float4*>(sGt + wave * W + 16 * mt + 4 * q) = make_float4(v[0], v[1], v[2], v[3]);
      }
      __syncthreads();
      for (int f = threadIdx.x; f < W; f += blockDim.x) {
        float s0 = 0.f;
#pragma unroll
        for (int w = 0; w < kB16W; ++w) s0 += sGt[w * W + f];
        Gt_part[((int64_t)t * nvb + vb) * W + f] = s0;
      }
    }
    if (vvalid) {
      float* dst = Gv + ((int64_t)ch * V + i_raw) * W;
#pragma unroll
      for (int mt = 0; mt < NT; ++mt)
        *reinterpret_cast<float4*>(dst + 16 * mt + 4 * q) = make_float4(gv[mt][0], gv[mt][1], gv[mt][2], gv[mt][3]);
    }
  }
  __syncthreads();

  // ---- this work-group's weight-gradient partial --------------------------
  const int n_out = quat ? 7 : 6;
  const int64_t len = (int64_t)(H - 1) * ((int64_t)W * W + W) + n_out * (int64_t)W + n_out;
  float* dst = gW_part + (int64_t)blockIdx.x * len;
#pragma unroll
  for (int l = 1; l < H; ++l) {
    float* dl = dst + (int64_t)(l - 1) * ((int64_t)W * W + W);
#pragma unroll
    for (int k = 0; k < NTT; ++k) {
      const unsigned tau = (unsigned)wave + kB16W * k;
      if (tau < (unsigned)(NT * NT)) {
        const int mt = tau / NT, kt = tau % NT;
#pragma unroll
        for (int r = 0; r < 4; ++r) dl[(16 * mt + 4 * q + r) * W + 16 * kt + c] = accW[l - 1][k][r];
      }
    }
    for (int e = threadIdx.x; e < W; e += blockDim.x) {
      float s0 = 0.f;
      for (int w = 0; w < kB16W; ++w) s0 += sGb[w * NB + (l - 1) * W + e];
      dl[(int64_t)W * W + e] = s0;
    }
  }
  float* dout = dst + (int64_t)(H - 1) * ((int64_t)W * W + W);
#pragma unroll
  for (int k = 0; k < NTO; ++k) {
    const int kt = wave + kB16W * k;
    if (kt < NT) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (4 * q + r < n_out) dout[(4 * q + r) * W + 16 * kt + c] = accO[k][r];
    }
  }
  if ((int)threadIdx.x < n_out) {
    float s0 = 0.f;
    for (int w = 0; w < kB16W; ++w) s0 += sGb[w * NB + (H - 1) * W + threadIdx.x];
    dout[n_out * W + threadIdx.x] = s0;
  }
}

// Gv[i][o] = sum over chunks of Gv_part[chunk][i][o]
__global__ void k_gv_reduce(const float* __restrict__ part, int64_t n, int nch, float* __restrict__ Gv) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  float s = 0.f;
  for (int k = 0; k < nch; ++k) s += part[(int64_t)k * n + e];
  Gv[e] = s;
}

// Fixed-order sums of partials: in a block of kRG x kRE threads, thread
// (g, e) adds the parts p = g, g + kRG, ... of entry e in order, then the kRG
// group sums are added in g order. Reads are coalesced over e.
constexpr int kRG = 16;
constexpr int kRE = 64;

// dst[e] = sum over p of part[p * len + e]
__global__ __launch_bounds__(kRG * kRE) void k_sum_parts(const float* __restrict__ part, int64_t len, int nparts,
                                                         float* __restrict__ dst) {
  __shared__ float red[kRG][kRE + 1];
  const int el = threadIdx.x % kRE, g = threadIdx.x / kRE;
  const int64_t e = blockIdx.x * (int64_t)kRE + el;
  float s0 = 0.f;
  if (e < len)
    for (int p = g; p < nparts; p += kRG) s0 += part[(int64_t)p * len + e];
  red[g][el] = s0;
  __syncthreads();
  if (g == 0 && e < len) {
    float t = 0.f;
    for (int k = 0; k < kRG; ++k) t += red[k][el];
    dst[e] = t;
  }
}

// Gt[t][o] = sum over work-groups p of Gt_part[t][p][o]
__global__ __launch_bounds__(kRG * kRE) void k_gt_reduce(const float* __restrict__ part, int T, int nwg, int W,
                                                         float* __restrict__ Gt) {
  __shared__ float red[kRG][kRE + 1];
  const int el = threadIdx.x % kRE, g = threadIdx.x / kRE;
  const int64_t e = blockIdx.x * (int64_t)kRE + el;
  const bool ok = e < (int64_t)T * W;
  float s0 = 0.f;
  if (ok) {
    const int64_t t = e / W, o = e % W;
    for (int p = g; p < nwg; p += kRG) s0 += part[(t * nwg + p) * W + o];
  }
  red[g][el] = s0;
  __syncthreads();
  if (g == 0 && ok) {
    float t = 0.f;
    for (int k = 0; k < kRG; ++k) t += red[k][el];
    Gt[e] = t;
  }
}

// First layer, z part, stage 1: per block of kFLV vertices and per output
// unit o, sum_i Gv[i][o] z_i[k] (k < Fz), in fixed order (vertex sub-streams
// of the block, then their sums in order). part [block][W][8]; the block
// count is npg_first_layer_blocks(V).
constexpr int kFLV = 64;
__global__ __launch_bounds__(256) void k_first_layer_z(const float* __restrict__ Gv, const float* __restrict__ z,
                                                       int64_t V, int W, int Fz, int bf16,
                                                       float* __restrict__ part) {
  __shared__ float red[256][9];
  const int o = threadIdx.x % W, sub = threadIdx.x / W, nsub = 256 / W;
  const int64_t i0 = (int64_t)blockIdx.x * kFLV;
  const int64_t i1 = i0 + kFLV < V ? i0 + kFLV : V;
  float acc[8];
  for (int k = 0; k < 8; ++k) acc[k] = 0.f;
  for (int64_t i = i0 + sub; i < i1; i += nsub) {
    const float gv = Gv[i * W + o];
    for (int k = 0; k < Fz; ++k) acc[k] = fmaf(gv, rnd(z[i * Fz + k], bf16), acc[k]);
  }
  for (int k = 0; k < 8; ++k) red[threadIdx.x][k] = acc[k];
  __syncthreads();
  if (sub == 0) {
    for (int k = 0; k < Fz; ++k) {
      float t = 0.f;
      for (int u = 0; u < nsub; ++u) t += red[u * W + o][k];
      part[((int64_t)blockIdx.x * W + o) * 8 + k] = t;
    }
  }
}

// First layer, stage 2 (one block per output unit o): gW1 z part = sum over
// blocks of the stage-1 partials; gamma part = sum_t Gt[t][o] gamma_t;
// gb1[o] = sum_t Gt[t][o]. Fixed-order tree reductions.
__global__ __launch_bounds__(256) void k_first_layer(const float* __restrict__ part, int nb,
                                                     const float* __restrict__ Gt, const float* __restrict__ gam,
                                                     int T, int W, int Din, int Fz, int bf16,
                                                     float* __restrict__ g1) {
  constexpr int kN = 8 + 16 + 1;  // z part, gamma part, bias
  __shared__ float red[256][kN];
  const int o = blockIdx.x;
  const int Dt = Din - Fz;
  float acc[kN];
  for (int k = 0; k < kN; ++k) acc[k] = 0.f;
  for (int b = threadIdx.x; b < nb; b += 256)
    for (int k = 0; k < Fz; ++k) acc[k] += part[((int64_t)b * W + o) * 8 + k];
  for (int t = threadIdx.x; t < T; t += 256) {
    const float v = Gt[(int64_t)t * W + o];
    acc[8 + 16] += v;
    for (int k = 0; k < Dt; ++k) acc[8 + k] = fmaf(v, rnd(gam[(int64_t)t * Dt + k], bf16), acc[8 + k]);
  }
  for (int k = 0; k < kN; ++k) red[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < kN; ++k) red[threadIdx.x][k] += red[threadIdx.x + st][k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < Fz; ++k) g1[(int64_t)o * Din + k] = red[0][k];
    for (int k = 0; k < Dt; ++k) g1[(int64_t)o * Din + Fz + k] = red[0][8 + k];
    g1[(int64_t)W * Din + o] = red[0][8 + 16];
  }
}

// gz[i][k] = sum_o W1[o][k] Gv[i][o], k < Fz: one wave per vertex, lanes over
// o, then a fixed butterfly over the wave
__global__ __launch_bounds__(256) void k_gz(const float* __restrict__ mlp, const float* __restrict__ Gv, int64_t V,
                                            int W, int Din, int Fz, int bf16, float* __restrict__ gz) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= V) return;  // uniform over the wave; no barriers below
  float acc[8];
  for (int k = 0; k < 8; ++k) acc[k] = 0.f;
  for (int o = lane; o < W; o += 64) {
    const float gv = Gv[i * W + o];
    for (int k = 0; k < Fz; ++k) acc[k] = fmaf(rnd(mlp[(int64_t)o * Din + k], bf16), gv, acc[k]);
  }
  for (int k = 0; k < 8; ++k)
    for (int m = 32; m > 0; m >>= 1) acc[k] += __shfl_xor(acc[k], m);
  if (lane == 0)
    for (int k = 0; k < Fz; ++k) gz[i * Fz + k] = acc[k];
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <int W, int H>
size_t fwd_lds() {
  return sizeof(float) * ((size_t)(H - 1) * W * (W + 4) + 16 * (W + 4) + (H - 1) * W + 16);
}
template <int W, int H>
size_t bwd_lds() {
  return sizeof(float) * bwd_lds_floats<W, H>();
}

template <int W, int H, bool STORE>
hipError_t launch_fwd_k(const npg_plan* P, float4* xhat, ActP ap, float4* nhat, float* act) {
  size_t lds = fwd_lds<W, H>();
  hipError_t e = hipFuncSetAttribute((const void*)k_decode_fwd<W, H, STORE>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_decode_fwd<W, H, STORE>), dim3(P->n_cu), dim3(512), lds, P->stream, P->wpack, P->mlpA,
                     P->mlpB, P->xyz, xhat, P->V, P->T, ap, P->cfg.alpha_t, (int)(P->n_out == 7), P->nrm,
                     nhat, act);
  return hipGetLastError();
}
template <int W, int H>
hipError_t launch_fwd(const npg_plan* P, float4* xhat, ActP ap, float4* nhat, float* act) {
  if (H > 1 && act) return launch_fwd_k<W, H, (H > 1)>(P, xhat, ap, nhat, act);
  return launch_fwd_k<W, H, false>(P, xhat, ap, nhat, nullptr);
}

template <int W, int H, bool STORED>
hipError_t launch_bwd_k(const npg_plan* P, const float4* gxhat, ActP ap, const float* act) {
  size_t lds = bwd_lds<W, H>();
  hipError_t e = hipFuncSetAttribute((const void*)k_decode_bwd<W, H, STORED>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_decode_bwd<W, H, STORED>), dim3(P->mlp_grid), dim3(256), lds, P->stream, P->wpack,
                     P->mlpA, P->mlpB, P->xyz, gxhat, P->V, P->T, ap, P->cfg.alpha_t, (int)(P->n_out == 7),
                     P->n_vblk_mlp, P->mlp_nch, P->mlp_nch > 1 ? P->Gv_part : P->Gv, P->Gt_part, P->gW_part, act);
  return hipGetLastError();
}
template <int W, int H>
hipError_t launch_bwd(const npg_plan* P, const float4* gxhat, ActP ap, const float* act) {
  if (H > 1 && act) return launch_bwd_k<W, H, (H > 1)>(P, gxhat, ap, act);
  return launch_bwd_k<W, H, false>(P, gxhat, ap, nullptr);
}

inline int is_bf16(const npg_plan* P) { return P->cfg.precision == NPG_PREC_BF16; }

hipError_t prep(const npg_plan* P, const float* params, const float* z) {
  const float* mlp = params + P->mlp_off;
  const WPack wpk(P->W, P->H);
  const int bf = is_bf16(P);
  hipLaunchKernelGGL(k_prep_weights, dim3(nblk(wpk.total, 256)), dim3(256), 0, P->stream, mlp, P->W, P->H,
                     P->Din, P->n_out, P->wpack);
  if (bf)
    hipLaunchKernelGGL(k_pack_bf16, dim3(nblk(wpk.total, 256)), dim3(256), 0, P->stream, P->wpack, wpk.total,
                       P->wpack16);
  hipLaunchKernelGGL(k_prep_A, dim3(nblk(P->V * P->W, 256)), dim3(256), 0, P->stream, mlp, z, P->V, P->W,
                     P->Din, P->Fz, bf, P->mlpA);
  hipLaunchKernelGGL(k_prep_B, dim3(nblk((int64_t)P->T * P->W, 256)), dim3(256), 0, P->stream, mlp, P->gam,
                     P->T, P->W, P->Din, P->Fz, bf, P->mlpB);
  return hipGetLastError();
}

template <int W, int H>
size_t fwd16_lds() {
  return sizeof(uint16_t) * ((size_t)((H - 1) * W + 16) * WLds<W>::LD) + sizeof(float) * ((size_t)(H - 1) * W + 16);
}

// Forward items: 16-vertex blocks times chunks of pc frame pairs, dealt to
// nw waves; pc minimizes the largest per-wave pair count (the longest chunk
// on a tie, so A_i is loaded least often).
void fwd16_schedule(int64_t V, int T, int64_t nw, int* pc, int* nch) {
  const int64_t nvb = (V + 15) / 16;
  const int np = (T + 1) / 2;
  int64_t best = -1;
  for (int c = 1; c <= np; ++c) {
    const int n = (np + c - 1) / c;
    const int64_t load = (nvb * n + nw - 1) / nw * c;
    if (best < 0 || load <= best) {
      best = load;
      *pc = c;
      *nch = n;
    }
  }
}

template <int W, int H>
hipError_t launch_fwd16(const npg_plan* P, float4* xhat, ActP ap, float4* nhat) {
  size_t lds = fwd16_lds<W, H>();
  hipError_t e = hipFuncSetAttribute((const void*)k_decode_fwd16<W, H>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int pc = 1, nch = 1;
  fwd16_schedule(P->V, P->T, (int64_t)P->n_cu * 8, &pc, &nch);
  hipLaunchKernelGGL((k_decode_fwd16<W, H>), dim3(P->n_cu), dim3(512), lds, P->stream, P->wpack16, P->wpack,
                     P->mlpA, P->mlpB, P->xyz, xhat, P->V, P->T, ap, P->cfg.alpha_t, (int)(P->n_out == 7), P->nrm,
                     nhat, pc, nch);
  return hipGetLastError();
}

template <int W, int H>
hipError_t launch_bwd16(const npg_plan* P, const float4* gxhat, ActP ap) {
  size_t lds = bwd16_lds_bytes<W, H>();
  hipError_t e = hipFuncSetAttribute((const void*)k_decode_bwd16<W, H>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_decode_bwd16<W, H>), dim3(P->mlp_grid), dim3(64 * kB16W), lds, P->stream, P->wpack16,
                     P->wpack, P->mlpA, P->mlpB, P->xyz, gxhat, P->V, P->T, ap, P->cfg.alpha_t,
                     (int)(P->n_out == 7), P->n_vblk_mlp, P->mlp_nch, P->mlp_nch > 1 ? P->Gv_part : P->Gv,
                     P->Gt_part, P->gW_part);
  return hipGetLastError();
}

#define NPG_DISPATCH(FN, ...)                                        \
  switch (P->W * 10 + P->H) {                                        \
    case 321: return FN<32, 1>(__VA_ARGS__);                         \
    case 322: return FN<32, 2>(__VA_ARGS__);                         \
    case 323: return FN<32, 3>(__VA_ARGS__);                         \
    case 641: return FN<64, 1>(__VA_ARGS__);                         \
    case 642: return FN<64, 2>(__VA_ARGS__);                         \
    case 643: return FN<64, 3>(__VA_ARGS__);                         \
    case 1281: return FN<128, 1>(__VA_ARGS__);                       \
    case 1282: return FN<128, 2>(__VA_ARGS__);                       \
    case 1283: return FN<128, 3>(__VA_ARGS__);                       \
    default: return hipErrorInvalidValue;                            \
  }

}  // namespace

int64_t npg_wpack_len(int W, int H) { return WPack(W, H).total; }
int64_t npg_gw_part_len(int W, int H, int n_out) {
  return (int64_t)(H - 1) * ((int64_t)W * W + W) + n_out * (int64_t)W + n_out;
}

// Work items of the MLP backward (both precisions): blocks of 64 vertices
// times nch frame chunks (balanced split of the T frames, at most tc_max
// frames each when tc_max > 0), dealt round-robin to grid = min(items, n_cu)
// persistent work-groups. nch minimizes the largest per-group frame count
// (fewest chunks on a tie).
void npg_mlp_schedule(int64_t V, int T, int n_cu, int tc_max, int* nvb, int* nch, int* grid) {
  const int nb = (int)((V + 63) / 64);
  const int n_min = tc_max > 0 ? (T + tc_max - 1) / tc_max : 1;
  int best_n = n_min;
  int64_t best = -1;
  for (int n = n_min; n <= std::min(T, n_min + 63); ++n) {
    const int64_t items = (int64_t)nb * n;
    const int G = (int)std::min<int64_t>(items, n_cu);
    std::vector<int64_t> load(G, 0);
    for (int64_t it = 0; it < items; ++it) {
      const int ch = (int)(it / nb);
      load[it % G] += (int64_t)T * (ch + 1) / n - (int64_t)T * ch / n;
    }
    const int64_t mk = *std::max_element(load.begin(), load.end());
    if (best < 0 || mk < best) {
      best = mk;
      best_n = n;
    }
  }
  *nvb = nb;
  *nch = best_n;
  *grid = (int)std::min<int64_t>((int64_t)nb * best_n, n_cu);
}
int npg_mlp_bf16_frames() { return kB16TC; }
int64_t npg_first_layer_blocks(int64_t V) { return (V + kFLV - 1) / kFLV; }

hipError_t npg_launch_decode_fwd(const npg_plan* P, const float* params, const float* z, float4* xhat,
                                 float4* nhat, float* act) {
  hipError_t e = prep(P, params, z);
  if (e != hipSuccess) return e;
  const bool relu = P->cfg.act == NPG_ACT_RELU;
  ActP ap{relu, relu ? 0.f : P->cfg.leaky_slope};
  if (is_bf16(P)) {
    NPG_DISPATCH(launch_fwd16, P, xhat, ap, nhat);
  }
  NPG_DISPATCH(launch_fwd, P, xhat, ap, nhat, act);
}

static hipError_t decode_bwd_tail(const npg_plan* P, const float* params, const float* z, float* grad, float* gz) {
  const float* mlp = params + P->mlp_off;
  float* gmlp = grad + P->mlp_off;
  const int64_t l0 = (int64_t)P->W * P->Din + P->W;
  const bool bf = is_bf16(P);
  const int64_t TW = (int64_t)P->T * P->W;
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk(P->gw_part_len, kRE)), dim3(kRG * kRE), 0, P->stream, P->gW_part,
                     P->gw_part_len, P->mlp_grid, gmlp + l0);
  hipLaunchKernelGGL(k_gt_reduce, dim3(nblk(TW, kRE)), dim3(kRG * kRE), 0, P->stream, P->Gt_part, P->T,
                     P->n_vblk_mlp, P->W, P->Gt);
  if (P->mlp_nch > 1)
    hipLaunchKernelGGL(k_gv_reduce, dim3(nblk(P->V * P->W, 256)), dim3(256), 0, P->stream, P->Gv_part,
                       P->V * P->W, P->mlp_nch, P->Gv);
  const int nb = (int)nblk(P->V, kFLV);
  hipLaunchKernelGGL(k_first_layer_z, dim3(nb), dim3(256), 0, P->stream, P->Gv, z, P->V, P->W, P->Fz, (int)bf,
                     P->fl_part);
  hipLaunchKernelGGL(k_first_layer, dim3(P->W), dim3(256), 0, P->stream, P->fl_part, nb, P->Gt, P->gam, P->T,
                     P->W, P->Din, P->Fz, (int)bf, gmlp);
  hipLaunchKernelGGL(k_gz, dim3(nblk(P->V, 4)), dim3(256), 0, P->stream, mlp, P->Gv, P->V, P->W, P->Din, P->Fz,
                     (int)bf, gz);
  return hipGetLastError();
}

hipError_t npg_launch_decode_bwd(const npg_plan* P, const float* params, const float* z, const float4* gxhat,
                                 float* grad, float* gz, const float* act) {
  hipError_t e = prep(P, params, z);
  if (e != hipSuccess) return e;
  const bool relu = P->cfg.act == NPG_ACT_RELU;
  ActP ap{relu, relu ? 0.f : P->cfg.leaky_slope};
  e = is_bf16(P) ? [&]() -> hipError_t { NPG_DISPATCH(launch_bwd16, P, gxhat, ap); }()
                 : [&]() -> hipError_t { NPG_DISPATCH(launch_bwd, P, gxhat, ap, act); }();
  if (e != hipSuccess) return e;
  return decode_bwd_tail(P, params, z, grad, gz);
}
