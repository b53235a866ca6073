// Learned per-sample weights for the sample-set filter (gfx950, wave64).
//
// The weighted mean of Sec. 5 Eq. 3 takes its weights from a small MLP on eight
// per-sample features, normalised over each set with a softmax (the learned
// replacement of the hand-set Gaussian of Sec. 5 Eq. 4):
//   O(p) = sum_s softmax(m)_s c_s,  m_s = MLP(standardised features of s).
//
// Inference (k_filter_learned): a wave owns 16 consecutive output pixels and
// streams their records (contiguous in the CSR arena) 64 at a time through the MLP
// on the matrix cores (v_mfma_f32_32x32x16_bf16: bfloat16 weights, operands as
// bfloat16 hi/lo pairs, float32 accumulate). The layers are evaluated transposed,
// H^T = W^T X^T (rows = hidden units, columns = samples): then the accumulator
// layout of layer 1 is exactly the B-operand layout of layer 2 (per lane: four
// consecutive hidden units of one sample), so the hidden activations never leave
// registers. The set softmax is a segmented reduction across the wave's lanes.
//
// Training (k_mlp_train_grad): one wave per pixel of the minibatch, on the matrix
// cores as well: a forward pass over the set gives the softmax statistics and
// O(p); a second pass recomputes the forward pass, back-propagates
// dL/dm_s = a_s (c_s - O) . dL/dO through the MLP (dz1 = W2 dz2 on the matrix
// cores, again without moving data between lanes), and accumulates dW2 = H1^T DZ2
// over the records with the operands read transposed from LDS; the small
// gradients (W1, W3, biases) stay on the vector units. k_mlp_adam applies Adam to
// the float32 masters.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_device.h"
#include "sg_internal.h"

namespace sg {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kNF = 8, kNH = 64;
constexpr int kOffW2 = kNF * kNH;            // W2 inside the bfloat16 weight block
constexpr int kOffW3 = kOffW2 + kNH * kNH;   // W3
constexpr int kOffB3 = 2 * kNH, kOffMean = 2 * kNH + 4;  // inside the float32 block: b1, b2, b3, pad, mean, 1 / std

__device__ __forceinline__ uint32_t bf16_bits(float v) {  // round to nearest even
  const uint32_t u = __float_as_uint(v);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_to_f(uint32_t b) { return __uint_as_float((b & 0xFFFFu) << 16); }

// An operand of the matrix cores (a standardised feature, a layer-1 activation)
// enters as two bfloat16 values, hi = bf16(v) and lo = bf16(v - hi) (v - hi is
// exact in float32), so it carries about 16 significant bits; W v = W hi + W lo
// takes two products. The kernel is bound by its vector work (features, GELU),
// so the second product costs little, and no value is rounded to 8 bits.
struct SplitBf16 {
  uint32_t hi, lo;
};
__device__ __forceinline__ SplitBf16 split_bf16(float v) {
  SplitBf16 r;
  r.hi = bf16_bits(v);
  r.lo = bf16_bits(v - bf16_to_f(r.hi));
  return r;
}
__device__ __forceinline__ float split_value(float v) {
  const SplitBf16 r = split_bf16(v);
  return bf16_to_f(r.hi) + bf16_to_f(r.lo);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Two values to packed bfloat16 (round to nearest even, a in the low half): one
// v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
// hi/lo split of two values as packed pairs (same values as split_bf16)
__device__ __forceinline__ void split_pack(float a, float b, uint32_t& hi, uint32_t& lo) {
  hi = pack_bf16(a, b);
  lo = pack_bf16(a - __uint_as_float(hi << 16), b - __uint_as_float(hi & 0xFFFF0000u));
}
__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// GELU(z) = z Phi(z) = z/2 + (|z|/2) erf(|z| / sqrt 2), with erf from Abramowitz and
// Stegun 7.1.28 (|error| <= 3e-7 for x >= 0):
//   erf(x) = 1 - 1 / (1 + a1 x + a2 x^2 + ... + a6 x^6)^16.
// The kernels evaluate it at y = z/2 (the matrix products use W/2 and b/2, which
// are exact in bfloat16): x = sqrt(2) |y|, so the polynomial in |y| has
// coefficients a_k 2^(k/2) and constant term 1, and GELU = y + |y| erf. Six
// multiply-adds, four squarings, one reciprocal and one subtraction; for large
// |y| the 16th power overflows to +inf and erf = 1 exactly.
constexpr float kE1 = static_cast<float>(0.0705230784 * 1.4142135623730951);
constexpr float kE2 = static_cast<float>(0.0422820123 * 2.0);
constexpr float kE3 = static_cast<float>(0.0092705272 * 2.8284271247461903);
constexpr float kE4 = static_cast<float>(0.0001520143 * 4.0);
constexpr float kE5 = static_cast<float>(0.0002765672 * 5.6568542494923806);
constexpr float kE6 = static_cast<float>(0.0000430638 * 8.0);
constexpr float kInvSqrt2Pi = 0.3989422804014327f;
constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ float erf_of_half(float y) {  // erf(sqrt(2) |y|)
  const float a = fabsf(y);
  float q = fmaf(kE6, a, kE5);
  q = fmaf(q, a, kE4);
  q = fmaf(q, a, kE3);
  q = fmaf(q, a, kE2);
  q = fmaf(q, a, kE1);
  q = fmaf(q, a, 1.0f);
  q *= q;
  q *= q;
  q *= q;
  q *= q;
  return 1.0f - __builtin_amdgcn_rcpf(q);
}
// GELU(2y) from y = z/2
__device__ __forceinline__ float gelu_half(float y) { return fmaf(fabsf(y), erf_of_half(y), y); }

// Inference evaluates GELU(2y) = g(y) = y + |y| erf(sqrt(2) |y|) from a chord
// table: y in [-4, 4) is cut into kGeluCells cells of width h = 1/128, and on cell
// i the kernel takes the chord of g between the cell's ends, stored as (slope,
// intercept) so that g(y) ~ slope y + intercept. A chord is within
// h^2 max|g''| / 8 = 2.5e-5 of g (g''(y) = 4 phi(2y) (2 - 4y^2) <= 8 phi(0));
// beyond [-4, 4) the end cells extrapolate g = 2y above (erf(4 sqrt 2) rounds to 1
// in float32) and g ~ 0 below (|g| < 1e-14 at y = -4). Five vector instructions and
// one LDS read per activation, against nine and a reciprocal for a polynomial
// erf; training keeps 7.1.28, whose derivative it also needs.
constexpr int kGeluCells = 1024;
constexpr float kGeluPerUnit = 128.0f;  // cells per unit of y; cell 0 starts at y = -4
constexpr int kGeluCellsPerThread = 4;

// Fills the table (kGeluCells entries) from threads tid = 0 .. kGeluCells / 4 - 1,
// each taking four consecutive cells, with the shared ends evaluated once.
__device__ __forceinline__ void fill_gelu_table(float2* tab, int tid) {
  const int i0 = kGeluCellsPerThread * tid;
  float y0 = -4.0f + static_cast<float>(i0) / kGeluPerUnit;
  float g0 = fmaf(fabsf(y0), erff(1.4142135623730951f * fabsf(y0)), y0);
#pragma unroll
  for (int k = 0; k < kGeluCellsPerThread; ++k) {
    const float y1 = -4.0f + static_cast<float>(i0 + k + 1) / kGeluPerUnit;  // exact
    const float g1 = fmaf(fabsf(y1), erff(1.4142135623730951f * fabsf(y1)), y1);
    const float slope = (g1 - g0) * kGeluPerUnit;
    tab[i0 + k] = make_float2(slope, fmaf(-slope, y0, g0));
    y0 = y1;
    g0 = g1;
  }
}
__device__ __forceinline__ float gelu_half_table(const float2* tab, float y) {
  // cell index clamped to the table (a NaN y lands in some cell; the result stays NaN)
  const float t = __builtin_amdgcn_fmed3f(fmaf(y, kGeluPerUnit, 4.0f * kGeluPerUnit), 0.0f,
                                          static_cast<float>(kGeluCells - 1));
  const float2 e = tab[static_cast<uint32_t>(t)];
  return fmaf(e.x, y, e.y);
}
__device__ __forceinline__ float gelu(float z) { return gelu_half(0.5f * z); }
// GELU'(z) = Phi(z) + z phi(z)
__device__ __forceinline__ float gelu_grad(float z) {
  const float e = erf_of_half(0.5f * z);
  const float cdf = 0.5f + (z >= 0.0f ? 0.5f * e : -0.5f * e);
  const float pdf = kInvSqrt2Pi * __builtin_amdgcn_exp2f(-0.5f * kLog2e * z * z);
  return fmaf(z, pdf, cdf);
}
// bfloat16 bits of w / 2 (exact for every normal bfloat16)
__device__ __forceinline__ uint32_t bf16_half_bits(uint16_t b) {
  return __float_as_uint(__uint_as_float(static_cast<uint32_t>(b) << 16) * 0.5f) >> 16;
}

__device__ __forceinline__ void wave_lds_fence_l() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Per-pixel context and the eight features of one sample.

struct PixelCtx {
  float x, y, dp;
  int f;
  float medr, medg, medb;
  float x7;  // log(1 + n) / log(1 + (2r+1)^2 (2w+1))
};

struct FeatureArgs {
  gp<const float> rel;        // relative maps of this output frame, [2w+1][kRelStride]
  gp<const uint16_t> depth;   // stored depth planes
  int width, height, n_frames, pw, w;
  size_t dplane;  // binary16 entries per depth plane
  float inv_w, cx, cy;
  float inv_fx, inv_fy, inv_width;  // reciprocals, once per kernel (no division per sample)
};

__device__ __forceinline__ FeatureArgs feature_args(gp<const uint16_t> depth, int width, int height, int n_frames,
                                                    int w, float fx, float fy, float cx, float cy) {
  FeatureArgs fa;
  fa.rel = nullptr;
  fa.depth = depth;
  fa.width = width;
  fa.height = height;
  fa.n_frames = n_frames;
  fa.pw = stored_pitch(width);
  fa.w = w;
  fa.dplane = depth_plane_elems(width, height);
  fa.inv_w = w > 0 ? 1.0f / static_cast<float>(w) : 0.0f;
  fa.cx = cx;
  fa.cy = cy;
  fa.inv_fx = 1.0f / fx;
  fa.inv_fy = 1.0f / fy;
  fa.inv_width = 1.0f / static_cast<float>(width);
  return fa;
}

__device__ __forceinline__ bool valid_depth(float d) { return d > 0.0f && d < INFINITY; }

// A record id names frame slot id >> 22 of the window and source pixel id & (2^22 - 1);
// one that lies outside the clip (sets from another gather) is skipped, not read.
__device__ __forceinline__ bool id_in_clip(const FeatureArgs& a, int f, uint32_t id) {
  const int slot = static_cast<int>(id >> SG_ID_SHIFT);
  const int j = f + slot - a.w;
  const uint32_t q = id & ((1u << SG_ID_SHIFT) - 1u);
  return slot <= 2 * a.w && j >= 0 && j < a.n_frames &&
         q < static_cast<uint32_t>(a.width) * static_cast<uint32_t>(a.height);
}

__device__ __forceinline__ void sample_features(const FeatureArgs& a, const PixelCtx& px, uint32_t id,
                                                uint2 rec, float* feat) {
  const int slot = static_cast<int>(id >> SG_ID_SHIFT);
  const int dj = slot - a.w;
  const int j = px.f + dj;
  const int q = static_cast<int>(id & ((1u << SG_ID_SHIFT) - 1u));
  // row by the reciprocal of the width (off by at most one, corrected below)
  int qy = static_cast<int>(static_cast<float>(q) * a.inv_width);
  int qx = q - qy * a.width;
  if (qx < 0) { --qy; qx += a.width; }
  if (qx >= a.width) { ++qy; qx -= a.width; }
  gp<const float> m = a.rel + slot * kRelStride;
  const float a0 = fmaf(m[0], px.x, fmaf(m[1], px.y, m[2]));
  const float a1 = fmaf(m[3], px.x, fmaf(m[4], px.y, m[5]));
  const float a2 = fmaf(m[6], px.x, fmaf(m[7], px.y, m[8]));
  const float y0 = fmaf(px.dp, a0, m[9]), y1 = fmaf(px.dp, a1, m[10]), z = fmaf(px.dp, a2, m[11]);
  const float rz = __builtin_amdgcn_rcpf(z);
  const float u = y0 * rz, v = y1 * rz;
  // metric: X - o_f and X - o_J in frame-J axes (undo K on the folded map)
  const float ax = (px.dp * a0 - a.cx * px.dp * a2) * a.inv_fx;
  const float ay = (px.dp * a1 - a.cy * px.dp * a2) * a.inv_fy;
  const float az = px.dp * a2;
  const float tx = (m[9] - a.cx * m[11]) * a.inv_fx, ty = (m[10] - a.cy * m[11]) * a.inv_fy, tzv = m[11];
  const float bx = ax + tx, by = ay + ty, bz = az + tzv;
  // 1 - cos(angle) = |a/|a| - b/|b||^2 / 2: no cancellation for nearly parallel rays
  const float ra = rsqrtf(ax * ax + ay * ay + az * az), rb = rsqrtf(bx * bx + by * by + bz * bz);
  const float ux = ax * ra - bx * rb, uy = ay * ra - by * rb, uz = az * ra - bz * rb;
  const float one_minus_cos = 0.5f * (ux * ux + uy * uy + uz * uz);
  // depth gradient at q in J (apron neighbours read as invalid), from the paired
  // depth plane: the words of columns qx - 1 .. qx + 1 in q's pair row hold q's row
  // and one vertical neighbour; one word of the pair row above (q on the pair's
  // first row) or below (on its second) holds the other
  gp<const uint32_t> dw = reinterpret_cast<gp<const uint32_t>>(a.depth + static_cast<size_t>(j) * a.dplane);
  const uint32_t row = static_cast<uint32_t>(qy + SG_APRON);
  const uint32_t at = __umul24(row >> 1, static_cast<uint32_t>(a.pw)) + static_cast<uint32_t>(qx + SG_APRON);
  const uint32_t wl = dw[at - 1], wc = dw[at], wr = dw[at + 1];
  const bool second = (row & 1u) != 0u;
  const uint32_t wo = dw[second ? at + static_cast<uint32_t>(a.pw) : at - static_cast<uint32_t>(a.pw)];
  const uint32_t sh = second ? 16u : 0u;
  const float d0 = h2f(wc >> sh);
  const float dxp = h2f(wr >> sh), dxm = h2f(wl >> sh);
  const float dyp = h2f(second ? wo : wc >> 16), dym = h2f(second ? wc : wo >> 16);
  float gx = 0.0f, gy = 0.0f;
  const bool vxp = valid_depth(dxp), vxm = valid_depth(dxm), vyp = valid_depth(dyp), vym = valid_depth(dym);
  if (vxp && vxm) gx = 0.5f * (dxp - dxm); else if (vxp) gx = dxp - d0; else if (vxm) gx = d0 - dxm;
  if (vyp && vym) gy = 0.5f * (dyp - dym); else if (vyp) gy = dyp - d0; else if (vym) gy = d0 - dym;
  const float cr = h2f(rec.x), cg = h2f(rec.x >> 16), cb = h2f(rec.y);
  const float er = cr - px.medr, eg = cg - px.medg, eb = cb - px.medb;
  feat[0] = h2f(rec.y >> 16);
  feat[1] = sqrtf(er * er + eg * eg + eb * eb);
  feat[2] = fabsf(static_cast<float>(dj)) * a.inv_w;
  feat[3] = sqrtf((qx - u) * (qx - u) + (qy - v) * (qy - v));
  feat[4] = one_minus_cos;
  feat[5] = sqrtf(gx * gx + gy * gy) * __builtin_amdgcn_rcpf(d0);
  feat[6] = px.x7;
  feat[7] = static_cast<float>(dj) * a.inv_w;
}

// Lower median (sorted[(n - 1) / 2]) of each colour channel over records [s, e),
// by binary search on binary16 bit patterns (colours are non-negative, so the
// patterns order like the values). Lanes lane0 .. lane0 + width - 1 cooperate.
template <int kWidth>
__device__ __forceinline__ void set_median(gp<const uint2> crho, int64_t s, int64_t e, int sub,
                                           float& mr, float& mg, float& mb) {
  const int64_t n = e - s;
  mr = mg = mb = 0.0f;
  if (n <= 0) return;
  const int need = static_cast<int>((n - 1) / 2 + 1);
  uint32_t lo[3] = {0u, 0u, 0u}, hi[3] = {0x7BFFu, 0x7BFFu, 0x7BFFu};
  for (int it = 0; it < 15; ++it) {
    uint32_t mid[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) mid[c] = (lo[c] + hi[c]) >> 1;
    int cnt[3] = {0, 0, 0};
    for (int64_t i = s + sub; i < e; i += kWidth) {
      const uint2 r = ld2(crho + i);
      cnt[0] += (r.x & 0xFFFFu) <= mid[0];
      cnt[1] += (r.x >> 16) <= mid[1];
      cnt[2] += (r.y & 0xFFFFu) <= mid[2];
    }
#pragma unroll
    for (int off = kWidth / 2; off > 0; off >>= 1)
#pragma unroll
      for (int c = 0; c < 3; ++c) cnt[c] += __shfl_xor(cnt[c], off, kWidth);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (cnt[c] >= need) hi[c] = mid[c]; else lo[c] = mid[c] + 1;
    }
  }
  mr = h2f(lo[0]);
  mg = h2f(lo[1]);
  mb = h2f(lo[2]);
}

// ---------------------------------------------------------------------------
// a7: learned filter (inference).

constexpr int kFlatPix = 16;  // output pixels per wave of the learned filter

// Lower median per channel over records [s, e) when every colour is one of the 256
// staged codes c / 255 (binary16 bits code[c], increasing in c): binary search over
// c, 8 steps. Lanes sub = 0 .. kWidth - 1 cooperate.
template <int kWidth>
__device__ __forceinline__ void set_median_codes(gp<const uint2> crho, int64_t s, int64_t e, int sub,
                                                 const uint16_t* __restrict__ code, float* med) {
  const int64_t n = e - s;
  med[0] = med[1] = med[2] = 0.0f;
  if (n <= 0) return;
  const int need = static_cast<int>((n - 1) / 2 + 1);
  int lo[3] = {0, 0, 0}, hi[3] = {255, 255, 255};
  for (int it = 0; it < 8; ++it) {
    uint32_t t[3];
    int cnt[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) t[c] = code[(lo[c] + hi[c]) >> 1];
    for (int64_t i = s + sub; i < e; i += kWidth) {
      const uint2 r = ld2(crho + i);
      cnt[0] += (r.x & 0xFFFFu) <= t[0];
      cnt[1] += (r.x >> 16) <= t[1];
      cnt[2] += (r.y & 0xFFFFu) <= t[2];
    }
#pragma unroll
    for (int off = kWidth / 2; off > 0; off >>= 1)
#pragma unroll
      for (int c = 0; c < 3; ++c) cnt[c] += __shfl_xor(cnt[c], off, kWidth);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int mid = (lo[c] + hi[c]) >> 1;
      if (cnt[c] >= need) hi[c] = mid; else lo[c] = mid + 1;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) med[c] = h2f(code[lo[c]]);
}

// A operands of the matrix products in LDS, one 16-byte entry per lane: entries
// 0, 1 = layer 1 tiles, 2 + 4 t2 + s = layer 2 output tile t2, K-step s.
constexpr int kAOps = 10;

// v_mfma_f32_32x32x16_bf16: lane (hi32, col) holds A[col][8 hi32 + j] and
// B[8 hi32 + j][col], j = 0..7. Layer 2 (and its backward) take their B operand
// straight from the accumulator of the layer before: K element (hi32, j) of K-step
// s is hidden unit 32(s/2) + 8(2(s%2) + j/4) + 4 hi32 + j%4, which is element
// 8(s%2) + j of this lane's accumulator tile s/2 (no data movement between lanes).
__device__ __forceinline__ int kstep_unit(int s, int hi32, int j) {
  return 32 * (s / 2) + 8 * (2 * (s % 2) + j / 4) + 4 * hi32 + j % 4;
}

// Layer 1, tile t: K = 16 = the 8 features' hi parts (hi32 = 0) and lo parts
// (hi32 = 1), so both halves hold W1[j][32t + col], halved (y = z/2).
template <typename P>
__device__ __forceinline__ u32x4 a_operand_l1(P mw, int t, int col) {
  u32x4 v;
#pragma unroll
  for (int p = 0; p < 4; ++p)
    v[p] = bf16_half_bits(mw[(2 * p) * kNH + 32 * t + col]) |
           (bf16_half_bits(mw[(2 * p + 1) * kNH + 32 * t + col]) << 16);
  return v;
}

// Layer 2, output tile t2, K-step s: W2[kstep_unit(s, hi32, j)][32 t2 + col], halved.
template <typename P>
__device__ __forceinline__ u32x4 a_operand_l2(P mw, int t2, int s, int hi32, int col) {
  u32x4 v;
#pragma unroll
  for (int p = 0; p < 4; ++p)
    v[p] = bf16_half_bits(mw[kOffW2 + kstep_unit(s, hi32, 2 * p) * kNH + 32 * t2 + col]) |
           (bf16_half_bits(mw[kOffW2 + kstep_unit(s, hi32, 2 * p + 1) * kNH + 32 * t2 + col]) << 16);
  return v;
}

// The MLP on the wave's 64 samples (features staged in xs[0] (hi) / xs[1] (lo),
// one uint4 per sample): returns the logit of the lane's own sample.
// kTable: GELU from the chord table s_gelu (inference); otherwise 7.1.28 (training).
template <bool kTable>
__device__ __forceinline__ float mlp_logits_64(const u32x4 (*s_a)[64], const uint4* xs_hi, const uint4* xs_lo,
                                               const float* s_bh, const float* s_w3, float b3, int hi32,
                                               int col, const float2* s_gelu) {
  const int lane = 32 * hi32 + col;
  float m_own = 0.0f;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    // B operand of layer 1: sample 32u + col, hi parts (hi32 = 0) or lo parts (hi32 = 1)
    const uint4 xv = (hi32 ? xs_lo : xs_hi)[32 * u + col];
    const bf16x8 bx = as_bf16x8(u32x4{xv.x, xv.y, xv.z, xv.w});
    // layer 1 + GELU; element a of tile t is hidden 32t + 8(a/4) + 4 hi32 + a%4
    uint32_t ph[2][8], pl[2][8];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      // y = z/2: the accumulator starts at b/2
      v16f c;
#pragma unroll
      for (int a = 0; a < 16; ++a) c[a] = s_bh[32 * t + 8 * (a / 4) + 4 * hi32 + a % 4];
      const v16f d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(s_a[t][lane]), bx, c, 0, 0, 0);
#pragma unroll
      for (int p = 0; p < 8; ++p)
        split_pack(kTable ? gelu_half_table(s_gelu, d[2 * p]) : gelu_half(d[2 * p]),
                   kTable ? gelu_half_table(s_gelu, d[2 * p + 1]) : gelu_half(d[2 * p + 1]), ph[t][p], pl[t][p]);
    }
    // layer 2 (hi and lo passes) and the output unit on the vector units
    float mpart = 0.0f;
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2) {
      v16f d;
#pragma unroll
      for (int a = 0; a < 16; ++a) d[a] = s_bh[kNH + 32 * t2 + 8 * (a / 4) + 4 * hi32 + a % 4];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int t = st / 2, p0 = 4 * (st % 2);
        const u32x4 bh = {ph[t][p0], ph[t][p0 + 1], ph[t][p0 + 2], ph[t][p0 + 3]};
        const u32x4 bl = {pl[t][p0], pl[t][p0 + 1], pl[t][p0 + 2], pl[t][p0 + 3]};
        const bf16x8 a2 = as_bf16x8(s_a[2 + 4 * t2 + st][lane]);
        d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, as_bf16x8(bh), d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, as_bf16x8(bl), d, 0, 0, 0);
      }
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int hid = 32 * t2 + 8 * q4 + 4 * hi32 + r;
          mpart = fmaf(s_w3[hid], kTable ? gelu_half_table(s_gelu, d[4 * q4 + r]) : gelu_half(d[4 * q4 + r]),
                       mpart);
        }
    }
    const float msum = mpart + __shfl_xor(mpart, 32, 64) + b3;
    if (u == hi32) m_own = msum;
    // the two halves run one after the other: interleaving them (the compiler's
    // choice) keeps eight 16-register accumulators live and halves the waves per SIMD
    __builtin_amdgcn_sched_barrier(0);
  }
  return m_own;
}

// Per output pixel of a wave, in LDS.
struct FlatPixel {
  int64_t s, e;                  // CSR range
  float x, y, dp, x7;
  float med[3], cref[3];
  int f, fo;
  float run_m, run_z, acc[3];    // online softmax state
};

// ---------------------------------------------------------------------------
// a7: learned filter (inference). Each wave owns kFlatPix consecutive output
// pixels and streams their records, which are contiguous in the CSR arena, 64 at
// a time: lane l takes record base + l, so every matrix-core column is a real
// sample except in the wave's last step, whatever the set sizes. The set softmax
// is a segmented reduction across lanes (records are sorted by pixel): a
// segmented max scan, then segmented sums of e^(m - max) and e^(m - max) c; the
// last lane of each pixel's run merges the run into that pixel's online state.

__global__ __launch_bounds__(256) void k_filter_learned(
    const uint2* __restrict__ rgbd, const uint16_t* __restrict__ depth, const float* __restrict__ rel,
    int width, int height, int n_frames, int f0, int w, float log_norm, float fx, float fy, float cx, float cy,
    int64_t n_pix, const int64_t* __restrict__ offsets, const uint32_t* __restrict__ ids,
    const uint2* __restrict__ crho, int64_t capacity, const uint16_t* __restrict__ mw,
    const float* __restrict__ mb, float* __restrict__ out) {
  __shared__ float s_bh[2 * kNH];  // b1 / 2, b2 / 2
  __shared__ float s_w3[kNH];
  __shared__ float s_std[2 * kNF];  // mean, 1 / std
  __shared__ uint16_t s_code[256];  // binary16 bits of c / 255
  __shared__ uint4 s_x[2][4][64];   // hi / lo parts; per wave: 64 samples x 8 bfloat16 features
  __shared__ FlatPixel s_px[4][kFlatPix];
  __shared__ u32x4 s_a[kAOps][64];
  __shared__ float2 s_gelu[kGeluCells];
  const int tid = threadIdx.x + threadIdx.y * 64;
  static_assert(kGeluCells == 256 * kGeluCellsPerThread, "one table slice per thread");
  fill_gelu_table(s_gelu, tid);
  for (int i = tid; i < 2 * kNH; i += 256) s_bh[i] = 0.5f * mb[i];
  for (int i = tid; i < kNH; i += 256) s_w3[i] = bf16_to_f(mw[kOffW3 + i]);
  for (int i = tid; i < 2 * kNF; i += 256) s_std[i] = mb[kOffMean + i];
  s_code[tid] = static_cast<uint16_t>(f2h(static_cast<float>(tid) / 255.0f));  // as staged

  const int lane = threadIdx.x, wv = threadIdx.y;
  const int hi32 = lane >> 5, col = lane & 31;
  const int64_t p0 = (static_cast<int64_t>(blockIdx.x) * 4 + wv) * kFlatPix;
  const int64_t plane = static_cast<int64_t>(width) * height;
  const int pw = stored_pitch(width);
  const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
  FlatPixel* px = s_px[wv];

  // A operands (rows = hidden units), the same for every wave: staged once per
  // workgroup in LDS (registers are the kernel's occupancy limit).
  if (wv == 0) {
#pragma unroll
    for (int t = 0; t < 2; ++t) s_a[t][lane] = a_operand_l1(mw, t, col);
  }
  // Layer 2: output tile t2, K-step s (the hi and lo passes share it).
  if (wv == 1) {
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
      for (int st = 0; st < 4; ++st) s_a[2 + 4 * t2 + st][lane] = a_operand_l2(mw, t2, st, hi32, col);
  }
  __syncthreads();
  const float b3 = mb[kOffB3];

  // 1. per-pixel context (lane k < kFlatPix: pixel p0 + k)
  if (lane < kFlatPix) {
    FlatPixel& q = px[lane];
    const int64_t pix = p0 + lane;
    q.run_m = -INFINITY;
    q.run_z = 0.0f;
    q.acc[0] = q.acc[1] = q.acc[2] = 0.0f;
    q.med[0] = q.med[1] = q.med[2] = 0.0f;
    if (pix < n_pix) {
      q.fo = static_cast<int>(pix / plane);
      const int64_t self = pix - q.fo * plane;
      const int y = static_cast<int>(self / width), x = static_cast<int>(self - static_cast<int64_t>(y) * width);
      q.f = f0 + q.fo;
      const size_t pi = static_cast<size_t>(q.f) * pplane + padded_index(x, y, pw);
      const uint2 ref = ld2(to_global(rgbd) + pi);
      q.cref[0] = h2f(ref.x);
      q.cref[1] = h2f(ref.x >> 16);
      q.cref[2] = h2f(ref.y);
      q.x = static_cast<float>(x);
      q.y = static_cast<float>(y);
      q.dp = h2f(ref.y >> 16);  // the depth channel holds the depth plane's binary16
      q.s = offsets[pix];
      q.e = offsets[pix + 1];
      q.x7 = __logf(1.0f + static_cast<float>(q.e - q.s)) / log_norm;
    } else {
      q.fo = 0;
      q.f = f0;
      q.s = q.e = -1;  // not a pixel
    }
  }
  wave_lds_fence_l();
  // The wave's records are [rs, re): the pixels' ranges are consecutive CSR entries.
  // Offsets that decrease (not produced by a count pass) make every pixel of the
  // wave NaN; a pixel whose set ends past the arena is NaN, and so are the pixels
  // after it; nothing outside [0, capacity) is read.
  const int64_t rs = px[0].s;
  int last = -1;
  bool wave_bad = rs < 0 && p0 < n_pix;
  for (int k = 0; k < kFlatPix; ++k) {
    if (px[k].s < 0 && px[k].e < 0) break;  // past the last pixel
    if (px[k].e < px[k].s || px[k].s != (k == 0 ? rs : px[k - 1].e)) wave_bad = true;
    if (!wave_bad && px[k].e <= capacity) last = k;
  }
  if (wave_bad) last = -1;
  const int64_t re = last >= 0 ? px[last].e : rs;
  // run ends relative to rs (a wave's records number far below 2^31), wave-uniform
  int rend[kFlatPix];
#pragma unroll
  for (int j = 0; j < kFlatPix; ++j)
    rend[j] = __builtin_amdgcn_readfirstlane(j <= last ? static_cast<int>(px[j].e - rs) : 0x7FFFFFFF);

  // 2. medians: four pixels at a time, 16 lanes each
  for (int r = 0; r < kFlatPix / 4; ++r) {
    const int k = 4 * r + lane / 16;
    const bool ok = k <= last;
    float med[3];
    set_median_codes<16>(to_global(crho), ok ? px[k].s : 0, ok ? px[k].e : 0, lane % 16, s_code, med);
    if (ok && lane % 16 == 0) {
      px[k].med[0] = med[0];
      px[k].med[1] = med[1];
      px[k].med[2] = med[2];
    }
  }
  wave_lds_fence_l();

  const FeatureArgs fa = feature_args(to_global(depth), width, height, n_frames, w, fx, fy, cx, cy);

  // 3. stream the records
  for (int64_t base = rs; base < re; base += 64) {
    const int64_t idx = base + lane;
    bool live = idx < re;
    // pixel of the record: the number of wave pixels whose range ends at or before
    // it (32-bit compares against scalar registers)
    int k = 0;
    const int ri = static_cast<int>(idx - rs);
#pragma unroll
    for (int j = 0; j < kFlatPix; ++j) k += rend[j] <= ri ? 1 : 0;
    if (k > last) live = false;
    uint2 rec = make_uint2(0u, 0u);
    float feat[kNF] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (live) {
      const FlatPixel& q = px[k];
      const uint32_t id = ids[idx];
      live = id_in_clip(fa, q.f, id);
      if (live) {
        rec = ld2(to_global(crho) + idx);
        PixelCtx pc;
        pc.x = q.x;
        pc.y = q.y;
        pc.dp = q.dp;
        pc.f = q.f;
        pc.medr = q.med[0];
        pc.medg = q.med[1];
        pc.medb = q.med[2];
        pc.x7 = q.x7;
        FeatureArgs fk = fa;
        fk.rel = to_global(rel) + static_cast<size_t>(q.fo) * (2 * w + 1) * kRelStride;
        sample_features(fk, pc, id, rec, feat);
      }
    }
    uint32_t xh[4], xl[4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
      split_pack((feat[2 * p] - s_std[2 * p]) * s_std[kNF + 2 * p],
                 (feat[2 * p + 1] - s_std[2 * p + 1]) * s_std[kNF + 2 * p + 1], xh[p], xl[p]);
    s_x[0][wv][lane] = make_uint4(xh[0], xh[1], xh[2], xh[3]);
    s_x[1][wv][lane] = make_uint4(xl[0], xl[1], xl[2], xl[3]);
    wave_lds_fence_l();
    const float m_own = mlp_logits_64<true>(s_a, s_x[0][wv], s_x[1][wv], s_bh, s_w3, b3, hi32, col, s_gelu);

    // segmented softmax over the lanes: key = pixel (dead lanes get keys of their own)
    // (every shuffle runs on all 64 lanes: a lane that skipped one would leave its
    // value unread by the lanes that take it)
    const int key = live ? k : kFlatPix + lane;
    const int key_next = __shfl_down(key, 1, 64);
    const bool is_last = lane == 63 || key_next != key;
    const uint64_t last_mask = __ballot(is_last);
    const int seg_end = lane + __builtin_ctzll(last_mask >> lane);
    bool same[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      const int key_prev = __shfl_up(key, 1 << l, 64);
      same[l] = lane >= (1 << l) && key_prev == key;
    }
    float mx = live ? m_own : -INFINITY;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      const float o = __shfl_up(mx, 1 << l, 64);
      if (same[l]) mx = fmaxf(mx, o);
    }
    const float seg_max = __shfl(mx, seg_end, 64);
    const float ew = live ? __builtin_amdgcn_exp2f((m_own - seg_max) * kLog2e) : 0.0f;
    float v[4] = {ew, ew * h2f(rec.x), ew * h2f(rec.x >> 16), ew * h2f(rec.y)};
#pragma unroll
    for (int l = 0; l < 6; ++l) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float o = __shfl_up(v[c], 1 << l, 64);
        if (same[l]) v[c] += o;
      }
    }
    if (is_last && live) {
      FlatPixel& q = px[k];
      const float nm = fmaxf(q.run_m, seg_max);
      const float so = q.run_z > 0.0f ? __builtin_amdgcn_exp2f((q.run_m - nm) * kLog2e) : 0.0f;
      const float sn = __builtin_amdgcn_exp2f((seg_max - nm) * kLog2e);
      q.run_z = q.run_z * so + v[0] * sn;
      q.acc[0] = q.acc[0] * so + v[1] * sn;
      q.acc[1] = q.acc[1] * so + v[2] * sn;
      q.acc[2] = q.acc[2] * so + v[3] * sn;
      q.run_m = nm;
    }
    wave_lds_fence_l();
  }

  // 4. outputs
  if (lane < kFlatPix && p0 + lane < n_pix) {
    const FlatPixel& q = px[lane];
    float* o = out + static_cast<size_t>(p0 + lane) * 3;
    if (lane > last) {
      o[0] = o[1] = o[2] = __builtin_nanf("");
    } else if (q.run_z > 0.0f) {
      const float inv = 1.0f / q.run_z;
      o[0] = q.acc[0] * inv;
      o[1] = q.acc[1] * inv;
      o[2] = q.acc[2] * inv;
    } else {
      o[0] = q.cref[0];
      o[1] = q.cref[1];
      o[2] = q.cref[2];
    }
  }
}

// ---------------------------------------------------------------------------
// a8: training. One wave (block of 64) per minibatch pixel at a time.

constexpr int kTS = 65;  // LDS row stride (odd: conflict-free column access)

struct TrainArgs {
  const uint2* rgbd;
  const uint16_t* depth;
  const float* rel;
  int width, height, n_frames, f0, w;
  float log_norm, fx, fy, cx, cy;
  const int64_t* offsets;
  const uint32_t* ids;
  const uint2* crho;
  int64_t capacity, n_all;
  const int32_t* pixel_idx;
  int n_pix;
  const float* clean;
  const uint16_t* mw;
  const float* mb;
  float* grad;
  float* loss;
};

// The kernels' view of TrainArgs: every pointer in the global address space
// (pointers inside a by-value argument struct are otherwise generic).
struct TrainDev {
  gp<const uint2> rgbd;
  gp<const uint16_t> depth;
  gp<const float> rel;
  int width, height, n_frames, f0, w;
  float log_norm, fx, fy, cx, cy;
  gp<const int64_t> offsets;
  gp<const uint32_t> ids;
  gp<const uint2> crho;
  int64_t capacity, n_all;
  gp<const int32_t> pixel_idx;
  int n_pix;
  gp<const float> clean;
  gp<const uint16_t> mw;
  gp<const float> mb;
  gp<float> grad;
  gp<float> loss;
};

__device__ __forceinline__ TrainDev dev_args(const TrainArgs& a) {
  TrainDev d;
  d.rgbd = to_global(a.rgbd);
  d.depth = to_global(a.depth);
  d.rel = to_global(a.rel);
  d.width = a.width;
  d.height = a.height;
  d.n_frames = a.n_frames;
  d.f0 = a.f0;
  d.w = a.w;
  d.log_norm = a.log_norm;
  d.fx = a.fx;
  d.fy = a.fy;
  d.cx = a.cx;
  d.cy = a.cy;
  d.offsets = to_global(a.offsets);
  d.ids = to_global(a.ids);
  d.crho = to_global(a.crho);
  d.capacity = a.capacity;
  d.n_all = a.n_all;
  d.pixel_idx = to_global(a.pixel_idx);
  d.n_pix = a.n_pix;
  d.clean = to_global(a.clean);
  d.mw = to_global(a.mw);
  d.mb = to_global(a.mb);
  d.grad = to_global(a.grad);
  d.loss = to_global(a.loss);
  return d;
}

__device__ __forceinline__ void add_f32(gp<float> p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Backward A operand, rows = layer-1 unit i = 32 t1 + col, K-step s over layer-2
// units in the accumulator order: W2[i][kstep_unit(s, hi32, j)] (not halved).
template <typename P>
__device__ __forceinline__ u32x4 a_operand_back(P mw, int t1, int s, int hi32, int col) {
  u32x4 v;
  const int row = kOffW2 + (32 * t1 + col) * kNH;
#pragma unroll
  for (int p = 0; p < 4; ++p)
    v[p] = static_cast<uint32_t>(mw[row + kstep_unit(s, hi32, 2 * p)]) |
           (static_cast<uint32_t>(mw[row + kstep_unit(s, hi32, 2 * p + 1)]) << 16);
  return v;
}

// 8 float32 values as bfloat16 hi / lo operand halves
__device__ __forceinline__ void split8(const float (&v)[8], bf16x8& hi, bf16x8& lo) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) split_pack(v[2 * p], v[2 * p + 1], h[p], l[p]);
  hi = as_bf16x8(u32x4{h[0], h[1], h[2], h[3]});
  lo = as_bf16x8(u32x4{l[0], l[1], l[2], l[3]});
}

// One wave per minibatch pixel at a time, 64 of its records per step (lane =
// record). Pass 1: the inference kernel's matrix-core forward gives the logits,
// an online softmax per lane and a merge over the wave give O(p), the loss and
// dL/dO. Pass 2, per step and per 32-record half: layer 1 and layer 2 forward on
// the matrix cores (transposed: rows = hidden units, columns = records), then
//   dm_s   = a_s (c_s - O) . dL/dO               (a_s = softmax weight)
//   dz2_s  = dm_s w3 * GELU'(z2_s)
//   dz1^T  = W2 dz2^T * GELU'(z1)                 (matrix cores, hi / lo dz2)
// and, with the step's h1, dz2, dz1, h2, x in LDS as [record][unit] rows,
//   dW2   += H1^T DZ2 over the step's 64 records   (matrix cores: operands read
//            transposed from LDS, hi*hi + hi*lo + lo*hi products, float32
//            accumulators held for the whole kernel)
//   dW1, dW3, db1, db2, db3 on the vector units (lane = unit).
// The gradients are summed into ta.grad (float32 atomics) at the end.
__global__ __launch_bounds__(64) void k_mlp_train_grad(TrainArgs ta_in) {
  const TrainDev ta = dev_args(ta_in);
  __shared__ float s_bh[2 * kNH];  // b1 / 2, b2 / 2
  __shared__ float s_w3[kNH];
  __shared__ float s_std[2 * kNF];  // mean, 1 / std
  __shared__ u32x4 s_a[kAOps][64];  // forward A operands
  __shared__ u32x4 s_ab[8][64];     // backward A operands, entry 4 t1 + s
  __shared__ uint4 s_x[2][64];      // hi / lo feature parts of the step's records
  __shared__ float s_h1[64 * kTS];  // [record][unit]
  __shared__ float s_dz2[64 * kTS];
  __shared__ float s_dz1[64 * kTS];
  __shared__ float s_h2[64 * kTS];
  __shared__ float s_xf[64 * 9];    // standardised features (hi + lo values)
  __shared__ float s_dm[64];
  const int lane = threadIdx.x;
  const int hi32 = lane >> 5, col = lane & 31;
  for (int i = lane; i < 2 * kNH; i += 64) s_bh[i] = 0.5f * ta.mb[i];
  s_w3[lane] = bf16_to_f(ta.mw[kOffW3 + lane]);
  if (lane < 2 * kNF) s_std[lane] = ta.mb[kOffMean + lane];
#pragma unroll
  for (int t = 0; t < 2; ++t) s_a[t][lane] = a_operand_l1(ta.mw, t, col);
#pragma unroll
  for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      s_a[2 + 4 * t2 + st][lane] = a_operand_l2(ta.mw, t2, st, hi32, col);
      s_ab[4 * t2 + st][lane] = a_operand_back(ta.mw, t2, st, hi32, col);
    }
  __syncthreads();
  const float b3 = ta.mb[kOffB3];

  const size_t plane = static_cast<size_t>(ta.width) * ta.height;
  FeatureArgs fa = feature_args(ta.depth, ta.width, ta.height, ta.n_frames, ta.w, ta.fx, ta.fy, ta.cx, ta.cy);

  // dW2 accumulators: tile (ti, tj), element a = dW2[32 ti + 8(a/4) + 4 hi32 + a%4][32 tj + col]
  v16f gw2[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int a = 0; a < 16; ++a) gw2[ti][tj][a] = 0.0f;
  // lane = unit: dW1 entries (k = lane/8, j = 8(lane%8) + jj), dW3[lane], db1[lane], db2[lane], db3
  float gw1[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float gw3 = 0.f, gb1 = 0.f, gb2 = 0.f, gb3 = 0.f;
  const float inv3n = 1.0f / (3.0f * static_cast<float>(ta.n_pix));

  for (int bi = blockIdx.x; bi < ta.n_pix; bi += gridDim.x) {
    const int64_t pix = ta.pixel_idx[bi];
    if (pix < 0 || pix >= ta.n_all) continue;
    const int fo = static_cast<int>(pix / static_cast<int64_t>(plane));
    const int64_t self = pix - static_cast<int64_t>(fo) * plane;
    const int y = static_cast<int>(self / ta.width), x = static_cast<int>(self - static_cast<int64_t>(y) * ta.width);
    const int64_t s = ta.offsets[pix], e = ta.offsets[pix + 1];
    if (s < 0 || e <= s || e > ta.capacity) continue;
    PixelCtx px;
    px.x = static_cast<float>(x);
    px.y = static_cast<float>(y);
    px.dp = depth_at(ta.depth, ta.width, ta.height, ta.f0 + fo, x, y);
    px.f = ta.f0 + fo;
    px.x7 = __logf(1.0f + static_cast<float>(e - s)) / ta.log_norm;
    set_median<64>(ta.crho, s, e, lane, px.medr, px.medg, px.medb);
    fa.rel = ta.rel + static_cast<size_t>(fo) * (2 * ta.w + 1) * kRelStride;

    // features of record base + lane into s_x (hi / lo) and, if asked, s_xf;
    // a record outside the set or the clip is dead (features 0, no weight)
    auto stage = [&](int64_t base, bool keep_f32, uint2& rec) -> bool {
      const int64_t idx = base + lane;
      const bool live = idx < e && id_in_clip(fa, px.f, ta.ids[idx]);
      float xs[kNF] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      rec = make_uint2(0u, 0u);
      if (live) {
        rec = ld2(ta.crho + idx);
        float feat[kNF];
        sample_features(fa, px, ta.ids[idx], rec, feat);
#pragma unroll
        for (int k = 0; k < kNF; ++k) xs[k] = (feat[k] - s_std[k]) * s_std[kNF + k];
      }
      uint32_t xh[4], xl[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) split_pack(xs[2 * q], xs[2 * q + 1], xh[q], xl[q]);
      s_x[0][lane] = make_uint4(xh[0], xh[1], xh[2], xh[3]);
      s_x[1][lane] = make_uint4(xl[0], xl[1], xl[2], xl[3]);
      if (keep_f32) {
#pragma unroll
        for (int k = 0; k < kNF; ++k) s_xf[lane * 9 + k] = split_value(xs[k]);
      }
      return live;
    };

    // pass 1: softmax statistics and O(p)
    float run_m = -INFINITY, run_z = 0.f, acc[3] = {0.f, 0.f, 0.f};
    for (int64_t base = s; base < e; base += 64) {
      uint2 rec;
      const bool live = stage(base, false, rec);
      wave_lds_fence_l();
      const float m = mlp_logits_64<false>(s_a, s_x[0], s_x[1], s_bh, s_w3, b3, hi32, col, nullptr);
      wave_lds_fence_l();
      if (live) {
        const float nm = fmaxf(run_m, m);
        const float sc = __expf(run_m - nm), ew = __expf(m - nm);
        run_z = fmaf(run_z, sc, ew);
        acc[0] = fmaf(acc[0], sc, ew * h2f(rec.x));
        acc[1] = fmaf(acc[1], sc, ew * h2f(rec.x >> 16));
        acc[2] = fmaf(acc[2], sc, ew * h2f(rec.y));
        run_m = nm;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float om = __shfl_xor(run_m, off, 64), oz = __shfl_xor(run_z, off, 64);
      const float o0 = __shfl_xor(acc[0], off, 64), o1 = __shfl_xor(acc[1], off, 64), o2 = __shfl_xor(acc[2], off, 64);
      const float nm = fmaxf(run_m, om);
      const float sa = run_z > 0.f ? __expf(run_m - nm) : 0.f, sb = oz > 0.f ? __expf(om - nm) : 0.f;
      run_z = run_z * sa + oz * sb;
      acc[0] = acc[0] * sa + o0 * sb;
      acc[1] = acc[1] * sa + o1 * sb;
      acc[2] = acc[2] * sa + o2 * sb;
      run_m = nm;
    }
    if (!(run_z > 0.0f)) continue;  // every record skipped: nothing to learn from (uniform)
    const float zinv = 1.0f / run_z;
    float o[3], dO[3];
    float l2 = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      o[c] = acc[c] * zinv;
      const float d = o[c] - ta.clean[static_cast<size_t>(bi) * 3 + c];
      l2 = fmaf(d, d, l2);
      dO[c] = 2.0f * d * inv3n;
    }
    if (lane == 0) add_f32(ta.loss, l2 * inv3n);

    // pass 2: backward, 64 records per step
    for (int64_t base = s; base < e; base += 64) {
      uint2 rec;
      const bool live = stage(base, true, rec);
      wave_lds_fence_l();
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int rs = 32 * u + col;  // record (within the step) of this lane's column
        // layer 1: y1 = z1 / 2, tile t element a = unit 32t + 8(a/4) + 4 hi32 + a%4
        const uint4 xv = (hi32 ? s_x[1] : s_x[0])[rs];
        const bf16x8 bx = as_bf16x8(u32x4{xv.x, xv.y, xv.z, xv.w});
        v16f y1[2];
        uint32_t ph[2][8], pl[2][8];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          v16f c;
#pragma unroll
          for (int a = 0; a < 16; ++a) c[a] = s_bh[32 * t + 8 * (a / 4) + 4 * hi32 + a % 4];
          y1[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(s_a[t][lane]), bx, c, 0, 0, 0);
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            split_pack(gelu_half(y1[t][2 * q]), gelu_half(y1[t][2 * q + 1]), ph[t][q], pl[t][q]);
            // h1 = hi + lo, as the matrix cores see it
            const int a0 = 2 * q;  // elements 2q, 2q + 1: units r0, r0 + 1
            const int r0 = 32 * t + 8 * (a0 / 4) + 4 * hi32 + a0 % 4, r1 = r0 + 1;
            s_h1[rs * kTS + r0] = __uint_as_float(ph[t][q] << 16) + __uint_as_float(pl[t][q] << 16);
            s_h1[rs * kTS + r1] =
                __uint_as_float(ph[t][q] & 0xFFFF0000u) + __uint_as_float(pl[t][q] & 0xFFFF0000u);
          }
        }
        // layer 2: y2 = z2 / 2, same element layout
        v16f y2[2];
#pragma unroll
        for (int t2 = 0; t2 < 2; ++t2) {
#pragma unroll
          for (int a = 0; a < 16; ++a) y2[t2][a] = s_bh[kNH + 32 * t2 + 8 * (a / 4) + 4 * hi32 + a % 4];
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            const int t = st / 2, p0 = 4 * (st % 2);
            const u32x4 bh = {ph[t][p0], ph[t][p0 + 1], ph[t][p0 + 2], ph[t][p0 + 3]};
            const u32x4 bl = {pl[t][p0], pl[t][p0 + 1], pl[t][p0 + 2], pl[t][p0 + 3]};
            const bf16x8 a2 = as_bf16x8(s_a[2 + 4 * t2 + st][lane]);
            y2[t2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, as_bf16x8(bh), y2[t2], 0, 0, 0);
            y2[t2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, as_bf16x8(bl), y2[t2], 0, 0, 0);
          }
        }
        // logit of record rs, then dm for it (its colour and liveness from lane rs)
        float mpart = 0.0f;
#pragma unroll
        for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
          for (int a = 0; a < 16; ++a) {
            const int j = 32 * t2 + 8 * (a / 4) + 4 * hi32 + a % 4;
            const float h2 = gelu_half(y2[t2][a]);
            s_h2[rs * kTS + j] = h2;
            mpart = fmaf(s_w3[j], h2, mpart);
          }
        const float m = mpart + __shfl_xor(mpart, 32, 64) + b3;
        const uint32_t rx = __shfl(rec.x, rs, 64), ry = __shfl(rec.y, rs, 64);
        const int live_rs = __shfl(live ? 1 : 0, rs, 64);
        float dm = 0.0f;
        if (live_rs) {
          const float a = __expf(m - run_m) * zinv;
          dm = a * ((h2f(rx) - o[0]) * dO[0] + (h2f(rx >> 16) - o[1]) * dO[1] + (h2f(ry) - o[2]) * dO[2]);
        }
        if (hi32 == 0) s_dm[rs] = dm;
        // dz2 = dm w3 GELU'(z2), z2 = 2 y2; as hi / lo B operands of the backward product
        uint32_t dh[2][8], dl[2][8];
#pragma unroll
        for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            float g[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int a = 2 * q + h;
              const int j = 32 * t2 + 8 * (a / 4) + 4 * hi32 + a % 4;
              g[h] = dm * s_w3[j] * gelu_grad(2.0f * y2[t2][a]);
              s_dz2[rs * kTS + j] = g[h];
            }
            split_pack(g[0], g[1], dh[t2][q], dl[t2][q]);
          }
        // dz1^T = W2 dz2^T, then * GELU'(z1), z1 = 2 y1
#pragma unroll
        for (int t1 = 0; t1 < 2; ++t1) {
          v16f d1;
#pragma unroll
          for (int a = 0; a < 16; ++a) d1[a] = 0.0f;
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            const int t = st / 2, p0 = 4 * (st % 2);
            const u32x4 bh = {dh[t][p0], dh[t][p0 + 1], dh[t][p0 + 2], dh[t][p0 + 3]};
            const u32x4 bl = {dl[t][p0], dl[t][p0 + 1], dl[t][p0 + 2], dl[t][p0 + 3]};
            const bf16x8 ab = as_bf16x8(s_ab[4 * t1 + st][lane]);
            d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, as_bf16x8(bh), d1, 0, 0, 0);
            d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, as_bf16x8(bl), d1, 0, 0, 0);
          }
#pragma unroll
          for (int a = 0; a < 16; ++a) {
            const int i = 32 * t1 + 8 * (a / 4) + 4 * hi32 + a % 4;
            s_dz1[rs * kTS + i] = d1[a] * gelu_grad(2.0f * y1[t1][a]);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      wave_lds_fence_l();
      // dW2 += H1^T DZ2 over the step's records: K = record, 16 per product
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          float va[8], vb[8];
#pragma unroll
          for (int jj = 0; jj < 8; ++jj) {
            const int r = 16 * ks + 8 * hi32 + jj;
            va[jj] = s_h1[r * kTS + 32 * t + col];
            vb[jj] = s_dz2[r * kTS + 32 * t + col];
          }
          split8(va, ah[t], al[t]);
          split8(vb, bh[t], bl[t]);
        }
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 2; ++tj) {
            gw2[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ti], bh[tj], gw2[ti][tj], 0, 0, 0);
            gw2[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ti], bl[tj], gw2[ti][tj], 0, 0, 0);
            gw2[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[ti], bh[tj], gw2[ti][tj], 0, 0, 0);
          }
      }
      // the small gradients on the vector units, lane = unit
      for (int r = 0; r < 64; ++r) {
        const float xk = s_xf[r * 9 + lane / 8];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) gw1[jj] = fmaf(xk, s_dz1[r * kTS + 8 * (lane % 8) + jj], gw1[jj]);
        const float dmr = s_dm[r];
        gw3 = fmaf(dmr, s_h2[r * kTS + lane], gw3);
        gb1 += s_dz1[r * kTS + lane];
        gb2 += s_dz2[r * kTS + lane];
        gb3 += dmr;
      }
      wave_lds_fence_l();
    }
  }
  // master order: W1 [8][64], W2 [64][64], W3 [64], b1 [64], b2 [64], b3
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int a = 0; a < 16; ++a) {
        const int i = 32 * ti + 8 * (a / 4) + 4 * hi32 + a % 4, j = 32 * tj + col;
        add_f32(ta.grad + (kOffW2 + i * kNH + j), gw2[ti][tj][a]);
      }
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) add_f32(ta.grad + ((lane / 8) * kNH + 8 * (lane % 8) + jj), gw1[jj]);
  add_f32(ta.grad + (kOffW3 + lane), gw3);
  add_f32(ta.grad + (SG_MLP_NW + lane), gb1);
  add_f32(ta.grad + (SG_MLP_NW + kNH + lane), gb2);
  if (lane == 0) add_f32(ta.grad + (SG_MLP_NW + 2 * kNH), gb3);
}

__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ master, float* __restrict__ mm,
                                                  float* __restrict__ vv, float* __restrict__ grad,
                                                  uint16_t* __restrict__ wb, float* __restrict__ bf,
                                                  float lr, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= SG_MLP_NPARAM) return;
  const float gv = grad[i];
  const float m = 0.9f * mm[i] + 0.1f * gv;
  const float v = 0.999f * vv[i] + 0.001f * gv * gv;
  mm[i] = m;
  vv[i] = v;
  const float p = master[i] - lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
  master[i] = p;
  grad[i] = 0.0f;
  if (i < SG_MLP_NW) wb[i] = static_cast<uint16_t>(bf16_bits(p));
  else bf[i - SG_MLP_NW] = p;  // b1, b2, b3 occupy the first 129 entries of b
}

__global__ void k_clear1(float* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0.0f;
}

// Feature statistics for the standardisation: adds, over the records of the
// minibatch pixels, the record count, sum x_k and sum x_k^2 of the raw features
// into moments[0], [1 + k], [9 + k] (float64). One wave per pixel.
__global__ __launch_bounds__(64) void k_feature_moments(TrainArgs ta_in, double* __restrict__ moments) {
  const TrainDev ta = dev_args(ta_in);
  const int lane = threadIdx.x;
  const size_t plane = static_cast<size_t>(ta.width) * ta.height;
  FeatureArgs fa = feature_args(ta.depth, ta.width, ta.height, ta.n_frames, ta.w, ta.fx, ta.fy, ta.cx, ta.cy);
  double cnt = 0.0, sum[kNF], sq[kNF];
#pragma unroll
  for (int k = 0; k < kNF; ++k) sum[k] = sq[k] = 0.0;
  for (int bi = blockIdx.x; bi < ta.n_pix; bi += gridDim.x) {
    const int64_t pix = ta.pixel_idx[bi];
    if (pix < 0 || pix >= ta.n_all) continue;
    const int fo = static_cast<int>(pix / static_cast<int64_t>(plane));
    const int64_t self = pix - static_cast<int64_t>(fo) * plane;
    const int y = static_cast<int>(self / ta.width), x = static_cast<int>(self - static_cast<int64_t>(y) * ta.width);
    const int64_t s = ta.offsets[pix], e = ta.offsets[pix + 1];
    if (s < 0 || e <= s || e > ta.capacity) continue;
    PixelCtx px;
    px.x = static_cast<float>(x);
    px.y = static_cast<float>(y);
    px.dp = depth_at(ta.depth, ta.width, ta.height, ta.f0 + fo, x, y);
    px.f = ta.f0 + fo;
    px.x7 = __logf(1.0f + static_cast<float>(e - s)) / ta.log_norm;
    set_median<64>(ta.crho, s, e, lane, px.medr, px.medg, px.medb);
    fa.rel = ta.rel + static_cast<size_t>(fo) * (2 * ta.w + 1) * kRelStride;
    for (int64_t idx = s + lane; idx < e; idx += 64) {
      const uint32_t id = ta.ids[idx];
      if (!id_in_clip(fa, px.f, id)) continue;
      float feat[kNF];
      sample_features(fa, px, id, ld2(ta.crho + idx), feat);
      cnt += 1.0;
#pragma unroll
      for (int k = 0; k < kNF; ++k) {
        sum[k] += feat[k];
        sq[k] += static_cast<double>(feat[k]) * feat[k];
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    cnt += __shfl_xor(cnt, off, 64);
#pragma unroll
    for (int k = 0; k < kNF; ++k) {
      sum[k] += __shfl_xor(sum[k], off, 64);
      sq[k] += __shfl_xor(sq[k], off, 64);
    }
  }
  if (lane == 0 && cnt > 0.0) {
    atomicAdd(&moments[0], cnt);
#pragma unroll
    for (int k = 0; k < kNF; ++k) {
      atomicAdd(&moments[1 + k], sum[k]);
      atomicAdd(&moments[1 + kNF + k], sq[k]);
    }
  }
}

// ---------------------------------------------------------------------------
// launchers

hipError_t launch_filter_learned(const LearnedJob& lj, hipStream_t st) {
  const int64_t waves = (lj.n_pix + kFlatPix - 1) / kFlatPix;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_filter_learned, dim3(static_cast<unsigned>(blocks)), dim3(64, 4), 0, st,
                     reinterpret_cast<const uint2*>(lj.rgbd), lj.depth, lj.rel, lj.width, lj.height,
                     lj.n_frames, lj.f0, lj.w, lj.log_norm, static_cast<float>(lj.fx), static_cast<float>(lj.fy),
                     static_cast<float>(lj.cx), static_cast<float>(lj.cy), lj.n_pix, lj.offsets, lj.ids,
                     reinterpret_cast<const uint2*>(lj.crho), lj.capacity, lj.mw, lj.mb, lj.out);
  return hipGetLastError();
}

static TrainArgs train_args(const LearnedJob& lj, const int32_t* pixel_idx, int n_pix) {
  TrainArgs ta{};
  ta.rgbd = reinterpret_cast<const uint2*>(lj.rgbd);
  ta.depth = lj.depth;
  ta.rel = lj.rel;
  ta.width = lj.width;
  ta.height = lj.height;
  ta.n_frames = lj.n_frames;
  ta.f0 = lj.f0;
  ta.w = lj.w;
  ta.log_norm = lj.log_norm;
  ta.fx = static_cast<float>(lj.fx);
  ta.fy = static_cast<float>(lj.fy);
  ta.cx = static_cast<float>(lj.cx);
  ta.cy = static_cast<float>(lj.cy);
  ta.offsets = lj.offsets;
  ta.ids = lj.ids;
  ta.crho = reinterpret_cast<const uint2*>(lj.crho);
  ta.capacity = lj.capacity;
  ta.n_all = lj.n_pix;
  ta.pixel_idx = pixel_idx;
  ta.n_pix = n_pix;
  return ta;
}

// Feature standardisation from accumulated moments (count, sums, sums of squares):
// mean = sum / n, variance = max(sum of squares / n - mean^2, 0) in float64; a
// feature whose standard deviation is not above 1e-12 max(|mean|, 1) gets 1.
// Writes the float32 mean and 1 / std into the MLP's parameter block.
__global__ __launch_bounds__(64) void k_standardise(const double* __restrict__ moments, float* __restrict__ mb) {
  const int k = threadIdx.x;
  if (k >= kNF) return;
  const double n = fmax(moments[0], 1.0);
  const double mean = moments[1 + k] / n;
  const double var = fmax(moments[1 + kNF + k] / n - mean * mean, 0.0);
  double sd = sqrt(var);
  if (!(sd > 1e-12 * fmax(fabs(mean), 1.0))) sd = 1.0;
  mb[kOffMean + k] = static_cast<float>(mean);
  mb[kOffMean + kNF + k] = static_cast<float>(1.0 / sd);
}

hipError_t launch_standardise(const double* moments, float* mlp_b, hipStream_t st) {
  hipLaunchKernelGGL(k_standardise, dim3(1), dim3(64), 0, st, moments, mlp_b);
  return hipGetLastError();
}

hipError_t launch_feature_moments(const LearnedJob& lj, const int32_t* pixel_idx, int n_pix, double* moments,
                                  hipStream_t st) {
  if (n_pix <= 0) return hipSuccess;
  const TrainArgs ta = train_args(lj, pixel_idx, n_pix);
  const int blocks = n_pix < 4096 ? n_pix : 4096;
  hipLaunchKernelGGL(k_feature_moments, dim3(blocks), dim3(64), 0, st, ta, moments);
  return hipGetLastError();
}

hipError_t launch_mlp_train(const LearnedJob& lj, const TrainJob& tj, hipStream_t st) {
  hipLaunchKernelGGL(k_clear1, dim3(1), dim3(64), 0, st, tj.loss);
  TrainArgs ta = train_args(lj, tj.pixel_idx, tj.n_pix);
  ta.clean = tj.clean;
  ta.mw = tj.w_bf16;
  ta.mb = tj.b_f32;
  ta.grad = tj.grad;
  ta.loss = tj.loss;
  if (tj.n_pix > 0) {
    const int blocks = tj.n_pix < 2048 ? tj.n_pix : 2048;
    hipLaunchKernelGGL(k_mlp_train_grad, dim3(blocks), dim3(64), 0, st, ta);
  }
  const float bc1 = 1.0f - powf(0.9f, static_cast<float>(tj.t));
  const float bc2 = 1.0f - powf(0.999f, static_cast<float>(tj.t));
  hipLaunchKernelGGL(k_mlp_adam, dim3((SG_MLP_NPARAM + 255) / 256), dim3(256), 0, st, tj.master, tj.adam_m,
                     tj.adam_v, tj.grad, tj.w_bf16, tj.b_f32, tj.lr, bc1, bc2);
  return hipGetLastError();
}

}  // namespace sg
