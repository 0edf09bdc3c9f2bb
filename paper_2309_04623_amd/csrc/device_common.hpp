// Device-side building blocks shared by the gfx950 kernels: vector types,
// MFMA wrappers, the operand permutations that let a 32x32 MFMA result feed
// the next MFMA directly, bf16 splitting, wave reductions and the
// counter-based SplitMix64 generator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nmf {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int WAVE = 64;
constexpr int TILE = 32;  // rows/cols of one 32x32 MFMA output

enum Prec { PREC_FP32 = 0, PREC_BF16X3 = 1 };

// ---------------------------------------------------------------------------
// 32x32 MFMA output layout (both v_mfma_f32_32x32x2_f32 and
// v_mfma_f32_32x32x16_bf16): lane l holds column (l & 31) and, in register
// i (0..15), row 8*(i/4) + 4*(l/32) + (i%4).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int acc_row(int i, int half) {
  return 8 * (i >> 2) + 4 * half + (i & 3);
}

// A 32x32 result used as the reduction operand of the next product sums over
// its rows.  The row order each lane supplies is fixed by the layout above,
// so the *other* operand is stored with its reduction index permuted within
// each aligned block of 32 so that every lane reads one contiguous run.
//   FP32 path (v_mfma_f32_32x32x2_f32, one value per lane per step):
//     row 8g + 4h + s  ->  position 16h + 4g + s
//   BF16 path (v_mfma_f32_32x32x16_bf16, eight values per lane per step):
//     row 16j + 8q + 4h + s  ->  position 16j + 8h + 4q + s
__host__ __device__ __forceinline__ int perm_f32(int r) {
  const int blk = r & ~31, x = r & 31;
  const int g = x >> 3, h = (x >> 2) & 1, s = x & 3;
  return blk + 16 * h + 4 * g + s;
}
__host__ __device__ __forceinline__ int perm_bf16(int r) {
  const int blk = r & ~31, x = r & 31;
  const int j = x >> 4, q = (x >> 3) & 1, h = (x >> 2) & 1, s = x & 3;
  return blk + 16 * j + 8 * h + 4 * q + s;
}
template <int PREC>
__host__ __device__ __forceinline__ int perm_red(int r) {
  return PREC == PREC_FP32 ? perm_f32(r) : perm_bf16(r);
}

// ---------------------------------------------------------------------------
// Operand-ordered factor layouts.  For each aligned block of 32 rows the
// values one MFMA operand load needs are stored as [load][lane][vector], so
// every load instruction of a wave reads one contiguous run (1 KB).
//   L  (rows x KP), A operand of Y = L Rt:
//     FP32 load u (0..KP/8-1), lane i + 32h: L(r, h*KP/2 + 4u + j), j < 4
//     BF16 load q (0..KP/16-1), lane i + 32h: L(r, 16q + 8h + e), e < 8
//   L^T (KP x rows) with the reduction index permuted (perm_f32/perm_bf16),
//   A operand of num/den for output tile t = k / 32:
//     FP32 load u (0..3):  lane m + 32h holds rows 8u + 4h + j, j < 4
//     BF16 load q (0..1):  lane m + 32h holds rows 16q + 8e' + 4h + s
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int64_t lop_f32(int r, int k, int KP) {
  const int rb = r >> 5, i = r & 31, hk = KP >> 1;
  const int h = k >= hk, kk = k - h * hk;
  return (((int64_t)rb * (KP >> 3) + (kk >> 2)) * 64 + i + 32 * h) * 4 + (kk & 3);
}
__host__ __device__ __forceinline__ int64_t lop_bf16(int r, int k, int KP) {
  const int rb = r >> 5, i = r & 31;
  const int q = k >> 4, h = (k >> 3) & 1, e = k & 7;
  return (((int64_t)rb * (KP >> 4) + q) * 64 + i + 32 * h) * 8 + e;
}
__host__ __device__ __forceinline__ int64_t ltop_f32(int k, int r, int KP) {
  const int t = k >> 5, m = k & 31, rb = r >> 5, x = r & 31;
  const int g = x >> 3, h = (x >> 2) & 1, s = x & 3;
  return ((((int64_t)rb * (KP >> 5) + t) * 4 + g) * 64 + m + 32 * h) * 4 + s;
}
__host__ __device__ __forceinline__ int64_t ltop_bf16(int k, int r, int KP) {
  const int t = k >> 5, m = k & 31, rb = r >> 5, x = r & 31;
  const int q = x >> 4, e4 = (x >> 3) & 1, h = (x >> 2) & 1, s = x & 3;
  return ((((int64_t)rb * (KP >> 5) + t) * 2 + q) * 64 + m + 32 * h) * 8 + 4 * e4 + s;
}

__device__ __forceinline__ f32x16 mfma_f32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// Split-precision product a*b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi.  The small
// terms go first so they are not absorbed by the large one.
__device__ __forceinline__ f32x16 mfma_bf16x3(bf16x8 ah, bf16x8 al, bf16x8 bh, bf16x8 bl,
                                              f32x16 c) {
  c = mfma_bf16(al, bh, c);
  c = mfma_bf16(ah, bl, c);
  return mfma_bf16(ah, bh, c);
}

// Round-to-nearest-even split x = hi + lo (+ a remainder below 2^-16 |x|).
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// The same split for eight values at once (two values per conversion
// instruction): x = hi + lo + a remainder below 2^-16 |x| per element.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split8_bf16(const float* x, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const f32x2 v = {x[e], x[e + 1]};
    const bf16x2 h = __builtin_convertvector(v, bf16x2);
    const f32x2 hf = __builtin_convertvector(h, f32x2);
    const bf16x2 l = __builtin_convertvector(v - hf, bf16x2);
    hi[e] = h[0];
    hi[e + 1] = h[1];
    lo[e] = l[0];
    lo[e + 1] = l[1];
  }
}

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.f;
  return z;
}

// ---------------------------------------------------------------------------
// Wave-level reductions (fixed order, deterministic).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood 2014) in counter mode.
// ---------------------------------------------------------------------------
constexpr uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ull;
__host__ __device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ uint64_t sm_key(uint64_t seed, int matrix_id) {
  return sm_mix(seed + (uint64_t)(matrix_id + 1) * SM_GAMMA);
}
__host__ __device__ __forceinline__ float sm_uniform(uint64_t key, uint64_t index) {
  const uint64_t u = sm_mix(key + (index + 1) * SM_GAMMA);
  return ((float)(u >> 41) + 0.5f) * (1.0f / 8388608.0f);
}

// Multiplicative-update factor applied to ``old``: old * num / den, or old
// when den == 0, then floored.  Computed in FP64 so that a tiny positive
// denominator cannot overflow an FP32 quotient.
__device__ __forceinline__ float mu_apply(float old, float num, float den, float eps) {
  double v = den > 0.f ? (double)old * (double)num / (double)den : (double)old;
  if (v > 3.4028234663852886e38) v = 3.4028234663852886e38;
  const float r = (float)v;
  return (r > eps || r != r) ? r : eps;  // a NaN propagates to the objective check
}

__device__ __forceinline__ float mu_apply_d(float old, double num, double den, float eps) {
  double v = den > 0.0 ? (double)old * num / den : (double)old;
  if (v > 3.4028234663852886e38) v = 3.4028234663852886e38;
  const float r = (float)v;
  return (r > eps || r != r) ? r : eps;
}

}  // namespace nmf
