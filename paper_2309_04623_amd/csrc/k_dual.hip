// Fused multiplicative-update half-step (Eq. 3 of arXiv:2309.04623) for
// gfx950.
//
// A workgroup of NW waves owns one 32-column tile of the data matrix D
// (R x C) and a chunk of its 32-row tiles; wave w takes row tiles w, w+NW, ...
// For every 32x32 tile a wave
//   1. forms Y = L[rows] * Rt[:, cols] on MFMA (the model W H, Eq. 1),
//   2. reads D and the weights Mw for the same tile, stored in MFMA
//      accumulator order so that the wave fetches them with four fully
//      coalesced 16-byte-per-lane loads (the next tile is prefetched while
//      this one computes),
//      and forms A = Mw o D, Z = Mw o Y and the residual term Mw (D - Y)^2
//      (Eq. 2),
//   3. accumulates num += L^T A and den += L^T Z on MFMA, fed straight from
//      the registers of step 1: the 32x32 accumulator layout is the
//      B-operand layout of the next 32x32 MFMA up to a fixed permutation of
//      the reduction index, and the L^T operand is stored with that
//      permutation applied.
// Y, A and Z never leave registers.  The NW partial sums are combined
// through LDS in a fixed order (bitwise reproducible).
//
// Modes:
//   MODE_UPDATE  one chunk covers all rows: apply Rt <- max(Rt o num/den, eps)
//                to the tile and write the layouts the other half-step reads
//                (the H-rule of Eq. 3 on V; also yields J for W, H).
//   MODE_SPLIT   write num/den partials for the chunk; the finish kernel sums
//                them (the W-rule, on V^T).
//   MODE_OBJ     objective only.
//
// FP32 products use v_mfma_f32_32x32x2_f32.  The split-precision products
// use v_mfma_f32_32x32x16_bf16 three times (hi*hi + hi*lo + lo*hi) with FP32
// accumulation.

#include "device_common.hpp"
#include "kernels.hpp"

namespace nmf {

// p points at lane * 4 floats inside a 1024-float tile; load u reads floats
// [u * 256 + lane * 4, +4), so each load instruction covers one contiguous
// kilobyte.
__device__ __forceinline__ void load_tile(const float* p, f32x4 (&v)[4]) {
  const f32x4* q = reinterpret_cast<const f32x4*>(p);
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(q + 64 * u);
}

// Weights of one tile as a wave holds them: FP32 values (16 per lane, loaded
// like the data) or, for binary weights, one 16-bit mask per lane.
template <bool BIN>
struct MaskTile {
  f32x4 v[4];
  __device__ __forceinline__ void load(const float* pw, const uint16_t*, int64_t t) {
    load_tile(pw + t * 1024, v);
  }
  __device__ __forceinline__ float get(int i) const { return v[i >> 2][i & 3]; }
};
template <>
struct MaskTile<true> {
  uint32_t b;
  __device__ __forceinline__ void load(const float*, const uint16_t* pb, int64_t t) {
    b = __builtin_nontemporal_load(pb + t * 64);
  }
  __device__ __forceinline__ float get(int i) const { return (b >> i) & 1u ? 1.f : 0.f; }
};

// Operand registers of one 32-row tile: the L rows (A operand of Y = L Rt)
// and the permuted L^T block (A operand of num/den).
template <int PREC, int KP>
struct Ops {
  static constexpr int MT = KP / 32;
  static constexpr int NL_F32 = (PREC == PREC_FP32) ? KP / 8 : 1;
  static constexpr int NL_BF = (PREC == PREC_FP32) ? 1 : KP / 16;
  static constexpr int NT_F32 = (PREC == PREC_FP32) ? MT * 4 : 1;
  static constexpr int NT_BF = (PREC == PREC_FP32) ? 1 : MT * 2;
  f32x4 lq[NL_F32];
  bf16x8 lh[NL_BF], ll[NL_BF];
  f32x4 tq[NT_F32];
  bf16x8 th[NT_BF], tl[NT_BF];
};

// Operand loads read the operand-ordered factor layouts (lop_*, ltop_*):
// one contiguous kilobyte per load instruction.
template <int PREC, int KP>
__device__ __forceinline__ void load_l(Ops<PREC, KP>& o, const DualArgs& a, int r0, int lane) {
  const int64_t rb = r0 >> 5;
  if constexpr (PREC == PREC_FP32) {
    const f32x4* lp = reinterpret_cast<const f32x4*>(a.L + rb * (KP / 8) * 256) + lane;
#pragma unroll
    for (int u = 0; u < KP / 8; ++u) o.lq[u] = lp[64 * u];
  } else {
    const bf16x8* lph = reinterpret_cast<const bf16x8*>(a.Lh + rb * (KP / 16) * 512) + lane;
    const bf16x8* lpl = reinterpret_cast<const bf16x8*>(a.Ll + rb * (KP / 16) * 512) + lane;
#pragma unroll
    for (int q = 0; q < KP / 16; ++q) {
      o.lh[q] = lph[64 * q];
      o.ll[q] = lpl[64 * q];
    }
  }
}

template <int PREC, int KP>
__device__ __forceinline__ void load_lt_tile(Ops<PREC, KP>& o, const DualArgs& a, int r0, int lane,
                                             int t) {
  constexpr int MT = KP / 32;
  const int64_t blk = (int64_t)(r0 >> 5) * MT + t;
  if constexpr (PREC == PREC_FP32) {
    const f32x4* lt = reinterpret_cast<const f32x4*>(a.LT + blk * 1024) + lane;
#pragma unroll
    for (int u = 0; u < 4; ++u) o.tq[4 * t + u] = lt[64 * u];
  } else {
    const bf16x8* lh = reinterpret_cast<const bf16x8*>(a.LTh + blk * 1024) + lane;
    const bf16x8* ll = reinterpret_cast<const bf16x8*>(a.LTl + blk * 1024) + lane;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      o.th[2 * t + q] = lh[64 * q];
      o.tl[2 * t + q] = ll[64 * q];
    }
  }
}

template <int PREC, int KP>
__device__ __forceinline__ void load_ops(Ops<PREC, KP>& o, const DualArgs& a, int r0, int lane) {
  load_l<PREC, KP>(o, a, r0, lane);
#pragma unroll
  for (int t = 0; t < KP / 32; ++t) load_lt_tile<PREC, KP>(o, a, r0, lane, t);
}

template <int PREC, int KP, int MODE, int NW, int PIPE, bool BIN>
__global__ __launch_bounds__(64 * NW, (KP <= 32 && PIPE <= 2) ? 2 : 1) void k_dual(DualArgs a) {
  static_assert(KP % 32 == 0, "KP must be a multiple of 32");
  constexpr int MT = KP / 32;  // 32-row tiles of the num/den outputs
  if (MODE != MODE_OBJ && a.stop_req && *a.stop_req) {
    // the stop test passed after an earlier iteration: nothing to do
    if (a.stop_seen && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *a.stop_seen = 1;
    return;
  }
  __shared__ float red[(NW > 1) ? (NW - 1) * 2 * 16 * 64 : 1];
  __shared__ double jred[NW];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int half = lane >> 5;
  // Workgroups are handed to the 8 XCDs round-robin in launch order; renumber
  // them so that each XCD runs one contiguous range of (split, tile) in
  // split-major order, and the workgroups that read the same rows of the
  // left factor share that XCD's L2 instead of each XCD fetching them.
  const int nb = gridDim.x * gridDim.y;
  const int lin = blockIdx.y * gridDim.x + blockIdx.x;
  const int per = nb >> 3, rem = nb & 7, xcd = lin & 7;
  const int lin2 = xcd * per + min(xcd, rem) + (lin >> 3);
  const int bx = lin2 % gridDim.x, by = lin2 / gridDim.x;
  const int tc = bx;
  const int c0 = tc * TILE;
  const int t_begin = by * a.tiles_per_split;
  const int t_end = min(t_begin + a.tiles_per_split, a.RT);

  // ---- right-factor tile, resident for the whole block ------------------
  // FP32: product step j uses reduction index half*KP/2 + j.
  // BF16: product step j uses reduction indices 16j + 8*half + e, e = 0..7.
  constexpr int NR_F32 = (PREC == PREC_FP32) ? KP / 2 : 1;
  constexpr int NR_BF = (PREC == PREC_FP32) ? 1 : KP / 16;
  float rt[NR_F32];
  bf16x8 rth[NR_BF], rtl[NR_BF];
  if constexpr (PREC == PREC_FP32) {
    const float* rp = a.Rt + (int64_t)(half * (KP / 2)) * a.ldr + c0 + col;
#pragma unroll
    for (int j = 0; j < KP / 2; ++j) rt[j] = rp[(int64_t)j * a.ldr];
  } else {
#pragma unroll
    for (int j = 0; j < KP / 16; ++j) {
      const float* rp = a.Rt + (int64_t)(16 * j + 8 * half) * a.ldr + c0 + col;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        __bf16 hi, lo;
        split_bf16(rp[(int64_t)e * a.ldr], hi, lo);
        rth[j][e] = hi;
        rtl[j][e] = lo;
      }
    }
  }

  f32x16 num[MT], den[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    num[t] = zero16();
    den[t] = zero16();
  }
  double jacc = 0.0;

  const int64_t tile_base = (int64_t)tc * a.RT;
  const float* dcol = a.D + tile_base * 1024 + lane * 4;
  const float* mcol = BIN ? nullptr : a.Mw + tile_base * 1024 + lane * 4;
  const uint16_t* bcol = BIN ? a.Mb + tile_base * 64 + lane : nullptr;
  using MK = MaskTile<BIN>;
  // PIPE 0: operands loaded at their use (large KP); PIPE 1: all operands of
  // a tile loaded at its start; PIPE 2: operands and data of the wave's next
  // tile loaded one tile ahead, so every wait covers loads issued a full
  // tile earlier; PIPE 3: as 2 with the data two tiles ahead.
  using O = Ops<PREC, KP>;
  constexpr int PFD = PIPE == 3 ? 2 : 1;  // data prefetch distance in tiles
  const auto ops_for = [&](O& o, int r0) { load_ops<PREC, KP>(o, a, r0, lane); };

  // One tile: consume (dv, mv, oc); prefetch the wave's next tile's data into
  // (dn, mn) and, with PIPE 2, its operands into on.
  auto step = [&](const int tr, const f32x4 (&dv)[4], const MK& mv, O& oc, f32x4 (&dn)[4], MK& mn,
                  O& on) {
    const int r0 = tr * TILE;
    // Unconditional (past the end a step re-reads its own tile) so that the
    // number of loads in flight is static and the waits below stay precise.
    const int trn = (tr + NW < t_end) ? tr + NW : tr;
    const int trd = (tr + PFD * NW < t_end) ? tr + PFD * NW : tr;
    if constexpr (PIPE >= 2) {
      ops_for(on, trn * TILE);
    } else if constexpr (PIPE == 1) {
      ops_for(oc, r0);
    }
    __builtin_amdgcn_sched_barrier(0);
    load_tile(dcol + (int64_t)trd * 1024, dn);
    mn.load(mcol, bcol, trd);
    __builtin_amdgcn_sched_barrier(0);

    // ---- Y = L[r0:r0+32, :] * Rt ------------------------------------------
    f32x16 y = zero16();
    if constexpr (PIPE == 0) load_l<PREC, KP>(oc, a, r0, lane);
    if constexpr (PREC == PREC_FP32) {
#pragma unroll
      for (int u = 0; u < KP / 8; ++u) {
        y = mfma_f32(oc.lq[u][0], rt[4 * u + 0], y);
        y = mfma_f32(oc.lq[u][1], rt[4 * u + 1], y);
        y = mfma_f32(oc.lq[u][2], rt[4 * u + 2], y);
        y = mfma_f32(oc.lq[u][3], rt[4 * u + 3], y);
      }
    } else {
#pragma unroll
      for (int j = 0; j < KP / 16; ++j) y = mfma_bf16x3(oc.lh[j], oc.ll[j], rth[j], rtl[j], y);
    }

    // ---- elementwise: A = Mw o D, Z = Mw o Y, J += Mw (D - Y)^2 ------------
    float av[16], zv[16];
    float js = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const float d = dv[i >> 2][i & 3];
      const float m = mv.get(i);
      // binary weights: the staged data is already 0 where the weight is
      av[i] = BIN ? d : m * d;
      zv[i] = m * y[i];
      if constexpr (MODE != MODE_SPLIT) {
        const float r = d - y[i];
        js = fmaf(m * r, r, js);
      }
    }
    if constexpr (MODE != MODE_SPLIT) jacc += (double)js;

    // ---- num += L^T A, den += L^T Z ----------------------------------------
    if constexpr (MODE != MODE_OBJ) {
      if constexpr (PREC == PREC_FP32) {
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          if constexpr (PIPE == 0) load_lt_tile<PREC, KP>(oc, a, r0, lane, t);
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            num[t] = mfma_f32(oc.tq[4 * t + (i >> 2)][i & 3], av[i], num[t]);
            den[t] = mfma_f32(oc.tq[4 * t + (i >> 2)][i & 3], zv[i], den[t]);
          }
        }
      } else {
        bf16x8 ah[2], al[2], zh[2], zl[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            __bf16 hi, lo;
            split_bf16(av[8 * j + e], hi, lo);
            ah[j][e] = hi;
            al[j][e] = lo;
            split_bf16(zv[8 * j + e], hi, lo);
            zh[j][e] = hi;
            zl[j][e] = lo;
          }
        }
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          if constexpr (PIPE == 0) load_lt_tile<PREC, KP>(oc, a, r0, lane, t);
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            num[t] = mfma_bf16x3(oc.th[2 * t + j], oc.tl[2 * t + j], ah[j], al[j], num[t]);
            den[t] = mfma_bf16x3(oc.th[2 * t + j], oc.tl[2 * t + j], zh[j], zl[j], den[t]);
          }
        }
      }
    }
  };

  int tr = t_begin + wave;
  if constexpr (PFD == 1) {
    f32x4 dA[4], dB[4];
    MK mA, mB;
    O oA, oB;
    if (tr < t_end) {
      if constexpr (PIPE >= 2) ops_for(oA, tr * TILE);
      load_tile(dcol + (int64_t)tr * 1024, dA);
      mA.load(mcol, bcol, tr);
    }
    for (; tr < t_end; tr += 2 * NW) {
      step(tr, dA, mA, oA, dB, mB, oB);
      if (tr + NW >= t_end) break;
      step(tr + NW, dB, mB, oB, dA, mA, oA);
    }
  } else {
    // data two tiles ahead: three data buffers, two operand sets
    f32x4 dA[4], dB[4], dC[4];
    MK mA, mB, mC;
    O oA, oB;
    if (tr < t_end) {
      ops_for(oA, tr * TILE);
      load_tile(dcol + (int64_t)tr * 1024, dA);
      mA.load(mcol, bcol, tr);
      const int t1 = (tr + NW < t_end) ? tr + NW : tr;
      load_tile(dcol + (int64_t)t1 * 1024, dB);
      mB.load(mcol, bcol, t1);
    }
    for (; tr < t_end; tr += 6 * NW) {
      step(tr, dA, mA, oA, dC, mC, oB);
      if (tr + NW >= t_end) break;
      step(tr + NW, dB, mB, oB, dA, mA, oA);
      if (tr + 2 * NW >= t_end) break;
      step(tr + 2 * NW, dC, mC, oA, dB, mB, oB);
      if (tr + 3 * NW >= t_end) break;
      step(tr + 3 * NW, dA, mA, oB, dC, mC, oA);
      if (tr + 4 * NW >= t_end) break;
      step(tr + 4 * NW, dB, mB, oA, dA, mA, oB);
      if (tr + 5 * NW >= t_end) break;
      step(tr + 5 * NW, dC, mC, oB, dB, mB, oA);
    }
  }

  // ---- combine the NW waves' sums in a fixed order -----------------------
  if constexpr (NW > 1 && MODE != MODE_OBJ) {
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      if (wave > 0) {
        float* dst = red + (wave - 1) * 2 * 1024;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          dst[i * 64 + lane] = num[t][i];
          dst[1024 + i * 64 + lane] = den[t][i];
        }
      }
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int w = 0; w < NW - 1; ++w) {
          const float* src = red + w * 2 * 1024;
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            num[t][i] += src[i * 64 + lane];
            den[t][i] += src[1024 + i * 64 + lane];
          }
        }
      }
      __syncthreads();
    }
  }
  if constexpr (MODE != MODE_SPLIT) {
    const double js = wave_sum(jacc);
    if (lane == 0) jred[wave] = js;
    __syncthreads();
    if (threadIdx.x == 0 && a.Jpart) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += jred[w];
      a.Jpart[lin2] = s;
    }
  }
  if constexpr (MODE == MODE_SPLIT) {
    if (wave != 0) return;
    float* pn = a.partial + (int64_t)by * 2 * KP * a.C_pad;
    float* pd = pn + (int64_t)KP * a.C_pad;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int k = 32 * t + acc_row(i, half);
        pn[(int64_t)k * a.C_pad + c0 + col] = num[t][i];
        pd[(int64_t)k * a.C_pad + c0 + col] = den[t][i];
      }
    }
  }

  if constexpr (MODE == MODE_UPDATE) {
    // Wave 0 applies the update and writes the KP x C layout (coalesced per
    // row); the new 32 x KP tile is staged in LDS so that all waves write
    // the operand-ordered copies the other half-step reads as contiguous
    // chunks (this tile's 32 columns own exactly one chunk of each).
    __shared__ float stage[32][KP + 1];
    if (wave == 0) {
      const int c = c0 + col;
      const bool cval = c < a.C_valid;
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        float old[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) old[i] = a.Rt[(int64_t)(32 * t + acc_row(i, half)) * a.ldr + c];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int k = 32 * t + acc_row(i, half);
          float nv = 0.f;
          if (cval && k < a.K) nv = mu_apply(old[i], num[t][i], den[t][i], a.eps);
          a.Rt_out[(int64_t)k * a.ldr + c] = nv;
          stage[col][k] = nv;
        }
      }
    }
    __syncthreads();
    const int64_t base = (int64_t)tc * 32 * KP;
    for (int o = threadIdx.x; o < 32 * KP; o += 64 * NW) {
      if constexpr (PREC == PREC_FP32) {
        {  // lop_f32 chunk: o = (u * 64 + lane) * 4 + j
          const int ln = (o >> 2) & 63, u = o >> 8, j = o & 3;
          const int k = (ln >> 5) * (KP / 2) + 4 * u + j;
          a.RtT[base + o] = stage[ln & 31][k];
        }
        {  // ltop_f32 chunk: o = ((t * 4 + g) * 64 + lane) * 4 + s
          const int t = o >> 10, g = (o >> 8) & 3, ln = (o >> 2) & 63, sx = o & 3;
          const int k = 32 * t + (ln & 31), x = 8 * g + 4 * (ln >> 5) + sx;
          a.Rtp[base + o] = stage[x][k];
        }
      } else {
        __bf16 hi, lo;
        {  // lop_bf16 chunk: o = (q * 64 + lane) * 8 + e
          const int q = o >> 9, ln = (o >> 3) & 63, e = o & 7;
          const int k = 16 * q + 8 * (ln >> 5) + e;
          split_bf16(stage[ln & 31][k], hi, lo);
          a.RtTh[base + o] = hi;
          a.RtTl[base + o] = lo;
        }
        {  // ltop_bf16 chunk: o = ((t * 2 + q) * 64 + lane) * 8 + e
          const int t = o >> 10, q = (o >> 9) & 1, ln = (o >> 3) & 63, e = o & 7;
          const int k = 32 * t + (ln & 31);
          const int x = 16 * q + 8 * (e >> 2) + 4 * (ln >> 5) + (e & 3);
          split_bf16(stage[x][k], hi, lo);
          a.Rtph[base + o] = hi;
          a.Rtpl[base + o] = lo;
        }
      }
    }
  }
}

template <int PREC, int KP, int MODE, int PIPE, bool BIN>
static hipError_t launch_bin(int nw, const DualArgs& a, dim3 g, hipStream_t s) {
  switch (nw) {
    case 1: hipLaunchKernelGGL((k_dual<PREC, KP, MODE, 1, PIPE, BIN>), g, dim3(64), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_dual<PREC, KP, MODE, 2, PIPE, BIN>), g, dim3(128), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_dual<PREC, KP, MODE, 4, PIPE, BIN>), g, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC, int KP, int MODE, int PIPE>
static hipError_t launch_nw(int nw, const DualArgs& a, dim3 g, hipStream_t s) {
  return a.Mb ? launch_bin<PREC, KP, MODE, PIPE, true>(nw, a, g, s)
              : launch_bin<PREC, KP, MODE, PIPE, false>(nw, a, g, s);
}

template <int PREC, int KP, int MODE>
static hipError_t launch_mode(int nw, int pipe, const DualArgs& a, dim3 g, hipStream_t s) {
  if constexpr (KP <= 64) {
    if (pipe == 3) return launch_nw<PREC, KP, MODE, 3>(nw, a, g, s);
    if (pipe == 2) return launch_nw<PREC, KP, MODE, 2>(nw, a, g, s);
    return launch_nw<PREC, KP, MODE, 1>(nw, a, g, s);
  } else {
    return launch_nw<PREC, KP, MODE, 0>(nw, a, g, s);
  }
}

template <int PREC, int KP>
static hipError_t launch_kp(int mode, int nw, int pipe, const DualArgs& a, dim3 g, hipStream_t s) {
  switch (mode) {
    case MODE_UPDATE: return launch_mode<PREC, KP, MODE_UPDATE>(nw, pipe, a, g, s);
    case MODE_SPLIT: return launch_mode<PREC, KP, MODE_SPLIT>(nw, pipe, a, g, s);
    default: return launch_mode<PREC, KP, MODE_OBJ>(nw, pipe, a, g, s);
  }
}

template <int PREC>
static hipError_t launch_prec(int kp, int mode, int nw, int pipe, const DualArgs& a, dim3 g,
                              hipStream_t s) {
  switch (kp) {
    case 32: return launch_kp<PREC, 32>(mode, nw, pipe, a, g, s);
    case 64: return launch_kp<PREC, 64>(mode, nw, pipe, a, g, s);
    case 96: return launch_kp<PREC, 96>(mode, nw, pipe, a, g, s);
    case 128: return launch_kp<PREC, 128>(mode, nw, pipe, a, g, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_dual(int prec, int kp, int mode, int nw, int pipe, const DualArgs& a, int grid_x,
                       int grid_y, hipStream_t s) {
  const dim3 g(grid_x, grid_y);
  if (prec == PREC_FP32) return launch_prec<PREC_FP32>(kp, mode, nw, pipe, a, g, s);
  return launch_prec<PREC_BF16X3>(kp, mode, nw, pipe, a, g, s);
}

}  // namespace nmf
