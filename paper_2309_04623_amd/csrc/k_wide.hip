// Fused multiplicative-update half-step (Eq. 3 of arXiv:2309.04623) for
// wide bases (padded component count KP >= 96) on gfx950.
//
// The arithmetic is the one of k_dual (Y = L Rt in MFMA registers, the
// weights, the residual term of Eq. 2 and num/den = L^T (Mw o D), L^T (Mw o Y)
// fed straight from the Y accumulators), but the work is laid out for a
// left factor whose operand set no longer fits a single wave's loads:
//
//   * a workgroup of four waves owns four adjacent 32-column tiles, one per
//     wave, and walks the 32-row tiles of its row chunk in order;
//   * the operand set of each row tile (its rows of L in the Y-operand order
//     and the permuted L^T block in the num/den-operand order, KP * 256
//     bytes in FP32 or as bf16 hi/lo pairs) is fetched ONCE per workgroup
//     and shared through LDS;
//   * every fetch is an LDS DMA (global_load_lds_dwordx4: each lane's 16
//     bytes land in LDS without passing through registers), issued one row
//     tile ahead into the other half of a double buffer, or, with bit-mask
//     weights at KP = 128, two row tiles ahead into three buffers (the
//     weight bits then travel by DMA too): the operand set by all waves, the
//     data (and weight) tile of each wave's column into that wave's own
//     slot.  The only wait is the one before the barrier that closes each
//     row tile, so the fetches overlap whole tiles of MFMA work and cost no
//     registers;
//   * each wave keeps its column tile's right-factor operands and its
//     num/den accumulators (2 * KP / 32 MFMA tiles) in registers (one wave
//     per SIMD).
// Compared with one workgroup per column tile this divides the L2 traffic
// of the left factor by four.  Reductions keep a fixed order (each wave sums
// its row tiles in order; the waves' objective terms are added in wave
// order), so results are bitwise reproducible.

#include "device_common.hpp"
#include "kernels.hpp"

namespace nmf {

constexpr int WIDE_NW = 4;  // waves (column tiles) per workgroup

// LDS layout (bytes): [NB operand sets of KP * 256][per wave: NB data tiles
// of 4 KB][per wave: NB weight tiles of 4 KB, FP32 weights when they fit, or
// NB bit tiles of 128 bytes in the three-buffer form], NB = 3 for the
// cross-tile pipelined loop (KP <= 96) and the three-buffer form, else 2.
// The update epilogue reuses the space from 0 to stage each wave's new
// 32 x KP tile.
constexpr int LDS_MAX = 160 * 1024 - 256;  // dynamic part (the static part holds 32 bytes)
template <int KP>
__host__ __device__ constexpr bool wide_xp() {
  return KP <= 96 && 3 * KP * 256 + WIDE_NW * 3 * 4096 <= LDS_MAX;
}
// Split-precision tiles without the cross-tile pipeline take three buffers
// when they fit: fetches run two row tiles ahead.
template <int KP, bool BIN>
__host__ __device__ constexpr bool wide_tb() {
  return BIN && !wide_xp<KP>() && 3 * KP * 256 + WIDE_NW * 3 * (4096 + 128) <= LDS_MAX;
}
template <int KP, bool BIN>
__host__ __device__ constexpr int wide_nbuf() {
  return (wide_xp<KP>() || wide_tb<KP, BIN>()) ? 3 : 2;
}
template <int KP, bool BIN>
__host__ __device__ constexpr int wide_ops_bytes() {
  return wide_nbuf<KP, BIN>() * KP * 256;
}
template <int KP, bool BIN>
__host__ __device__ constexpr int wide_slot_bytes() {  // data (or weight) slots of all waves
  return WIDE_NW * wide_nbuf<KP, BIN>() * 4096;
}
// FP32 weight tiles go through LDS when they fit; otherwise they are loaded
// into registers one step ahead.
template <int KP, bool BIN>
__host__ __device__ constexpr bool wide_mw_dma() {
  return !BIN && wide_ops_bytes<KP, BIN>() + 2 * wide_slot_bytes<KP, BIN>() <= LDS_MAX;
}
template <int KP, bool BIN>
__host__ __device__ constexpr int wide_lds_bytes() {
  return wide_ops_bytes<KP, BIN>() + wide_slot_bytes<KP, BIN>() * (wide_mw_dma<KP, BIN>() ? 2 : 1) +
         (wide_tb<KP, BIN>() ? WIDE_NW * 3 * 128 : 0);
}
template <int KP>
__host__ __device__ constexpr int wide_stage_bytes() {
  return WIDE_NW * 32 * (KP + 1) * 4;
}

// One LDS DMA of 16 bytes per lane: lane i's bytes land at lds + 16 i.
__device__ __forceinline__ void dma16(const void* src, unsigned char* lds) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}
// The same for data read once per launch: streamed (non-temporal), so it
// does not displace the operand sets every workgroup re-reads from L2.
__device__ __forceinline__ void dma16_stream(const void* src, unsigned char* lds) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds, 16, 0,
                                   2 /* nt */);
}
// The same with 4 bytes per lane: lane i's bytes land at lds + 4 i.
__device__ __forceinline__ void dma4(const void* src, unsigned char* lds) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds, 4, 0, 0);
}

// Places a register value at this point of the instruction stream: it is
// computed before this point and, used as an input, not hoisted above it
// (an empty statement on one register: no instruction, no memory access).
template <class T>
__device__ __forceinline__ void pin(T& x) {
  asm volatile("" : "+v"(x));
}

template <int PREC, int KP, int MODE, bool BIN>
__global__ __launch_bounds__(64 * WIDE_NW, 1) void k_wide(DualArgs a) {
  static_assert(KP % 32 == 0 && KP >= 64, "wide kernel needs KP a multiple of 32, >= 64");
  static_assert(wide_lds_bytes<KP, BIN>() <= LDS_MAX && wide_stage_bytes<KP>() <= LDS_MAX,
                "LDS budget");
  constexpr int MT = KP / 32;
  constexpr int NV = KP * 16;                     // 16-byte vectors per operand set
  constexpr int PT = NV / (64 * WIDE_NW);         // per thread
  constexpr int NCH = PREC == PREC_FP32 ? 2 : 4;  // contiguous source chunks
  constexpr int CV = NV / NCH;                    // vectors per chunk
  constexpr int ESZ = PREC == PREC_FP32 ? 4 : 2;  // bytes per element
  constexpr int OPS = KP * 256;                   // bytes per operand set
  constexpr int NBUF = wide_nbuf<KP, BIN>();      // operand / data buffers
  constexpr bool XP = wide_xp<KP>();              // cross-tile pipelined loop
  constexpr int DATA0 = wide_ops_bytes<KP, BIN>();  // data slots
  constexpr int MW0 = DATA0 + wide_slot_bytes<KP, BIN>();  // weight slots (FP32 weights)
  constexpr bool MWD = wide_mw_dma<KP, BIN>();
  // operand reads pinned one MFMA group ahead of their use (beyond KP = 128
  // the pinned order runs out of registers and the compiler's order is kept)
  constexpr bool RA = KP <= 128;
  if (MODE != MODE_OBJ && a.stop_req && *a.stop_req) {
    if (a.stop_seen && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *a.stop_seen = 1;
    return;
  }
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double jred[WIDE_NW];
  const int tid = threadIdx.x;
  // wave index as a uniform (scalar) value, so that everything derived from
  // it (column tile, fetch chunk, base addresses) lives in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int col = lane & 31;
  const int half = lane >> 5;
  // XCD-aware renumbering (launch order is dealt round-robin over the 8
  // XCDs): each XCD runs a contiguous range of (chunk, group) in chunk-major
  // order, so the workgroups reading the same rows of L share its L2.
  const int nb = gridDim.x * gridDim.y;
  const int lin = blockIdx.y * gridDim.x + blockIdx.x;
  const int per = nb >> 3, rem = nb & 7, xcd = lin & 7;
  const int lin2 = xcd * per + min(xcd, rem) + (lin >> 3);
  const int bx = lin2 % gridDim.x, by = lin2 / gridDim.x;
  const int ncol = a.C_pad >> 5;
  const int tc = bx * WIDE_NW + wave;
  const bool active = tc < ncol;
  // a wave past the last column tile shadows the last one (results unused)
  const int c0 = (active ? tc : ncol - 1) * TILE;
  const int t_begin = by * a.tiles_per_split;
  const int t_end = min(t_begin + a.tiles_per_split, a.RT);

  // ---- operand-set fetch ----------------------------------------------------
  // Wave w fetches chunk w (bf16: L hi, L lo, L^T hi, L^T lo) or half of
  // chunk w / 2 (FP32: L, L^T), so its source array is wave-uniform; every
  // chunk of row block rb starts at element rb * KP * 32 of its array.
  constexpr int LS = 64 * WIDE_NW / NCH;  // lanes fetching one chunk
  static_assert(CV % LS == 0 && CV / LS == PT, "operand chunk split");
  const int chunk = (wave * NCH) / WIDE_NW;
  const int cl0 = (wave - chunk * (WIDE_NW / NCH)) * 64;  // first vector of this wave
  const unsigned char* csrc;
  if constexpr (PREC == PREC_FP32) {
    csrc = reinterpret_cast<const unsigned char*>(chunk == 0 ? a.L : a.LT);
  } else {
    const __bf16* p = chunk == 0 ? a.Lh : chunk == 1 ? a.Ll : chunk == 2 ? a.LTh : a.LTl;
    csrc = reinterpret_cast<const unsigned char*>(p);
  }
  // addresses are a uniform base plus a 32-bit lane offset (scalar base
  // registers, one vector register per address)
  const uint32_t lofs = (uint32_t)lane * 16;
  auto fetch_ops = [&](int rb, int buf) {
    const unsigned char* src = csrc + (int64_t)rb * KP * 32 * ESZ + cl0 * 16;
    unsigned char* dst = smem + buf * OPS + (chunk * CV + cl0) * 16;
#pragma unroll
    for (int u = 0; u < PT; ++u) dma16(src + (lofs + LS * 16 * u), dst + LS * 16 * u);
  };

  // ---- right-factor operands of this wave's column tile (resident) --------
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

  // ---- data tiles of this wave's column -------------------------------------
  // A tile is 4 KB in MFMA accumulator order (lane l's 16 values at bytes
  // [u * 1024 + 16 l, +16), u < 4): four DMAs land it in the wave's slot in
  // the same order.  Binary weights (16 bits per lane) come by a plain load.
  const int64_t tile_base = (int64_t)(c0 >> 5) * a.RT;
  const unsigned char* dcol = reinterpret_cast<const unsigned char*>(a.D + tile_base * 1024);
  const unsigned char* mcol =
      BIN ? nullptr : reinterpret_cast<const unsigned char*>(a.Mw + tile_base * 1024);
  const unsigned char* bcol =
      BIN ? reinterpret_cast<const unsigned char*>(a.Mb + tile_base * 64) : nullptr;
  auto load_bits = [&](int tr) -> uint32_t {
    return __builtin_nontemporal_load(
        reinterpret_cast<const uint16_t*>(bcol + (int64_t)tr * 128 + (uint32_t)lane * 2));
  };
  unsigned char* dslot = smem + DATA0 + wave * NBUF * 4096;
  unsigned char* mslot = smem + MW0 + wave * NBUF * 4096;
  auto fetch_data = [&](int tr, int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      dma16_stream(dcol + (int64_t)tr * 4096 + (lofs + u * 1024), dslot + buf * 4096 + u * 1024);
    if constexpr (MWD) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        dma16_stream(mcol + (int64_t)tr * 4096 + (lofs + u * 1024), mslot + buf * 4096 + u * 1024);
    }
  };
  // weights through registers (when their LDS slots do not fit)
  auto load_w = [&](int tr, f32x4(&w)[4]) {
    if constexpr (!BIN && !MWD) {
      const f32x4* q = reinterpret_cast<const f32x4*>(mcol + (int64_t)tr * 4096 + lofs);
#pragma unroll
      for (int u = 0; u < 4; ++u) w[u] = __builtin_nontemporal_load(q + 64 * u);
    }
  };

  // The work of one 32 x 32 tile of this wave's column, in three parts:
  //   y_part:    Y = L Rt on MFMA from the L operands in operand buffer ``ob``;
  //   elem_part: weights, residual term and the num/den B operands
  //              (A = Mw o D, Z = Mw o Y, split into bf16 hi/lo for the
  //              split-precision products) from the data in slot ``db``;
  //   nd_part:   num += L^T A, den += L^T Z from the L^T operands in ``ob``.
  // Operand reads from LDS run one MFMA group ahead of their use; the
  // num/den products are interleaved over all output tiles.
  constexpr int NB = PREC == PREC_FP32 ? 16 : 4;  // registers of the B operands
  struct BOps {
    float a[PREC == PREC_FP32 ? 16 : 1], z[PREC == PREC_FP32 ? 16 : 1];
    bf16x8 ah[2], al[2], zh[2], zl[2];
  };
  auto y_part = [&](int ob) -> f32x16 {
    const unsigned char* base = smem + ob * OPS;
    f32x16 y0 = zero16();
    if constexpr (PREC == PREC_FP32) {
      const f32x4* L = reinterpret_cast<const f32x4*>(base) + lane;
      constexpr int NU = KP / 8;
      f32x4 cq = L[0];
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        f32x4 nq = cq;
        if (u + 1 < NU) nq = L[64 * (u + 1)];
        if constexpr (RA && !XP) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < 4; ++j) y0 = mfma_f32(cq[j], rt[4 * u + j], y0);
        if constexpr (RA && !XP) __builtin_amdgcn_sched_barrier(0);
        cq = nq;
      }
    } else {
      const bf16x8* Lh = reinterpret_cast<const bf16x8*>(base) + lane;
      const bf16x8* Ll = Lh + CV;
      constexpr int NQ = KP / 16;
      bf16x8 ch = Lh[0], cl = Ll[0];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        bf16x8 nh = ch, nl = cl;
        if (q + 1 < NQ) {
          nh = Lh[64 * (q + 1)];
          nl = Ll[64 * (q + 1)];
        }
        if constexpr (RA && !XP) __builtin_amdgcn_sched_barrier(0);
        y0 = mfma_bf16x3(ch, cl, rth[q], rtl[q], y0);  // the small terms first
        if constexpr (RA && !XP) __builtin_amdgcn_sched_barrier(0);
        ch = nh;
        cl = nl;
      }
    }
    return y0;
  };
  auto elem_part = [&](const f32x16& y, int db, uint32_t mb, const f32x4(&wr)[4], BOps& B) {
    const f32x4* dp = reinterpret_cast<const f32x4*>(dslot + db * 4096) + lane;
    const f32x4* mp = reinterpret_cast<const f32x4*>(mslot + db * 4096) + lane;
    f32x4 dv[4], mv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      dv[u] = dp[64 * u];
      if constexpr (MWD) mv[u] = mp[64 * u];
      else if constexpr (!BIN) mv[u] = wr[u];
    }
    float av[16], zv[16];
    float js = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const float d = dv[i >> 2][i & 3];
      // the residual term in every mode: the split pass reports it too when
      // asked (and without it the compiler's register allocation of the
      // split kernel spills)
      const float r = d - y[i];
      if constexpr (BIN) {
        // weight bit i as an all-ones / all-zeros mask (one bit-field
        // extract): masking by AND gives exactly 1 * x or +0 (x >= 0 for y)
        const int mk = (int)(mb << (31 - i)) >> 31;
        av[i] = d;  // the staged data is already 0 where the weight is
        zv[i] = __int_as_float(__float_as_int(y[i]) & mk);
        const float rm = __int_as_float(__float_as_int(r) & mk);
        js = fmaf(rm, rm, js);
      } else {
        const float m = mv[i >> 2][i & 3];
        av[i] = m * d;
        zv[i] = m * y[i];
        js = fmaf(m * r, r, js);
      }
    }
    jacc += (double)js;
    if constexpr (MODE == MODE_OBJ) return;
    if constexpr (PREC == PREC_FP32) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        B.a[i] = av[i];
        B.z[i] = zv[i];
      }
    } else {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        split8_bf16(av + 8 * j, B.ah[j], B.al[j]);
        split8_bf16(zv + 8 * j, B.zh[j], B.zl[j]);
      }
    }
  };
  auto nd_part = [&](int ob, const BOps& B) {
    if constexpr (MODE == MODE_OBJ) return;
    const unsigned char* base = smem + ob * OPS;
    if constexpr (PREC == PREC_FP32) {
      const f32x4* LT = reinterpret_cast<const f32x4*>(base) + CV + lane;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        f32x4 tq[MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) tq[t] = LT[64 * (4 * t + u)];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            num[t] = mfma_f32(tq[t][j], B.a[4 * u + j], num[t]);
            den[t] = mfma_f32(tq[t][j], B.z[4 * u + j], den[t]);
          }
        }
      }
    } else {
      const bf16x8* LTh = reinterpret_cast<const bf16x8*>(base) + 2 * CV + lane;
      const bf16x8* LTl = LTh + CV;
      // per accumulator the order is the split-precision one (lo*hi, hi*lo,
      // then hi*hi), over the two 16-row halves in turn
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        bf16x8 th[MT], tl[MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          th[t] = LTh[64 * (2 * t + q)];
          tl[t] = LTl[64 * (2 * t + q)];
        }
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          num[t] = mfma_bf16(tl[t], B.ah[q], num[t]);
          den[t] = mfma_bf16(tl[t], B.zh[q], den[t]);
        }
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          num[t] = mfma_bf16(th[t], B.al[q], num[t]);
          den[t] = mfma_bf16(th[t], B.zl[q], den[t]);
        }
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          num[t] = mfma_bf16(th[t], B.ah[q], num[t]);
          den[t] = mfma_bf16(th[t], B.zh[q], den[t]);
        }
      }
    }
  };
  // Split-precision tile in an explicit instruction order, so that the
  // vector work sits between independent matrix products (one wave per
  // SIMD cannot hide it otherwise):
  //   (1) Y = L Rt, operand reads two product groups ahead, with the RNE
  //       split of A = Mw o D into bf16 hi/lo spread over the groups;
  //   (2) num of rows 0-15 (lane half 0 of the reduction) beside Z = Mw o Y,
  //       the objective terms and the split of Z for rows 0-15;
  //   (3) den of rows 0-15 beside the same for rows 16-31;
  //   (4) num, then den, of rows 16-31.
  // Every accumulator receives its products in the order of the plain form
  // and the objective terms are summed in element order (with bit-mask
  // weights the results are the same bits); a weighted product is rounded
  // to FP32 before it is split.  ``issue(s)`` is called at the start of
  // product group s (s < KP / 16 + 3 * KP / 32) so that a caller can spread
  // its memory fetches over the tile.
  auto compute_x4 = [&](int buf, uint32_t mb, const f32x4(&wr)[4], auto&& issue) {
    constexpr int NQ = KP / 16;
    const unsigned char* base = smem + buf * OPS;
    const f32x4* dp = reinterpret_cast<const f32x4*>(dslot + buf * 4096) + lane;
    const f32x4* mp = reinterpret_cast<const f32x4*>(mslot + buf * 4096) + lane;
    const bf16x8* Lh = reinterpret_cast<const bf16x8*>(base) + lane;
    const bf16x8* Ll = Lh + CV;
    const bf16x8* LTh = Lh + 2 * CV;
    const bf16x8* LTl = Lh + 3 * CV;
    bf16x8 lh[NQ], ll[NQ];
    f32x4 dq[4], wq[4];
    lh[0] = Lh[0];
    ll[0] = Ll[0];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      dq[u] = dp[64 * u];
      if constexpr (MWD) wq[u] = mp[64 * u];
      else if constexpr (!BIN) wq[u] = wr[u];
    }
    lh[1] = Lh[64];
    ll[1] = Ll[64];
    __builtin_amdgcn_sched_barrier(0);
    float dv[16], mv[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      dv[i] = dq[i >> 2][i & 3];
      mv[i] = BIN ? 1.f : wq[i >> 2][i & 3];
    }
    uint32_t ahp[8], alp[8], zhp[8], zlp[8];
    auto split2 = [](float x0, float x1, uint32_t& hi, uint32_t& lo) {
      const f32x2 v = {x0, x1};
      const bf16x2 h = __builtin_convertvector(v, bf16x2);
      const bf16x2 l = __builtin_convertvector(v - __builtin_convertvector(h, f32x2), bf16x2);
      hi = __builtin_bit_cast(uint32_t, h);
      lo = __builtin_bit_cast(uint32_t, l);
    };
    auto pack = [](const uint32_t* p) {
      typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
      const u32x4 v = {p[0], p[1], p[2], p[3]};
      return __builtin_bit_cast(bf16x8, v);
    };
    bf16x8 th[MT], tl[MT];
    // (1)
    f32x16 y = zero16();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (q + 2 < NQ) {
        lh[q + 2] = Lh[64 * (q + 2)];
        ll[q + 2] = Ll[64 * (q + 2)];
      }
      if (q == NQ - 2) {  // the num/den operands of rows 0-15
#pragma unroll
        for (int t = 0; t < MT; ++t) tl[t] = LTl[64 * (2 * t)];
      }
      if (q == NQ - 1) {
#pragma unroll
        for (int t = 0; t < MT; ++t) th[t] = LTh[64 * (2 * t)];
      }
      issue(q);
      y = mfma_bf16(ll[q], rth[q], y);
      y = mfma_bf16(lh[q], rtl[q], y);
      y = mfma_bf16(lh[q], rth[q], y);
#pragma unroll
      for (int pr = (8 * q) / NQ; pr < (8 * (q + 1)) / NQ; ++pr) {
        float x0 = dv[2 * pr], x1 = dv[2 * pr + 1];
        pin(x0);
        pin(x1);
        split2(__fmul_rn(mv[2 * pr], x0), __fmul_rn(mv[2 * pr + 1], x1), ahp[pr], alp[pr]);
        pin(ahp[pr]);
        pin(alp[pr]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    const bf16x8 ah0 = pack(ahp), al0 = pack(alp), ah1 = pack(ahp + 4), al1 = pack(alp + 4);
    float js = 0.f;
    float zv[16];
    auto elem = [&](int i) {
      float yi = y[i];
      pin(yi);
      const float r = dv[i] - yi;
      if constexpr (BIN) {
        const int mk = (int)(mb << (31 - i)) >> 31;
        zv[i] = __int_as_float(__float_as_int(yi) & mk);
        const float rm = __int_as_float(__float_as_int(r) & mk);
        js = fmaf(rm, rm, js);
      } else {
        zv[i] = __fmul_rn(mv[i], yi);
        js = fmaf(mv[i] * r, r, js);
      }
      pin(zv[i]);
      pin(js);
    };
    auto zsplit = [&](int i, int k) {
      float z0 = zv[i], z1 = zv[i + 1];
      pin(z0);
      pin(z1);
      split2(z0, z1, zhp[k], zlp[k]);
      pin(zhp[k]);
      pin(zlp[k]);
    };
    // (2) num, rows 0-15; element work 0-7 (one element or one pair split
    // per product)
#pragma unroll
    for (int m = 0; m < 3 * MT; ++m) {
      const int t = m % MT, s = m / MT;
      issue(NQ + m);
      if (s == 0) num[t] = mfma_bf16(tl[t], ah0, num[t]);
      else if (s == 1) num[t] = mfma_bf16(th[t], al0, num[t]);
      else num[t] = mfma_bf16(th[t], ah0, num[t]);
      if (m < 8) elem(m);
      else if (m < 12) zsplit(2 * (m - 8), m - 8);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (3 * MT < 12) {  // MT < 4: the rest of the element work of rows 0-15
#pragma unroll
      for (int m = 3 * MT; m < 12; ++m) {
        if (m < 8) elem(m);
        else zsplit(2 * (m - 8), m - 8);
      }
    }
    const bf16x8 zh0 = pack(zhp), zl0 = pack(zlp);
    // (3) den, rows 0-15; element work 8-15, and the operands of rows 16-31
#pragma unroll
    for (int m = 0; m < 3 * MT; ++m) {
      const int t = m % MT, s = m / MT;
      if (s == 0) den[t] = mfma_bf16(tl[t], zh0, den[t]);
      else if (s == 1) den[t] = mfma_bf16(th[t], zl0, den[t]);
      else den[t] = mfma_bf16(th[t], zh0, den[t]);
      if (m < 8) elem(8 + m);
      else if (m < 12) zsplit(8 + 2 * (m - 8), 4 + m - 8);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (3 * MT < 12) {
#pragma unroll
      for (int m = 3 * MT; m < 12; ++m) {
        if (m < 8) elem(8 + m);
        else zsplit(8 + 2 * (m - 8), 4 + m - 8);
      }
    }
    jacc += (double)js;
    const bf16x8 zh1 = pack(zhp + 4), zl1 = pack(zlp + 4);
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      tl[t] = LTl[64 * (2 * t + 1)];
      th[t] = LTh[64 * (2 * t + 1)];
    }
    // (4) rows 16-31
#pragma unroll
    for (int t = 0; t < MT; ++t) num[t] = mfma_bf16(tl[t], ah1, num[t]);
#pragma unroll
    for (int t = 0; t < MT; ++t) den[t] = mfma_bf16(tl[t], zh1, den[t]);
#pragma unroll
    for (int t = 0; t < MT; ++t) num[t] = mfma_bf16(th[t], al1, num[t]);
#pragma unroll
    for (int t = 0; t < MT; ++t) den[t] = mfma_bf16(th[t], zl1, den[t]);
#pragma unroll
    for (int t = 0; t < MT; ++t) num[t] = mfma_bf16(th[t], ah1, num[t]);
#pragma unroll
    for (int t = 0; t < MT; ++t) den[t] = mfma_bf16(th[t], zh1, den[t]);
  };
  auto compute = [&](int buf, uint32_t mb, const f32x4(&wr)[4]) {
    if constexpr (PREC == PREC_BF16X3 && MODE != MODE_OBJ && KP <= 128) {
      compute_x4(buf, mb, wr, [](int) {});
      return;
    }
    const f32x16 y = y_part(buf);
    if constexpr (RA) __builtin_amdgcn_sched_barrier(0);
    BOps B;
    elem_part(y, buf, mb, wr, B);
    if constexpr (RA) __builtin_amdgcn_sched_barrier(0);
    nd_part(buf, B);
  };

  // ---- main loop over the row tiles of the chunk ---------------------------
  // Every step issues the same fetches (past the end of the chunk they
  // re-read its last tile into an unused buffer; a wave without a column
  // tile computes on the group's last one and discards the result).  The
  // compiler waits for the DMAs before each barrier.
  uint32_t bA = 0, bB = 0, bC = 0;
  f32x4 wA[4], wB[4], wC[4];
  int tr = t_begin;
  if constexpr (XP) {
    // Cross-tile pipeline over three buffers: step r computes Y of tile r+1
    // (its operands arrived a step earlier) while the vector units finish
    // tile r (elementwise part, from the Y computed in step r-1), then the
    // num/den products of tile r; the fetches of step r bring the operands
    // of tile r+2 and the data of tile r+1.  A wave thus always has MFMA
    // work independent of its vector work.
    f32x16 y;
    if (tr < t_end) {
      fetch_ops(tr, 0);
      fetch_ops(min(tr + 1, t_end - 1), 1);
      fetch_data(tr, 0);
      load_w(tr, wA);
      if constexpr (BIN) bA = load_bits(tr);
      __syncthreads();
      y = y_part(0);
    }
    auto step = [&](int r, int o0, int o1, int o2, uint32_t mb, const f32x4(&wr)[4],
                    uint32_t& mbn, f32x4(&wrn)[4]) {
      const int nd = min(r + 1, t_end - 1), no = min(r + 2, t_end - 1);
      fetch_ops(no, o2);
      fetch_data(nd, o1);
      load_w(nd, wrn);
      if constexpr (BIN) mbn = load_bits(nd);
      __builtin_amdgcn_sched_barrier(0);  // issue the fetches before the tile's work
      const f32x16 yn = y_part(o1);
      BOps B;
      elem_part(y, o0, mb, wr, B);
      nd_part(o0, B);
      y = yn;
      // instruction order of the step: Y's operand reads one product group
      // ahead, each product group followed by a share of the vector work,
      // then the num/den products with their reads
      if constexpr (PREC == PREC_BF16X3) {
        constexpr int NQ = KP / 16;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);  // DS reads
          __builtin_amdgcn_sched_group_barrier(0x008, 3, 0);  // MFMA
          __builtin_amdgcn_sched_group_barrier(0x002, 20, 0);  // VALU
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          __builtin_amdgcn_sched_group_barrier(0x100, 2 * MT, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 6 * MT, 0);
        }
      }
      __syncthreads();
    };
    for (; tr < t_end; tr += 3) {
      step(tr, 0, 1, 2, bA, wA, bB, wB);
      if (tr + 1 >= t_end) break;
      step(tr + 1, 1, 2, 0, bB, wB, bC, wC);
      if (tr + 2 >= t_end) break;
      step(tr + 2, 2, 0, 1, bC, wC, bA, wA);
    }
  } else if constexpr (NBUF == 3) {
    // Operand sets, data tiles and weight bits are fetched two row tiles
    // ahead into three buffers.  The barrier closing step r waits only
    // until the fetches of tile r + 2 (issued at the start of step r) are
    // the ones in flight (memory loads complete in issue order), so
    // everything tile r + 1 needs has landed.  The buffer they fill was last
    // read in step r - 1, which every wave has left.
    constexpr int NV_STEP = PT + 5;
    static_assert(BIN && NV_STEP < 64, "three buffers take bit-mask weights");
    // s_waitcnt: vmcnt <= NV_STEP, lgkmcnt 0, expcnt untouched
    constexpr int WAIT_PREV = (NV_STEP & 15) | (7 << 4) | (0 << 8) | ((NV_STEP >> 4) << 14);
    auto close_step = [&]() {
      __builtin_amdgcn_s_waitcnt(WAIT_PREV);
      __builtin_amdgcn_s_barrier();
    };
    unsigned char* bslot = smem + DATA0 + wide_slot_bytes<KP, BIN>() + wave * 3 * 128;
    auto fetch_bits = [&](int t, int buf) {
      if (lane < 32) dma4(bcol + (int64_t)t * 128 + lofs / 4, bslot + buf * 128);
    };
    const f32x4 wnone[4] = {};
    if (tr < t_end) {
      const int n1 = min(tr + 1, t_end - 1);
      fetch_ops(tr, 0);
      fetch_data(tr, 0);
      fetch_bits(tr, 0);
      fetch_ops(n1, 1);
      fetch_data(n1, 1);
      fetch_bits(n1, 1);
    }
    close_step();
    int cur = 0;
    for (; tr < t_end; ++tr) {
      const int n2 = min(tr + 2, t_end - 1), buf2 = cur == 0 ? 2 : cur - 1;
      const uint32_t mb = *reinterpret_cast<const uint16_t*>(bslot + cur * 128 + lane * 2);
      if constexpr (PREC == PREC_BF16X3 && MODE != MODE_OBJ && KP <= 128) {
        // the fetches of tile r + 2 spread over the tile's products, one
        // load per product group, so that the memory pipeline never backs
        // up into the instruction stream
        const unsigned char* osrc = csrc + (int64_t)n2 * KP * 32 * ESZ + cl0 * 16;
        unsigned char* odst = smem + buf2 * OPS + (chunk * CV + cl0) * 16;
        compute_x4(cur, mb, wnone, [&](int piece) {
          if (piece < PT) {
            dma16(osrc + (lofs + LS * 16 * piece), odst + LS * 16 * piece);
          } else if (piece < PT + 4) {
            const int u = piece - PT;
            dma16_stream(dcol + (int64_t)n2 * 4096 + (lofs + u * 1024),
                         dslot + buf2 * 4096 + u * 1024);
          } else if (piece == PT + 4) {
            fetch_bits(n2, buf2);
          }
        });
      } else {
        fetch_ops(n2, buf2);
        fetch_data(n2, buf2);
        fetch_bits(n2, buf2);
        __builtin_amdgcn_sched_barrier(0);
        compute(cur, mb, wnone);
      }
      close_step();
      cur = cur == 2 ? 0 : cur + 1;
    }
    // the fetches still in flight land in buffers the epilogue reuses
    __syncthreads();
  } else {
    if (tr < t_end) {
      fetch_ops(tr, 0);
      fetch_data(tr, 0);
      load_w(tr, wA);
      if constexpr (BIN) bA = load_bits(tr);
    }
    __syncthreads();
    // Two row tiles per trip: the buffer indices are compile-time constants.
    for (; tr < t_end; tr += 2) {
      const int n1 = min(tr + 1, t_end - 1);
      fetch_ops(n1, 1);
      fetch_data(n1, 1);
      load_w(n1, wB);
      if constexpr (BIN) bB = load_bits(n1);
      __builtin_amdgcn_sched_barrier(0);  // issue the fetches before the tile's work
      compute(0, bA, wA);
      __syncthreads();
      if (tr + 1 >= t_end) break;
      const int n2 = min(tr + 2, t_end - 1);
      fetch_ops(n2, 0);
      fetch_data(n2, 0);
      load_w(n2, wA);
      if constexpr (BIN) bA = load_bits(n2);
      __builtin_amdgcn_sched_barrier(0);
      compute(1, bB, wB);
      __syncthreads();
    }
  }
  if (!active) jacc = 0.0;

  {
    const double js = wave_sum(jacc);
    if (lane == 0) jred[wave] = js;
    __syncthreads();
    if (tid == 0 && a.Jpart) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < WIDE_NW; ++w) s += jred[w];
      a.Jpart[lin2] = s;
    }
  }
  if constexpr (MODE == MODE_SPLIT) {
    if (!active) return;
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
    // Each wave applies the update to its tile, writes the KP x C layout,
    // and stages the new 32 x KP tile in LDS (free after the loop's last
    // barrier) to write the operand-ordered copies the other half-step
    // reads as contiguous chunks.
    float* stage = reinterpret_cast<float*>(smem) + wave * 32 * (KP + 1);
    if (active) {
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
          stage[col * (KP + 1) + k] = nv;
        }
      }
    }
    __syncthreads();
    if (!active) return;
    const int64_t base = (int64_t)tc * 32 * KP;
    for (int o = lane; o < 32 * KP; o += 64) {
      if constexpr (PREC == PREC_FP32) {
        {  // lop_f32 chunk: o = (u * 64 + ln) * 4 + j
          const int ln = (o >> 2) & 63, u = o >> 8, j = o & 3;
          const int k = (ln >> 5) * (KP / 2) + 4 * u + j;
          a.RtT[base + o] = stage[(ln & 31) * (KP + 1) + k];
        }
        {  // ltop_f32 chunk: o = ((t * 4 + g) * 64 + ln) * 4 + s
          const int t = o >> 10, g = (o >> 8) & 3, ln = (o >> 2) & 63, sx = o & 3;
          const int k = 32 * t + (ln & 31), x = 8 * g + 4 * (ln >> 5) + sx;
          a.Rtp[base + o] = stage[x * (KP + 1) + k];
        }
      } else {
        __bf16 hi, lo;
        {  // lop_bf16 chunk: o = (q * 64 + ln) * 8 + e
          const int q = o >> 9, ln = (o >> 3) & 63, e = o & 7;
          const int k = 16 * q + 8 * (ln >> 5) + e;
          split_bf16(stage[(ln & 31) * (KP + 1) + k], hi, lo);
          a.RtTh[base + o] = hi;
          a.RtTl[base + o] = lo;
        }
        {  // ltop_bf16 chunk: o = ((t * 2 + q) * 64 + ln) * 8 + e
          const int t = o >> 10, q = (o >> 9) & 1, ln = (o >> 3) & 63, e = o & 7;
          const int k = 32 * t + (ln & 31);
          const int x = 16 * q + 8 * (e >> 2) + 4 * (ln >> 5) + (e & 3);
          split_bf16(stage[x * (KP + 1) + k], hi, lo);
          a.Rtph[base + o] = hi;
          a.Rtpl[base + o] = lo;
        }
      }
    }
  }
}

template <int PREC, int KP, int MODE, bool BIN>
static hipError_t wide_go(const DualArgs& a, dim3 g, hipStream_t s) {
  constexpr int l1 = wide_lds_bytes<KP, BIN>();
  constexpr int l2 = MODE == MODE_UPDATE ? wide_stage_bytes<KP>() : 0;
  constexpr int lds = l1 > l2 ? l1 : l2;
  auto fn = k_wide<PREC, KP, MODE, BIN>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, g, dim3(64 * WIDE_NW), lds, s, a);
  return hipGetLastError();
}

template <int PREC, int KP>
static hipError_t wide_kp(int mode, const DualArgs& a, dim3 g, hipStream_t s) {
  const bool bin = a.Mb != nullptr;
  switch (mode) {
    case MODE_UPDATE:
      return bin ? wide_go<PREC, KP, MODE_UPDATE, true>(a, g, s)
                 : wide_go<PREC, KP, MODE_UPDATE, false>(a, g, s);
    case MODE_SPLIT:
      return bin ? wide_go<PREC, KP, MODE_SPLIT, true>(a, g, s)
                 : wide_go<PREC, KP, MODE_SPLIT, false>(a, g, s);
    default:
      return bin ? wide_go<PREC, KP, MODE_OBJ, true>(a, g, s)
                 : wide_go<PREC, KP, MODE_OBJ, false>(a, g, s);
  }
}

template <int PREC>
static hipError_t wide_prec(int kp, int mode, const DualArgs& a, dim3 g, hipStream_t s) {
  switch (kp) {
    case 96: return wide_kp<PREC, 96>(mode, a, g, s);
    case 128: return wide_kp<PREC, 128>(mode, a, g, s);
    case 160: return wide_kp<PREC, 160>(mode, a, g, s);
    case 192: return wide_kp<PREC, 192>(mode, a, g, s);
    case 224: return wide_kp<PREC, 224>(mode, a, g, s);
    default: return hipErrorInvalidValue;
  }
}

int wide_groups(int col_tiles) { return (col_tiles + WIDE_NW - 1) / WIDE_NW; }

hipError_t launch_wide(int prec, int kp, int mode, const DualArgs& a, int grid_y, hipStream_t s) {
  const dim3 g(wide_groups(a.C_pad / TILE), grid_y);
  if (prec == PREC_FP32) return wide_prec<PREC_FP32>(kp, mode, a, g, s);
  return wide_prec<PREC_BF16X3>(kp, mode, a, g, s);
}

}  // namespace nmf
