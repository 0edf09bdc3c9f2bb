// Target modelling through per-frame masked Gram matrices (Sec. 4.1 with
// the W-rule of Eq. 3 and H fixed), one persistent launch for all frames.
//
// For a frame with pixels S, weights m and data t the W-rule denominator
// [m o (c H)] H^T equals c G with G = H diag(m) H^T (exact re-association),
// and the numerator is the constant b = H (m o t).  Each workgroup takes
// frames from a device queue; per frame it
//   1. streams the frame's pixels in chunks of 32, staging the gathered rows
//      of H^T (K values per pixel), m and t in LDS, and accumulates the
//      upper-triangle 32x32 tiles of G on MFMA (tiles spread over the
//      waves) and b on the vector units (FP64 sums, each component's pixels
//      split over the groups of threads that fit the workgroup);
//   2. for K <= 128 hands G, b and the start to k_gram_iter (below), which
//      iterates several frames per compute unit with a row of G per lane;
//      for larger K writes G to LDS and runs all iterations
//      c_j <- max(c_j b_j / (c G)_j, eps) itself, with c in LDS.
// Pixels appear only through the staged chunks, so dense frames (all
// pixels, weight row of M_T) and CSR frames share the kernel.
//
// G tiles take FP32 products (v_mfma_f32_32x32x2_f32 on the staged rows,
// (H o m) H^T) or split-precision ones: G = (H o sqrt m)(H o sqrt m)^T, the
// chunk's H o sqrt m staged transposed (component rows, pixels along the
// row) as one bf16 hi/lo pair that serves both operands, so that every
// operand of v_mfma_f32_32x32x16_bf16 is one 16-byte LDS read; each tile
// then takes two reduction steps of three products per chunk.  The same
// staging pass adds the chunk's b terms (h m) t in FP64.

#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"

namespace nmf {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// One LDS DMA of 16 bytes per lane: lane i's bytes land at lds + 16 i.
__device__ __forceinline__ void gram_dma16(const void* src, float* lds) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}
// The same with 4 bytes per lane: lane i's bytes land at lds + 4 i.
__device__ __forceinline__ void gram_dma4(const void* src, float* lds) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds, 4, 0, 0);
}

template <int KP>
__host__ __device__ constexpr int gram_tiles() {
  return (KP / 32) * (KP / 32 + 1) / 2;
}

// Upper-triangle tile index -> (mi, mj), row-major over mi <= mj.
__device__ __forceinline__ void tile_of(int idx, int nb, int& mi, int& mj) {
  mi = 0;
  while (idx >= nb - mi) {
    idx -= nb - mi;
    ++mi;
  }
  mj = mi + idx;
}

template <int KP>
__host__ __device__ constexpr int gram_waves() {
  return KP <= 128 ? 4 : 8;
}

// How the split form spreads the tiles of G over the waves so that a wave
// reads each 32-component block of the staged operand once per reduction
// step and uses it for several tiles (the staged array is both operands):
//   1 (4 or 3 blocks, four waves): wave w takes blocks p = w, q = w + 1,
//     r = w + 2 (mod NB) and the tiles (p,p), (p,q) and, for NB = 4 and
//     w < 2, (p,r); three waves for NB = 3;
//   2 (7 blocks, eight waves): wave w < 7 takes the blocks of the line
//     {w, w + 1, w + 3} (mod 7) of the Fano plane, whose seven lines hold
//     every pair of blocks exactly once, and the tiles (w,w+1), (w,w+3),
//     (w+1,w+3) and, for w < 4, (w,w); wave 7 takes the blocks 4, 5, 6 and
//     their diagonal tiles, so each SIMD (waves w and w + 4) has seven;
//   0: tile t to wave t mod NWV, each tile reading both its operands.
template <int KP, int PREC>
__host__ __device__ constexpr int gram_pattern() {
  return PREC != PREC_BF16X3 ? 0 : (KP == 96 || KP == 128) ? 1 : KP == 224 ? 2 : 0;
}

// Transposed bf16 staging: a row per component, 16 dwords (32 pixels) used
// of GT_STRIDE (the pad keeps the per-lane 16-byte reads conflict-free).
constexpr int GT_STRIDE = 20;

// Rows of each staged bf16 array: KP, or for KP > 128 only K (components
// K.. are never staged: the tiles that read past row K land in rows and
// columns of G that are never used, and stay inside the allocation, which
// holds at least 4 KP floats after the staging area).
__host__ __device__ constexpr int gram_staged_rows(int K, int KP) { return KP <= 128 ? KP : K; }

// LDS floats of the pixel loop with rows gathered PF chunks ahead of their
// first use: gathered rows [PF+1][32][KP], rings of pixel indices, weights
// and square-rooted weights [PF+2][32] each, the raw pixel indices, weights
// and data as fetched [2][3][32], a ring of the FP64 products m t
// [PF+2][32], and (bf16x3) two transposed hi/lo pairs [2][2][rows][GT_STRIDE]
__host__ __device__ constexpr int gram_stage_floats(int K, int KP, int prec, int pf) {
  return 32 * (pf + 1) * KP + 96 * (pf + 2) + 192 + 64 * (pf + 2) +
         (prec == PREC_BF16X3 ? 4 * gram_staged_rows(K, KP) * GT_STRIDE : 0);
}

template <int KP, bool RAGGED, int PREC, bool FORM, int PF>
__global__ __launch_bounds__(64 * gram_waves<KP>()) void k_gram(GramArgs a) {
  static_assert(PF == 1 || PF == 2, "rows gathered one or two chunks ahead");
  static_assert(!FORM || KP <= 128, "the two-phase form keeps a row of G per lane");
  static_assert(FORM || KP > 128, "K <= 128 iterates in k_gram_iter");
  extern __shared__ __align__(16) float lds[];
  __shared__ int qslot;
  __shared__ double wsel[2][gram_waves<KP>()];
  constexpr int NB = KP / 32;
  constexpr int NT = gram_tiles<KP>();
  constexpr int NWV = gram_waves<KP>();
  constexpr int NTH = 64 * NWV;
  constexpr int GP = gram_pattern<KP, PREC>();
  constexpr int TPW = GP == 1 ? (NB == 4 ? 3 : 2) : GP == 2 ? 4 : (NT + NWV - 1) / NWV;
  // blocks of a pattern tile: slot s multiplies block LA[s] by block LB[s]
  constexpr int LA[4] = {0, 0, 0, 1};
  constexpr int LB[4] = {0, 1, 2, 2};
  constexpr int KQ = KP / 4;
  constexpr int FOLD = 8;  // chunks summed in FP32 before folding into FP64
  // b = H (m o t) on groups of KP threads, thread (bgrp, bcomp) summing
  // component bcomp over its group's pixels of each chunk: FP32 form, BG
  // groups of BPX consecutive pixels; split form, SG groups that take every
  // SG-th group of eight pixels in the staging pass
  constexpr int BG = NTH / KP >= 8 ? 8 : NTH / KP >= 4 ? 4 : NTH / KP >= 2 ? 2 : 1;
  constexpr int BPX = 32 / BG;
  constexpr int SG = NTH / KP < 4 ? NTH / KP : 4;
  constexpr int NBG = PREC == PREC_BF16X3 ? SG : BG;
  const int K = a.K;
  // PF: chunks gathered ahead of their first use; LEAD: chunks staged ahead
  // of the one multiplied (split form); GA: chunks gathered ahead of the one
  // multiplied
  constexpr int LEAD = PREC == PREC_BF16X3 ? 1 : 0, GA = PF + LEAD;
  // ring slots: chunks c + LEAD .. c + GA + 1 are live while chunk c is
  // multiplied (the split form no longer needs chunk c's)
  constexpr int NH = PF + 1, NM = GA + 2 - LEAD;
  // [NH][32][KP] gathered H^T rows (the chunk in use and the next PF)
  float* Hsb = lds;
  // rings of NM chunks' pixel indices, weights and square roots of the
  // weights ([NM][32] each)
  int* pixr = reinterpret_cast<int*>(lds + 32 * NH * KP);
  float* msr = lds + 32 * NH * KP + 32 * NM;
  float* qsr = msr + 32 * NM;
  // two chunks' raw pixel indices, weights and data, as fetched ([2][3][32])
  float* rawr = qsr + 32 * NM;
  // ring of the pixels' m t in FP64 (exact products of the two floats)
  double* mtr = reinterpret_cast<double*>(rawr + 192);
  // two buffers of bf16 hi/lo of (H o sqrt m)^T, [2][2][rows][GT_STRIDE]
  // dwords (2 pixels each)
  uint32_t* wT = reinterpret_cast<uint32_t*>(mtr + 32 * NM);
  const int WB = gram_staged_rows(K, KP) * GT_STRIDE;  // dwords of one hi or lo array
  float* G = lds;             // [K][K] after the pixel loop (aliases the above)
  const int goff = (max(K * K, gram_stage_floats(K, KP, PREC, PF)) + 3) & ~3;
  double* bsh = reinterpret_cast<double*>(lds + goff);  // [KP]
  float* csh = reinterpret_cast<float*>(bsh + KP);      // [KP]

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int col = lane & 31, half = lane >> 5;
  const int bgrp = tid / KP, bcomp = tid - bgrp * KP;
  int tmi[TPW], tmj[TPW];
  int blk[3] = {0, 0, 0};  // the wave's blocks (patterns 1 and 2)
  int bused = 0;           // which of them its tiles read
  bool diag3 = false;      // pattern 2, wave 7: the tiles (4,4), (5,5), (6,6)
  if constexpr (GP == 0) {
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int idx = wave + NWV * q;
      if (idx < NT) {
        tile_of(idx, NB, tmi[q], tmj[q]);
      } else {
        tmi[q] = -1;
        tmj[q] = -1;
      }
    }
  } else {
    static_assert(GP != 1 || (NWV == 4 && (NB == 3 || NB == 4)), "row pattern");
    static_assert(GP != 2 || (NWV == 8 && NB == 7), "Fano pattern");
    int ntl;
    if constexpr (GP == 1) {
      blk[0] = wave;
      blk[1] = (wave + 1) % NB;
      blk[2] = (wave + 2) % NB;
      ntl = NB == 4 ? (wave < 2 ? 3 : 2) : (wave < 3 ? 2 : 0);
    } else {
      blk[0] = wave < 7 ? wave : 4;
      blk[1] = wave < 7 ? (wave + 1) % 7 : 5;
      blk[2] = wave < 7 ? (wave + 3) % 7 : 6;
      ntl = wave < 7 ? 4 : 0;
      diag3 = wave == 7;
    }
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      tmi[q] = q < ntl ? blk[LA[q]] : -1;
      tmj[q] = q < ntl ? blk[LB[q]] : -1;
    }
    if constexpr (GP == 2) {
      // waves 4-6 leave their diagonal tile to wave 7, which has no line:
      // seven tiles per SIMD (waves w and w + 4 share one)
      if (wave >= 4 && wave < 7) tmi[0] = tmj[0] = -1;
      if (diag3) {
        tmi[0] = tmj[0] = 4;
        tmi[1] = tmj[1] = 5;
        tmi[2] = tmj[2] = 6;
      }
    }
#pragma unroll
    for (int q = 0; q < TPW; ++q)
      if (tmi[q] >= 0) bused |= diag3 ? 1 << q : (1 << LA[q]) | (1 << LB[q]);
  }
  const uint64_t key = sm_key(a.seed, 2);
  int bad = 0;

  while (true) {
    if (tid == 0) qslot = atomicAdd(a.queue, 1);
    __syncthreads();
    const int qi = qslot;
    __syncthreads();
    if (qi >= a.F) break;
    const int f = a.order ? a.order[qi] : qi;
    const uint64_t tick0 = wall_clock64();
    if (a.visits && tid == 0) atomicAdd(a.visits + f, 1);

    int64_t s = 0, e = a.P;
    if constexpr (RAGGED) {
      s = a.offsets[f];
      e = a.offsets[f + 1];
      if (!(s >= 0 && s <= e && e <= a.nnz)) {
        bad |= 16;
        s = e = 0;
      }
    }

    // Totals: FP64 when they fit the register file (KP <= 160), else FP32.
    constexpr bool TOT64 = KP <= 160;
    using tot_t = typename std::conditional<TOT64, double, float>::type;
    f32x16 acc[TPW];
    tot_t tot[TPW][16];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      acc[q] = zero16();
#pragma unroll
      for (int r = 0; r < 16; ++r) tot[q][r] = 0;
    }
    auto fold = [&]() {
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[q][r] += (tot_t)acc[q][r];
        acc[q] = zero16();
      }
    };
    double bacc = 0.0;
    int nfold = 0;

    // Pixel chunks of 32 in a software pipeline: while the tiles of chunk c
    // are multiplied, the split form stages chunk c + 1 (into the other
    // buffer), the rows of H^T of chunk c + GA are gathered by LDS DMA (one
    // 16-byte piece per lane, no registers), the raw pixel indices, weights
    // and data of chunk c + GA + 2 are fetched by LDS DMA too, and those of
    // chunk c + GA + 1 (fetched one chunk earlier) are checked into the ring.
    // Each chunk ends with one barrier; with PF = 2 a wave waits there for
    // its older DMAs only (vmcnt of the pieces it issued this chunk, first
    // used two chunks later, stay in flight).  A pixel outside the frame or
    // with an invalid index gathers row 0 (finite) under weight 0, so it
    // adds exactly nothing.
    // The pixel data of a chunk are fetched and checked by lanes 0-31 of the
    // last wave (the meta lanes), the wave with the fewest tiles and no
    // staging share at K > 128.
    const bool mw = wave == NWV - 1 && lane < 32;
    const int ml = lane;
    int mp = 0;
    float mm = 0.f, mt = 0.f;
    auto meta_load = [&](int64_t b0) {  // meta lanes: chunk at b0
      const int64_t jj = b0 + ml;
      mp = -1;
      mm = 0.f;
      mt = 0.f;
      if (jj < e) {
        if constexpr (RAGGED) {
          mp = a.pix[jj];
          mm = a.wt ? a.wt[jj] : 1.0f;
          mt = a.val[jj];
        } else {
          mp = (int)jj;
          mm = a.MT[(int64_t)f * a.P + jj];
          mt = a.T[(int64_t)f * a.P + jj];
        }
      }
    };
    auto meta_fetch = [&](int rs, int64_t b0) {  // meta lanes: chunk at b0, by DMA
      const int64_t jj = min(b0 + ml, e - 1);  // lanes past the frame: any valid entry
      float* rw = rawr + 96 * rs;
      if constexpr (RAGGED) {
        gram_dma4(a.pix + jj, rw);
        if (a.wt) gram_dma4(a.wt + jj, rw + 32);
        gram_dma4(a.val + jj, rw + 64);
      } else {
        gram_dma4(a.MT + (int64_t)f * a.P + jj, rw + 32);
        gram_dma4(a.T + (int64_t)f * a.P + jj, rw + 64);
      }
    };
    auto meta_take = [&](int rs, int64_t b0) {  // meta lanes: fetched values
      const int64_t jj = b0 + ml;
      const float* rw = rawr + 96 * rs;
      mp = -1;
      mm = 0.f;
      mt = 0.f;
      if (jj < e) {
        if constexpr (RAGGED) {
          mp = __builtin_bit_cast(int, rw[ml]);
          mm = a.wt ? rw[32 + ml] : 1.0f;
        } else {
          mp = (int)jj;
          mm = rw[32 + ml];
        }
        mt = rw[64 + ml];
      }
    };
    auto meta_store = [&](int slot, int64_t b0) {  // meta lanes: validated
      const int64_t jj = b0 + ml;
      float m = 0.f, t = 0.f;
      int prow = 0;
      if (jj < e) {
        m = mm;
        t = mt;
        prow = mp;
        if (RAGGED && (prow < 0 || prow >= a.P)) {
          bad |= 16;
          m = 0.f;
          prow = 0;
        }
        if (!(m >= 0.f) || isinf(m)) {
          bad |= 4;
          m = 0.f;
        }
        if (a.binary) m = m > 0.f ? 1.f : 0.f;
        if (m > 0.f) {
          if (!isfinite(t)) {
            bad |= 1;
            t = 0.f;
          } else if (t < 0.f) {
            if (a.clip_negative) {
              m = 0.f;
              t = 0.f;
            } else {
              bad |= 2;
            }
          }
        } else {
          t = 0.f;
        }
      }
      pixr[32 * slot + ml] = prow;
      msr[32 * slot + ml] = m;
      qsr[32 * slot + ml] = sqrtf(m);
      mtr[32 * slot + ml] = (double)m * (double)t;
    };
    auto gather = [&](int slot, float* dst) {  // all waves: 32 rows of H^T
#pragma unroll
      for (int i = wave; i < KQ / 2; i += NWV) {
        const int x = 64 * i + lane, jr = x / KQ, kq = x - jr * KQ;
        gram_dma16(a.HT + lop_f32(pixr[32 * slot + jr], 4 * kq, KP), dst + 256 * i);
      }
    };
    // DMA instructions a wave issues per chunk: at least NDMA
    constexpr int NDMA = (KQ / 2) / NWV;
    static_assert(NDMA >= 1 && NDMA < 64, "gather instructions per wave");
    // barrier that leaves this wave's newest n VMEM operations in flight
    // (LDS operations all complete); the empty asm statements keep the
    // compiler from moving memory accesses across it
    auto barrier_vm = [](auto n) {
      constexpr int v = decltype(n)::value;
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_waitcnt((v & 15) | (7 << 4) | (0 << 8) | ((v >> 4) << 14));
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
    };
    // split form: transposed staging of w = h sqrt(m) of one chunk into
    // buffer wb, thread (bgrp, bcomp) -> component bcomp, pixels 8 q .. 8 q
    // + 7 for q = bgrp, bgrp + SG, ... < 4: the reads of Hs are consecutive
    // across threads, each thread writes its four pixel pairs of hi and of
    // lo as one 16-byte word (the row stride keeps those conflict-free, as
    // for the operand reads); the same pass adds the chunk's b terms
    auto stage = [&](const float* Hsrc, int slot, int wb) {
      const float* qsl = qsr + 32 * slot;
      const double* mtl = mtr + 32 * slot;
      uint32_t* dhi = wT + wb * 2 * WB;
      uint32_t* dlo = dhi + WB;
      // components K.. are not staged (see gram_staged_rows)
      if (bgrp < SG && bcomp < K) {
        for (int q = bgrp; q < 4; q += SG) {
          float h[8], qv[8];
          double mt[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) h[u] = Hsrc[(8 * q + u) * KP + bcomp];
#pragma unroll
          for (int u4 = 0; u4 < 2; ++u4) {
            const f32x4 q4 = *reinterpret_cast<const f32x4*>(qsl + 8 * q + 4 * u4);
#pragma unroll
            for (int u = 0; u < 4; ++u) qv[4 * u4 + u] = q4[u];
          }
#pragma unroll
          for (int u2 = 0; u2 < 4; ++u2) {
            const f64x2 m2 = *reinterpret_cast<const f64x2*>(mtl + 8 * q + 2 * u2);
            mt[2 * u2] = m2[0];
            mt[2 * u2 + 1] = m2[1];
          }
          u32x4 hi4, lo4;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const f32x2 wv = {h[2 * v] * qv[2 * v], h[2 * v + 1] * qv[2 * v + 1]};
            const bf16x2 wh = __builtin_convertvector(wv, bf16x2);
            const bf16x2 wl = __builtin_convertvector(wv - __builtin_convertvector(wh, f32x2), bf16x2);
            hi4[v] = __builtin_bit_cast(uint32_t, wh);
            lo4[v] = __builtin_bit_cast(uint32_t, wl);
          }
          const int o = bcomp * GT_STRIDE + 4 * q;
          *reinterpret_cast<u32x4*>(dhi + o) = hi4;
          *reinterpret_cast<u32x4*>(dlo + o) = lo4;
#pragma unroll
          for (int u = 0; u < 8; ++u) bacc = fma((double)h[u], mt[u], bacc);
        }
      }
    };
    if (s < e) {
      if (mw) {
#pragma unroll
        for (int x = 0; x <= GA; ++x) {
          meta_load(s + 32 * x);
          meta_store(x, s + 32 * x);
        }
        if (s + 32 * (GA + 1) < e) meta_fetch((GA + 1) & 1, s + 32 * (GA + 1));
      }
      __syncthreads();
#pragma unroll
      for (int x = 0; x < GA; ++x)
        if (s + 32 * x < e) gather(x, Hsb + x * 32 * KP);
      __syncthreads();
      if constexpr (LEAD == 1) {
        stage(Hsb, 0, 0);
        __syncthreads();
      }
    }
    int c = 0;
    for (int64_t base = s; base < e; base += 32, ++c) {
      const int sl = c % NM;
      const float* Hs = Hsb + (c % NH) * 32 * KP;
      const float* ms = msr + 32 * sl;
      // chunk c + GA + 2's pixel data (before the gather: older DMAs land
      // first)
      if (mw && base + 32 * (GA + 2) < e) meta_fetch((c + GA) & 1, base + 32 * (GA + 2));
      const bool ahead = base + 32 * GA < e;
      if (ahead) gather((c + GA) % NM, Hsb + ((c + GA) % NH) * 32 * KP);

      // ---- G tiles: G[mi-block, mj-block] += (H o m) H^T over the chunk ---
      auto tiles = [&]() {
        if constexpr (GP != 0) {
          // each of the wave's blocks read once per reduction step
          const uint32_t* whi = wT + (c & 1) * 2 * WB;
          const uint32_t* wlo = whi + WB;
#pragma unroll
          for (int ks = 0; ks < 2; ++ks) {
            const int d = 8 * ks + 4 * half;
            bf16x8 bh[3], bl[3];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
              const bool used = (bused >> l) & 1;
              const int r = (32 * blk[l] + col) * GT_STRIDE + d;
              bh[l] = used ? *reinterpret_cast<const bf16x8*>(whi + r) : bf16x8{};
              bl[l] = used ? *reinterpret_cast<const bf16x8*>(wlo + r) : bf16x8{};
            }
            if (GP == 2 && diag3) {
#pragma unroll
              for (int q = 0; q < 3; ++q) acc[q] = mfma_bf16x3(bh[q], bl[q], bh[q], bl[q], acc[q]);
            } else {
#pragma unroll
              for (int q = 0; q < TPW; ++q)
                if (tmi[q] >= 0)
                  acc[q] = mfma_bf16x3(bh[LA[q]], bl[LA[q]], bh[LB[q]], bl[LB[q]], acc[q]);
            }
          }
          return;
        }
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
          if (tmi[q] >= 0) {
            if constexpr (PREC == PREC_BF16X3 && GP == 0) {
              // reduction step ks covers pixels 16 ks .. 16 ks + 15; lane
              // half h holds pixels 16 ks + 8 h .. + 7 (dwords 8 ks + 4 h ..)
              const uint32_t* whi = wT + (c & 1) * 2 * WB;
              const uint32_t* wlo = whi + WB;
              const int ra = (32 * tmi[q] + col) * GT_STRIDE, rb = (32 * tmj[q] + col) * GT_STRIDE;
#pragma unroll
              for (int ks = 0; ks < 2; ++ks) {
                const int d = 8 * ks + 4 * half;
                const bf16x8 ah = *reinterpret_cast<const bf16x8*>(whi + ra + d);
                const bf16x8 al = *reinterpret_cast<const bf16x8*>(wlo + ra + d);
                const bf16x8 bh = *reinterpret_cast<const bf16x8*>(whi + rb + d);
                const bf16x8 bl = *reinterpret_cast<const bf16x8*>(wlo + rb + d);
                acc[q] = mfma_bf16x3(ah, al, bh, bl, acc[q]);
              }
            } else {
              const float* ha = Hs + 32 * tmi[q] + col;
              const float* hb = Hs + 32 * tmj[q] + col;
#pragma unroll
              for (int u = 0; u < 16; ++u) {
                const int jr = 2 * u + half;
                acc[q] = mfma_f32(ha[jr * KP] * ms[jr], hb[jr * KP], acc[q]);
              }
            }
          }
        }
      };
      if constexpr (PREC == PREC_BF16X3) {
        // the two waves of a SIMD (wave w and w + 4 of eight) take the two
        // parts in opposite orders, so one multiplies while the other stages
        const bool next = base + 32 < e;
        if (NWV == 8 && (wave & 4)) {
          if (next) stage(Hsb + ((c + 1) % NH) * 32 * KP, (c + 1) % NM, (c + 1) & 1);
          tiles();
        } else {
          tiles();
          if (next) stage(Hsb + ((c + 1) % NH) * 32 * KP, (c + 1) % NM, (c + 1) & 1);
        }
      } else {
        tiles();
        // ---- b += H (m o t), FP32 form: thread (bgrp, bcomp) sums pixels
        // bgrp*BPX .. bgrp*BPX + BPX - 1 ------------------------------------
        if (bgrp < BG && bcomp < K) {
#pragma unroll
          for (int u = 0; u < BPX; ++u) {
            const int jr = bgrp * BPX + u;
            bacc = fma((double)Hs[jr * KP + bcomp], mtr[32 * sl + jr], bacc);
          }
        }
      }
      // Two-level sum: FOLD chunks in the FP32 MFMA accumulators, then into
      // FP64 totals (G entries are sums of up to P_f / 2 positive terms).
      if (++nfold == FOLD) {
        nfold = 0;
        fold();
      }
      if (mw) {
        meta_take((c + GA + 1) & 1, base + 32 * (GA + 1));
        meta_store((c + GA + 1) % NM, base + 32 * (GA + 1));
      }
      // the rows used next chunk landed (every wave's); with PF = 2 those
      // gathered this chunk stay in flight
      if (PF == 2 && ahead)
        barrier_vm(std::integral_constant<int, NDMA>{});
      else
        barrier_vm(std::integral_constant<int, 0>{});
    }
    fold();
    // b: the groups' partial sums in group order (bsh is not aliased by the
    // staging area, so this needs no barrier before it)
#pragma unroll
    for (int gi = 0; gi < NBG; ++gi) {
      if (bgrp == gi) bsh[bcomp] = bcomp < K ? (gi == 0 ? bacc : bsh[bcomp] + bacc) : 0.0;
      if (NBG > 1) __syncthreads();
    }

    // ---- G to LDS (both triangles), b and the starting coefficients -------
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      if (tmi[q] >= 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 32 * tmi[q] + acc_row(r, half);
          const int cg = 32 * tmj[q] + col;
          if (row < K && cg < K) {
            const float v = (float)tot[q][r];
            G[row * K + cg] = v;
            if (tmi[q] != tmj[q]) G[cg * K + row] = v;
          }
        }
      }
    }
    if (tid < KP) {
      float c0 = 0.f;
      if (tid < K) {
        c0 = a.C_init ? a.C_init[(int64_t)f * K + tid] : sm_uniform(key, (uint64_t)f * K + tid);
        // a warm start is clamped to the floor (a zero would never move)
        if (a.warm) c0 = fmaxf(c0, a.eps);
      }
      csh[tid] = c0;
    }
    __syncthreads();

    bool warm_kept = false;  // the same in every thread
    if (a.warm) {
      // Warm start with fallback: the supplied coefficients are kept only if
      // their objective is not above that of the seeded cold start (the two
      // are compared as c G c^T - 2 b c^T; the frame's constant cancels).
      double qw = 0.0, qc = 0.0;
      if (tid < K) {
        double gw = 0.0, gc = 0.0;
        for (int i = 0; i < K; ++i) {
          const double g = G[tid * K + i];
          gw += g * (double)csh[i];
          gc += g * (double)sm_uniform(key, (uint64_t)f * K + i);
        }
        const double cw = csh[tid], cc = sm_uniform(key, (uint64_t)f * K + tid);
        qw = cw * (gw - 2.0 * bsh[tid]);
        qc = cc * (gc - 2.0 * bsh[tid]);
      }
      qw = wave_sum(qw);
      qc = wave_sum(qc);
      if (lane == 0) {
        wsel[0][wave] = qw;
        wsel[1][wave] = qc;
      }
      __syncthreads();
      double sw = 0.0, sc = 0.0;
#pragma unroll
      for (int w = 0; w < NWV; ++w) {
        sw += wsel[0][w];
        sc += wsel[1][w];
      }
      const bool keep = sw <= sc;  // false for a non-finite warm objective
      warm_kept = keep;
      if (!keep && tid < K) csh[tid] = sm_uniform(key, (uint64_t)f * K + tid);
      if (a.fallback && tid == 0) a.fallback[f] = keep ? 0 : 1;
      __syncthreads();
    }

    if constexpr (FORM) {
      // hand G, b and the start over to the iterating launch
      float* Go = a.Gf + (int64_t)f * K * K;
      for (int x = tid; x < K * K; x += NTH) Go[x] = G[x];
      if (tid < KP) {
        a.bf[(int64_t)f * KP + tid] = bsh[tid];
        a.cf[(int64_t)f * KP + tid] = csh[tid];
      }
      if (a.ticks && tid == 0) a.ticks[2 * (int64_t)f] = tick0;
      __syncthreads();  // LDS is reused by the next frame
      continue;
    }

    if constexpr (!FORM) {
      // ---- iterations (K > 128): (c G)_j, half a row of G per thread -----
      // Two threads, j and j + 256, share row j of the product: each keeps
      // KP/2 entries of row j of G (G is symmetric: row j is column j) in
      // registers and sums that half of the components, the upper one
      // leaves its sum in LDS for the lower one, which owns coefficient j.
      // Optional per-frame stop rule: every
      // check_every iterations the model change since the previous check,
      // d = c - c_prev, is tested against the model, d G d^T <= tol^2 c G c^T
      // (both in FP64; c G is the denominator just formed, d G one more
      // product).  A warm-started frame that has not met the rule by the cap
      // restarts from the cold start.
      static_assert(NTH == 512 && KP <= 256, "two threads per row of G");
      const int j = tid & 255, hf = tid >> 8;
      const bool own = hf == 0 && j < K;  // thread owns coefficient j
      const double bj = own ? bsh[j] : 0.0;
      float* psh = reinterpret_cast<float*>(bsh);  // upper half's sums (b is in bj now)
      const f32x4* c4 = reinterpret_cast<const f32x4*>(csh);
      float* dsh = csh + KP;
      const f32x4* d4 = reinterpret_cast<const f32x4*>(dsh);
      const int ce = a.check_every;
      __shared__ int run_sh[2];  // iterations run, rule met
      // thread (j, hf) holds G[j][hf KH + i], i < KH (zero past K); each
      // index i goes into partial sum i % 4
      constexpr int KH = KP / 2;
      float g[KH];
#pragma unroll
      for (int i = 0; i < KH; ++i) {
        const int col = hf * KH + i;
        g[i] = (j < K && col < K) ? G[j * K + col] : 0.f;
      }
      auto matvec_part = [&](const float* v, const f32x4* v4) -> float {
        (void)v;
        float d0 = 0.f, d1 = 0.f, d2 = 0.f, d3 = 0.f;
#pragma unroll
        for (int i4 = 0; i4 < KH / 4; ++i4) {
          const f32x4 cv = v4[hf * (KH / 4) + i4];
          d0 = fmaf(cv[0], g[4 * i4 + 0], d0);
          d1 = fmaf(cv[1], g[4 * i4 + 1], d1);
          d2 = fmaf(cv[2], g[4 * i4 + 2], d2);
          d3 = fmaf(cv[3], g[4 * i4 + 3], d3);
        }
        return (d0 + d1) + (d2 + d3);
      };
      __syncthreads();  // every bj is read before psh (over b) is written
      int its_total = 0;
      bool met = false;
      for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
          // the warm start missed the rule by the cap: cold start, same cap
          if (!(warm_kept && ce > 0 && !met)) break;
          if (tid < KP) csh[tid] = tid < K ? sm_uniform(key, (uint64_t)f * K + tid) : 0.f;
          if (a.fallback && tid == 0) a.fallback[f] = 2;
          __syncthreads();
        }
        float cj = own ? csh[j] : 0.f, cp = cj;
        int it = 0, next_check = ce > 0 ? ce : -1;  // iteration of the next stop-rule check
        bool stop = false;
        for (; it < a.iters; ++it) {
          float den = matvec_part(csh, c4);
          if (hf == 1 && j < K) psh[j] = den;
          __syncthreads();
          if (own) den += psh[j];
          if (it == next_check) {
            next_check += ce;
            const float dj = own ? cj - cp : 0.f;
            if (hf == 0 && j < KP) dsh[j] = dj;
            __syncthreads();
            float dg = matvec_part(dsh, d4);
            if (hf == 1 && j < K) psh[j] = dg;
            __syncthreads();
            if (own) dg += psh[j];
            const double q1 = wave_sum(own ? (double)dj * (double)dg : 0.0);
            const double q2 = wave_sum(own ? (double)cj * (double)den : 0.0);
            if (lane == 0) {
              wsel[0][wave] = q1;
              wsel[1][wave] = q2;
            }
            __syncthreads();
            double s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int w = 0; w < NWV; ++w) {
              s1 += wsel[0][w];
              s2 += wsel[1][w];
            }
            if (s1 <= a.tol2 * s2) {  // the same value in every thread
              stop = true;
              break;
            }
            cp = cj;
          }
          if (own) {
            cj = mu_apply_d(cj, bj, (double)den, a.eps);
            csh[j] = cj;
          }
          __syncthreads();
        }
        if (tid == 0) {
          run_sh[0] = it;
          run_sh[1] = stop ? 1 : 0;
        }
        __syncthreads();
        its_total += run_sh[0];
        met = run_sh[1] != 0;
        __syncthreads();
      }
      if (a.iters_out && tid == 0) a.iters_out[f] = its_total;
      if (tid < K) a.C_out[(int64_t)f * K + tid] = csh[tid];
      if (a.ticks && tid == 0) {
        a.ticks[2 * (int64_t)f] = tick0;
        a.ticks[2 * (int64_t)f + 1] = wall_clock64();
      }
    }
    __syncthreads();  // LDS is reused by the next frame
  }
  if (bad) atomicOr(a.status, bad);
}

size_t gram_lds_bytes(int K, int KP, int prec, int ahead) {
  const int goff = (std::max(K * K, gram_stage_floats(K, KP, prec, ahead)) + 3) & ~3;
  return (size_t)goff * 4 + (size_t)KP * 8 + (size_t)KP * 4 * 2;  // G | b | c, d
}

template <int KP, bool RAGGED, int PREC, bool FORM, int PF>
static hipError_t gram_launch(const GramArgs& a, int max_blocks, hipStream_t s, int* grid_out) {
  const size_t lds = gram_lds_bytes(a.K, KP, PREC, PF);
  auto fn = k_gram<KP, RAGGED, PREC, FORM, PF>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * gram_waves<KP>(), lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int grid = std::max(1, std::min(a.F, cus * per_cu));
  if (max_blocks > 0) grid = std::min(grid, max_blocks);
  if (grid_out) *grid_out = grid;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(64 * gram_waves<KP>()), lds, s, a);
  return hipGetLastError();
}

template <bool RAGGED, int PREC, bool FORM, int PF>
static hipError_t gram_kp(int kp, const GramArgs& a, int max_blocks, hipStream_t s, int* g) {
  if constexpr (FORM) {  // K <= 128: G formed here, iterated by k_gram_iter
    switch (kp) {
      case 32: return gram_launch<32, RAGGED, PREC, true, PF>(a, max_blocks, s, g);
      case 64: return gram_launch<64, RAGGED, PREC, true, PF>(a, max_blocks, s, g);
      case 96: return gram_launch<96, RAGGED, PREC, true, PF>(a, max_blocks, s, g);
      case 128: return gram_launch<128, RAGGED, PREC, true, PF>(a, max_blocks, s, g);
      default: break;
    }
  } else {
    switch (kp) {
      case 160: return gram_launch<160, RAGGED, PREC, false, PF>(a, max_blocks, s, g);
      case 192: return gram_launch<192, RAGGED, PREC, false, PF>(a, max_blocks, s, g);
      case 224: return gram_launch<224, RAGGED, PREC, false, PF>(a, max_blocks, s, g);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

template <bool FORM, int PF>
static hipError_t gram_form(int kp, bool ragged, const GramArgs& a, int max_blocks, hipStream_t s,
                            int* grid_out) {
  if (a.prec == PREC_BF16X3)
    return ragged ? gram_kp<true, PREC_BF16X3, FORM, PF>(kp, a, max_blocks, s, grid_out)
                  : gram_kp<false, PREC_BF16X3, FORM, PF>(kp, a, max_blocks, s, grid_out);
  return ragged ? gram_kp<true, PREC_FP32, FORM, PF>(kp, a, max_blocks, s, grid_out)
                : gram_kp<false, PREC_FP32, FORM, PF>(kp, a, max_blocks, s, grid_out);
}

hipError_t launch_gram(int kp, bool ragged, const GramArgs& a, int max_blocks, hipStream_t s,
                       int* grid_out, bool form) {
  if (a.ahead != 1 && a.ahead != 2) return hipErrorInvalidValue;
  if (a.ahead == 1)
    return form ? gram_form<true, 1>(kp, ragged, a, max_blocks, s, grid_out)
                : gram_form<false, 1>(kp, ragged, a, max_blocks, s, grid_out);
  return form ? gram_form<true, 2>(kp, ragged, a, max_blocks, s, grid_out)
              : gram_form<false, 2>(kp, ragged, a, max_blocks, s, grid_out);
}

// ---------------------------------------------------------------------------
// Iterations of the two-phase form (K <= 128): one frame per workgroup of
// KR / 32 waves rounded up.  Lanes l and l + 32 of wave w share row
// j = 32 w + l of the product: each keeps half of row j of the frame's G in
// registers (KR / 2 entries; G is symmetric, so row j is column j), the two
// half sums meet through a lane swap (v_permlane32_swap, no LDS) and are
// added in the same order in both lanes, and lane l updates coefficient j.  The coefficients travel
// through a double buffer in LDS, so one barrier per iteration suffices
// (iteration t reads buffer t % 2 and writes the other).  The update and the
// stop rule are those of the one-launch form of k_gram for larger K (FP64
// ratio and objective sums, four FP32 partial sums per half row).
// ---------------------------------------------------------------------------
template <int KR>
__host__ __device__ constexpr int gram_iter_threads() {
  return 64 * ((KR + 31) / 32);
}

template <int KP, int KR>
__global__ __launch_bounds__(gram_iter_threads<KR>()) void k_gram_iter(GramArgs a) {
  static_assert(KR % 8 == 0 && KR <= KP, "row length: K rounded up to 8");
  constexpr int NT = gram_iter_threads<KR>();
  constexpr int NW = NT / 64;
  constexpr int KH = KR / 2;  // entries of a half row (the zero padding past KR left out)
  __shared__ __align__(16) float cb[2][KP];
  __shared__ __align__(16) float dsh[KP];
  __shared__ double wsel[2][NW];
  const int f = blockIdx.x;
  if (f >= a.F) return;
  const int K = a.K;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int j = 32 * wave + (lane & 31), hf = lane >> 5;
  const bool own = hf == 0 && j < K;  // lane that writes coefficient j
  const uint64_t key = sm_key(a.seed, 2);
  float g[KH];
  const float* Gr = a.Gf + (int64_t)f * K * K + (j < K ? j : 0) * K;
#pragma unroll
  for (int i = 0; i < KH; ++i) {
    const int col = hf * KH + i;
    g[i] = (j < K && col < K) ? Gr[col] : 0.f;
  }
  const double bj = j < K ? a.bf[(int64_t)f * KP + j] : 0.0;
  const bool warm_kept = a.warm && a.fallback && a.fallback[f] == 0;
  const int ce = a.check_every;
  auto sync = [&]() {
    if constexpr (NW == 1) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  };
  // (v G)_j, the same value in both lanes of row j
  auto matvec = [&](const float* v) -> float {
    const f32x4* v4 = reinterpret_cast<const f32x4*>(v) + hf * (KH / 4);
    float d0 = 0.f, d1 = 0.f, d2 = 0.f, d3 = 0.f;
#pragma unroll
    for (int i4 = 0; i4 < KH / 4; ++i4) {
      const f32x4 cv = v4[i4];
      d0 = fmaf(cv[0], g[4 * i4 + 0], d0);
      d1 = fmaf(cv[1], g[4 * i4 + 1], d1);
      d2 = fmaf(cv[2], g[4 * i4 + 2], d2);
      d3 = fmaf(cv[3], g[4 * i4 + 3], d3);
    }
    // v_permlane32_swap of the value with itself: element 0 holds the
    // lower lane's value of the pair (l mod 32), element 1 the upper's
    const uint32_t pb = __builtin_bit_cast(uint32_t, (d0 + d1) + (d2 + d3));
    const auto pr = __builtin_amdgcn_permlane32_swap(pb, pb, false, false);
    return __builtin_bit_cast(float, (uint32_t)pr[0]) + __builtin_bit_cast(float, (uint32_t)pr[1]);
  };
  // a sum over all coefficients, the same value in every thread: per wave
  // in a fixed order, then the waves in order
  auto block_sum2 = [&](double x1, double x2, double& s1, double& s2) {
    x1 = wave_sum(x1);
    x2 = wave_sum(x2);
    if constexpr (NW == 1) {
      s1 = x1;
      s2 = x2;
    } else {
      if (lane == 0) {
        wsel[0][wave] = x1;
        wsel[1][wave] = x2;
      }
      __syncthreads();
      s1 = 0.0;
      s2 = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        s1 += wsel[0][w];
        s2 += wsel[1][w];
      }
      __syncthreads();
    }
  };
  float cj = j < KP ? a.cf[(int64_t)f * KP + j] : 0.f;
  int its_total = 0;
  bool met = false;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      // the warm start missed the rule by the cap: cold start, same cap
      if (!(warm_kept && ce > 0 && !met)) break;
      cj = j < K ? sm_uniform(key, (uint64_t)f * K + j) : 0.f;
      if (tid == 0) a.fallback[f] = 2;
    }
    if (hf == 0 && j < KP) cb[0][j] = cj;
    sync();
    float cp = cj;
    int it = 0, next_check = ce > 0 ? ce : -1;  // iteration of the next stop-rule check
    bool stop = false;
    for (; it < a.iters; ++it) {
      const float* cur = cb[it & 1];
      const float den = matvec(cur);
      if (it == next_check) {
        next_check += ce;
        const float dj = j < K ? cj - cp : 0.f;
        if (hf == 0 && j < KP) dsh[j] = dj;
        sync();
        const float dg = matvec(dsh);
        double s1, s2;
        block_sum2(own ? (double)dj * (double)dg : 0.0, own ? (double)cj * (double)den : 0.0, s1,
                   s2);
        if (s1 <= a.tol2 * s2) {  // the same value in every thread
          stop = true;
          break;
        }
        cp = cj;
      }
      if (j < K) cj = mu_apply_d(cj, bj, (double)den, a.eps);
      if (hf == 0 && j < KP) cb[(it + 1) & 1][j] = cj;
      sync();
    }
    its_total += it;
    met = stop;
  }
  if (a.iters_out && tid == 0) a.iters_out[f] = its_total;
  if (own) a.C_out[(int64_t)f * K + j] = cj;
  if (a.ticks && tid == 0) a.ticks[2 * (int64_t)f + 1] = wall_clock64();
}

template <int KP, int KR>
static void gram_iter_go(const GramArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_gram_iter<KP, KR>), dim3(a.F), dim3(gram_iter_threads<KR>()), 0, s, a);
}

// The products of a row with G run over K rounded up to 8 (the rest of a
// KP-long row is zero padding), so the kernel comes in one form per K / 8.
template <int KP>
static hipError_t gram_iter_kp(int K, const GramArgs& a, hipStream_t s) {
  const int r = (K + 7) / 8 * 8;
  switch (KP - r) {
    case 0: gram_iter_go<KP, KP>(a, s); break;
    case 8: gram_iter_go<KP, KP - 8>(a, s); break;
    case 16: gram_iter_go<KP, KP - 16>(a, s); break;
    case 24: gram_iter_go<KP, KP - 24>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gram_iter(int kp, const GramArgs& a, hipStream_t s) {
  if (a.F <= 0) return hipSuccess;
  if (a.K < 1 || a.K > kp || kp - a.K >= 32) return hipErrorInvalidValue;
  switch (kp) {
    case 32: return gram_iter_kp<32>(a.K, a, s);
    case 64: return gram_iter_kp<64>(a.K, a, s);
    case 96: return gram_iter_kp<96>(a.K, a, s);
    case 128: return gram_iter_kp<128>(a.K, a, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Longest-first frame order for the persistent queue: one workgroup bitonic
// sort of (size, index) pairs, descending size then ascending index.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_frame_order(const int64_t* offsets, int f, int n2,
                                                     int* order) {
  __shared__ int ks[MAX_SORT_FRAMES];
  __shared__ int vs[MAX_SORT_FRAMES];
  for (int i = threadIdx.x; i < n2; i += 1024) {
    if (i < f) {
      const int64_t d = offsets[i + 1] - offsets[i];
      ks[i] = d < 0 ? 0 : (d > 0x7fffffff ? 0x7fffffff : (int)d);
    } else {
      ks[i] = -1;
    }
    vs[i] = i;
  }
  __syncthreads();
  for (int size = 2; size <= n2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < n2; i += 1024) {
        const int jx = i ^ stride;
        if (jx > i) {
          // "before" = larger size, then smaller index
          const bool desc = (i & size) == 0;
          const bool i_before = ks[i] > ks[jx] || (ks[i] == ks[jx] && vs[i] < vs[jx]);
          if (desc != i_before) {
            const int tk = ks[i], tv = vs[i];
            ks[i] = ks[jx];
            vs[i] = vs[jx];
            ks[jx] = tk;
            vs[jx] = tv;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < f; i += 1024) order[i] = vs[i];
}

// More frames: a stable least-significant-digit radix sort (4-bit digits,
// eight passes) of key = INT32_MAX - size with the frame index as value, in
// one workgroup over global ping-pong buffers (tmp: 4 f ints).  Stability
// keeps equal sizes in increasing index order, as the bitonic sort orders
// them.  Thread t owns the contiguous element range [t C, (t+1) C).
__global__ __launch_bounds__(1024) void k_frame_order_radix(const int64_t* offsets, int f,
                                                           int* tmp, int* order) {
  constexpr int NT = 1024, ND = 16;
  __shared__ int cnt[ND * NT];  // digit-major: cnt[d * NT + t]
  __shared__ int part[NT];
  const int t = threadIdx.x;
  const int C = (f + NT - 1) / NT;
  const int b0 = min(t * C, f), b1 = min(b0 + C, f);
  int* ka = tmp;
  int* va = tmp + f;
  int* kb = tmp + 2 * f;
  int* vb = tmp + 3 * f;
  for (int i = b0; i < b1; ++i) {
    const int64_t d = offsets[i + 1] - offsets[i];
    const int sz = d < 0 ? 0 : (d > 0x7fffffff ? 0x7fffffff : (int)d);
    ka[i] = 0x7fffffff - sz;
    va[i] = i;
  }
  __syncthreads();
  for (int pass = 0; pass < 8; ++pass) {
    const int sh = 4 * pass;
    int c[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) c[d] = 0;
    for (int i = b0; i < b1; ++i) ++c[(ka[i] >> sh) & 15];
#pragma unroll
    for (int d = 0; d < ND; ++d) cnt[d * NT + t] = c[d];
    __syncthreads();
    // exclusive scan of cnt in digit-major order: thread t owns entries
    // [16 t, 16 t + 16)
    int loc = 0;
#pragma unroll
    for (int q = 0; q < ND; ++q) loc += cnt[16 * t + q];
    part[t] = loc;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
      const int v = t >= off ? part[t - off] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    int run = part[t] - loc;
#pragma unroll
    for (int q = 0; q < ND; ++q) {
      const int v = cnt[16 * t + q];
      cnt[16 * t + q] = run;
      run += v;
    }
    __syncthreads();
#pragma unroll
    for (int d = 0; d < ND; ++d) c[d] = cnt[d * NT + t];
    for (int i = b0; i < b1; ++i) {
      const int k = ka[i];
      const int pos = c[(k >> sh) & 15]++;
      kb[pos] = k;
      vb[pos] = va[i];
    }
    __syncthreads();
    int* x = ka; ka = kb; kb = x;
    x = va; va = vb; vb = x;
  }
  for (int i = b0; i < b1; ++i) order[i] = va[i];
}

hipError_t launch_frame_order(const int64_t* offsets, int f, int* order, int* tmp,
                              hipStream_t s) {
  if (f > MAX_SORT_FRAMES) {
    if (!tmp) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_frame_order_radix, dim3(1), dim3(1024), 0, s, offsets, f, tmp, order);
    return hipGetLastError();
  }
  int n2 = 1;
  while (n2 < f) n2 <<= 1;
  hipLaunchKernelGGL(k_frame_order, dim3(1), dim3(1024), 0, s, offsets, f, n2, order);
  return hipGetLastError();
}

}  // namespace nmf
