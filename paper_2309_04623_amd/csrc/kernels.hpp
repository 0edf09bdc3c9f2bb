// Internal launch interface between the host library (api.cpp) and the
// gfx950 kernels.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nmf {

// One multiplicative-update half-step over a data matrix D (R x C, padded to
// multiples of 32) with weights Mw of the same shape:
//   Y   = L Rt                      (L: R x K rows, Rt: K x C tile)
//   num = L^T (Mw o D),  den = L^T (Mw o Y)   (reduced over R)
// and optionally J = sum Mw (D - Y)^2.
// The H-rule of Eq. 3 is this step on (D = V, L = W, Rt = H); the W-rule is
// the same step on the transposed problem (D = V^T, L = H^T, Rt = W^T).
//
// D and Mw are stored tiled: 32x32 tiles, column-tile-major (tile (tr, tc)
// at index tc * RT + tr), and inside a tile in MFMA accumulator order:
// register i of lane l (column l % 32, row acc_row(i, l / 32)) at
// (i / 4) * 256 + l * 4 + i % 4.
struct DualArgs {
  const float* D;
  const float* Mw;
  // binary weights instead of Mw (nullable): per tile 64 x 16 bits, lane l's
  // bit i is the weight of its register i (same placement as the tile slots)
  const uint16_t* Mb;
  int RT;               // row tiles (R_pad / 32)
  int tiles_per_split;  // row tiles per grid-y chunk
  int C_pad, C_valid;
  // left factor rows (R_pad x KP) in the operand order lop_f32 / lop_bf16
  const float* L;
  const __bf16* Lh;
  const __bf16* Ll;
  // left factor transposed (KP x R_pad) in the operand order ltop_f32 / ltop_bf16
  const float* LT;
  const __bf16* LTh;
  const __bf16* LTl;
  int64_t ldlt;
  // right factor (KP x C_pad, row-major)
  const float* Rt;
  int64_t ldr;
  // outputs
  float* partial;  // split mode: [split][2][KP][C_pad]
  double* Jpart;   // per-block objective partial (nullable)
  // update mode: the new right factor and the layouts the other half-step reads
  float* Rt_out;   // KP x C_pad (may equal Rt)
  float* RtT;      // C_pad x KP FP32
  __bf16* RtTh;    // C_pad x KP bf16 hi
  __bf16* RtTl;    // C_pad x KP bf16 lo
  float* Rtp;      // KP x C_pad FP32, permuted (FP32 operand order)
  __bf16* Rtph;    // KP x C_pad bf16 hi, permuted (bf16 operand order)
  __bf16* Rtpl;
  int K;
  float eps;
  // on-device stop (nullable): a set *stop_req makes the launch return at
  // once; the first block of an update-mode launch that sees it also sets
  // *stop_seen, which the finish kernel reads (the finish launch that sets
  // *stop_req must not read it, so the two flags trail each other by one
  // launch)
  const int* stop_req;
  int* stop_seen;
};

enum DualMode { MODE_UPDATE = 0, MODE_SPLIT = 1, MODE_OBJ = 2 };

// nw = waves per workgroup (1, 2 or 4); pipe = operand pipelining (2: the
// next tile's operands and data one tile ahead, KP <= 64 only; otherwise the
// current tile's operands at its start, or at their use for KP > 64);
// grid = (C_pad / 32, splits).
hipError_t launch_dual(int prec, int kp, int mode, int nw, int pipe, const DualArgs& a, int grid_x,
                       int grid_y, hipStream_t s);

// Wide-basis form of the same half-step (KP = 96..224): a workgroup of four
// waves owns four adjacent column tiles (one per wave) and shares each row
// tile's left-factor operand set through LDS.  grid = (wide_groups(C_pad /
// 32), splits); the objective partials are indexed by workgroup and are
// written in every mode when Jpart is set.
int wide_groups(int col_tiles);
hipError_t launch_wide(int prec, int kp, int mode, const DualArgs& a, int grid_y, hipStream_t s);

// Finishes a split half-step: sums the partials in a fixed order, applies
// the update to the factor (old value read from t, the KP x C_pad layout)
// and refreshes every layout.  Optionally also sums the objective partials
// of the preceding H-rule pass into Jhist[*iter] and advances *iter.
// With a stop test (check_every > 0, tol > 0): at t = *iter, a multiple of
// check_every and >= check_every, the iteration is the last one when
// (Jhist[t - c] - Jhist[t]) / Jhist[t - c] < tol; *stop_req is then set.
struct FinishArgs {
  const float* partial;  // [S][2][KP][C_pad]
  int S, KP, C_pad, C_valid, K;
  float eps;
  int prec;
  float* m;          // C_pad x KP
  __bf16* mh;        // C_pad x KP bf16 hi/lo
  __bf16* ml;
  float* t;          // KP x C_pad (holds the current values)
  float* tp;         // KP x C_pad permuted, FP32 operand order
  __bf16* tph;       // KP x C_pad permuted, bf16 operand order
  __bf16* tpl;
  const double* Jpart;  // nullable
  int nJ;
  double* Jhist;
  int* iter;
  int* status;
  int check_every;
  double tol;
  int* stop_req;         // nullable: set when the stop test passes
  const int* stop_seen;  // nullable: when set, the launch returns at once
};
hipError_t launch_finish(const FinishArgs& a, hipStream_t s);

hipError_t launch_set_int(int* p, int v, hipStream_t s);
hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t s);

// Layout fill of a factor: from a user matrix (rows x K, row-major, or
// K x rows if ``user_is_kxr``), or from the seeded generator when src is
// null, write every internal layout; padding entries are 0.
struct FactorFillArgs {
  const float* src;
  int user_is_kxr;
  uint64_t seed;
  int matrix_id;
  int rows, rows_pad, K, KP;
  float* m;
  __bf16* mh;
  __bf16* ml;
  float* t;
  float* tp;
  __bf16* tph;
  __bf16* tpl;
};
hipError_t launch_factor_fill(const FactorFillArgs& a, hipStream_t s);

// Copy the K x rows block of a transposed layout (KP x rows_pad) out to a user
// matrix, either rows x K (transpose) or K x rows.
hipError_t launch_factor_out(const float* t, int rows, int rows_pad, int K, int KP,
                             int out_is_kxr, float* out, hipStream_t s);

// Data staging: Vhat = V where M > 0 else 0 and the weights, written as the
// tiled layouts of the two half-steps (D: n x p tiles, DT: p x n tiles);
// flags bad data under positive weight; per-block partial sums of
// M * Vhat^2.
struct StageArgs {
  const float* V;
  const float* M;
  int64_t n, p;
  int n_pad, p_pad;
  int clip_negative;
  float* D;    // tiled n_pad x p_pad (nullable)
  float* Mw;
  float* DT;   // tiled p_pad x n_pad (nullable)
  float* MwT;
  int* status; // bit 0: non-finite data, bit 1: negative data, bit 2: bad weight
  double* part;
  // binary weights: weight = (M > 0); bit tiles written instead of Mw / MwT
  int binary;
  uint16_t* B;   // bits of the D tiles (with D)
  uint16_t* BT;  // bits of the DT tiles (with DT)
};
hipError_t launch_stage(const StageArgs& a, int* nblocks_out, hipStream_t s);

// Fixed-order FP64 sum of ``n`` partials into out[0], or out[*out_index]
// when out_index is given (single block).  With ``status``: status |= 8 if
// the sum is not finite.
hipError_t launch_reduce_f64(const double* part, int n, double* out, int* status, hipStream_t s,
                             const int* out_index = nullptr);

hipError_t launch_init_uniform(uint64_t seed, int matrix_id, int64_t count, float* out,
                               hipStream_t s);

// Unit-L2 normalisation of the K basis rows (k x P_pad master plus layouts)
// with the inverse scale moved into the coefficient rows.
hipError_t launch_normalize(float* Ht, int KP, int p_pad, int K, float* Wm, int n_pad,
                            hipStream_t s);

// Subtraction kernel.
hipError_t launch_subtract(const float* H, const float* C, const float* T, const float* MT,
                           int64_t f, int k, int64_t p, const float* scale, float* model,
                           float* resid, hipStream_t s);

// Per-frame objective sum_p m (t - c H)^2 for dense frames, with the
// weights staged as the projection stages them (binary: m > 0 counts as 1;
// clip_negative: negative data under weight is treated as masked).
hipError_t launch_frame_objective(const float* H, const float* C, const float* T,
                                  const float* MT, int64_t f, int k, int64_t p, int binary,
                                  int clip_negative, double* out, hipStream_t s);

// Masked-Gram projection: one persistent launch over all frames.
struct GramArgs {
  const float* HT;  // H transposed (P_pad x KP) in the lop_f32 operand order
  int K, P, F;
  // dense frames (F x P), or CSR frames
  const float* T;
  const float* MT;
  const int64_t* offsets;
  int64_t nnz;
  const int32_t* pix;
  const float* val;
  const float* wt;     // nullable: weights 1
  const int* order;    // nullable: processing order
  const float* C_init; // nullable: seeded U(0,1), matrix 2
  uint64_t seed;
  int iters;
  float eps;
  int clip_negative;
  int binary;          // every positive weight counts as 1
  float* C_out;        // F x K
  int* queue;          // zeroed before the launch
  int* status;         // bits as staging, plus 16 = bad CSR entry
  uint64_t* ticks;     // nullable: 2 per frame
  int warm;            // C_init is a warm start: fall back to the cold start
                       // per frame when its objective is lower
  int* fallback;       // nullable: per frame, 1 where the cold start was used
  int prec;            // products of G: PREC_FP32 or PREC_BF16X3
  // per-frame stop rule (check_every > 0): stop when the model change since
  // the previous check satisfies d G d^T <= tol2 * c G c^T; a warm start
  // that misses it by the cap restarts cold (fallback = 2)
  int check_every;
  double tol2;
  int* iters_out;      // nullable: iterations run per frame
  // two-phase form (K <= 128): the forming launch writes each frame's G
  // (K x K FP32), b (KP FP64) and starting coefficients (KP FP32) here, the
  // iterating launch reads them
  float* Gf;
  double* bf;
  float* cf;
  int* visits;  // nullable: per frame, incremented each time a workgroup takes it
  int ahead;    // chunks of pixel rows gathered ahead of their first use: 1 or 2
};
size_t gram_lds_bytes(int K, int KP, int prec, int ahead);
// form = true (required for KP <= 128, refused above): the launch only
// forms G, b and the start of every frame (Gf, bf, cf; warm-start decision
// included); launch_gram_iter then runs the iterations, one frame per
// workgroup of ceil(K / 32) waves (two lanes per row of G).
// form = false (KP > 128): one launch forms G and iterates each frame.
hipError_t launch_gram(int kp, bool ragged, const GramArgs& a, int max_blocks, hipStream_t s,
                       int* grid_out, bool form = false);
hipError_t launch_gram_iter(int kp, const GramArgs& a, hipStream_t s);
// Longest-first processing order of CSR frames (equal sizes by index): a
// bitonic sort in LDS up to MAX_SORT_FRAMES frames, a radix sort over
// ``tmp`` (4 f ints of device scratch) beyond.
constexpr int MAX_SORT_FRAMES = 8192;
hipError_t launch_frame_order(const int64_t* offsets, int f, int* order, int* tmp,
                              hipStream_t s);

// ---- reference selection, best factor, sequential build --------------------
// d[f, n] = sum over pixels valid in both of (T - V)^2 (FP32 per 64-pixel
// chunk, FP64 across chunks); status |= 1 for non-finite data under weight.
hipError_t launch_frame_dist(const float* T, const float* MT, const float* V, const float* M,
                             int f, int n, int64_t p, double* dist, int* status, hipStream_t s);
// idx[f, r] = reference of rank r < n_sel by (distance, index).
hipError_t launch_select_rank(const double* dist, int f, int n, int n_sel, int32_t* idx,
                              hipStream_t s);
hipError_t launch_best_factor(const float* H, const float* C, const float* T, const float* MT,
                              const float* region, int64_t f, int k, int64_t p, float s_lo,
                              float s_hi, float* scale, hipStream_t s);
// Start of stage j (of K) of the component-by-component build.
hipError_t launch_seq_start(const float* Wp, const float* Hp, int64_t n, int64_t p, int j, int K,
                            uint64_t seed, float* W0, float* H0, hipStream_t s);

// ---- learned warm start ---------------------------------------------------
enum { ACT_NONE = 0, ACT_GELU = 1 };
struct LinearArgs {
  const float* A;  // A(i, k) = A[i * sa0 + k * sa1]
  int64_t sa0, sa1;
  const float* B;  // B(k, j) = B[k * sb0 + j * sb1]
  int64_t sb0, sb1;
  const float* bias;  // nullable, N
  float* C;           // M x N, row stride ldc (pre-activation)
  float* Hact;        // act(C) when act != ACT_NONE
  int64_t ldc;
  int M, N, Kd;
  int act;
  int x3;  // 1: split-precision bf16x3 products, 0: bf16 operands
};
hipError_t launch_linear(const LinearArgs& a, hipStream_t s);
hipError_t launch_head(const float* z, const float* s, int B, int K, float floor_rel, float* w,
                       hipStream_t st);
hipError_t launch_head_bwd(const float* dw, const float* z, const float* s, int B, int K,
                           float* dz, hipStream_t st);
hipError_t launch_gelu_bwd(const float* dh, const float* a, int64_t n, float* da, hipStream_t st);
hipError_t launch_loss(const float* w, const float* cstar, const float* U, const float* V, int B,
                       int K, float* dw, double* lrow, hipStream_t st);
hipError_t launch_sub(const float* a, const float* b, int64_t n, float* out, hipStream_t st);
hipError_t launch_colsum(const float* d, int B, int N, float* out, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, int t, hipStream_t st);
hipError_t launch_gather_cur(const float* src, const int* perm, const int* ctr, int rows, int n,
                             float* out, hipStream_t st);
hipError_t launch_adam_dev(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                           float b1, float b2, float eps, const float* coef, hipStream_t st);
hipError_t launch_train_ctr(int* ctr, float* coef, int advance, int b, float b1, float b2,
                            hipStream_t st);
hipError_t launch_loss_accum(const double* lrow, int b, double* acc, int reset, hipStream_t st);
hipError_t launch_gather(const float* src, const int* idx, int rows, int n, float* out,
                         hipStream_t st);
hipError_t launch_pool(const float* T, const float* MT, int f, int ny, int nx, float* X, float* s,
                       hipStream_t st);
hipError_t launch_normal_init(float* p, int64_t n, float std, uint64_t seed, int stream_id,
                              hipStream_t st);

}  // namespace nmf
