// Streaming kernels around the fused half-step: data staging, factor
// layouts, the W-rule finish, fixed-order FP64 reductions, seeded init,
// basis normalisation, model-PSF subtraction and per-frame objectives.

#include "device_common.hpp"
#include "kernels.hpp"

namespace nmf {

// ---------------------------------------------------------------------------
// Staging (masked pixels are missing data: Vhat = V where M > 0, else 0)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_stage(StageArgs a) {
  __shared__ float tv[32][33];
  __shared__ float tm[32][33];
  __shared__ double red[256];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int cb = blockIdx.x * 32, rb = blockIdx.y * 32;
  int bad = 0;
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = rb + ty + 8 * q, c = cb + tx;
    float v = 0.f, m = 0.f;
    if (r < a.n && c < a.p) {
      v = a.V[(int64_t)r * a.p + c];
      m = a.M[(int64_t)r * a.p + c];
      if (!(m >= 0.f) || isinf(m)) {  // negative, NaN or Inf weight
        bad |= 4;
        m = 0.f;
      }
      if (a.binary) m = m > 0.f ? 1.f : 0.f;
      if (m > 0.f) {
        if (!isfinite(v)) {
          bad |= 1;
          v = 0.f;
        } else if (v < 0.f) {
          if (a.clip_negative) {
            m = 0.f;
            v = 0.f;
          } else {
            bad |= 2;
          }
        }
      } else {
        v = 0.f;
      }
      acc += (double)m * (double)v * (double)v;
    }
    tv[ty + 8 * q][tx] = v;
    tm[ty + 8 * q][tx] = m;
  }
  __syncthreads();
  // Tiled copies.  Slot o of a tile holds register i of lane ln with
  // o = (i / 4) * 256 + ln * 4 + i % 4, so that load u of a wave reads the
  // contiguous kilobyte [u * 256, u * 256 + 256) floats; (row, col) =
  // (acc_row(i, ln / 32), ln % 32).
  const int64_t tileA = ((int64_t)blockIdx.x * (a.n_pad / 32) + blockIdx.y) * 1024;
  const int64_t tileB = ((int64_t)blockIdx.y * (a.p_pad / 32) + blockIdx.x) * 1024;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int o = threadIdx.x + 256 * q;
    const int u = o >> 8, ln = (o & 255) >> 2, i = 4 * u + (o & 3);
    const int tr = acc_row(i, ln >> 5), tcol = ln & 31;
    if (a.D) {
      a.D[tileA + o] = tv[tr][tcol];
      if (!a.binary) a.Mw[tileA + o] = tm[tr][tcol];
    }
    if (a.DT) {
      a.DT[tileB + o] = tv[tcol][tr];
      if (!a.binary) a.MwT[tileB + o] = tm[tcol][tr];
    }
  }
  // Binary weights: lane ln of a tile keeps bit i for its register i.
  if (a.binary && threadIdx.x < 128) {
    const int ln = threadIdx.x & 63, half = ln >> 5, c = ln & 31;
    const bool tr_side = threadIdx.x >= 64;
    uint32_t bits = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = acc_row(i, half);
      const float m = tr_side ? tm[c][r] : tm[r][c];
      bits |= (m > 0.f ? 1u : 0u) << i;
    }
    if (!tr_side && a.D) a.B[(tileA >> 4) + ln] = (uint16_t)bits;
    if (tr_side && a.DT) a.BT[(tileB >> 4) + ln] = (uint16_t)bits;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
  if (bad) atomicOr(a.status, bad);
}

hipError_t launch_stage(const StageArgs& a, int* nblocks_out, hipStream_t s) {
  const dim3 g(a.p_pad / 32, a.n_pad / 32);
  *nblocks_out = g.x * g.y;
  hipLaunchKernelGGL(k_stage, g, dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed-order FP64 reduction (single block)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce_f64(const double* part, int n, double* out,
                                                   int* status, const int* out_index) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[out_index ? *out_index : 0] = red[0];
    if (status && !isfinite(red[0])) atomicOr(status, 8);
  }
}

hipError_t launch_reduce_f64(const double* part, int n, double* out, int* status, hipStream_t s,
                             const int* out_index) {
  hipLaunchKernelGGL(k_reduce_f64, dim3(1), dim3(256), 0, s, part, n, out, status, out_index);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Seeded init
// ---------------------------------------------------------------------------
__global__ void k_init_uniform(uint64_t key, int64_t count, float* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = sm_uniform(key, (uint64_t)i);
}

hipError_t launch_init_uniform(uint64_t seed, int matrix_id, int64_t count, float* out,
                               hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(k_init_uniform, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256),
                     0, s, sm_key(seed, matrix_id), count, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Factor layouts
// ---------------------------------------------------------------------------
__device__ __forceinline__ void store_layouts(int r, int k, float v, int rows_pad, int KP,
                                              float* m, __bf16* mh, __bf16* ml, float* t,
                                              float* tp, __bf16* tph, __bf16* tpl) {
  __bf16 hi, lo;
  split_bf16(v, hi, lo);
  m[lop_f32(r, k, KP)] = v;
  mh[lop_bf16(r, k, KP)] = hi;
  ml[lop_bf16(r, k, KP)] = lo;
  t[(int64_t)k * rows_pad + r] = v;
  tp[ltop_f32(k, r, KP)] = v;
  tph[ltop_bf16(k, r, KP)] = hi;
  tpl[ltop_bf16(k, r, KP)] = lo;
}

__global__ __launch_bounds__(256) void k_factor_fill(FactorFillArgs a) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= a.rows_pad) return;
  float v = 0.f;
  if (r < a.rows && k < a.K) {
    const int64_t idx = a.user_is_kxr ? (int64_t)k * a.rows + r : (int64_t)r * a.K + k;
    v = a.src ? a.src[idx] : sm_uniform(sm_key(a.seed, a.matrix_id), (uint64_t)idx);
  }
  store_layouts(r, k, v, a.rows_pad, a.KP, a.m, a.mh, a.ml, a.t, a.tp, a.tph, a.tpl);
}

hipError_t launch_factor_fill(const FactorFillArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_factor_fill, dim3((a.rows_pad + 255) / 256, a.KP), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_factor_out(const float* t, int rows, int rows_pad, int K,
                                                   int out_is_kxr, float* out) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= rows) return;
  const float v = t[(int64_t)k * rows_pad + r];
  if (out_is_kxr)
    out[(int64_t)k * rows + r] = v;
  else
    out[(int64_t)r * K + k] = v;
}

hipError_t launch_factor_out(const float* t, int rows, int rows_pad, int K, int KP,
                             int out_is_kxr, float* out, hipStream_t s) {
  (void)KP;
  hipLaunchKernelGGL(k_factor_out, dim3((rows + 255) / 256, K), dim3(256), 0, s, t, rows,
                     rows_pad, K, out_is_kxr, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Finish of a split half-step: fixed-order sum over the partials, the update,
// every layout; block (0, 0) also sums the H-rule objective partials.
// Block = 64 columns x 4 groups of splits.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_finish(FinishArgs a) {
  if (a.stop_seen && *a.stop_seen) return;  // an earlier iteration was the last
  __shared__ double rn[4][64];
  __shared__ double rd[4][64];
  __shared__ double rj[256];
  const int cx = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cx;
  const int k = blockIdx.y;
  double num = 0.0, den = 0.0;
  if (c < a.C_pad) {
    const int64_t stride = (int64_t)a.KP * a.C_pad;
    const float* pn = a.partial + (int64_t)k * a.C_pad + c;
    for (int s = g; s < a.S; s += 4) {
      num += pn[(int64_t)(2 * s) * stride];
      den += pn[(int64_t)(2 * s + 1) * stride];
    }
  }
  rn[g][cx] = num;
  rd[g][cx] = den;
  __syncthreads();
  if (g == 0 && c < a.C_pad) {
    num = ((rn[0][cx] + rn[1][cx]) + rn[2][cx]) + rn[3][cx];
    den = ((rd[0][cx] + rd[1][cx]) + rd[2][cx]) + rd[3][cx];
    float nv = 0.f;
    const int64_t it = (int64_t)k * a.C_pad + c;
    if (k < a.K && c < a.C_valid) nv = mu_apply_d(a.t[it], num, den, a.eps);
    a.t[it] = nv;
    a.m[lop_f32(c, k, a.KP)] = nv;
    if (a.prec == PREC_FP32) {
      a.tp[ltop_f32(k, c, a.KP)] = nv;
    } else {
      __bf16 hi, lo;
      split_bf16(nv, hi, lo);
      a.mh[lop_bf16(c, k, a.KP)] = hi;
      a.ml[lop_bf16(c, k, a.KP)] = lo;
      a.tph[ltop_bf16(k, c, a.KP)] = hi;
      a.tpl[ltop_bf16(k, c, a.KP)] = lo;
    }
  }
  if (a.Jpart && blockIdx.x == 0 && blockIdx.y == 0) {
    double sj = 0.0;
    for (int i = threadIdx.x; i < a.nJ; i += 256) sj += a.Jpart[i];
    rj[threadIdx.x] = sj;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) rj[threadIdx.x] += rj[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const int t = *a.iter;
      const double J = rj[0];
      a.Jhist[t] = J;
      *a.iter = t + 1;
      if (!isfinite(J)) atomicOr(a.status, 8);
      // Stop rule on the relative decrease of the objective over the last
      // check_every iterations; J is the cost of the iterate entering
      // iteration t, so when it passes iteration t is the last one.
      const int c = a.check_every;
      if (a.stop_req && c > 0 && t >= c && t % c == 0) {
        const double j0 = a.Jhist[t - c];
        if (j0 > 0.0 && (j0 - J) / j0 < a.tol) *a.stop_req = 1;
      }
    }
  }
}

hipError_t launch_finish(const FinishArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3((a.C_pad + 63) / 64, a.KP), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ void k_set_int(int* p, int v) { *p = v; }

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_int(int* p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = v;
}

hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Basis normalisation: H_k <- H_k / ||H_k||, W[:, k] <- W[:, k] ||H_k||
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_normalize(float* Ht, int p_pad, float* Wt, int n_pad) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  float* hr = Ht + (int64_t)k * p_pad;
  double s = 0.0;
  for (int i = threadIdx.x; i < p_pad; i += 256) s += (double)hr[i] * (double)hr[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double d = red[0] > 0.0 ? sqrt(red[0]) : 1.0;
  for (int i = threadIdx.x; i < p_pad; i += 256) hr[i] = (float)((double)hr[i] / d);
  float* wr = Wt + (int64_t)k * n_pad;
  for (int i = threadIdx.x; i < n_pad; i += 256) wr[i] = (float)((double)wr[i] * d);
}

hipError_t launch_normalize(float* Ht, int KP, int p_pad, int K, float* Wt, int n_pad,
                            hipStream_t s) {
  (void)KP;
  hipLaunchKernelGGL(k_normalize, dim3(K), dim3(256), 0, s, Ht, p_pad, Wt, n_pad);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Subtraction: model = C H (FP64 accumulation), residual = T - s * model,
// NaN where the frame's weight is 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_subtract(const float* H, const float* C, const float* T,
                                                 const float* MT, int k, int64_t p,
                                                 const float* scale, float* model,
                                                 float* resid) {
  extern __shared__ float cs[];
  const int64_t f = blockIdx.y;
  for (int i = threadIdx.x; i < k; i += 256) cs[i] = C[f * k + i];
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= p) return;
  double acc = 0.0;
  for (int i = 0; i < k; ++i) acc = fma((double)cs[i], (double)H[(int64_t)i * p + j], acc);
  const float mdl = (float)acc;
  const float sf = scale ? scale[f] : 1.0f;
  const int64_t o = f * p + j;
  if (model) model[o] = mdl;
  const float t = T[o];
  resid[o] = MT[o] > 0.f ? (float)((double)t - (double)sf * acc) : __builtin_nanf("");
}

hipError_t launch_subtract(const float* H, const float* C, const float* T, const float* MT,
                           int64_t f, int k, int64_t p, const float* scale, float* model,
                           float* resid, hipStream_t s) {
  const dim3 g((unsigned)((p + 255) / 256), (unsigned)f);
  hipLaunchKernelGGL(k_subtract, g, dim3(256), k * sizeof(float), s, H, C, T, MT, k, p, scale,
                     model, resid);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-frame objective sum_p m (t - c H)^2 (FP64)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_frame_objective(const float* H, const float* C,
                                                        const float* T, const float* MT, int k,
                                                        int64_t p, int binary, int clip_negative,
                                                        double* out) {
  extern __shared__ float cs[];
  __shared__ double red[256];
  const int64_t f = blockIdx.x;
  for (int i = threadIdx.x; i < k; i += 256) cs[i] = C[f * k + i];
  __syncthreads();
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < p; j += 256) {
    float m = MT[f * p + j];
    if (binary) m = m > 0.f ? 1.f : 0.f;
    const float t = T[f * p + j];
    if (clip_negative && t < 0.f) m = 0.f;
    if (m > 0.f) {
      double acc = 0.0;
      for (int i = 0; i < k; ++i) acc = fma((double)cs[i], (double)H[(int64_t)i * p + j], acc);
      const double d = (double)t - acc;
      s += (double)m * d * d;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[f] = red[0];
}

hipError_t launch_frame_objective(const float* H, const float* C, const float* T,
                                  const float* MT, int64_t f, int k, int64_t p, int binary,
                                  int clip_negative, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_frame_objective, dim3((unsigned)f), dim3(256), k * sizeof(float), s, H, C,
                     T, MT, k, p, binary, clip_negative, out);
  return hipGetLastError();
}

}  // namespace nmf
