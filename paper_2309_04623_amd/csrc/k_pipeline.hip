// Steps around the factorisation on gfx950:
//   * masked Euclidean distances of target frames to the reference library
//     and the per-target selection of the closest references (Sec. 4.1:
//     a percentage of the closest frames, by the Euclidean norm, builds the
//     basis; Sec. 5.3: the largest SNR gain);
//   * the best factor of each frame's model PSF (Sec. 2 / Sec. 4.1): the
//     scale that minimises the variance of t - s (c H) over the frame's
//     valid pixels inside an optional region, clamped to a range;
//   * the start of each stage of the component-by-component basis build
//     (Sec. 2): the previous stage's components plus one seeded new one.

#include "device_common.hpp"
#include "kernels.hpp"

namespace nmf {

// ---------------------------------------------------------------------------
// Distances d[f, n] = sum_p [MT_fp > 0][M_np > 0] (T_fp - V_np)^2.
// A workgroup owns 64 references x 8 targets and walks the pixels in chunks
// of 64 staged in LDS (masked values replaced by 0, validity kept apart, so
// NaN under zero weight never reaches a sum).  Thread (r, s) accumulates
// reference r against the 8 targets over pixels s, s + 4, ... of a chunk in
// FP32, folded into FP64 once per chunk; the four pixel slices are added in
// a fixed order at the end.
// ---------------------------------------------------------------------------
constexpr int FD_REF = 64, FD_TGT = 8, FD_PIX = 64;

__global__ __launch_bounds__(256) void k_frame_dist(const float* T, const float* MT,
                                                   const float* V, const float* M, int f,
                                                   int n, int64_t p, double* dist,
                                                   int* status) {
  __shared__ float vs[FD_REF][FD_PIX + 1], vv[FD_REF][FD_PIX + 1];
  __shared__ float ts[FD_TGT][FD_PIX], tv[FD_TGT][FD_PIX];
  __shared__ double red[4][FD_TGT][FD_REF];
  const int tid = threadIdx.x;
  const int n0 = blockIdx.x * FD_REF, f0 = blockIdx.y * FD_TGT;
  const int r = tid & 63, sl = tid >> 6;
  double acc64[FD_TGT];
#pragma unroll
  for (int g = 0; g < FD_TGT; ++g) acc64[g] = 0.0;
  int bad = 0;
  for (int64_t c0 = 0; c0 < p; c0 += FD_PIX) {
    for (int i = tid; i < FD_REF * FD_PIX; i += 256) {
      const int rr = i / FD_PIX, x = i % FD_PIX;
      const int64_t c = c0 + x;
      float v = 0.f, ok = 0.f;
      if (n0 + rr < n && c < p) {
        const int64_t o = (int64_t)(n0 + rr) * p + c;
        if (M[o] > 0.f) {
          v = V[o];
          ok = 1.f;
          if (!isfinite(v)) bad = 1;
        }
      }
      vs[rr][x] = v;
      vv[rr][x] = ok;
    }
    for (int i = tid; i < FD_TGT * FD_PIX; i += 256) {
      const int g = i / FD_PIX, x = i % FD_PIX;
      const int64_t c = c0 + x;
      float t = 0.f, ok = 0.f;
      if (f0 + g < f && c < p) {
        const int64_t o = (int64_t)(f0 + g) * p + c;
        if (MT[o] > 0.f) {
          t = T[o];
          ok = 1.f;
          if (!isfinite(t)) bad = 1;
        }
      }
      ts[g][x] = t;
      tv[g][x] = ok;
    }
    __syncthreads();
    float acc[FD_TGT];
#pragma unroll
    for (int g = 0; g < FD_TGT; ++g) acc[g] = 0.f;
    for (int x = sl; x < FD_PIX; x += 4) {
      const float v = vs[r][x], okv = vv[r][x];
#pragma unroll
      for (int g = 0; g < FD_TGT; ++g) {
        const float d = ts[g][x] - v;
        acc[g] = fmaf(okv * tv[g][x] * d, d, acc[g]);
      }
    }
#pragma unroll
    for (int g = 0; g < FD_TGT; ++g) acc64[g] += (double)acc[g];
    __syncthreads();
  }
#pragma unroll
  for (int g = 0; g < FD_TGT; ++g) red[sl][g][r] = acc64[g];
  __syncthreads();
  for (int i = tid; i < FD_TGT * FD_REF; i += 256) {
    const int g = i / FD_REF, rr = i % FD_REF;
    if (f0 + g < f && n0 + rr < n)
      dist[(int64_t)(f0 + g) * n + n0 + rr] =
          ((red[0][g][rr] + red[1][g][rr]) + red[2][g][rr]) + red[3][g][rr];
  }
  if (bad) atomicOr(status, 1);
}

hipError_t launch_frame_dist(const float* T, const float* MT, const float* V, const float* M,
                             int f, int n, int64_t p, double* dist, int* status, hipStream_t s) {
  const dim3 g((n + FD_REF - 1) / FD_REF, (f + FD_TGT - 1) / FD_TGT);
  hipLaunchKernelGGL(k_frame_dist, g, dim3(256), 0, s, T, MT, V, M, f, n, p, dist, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Selection by rank: reference i of target f has rank #{j : key_j < key_i}
// with key = (distance, index) (a NaN distance counts as +inf); the ones with
// rank < n_sel are written at their rank.  Exact and order-independent.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_select_rank(const double* dist, int n, int n_sel,
                                                    int32_t* idx) {
  __shared__ double ds[256];
  const int f = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const double* d = dist + (int64_t)f * n;
  double di = i < n ? d[i] : 0.0;
  if (di != di) di = __builtin_inf();
  int rank = 0;
  for (int j0 = 0; j0 < n; j0 += 256) {
    const int j = j0 + threadIdx.x;
    double dj = j < n ? d[j] : 0.0;
    if (dj != dj) dj = __builtin_inf();
    ds[threadIdx.x] = dj;
    __syncthreads();
    const int m = min(256, n - j0);
    for (int q = 0; q < m; ++q) {
      const double x = ds[q];
      rank += (x < di || (x == di && j0 + q < i)) ? 1 : 0;
    }
    __syncthreads();
  }
  if (i < n && rank < n_sel) idx[(int64_t)f * n_sel + rank] = i;
}

hipError_t launch_select_rank(const double* dist, int f, int n, int n_sel, int32_t* idx,
                              hipStream_t s) {
  const dim3 g((n + 255) / 256, f);
  hipLaunchKernelGGL(k_select_rank, g, dim3(256), 0, s, dist, n, n_sel, idx);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Best factor: one workgroup per frame.  The model m_p = sum_k c_k H_kp is
// formed per pixel (FP64 accumulation, as the subtraction forms it) and the
// moments n, sum t, sum m, sum t^2, sum t m, sum m^2 over the used pixels
// are accumulated in FP64 and reduced in a fixed order; then
//   s = cov(t, m) / var(m), clamped to [s_lo, s_hi];
// s = 1 with fewer than two pixels or var(m) <= 1e-12 mean(m^2).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_best_factor(const float* H, const float* C,
                                                    const float* T, const float* MT,
                                                    const float* region, int k, int64_t p,
                                                    float s_lo, float s_hi, float* scale) {
  extern __shared__ float cs[];
  __shared__ double red[6][256];
  const int64_t f = blockIdx.x;
  for (int i = threadIdx.x; i < k; i += 256) cs[i] = C[f * k + i];
  __syncthreads();
  double mo[6] = {0, 0, 0, 0, 0, 0};  // n, St, Sm, Stt, Stm, Smm
  for (int64_t j = threadIdx.x; j < p; j += 256) {
    const int64_t o = f * p + j;
    if (!(MT[o] > 0.f) || (region && !(region[j] > 0.f))) continue;
    double m = 0.0;
    for (int i = 0; i < k; ++i) m = fma((double)cs[i], (double)H[(int64_t)i * p + j], m);
    const double t = (double)T[o];
    mo[0] += 1.0;
    mo[1] += t;
    mo[2] += m;
    mo[3] += t * t;
    mo[4] += t * m;
    mo[5] += m * m;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) red[q][threadIdx.x] = mo[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 6; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nn = red[0][0];
    double s = 1.0;
    if (nn >= 2.0) {
      const double mt = red[1][0] / nn, mm = red[2][0] / nn;
      const double var_m = red[5][0] / nn - mm * mm;
      const double cov = red[4][0] / nn - mt * mm;
      if (var_m > 1e-12 * (red[5][0] / nn)) {
        s = cov / var_m;
        s = s < (double)s_lo ? (double)s_lo : s;
        s = s > (double)s_hi ? (double)s_hi : s;
      }
    }
    scale[f] = (float)s;
  }
}

hipError_t launch_best_factor(const float* H, const float* C, const float* T, const float* MT,
                              const float* region, int64_t f, int k, int64_t p, float s_lo,
                              float s_hi, float* scale, hipStream_t s) {
  hipLaunchKernelGGL(k_best_factor, dim3((unsigned)f), dim3(256), k * sizeof(float), s, H, C, T,
                     MT, region, k, p, s_lo, s_hi, scale);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stage j start of the component-by-component build: W0 (n x j) = [W_prev |
// w], H0 (j x p) = [H_prev; h], with w_r = U(key(seed, 3), r K + j - 1) and
// h_c = U(key(seed, 4), (j - 1) p + c) (their places in n x K and K x p
// matrices).  W_prev / H_prev (n x (j-1), (j-1) x p) may be null for j = 1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_seq_start(const float* Wp, const float* Hp, int64_t n,
                                                  int64_t p, int j, int K, uint64_t seed,
                                                  float* W0, float* H0) {
  const uint64_t kw = sm_key(seed, 3), kh = sm_key(seed, 4);
  const int64_t nw = n * j, nh = (int64_t)j * p;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nw + nh;
       i += (int64_t)gridDim.x * 256) {
    if (i < nw) {
      const int64_t r = i / j, c = i % j;
      W0[i] = c < j - 1 ? Wp[r * (j - 1) + c] : sm_uniform(kw, (uint64_t)(r * K + j - 1));
    } else {
      const int64_t q = i - nw, r = q / p, c = q % p;
      H0[q] = r < j - 1 ? Hp[q] : sm_uniform(kh, (uint64_t)((int64_t)(j - 1) * p + c));
    }
  }
}

hipError_t launch_seq_start(const float* Wp, const float* Hp, int64_t n, int64_t p, int j, int K,
                            uint64_t seed, float* W0, float* H0, hipStream_t s) {
  const int64_t tot = (n + p) * j;
  const unsigned g = (unsigned)std::min<int64_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_seq_start, dim3(g), dim3(256), 0, s, Wp, Hp, n, p, j, K, seed, W0, H0);
  return hipGetLastError();
}

}  // namespace nmf
