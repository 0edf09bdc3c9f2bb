// Learned warm start for target modelling: the kernels of a small MLP that
// predicts a frame's projection coefficients from its masked-mean-pooled
// image (forward, backward, Adam), and the pooling itself.  The network is
// not in the paper; it only supplies the starting point of the Eq. 3
// W-rule iteration, which is unchanged.
//
// GEMMs run on v_mfma_f32_32x32x16_bf16 with FP32 accumulation, operands
// rounded to bf16 (one product) or split hi + lo (three products, ~FP32
// accuracy).  Operands are FP32 in memory with arbitrary strides, so the
// same kernel serves X W, dZ W^T and X^T dZ.

#include "device_common.hpp"
#include "kernels.hpp"

namespace nmf {

// ---------------------------------------------------------------------------
// C[M x N] = A[M x Kd] B[Kd x N] (+ bias[N]); A(i,k) = A[i*sa0 + k*sa1],
// B(k,j) = B[k*sb0 + j*sb1].  Block = 4 waves, 64 x 64 output tile, k-step 32.
// ---------------------------------------------------------------------------
template <int X3>
__global__ __launch_bounds__(256) void k_linear(LinearArgs a) {
  __shared__ __bf16 As[2][64][40];  // [hi/lo][row][k] (+8 pad)
  __shared__ __bf16 Bs[2][64][40];  // [hi/lo][col][k]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int col = lane & 31, half = lane >> 5;
  const int bm = blockIdx.y * 64, bn = blockIdx.x * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x16 acc = zero16();
  for (int k0 = 0; k0 < a.Kd; k0 += 32) {
    // stage 64 x 32 of A and 32 x 64 of B (8 elements each per thread)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q;
      const int r = e >> 5, kk = e & 31;
      const int gi = bm + r, gk = k0 + kk;
      float va = 0.f;
      if (gi < a.M && gk < a.Kd) va = a.A[(int64_t)gi * a.sa0 + (int64_t)gk * a.sa1];
      __bf16 hi, lo;
      split_bf16(va, hi, lo);
      As[0][r][kk] = hi;
      As[1][r][kk] = lo;
      const int gj = bn + r;
      float vb = 0.f;
      if (gj < a.N && gk < a.Kd) vb = a.B[(int64_t)gk * a.sb0 + (int64_t)gj * a.sb1];
      split_bf16(vb, hi, lo);
      Bs[0][r][kk] = hi;
      Bs[1][r][kk] = lo;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 32; ks += 16) {
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&As[0][wm + col][ks + 8 * half]);
      const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&Bs[0][wn + col][ks + 8 * half]);
      if constexpr (X3) {
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(&As[1][wm + col][ks + 8 * half]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&Bs[1][wn + col][ks + 8 * half]);
        acc = mfma_bf16x3(ah, al, bh, bl, acc);
      } else {
        acc = mfma_bf16(ah, bh, acc);
      }
    }
    __syncthreads();
  }
  const int j = bn + wn + col;
  if (j >= a.N) return;
  const float bias = a.bias ? a.bias[j] : 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = bm + wm + acc_row(i, half);
    if (r < a.M) {
      const float z = acc[i] + bias;
      a.C[(int64_t)r * a.ldc + j] = z;
      if (a.act == ACT_GELU) a.Hact[(int64_t)r * a.ldc + j] = 0.5f * z * (1.f + erff(z * 0.70710678118654752f));
    }
  }
}

hipError_t launch_linear(const LinearArgs& a, hipStream_t s) {
  const dim3 g((a.N + 63) / 64, (a.M + 63) / 64);
  if (a.x3)
    hipLaunchKernelGGL(k_linear<1>, g, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_linear<0>, g, dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Output head: w = s * softplus(z), floored at floor_rel * s.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float softplus_f(float z) {
  return z > 20.f ? z : log1pf(expf(z));
}
__device__ __forceinline__ float sigmoid_f(float z) { return 1.f / (1.f + expf(-z)); }
constexpr float FLOOR_REL = 1e-6f;

__global__ void k_head(const float* z, const float* s, int B, int K, float floor_rel, float* w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * K) return;
  const float sf = s[i / K];
  w[i] = fmaxf(sf * softplus_f(z[i]), floor_rel * sf);
}

// dz = dw * s * sigmoid(z)
__global__ void k_head_bwd(const float* dw, const float* z, const float* s, int B, int K,
                           float* dz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * K) return;
  const float sp = softplus_f(z[i]);
  dz[i] = sp > FLOOR_REL ? dw[i] * s[i / K] * sigmoid_f(z[i]) : 0.f;  // floored outputs pass no gradient
}

// da = dh * gelu'(a)
__global__ void k_gelu_bwd(const float* dh, const float* a, int64_t n, float* da) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float u = a[i];
  const float g = 0.5f * (1.f + erff(u * 0.70710678118654752f)) + u * 0.3989422804014327f * expf(-0.5f * u * u);
  da[i] = dh[i] * g;
}

// Loss L = mean_f d_f G d_f^T / (c*_f G c*_f^T) with U = d G and V = c* G
// precomputed (d = w - c*); writes dL/dw = 2 U / (den_f B) and one loss
// term per row (FP64 row sums).
__global__ void k_loss(const float* w, const float* cstar, const float* U, const float* V, int B,
                       int K, float* dw, double* lrow) {
  const int f = blockIdx.x;
  __shared__ double rn[64], rd[64];
  double an = 0.0, ad = 0.0;
  for (int k = threadIdx.x; k < K; k += 64) {
    const int64_t i = (int64_t)f * K + k;
    an += (double)(w[i] - cstar[i]) * (double)U[i];
    ad += (double)cstar[i] * (double)V[i];
  }
  rn[threadIdx.x] = an;
  rd[threadIdx.x] = ad;
  __syncthreads();
  for (int o = 32; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      rn[threadIdx.x] += rn[threadIdx.x + o];
      rd[threadIdx.x] += rd[threadIdx.x + o];
    }
    __syncthreads();
  }
  const double den = rd[0] > 0.0 ? rd[0] : 1.0;
  for (int k = threadIdx.x; k < K; k += 64) {
    const int64_t i = (int64_t)f * K + k;
    dw[i] = (float)(2.0 * (double)U[i] / (den * (double)B));
  }
  if (threadIdx.x == 0) lrow[f] = rn[0] / den;
}

// d = w - wstar (the left operand of U = d G)
__global__ void k_sub(const float* a, const float* b, int64_t n, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

// Column sums (bias gradients), fixed order: one thread per column.
__global__ void k_colsum(const float* d, int B, int N, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double s = 0.0;
  for (int r = 0; r < B; ++r) s += d[(int64_t)r * N + j];
  out[j] = (float)s;
}

// Adam over one contiguous parameter block.
__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Gather rows: out[r] = src[idx[r]] (row length n).
__global__ void k_gather(const float* src, const int* idx, int rows, int n, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * n) return;
  const int r = (int)(i / n), c = (int)(i % n);
  out[i] = src[(int64_t)idx[r] * n + c];
}

// ---- training steps replayed from one captured graph ----------------------
// The minibatch cursor, the Adam step t and the bias corrections
// c1 = 1 - b1^t, c2 = 1 - b2^t live in device memory and advance on the
// device after each step, so an epoch of steps is a fixed sequence of
// launches.  ctr = {cursor, t}, coef = {c1, c2}.
__global__ void k_gather_cur(const float* src, const int* perm, const int* ctr, int rows, int n,
                             float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * n) return;
  const int r = (int)(i / n), c = (int)(i % n);
  out[i] = src[(int64_t)perm[ctr[0] + r] * n + c];
}

__global__ void k_adam_dev(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                           float b1, float b2, float eps, const float* coef) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float c1 = coef[0], c2 = coef[1];
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_train_ctr(int* ctr, float* coef, int advance, int b, float b1, float b2) {
  if (threadIdx.x != 0) return;
  if (advance) {
    ctr[0] += b;
    ctr[1] += 1;
  } else {
    ctr[0] = 0;
    ctr[1] = 1;
  }
  coef[0] = 1.f - powf(b1, (float)ctr[1]);
  coef[1] = 1.f - powf(b2, (float)ctr[1]);
}

// acc (+)= sum of the b per-row loss terms, reduced in a fixed order.
__global__ __launch_bounds__(256) void k_loss_accum(const double* lrow, int b, double* acc,
                                                   int reset) {
  __shared__ double red[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < b; i += 256) v += lrow[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[0] = reset ? red[0] : acc[0] + red[0];
}

// Masked-mean pooling of dense frames (F x ny*nx) to F x 1024 and the
// per-frame masked mean s (1 when no pixel has weight or the mean is <= 0).
__global__ __launch_bounds__(256) void k_pool(const float* T, const float* MT, int ny, int nx,
                                             float* X, float* s_out) {
  const int f = blockIdx.x;
  const int64_t P = (int64_t)ny * nx;
  const float* t = T + (int64_t)f * P;
  const float* m = MT + (int64_t)f * P;
  __shared__ double rs[256];
  __shared__ int rc[256];
  double sum = 0.0;
  int cnt = 0;
  for (int64_t j = threadIdx.x; j < P; j += 256)
    if (m[j] > 0.f) {
      sum += t[j];
      ++cnt;
    }
  rs[threadIdx.x] = sum;
  rc[threadIdx.x] = cnt;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      rs[threadIdx.x] += rs[threadIdx.x + o];
      rc[threadIdx.x] += rc[threadIdx.x + o];
    }
    __syncthreads();
  }
  double sf = rc[0] > 0 ? rs[0] / rc[0] : 1.0;
  if (!(sf > 0.0)) sf = 1.0;
  if (threadIdx.x == 0) s_out[f] = (float)sf;
  const int by = (ny + 31) / 32, bx = (nx + 31) / 32;
  for (int q = threadIdx.x; q < 1024; q += 256) {
    const int gi = q >> 5, gj = q & 31;
    double bs = 0.0;
    int bc = 0;
    for (int y = gi * by; y < min(gi * by + by, ny); ++y)
      for (int x = gj * bx; x < min(gj * bx + bx, nx); ++x) {
        const int64_t j = (int64_t)y * nx + x;
        if (m[j] > 0.f) {
          bs += t[j];
          ++bc;
        }
      }
    X[(int64_t)f * 1024 + q] = bc > 0 ? (float)(bs / bc / sf) : 0.f;
  }
}

// Normal(0, std) fill from the counter-based generator (Box-Muller on two
// SplitMix64 uniforms per element).
__global__ void k_normal_init(float* p, int64_t n, float std, uint64_t key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float u1 = sm_uniform(key, (uint64_t)(2 * i));
  const float u2 = sm_uniform(key, (uint64_t)(2 * i + 1));
  p[i] = std * sqrtf(-2.f * logf(u1)) * cosf(6.283185307179586f * u2);
}

static inline dim3 grid1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_head(const float* z, const float* s, int B, int K, float floor_rel, float* w,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_head, grid1((int64_t)B * K), dim3(256), 0, st, z, s, B, K, floor_rel, w);
  return hipGetLastError();
}
hipError_t launch_head_bwd(const float* dw, const float* z, const float* s, int B, int K,
                           float* dz, hipStream_t st) {
  hipLaunchKernelGGL(k_head_bwd, grid1((int64_t)B * K), dim3(256), 0, st, dw, z, s, B, K, dz);
  return hipGetLastError();
}
hipError_t launch_gelu_bwd(const float* dh, const float* a, int64_t n, float* da, hipStream_t st) {
  hipLaunchKernelGGL(k_gelu_bwd, grid1(n), dim3(256), 0, st, dh, a, n, da);
  return hipGetLastError();
}
hipError_t launch_loss(const float* w, const float* cstar, const float* U, const float* V, int B,
                       int K, float* dw, double* lrow, hipStream_t st) {
  hipLaunchKernelGGL(k_loss, dim3(B), dim3(64), 0, st, w, cstar, U, V, B, K, dw, lrow);
  return hipGetLastError();
}
hipError_t launch_sub(const float* a, const float* b, int64_t n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sub, grid1(n), dim3(256), 0, st, a, b, n, out);
  return hipGetLastError();
}
hipError_t launch_colsum(const float* d, int B, int N, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, grid1(N), dim3(256), 0, st, d, B, N, out);
  return hipGetLastError();
}
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, int t, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, grid1(n), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t launch_gather(const float* src, const int* idx, int rows, int n, float* out,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_gather, grid1((int64_t)rows * n), dim3(256), 0, st, src, idx, rows, n, out);
  return hipGetLastError();
}
hipError_t launch_gather_cur(const float* src, const int* perm, const int* ctr, int rows, int n,
                             float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_cur, grid1((int64_t)rows * n), dim3(256), 0, st, src, perm, ctr,
                     rows, n, out);
  return hipGetLastError();
}
hipError_t launch_adam_dev(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                           float b1, float b2, float eps, const float* coef, hipStream_t st) {
  hipLaunchKernelGGL(k_adam_dev, grid1(n), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, coef);
  return hipGetLastError();
}
hipError_t launch_train_ctr(int* ctr, float* coef, int advance, int b, float b1, float b2,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_train_ctr, dim3(1), dim3(64), 0, st, ctr, coef, advance, b, b1, b2);
  return hipGetLastError();
}
hipError_t launch_loss_accum(const double* lrow, int b, double* acc, int reset, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_accum, dim3(1), dim3(256), 0, st, lrow, b, acc, reset);
  return hipGetLastError();
}
hipError_t launch_pool(const float* T, const float* MT, int f, int ny, int nx, float* X, float* s,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_pool, dim3(f), dim3(256), 0, st, T, MT, ny, nx, X, s);
  return hipGetLastError();
}

hipError_t launch_normal_init(float* p, int64_t n, float std, uint64_t seed, int stream_id,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_normal_init, grid1(n), dim3(256), 0, st, p, n, std, sm_key(seed, stream_id));
  return hipGetLastError();
}

}  // namespace nmf
