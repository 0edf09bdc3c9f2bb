// Host side of the C ABI declared in include/nmf_mi355x.h: argument checks,
// the device workspace, iteration control and kernel sequencing.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/nmf_mi355x.h"
#include "kernels.hpp"

using namespace nmf;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct nmf_handle_s {
  int device = 0;
  std::unordered_map<std::string, DevBuf> bufs;
  size_t total = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double* pinned = nullptr;  // host staging for objective values
  size_t pinned_count = 0;
  // live kernel timing
  bool prof = false;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> ev_pool;
  std::vector<Rec> pending;
  double prof_ms[NMF_K_COUNT] = {};
  int64_t prof_n[NMF_K_COUNT] = {};
  // captured launch sequences, keyed by operation and every argument
  hipStream_t cap = nullptr;
  std::unordered_map<std::string, hipGraphExec_t> graphs;
};

namespace {

#define LAUNCH(cls, expr) HIP_TRY(timed(h, (cls), s, [&]() { return (expr); }))

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(NMF_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int ws_get(nmf_handle h, const std::string& name, size_t bytes, void** out) {
  bytes = std::max<size_t>(bytes, 256);
  DevBuf& b = h->bufs[name];
  if (b.bytes < bytes) {
    if (b.p) {
      (void)hipDeviceSynchronize();
      (void)hipFree(b.p);
      h->total -= b.bytes;
      b.p = nullptr;
      b.bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(NMF_ERR_NOMEM, "device workspace allocation of " + std::to_string(bytes) +
                                     " bytes for '" + name + "' failed");
    }
    b.p = p;
    b.bytes = bytes;
    h->total += bytes;
  }
  *out = b.p;
  return NMF_OK;
}

template <typename T>
int ws(nmf_handle h, const std::string& name, size_t count, T** out) {
  void* p = nullptr;
  int rc = ws_get(h, name, count * sizeof(T), &p);
  *out = static_cast<T*>(p);
  return rc;
}

int pinned_get(nmf_handle h, size_t count, double** out) {
  if (h->pinned_count < count) {
    if (h->pinned) (void)hipHostFree(h->pinned);
    h->pinned = nullptr;
    h->pinned_count = 0;
    if (hipHostMalloc((void**)&h->pinned, count * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
      (void)hipGetLastError();
      return fail(NMF_ERR_NOMEM, "pinned host allocation failed");
    }
    h->pinned_count = count;
  }
  *out = h->pinned;
  return NMF_OK;
}

hipEvent_t pool_event(nmf_handle h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch ``fn`` on stream s; with timing on, bracket it with two events.
template <typename F>
hipError_t timed(nmf_handle h, int cls, hipStream_t s, F fn) {
  if (!h->prof) return fn();
  hipEvent_t a = pool_event(h), b = pool_event(h);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = fn();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  h->pending.push_back({cls, a, b});
  return e;
}

hipError_t prof_drain(nmf_handle h) {
  for (auto& r : h->pending) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return e;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    h->prof_ms[r.cls] += ms;
    h->prof_n[r.cls] += 1;
    h->ev_pool.push_back(r.a);
    h->ev_pool.push_back(r.b);
  }
  h->pending.clear();
  return hipSuccess;
}

// Runs ``enqueue(stream)`` either directly on ``s`` (timing on, or graphs
// off) or as a hipGraph captured once on the handle's capture stream and
// replayed on ``s``; the graph is cached under ``key``.
template <typename F>
hipError_t run_graph(nmf_handle h, const std::string& key, hipStream_t s, F enqueue) {
  if (h->prof) return enqueue(s);
  auto it = h->graphs.find(key);
  if (it == h->graphs.end()) {
    hipError_t e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t ee = enqueue(h->cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(h->cap, &graph);
    if (ee != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return ee;
    }
    if (e != hipSuccess) return e;
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    if (h->graphs.size() > 64) {
      for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
      h->graphs.clear();
    }
    it = h->graphs.emplace(key, exec).first;
  }
  return hipGraphLaunch(it->second, s);
}

std::string key_of(const char* op, std::initializer_list<uint64_t> vals) {
  std::string k(op);
  char buf[24];
  for (uint64_t v : vals) {
    std::snprintf(buf, sizeof(buf), ":%llx", (unsigned long long)v);
    k += buf;
  }
  return k;
}

inline int round_up(int64_t x, int m) { return (int)((x + m - 1) / m * m); }

// All layouts of one factor matrix with ``rows`` rows of K components
// (W: rows = n; H: rows = p, stored transposed as K x p in ``t``).
struct Factor {
  float* m = nullptr;
  __bf16* mh = nullptr;
  __bf16* ml = nullptr;
  float* t = nullptr;
  float* tp = nullptr;
  __bf16* tph = nullptr;
  __bf16* tpl = nullptr;
  int rows = 0, rows_pad = 0, KP = 0;
};

int factor_alloc(nmf_handle h, const std::string& pfx, int rows, int rows_pad, int KP, Factor* f) {
  const size_t n = (size_t)rows_pad * KP;
  int rc;
  if ((rc = ws(h, pfx + ".m", n, &f->m))) return rc;
  if ((rc = ws(h, pfx + ".mh", n, &f->mh))) return rc;
  if ((rc = ws(h, pfx + ".ml", n, &f->ml))) return rc;
  if ((rc = ws(h, pfx + ".t", n, &f->t))) return rc;
  if ((rc = ws(h, pfx + ".tp", n, &f->tp))) return rc;
  if ((rc = ws(h, pfx + ".tph", n, &f->tph))) return rc;
  if ((rc = ws(h, pfx + ".tpl", n, &f->tpl))) return rc;
  f->rows = rows;
  f->rows_pad = rows_pad;
  f->KP = KP;
  return NMF_OK;
}

FactorFillArgs fill_args(const Factor& f, const float* src, int user_is_kxr, uint64_t seed,
                         int matrix_id, int K) {
  FactorFillArgs a{};
  a.src = src;
  a.user_is_kxr = user_is_kxr;
  a.seed = seed;
  a.matrix_id = matrix_id;
  a.rows = f.rows;
  a.rows_pad = f.rows_pad;
  a.K = K;
  a.KP = f.KP;
  a.m = f.m;
  a.mh = f.mh;
  a.ml = f.ml;
  a.t = f.t;
  a.tp = f.tp;
  a.tph = f.tph;
  a.tpl = f.tpl;
  return a;
}

int check_params(const nmf_params* prm, int64_t rows, int64_t cols, bool need_k_le) {
  if (!prm) return fail(NMF_ERR_ARG, "params is NULL");
  if (prm->struct_size != sizeof(nmf_params))
    return fail(NMF_ERR_ARG, "nmf_params.struct_size mismatch (expected " +
                                 std::to_string(sizeof(nmf_params)) + ")");
  if (prm->k < 1) return fail(NMF_ERR_ARG, "k must be >= 1");
  if (need_k_le && (prm->k > rows || prm->k > cols))
    return fail(NMF_ERR_ARG, "k must not exceed min(n, p)");
  if (prm->max_iter < 0) return fail(NMF_ERR_ARG, "max_iter must be >= 0");
  if (prm->check_every < 0) return fail(NMF_ERR_ARG, "check_every must be >= 0");
  if (!(prm->tol >= 0.0)) return fail(NMF_ERR_ARG, "tol must be >= 0");
  if (prm->precision != NMF_PREC_FP32 && prm->precision != NMF_PREC_BF16X3)
    return fail(NMF_ERR_ARG, "unknown precision");
  if (!(prm->floor_eps >= 0.f) || !std::isfinite(prm->floor_eps))
    return fail(NMF_ERR_ARG, "floor_eps must be finite and >= 0");
  if (prm->split < 0) return fail(NMF_ERR_ARG, "split must be >= 0");
  if (prm->waves != 0 && prm->waves != 1 && prm->waves != 2 && prm->waves != 4)
    return fail(NMF_ERR_ARG, "waves must be 0, 1, 2 or 4");
  if (prm->pipeline < 0 || prm->pipeline > 2) return fail(NMF_ERR_ARG, "pipeline must be 0, 1 or 2");
  return NMF_OK;
}

int kp_for(int k) { return round_up(k, 32); }
constexpr int KP_MAX = 128;
constexpr int64_t DIM_MAX = (int64_t)1 << 30;

int check_dims(int64_t a, int64_t b, const char* what) {
  if (a <= 0 || b <= 0) return fail(NMF_ERR_SHAPE, std::string(what) + ": dimensions must be > 0");
  if (a > DIM_MAX || b > DIM_MAX || a * b > ((int64_t)1 << 40))
    return fail(NMF_ERR_SHAPE, std::string(what) + ": dimensions too large");
  return NMF_OK;
}

// Splits of the long reduction axis of the W-rule: enough blocks to fill
// 256 compute units several times over, at least two 32-row blocks each.
int auto_split(int col_tiles, int r_pad, int requested) {
  const int max_split = std::max(1, r_pad / 64);
  int s = requested > 0 ? requested : std::max(1, (2048 + col_tiles - 1) / col_tiles);
  return std::min(s, max_split);
}

int status_from_stage(int st) {
  if (st & 4) return fail(NMF_ERR_NEGATIVE, "negative or non-finite weight");
  if (st & 1) return fail(NMF_ERR_NONFINITE, "non-finite data under positive weight");
  if (st & 2) return fail(NMF_ERR_NEGATIVE, "negative data under positive weight");
  return NMF_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

const char* nmf_status_string(int status) {
  switch (status) {
    case NMF_OK: return "ok";
    case NMF_ERR_ARG: return "invalid argument";
    case NMF_ERR_SHAPE: return "invalid shape";
    case NMF_ERR_NONFINITE: return "non-finite data under positive weight";
    case NMF_ERR_NEGATIVE: return "negative data or weight";
    case NMF_ERR_DIVERGED: return "objective diverged";
    case NMF_ERR_HIP: return "HIP runtime error";
    case NMF_ERR_NOMEM: return "out of device memory";
    case NMF_ERR_UNSUPPORTED: return "unsupported request";
    case NMF_WARN_NONMONOTONE: return "warning: objective not monotone";
    case NMF_WARN_MAXITER: return "warning: tolerance not reached";
    default: return "unknown status";
  }
}

const char* nmf_last_error(void) { return g_last_error.c_str(); }

void nmf_params_default(nmf_params* prm) {
  if (!prm) return;
  std::memset(prm, 0, sizeof(*prm));
  prm->struct_size = sizeof(nmf_params);
  prm->k = 1;
  prm->max_iter = 200;
  prm->check_every = 0;
  prm->tol = 0.0;
  prm->seed = 0;
  prm->precision = NMF_PREC_FP32;
  prm->flags = 0;
  prm->floor_eps = 1e-30f;
  prm->split = 0;
  prm->waves = 0;
  prm->pipeline = 0;
}

int nmf_create(int hip_device, nmf_handle* out) {
  if (!out) return fail(NMF_ERR_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return fail(NMF_ERR_HIP, "no HIP device available");
  }
  if (hip_device < 0 || hip_device >= count) return fail(NMF_ERR_ARG, "device index out of range");
  nmf_handle h = new (std::nothrow) nmf_handle_s();
  if (!h) return fail(NMF_ERR_NOMEM, "host allocation failed");
  h->device = hip_device;
  DeviceGuard g(hip_device);
  if (!g.ok) {
    delete h;
    return fail(NMF_ERR_HIP, "hipSetDevice failed");
  }
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
      hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) {
    delete h;
    return fail(NMF_ERR_HIP, "hipEventCreate/hipStreamCreate failed");
  }
  *out = h;
  return NMF_OK;
}

int nmf_destroy(nmf_handle h) {
  if (!h) return NMF_OK;
  DeviceGuard g(h->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : h->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  if (h->pinned) (void)hipHostFree(h->pinned);
  (void)prof_drain(h);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  delete h;
  return NMF_OK;
}

size_t nmf_workspace_bytes(nmf_handle h) { return h ? h->total : 0; }

int nmf_init_uniform(nmf_handle h, uint64_t seed, int32_t matrix_id, int64_t rows, int64_t cols,
                     float* out, void* stream) {
  if (!out) return fail(NMF_ERR_ARG, "out is NULL");
  if (matrix_id < 0) return fail(NMF_ERR_ARG, "matrix_id must be >= 0");
  int rc = check_dims(rows, cols, "init");
  if (rc) return rc;
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  LAUNCH(NMF_K_OTHER, launch_init_uniform(seed, matrix_id, rows * cols, out, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  return NMF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
namespace {

// Launch shape of one fused half-step: waves per workgroup and the number of
// row chunks (grid y).
struct PassCfg {
  int nw = 1;
  int splits = 1;
  int tiles_per_split = 1;
  int pipe = 1;
};

int pipe_for(int KP, int req) { return KP > 64 ? 0 : (req > 0 ? req : 2); }

// Resident waves per SIMD of the fused kernels by padded component count
// (from their register use).
int occupancy_for(int KP) { return KP <= 64 ? 2 : 1; }
constexpr int SIMDS = 1024;  // 256 compute units x 4

PassCfg cfg_whole(int col_tiles, int RT, int KP, int req_nw) {
  PassCfg c;
  const int cap = SIMDS * occupancy_for(KP);
  c.nw = KP >= 128 ? 2 : 1;  // one wave per workgroup spills at KP = 128
  if (req_nw > 0) {
    c.nw = req_nw;
  } else {
    for (int nw : {4, 2}) {
      if ((int64_t)col_tiles * nw <= cap && RT >= nw) {
        c.nw = nw;
        break;
      }
    }
  }
  c.splits = 1;
  c.tiles_per_split = RT;
  c.pipe = pipe_for(KP, 0);
  return c;
}

PassCfg cfg_split(int col_tiles, int RT, int KP, int req_split, int req_nw) {
  PassCfg c;
  c.nw = req_nw > 0 ? req_nw : 4;
  const int cap = SIMDS * occupancy_for(KP);
  int S = req_split > 0 ? req_split : std::max(1, cap / std::max(1, col_tiles * c.nw));
  S = std::min(S, std::max(1, RT / c.nw));
  c.tiles_per_split = (RT + S - 1) / S;
  c.splits = (RT + c.tiles_per_split - 1) / c.tiles_per_split;
  c.pipe = pipe_for(KP, 0);
  return c;
}

DualArgs pass_args(const float* D, const float* Mw, int RT, int C_pad, int C_valid, const Factor& L,
                   const float* Rt, int K, float eps) {
  DualArgs a{};
  a.D = D;
  a.Mw = Mw;
  a.RT = RT;
  a.tiles_per_split = RT;
  a.C_pad = C_pad;
  a.C_valid = C_valid;
  a.L = L.m;
  a.Lh = L.mh;
  a.Ll = L.ml;
  a.LT = L.tp;
  a.LTh = L.tph;
  a.LTl = L.tpl;
  a.ldlt = L.rows_pad;
  a.Rt = Rt;
  a.ldr = C_pad;
  a.K = K;
  a.eps = eps;
  return a;
}

FinishArgs finish_args(const float* partial, int S, const Factor& f, int C_valid, int K,
                       float eps, int prec) {
  FinishArgs a{};
  a.partial = partial;
  a.S = S;
  a.KP = f.KP;
  a.C_pad = f.rows_pad;
  a.C_valid = C_valid;
  a.K = K;
  a.eps = eps;
  a.prec = prec;
  a.m = f.m;
  a.mh = f.mh;
  a.ml = f.ml;
  a.t = f.t;
  a.tp = f.tp;
  a.tph = f.tph;
  a.tpl = f.tpl;
  return a;
}

constexpr int GRAM_K_MAX = 200;  // G (K x K FP32) must fit the 160 KB LDS

struct GramCall {
  const float* H = nullptr;
  int K = 0;
  int64_t p = 0, f = 0;
  const float* T = nullptr;   // dense frames
  const float* MT = nullptr;
  const int64_t* offsets = nullptr;  // CSR frames
  int64_t nnz = 0;
  const int32_t* pix = nullptr;
  const float* val = nullptr;
  const float* wt = nullptr;
  const nmf_params* prm = nullptr;
  const float* C_init = nullptr;
  float* C_out = nullptr;
  uint64_t* ticks = nullptr;
};

// Masked-Gram projection of dense or CSR frames: H layouts, (for CSR) the
// longest-first order, and the persistent kernel, captured as one graph.
int project_gram(nmf_handle h, const GramCall& c, hipStream_t s, nmf_report* rep) {
  const bool ragged = c.offsets != nullptr;
  const int K = c.K, KP = kp_for(K);
  const int p_pad = round_up(c.p, 32);
  DeviceGuard g(h->device);
  if (!g.ok) return fail(NMF_ERR_HIP, "hipSetDevice failed");
  int rc;
  Factor Hf;
  int *queue, *stat, *order = nullptr;
  if ((rc = factor_alloc(h, "GH", (int)c.p, p_pad, KP, &Hf)) || (rc = ws(h, "gqueue", 1, &queue)) ||
      (rc = ws(h, "gstat", 1, &stat)))
    return rc;
  const bool sorted = ragged && c.f <= MAX_SORT_FRAMES && c.f > 1;
  if (sorted && (rc = ws(h, "gorder", (size_t)c.f, &order))) return rc;
  GramArgs a{};
  a.HT = Hf.m;
  a.K = K;
  a.P = (int)c.p;
  a.F = (int)c.f;
  a.T = c.T;
  a.MT = c.MT;
  a.offsets = c.offsets;
  a.nnz = c.nnz;
  a.pix = c.pix;
  a.val = c.val;
  a.wt = c.wt;
  a.order = order;
  a.C_init = c.C_init;
  a.seed = c.prm->seed;
  a.iters = c.prm->max_iter;
  a.eps = c.prm->floor_eps;
  a.clip_negative = (c.prm->flags & NMF_F_CLIP_NEGATIVE) ? 1 : 0;
  a.C_out = c.C_out;
  a.queue = queue;
  a.status = stat;
  a.ticks = c.ticks;
  const FactorFillArgs fa = fill_args(Hf, c.H, 1, 0, 1, K);
  auto enqueue = [&](hipStream_t s) -> hipError_t {
    hipError_t e;
    if ((e = timed(h, NMF_K_OTHER, s, [&]() { return launch_set_int(queue, 0, s); }))) return e;
    if ((e = timed(h, NMF_K_OTHER, s, [&]() { return launch_set_int(stat, 0, s); }))) return e;
    if ((e = timed(h, NMF_K_OTHER, s, [&]() { return launch_factor_fill(fa, s); }))) return e;
    if (sorted &&
        (e = timed(h, NMF_K_OTHER, s, [&]() { return launch_frame_order(c.offsets, a.F, order, s); })))
      return e;
    return timed(h, NMF_K_PROJECT, s, [&]() { return launch_gram(KP, ragged, a, 0, s, nullptr); });
  };
  const std::string key =
      key_of(ragged ? "gramR" : "gramD",
             {(uint64_t)c.H, (uint64_t)K, (uint64_t)c.p, (uint64_t)c.f, (uint64_t)c.T,
              (uint64_t)c.MT, (uint64_t)c.offsets, (uint64_t)c.nnz, (uint64_t)c.pix,
              (uint64_t)c.val, (uint64_t)c.wt, (uint64_t)c.C_init, (uint64_t)c.C_out,
              (uint64_t)c.ticks, (uint64_t)c.prm->seed, (uint64_t)c.prm->max_iter,
              (uint64_t)c.prm->flags, (uint64_t)__builtin_bit_cast(uint32_t, c.prm->floor_eps),
              (uint64_t)Hf.m, (uint64_t)queue, (uint64_t)stat, (uint64_t)order});
  HIP_TRY(hipEventRecord(h->ev0, s));
  HIP_TRY(run_graph(h, key, s, enqueue));
  HIP_TRY(hipEventRecord(h->ev1, s));
  if (c.prm->flags & NMF_F_ASYNC) return NMF_OK;
  int st = 0;
  HIP_TRY(hipMemcpyAsync(&st, stat, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  if (st & 16) return fail(NMF_ERR_ARG, "CSR offsets or pixel indices out of range");
  if (c.prm->flags & NMF_F_VALIDATE_DATA) {
    if ((rc = status_from_stage(st))) return rc;
  } else if ((rc = status_from_stage(st & 4))) {
    return rc;
  }
  if (rep) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
    rep->iters_run = c.prm->max_iter;
    rep->status_flags = 0;
    rep->objective = 0.0;
    rep->objective_rel = 0.0;
    rep->elapsed_ms = ms;
  }
  return NMF_OK;
}

}  // namespace

extern "C" {

int nmf_objective(nmf_handle h, const float* V, const float* M, const float* W, const float* H,
                  int64_t n, int64_t p, int32_t k, int32_t precision, double* J_out,
                  void* stream) {
  if (!V || !M || !W || !H || !J_out) return fail(NMF_ERR_ARG, "NULL array argument");
  int rc = check_dims(n, p, "objective");
  if (rc) return rc;
  if (k < 1 || k > n || k > p) return fail(NMF_ERR_ARG, "k must be in [1, min(n, p)]");
  if (precision != NMF_PREC_FP32 && precision != NMF_PREC_BF16X3)
    return fail(NMF_ERR_ARG, "unknown precision");
  const int KP = kp_for(k);
  if (KP > KP_MAX) return fail(NMF_ERR_UNSUPPORTED, "k > 128 is not supported by this build");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  const int n_pad = round_up(n, 32), p_pad = round_up(p, 32);
  float *D, *Mw;
  double *part, *Jdev;
  int* stat;
  Factor Wf, Hf;
  const int nblk = std::max((n_pad / 32) * (p_pad / 32), p_pad / 32);
  if ((rc = ws(h, "D", (size_t)n_pad * p_pad, &D)) || (rc = ws(h, "Mw", (size_t)n_pad * p_pad, &Mw)) ||
      (rc = ws(h, "stat", 1, &stat)) || (rc = ws(h, "Jdev", 2, &Jdev)) ||
      (rc = ws(h, "part", (size_t)nblk, &part)) ||
      (rc = factor_alloc(h, "W", (int)n, n_pad, KP, &Wf)) ||
      (rc = factor_alloc(h, "H", (int)p, p_pad, KP, &Hf)))
    return rc;
  HIP_TRY(hipMemsetAsync(stat, 0, sizeof(int), s));
  StageArgs sa{V, M, n, p, n_pad, p_pad, 0, D, Mw, nullptr, nullptr, stat, part};
  int sblocks = 0;
  LAUNCH(NMF_K_OTHER, launch_stage(sa, &sblocks, s));
  LAUNCH(NMF_K_OTHER, launch_factor_fill(fill_args(Wf, W, 0, 0, 0, k), s));
  LAUNCH(NMF_K_OTHER, launch_factor_fill(fill_args(Hf, H, 1, 0, 1, k), s));
  DualArgs a = pass_args(D, Mw, n_pad / 32, p_pad, (int)p, Wf, Hf.t, k, 0.f);
  a.Jpart = part;
  const PassCfg pc = cfg_whole(p_pad / 32, n_pad / 32, KP, 0);
  LAUNCH(NMF_K_OBJECTIVE, launch_dual(precision, KP, MODE_OBJ, pc.nw, pc.pipe, a, p_pad / 32, 1, s));
  LAUNCH(NMF_K_OTHER, launch_reduce_f64(part, p_pad / 32, Jdev, nullptr, s));
  int st = 0;
  HIP_TRY(hipMemcpyAsync(&st, stat, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(J_out, Jdev, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  return status_from_stage(st & 4);
}

// ---------------------------------------------------------------------------
int nmf_build_basis(nmf_handle h, const float* V, const float* M, int64_t n, int64_t p,
                    const nmf_params* prm, const float* W_init, const float* H_init,
                    float* W_out, float* H_out, double* obj_hist, nmf_report* rep,
                    void* stream) {
  if (!V || !M || !W_out || !H_out) return fail(NMF_ERR_ARG, "NULL array argument");
  int rc = check_dims(n, p, "build_basis");
  if (rc) return rc;
  if ((rc = check_params(prm, n, p, true))) return rc;
  if (rep && rep->struct_size != sizeof(nmf_report))
    return fail(NMF_ERR_ARG, "nmf_report.struct_size mismatch");
  if ((const float*)W_out == V || (const float*)W_out == M || (const float*)H_out == V ||
      (const float*)H_out == M || W_out == H_out || (W_init && W_init == H_out) ||
      (H_init && H_init == W_out))
    return fail(NMF_ERR_ARG, "forbidden aliasing between arguments");
  const int K = prm->k;
  const int KP = kp_for(K);
  if (KP > KP_MAX) return fail(NMF_ERR_UNSUPPORTED, "k > 128 is not supported by this build");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  const int T = prm->max_iter;
  const int prec = prm->precision;
  const float eps = prm->floor_eps;
  DeviceGuard g(h->device);
  if (!g.ok) return fail(NMF_ERR_HIP, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;

  const int n_pad = round_up(n, 32), p_pad = round_up(p, 32);
  const int ntile = n_pad / 32, ptile = p_pad / 32;
  PassCfg ca = cfg_whole(ptile, ntile, KP, prm->waves);
  PassCfg cb = cfg_split(ntile, ptile, KP, prm->split, prm->waves);
  ca.pipe = cb.pipe = pipe_for(KP, prm->pipeline);

  float *D, *Mw, *DT, *MwT, *partial;
  double *part, *Jhist, *sum_mv2;
  int *stat, *iter;
  Factor Wf, Hf;
  const size_t nel = (size_t)n_pad * p_pad;
  const int nblk = std::max(ntile * ptile, ptile);
  if ((rc = ws(h, "D", nel, &D)) || (rc = ws(h, "Mw", nel, &Mw)) || (rc = ws(h, "DT", nel, &DT)) ||
      (rc = ws(h, "MwT", nel, &MwT)) ||
      (rc = ws(h, "partial", (size_t)cb.splits * 2 * KP * n_pad, &partial)) ||
      (rc = ws(h, "part", (size_t)nblk, &part)) || (rc = ws(h, "Jhist", (size_t)T + 2, &Jhist)) ||
      (rc = ws(h, "summv2", 1, &sum_mv2)) || (rc = ws(h, "stat", 1, &stat)) ||
      (rc = ws(h, "iter", 1, &iter)) ||
      (rc = factor_alloc(h, "W", (int)n, n_pad, KP, &Wf)) ||
      (rc = factor_alloc(h, "H", (int)p, p_pad, KP, &Hf)))
    return rc;
  double* hostJ = nullptr;
  if ((rc = pinned_get(h, (size_t)T + 2, &hostJ))) return rc;

  HIP_TRY(hipEventRecord(h->ev0, s));
  HIP_TRY(hipMemsetAsync(stat, 0, sizeof(int), s));
  LAUNCH(NMF_K_OTHER, launch_set_int(iter, 0, s));
  StageArgs sa{V, M, n, p, n_pad, p_pad, (prm->flags & NMF_F_CLIP_NEGATIVE) ? 1 : 0,
               D, Mw, DT, MwT, stat, part};
  int sblocks = 0;
  LAUNCH(NMF_K_OTHER, launch_stage(sa, &sblocks, s));
  LAUNCH(NMF_K_OTHER, launch_reduce_f64(part, sblocks, sum_mv2, nullptr, s));
  LAUNCH(NMF_K_OTHER, launch_factor_fill(fill_args(Wf, W_init, 0, prm->seed, 0, K), s));
  LAUNCH(NMF_K_OTHER, launch_factor_fill(fill_args(Hf, H_init, 1, prm->seed, 1, K), s));

  if ((prm->flags & NMF_F_VALIDATE_DATA) && !(prm->flags & NMF_F_ASYNC)) {
    int st = 0;
    HIP_TRY(hipMemcpyAsync(&st, stat, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if ((rc = status_from_stage(st))) return rc;
  }

  // H-rule over V: one workgroup per 32-pixel tile, all images.
  DualArgs A = pass_args(D, Mw, ntile, p_pad, (int)p, Wf, Hf.t, K, eps);
  A.Jpart = part;
  A.Rt_out = Hf.t;
  A.RtT = Hf.m;
  A.RtTh = Hf.mh;
  A.RtTl = Hf.ml;
  A.Rtp = Hf.tp;
  A.Rtph = Hf.tph;
  A.Rtpl = Hf.tpl;
  // W-rule over V^T: 32-image tiles x chunks of pixel tiles, then the finish.
  DualArgs B = pass_args(DT, MwT, ptile, n_pad, (int)n, Hf, Wf.t, K, eps);
  B.tiles_per_split = cb.tiles_per_split;
  B.partial = partial;
  FinishArgs F = finish_args(partial, cb.splits, Wf, (int)n, K, eps, prec);
  F.Jpart = part;
  F.nJ = ptile;
  F.Jhist = Jhist;
  F.iter = iter;
  F.status = stat;

  const int c = (prm->tol > 0.0 && prm->check_every > 0) ? prm->check_every : 0;
  // Iterations run as replays of a captured graph of ``chunk`` iterations
  // (the finish kernel advances the device iteration counter, so every
  // chunk is the same launch sequence).
  const int chunk = c ? c : std::min(T, 64);
  auto enqueue_iters = [&](hipStream_t s, int count) -> hipError_t {
    hipError_t e;
    for (int i = 0; i < count; ++i) {
      if ((e = timed(h, NMF_K_HRULE, s,
                     [&]() { return launch_dual(prec, KP, MODE_UPDATE, ca.nw, ca.pipe, A, ptile, 1, s); })))
        return e;
      if ((e = timed(h, NMF_K_WRULE, s, [&]() {
             return launch_dual(prec, KP, MODE_SPLIT, cb.nw, cb.pipe, B, ntile, cb.splits, s);
           })))
        return e;
      if ((e = timed(h, NMF_K_WFINISH, s, [&]() { return launch_finish(F, s); }))) return e;
    }
    return hipSuccess;
  };
  auto iter_key = [&](int count) {
    return key_of("iters", {(uint64_t)D, (uint64_t)DT, (uint64_t)Wf.m, (uint64_t)Hf.m,
                            (uint64_t)partial, (uint64_t)part, (uint64_t)Jhist, (uint64_t)iter,
                            (uint64_t)stat, (uint64_t)n, (uint64_t)p, (uint64_t)K,
                            (uint64_t)prec, (uint64_t)__builtin_bit_cast(uint32_t, eps),
                            (uint64_t)ca.nw, (uint64_t)cb.nw, (uint64_t)cb.splits,
                            (uint64_t)count});
  };
  int t = 0;
  bool stopped = false;
  int pending_check = -1;  // iteration whose J copy is in flight
  hipEvent_t chk = nullptr;
  if (c) HIP_TRY(hipEventCreateWithFlags(&chk, hipEventDisableTiming));
  while (t < T) {
    const int count = std::min(chunk, T - t);
    HIP_TRY(run_graph(h, iter_key(count), s, [&](hipStream_t st) { return enqueue_iters(st, count); }));
    t += count;
    if (!c) continue;
    // J of the last iteration of a chunk is known once that chunk completes;
    // decide on the previous chunk's value so that one chunk stays queued.
    if (pending_check >= 0) {
      HIP_TRY(hipEventSynchronize(chk));
      const int t1 = pending_check;
      if (t1 >= c) {
        const double j0 = hostJ[t1 - c], j1 = hostJ[t1];
        if (!std::isfinite(j1)) break;
        if (j0 > 0 && (j0 - j1) / j0 < prm->tol) {
          stopped = true;
          break;
        }
      }
    }
    HIP_TRY(hipMemcpyAsync(hostJ + (t - 1), Jhist + (t - 1), sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(chk, s));
    pending_check = t - 1;
  }
  if (chk) {
    (void)hipEventSynchronize(chk);
    (void)hipEventDestroy(chk);
  }
  const int iters_run = t;
  // Objective after the last iteration.
  LAUNCH(NMF_K_OBJECTIVE, launch_dual(prec, KP, MODE_OBJ, ca.nw, ca.pipe, A, ptile, 1, s));
  LAUNCH(NMF_K_OTHER, launch_reduce_f64(part, ptile, Jhist + iters_run, stat, s));
  if (prm->flags & NMF_F_NORMALIZE_H) LAUNCH(NMF_K_OTHER, launch_normalize(Hf.t, KP, p_pad, K, Wf.t, n_pad, s));
  LAUNCH(NMF_K_OTHER, launch_factor_out(Wf.t, (int)n, n_pad, K, KP, 0, W_out, s));
  LAUNCH(NMF_K_OTHER, launch_factor_out(Hf.t, (int)p, p_pad, K, KP, 1, H_out, s));
  HIP_TRY(hipEventRecord(h->ev1, s));
  if (prm->flags & NMF_F_ASYNC) {
    if (rep) {
      rep->iters_run = iters_run;
      rep->status_flags = 0;
    }
    return NMF_OK;
  }
  int st = 0;
  double mv2 = 0.0;
  HIP_TRY(hipMemcpyAsync(&st, stat, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&mv2, sum_mv2, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hostJ, Jhist, sizeof(double) * (iters_run + 1), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
  if (obj_hist) std::memcpy(obj_hist, hostJ, sizeof(double) * (iters_run + 1));
  if (prm->flags & NMF_F_VALIDATE_DATA) {
    if ((rc = status_from_stage(st))) return rc;
  } else if ((rc = status_from_stage(st & 4))) {
    return rc;
  }
  int result = NMF_OK;
  int warn = 0;
  for (int i = 0; i <= iters_run; ++i)
    if (!std::isfinite(hostJ[i])) return fail(NMF_ERR_DIVERGED, "objective became non-finite");
  for (int i = 0; i < iters_run; ++i)
    if (hostJ[i + 1] > hostJ[i] * (1.0 + 1e-5) + 1e-300) warn |= 1 << NMF_WARN_NONMONOTONE;
  if (c && !stopped && iters_run == T) warn |= 1 << NMF_WARN_MAXITER;
  if (warn & (1 << NMF_WARN_NONMONOTONE)) result = NMF_WARN_NONMONOTONE;
  else if (warn & (1 << NMF_WARN_MAXITER)) result = NMF_WARN_MAXITER;
  if (rep) {
    rep->iters_run = iters_run;
    rep->status_flags = warn;
    rep->objective = hostJ[iters_run];
    rep->objective_rel = mv2 > 0 ? hostJ[iters_run] / mv2 : 0.0;
    rep->elapsed_ms = ms;
  }
  return result;
}

// ---------------------------------------------------------------------------
int nmf_project(nmf_handle h, const float* H, int64_t k, int64_t p, const float* T,
                const float* M_T, int64_t f, const nmf_params* prm, const float* C_init,
                float* C_out, double* obj_out, nmf_report* rep, void* stream) {
  if (!H || !T || !M_T || !C_out) return fail(NMF_ERR_ARG, "NULL array argument");
  int rc = check_dims(f, p, "project");
  if (rc) return rc;
  if ((rc = check_params(prm, f, p, false))) return rc;
  if (prm->k != k) return fail(NMF_ERR_ARG, "params.k must equal k");
  if (k > p) return fail(NMF_ERR_ARG, "k must not exceed p");
  if (rep && rep->struct_size != sizeof(nmf_report))
    return fail(NMF_ERR_ARG, "nmf_report.struct_size mismatch");
  if ((const float*)C_out == H || (const float*)C_out == T || (const float*)C_out == M_T)
    return fail(NMF_ERR_ARG, "forbidden aliasing between arguments");
  const int K = (int)k;
  const int KP = kp_for(K);
  if (prm->flags & NMF_F_MASKED_GRAM) {
    if (K > GRAM_K_MAX) return fail(NMF_ERR_UNSUPPORTED, "masked-Gram projection needs k <= 200");
    if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
    GramCall gc{};
    gc.H = H;
    gc.K = K;
    gc.p = p;
    gc.f = f;
    gc.T = T;
    gc.MT = M_T;
    gc.prm = prm;
    gc.C_init = C_init;
    gc.C_out = C_out;
    int rc2 = project_gram(h, gc, (hipStream_t)stream, rep);
    if (rc2 < 0 || !obj_out) return rc2;
    DeviceGuard g(h->device);
    hipStream_t s = (hipStream_t)stream;
    LAUNCH(NMF_K_OTHER, launch_frame_objective(H, C_out, T, M_T, f, K, p, obj_out, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(prof_drain(h));
    return rc2;
  }
  if (KP > KP_MAX) return fail(NMF_ERR_UNSUPPORTED, "k > 128 is not supported by this build");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  const int prec = prm->precision;
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  const int f_pad = round_up(f, 32), p_pad = round_up(p, 32);
  const int ftile = f_pad / 32, ptile = p_pad / 32;
  PassCfg cb = cfg_split(ftile, ptile, KP, prm->split, prm->waves);
  cb.pipe = pipe_for(KP, prm->pipeline);
  float *DT, *MwT, *partial;
  double* part;
  int* stat;
  Factor Cf, Hf;
  const size_t nel = (size_t)f_pad * p_pad;
  if ((rc = ws(h, "pDT", nel, &DT)) || (rc = ws(h, "pMwT", nel, &MwT)) ||
      (rc = ws(h, "ppartial", (size_t)cb.splits * 2 * KP * f_pad, &partial)) ||
      (rc = ws(h, "ppart", (size_t)ftile * ptile, &part)) ||
      (rc = ws(h, "stat", 1, &stat)) || (rc = factor_alloc(h, "C", (int)f, f_pad, KP, &Cf)) ||
      (rc = factor_alloc(h, "PH", (int)p, p_pad, KP, &Hf)))
    return rc;
  HIP_TRY(hipEventRecord(h->ev0, s));
  HIP_TRY(hipMemsetAsync(stat, 0, sizeof(int), s));
  StageArgs sa{T, M_T, f, p, f_pad, p_pad, (prm->flags & NMF_F_CLIP_NEGATIVE) ? 1 : 0,
               nullptr, nullptr, DT, MwT, stat, part};
  int sblocks = 0;
  LAUNCH(NMF_K_OTHER, launch_stage(sa, &sblocks, s));
  LAUNCH(NMF_K_OTHER, launch_factor_fill(fill_args(Hf, H, 1, 0, 1, K), s));
  LAUNCH(NMF_K_OTHER, launch_factor_fill(fill_args(Cf, C_init, 0, prm->seed, 2, K), s));
  if ((prm->flags & NMF_F_VALIDATE_DATA) && !(prm->flags & NMF_F_ASYNC)) {
    int st = 0;
    HIP_TRY(hipMemcpyAsync(&st, stat, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if ((rc = status_from_stage(st))) return rc;
  }
  DualArgs B = pass_args(DT, MwT, ptile, f_pad, (int)f, Hf, Cf.t, K, prm->floor_eps);
  B.tiles_per_split = cb.tiles_per_split;
  B.partial = partial;
  FinishArgs F = finish_args(partial, cb.splits, Cf, (int)f, K, prm->floor_eps, prec);
  for (int it = 0; it < prm->max_iter; ++it) {
    LAUNCH(NMF_K_PROJECT, launch_dual(prec, KP, MODE_SPLIT, cb.nw, cb.pipe, B, ftile, cb.splits, s));
    LAUNCH(NMF_K_PROJECT, launch_finish(F, s));
  }
  LAUNCH(NMF_K_OTHER, launch_factor_out(Cf.t, (int)f, f_pad, K, KP, 0, C_out, s));
  if (obj_out) LAUNCH(NMF_K_OTHER, launch_frame_objective(H, C_out, T, M_T, f, K, p, obj_out, s));
  HIP_TRY(hipEventRecord(h->ev1, s));
  if (prm->flags & NMF_F_ASYNC) return NMF_OK;
  int st = 0;
  HIP_TRY(hipMemcpyAsync(&st, stat, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  if (prm->flags & NMF_F_VALIDATE_DATA) {
    if ((rc = status_from_stage(st))) return rc;
  } else if ((rc = status_from_stage(st & 4))) {
    return rc;
  }
  if (rep) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
    rep->iters_run = prm->max_iter;
    rep->status_flags = 0;
    rep->objective = 0.0;
    rep->objective_rel = 0.0;
    rep->elapsed_ms = ms;
  }
  return NMF_OK;
}

int nmf_project_ragged(nmf_handle h, const float* H, int64_t k, int64_t p, int64_t f,
                       const int64_t* offsets, int64_t nnz, const int32_t* pix,
                       const float* val, const float* wt, const nmf_params* prm,
                       const float* C_init, float* C_out, uint64_t* frame_ticks,
                       nmf_report* rep, void* stream) {
  if (!H || !offsets || !C_out || (nnz > 0 && (!pix || !val)))
    return fail(NMF_ERR_ARG, "NULL array argument");
  int rc = check_dims(f, p, "project_ragged");
  if (rc) return rc;
  if (f > 0x7fffffff || p > 0x7fffffff) return fail(NMF_ERR_SHAPE, "f and p must fit in int32");
  if (nnz < 0) return fail(NMF_ERR_SHAPE, "nnz must be >= 0");
  if ((rc = check_params(prm, f, p, false))) return rc;
  if (prm->k != k) return fail(NMF_ERR_ARG, "params.k must equal k");
  if (k > p) return fail(NMF_ERR_ARG, "k must not exceed p");
  if (k > GRAM_K_MAX) return fail(NMF_ERR_UNSUPPORTED, "ragged projection needs k <= 200");
  if (prm->precision != NMF_PREC_FP32)
    return fail(NMF_ERR_UNSUPPORTED, "ragged projection runs FP32 products in this build");
  if (rep && rep->struct_size != sizeof(nmf_report))
    return fail(NMF_ERR_ARG, "nmf_report.struct_size mismatch");
  if ((const float*)C_out == H || (const float*)C_out == val || (const float*)C_out == wt)
    return fail(NMF_ERR_ARG, "forbidden aliasing between arguments");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  GramCall gc{};
  gc.H = H;
  gc.K = (int)k;
  gc.p = p;
  gc.f = f;
  gc.offsets = offsets;
  gc.nnz = nnz;
  gc.pix = pix;
  gc.val = val;
  gc.wt = wt;
  gc.prm = prm;
  gc.C_init = C_init;
  gc.C_out = C_out;
  gc.ticks = frame_ticks;
  return project_gram(h, gc, (hipStream_t)stream, rep);
}

double nmf_device_clock_khz(nmf_handle h) {
  if (!h) return 0.0;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device) != hipSuccess)
    return 0.0;
  return (double)khz;
}

// ---------------------------------------------------------------------------
int nmf_subtract(nmf_handle h, const float* H, const float* C, const float* T, const float* M_T,
                 int64_t f, int64_t k, int64_t p, const float* scale, float* model_out,
                 float* resid_out, void* stream) {
  if (!H || !C || !T || !M_T || !resid_out) return fail(NMF_ERR_ARG, "NULL array argument");
  int rc = check_dims(f, p, "subtract");
  if (rc) return rc;
  if (k < 1 || k > 4096) return fail(NMF_ERR_ARG, "k must be in [1, 4096]");
  if (f > 65535) return fail(NMF_ERR_SHAPE, "more than 65535 frames per call");
  if ((const float*)resid_out == T || (const float*)resid_out == M_T || resid_out == model_out ||
      (const float*)resid_out == H || (const float*)resid_out == C)
    return fail(NMF_ERR_ARG, "forbidden aliasing between arguments");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  LAUNCH(NMF_K_SUBTRACT, launch_subtract(H, C, T, M_T, f, (int)k, p, scale, model_out, resid_out, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  return NMF_OK;
}

int nmf_profile_enable(nmf_handle h, int on) {
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  HIP_TRY(prof_drain(h));
  h->prof = on != 0;
  if (h->prof)
    for (int i = 0; i < NMF_K_COUNT; ++i) {
      h->prof_ms[i] = 0.0;
      h->prof_n[i] = 0;
    }
  return NMF_OK;
}

int nmf_profile_get(nmf_handle h, int32_t kernel_class, int64_t* count, double* total_ms) {
  if (kernel_class < 0 || kernel_class >= NMF_K_COUNT)
    return fail(NMF_ERR_ARG, "kernel_class out of range");
  if (!count || !total_ms) return fail(NMF_ERR_ARG, "NULL output");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  HIP_TRY(prof_drain(h));
  *count = h->prof_n[kernel_class];
  *total_ms = h->prof_ms[kernel_class];
  return NMF_OK;
}

}  // extern "C"
