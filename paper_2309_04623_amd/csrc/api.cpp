// Host side of the C ABI declared in include/nmf_mi355x.h: argument checks,
// the device workspace, iteration control and kernel sequencing.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/nmf_mi355x.h"
#include "device_common.hpp"
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

// Scratch memory of the allocation-free entry point (nmf_closest_frames_noalloc):
// a file-scope device array, one copy per GPU the library runs on, held
// until the process ends.  Host code never uses the array's name as an
// address: each device's copy is located once with hipGetSymbolAddress (at
// the first nmf_create on that device) and only that address is used.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(16) << 20;
constexpr size_t NOALLOC_STATUS_BYTES = 256;  // status word, then the distances
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
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
  // autotuned launch shapes: key -> (waves, pipeline, splits, microseconds)
  struct Tuned {
    int nw, pipe, splits;
    float us;
  };
  std::unordered_map<std::string, Tuned> tuned;
  int64_t last_fallbacks = -1;  // frames of the last warm start that fell back
  std::vector<int32_t> last_frame_iters;  // of the last Gram projection with a stop rule
  std::vector<int32_t> last_frame_visits;  // of the last Gram projection
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
  if (prm->pipeline < 0 || prm->pipeline > 3) return fail(NMF_ERR_ARG, "pipeline must be 0..3");
  return NMF_OK;
}

int kp_for(int k) { return round_up(k, 32); }
constexpr int KP_MAX = 224;  // K <= 224
constexpr int KP_WIDE = 96;   // from here on the wide-basis half-step runs
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
  if (hip_device < MAX_DEVICES) {
    // once per device, with that device current: the address of this
    // device's copy of the scratch array
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[hip_device]) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        (void)hipStreamDestroy(h->cap);
        (void)hipEventDestroy(h->ev0);
        (void)hipEventDestroy(h->ev1);
        delete h;
        return fail(NMF_ERR_HIP, "hipGetSymbolAddress of the scratch array failed");
      }
      g_scratch_ptr[hip_device] = ptr;
    }
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

// Default launch shapes (measured on the STIS-shaped workload, 500 x 40000,
// K = 30): the update pass runs four waves per workgroup in FP32 and one in
// bf16x3 (whose fused kernel then stays at two waves per SIMD); the split pass
// takes about one workgroup per compute unit, four waves (FP32) or two
// (bf16x3).  The autotuner replaces these per shape on request.
PassCfg cfg_whole(int col_tiles, int RT, int KP, int prec, int req_nw) {
  PassCfg c;
  if (KP >= KP_WIDE) {  // one workgroup per four column tiles, all rows
    c.nw = 4;
    c.splits = 1;
    c.tiles_per_split = RT;
    c.pipe = 0;
    return c;
  }
  const int cap = SIMDS * occupancy_for(KP);
  c.nw = KP >= 128 ? 2 : 1;  // one wave per workgroup spills at KP = 128
  if (req_nw > 0) {
    c.nw = req_nw;
  } else if (KP <= 64 && prec == NMF_PREC_FP32 && RT >= 4) {
    c.nw = 4;
  } else if (KP > 64) {
    for (int nw : {4, 2}) {
      if ((int64_t)col_tiles * nw <= cap && RT >= nw) {
        c.nw = nw;
        break;
      }
    }
  }
  c.splits = 1;
  c.tiles_per_split = RT;
  c.pipe = KP > 64 ? 0 : (prec == NMF_PREC_FP32 ? 2 : 1);
  return c;
}

PassCfg cfg_split(int col_tiles, int RT, int KP, int prec, int req_split, int req_nw) {
  PassCfg c;
  if (KP >= KP_WIDE) {
    // about one workgroup (four waves, one per SIMD) per compute unit
    const int groups = wide_groups(col_tiles);
    int S = req_split > 0 ? req_split : std::max(1, (256 + groups - 1) / groups);
    S = std::min(S, std::max(1, RT / 2));
    c.nw = 4;
    c.tiles_per_split = (RT + S - 1) / S;
    c.splits = (RT + c.tiles_per_split - 1) / c.tiles_per_split;
    c.pipe = 0;
    return c;
  }
  c.nw = req_nw > 0 ? req_nw : (prec == NMF_PREC_FP32 || KP > 64 ? 4 : 2);
  int S = req_split > 0 ? req_split : std::max(1, 256 / std::max(1, col_tiles));
  S = std::min(S, std::max(1, RT / c.nw));
  c.tiles_per_split = (RT + S - 1) / S;
  c.splits = (RT + c.tiles_per_split - 1) / c.tiles_per_split;
  c.pipe = pipe_for(KP, 0);
  return c;
}

// Launches one fused half-step over ``col_tiles`` column tiles with the
// shape ``c``: the wide-basis kernel from KP_WIDE components on, else the
// single-column-tile kernel.
hipError_t launch_pass(int prec, int KP, int mode, const PassCfg& c, const DualArgs& a,
                       int col_tiles, hipStream_t s) {
  if (KP >= KP_WIDE) return launch_wide(prec, KP, mode, a, c.splits, s);
  return launch_dual(prec, KP, mode, c.nw, c.pipe, a, col_tiles, c.splits, s);
}

// Number of objective partials (one per workgroup) of a launch_pass.
int pass_blocks(int KP, const PassCfg& c, int col_tiles) {
  return (KP >= KP_WIDE ? wide_groups(col_tiles) : col_tiles) * c.splits;
}

// Times candidate launch shapes of one fused half-step on the staged data
// and returns the fastest; cached per key in the handle.  A pass that may be
// split is timed in split mode, one that updates in place is timed in update
// mode; either way every output goes to a scratch buffer, so nothing the
// iteration reads is written.
int autotune_pass(nmf_handle h, const std::string& key, int prec, int KP, const DualArgs& base,
                  int col_tiles, int RT, bool allow_split, hipStream_t s, PassCfg* out) {
  auto it = h->tuned.find(key);
  if (it != h->tuned.end()) {
    out->nw = it->second.nw;
    out->pipe = it->second.pipe;
    out->splits = it->second.splits;
    out->tiles_per_split = (RT + out->splits - 1) / out->splits;
    return NMF_OK;
  }
  std::vector<int> split_opts = {1};
  if (allow_split)
    for (int sp : {2, 4, 8, 16, 32, 64, 128})
      if (sp <= RT) split_opts.push_back(sp);
  int rc;
  float* scratch = nullptr;
  const int max_split = split_opts.back();
  const size_t plane = (size_t)KP * base.C_pad;
  // update mode: new factor (KP x C) + two FP32 or four bf16 copies + J partials
  const size_t need = allow_split ? (size_t)max_split * 2 * plane : 3 * plane + 2 * (size_t)col_tiles;
  if ((rc = ws(h, "tune.partial", need, &scratch))) return rc;
  const int mode = allow_split ? MODE_SPLIT : MODE_UPDATE;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best = 1e30f;
  PassCfg bc = *out;
  for (int nw : {1, 2, 4}) {
    for (int pipe : {1, 2, 3}) {
      if (KP > 64 && pipe >= 2) continue;
      if (KP >= 128 && nw == 1) continue;
      for (int sp : split_opts) {
        const int tps = (RT + sp - 1) / sp;
        const int S = (RT + tps - 1) / tps;
        if (tps < nw) continue;
        DualArgs a = base;
        a.tiles_per_split = tps;
        if (allow_split) {
          a.partial = scratch;
          a.Jpart = nullptr;
        } else {
          a.Rt_out = scratch;
          a.RtT = scratch + plane;
          a.Rtp = scratch + 2 * plane;
          a.RtTh = (__bf16*)(scratch + plane);
          a.RtTl = a.RtTh + plane;
          a.Rtph = (__bf16*)(scratch + 2 * plane);
          a.Rtpl = a.Rtph + plane;
          a.Jpart = (double*)(scratch + 3 * plane);
        }
        const int pp = pipe_for(KP, pipe);
        hipError_t e = launch_dual(prec, KP, mode, nw, pp, a, col_tiles, S, s);
        if (e != hipSuccess) continue;
        HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r) HIP_TRY(launch_dual(prec, KP, mode, nw, pp, a, col_tiles, S, s));
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        // a split costs an extra finish pass over S partials: charge it
        const float us = ms * 1e3f / 3.f + (sp > 1 ? 0.02f * S : 0.f);
        if (us < best) {
          best = us;
          bc.nw = nw;
          bc.pipe = pp;
          bc.splits = S;
          bc.tiles_per_split = tps;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->tuned[key] = {bc.nw, bc.pipe, bc.splits, best};
  *out = bc;
  return NMF_OK;
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
  const bool sorted = ragged && c.f > 1;
  int* sort_tmp = nullptr;
  if (sorted && (rc = ws(h, "gorder", (size_t)c.f, &order))) return rc;
  if (sorted && c.f > MAX_SORT_FRAMES && (rc = ws(h, "gsorttmp", 4 * (size_t)c.f, &sort_tmp)))
    return rc;
  const bool warm = (c.prm->flags & NMF_F_WARM_START) != 0;
  if (warm && !c.C_init) return fail(NMF_ERR_ARG, "NMF_F_WARM_START needs C_init");
  int* fb = nullptr;
  if (warm && (rc = ws(h, "gfallback", (size_t)c.f, &fb))) return rc;
  // per-frame stop rule: on when tol > 0 and check_every > 0
  const int ce = (c.prm->tol > 0.0 && c.prm->check_every > 0) ? c.prm->check_every : 0;
  int* its = nullptr;
  if (ce && (rc = ws(h, "giters", (size_t)c.f, &its))) return rc;
  int* visits = nullptr;
  if ((rc = ws(h, "gvisits", (size_t)c.f, &visits))) return rc;
  // K <= 128: two launches, G formed by workgroups of four waves, then
  // iterated by small workgroups that keep a row of G per lane (several
  // frames per compute unit)
  const bool two_phase = KP <= 128;
  float *Gf = nullptr, *cf = nullptr;
  double* bf = nullptr;
  if (two_phase && ((rc = ws(h, "gG", (size_t)c.f * K * K, &Gf)) ||
                    (rc = ws(h, "gb", (size_t)c.f * KP, &bf)) ||
                    (rc = ws(h, "gc", (size_t)c.f * KP, &cf))))
    return rc;
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
  a.binary = (c.prm->flags & NMF_F_BINARY_WEIGHTS) ? 1 : 0;
  a.C_out = c.C_out;
  a.queue = queue;
  a.status = stat;
  a.ticks = c.ticks;
  a.warm = warm ? 1 : 0;
  a.fallback = fb;
  a.prec = c.prm->precision;
  a.check_every = ce;
  a.tol2 = ce ? c.prm->tol * c.prm->tol : 0.0;
  a.iters_out = its;
  a.Gf = Gf;
  a.bf = bf;
  a.cf = cf;
  a.visits = visits;
  // rows of H^T gathered two chunks ahead of their use, one for the split
  // form above K = 128 (measured faster there; NMF_F_AUTOTUNE times both)
  a.ahead = (KP > 128 && c.prm->precision == NMF_PREC_BF16X3) ? 1 : 2;
  const FactorFillArgs fa = fill_args(Hf, c.H, 1, 0, 1, K);
  auto enqueue = [&](hipStream_t s) -> hipError_t {
    hipError_t e;
    if ((e = timed(h, NMF_K_OTHER, s, [&]() { return launch_set_int(queue, 0, s); }))) return e;
    if ((e = timed(h, NMF_K_OTHER, s, [&]() { return launch_set_int(stat, 0, s); }))) return e;
    if ((e = timed(h, NMF_K_OTHER, s, [&]() { return launch_fill_int(visits, a.F, 0, s); })))
      return e;
    if ((e = timed(h, NMF_K_OTHER, s, [&]() { return launch_factor_fill(fa, s); }))) return e;
    if (sorted &&
        (e = timed(h, NMF_K_OTHER, s,
                   [&]() { return launch_frame_order(c.offsets, a.F, order, sort_tmp, s); })))
      return e;
    if ((e = timed(h, NMF_K_PROJECT, s,
                   [&]() { return launch_gram(KP, ragged, a, 0, s, nullptr, two_phase); })))
      return e;
    if (!two_phase) return hipSuccess;
    return timed(h, NMF_K_PROJECT, s, [&]() { return launch_gram_iter(KP, a, s); });
  };
  // Autotuning: the gather depth of the pixel loop (rows of H^T one or two
  // chunks ahead of their use) timed on this call's own inputs, the second
  // of two eager runs of the whole sequence per candidate; the choice is
  // cached per shape.  Both depths compute the same bits, and every output
  // is written again by the run that follows.
  if (c.prm->flags & NMF_F_AUTOTUNE) {
    const std::string tkey =
        key_of(ragged ? "gram.csr" : "gram.dense",
               {(uint64_t)K, (uint64_t)c.p, (uint64_t)c.f, (uint64_t)c.nnz,
                (uint64_t)c.prm->precision, (uint64_t)c.prm->max_iter, (uint64_t)ce,
                (uint64_t)(warm ? 1 : 0)});
    auto it = h->tuned.find(tkey);
    if (it != h->tuned.end()) {
      a.ahead = it->second.pipe;
    } else {
      hipEvent_t e0, e1;
      HIP_TRY(hipEventCreate(&e0));
      HIP_TRY(hipEventCreate(&e1));
      float best = 1e30f;
      int best_pf = 2;
      for (int pf : {1, 2}) {
        a.ahead = pf;
        HIP_TRY(enqueue(s));
        HIP_TRY(hipEventRecord(e0, s));
        HIP_TRY(enqueue(s));
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms * 1e3f < best) {
          best = ms * 1e3f;
          best_pf = pf;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      a.ahead = best_pf;
      h->tuned[tkey] = {KP <= 128 ? 4 : 8, best_pf, 1, best};
    }
  }
  const std::string key =
      key_of(ragged ? "gramR" : "gramD",
             {(uint64_t)c.H, (uint64_t)K, (uint64_t)c.p, (uint64_t)c.f, (uint64_t)c.T,
              (uint64_t)c.MT, (uint64_t)c.offsets, (uint64_t)c.nnz, (uint64_t)c.pix,
              (uint64_t)c.val, (uint64_t)c.wt, (uint64_t)c.C_init, (uint64_t)c.C_out,
              (uint64_t)c.ticks, (uint64_t)c.prm->seed, (uint64_t)c.prm->max_iter,
              (uint64_t)c.prm->flags, (uint64_t)c.prm->precision,
              (uint64_t)__builtin_bit_cast(uint32_t, c.prm->floor_eps), (uint64_t)ce,
              __builtin_bit_cast(uint64_t, a.tol2), (uint64_t)its, (uint64_t)Hf.m,
              (uint64_t)queue, (uint64_t)stat, (uint64_t)order, (uint64_t)sort_tmp,
              (uint64_t)fb, (uint64_t)Gf, (uint64_t)bf, (uint64_t)cf, (uint64_t)visits,
              (uint64_t)a.ahead});
  HIP_TRY(hipEventRecord(h->ev0, s));
  HIP_TRY(run_graph(h, key, s, enqueue));
  HIP_TRY(hipEventRecord(h->ev1, s));
  if (c.prm->flags & NMF_F_ASYNC) return NMF_OK;
  int st = 0;
  HIP_TRY(hipMemcpyAsync(&st, stat, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  if (st & 16) return fail(NMF_ERR_ARG, "CSR offsets or pixel indices out of range");
  int64_t nfb = 0;
  std::vector<int> hfb;
  if (warm) {
    hfb.resize((size_t)c.f);
    HIP_TRY(hipMemcpy(hfb.data(), fb, (size_t)c.f * sizeof(int), hipMemcpyDeviceToHost));
    for (int v : hfb) nfb += v != 0;
    h->last_fallbacks = nfb;
  }
  // With a stop rule: iterations per frame (a warm start restarted cold
  // counts both runs); a frame that ran to the cap of its last run did not
  // meet the rule.
  h->last_frame_visits.resize((size_t)c.f);
  HIP_TRY(hipMemcpy(h->last_frame_visits.data(), visits, (size_t)c.f * sizeof(int),
                    hipMemcpyDeviceToHost));
  int iters_run = c.prm->max_iter, unmet = 0;
  h->last_frame_iters.clear();
  if (ce) {
    h->last_frame_iters.resize((size_t)c.f);
    HIP_TRY(hipMemcpy(h->last_frame_iters.data(), its, (size_t)c.f * sizeof(int),
                      hipMemcpyDeviceToHost));
    iters_run = 0;
    for (int64_t i = 0; i < c.f; ++i) {
      const int t = h->last_frame_iters[(size_t)i];
      const int runs = (warm && hfb[(size_t)i] == 2) ? 2 : 1;
      iters_run = std::max(iters_run, t);
      unmet += t == runs * c.prm->max_iter;
    }
  }
  if (c.prm->flags & NMF_F_VALIDATE_DATA) {
    if ((rc = status_from_stage(st))) return rc;
  } else if ((rc = status_from_stage(st & 4))) {
    return rc;
  }
  if (rep) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
    rep->iters_run = iters_run;
    rep->status_flags = (nfb > 0 ? NMF_RS_WARM_FALLBACK : 0) | (unmet ? 1 << NMF_WARN_MAXITER : 0);
    rep->objective = 0.0;
    rep->objective_rel = 0.0;
    rep->elapsed_ms = ms;
  }
  return unmet ? NMF_WARN_MAXITER : NMF_OK;
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
  if (KP > KP_MAX) return fail(NMF_ERR_UNSUPPORTED, "k > 224 is not supported by this build");
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
  const PassCfg pc = cfg_whole(p_pad / 32, n_pad / 32, KP, precision, 0);
  LAUNCH(NMF_K_OBJECTIVE, launch_pass(precision, KP, MODE_OBJ, pc, a, p_pad / 32, s));
  LAUNCH(NMF_K_OTHER, launch_reduce_f64(part, pass_blocks(KP, pc, p_pad / 32), Jdev, nullptr, s));
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
  if (KP > KP_MAX) return fail(NMF_ERR_UNSUPPORTED, "k > 224 is not supported by this build");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  const int T = prm->max_iter;
  const int prec = prm->precision;
  const float eps = prm->floor_eps;
  DeviceGuard g(h->device);
  if (!g.ok) return fail(NMF_ERR_HIP, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;

  const int n_pad = round_up(n, 32), p_pad = round_up(p, 32);
  const int ntile = n_pad / 32, ptile = p_pad / 32;
  PassCfg ca = cfg_whole(ptile, ntile, KP, prec, prm->waves);
  PassCfg cb = cfg_split(ntile, ptile, KP, prec, prm->split, prm->waves);
  if (prm->pipeline > 0) ca.pipe = cb.pipe = pipe_for(KP, prm->pipeline);

  float *D, *Mw, *DT, *MwT, *partial;
  double *part, *Jhist, *sum_mv2;
  int *stat, *iter;
  Factor Wf, Hf;
  const size_t nel = (size_t)n_pad * p_pad;
  const int nblk = std::max(ntile * ptile, ptile);
  const bool binary = (prm->flags & NMF_F_BINARY_WEIGHTS) != 0;
  uint16_t *Bb = nullptr, *BbT = nullptr;
  Mw = MwT = nullptr;
  if (binary) {
    if ((rc = ws(h, "B", nel / 16, &Bb)) || (rc = ws(h, "BT", nel / 16, &BbT))) return rc;
  } else if ((rc = ws(h, "Mw", nel, &Mw)) || (rc = ws(h, "MwT", nel, &MwT))) {
    return rc;
  }
  if ((rc = ws(h, "D", nel, &D)) || (rc = ws(h, "DT", nel, &DT)) ||
      (rc = ws(h, "partial", (size_t)cb.splits * 2 * KP * n_pad, &partial)) ||
      (rc = ws(h, "part", (size_t)nblk, &part)) || (rc = ws(h, "Jhist", (size_t)T + 2, &Jhist)) ||
      (rc = ws(h, "summv2", 1, &sum_mv2)) || (rc = ws(h, "stat", 1, &stat)) ||
      (rc = ws(h, "iter", 4, &iter)) ||
      (rc = factor_alloc(h, "W", (int)n, n_pad, KP, &Wf)) ||
      (rc = factor_alloc(h, "H", (int)p, p_pad, KP, &Hf)))
    return rc;
  double* hostJ = nullptr;
  if ((rc = pinned_get(h, (size_t)T + 3, &hostJ))) return rc;

  // iter[0]: iterations done; iter[1]: stop requested by the stop test;
  // iter[2]: stop seen by an update pass (see the kernels' stop flags)
  int* stop_req = iter + 1;
  int* stop_seen = iter + 2;
  HIP_TRY(hipEventRecord(h->ev0, s));
  HIP_TRY(hipMemsetAsync(stat, 0, sizeof(int), s));
  HIP_TRY(hipMemsetAsync(iter, 0, 4 * sizeof(int), s));
  StageArgs sa{V, M, n, p, n_pad, p_pad, (prm->flags & NMF_F_CLIP_NEGATIVE) ? 1 : 0,
               D, Mw, DT, MwT, stat, part, binary ? 1 : 0, Bb, BbT};
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
  A.Mb = Bb;
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
  B.Mb = BbT;
  B.tiles_per_split = cb.tiles_per_split;
  B.partial = partial;
  // Warm start of the component initialisation (NMF_F_WARM_START with W_init
  // and H_init, e.g. a prior basis and the coefficients a network predicts
  // on it): the supplied start is kept only if its Eq. 2 cost is not above
  // that of the seeded cold start.  Decided once, before the first
  // iteration, with one synchronisation.
  bool fell_back = false;
  if (prm->flags & NMF_F_WARM_START) {
    if (!W_init || !H_init) return fail(NMF_ERR_ARG, "NMF_F_WARM_START needs W_init and H_init");
    double* Jwc;
    if ((rc = ws(h, "Jwarmcold", 2, &Jwc))) return rc;
    const int nO = pass_blocks(KP, ca, ptile);
    // cold start first, then the warm one, which normally stays in place
    for (int w = 0; w < 2; ++w) {
      const FactorFillArgs fw = fill_args(Wf, w ? W_init : nullptr, 0, prm->seed, 0, K);
      const FactorFillArgs fh = fill_args(Hf, w ? H_init : nullptr, 1, prm->seed, 1, K);
      LAUNCH(NMF_K_OTHER, launch_factor_fill(fw, s));
      LAUNCH(NMF_K_OTHER, launch_factor_fill(fh, s));
      LAUNCH(NMF_K_OBJECTIVE, launch_pass(prec, KP, MODE_OBJ, ca, A, ptile, s));
      LAUNCH(NMF_K_OTHER, launch_reduce_f64(part, nO, Jwc + (1 - w), nullptr, s));
    }
    double hj[2] = {0.0, 0.0};  // warm, cold
    HIP_TRY(hipMemcpyAsync(hj, Jwc, sizeof(hj), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    fell_back = !(hj[0] <= hj[1]);  // also for a non-finite warm cost
    if (fell_back) {
      LAUNCH(NMF_K_OTHER, launch_factor_fill(fill_args(Wf, nullptr, 0, prm->seed, 0, K), s));
      LAUNCH(NMF_K_OTHER, launch_factor_fill(fill_args(Hf, nullptr, 1, prm->seed, 1, K), s));
    }
    h->last_fallbacks = fell_back ? 1 : 0;
  }
  if ((prm->flags & NMF_F_AUTOTUNE) && KP < KP_WIDE) {
    const std::string ka = key_of("tuneA", {(uint64_t)n, (uint64_t)p, (uint64_t)KP, (uint64_t)prec});
    const std::string kb = key_of("tuneB", {(uint64_t)n, (uint64_t)p, (uint64_t)KP, (uint64_t)prec});
    if ((rc = autotune_pass(h, ka, prec, KP, A, ptile, ntile, false, s, &ca))) return rc;
    if ((rc = autotune_pass(h, kb, prec, KP, B, ntile, ptile, true, s, &cb))) return rc;
    if ((rc = ws(h, "partial", (size_t)cb.splits * 2 * KP * n_pad, &partial))) return rc;
    B.tiles_per_split = cb.tiles_per_split;
    B.partial = partial;
  }
  FinishArgs F = finish_args(partial, cb.splits, Wf, (int)n, K, eps, prec);
  F.Jpart = part;
  F.nJ = pass_blocks(KP, ca, ptile);
  F.Jhist = Jhist;
  F.iter = iter;
  F.status = stat;

  // Stop rule (Sec. 2: iterate until the change reaches a set value or the
  // iteration cap): evaluated on the device by the finish kernel from the
  // objective history, so no host round trip decides it; once it passes,
  // the remaining launches return at once.
  const int c = (prm->tol > 0.0 && prm->check_every > 0) ? prm->check_every : 0;
  if (c) {
    F.check_every = c;
    F.tol = prm->tol;
    F.stop_req = stop_req;
    F.stop_seen = stop_seen;
    A.stop_req = stop_req;
    A.stop_seen = stop_seen;
    B.stop_req = stop_req;
  }
  // Iterations run as replays of a captured graph of ``chunk`` iterations
  // (the finish kernel advances the device iteration counter, so every
  // chunk is the same launch sequence).
  const int chunk = c ? std::max(c, std::min(T, 64) / c * c) : std::min(T, 64);
  auto enqueue_iters = [&](hipStream_t s, int count) -> hipError_t {
    hipError_t e;
    for (int i = 0; i < count; ++i) {
      if ((e = timed(h, NMF_K_HRULE, s,
                     [&]() { return launch_pass(prec, KP, MODE_UPDATE, ca, A, ptile, s); })))
        return e;
      if ((e = timed(h, NMF_K_WRULE, s, [&]() {
             return launch_pass(prec, KP, MODE_SPLIT, cb, B, ntile, s);
           })))
        return e;
      if ((e = timed(h, NMF_K_WFINISH, s, [&]() { return launch_finish(F, s); }))) return e;
    }
    return hipSuccess;
  };
  // Every value baked into the captured launches is part of the key: buffer
  // addresses (they move when the workspace grows), the weight storage, the
  // launch shapes and the stop rule.
  auto iter_key = [&](int count) {
    return key_of("iters",
                  {(uint64_t)D, (uint64_t)DT, (uint64_t)Mw, (uint64_t)MwT, (uint64_t)Bb,
                   (uint64_t)BbT, (uint64_t)Wf.m, (uint64_t)Wf.mh, (uint64_t)Wf.ml,
                   (uint64_t)Wf.t, (uint64_t)Wf.tp, (uint64_t)Wf.tph, (uint64_t)Wf.tpl,
                   (uint64_t)Hf.m, (uint64_t)Hf.mh, (uint64_t)Hf.ml, (uint64_t)Hf.t,
                   (uint64_t)Hf.tp, (uint64_t)Hf.tph, (uint64_t)Hf.tpl, (uint64_t)partial,
                   (uint64_t)part, (uint64_t)Jhist, (uint64_t)iter, (uint64_t)stat, (uint64_t)n,
                   (uint64_t)p, (uint64_t)K, (uint64_t)prec, (uint64_t)binary,
                   (uint64_t)__builtin_bit_cast(uint32_t, eps), (uint64_t)ca.nw, (uint64_t)ca.pipe,
                   (uint64_t)ca.tiles_per_split, (uint64_t)cb.nw, (uint64_t)cb.pipe,
                   (uint64_t)cb.splits, (uint64_t)cb.tiles_per_split, (uint64_t)c,
                   __builtin_bit_cast(uint64_t, c ? prm->tol : 0.0), (uint64_t)count});
  };
  // The device decides the stop; the host only stops enqueueing chunks once
  // it has seen the flag.  After each chunk the flag is copied to pinned
  // memory, and the copy of the previous chunk is read only after the next
  // chunk is queued, so the device never idles waiting for the host.
  int t = 0;
  int* host_flags = reinterpret_cast<int*>(hostJ + T + 1);  // two ints after J
  hipEvent_t chk[2] = {nullptr, nullptr};
  int inflight = -1, slot = 0;
  if (c) {
    HIP_TRY(hipEventCreateWithFlags(&chk[0], hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&chk[1], hipEventDisableTiming));
    host_flags[0] = host_flags[1] = 0;
  }
  hipError_t loop_err = hipSuccess;
  while (t < T) {
    const int count = std::min(chunk, T - t);
    loop_err = run_graph(h, iter_key(count), s, [&](hipStream_t st) { return enqueue_iters(st, count); });
    if (loop_err != hipSuccess) break;
    t += count;
    if (!c) continue;
    if ((loop_err = hipMemcpyAsync(host_flags + slot, stop_req, sizeof(int),
                                   hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (loop_err = hipEventRecord(chk[slot], s)) != hipSuccess)
      break;
    if (inflight >= 0) {
      if ((loop_err = hipEventSynchronize(chk[inflight])) != hipSuccess) break;
      if (host_flags[inflight]) break;  // stopped during an earlier chunk
    }
    inflight = slot;
    slot ^= 1;
  }
  for (hipEvent_t e : chk) {
    if (!e) continue;
    (void)hipEventSynchronize(e);
    (void)hipEventDestroy(e);
  }
  HIP_TRY(loop_err);
  // Objective after the last iteration, stored at Jhist[iterations done].
  LAUNCH(NMF_K_OBJECTIVE, launch_pass(prec, KP, MODE_OBJ, ca, A, ptile, s));
  LAUNCH(NMF_K_OTHER, launch_reduce_f64(part, pass_blocks(KP, ca, ptile), Jhist, stat, s, iter));
  if (prm->flags & NMF_F_NORMALIZE_H) LAUNCH(NMF_K_OTHER, launch_normalize(Hf.t, KP, p_pad, K, Wf.t, n_pad, s));
  LAUNCH(NMF_K_OTHER, launch_factor_out(Wf.t, (int)n, n_pad, K, KP, 0, W_out, s));
  LAUNCH(NMF_K_OTHER, launch_factor_out(Hf.t, (int)p, p_pad, K, KP, 1, H_out, s));
  HIP_TRY(hipEventRecord(h->ev1, s));
  if (prm->flags & NMF_F_ASYNC) {
    if (rep) {
      rep->iters_run = c ? -1 : t;  // with a stop rule only the device knows
      rep->status_flags = 0;
    }
    return NMF_OK;
  }
  int st = 0;
  double mv2 = 0.0;
  int dev_flags[3] = {0, 0, 0};
  HIP_TRY(hipMemcpyAsync(&st, stat, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&mv2, sum_mv2, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(dev_flags, iter, sizeof(dev_flags), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hostJ, Jhist, sizeof(double) * (T + 1), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int iters_run = dev_flags[0];
  const bool stopped = dev_flags[1] != 0;
  if (iters_run < 0 || iters_run > T) return fail(NMF_ERR_HIP, "iteration counter out of range");
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
    rep->status_flags = warn | (fell_back ? NMF_RS_WARM_FALLBACK : 0);
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
    LAUNCH(NMF_K_OTHER, launch_frame_objective(H, C_out, T, M_T, f, K, p,
                                               (prm->flags & NMF_F_BINARY_WEIGHTS) ? 1 : 0,
                                               (prm->flags & NMF_F_CLIP_NEGATIVE) ? 1 : 0,
                                               obj_out, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(prof_drain(h));
    return rc2;
  }
  if (prm->flags & NMF_F_WARM_START)
    return fail(NMF_ERR_UNSUPPORTED, "NMF_F_WARM_START needs the masked-Gram form");
  if (prm->tol > 0.0 && prm->check_every > 0)
    return fail(NMF_ERR_UNSUPPORTED, "the projection stop rule needs the masked-Gram form");
  if (KP > KP_MAX) return fail(NMF_ERR_UNSUPPORTED, "k > 224 is not supported by this build");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  const int prec = prm->precision;
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  const int f_pad = round_up(f, 32), p_pad = round_up(p, 32);
  const int ftile = f_pad / 32, ptile = p_pad / 32;
  PassCfg cb = cfg_split(ftile, ptile, KP, prec, prm->split, prm->waves);
  if (prm->pipeline > 0) cb.pipe = pipe_for(KP, prm->pipeline);
  float *DT, *MwT, *partial;
  double* part;
  int* stat;
  Factor Cf, Hf;
  const size_t nel = (size_t)f_pad * p_pad;
  const bool binary = (prm->flags & NMF_F_BINARY_WEIGHTS) != 0;
  uint16_t* BbT = nullptr;
  MwT = nullptr;
  if (binary ? (rc = ws(h, "pBT", nel / 16, &BbT)) : (rc = ws(h, "pMwT", nel, &MwT))) return rc;
  if ((rc = ws(h, "pDT", nel, &DT)) ||
      (rc = ws(h, "ppartial", (size_t)cb.splits * 2 * KP * f_pad, &partial)) ||
      (rc = ws(h, "ppart", (size_t)ftile * ptile, &part)) ||
      (rc = ws(h, "stat", 1, &stat)) || (rc = factor_alloc(h, "C", (int)f, f_pad, KP, &Cf)) ||
      (rc = factor_alloc(h, "PH", (int)p, p_pad, KP, &Hf)))
    return rc;
  HIP_TRY(hipEventRecord(h->ev0, s));
  HIP_TRY(hipMemsetAsync(stat, 0, sizeof(int), s));
  StageArgs sa{T, M_T, f, p, f_pad, p_pad, (prm->flags & NMF_F_CLIP_NEGATIVE) ? 1 : 0,
               nullptr, nullptr, DT, MwT, stat, part, binary ? 1 : 0, nullptr, BbT};
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
  B.Mb = BbT;
  B.tiles_per_split = cb.tiles_per_split;
  B.partial = partial;
  FinishArgs F = finish_args(partial, cb.splits, Cf, (int)f, K, prm->floor_eps, prec);
  for (int it = 0; it < prm->max_iter; ++it) {
    LAUNCH(NMF_K_PROJECT, launch_pass(prec, KP, MODE_SPLIT, cb, B, ftile, s));
    LAUNCH(NMF_K_PROJECT, launch_finish(F, s));
  }
  LAUNCH(NMF_K_OTHER, launch_factor_out(Cf.t, (int)f, f_pad, K, KP, 0, C_out, s));
  if (obj_out)
    LAUNCH(NMF_K_OTHER, launch_frame_objective(H, C_out, T, M_T, f, K, p, binary ? 1 : 0,
                                               (prm->flags & NMF_F_CLIP_NEGATIVE) ? 1 : 0,
                                               obj_out, s));
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

int64_t nmf_warm_fallbacks(nmf_handle h) { return h ? h->last_fallbacks : -1; }

int64_t nmf_frame_iters(nmf_handle h, int32_t* iters_out, int64_t f) {
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  const int64_t have = (int64_t)h->last_frame_iters.size();
  if (!have || !iters_out) return have;
  if (f < have) return fail(NMF_ERR_ARG, "iters_out must hold every frame");
  std::copy(h->last_frame_iters.begin(), h->last_frame_iters.end(), iters_out);
  return have;
}

int64_t nmf_frame_visits(nmf_handle h, int32_t* visits_out, int64_t f) {
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  const int64_t have = (int64_t)h->last_frame_visits.size();
  if (!have || !visits_out) return have;
  if (f < have) return fail(NMF_ERR_ARG, "visits_out must hold every frame");
  std::copy(h->last_frame_visits.begin(), h->last_frame_visits.end(), visits_out);
  return have;
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

// ---------------------------------------------------------------------------
int nmf_closest_frames(nmf_handle h, const float* V, const float* M, int64_t n, int64_t p,
                       const float* T, const float* M_T, int64_t f, int64_t n_sel,
                       double* dist_out, int32_t* idx_out, void* stream) {
  if (!V || !M || !T || !M_T || !idx_out) return fail(NMF_ERR_ARG, "NULL array argument");
  int rc = check_dims(n, p, "closest_frames");
  if (rc || (rc = check_dims(f, p, "closest_frames"))) return rc;
  if (n > 0x7fffffff || f > 65535) return fail(NMF_ERR_SHAPE, "n must fit in int32, f <= 65535");
  if (n_sel < 1 || n_sel > n) return fail(NMF_ERR_ARG, "n_sel must be in [1, n]");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  double* dist = dist_out;
  int* stat;
  if ((rc = ws(h, "stat", 1, &stat))) return rc;
  if (!dist && (rc = ws(h, "cf.dist", (size_t)f * n, &dist))) return rc;
  LAUNCH(NMF_K_OTHER, launch_set_int(stat, 0, s));
  LAUNCH(NMF_K_OTHER, launch_frame_dist(T, M_T, V, M, (int)f, (int)n, p, dist, stat, s));
  LAUNCH(NMF_K_OTHER, launch_select_rank(dist, (int)f, (int)n, (int)n_sel, idx_out, s));
  int st = 0;
  HIP_TRY(hipMemcpyAsync(&st, stat, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  if (st & 1) return fail(NMF_ERR_NONFINITE, "non-finite data under positive weight");
  return NMF_OK;
}

int nmf_closest_frames_noalloc(nmf_handle h, const float* V, const float* M, int64_t n,
                               int64_t p, const float* T, const float* M_T, int64_t f,
                               int64_t n_sel, int32_t* idx_out, void* stream) {
  if (!V || !M || !T || !M_T || !idx_out) return fail(NMF_ERR_ARG, "NULL array argument");
  int rc = check_dims(n, p, "closest_frames_noalloc");
  if (rc || (rc = check_dims(f, p, "closest_frames_noalloc"))) return rc;
  if (n > 0x7fffffff || f > 65535) return fail(NMF_ERR_SHAPE, "n must fit in int32, f <= 65535");
  if (n_sel < 1 || n_sel > n) return fail(NMF_ERR_ARG, "n_sel must be in [1, n]");
  if ((uint64_t)f * (uint64_t)n > (NOALLOC_SCRATCH_BYTES - NOALLOC_STATUS_BYTES) / sizeof(double))
    return fail(NMF_ERR_UNSUPPORTED, "f * n exceeds the scratch capacity of " +
                                         std::to_string((NOALLOC_SCRATCH_BYTES - NOALLOC_STATUS_BYTES) /
                                                        sizeof(double)) +
                                         " distances");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  if (h->device >= MAX_DEVICES || !g_scratch_ptr[h->device])
    return fail(NMF_ERR_UNSUPPORTED, "no scratch array on this device");
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  unsigned char* base = static_cast<unsigned char*>(g_scratch_ptr[h->device]);
  int* stat = reinterpret_cast<int*>(base);
  double* dist = reinterpret_cast<double*>(base + NOALLOC_STATUS_BYTES);
  // the array keeps the previous call's contents: the status word starts at 0
  HIP_TRY(launch_set_int(stat, 0, s));
  HIP_TRY(launch_frame_dist(T, M_T, V, M, (int)f, (int)n, p, dist, stat, s));
  HIP_TRY(launch_select_rank(dist, (int)f, (int)n, (int)n_sel, idx_out, s));
  int st = 0;
  HIP_TRY(hipMemcpyAsync(&st, stat, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (st & 1) return fail(NMF_ERR_NONFINITE, "non-finite data under positive weight");
  return NMF_OK;
}

int nmf_best_factor(nmf_handle h, const float* H, const float* C, const float* T,
                    const float* M_T, const float* region, int64_t f, int64_t k, int64_t p,
                    float s_lo, float s_hi, float* scale_out, void* stream) {
  if (!H || !C || !T || !M_T || !scale_out) return fail(NMF_ERR_ARG, "NULL array argument");
  int rc = check_dims(f, p, "best_factor");
  if (rc) return rc;
  if (k < 1 || k > 4096) return fail(NMF_ERR_ARG, "k must be in [1, 4096]");
  if (f > 0x7fffffff) return fail(NMF_ERR_SHAPE, "too many frames");
  if (!(s_lo <= s_hi) || std::isnan(s_lo) || std::isnan(s_hi))
    return fail(NMF_ERR_ARG, "need s_lo <= s_hi");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  LAUNCH(NMF_K_OTHER, launch_best_factor(H, C, T, M_T, region, f, (int)k, p, s_lo, s_hi,
                                         scale_out, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  return NMF_OK;
}

int nmf_build_basis_sequential(nmf_handle h, const float* V, const float* M, int64_t n, int64_t p,
                               const nmf_params* prm, float* W_out, float* H_out,
                               double* obj_stages, nmf_report* rep, void* stream) {
  if (!V || !M || !W_out || !H_out) return fail(NMF_ERR_ARG, "NULL array argument");
  int rc = check_dims(n, p, "build_basis_sequential");
  if (rc) return rc;
  if ((rc = check_params(prm, n, p, true))) return rc;
  if (rep && rep->struct_size != sizeof(nmf_report))
    return fail(NMF_ERR_ARG, "nmf_report.struct_size mismatch");
  if (kp_for(prm->k) > KP_MAX) return fail(NMF_ERR_UNSUPPORTED, "k > 224 is not supported by this build");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  const int K = prm->k;
  float *I_W, *I_H, *B_W[2], *B_H[2];
  if ((rc = ws(h, "seq.IW", (size_t)n * K, &I_W)) || (rc = ws(h, "seq.IH", (size_t)K * p, &I_H)) ||
      (rc = ws(h, "seq.W0", (size_t)n * K, &B_W[0])) || (rc = ws(h, "seq.H0", (size_t)K * p, &B_H[0])) ||
      (rc = ws(h, "seq.W1", (size_t)n * K, &B_W[1])) || (rc = ws(h, "seq.H1", (size_t)K * p, &B_H[1])))
    return rc;
  nmf_params sp = *prm;
  sp.flags &= ~NMF_F_ASYNC;  // each stage's result is needed by the next one
  const float *Wp = nullptr, *Hp = nullptr;
  int64_t total_iters = 0;
  float total_ms = 0.f;
  int warn = 0, result = NMF_OK;
  nmf_report sr{};
  sr.struct_size = sizeof(nmf_report);
  for (int j = 1; j <= K; ++j) {
    float* Wo = j == K ? W_out : B_W[j & 1];
    float* Ho = j == K ? H_out : B_H[j & 1];
    LAUNCH(NMF_K_OTHER, launch_seq_start(Wp, Hp, n, p, j, K, prm->seed, I_W, I_H, s));
    sp.k = j;
    const int st = nmf_build_basis(h, V, M, n, p, &sp, I_W, I_H, Wo, Ho, nullptr, &sr, stream);
    if (st < 0) return st;
    if (st > 0) {
      warn |= sr.status_flags;
      if (result == NMF_OK || st == NMF_WARN_NONMONOTONE) result = st;
    }
    if (obj_stages) obj_stages[j - 1] = sr.objective;
    total_iters += sr.iters_run;
    total_ms += sr.elapsed_ms;
    Wp = Wo;
    Hp = Ho;
  }
  if (rep) {
    rep->iters_run = (int32_t)std::min<int64_t>(total_iters, 0x7fffffff);
    rep->status_flags = warn;
    rep->objective = sr.objective;
    rep->objective_rel = sr.objective_rel;
    rep->elapsed_ms = total_ms;
  }
  return result;
}

int nmf_autotune_report(nmf_handle h, char* buf, size_t cap) {
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  std::string out;
  for (const auto& kv : h->tuned) {
    char line[256];
    std::snprintf(line, sizeof(line), "%s: waves=%d pipeline=%d splits=%d %.2f us\n", kv.first.c_str(),
                  kv.second.nw, kv.second.pipe, kv.second.splits, kv.second.us);
    out += line;
  }
  if (buf && cap) {
    const size_t n = std::min(cap - 1, out.size());
    std::memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  return (int)h->tuned.size();
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

// ===========================================================================
// Learned warm start
// ===========================================================================
namespace {

constexpr int WS_IN = NMF_WS_IN, WS_H = NMF_WS_HIDDEN;
constexpr float WS_FLOOR = 1e-6f;

struct WsLayout {
  int64_t W1, b1, W2, b2, W3, b3, count;
  explicit WsLayout(int k) {
    W1 = 0;
    b1 = W1 + (int64_t)WS_IN * WS_H;
    W2 = b1 + WS_H;
    b2 = W2 + (int64_t)WS_H * WS_H;
    W3 = b2 + WS_H;
    b3 = W3 + (int64_t)WS_H * k;
    count = b3 + k;
  }
};

LinearArgs lin(const float* A, int64_t sa0, int64_t sa1, const float* B, int64_t sb0, int64_t sb1,
               const float* bias, float* C, float* Hact, int64_t ldc, int M, int N, int Kd, int act,
               int x3) {
  LinearArgs a{};
  a.A = A;
  a.sa0 = sa0;
  a.sa1 = sa1;
  a.B = B;
  a.sb0 = sb0;
  a.sb1 = sb1;
  a.bias = bias;
  a.C = C;
  a.Hact = Hact;
  a.ldc = ldc;
  a.M = M;
  a.N = N;
  a.Kd = Kd;
  a.act = act;
  a.x3 = x3;
  return a;
}

struct WsBufs {
  float *A1, *H1, *A2, *H2, *Z, *W, *D, *U, *V, *dW, *dZ, *dH, *dA, *grads, *Xb, *sb, *cb;
  double* lrow;
  int* idx;
};

int ws_bufs(nmf_handle h, int b, int k, int64_t nparam, WsBufs* o) {
  int rc;
  const size_t bh = (size_t)b * WS_H, bk = (size_t)b * k;
  if ((rc = ws(h, "ws.A1", bh, &o->A1)) || (rc = ws(h, "ws.H1", bh, &o->H1)) ||
      (rc = ws(h, "ws.A2", bh, &o->A2)) || (rc = ws(h, "ws.H2", bh, &o->H2)) ||
      (rc = ws(h, "ws.Z", bk, &o->Z)) || (rc = ws(h, "ws.W", bk, &o->W)) ||
      (rc = ws(h, "ws.D", bk, &o->D)) || (rc = ws(h, "ws.U", bk, &o->U)) ||
      (rc = ws(h, "ws.V", bk, &o->V)) ||
      (rc = ws(h, "ws.dW", bk, &o->dW)) || (rc = ws(h, "ws.dZ", bk, &o->dZ)) ||
      (rc = ws(h, "ws.dH", bh, &o->dH)) || (rc = ws(h, "ws.dA", bh, &o->dA)) ||
      (rc = ws(h, "ws.grads", (size_t)nparam, &o->grads)) ||
      (rc = ws(h, "ws.lrow", (size_t)b, &o->lrow)) || (rc = ws(h, "ws.Xb", (size_t)b * WS_IN, &o->Xb)) ||
      (rc = ws(h, "ws.sb", (size_t)b, &o->sb)) || (rc = ws(h, "ws.cb", bk, &o->cb)) ||
      (rc = ws(h, "ws.idx", (size_t)b, &o->idx)))
    return rc;
  return NMF_OK;
}

int x3_of(int precision) { return precision == NMF_PREC_BF16 ? 0 : 1; }

// Forward pass for b rows: activations into the buffers, predictions into W.
hipError_t ws_forward(nmf_handle h, const float* P, const WsLayout& L, const float* X, const float* s,
                      int b, int k, int x3, const WsBufs& B, float* Wout, hipStream_t st) {
  hipError_t e;
  LinearArgs l1 = lin(X, WS_IN, 1, P + L.W1, WS_H, 1, P + L.b1, B.A1, B.H1, WS_H, b, WS_H, WS_IN,
                      ACT_GELU, x3);
  if ((e = timed(h, NMF_K_OTHER, st, [&]() { return launch_linear(l1, st); }))) return e;
  LinearArgs l2 = lin(B.H1, WS_H, 1, P + L.W2, WS_H, 1, P + L.b2, B.A2, B.H2, WS_H, b, WS_H, WS_H,
                      ACT_GELU, x3);
  if ((e = timed(h, NMF_K_OTHER, st, [&]() { return launch_linear(l2, st); }))) return e;
  LinearArgs l3 = lin(B.H2, WS_H, 1, P + L.W3, k, 1, P + L.b3, B.Z, nullptr, k, b, k, WS_H,
                      ACT_NONE, x3);
  if ((e = timed(h, NMF_K_OTHER, st, [&]() { return launch_linear(l3, st); }))) return e;
  return timed(h, NMF_K_OTHER, st, [&]() { return launch_head(B.Z, s, b, k, WS_FLOOR, Wout, st); });
}

// Loss + backward for b rows (after ws_forward into B.W); gradients into
// B.grads in the parameter layout; per-row loss terms into B.lrow.
hipError_t ws_backward(nmf_handle h, const float* P, const WsLayout& L, const float* X,
                       const float* s, const float* cstar, const float* G, int b, int k, int x3,
                       const WsBufs& B, hipStream_t st) {
  hipError_t e;
  auto T = [&](auto fn) { return timed(h, NMF_K_OTHER, st, fn); };
  float* g = B.grads;
  // U = (w - c*) G and V = c* G, always with split products (small GEMMs)
  if ((e = T([&]() { return launch_sub(B.W, cstar, (int64_t)b * k, B.D, st); }))) return e;
  LinearArgs lu = lin(B.D, k, 1, G, k, 1, nullptr, B.U, nullptr, k, b, k, k, ACT_NONE, 1);
  if ((e = T([&]() { return launch_linear(lu, st); }))) return e;
  LinearArgs lv = lin(cstar, k, 1, G, k, 1, nullptr, B.V, nullptr, k, b, k, k, ACT_NONE, 1);
  if ((e = T([&]() { return launch_linear(lv, st); }))) return e;
  if ((e = T([&]() { return launch_loss(B.W, cstar, B.U, B.V, b, k, B.dW, B.lrow, st); }))) return e;
  // head
  if ((e = T([&]() { return launch_head_bwd(B.dW, B.Z, s, b, k, B.dZ, st); }))) return e;
  LinearArgs g3 = lin(B.H2, 1, WS_H, B.dZ, k, 1, nullptr, g + L.W3, nullptr, k, WS_H, k, b, ACT_NONE, x3);
  if ((e = T([&]() { return launch_linear(g3, st); }))) return e;
  if ((e = T([&]() { return launch_colsum(B.dZ, b, k, g + L.b3, st); }))) return e;
  // layer 2
  LinearArgs d2 = lin(B.dZ, k, 1, P + L.W3, 1, k, nullptr, B.dH, nullptr, WS_H, b, WS_H, k, ACT_NONE, x3);
  if ((e = T([&]() { return launch_linear(d2, st); }))) return e;
  if ((e = T([&]() { return launch_gelu_bwd(B.dH, B.A2, (int64_t)b * WS_H, B.dA, st); }))) return e;
  LinearArgs g2 = lin(B.H1, 1, WS_H, B.dA, WS_H, 1, nullptr, g + L.W2, nullptr, WS_H, WS_H, WS_H, b,
                      ACT_NONE, x3);
  if ((e = T([&]() { return launch_linear(g2, st); }))) return e;
  if ((e = T([&]() { return launch_colsum(B.dA, b, WS_H, g + L.b2, st); }))) return e;
  // layer 1
  LinearArgs d1 = lin(B.dA, WS_H, 1, P + L.W2, 1, WS_H, nullptr, B.dH, nullptr, WS_H, b, WS_H, WS_H,
                      ACT_NONE, x3);
  if ((e = T([&]() { return launch_linear(d1, st); }))) return e;
  if ((e = T([&]() { return launch_gelu_bwd(B.dH, B.A1, (int64_t)b * WS_H, B.dA, st); }))) return e;
  LinearArgs g1 = lin(X, 1, WS_IN, B.dA, WS_H, 1, nullptr, g + L.W1, nullptr, WS_H, WS_IN, WS_H, b,
                      ACT_NONE, x3);
  if ((e = T([&]() { return launch_linear(g1, st); }))) return e;
  return T([&]() { return launch_colsum(B.dA, b, WS_H, g + L.b1, st); });
}

}  // namespace

extern "C" {

int64_t nmf_warmstart_param_count(int32_t k) { return k > 0 ? WsLayout(k).count : 0; }

int nmf_warmstart_init(nmf_handle h, float* state, int32_t k, uint64_t seed, void* stream) {
  if (!state) return fail(NMF_ERR_ARG, "state is NULL");
  if (k < 1 || k > 4096) return fail(NMF_ERR_ARG, "k must be in [1, 4096]");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  const WsLayout L(k);
  HIP_TRY(hipMemsetAsync(state, 0, sizeof(float) * 3 * L.count, s));
  LAUNCH(NMF_K_OTHER, launch_normal_init(state + L.W1, L.b1 - L.W1, std::sqrt(2.f / WS_IN), seed, 10, s));
  LAUNCH(NMF_K_OTHER, launch_normal_init(state + L.W2, L.b2 - L.W2, std::sqrt(2.f / WS_H), seed, 11, s));
  LAUNCH(NMF_K_OTHER, launch_normal_init(state + L.W3, L.b3 - L.W3, std::sqrt(1.f / WS_H), seed, 12, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  return NMF_OK;
}

int nmf_warmstart_pool(nmf_handle h, const float* T, const float* M_T, int64_t f, int32_t ny,
                       int32_t nx, float* X_out, float* s_out, void* stream) {
  if (!T || !M_T || !X_out || !s_out) return fail(NMF_ERR_ARG, "NULL array argument");
  if (f < 1 || f > 0x7fffffff || ny < 1 || nx < 1) return fail(NMF_ERR_SHAPE, "bad frame shape");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  LAUNCH(NMF_K_OTHER, launch_pool(T, M_T, (int)f, ny, nx, X_out, s_out, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  return NMF_OK;
}

int nmf_warmstart_infer(nmf_handle h, const float* state, const float* X, const float* s_in,
                        int64_t f, int32_t k, int32_t precision, float* C_out, void* stream) {
  if (!state || !X || !s_in || !C_out) return fail(NMF_ERR_ARG, "NULL array argument");
  if (f < 1 || f > 0x7fffffff) return fail(NMF_ERR_SHAPE, "bad row count");
  if (k < 1 || k > 4096) return fail(NMF_ERR_ARG, "k must be in [1, 4096]");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  const WsLayout L(k);
  const int x3 = x3_of(precision);
  const int chunk = 4096;
  WsBufs B;
  int rc;
  if ((rc = ws_bufs(h, (int)std::min<int64_t>(f, chunk), k, L.count, &B))) return rc;
  for (int64_t r0 = 0; r0 < f; r0 += chunk) {
    const int b = (int)std::min<int64_t>(chunk, f - r0);
    HIP_TRY(ws_forward(h, state, L, X + r0 * WS_IN, s_in + r0, b, k, x3, B, C_out + r0 * k, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  return NMF_OK;
}

int nmf_warmstart_step(nmf_handle h, float* state, const float* X, const float* s_in,
                       const float* c_star, const float* G, int32_t b, int32_t k,
                       int32_t precision, float lr, int32_t step_index, float* grads_out,
                       double* loss_out, void* stream) {
  if (!state || !X || !s_in || !c_star || !G) return fail(NMF_ERR_ARG, "NULL array argument");
  if (b < 1 || b > 65535) return fail(NMF_ERR_SHAPE, "batch must be in [1, 65535]");
  if (k < 1 || k > 4096) return fail(NMF_ERR_ARG, "k must be in [1, 4096]");
  if (lr > 0.f && step_index < 1) return fail(NMF_ERR_ARG, "step_index counts from 1");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  const WsLayout L(k);
  const int x3 = x3_of(precision);
  WsBufs B;
  int rc;
  if ((rc = ws_bufs(h, b, k, L.count, &B))) return rc;
  HIP_TRY(ws_forward(h, state, L, X, s_in, b, k, x3, B, B.W, s));
  HIP_TRY(ws_backward(h, state, L, X, s_in, c_star, G, b, k, x3, B, s));
  if (grads_out)
    HIP_TRY(hipMemcpyAsync(grads_out, B.grads, sizeof(float) * L.count, hipMemcpyDeviceToDevice, s));
  if (lr > 0.f)
    LAUNCH(NMF_K_OTHER, launch_adam(state, B.grads, state + L.count, state + 2 * L.count, L.count,
                                    lr, 0.9f, 0.999f, 1e-8f, step_index, s));
  std::vector<double> lrow(b);
  HIP_TRY(hipMemcpyAsync(lrow.data(), B.lrow, sizeof(double) * b, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  double sum = 0.0;
  for (double v : lrow) sum += v;
  if (loss_out) *loss_out = sum / b;
  if (!std::isfinite(sum)) return fail(NMF_ERR_DIVERGED, "warm-start loss became non-finite");
  return NMF_OK;
}

int nmf_warmstart_train(nmf_handle h, float* state, const float* X, const float* s_in,
                        const float* c_star, const float* G, int64_t m, int32_t k,
                        int32_t precision, int32_t epochs, int32_t batch, float lr,
                        uint64_t seed, double* loss_hist, void* stream) {
  if (!state || !X || !s_in || !c_star || !G) return fail(NMF_ERR_ARG, "NULL array argument");
  if (m < 1 || m > 0x7fffffff) return fail(NMF_ERR_SHAPE, "bad row count");
  if (batch < 1 || batch > 65535) return fail(NMF_ERR_SHAPE, "batch must be in [1, 65535]");
  if (epochs < 0 || !(lr > 0.f)) return fail(NMF_ERR_ARG, "epochs >= 0 and lr > 0 required");
  if (k < 1 || k > 4096) return fail(NMF_ERR_ARG, "k must be in [1, 4096]");
  if (!h) return fail(NMF_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  hipStream_t s = (hipStream_t)stream;
  const WsLayout L(k);
  const int x3 = x3_of(precision);
  const int b = (int)std::min<int64_t>(batch, m);
  const int nb = (int)(m / b);  // full minibatches per epoch
  WsBufs B;
  int rc;
  int *perm_d, *ctr;
  float* coef;
  double* eacc;
  if ((rc = ws_bufs(h, b, k, L.count, &B)) || (rc = ws(h, "ws.perm", (size_t)m, &perm_d)) ||
      (rc = ws(h, "ws.ctr", 2, &ctr)) || (rc = ws(h, "ws.coef", 2, &coef)) ||
      (rc = ws(h, "ws.eacc", 1, &eacc)))
    return rc;
  constexpr float B1 = 0.9f, B2 = 0.999f, AEPS = 1e-8f;
  // An epoch is one captured graph: per minibatch the rows perm[cursor ..
  // cursor + b) are gathered, the forward and backward passes and the Adam
  // step run, the batch loss is added to the epoch sum, and the cursor and
  // step advance on the device.  The step count t runs on across epochs.
  LAUNCH(NMF_K_OTHER, launch_train_ctr(ctr, coef, 0, b, B1, B2, s));
  auto epoch = [&](hipStream_t st) -> hipError_t {
    hipError_t e;
    if ((e = launch_set_int(ctr, 0, st))) return e;  // cursor only; t continues
    for (int i = 0; i < nb; ++i) {
      if ((e = timed(h, NMF_K_OTHER, st, [&]() {
             return launch_gather_cur(X, perm_d, ctr, b, WS_IN, B.Xb, st);
           })))
        return e;
      if ((e = timed(h, NMF_K_OTHER, st,
                     [&]() { return launch_gather_cur(s_in, perm_d, ctr, b, 1, B.sb, st); })))
        return e;
      if ((e = timed(h, NMF_K_OTHER, st,
                     [&]() { return launch_gather_cur(c_star, perm_d, ctr, b, k, B.cb, st); })))
        return e;
      if ((e = ws_forward(h, state, L, B.Xb, B.sb, b, k, x3, B, B.W, st))) return e;
      if ((e = ws_backward(h, state, L, B.Xb, B.sb, B.cb, G, b, k, x3, B, st))) return e;
      if ((e = timed(h, NMF_K_OTHER, st, [&]() {
             return launch_adam_dev(state, B.grads, state + L.count, state + 2 * L.count, L.count,
                                    lr, B1, B2, AEPS, coef, st);
           })))
        return e;
      if ((e = timed(h, NMF_K_OTHER, st,
                     [&]() { return launch_loss_accum(B.lrow, b, eacc, i == 0, st); })))
        return e;
      if ((e = timed(h, NMF_K_OTHER, st,
                     [&]() { return launch_train_ctr(ctr, coef, 1, b, B1, B2, st); })))
        return e;
    }
    return hipSuccess;
  };
  const std::string key =
      key_of("wsTrain", {(uint64_t)state, (uint64_t)X, (uint64_t)s_in, (uint64_t)c_star,
                         (uint64_t)G, (uint64_t)m, (uint64_t)k, (uint64_t)x3, (uint64_t)b,
                         (uint64_t)__builtin_bit_cast(uint32_t, lr), (uint64_t)perm_d,
                         (uint64_t)ctr, (uint64_t)coef, (uint64_t)eacc, (uint64_t)B.Xb,
                         (uint64_t)B.grads, (uint64_t)B.lrow, (uint64_t)B.A1, (uint64_t)B.dA});
  std::vector<int> perm(m);
  for (int ep = 0; ep < epochs; ++ep) {
    // Fisher-Yates shuffle driven by the counter-based generator
    for (int64_t i = 0; i < m; ++i) perm[i] = (int)i;
    const uint64_t key_ep = sm_key(seed, 100 + ep);
    for (int64_t i = m - 1; i > 0; --i) {
      const uint64_t u = sm_mix(key_ep + (uint64_t)(i + 1) * SM_GAMMA);
      const int64_t j = (int64_t)(u % (uint64_t)(i + 1));
      std::swap(perm[i], perm[j]);
    }
    HIP_TRY(hipMemcpyAsync(perm_d, perm.data(), sizeof(int) * m, hipMemcpyHostToDevice, s));
    HIP_TRY(run_graph(h, key, s, epoch));
    double ep_loss = 0.0;
    HIP_TRY(hipMemcpyAsync(&ep_loss, eacc, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));  // also keeps perm alive for the copy
    if (loss_hist) loss_hist[ep] = nb ? ep_loss / ((double)nb * b) : 0.0;
    if (!std::isfinite(ep_loss)) return fail(NMF_ERR_DIVERGED, "warm-start loss became non-finite");
  }
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(prof_drain(h));
  return NMF_OK;
}

}  // extern "C"
