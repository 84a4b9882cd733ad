// C ABI of the library: argument validation (host only, before any launch),
// workspace layout, launch-grid choices and the order of kernel launches for
// E, E^H, E^H E and the CG solve.  No device memory is allocated here.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "nfs.h"
#include "nfs_internal.h"

using namespace nfs;

struct nfs_ctx {
  int device;
  int n_cu;
  bool profiling = false;
  bool graphs = false;
  int batch_mode = NFS_BATCH_STREAMS;
  // captured solves (nfs_set_graphs), at most kMaxGraphs; `done` is recorded
  // after each launch so that an evicted graph is destroyed only once its
  // last launch has finished
  struct Graph {
    hipGraphExec_t ex = nullptr;
    hipEvent_t done = nullptr;
    uint64_t last_use = 0;
  };
  std::unordered_map<std::string, Graph> graph_cache;
  uint64_t graph_clock = 0;
  std::vector<hipStream_t> bstreams;  // batched solves: forked streams (default priority)
  std::vector<hipEvent_t> bevents;    // ... and their join events
  hipEvent_t fork_event = nullptr;
  hipStream_t capture_stream = nullptr;  // graph capture only
  std::vector<hipEvent_t> pool;                 // idle events
  std::vector<std::pair<hipEvent_t, hipEvent_t>> rec[2];  // recorded (start, stop) per kind
  // autotuned encode shapes: key (op, precision, L, K, G, P) -> (MT, nsplit)
  std::map<std::string, std::pair<int, int>> tune;
  unsigned tune_generation = 0;  // bumped by every autotune (part of graph keys)
  void* scratch = nullptr;       // this device's copy of `scratch` (nfs_cg_solve_noalloc)
};

static std::string tune_key(int op, int prec, const nfs_problem* pr) {
  char b[128];
  snprintf(b, sizeof b, "%d/%d/%lld/%lld/%d/%d", op, prec, (long long)pr->n_vox, (long long)pr->n_samp, pr->n_coil,
           pr->n_basis);
  return b;
}

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

static int hip_fail(hipError_t e, const char* where) {
  return fail(NFS_EHIP, "%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
}

extern "C" const char* nfs_last_error(void) { return g_err.c_str(); }
extern "C" int nfs_version(void) { return 100; }

// Device scratch of nfs_cg_solve_noalloc: a file-scope device array, so
// that the call needs no allocation at all.  Its name is only a host-side
// stand-in; the device address of each GPU's copy comes from
// hipGetSymbolAddress (with that device current) and is kept per device.
constexpr size_t kScratchBytes = (size_t)NFS_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static std::unordered_map<int, void*> g_scratch_ptr;

static int scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return NFS_OK;
  }
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "nfs_create: hipGetDevice");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "nfs_create: hipSetDevice");
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  const hipError_t e2 = hipSetDevice(cur);
  if (e != hipSuccess) return hip_fail(e, "nfs_create: hipGetSymbolAddress(scratch)");
  if (e2 != hipSuccess) return hip_fail(e2, "nfs_create: hipSetDevice");
  if (!p || (uintptr_t)p % 256) return fail(NFS_EHIP, "nfs_create: scratch address %p not 256-byte aligned", p);
  g_scratch_ptr.emplace(device, p);
  *out = p;
  return NFS_OK;
}

extern "C" int nfs_create(nfs_ctx** ctx, int device) {
  if (!ctx) return fail(NFS_EINVAL, "nfs_create: ctx is NULL");
  *ctx = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "nfs_create: hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(NFS_EHIP, "nfs_create: device %d not present (%d devices)", device, n);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "nfs_create: hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(NFS_EUNSUPPORTED, "nfs_create: device %d is %s, not gfx950", device, prop.gcnArchName);
  void* sp = nullptr;
  const int rc = scratch_address(device, &sp);
  if (rc) return rc;
  nfs_ctx* c = new nfs_ctx;
  c->device = device;
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->scratch = sp;
  *ctx = c;
  return NFS_OK;
}

extern "C" int nfs_destroy(nfs_ctx* ctx) {
  if (!ctx) return NFS_OK;
  for (int k = 0; k < 2; ++k)
    for (auto& pr : ctx->rec[k]) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  for (auto& kv : ctx->graph_cache) {
    if (kv.second.done) (void)hipEventSynchronize(kv.second.done);
    (void)hipGraphExecDestroy(kv.second.ex);
    if (kv.second.done) (void)hipEventDestroy(kv.second.done);
  }
  for (auto st : ctx->bstreams) (void)hipStreamDestroy(st);
  for (auto e : ctx->bevents) (void)hipEventDestroy(e);
  if (ctx->fork_event) (void)hipEventDestroy(ctx->fork_event);
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  delete ctx;
  return NFS_OK;
}

static hipError_t take_event(nfs_ctx* ctx, hipEvent_t* e) {
  if (!ctx->pool.empty()) {
    *e = ctx->pool.back();
    ctx->pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

extern "C" int nfs_profile_enable(nfs_ctx* ctx, int on) {
  if (!ctx) return fail(NFS_EINVAL, "nfs_profile_enable: ctx is NULL");
  ctx->profiling = on != 0;
  return NFS_OK;
}

extern "C" int nfs_profile_read(nfs_ctx* ctx, int kind, int* count, double* total_ms) {
  if (!ctx || !count || !total_ms) return fail(NFS_EINVAL, "nfs_profile_read: NULL argument");
  if (kind < 0 || kind > 1) return fail(NFS_EINVAL, "nfs_profile_read: kind %d not 0 or 1", kind);
  double tot = 0.0;
  int n = 0;
  for (auto& pr : ctx->rec[kind]) {
    hipError_t e = hipEventSynchronize(pr.second);
    if (e != hipSuccess) return hip_fail(e, "nfs_profile_read: hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess) return hip_fail(e, "nfs_profile_read: hipEventElapsedTime");
    tot += ms;
    ++n;
    ctx->pool.push_back(pr.first);
    ctx->pool.push_back(pr.second);
  }
  ctx->rec[kind].clear();
  *count = n;
  *total_ms = tot;
  return NFS_OK;
}

// ---------------------------------------------------------------------------
// validation
static bool misaligned(const void* p, size_t a) { return p && ((uintptr_t)p % a) != 0; }

static int check_sizes(const nfs_problem* pr, const char* fn) {
  if (!pr) return fail(NFS_EINVAL, "%s: problem is NULL", fn);
  const int64_t lim = (int64_t)1 << 26;
  if (pr->n_vox < 0 || pr->n_vox > lim) return fail(NFS_ESHAPE, "%s: n_vox %lld outside [0, 2^26]", fn, (long long)pr->n_vox);
  if (pr->n_samp < 0 || pr->n_samp > lim) return fail(NFS_ESHAPE, "%s: n_samp %lld outside [0, 2^26]", fn, (long long)pr->n_samp);
  if (pr->n_coil < 1 || pr->n_coil > 64) return fail(NFS_ESHAPE, "%s: n_coil %d outside [1, 64]", fn, pr->n_coil);
  if (pr->n_basis < 0 || pr->n_basis > 31) return fail(NFS_ESHAPE, "%s: n_basis %d outside [0, 31]", fn, pr->n_basis);
  return NFS_OK;
}

static int check_problem(const nfs_problem* pr, const char* fn) {
  int rc = check_sizes(pr, fn);
  if (rc) return rc;
  const bool hasL = pr->n_vox > 0, hasK = pr->n_samp > 0, hasP = pr->n_basis > 0;
  if (hasL && !pr->sens) return fail(NFS_EINVAL, "%s: sens is NULL", fn);
  if (hasL && !pr->b0) return fail(NFS_EINVAL, "%s: b0 is NULL", fn);
  if (hasL && hasP && !pr->fields) return fail(NFS_EINVAL, "%s: fields is NULL", fn);
  if (hasK && !pr->t) return fail(NFS_EINVAL, "%s: t is NULL", fn);
  if (hasK && hasP && !pr->kcoef) return fail(NFS_EINVAL, "%s: kcoef is NULL", fn);
  if (misaligned(pr->sens, 8)) return fail(NFS_EINVAL, "%s: sens not 8-byte aligned", fn);
  if (misaligned(pr->fields, 4) || misaligned(pr->b0, 4) || misaligned(pr->kcoef, 4) || misaligned(pr->t, 4) ||
      misaligned(pr->icorr, 4))
    return fail(NFS_EINVAL, "%s: real array not 4-byte aligned", fn);
  return NFS_OK;
}

static int check_prec(int prec, const char* fn) {
  if (prec != NFS_FP32 && prec != NFS_BF16 && prec != NFS_FP16)
    return fail(NFS_EINVAL, "%s: unknown precision %d", fn, prec);
  return NFS_OK;
}

static int check_vec(const void* p, int64_t n, const char* fn, const char* name) {
  if (n > 0 && !p) return fail(NFS_EINVAL, "%s: %s is NULL", fn, name);
  if (misaligned(p, 8)) return fail(NFS_EINVAL, "%s: %s not 8-byte aligned", fn, name);
  return NFS_OK;
}

// ---------------------------------------------------------------------------
// workspace layout
static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  int64_t L, K, LC, KC;
  int G, P, NQ, NB, prec;
  EncodeShape shE, shH;
  size_t o_sA, o_sB, o_vA, o_vB, o_tmax, o_dataE, o_dataH, o_epart, o_hpart, o_bmax, o_unscale, o_sensj, o_smax;
  size_t o_r, o_p, o_q, o_b, o_part, o_alpha, o_scal, o_hist, o_info, o_stop, o_V, o_rpart, o_rn;
  size_t o_PE, o_PH;  // resident P (NFS_OP_CG_RESIDENT)
  size_t total;
};

static size_t epart_bytes(const EncodeShape& sh, int NB) { return (size_t)sh.nsplit * sh.HC * 16 * NB * 16 * 4; }
static size_t hpart_bytes(const EncodeShape& sh) { return (size_t)sh.nsplit * sh.HC * 16 * 8; }

static int choose_split(int64_t held_chunks, int64_t strm_chunks, int MT, int n_cu) {
  const int64_t gx = cdiv(held_chunks, (int64_t)kWaves * MT);
  if (gx <= 0) return 1;
  int64_t ns = cdiv(4LL * n_cu, gx);
  const int64_t maxs = strm_chunks / 32 > 1 ? strm_chunks / 32 : 1;
  if (ns > maxs) ns = maxs;
  if (ns > 64) ns = 64;
  if (ns < 1) ns = 1;
  return (int)ns;
}

// Encode shape of one direction: held-tile count MT and split count, from
// (in order) an explicit override, the context's autotuned entry, or the
// default heuristic.
static EncodeShape encode_shape(const nfs_ctx* ctx, const nfs_problem* pr, int op, int prec, int NQ, int NB,
                                int64_t HC, int64_t SC, const int* ov) {
  const int n_cu = ctx ? ctx->n_cu : 256;
  int MT = held_tiles(NB), ns = 0;
  if (ov) {
    MT = ov[0];
    ns = ov[1];
  } else if (ctx) {
    auto it = ctx->tune.find(tune_key(op, prec, pr));
    if (it != ctx->tune.end()) {
      MT = it->second.first;
      ns = it->second.second;
    }
  }
  if (ns < 1) ns = choose_split(HC, SC, MT, n_cu);
  EncodeShape sh{op, prec, NQ, NB, MT, HC, SC, ns, 0};
  sh.cps = cdiv(SC, ns > 0 ? ns : 1);
  return sh;
}

// ovE / ovH: optional {MT, nsplit} overrides of the E / E^H shapes (tuning)
static Layout make_layout(const nfs_ctx* ctx, const nfs_problem* pr, int op, int prec, int n_iter, int reorth,
                          const int* ovE = nullptr, const int* ovH = nullptr) {
  Layout y{};
  y.L = pr->n_vox;
  y.K = pr->n_samp;
  y.G = pr->n_coil;
  y.P = pr->n_basis;
  y.LC = cdiv(y.L, kChunk);
  y.KC = cdiv(y.K, kChunk);
  y.NQ = phase_instrs(y.P);
  y.NB = col_blocks(y.G);
  y.prec = prec;
  y.shE = encode_shape(ctx, pr, OP_E, prec, y.NQ, y.NB, y.KC, y.LC, ovE);
  y.shH = encode_shape(ctx, pr, OP_EH, prec, y.NQ, y.NB, y.LC, y.KC, ovH);
  const bool needE = op != NFS_OP_EH, needH = op != NFS_OP_E;
  const bool cg = op == NFS_OP_CG || op == NFS_OP_CG_RESIDENT;

  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += al(bytes);
    return at;
  };
  // phase parts: E streams voxels (role A) against held samples (role B);
  // E^H streams samples (role A) against held voxels (role B)
  y.o_vA = needE ? take((size_t)y.LC * phase_chunk_bytes(y.NQ)) : 0;
  y.o_sB = needE ? take((size_t)y.KC * phase_chunk_bytes(y.NQ)) : 0;
  y.o_sA = needH ? take((size_t)y.KC * phase_chunk_bytes(y.NQ)) : 0;
  y.o_vB = needH ? take((size_t)y.LC * phase_chunk_bytes(y.NQ)) : 0;
  y.o_tmax = take(2 * kMaxTerms * 4);
  y.o_bmax = take(kBmaxBlocks * 4);
  y.o_unscale = take(2 * 4);
  y.o_dataE = needE ? take((size_t)y.LC * y.NB * data_chunk_bytes(prec)) : 0;
  y.o_dataH = needH ? take((size_t)y.KC * y.NB * data_chunk_bytes(prec)) : 0;
  if (cg) {
    y.o_sensj = pr->icorr ? take((size_t)y.G * y.L * 8) : 0;
    y.o_smax = scaled_prec(prec) ? take((size_t)y.L * 4) : 0;
    y.o_r = take((size_t)y.L * 8);
    y.o_p = take((size_t)y.L * 8);
    y.o_q = take((size_t)y.L * 8);
    y.o_b = take((size_t)y.L * 8);
    y.o_part = take(4 * kCgBlocks * 8);
    y.o_alpha = take((size_t)(n_iter + 2) * 8);
    y.o_scal = take(4 * 8);
    y.o_hist = take((size_t)(n_iter + 1) * 3 * 8);
    y.o_info = take(2 * 4);
    y.o_stop = take(4);
    if (reorth) {
      y.o_V = take((size_t)(n_iter + 1) * y.L * 8);
      y.o_rn = take((size_t)y.L * 8);
      y.o_rpart = take((size_t)(n_iter + 1) * 2 * kCgBlocks * 8);
    }
  }
  if (op == NFS_OP_CG_RESIDENT) {
    y.o_PE = take(resident_P_bytes(y.KC, y.LC));
    y.o_PH = take(resident_P_bytes(y.LC, y.KC));
  }
  // split partials last: their sizes depend on the encode shapes
  y.o_epart = needE ? take(epart_bytes(y.shE, y.NB)) : 0;
  y.o_hpart = needH ? take(hpart_bytes(y.shH)) : 0;
  y.total = o;
  return y;
}

extern "C" int nfs_workspace_bytes(const nfs_ctx* ctx, const nfs_problem* prob, int op, int precision, int n_iter,
                                   int reorth, size_t* bytes) {
  const char* fn = "nfs_workspace_bytes";
  if (!bytes) return fail(NFS_EINVAL, "%s: bytes is NULL", fn);
  int rc = check_sizes(prob, fn);
  if (rc) return rc;
  if ((rc = check_prec(precision, fn))) return rc;
  if (op < NFS_OP_E || op > NFS_OP_CG_RESIDENT) return fail(NFS_EINVAL, "%s: unknown op %d", fn, op);
  const bool cg = op == NFS_OP_CG || op == NFS_OP_CG_RESIDENT;
  if (cg && n_iter < 0) return fail(NFS_EINVAL, "%s: n_iter %d < 0", fn, n_iter);
  if (cg && reorth && n_iter > kMaxReorth) return fail(NFS_EINVAL, "%s: reorth needs n_iter <= %d", fn, kMaxReorth);
  if (op == NFS_OP_CG_RESIDENT && precision != NFS_FP16)
    return fail(NFS_EUNSUPPORTED, "%s: the resident form takes NFS_FP16 operands", fn);
  *bytes = make_layout(ctx, prob, op, precision, cg ? n_iter : 0, cg ? (reorth != 0) : 0).total;
  return NFS_OK;
}

static int check_ws(const Layout& y, void* ws, size_t ws_bytes, const char* fn) {
  if (!ws) return fail(NFS_EWORKSPACE, "%s: workspace is NULL", fn);
  if ((uintptr_t)ws % 256) return fail(NFS_EWORKSPACE, "%s: workspace not 256-byte aligned", fn);
  if (ws_bytes < y.total)
    return fail(NFS_EWORKSPACE, "%s: workspace has %zu bytes, needs %zu", fn, ws_bytes, y.total);
  return NFS_OK;
}

template <class T>
static T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

#define NFS_TRY(expr, where)                  \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// ---------------------------------------------------------------------------
// launch sequences
struct Ctx {
  nfs_ctx* lib;
  const Layout& y;
  const nfs_problem* pr;
  const float2* sens;  // possibly intensity-corrected
  void* ws;
  hipStream_t s;
  const int* stop;
  const void* PE = nullptr;  // resident P of E and of E^H (non-split form), or NULL
  const void* PH = nullptr;
};

// Launch the encode kernel, bracketed by HIP events when profiling is on.
template <class F>
static int timed_encode(const Ctx& c, int kind, F&& launch) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c.lib->profiling) {
    NFS_TRY(take_event(c.lib, &e0), "profile: hipEventCreate");
    NFS_TRY(take_event(c.lib, &e1), "profile: hipEventCreate");
    NFS_TRY(hipEventRecord(e0, c.s), "profile: hipEventRecord");
  }
  NFS_TRY(launch(), kind ? "encode(EH)" : "encode(E)");
  if (c.lib->profiling) {
    NFS_TRY(hipEventRecord(e1, c.s), "profile: hipEventRecord");
    c.lib->rec[kind].emplace_back(e0, e1);
  }
  return NFS_OK;
}

static int seq_pack_coefs(const Ctx& c, bool forE, bool forH) {
  const Layout& y = c.y;
  const nfs_problem* p = c.pr;
  unsigned* tmax = at<unsigned>(c.ws, y.o_tmax);
  NFS_TRY(launch_term_absmax(p->t, p->kcoef, y.K, p->b0, p->fields, y.L, y.P, tmax, c.s), "term_absmax");
  if (forE) {
    NFS_TRY(launch_pack_phase(p->b0, p->fields, y.L, y.P, 1, 0, y.NQ, tmax, at<void>(c.ws, y.o_vA), c.s),
            "pack_phase");
    NFS_TRY(launch_pack_phase(p->t, p->kcoef, y.K, y.P, 0, 1, y.NQ, tmax, at<void>(c.ws, y.o_sB), c.s),
            "pack_phase");
  }
  if (forH) {
    NFS_TRY(launch_pack_phase(p->t, p->kcoef, y.K, y.P, 0, 0, y.NQ, tmax, at<void>(c.ws, y.o_sA), c.s),
            "pack_phase");
    NFS_TRY(launch_pack_phase(p->b0, p->fields, y.L, y.P, 1, 1, y.NQ, tmax, at<void>(c.ws, y.o_vB), c.s),
            "pack_phase");
  }
  return NFS_OK;
}

static float* unscale_slot(const Ctx& c, int which) {
  return scaled_prec(c.y.prec) ? at<float>(c.ws, c.y.o_unscale) + which : nullptr;
}

// The E operand: packed Q = S o rho (o wgt); bmax_ready: the FP16 scale
// bound of Q is already in bmax
static int pre_E(const Ctx& c, const float2* rho, bool bmax_ready, const float* wgt = nullptr) {
  const Layout& y = c.y;
  float* bmax = at<float>(c.ws, y.o_bmax);
  if (scaled_prec(y.prec) && !bmax_ready) NFS_TRY(launch_absmax(rho, c.sens, wgt, y.L, 1, 0, y.G, bmax, c.stop, c.s), "absmax(Q)");
  NFS_TRY(launch_pack_data(OP_E, y.prec, rho, c.sens, wgt, y.L, 1, 0, y.G, y.NB, y.LC, at<void>(c.ws, y.o_dataE),
                           bmax, at<float>(c.ws, y.o_unscale), c.stop, c.s),
          "pack_data(E)");
  return NFS_OK;
}

// The E^H operand from src (m [G][K]) (o wgt)
static int pre_EH(const Ctx& c, const float2* src, int64_t is, int64_t cs, const float* wgt = nullptr) {
  const Layout& y = c.y;
  float* bmax = at<float>(c.ws, y.o_bmax);
  if (scaled_prec(y.prec))
    NFS_TRY(launch_absmax(src, nullptr, wgt, y.K, is, cs, y.G, bmax, c.stop, c.s), "absmax(m)");
  NFS_TRY(launch_pack_data(OP_EH, y.prec, src, nullptr, wgt, y.K, is, cs, y.G, y.NB, y.KC, at<void>(c.ws, y.o_dataH),
                           bmax, at<float>(c.ws, y.o_unscale) + 1, c.stop, c.s),
          "pack_data(EH)");
  return NFS_OK;
}

// The E^H operand of E^H E, packed straight from the E partials
// (optionally weighted per sample: E^H diag(wgt * wmul) E)
static int mid_EHE(const Ctx& c, const float* wgt = nullptr, float wmul = 1.f) {
  const Layout& y = c.y;
  float* us = at<float>(c.ws, y.o_unscale);
  NFS_TRY(launch_pack_EH_from_epart(y.prec, at<float>(c.ws, y.o_epart), y.shE.nsplit, y.KC * 16, y.NB, y.K, y.G, y.L,
                                    wgt, wmul, us, us + 1, y.KC, at<void>(c.ws, y.o_dataH), c.stop, c.s),
          "pack_EH_from_epart");
  return NFS_OK;
}

// E part: rho -> epart (partials) via packed Q = S o rho (o wgt);
// bmax_ready: the FP16 scale bound of Q is already in bmax
static int seq_E(const Ctx& c, const float2* rho, const float* wgt = nullptr, bool bmax_ready = false) {
  const Layout& y = c.y;
  int rc = pre_E(c, rho, bmax_ready, wgt);
  if (rc) return rc;
  return timed_encode(c, 0, [&] {
    if (c.PE)
      return launch_resident(y.shE, c.PE, at<void>(c.ws, y.o_dataE), at<float>(c.ws, y.o_epart), c.sens, y.L, y.G,
                             c.stop, c.s);
    return launch_encode(y.shE, at<void>(c.ws, y.o_sB), at<void>(c.ws, y.o_vA), at<void>(c.ws, y.o_dataE),
                         at<float>(c.ws, y.o_epart), c.sens, y.L, y.G, at<unsigned>(c.ws, y.o_tmax), y.P + 1, c.stop,
                         c.s);
  });
}

// E^H part: src (m [G][K]) (o wgt) -> hpart (coil-combined partials)
static int seq_EH(const Ctx& c, const float2* src, int64_t is, int64_t cs, const float* wgt = nullptr) {
  const Layout& y = c.y;
  int rc = pre_EH(c, src, is, cs, wgt);
  if (rc) return rc;
  return timed_encode(c, 1, [&] {
    if (c.PH)
      return launch_resident(y.shH, c.PH, at<void>(c.ws, y.o_dataH), at<float>(c.ws, y.o_hpart), c.sens, y.L, y.G,
                             c.stop, c.s);
    return launch_encode(y.shH, at<void>(c.ws, y.o_vB), at<void>(c.ws, y.o_sA), at<void>(c.ws, y.o_dataH),
                         at<float>(c.ws, y.o_hpart), c.sens, y.L, y.G, at<unsigned>(c.ws, y.o_tmax), y.P + 1, c.stop,
                         c.s);
  });
}

// E^H E: p -> hpart; the E^H operand is packed straight from the E partials
// (optionally weighted per sample: E^H diag(wgt * wmul) E)
static int seq_EHE(const Ctx& c, const float2* p, bool bmax_ready = false, const float* wgt = nullptr,
                   float wmul = 1.f) {
  const Layout& y = c.y;
  int rc = seq_E(c, p, nullptr, bmax_ready);
  if (rc) return rc;
  if ((rc = mid_EHE(c, wgt, wmul))) return rc;
  return timed_encode(c, 1, [&] {
    if (c.PH)
      return launch_resident(y.shH, c.PH, at<void>(c.ws, y.o_dataH), at<float>(c.ws, y.o_hpart), c.sens, y.L, y.G,
                             c.stop, c.s);
    return launch_encode(y.shH, at<void>(c.ws, y.o_vB), at<void>(c.ws, y.o_sA), at<void>(c.ws, y.o_dataH),
                         at<float>(c.ws, y.o_hpart), c.sens, y.L, y.G, at<unsigned>(c.ws, y.o_tmax), y.P + 1, c.stop,
                         c.s);
  });
}

extern "C" int nfs_apply_E(nfs_ctx* ctx, const nfs_problem* prob, const float* rho, float* m, int precision,
                           void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nfs_apply_E";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  int rc = check_problem(prob, fn);
  if (rc) return rc;
  if ((rc = check_prec(precision, fn))) return rc;
  if ((rc = check_vec(rho, prob->n_vox, fn, "rho"))) return rc;
  if ((rc = check_vec(m, prob->n_samp, fn, "m"))) return rc;
  const Layout y = make_layout(ctx, prob, NFS_OP_E, precision, 0, 0);
  if ((rc = check_ws(y, ws, ws_bytes, fn))) return rc;
  if (y.K == 0) return NFS_OK;
  Ctx c{ctx, y, prob, reinterpret_cast<const float2*>(prob->sens), ws, (hipStream_t)stream, nullptr};
  if ((rc = seq_pack_coefs(c, true, false))) return rc;
  if ((rc = seq_E(c, reinterpret_cast<const float2*>(rho)))) return rc;
  NFS_TRY(launch_finish_E_to_m(at<float>(ws, y.o_epart), y.shE.nsplit, y.KC * 16, y.NB, y.K, y.G, unscale_slot(c, 0),
                               reinterpret_cast<float2*>(m), c.s),
          "finish_E_to_m");
  return NFS_OK;
}

extern "C" int nfs_apply_EH(nfs_ctx* ctx, const nfs_problem* prob, const float* m, float* x, int precision, void* ws,
                            size_t ws_bytes, void* stream) {
  const char* fn = "nfs_apply_EH";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  int rc = check_problem(prob, fn);
  if (rc) return rc;
  if ((rc = check_prec(precision, fn))) return rc;
  if ((rc = check_vec(m, prob->n_samp, fn, "m"))) return rc;
  if ((rc = check_vec(x, prob->n_vox, fn, "x"))) return rc;
  const Layout y = make_layout(ctx, prob, NFS_OP_EH, precision, 0, 0);
  if ((rc = check_ws(y, ws, ws_bytes, fn))) return rc;
  if (y.L == 0) return NFS_OK;
  Ctx c{ctx, y, prob, reinterpret_cast<const float2*>(prob->sens), ws, (hipStream_t)stream, nullptr};
  if ((rc = seq_pack_coefs(c, false, true))) return rc;
  if ((rc = seq_EH(c, reinterpret_cast<const float2*>(m), 1, y.K))) return rc;
  NFS_TRY(launch_finish_EH(at<float2>(ws, y.o_hpart), y.shH.nsplit, y.LC * 16, y.L, unscale_slot(c, 1),
                           reinterpret_cast<float2*>(x), c.s),
          "finish_EH");
  return NFS_OK;
}

extern "C" int nfs_apply_EHE(nfs_ctx* ctx, const nfs_problem* prob, const float* p, float* q, int precision,
                             void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nfs_apply_EHE";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  int rc = check_problem(prob, fn);
  if (rc) return rc;
  if ((rc = check_prec(precision, fn))) return rc;
  if ((rc = check_vec(p, prob->n_vox, fn, "p"))) return rc;
  if ((rc = check_vec(q, prob->n_vox, fn, "q"))) return rc;
  const Layout y = make_layout(ctx, prob, NFS_OP_EHE, precision, 0, 0);
  if ((rc = check_ws(y, ws, ws_bytes, fn))) return rc;
  if (y.L == 0) return NFS_OK;
  Ctx c{ctx, y, prob, reinterpret_cast<const float2*>(prob->sens), ws, (hipStream_t)stream, nullptr};
  if ((rc = seq_pack_coefs(c, true, true))) return rc;
  if ((rc = seq_EHE(c, reinterpret_cast<const float2*>(p)))) return rc;
  NFS_TRY(launch_finish_EH(at<float2>(ws, y.o_hpart), y.shH.nsplit, y.LC * 16, y.L, unscale_slot(c, 1),
                           reinterpret_cast<float2*>(q), c.s),
          "finish_EH");
  return NFS_OK;
}

static int check_cg_args(const nfs_ctx* ctx, const nfs_problem* prob, const float* m, const float* rho, int n_iter,
                         double tol, int replace_every, int reorth, int precision, const double* hist, const int* info,
                         const char* fn) {
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  int rc = check_problem(prob, fn);
  if (rc) return rc;
  if ((rc = check_prec(precision, fn))) return rc;
  if ((rc = check_vec(m, prob->n_samp, fn, "m"))) return rc;
  if ((rc = check_vec(rho, prob->n_vox, fn, "rho"))) return rc;
  if (n_iter < 0) return fail(NFS_EINVAL, "%s: n_iter %d < 0", fn, n_iter);
  if (!std::isfinite(tol) || tol < 0.0) return fail(NFS_EINVAL, "%s: tol must be finite and >= 0", fn);
  if (replace_every < 0) return fail(NFS_EINVAL, "%s: replace_every %d < 0", fn, replace_every);
  if (reorth != 0 && reorth != 1) return fail(NFS_EINVAL, "%s: reorth must be 0 or 1", fn);
  if (reorth && n_iter > kMaxReorth) return fail(NFS_EINVAL, "%s: reorth needs n_iter <= %d", fn, kMaxReorth);
  if (misaligned(hist, 8)) return fail(NFS_EINVAL, "%s: hist not 8-byte aligned", fn);
  if (misaligned(info, 4)) return fail(NFS_EINVAL, "%s: info not 4-byte aligned", fn);
  return NFS_OK;
}

// The launch sequence of one CG solve (arguments already checked).
// resident: build P once (the non-split form) and stream it in every E and
// E^H instead of rebuilding the phase tiles
static int run_cg(nfs_ctx* ctx, const nfs_problem* prob, const Layout& y, const float* m, float* rho, int n_iter,
                  double tol, int replace_every, int reorth, double* hist, int* info, void* ws, hipStream_t s,
                  bool resident = false, float* iterates = nullptr) {
  int rc;
  CgState st;
  st.r = at<float2>(ws, y.o_r);
  st.p = at<float2>(ws, y.o_p);
  st.q = at<float2>(ws, y.o_q);
  st.b = at<float2>(ws, y.o_b);
  st.part = at<double>(ws, y.o_part);
  st.alpha = at<double>(ws, y.o_alpha);
  st.scal = at<double>(ws, y.o_scal);
  st.hist = hist ? hist : at<double>(ws, y.o_hist);
  st.info = info ? info : at<int>(ws, y.o_info);
  st.stop = at<int>(ws, y.o_stop);
  st.V = reorth ? at<float2>(ws, y.o_V) : nullptr;
  st.rn = reorth ? at<float2>(ws, y.o_rn) : nullptr;
  st.iters = reinterpret_cast<float2*>(iterates);
  st.icorr = prob->icorr;
  st.rpart = reorth ? at<double>(ws, y.o_rpart) : nullptr;
  const bool f16ops = scaled_prec(y.prec);  // f16 operand fragments, power-of-two scaled
  st.smax = f16ops ? at<float>(ws, y.o_smax) : nullptr;
  st.bmax = f16ops ? at<float>(ws, y.o_bmax) : nullptr;
  st.L = y.L;
  int64_t nb = cdiv(y.L, 256);
  st.nblk = (int)(nb < 1 ? 1 : (nb > kCgBlocks ? kCgBlocks : nb));

  const float2* sens = reinterpret_cast<const float2*>(prob->sens);
  if (prob->icorr && y.L > 0) {
    float2* sj = at<float2>(ws, y.o_sensj);
    NFS_TRY(launch_scale_sens(sens, prob->icorr, y.G, y.L, sj, s), "scale_sens");
    sens = sj;
  }
  if (f16ops) NFS_TRY(launch_sens_absmax(sens, y.G, y.L, at<float>(ws, y.o_smax), s), "sens_absmax");
  Ctx c{ctx, y, prob, sens, ws, s, st.stop};
  float2* x = reinterpret_cast<float2*>(rho);
  const float2* hpart = at<float2>(ws, y.o_hpart);
  const int64_t hstride = y.LC * 16;
  const int ns = y.shH.nsplit;

  NFS_TRY(launch_cg_reset(st, s), "cg_reset");
  if ((rc = seq_pack_coefs(c, true, true))) return rc;
  if (resident) {
    const unsigned* tmax = at<unsigned>(ws, y.o_tmax);
    NFS_TRY(launch_build_P(y.NQ, at<void>(ws, y.o_sB), at<void>(ws, y.o_vA), y.KC, y.LC, tmax, y.P + 1,
                           at<void>(ws, y.o_PE), s),
            "build_P(E)");
    NFS_TRY(launch_build_P(y.NQ, at<void>(ws, y.o_vB), at<void>(ws, y.o_sA), y.LC, y.KC, tmax, y.P + 1,
                           at<void>(ws, y.o_PH), s),
            "build_P(EH)");
    c.PE = at<void>(ws, y.o_PE);
    c.PH = at<void>(ws, y.o_PH);
  }
  NFS_TRY(launch_cg_norm_m(st, reinterpret_cast<const float2*>(m), (int64_t)y.G * y.K, s), "cg_norm_m");
  if ((rc = seq_EH(c, reinterpret_cast<const float2*>(m), 1, y.K))) return rc;
  NFS_TRY(launch_cg_init(st, hpart, ns, hstride, unscale_slot(c, 1), x, y.L, s), "cg_init");
  NFS_TRY(launch_cg_start(st, n_iter, s), "cg_start");
  if (reorth) NFS_TRY(launch_cg_store_v(st, 0, s), "cg_store_v");
  for (int n = 0; n < n_iter; ++n) {
    if ((rc = seq_EHE(c, st.p, f16ops))) return rc;
    NFS_TRY(launch_cg_beta(st, hpart, ns, hstride, unscale_slot(c, 1), y.L, s), "cg_beta");
    // the re-orthogonalisation dot products come with the kernel that
    // writes the final r of this iteration (update, or the replacement)
    const bool replace = replace_every > 0 && (n + 1) % replace_every == 0 && n + 1 < n_iter;
    const int nv = reorth ? n + 1 : 0;
    NFS_TRY(launch_cg_update(st, x, y.L, n, replace ? 0 : nv, s), "cg_update");
    if (replace) {
      if ((rc = seq_EHE(c, x))) return rc;
      NFS_TRY(launch_cg_replace(st, hpart, ns, hstride, unscale_slot(c, 1), y.L, nv, s), "cg_replace");
    }
    if (reorth) NFS_TRY(launch_cg_reorth_apply(st, nv, !replace, s), "cg_reorth_apply");
    NFS_TRY(launch_cg_direction(st, y.L, n, n_iter, tol, s), "cg_direction");
  }
  NFS_TRY(launch_cg_finish(st, x, prob->icorr, y.L, s), "cg_finish");
  return NFS_OK;
}

// ---------------------------------------------------------------------------
// Optional hipGraph capture of whole solves (nfs_set_graphs).  A graph is
// keyed by every pointer and parameter the launch sequence bakes in; the
// first call captures and instantiates it, later identical calls replay it
// with one hipGraphLaunch.  Not used while the caller's stream is itself
// being captured (the launches then simply go into the caller's graph) or
// while kernel profiling is on.
static std::string graph_key(const nfs_ctx* ctx, const char* kind, const nfs_problem* probs, int n,
                             const void* const* ptrs, int np, int n_iter, double tol, int replace_every, int reorth,
                             int precision, const void* ws, size_t ws_bytes, const void* stream) {
  std::string k(kind);
  k.append(reinterpret_cast<const char*>(&ctx->tune_generation), sizeof ctx->tune_generation);
  auto add = [&](const void* p, size_t len) { k.append(static_cast<const char*>(p), len); };
  for (int i = 0; i < n; ++i) add(&probs[i], sizeof(nfs_problem));
  for (int i = 0; i < np; ++i) add(&ptrs[i], sizeof(void*));
  add(&n_iter, sizeof n_iter);
  add(&tol, sizeof tol);
  add(&replace_every, sizeof replace_every);
  add(&reorth, sizeof reorth);
  add(&precision, sizeof precision);
  add(&ws, sizeof ws);
  add(&ws_bytes, sizeof ws_bytes);
  add(&stream, sizeof stream);
  return k;
}

// Capture happens on a library-owned stream (the caller's stream may be the
// legacy null stream, which cannot be captured); the instantiated graph is
// then launched on the caller's stream, after the work already queued there.
constexpr size_t kMaxGraphs = 32;

// Drop the least recently used graph once the cache is full (callers that
// pass fresh output buffers on every call would otherwise grow it without
// bound); waits for that graph's last launch first.
static int evict_graph(nfs_ctx* ctx) {
  auto lru = ctx->graph_cache.begin();
  for (auto it = ctx->graph_cache.begin(); it != ctx->graph_cache.end(); ++it)
    if (it->second.last_use < lru->second.last_use) lru = it;
  if (lru == ctx->graph_cache.end()) return NFS_OK;
  if (lru->second.done) NFS_TRY(hipEventSynchronize(lru->second.done), "hipEventSynchronize");
  NFS_TRY(hipGraphExecDestroy(lru->second.ex), "hipGraphExecDestroy");
  if (lru->second.done) NFS_TRY(hipEventDestroy(lru->second.done), "hipEventDestroy");
  ctx->graph_cache.erase(lru);
  return NFS_OK;
}

template <class F>
static int run_maybe_graph(nfs_ctx* ctx, const std::string& key, hipStream_t s, F&& enqueue) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (s) NFS_TRY(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
  if (!ctx->graphs || ctx->profiling || cs != hipStreamCaptureStatusNone) return enqueue(s);
  auto it = ctx->graph_cache.find(key);
  if (it == ctx->graph_cache.end()) {
    if (!ctx->capture_stream) {
      int cur = 0;
      NFS_TRY(hipGetDevice(&cur), "hipGetDevice");
      NFS_TRY(hipSetDevice(ctx->device), "hipSetDevice");
      const hipError_t ec = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
      NFS_TRY(hipSetDevice(cur), "hipSetDevice");
      NFS_TRY(ec, "hipStreamCreateWithFlags");
    }
    hipStream_t cap = ctx->capture_stream;
    NFS_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    const int rc = enqueue(cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cap, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return hip_fail(e2, "hipGraphInstantiate");
    hipEvent_t done = nullptr;
    const hipError_t e3 = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e3 != hipSuccess) {
      (void)hipGraphExecDestroy(ex);
      return hip_fail(e3, "hipEventCreateWithFlags");
    }
    if (ctx->graph_cache.size() >= kMaxGraphs) {
      const int rc2 = evict_graph(ctx);
      if (rc2) {
        (void)hipGraphExecDestroy(ex);
        (void)hipEventDestroy(done);
        return rc2;
      }
    }
    it = ctx->graph_cache.emplace(key, nfs_ctx::Graph{ex, done, 0}).first;
  }
  it->second.last_use = ++ctx->graph_clock;
  NFS_TRY(hipGraphLaunch(it->second.ex, s), "hipGraphLaunch");
  NFS_TRY(hipEventRecord(it->second.done, s), "hipEventRecord");
  return NFS_OK;
}

extern "C" int nfs_set_graphs(nfs_ctx* ctx, int on) {
  if (!ctx) return fail(NFS_EINVAL, "nfs_set_graphs: ctx is NULL");
  ctx->graphs = on != 0;
  return NFS_OK;
}

extern "C" int nfs_cg_solve(nfs_ctx* ctx, const nfs_problem* prob, const float* m, float* rho, int n_iter,
                            double tol, int replace_every, int reorth, int precision, double* hist, int* info,
                            void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nfs_cg_solve";
  int rc = check_cg_args(ctx, prob, m, rho, n_iter, tol, replace_every, reorth, precision, hist, info, fn);
  if (rc) return rc;
  const Layout y = make_layout(ctx, prob, NFS_OP_CG, precision, n_iter, reorth);
  if ((rc = check_ws(y, ws, ws_bytes, fn))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const void* ptrs[4] = {m, rho, hist, info};
  const std::string key =
      graph_key(ctx, "cg", prob, 1, ptrs, 4, n_iter, tol, replace_every, reorth, precision, ws, ws_bytes, stream);
  return run_maybe_graph(ctx, key, s, [&](hipStream_t st) {
    return run_cg(ctx, prob, y, m, rho, n_iter, tol, replace_every, reorth, hist, info, ws, st);
  });
}

extern "C" int nfs_cg_solve_noalloc(nfs_ctx* ctx, const nfs_problem* prob, const float* m, float* rho, int n_iter,
                                    double tol, int replace_every, int reorth, int precision, double* hist, int* info,
                                    void* stream) {
  const char* fn = "nfs_cg_solve_noalloc";
  int rc = check_cg_args(ctx, prob, m, rho, n_iter, tol, replace_every, reorth, precision, hist, info, fn);
  if (rc) return rc;
  const Layout y = make_layout(ctx, prob, NFS_OP_CG, precision, n_iter, reorth);
  if (y.total > kScratchBytes)
    return fail(NFS_EWORKSPACE, "%s: the solve needs %zu bytes of scratch, more than the %zu the library holds", fn,
                y.total, kScratchBytes);
  if (!ctx->scratch) return fail(NFS_EHIP, "%s: no scratch address for device %d", fn, ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const void* ptrs[4] = {m, rho, hist, info};
  const std::string key = graph_key(ctx, "cgn", prob, 1, ptrs, 4, n_iter, tol, replace_every, reorth, precision,
                                    ctx->scratch, kScratchBytes, stream);
  return run_maybe_graph(ctx, key, s, [&](hipStream_t st) {
    return run_cg(ctx, prob, y, m, rho, n_iter, tol, replace_every, reorth, hist, info, ctx->scratch, st);
  });
}

extern "C" int nfs_cg_solve_resident(nfs_ctx* ctx, const nfs_problem* prob, const float* m, float* rho, int n_iter,
                                     double tol, int replace_every, int reorth, int precision, double* hist,
                                     int* info, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nfs_cg_solve_resident";
  int rc = check_cg_args(ctx, prob, m, rho, n_iter, tol, replace_every, reorth, precision, hist, info, fn);
  if (rc) return rc;
  if (precision != NFS_FP16) return fail(NFS_EUNSUPPORTED, "%s: the resident form takes NFS_FP16 operands", fn);
  const Layout y = make_layout(ctx, prob, NFS_OP_CG_RESIDENT, precision, n_iter, reorth);
  if ((rc = check_ws(y, ws, ws_bytes, fn))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const void* ptrs[4] = {m, rho, hist, info};
  const std::string key =
      graph_key(ctx, "cgr", prob, 1, ptrs, 4, n_iter, tol, replace_every, reorth, precision, ws, ws_bytes, stream);
  return run_maybe_graph(ctx, key, s, [&](hipStream_t st) {
    return run_cg(ctx, prob, y, m, rho, n_iter, tol, replace_every, reorth, hist, info, ws, st, true);
  });
}

extern "C" int nfs_cg_solve_traced(nfs_ctx* ctx, const nfs_problem* prob, const float* m, float* rho, int n_iter,
                                   double tol, int replace_every, int reorth, int precision, double* hist, int* info,
                                   float* iterates, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nfs_cg_solve_traced";
  int rc = check_cg_args(ctx, prob, m, rho, n_iter, tol, replace_every, reorth, precision, hist, info, fn);
  if (rc) return rc;
  if ((rc = check_vec(iterates, (int64_t)(n_iter + 1) * prob->n_vox, fn, "iterates"))) return rc;
  const Layout y = make_layout(ctx, prob, NFS_OP_CG, precision, n_iter, reorth);
  if ((rc = check_ws(y, ws, ws_bytes, fn))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const void* ptrs[5] = {m, rho, hist, info, iterates};
  const std::string key =
      graph_key(ctx, "cgt", prob, 1, ptrs, 5, n_iter, tol, replace_every, reorth, precision, ws, ws_bytes, stream);
  return run_maybe_graph(ctx, key, s, [&](hipStream_t st) {
    return run_cg(ctx, prob, y, m, rho, n_iter, tol, replace_every, reorth, hist, info, ws, st, false, iterates);
  });
}

// ---------------------------------------------------------------------------
// Stopping-criteria instrumentation: SSIM of iterates against a reference,
// and the L-curve corner.
static int check_ssim_dims(int n_img, int nx, int ny, int nz, const char* fn) {
  if (n_img < 0) return fail(NFS_EINVAL, "%s: n_img %d < 0", fn, n_img);
  if (nx < 11 || ny < 11 || !(nz == 1 || nz >= 11))
    return fail(NFS_ESHAPE, "%s: image %d x %d x %d: needs nx, ny >= 11 and nz == 1 or >= 11", fn, nx, ny, nz);
  if ((int64_t)nx * ny * nz > ((int64_t)1 << 26)) return fail(NFS_ESHAPE, "%s: image too large", fn);
  return NFS_OK;
}

extern "C" int nfs_ssim_workspace_bytes(int n_img, int nx, int ny, int nz, size_t* bytes) {
  const char* fn = "nfs_ssim_workspace_bytes";
  if (!bytes) return fail(NFS_EINVAL, "%s: bytes is NULL", fn);
  int rc = check_ssim_dims(n_img, nx, ny, nz, fn);
  if (rc) return rc;
  *bytes = ssim_workspace_bytes(n_img, nx, ny, nz);
  return NFS_OK;
}

extern "C" int nfs_ssim(nfs_ctx* ctx, const float* imgs, int n_img, const float* ref, int nx, int ny, int nz,
                        double* out, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nfs_ssim";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  int rc = check_ssim_dims(n_img, nx, ny, nz, fn);
  if (rc) return rc;
  const int64_t L = (int64_t)nx * ny * nz;
  if ((rc = check_vec(imgs, (int64_t)n_img * L, fn, "imgs"))) return rc;
  if ((rc = check_vec(ref, L, fn, "ref"))) return rc;
  if (n_img > 0 && !out) return fail(NFS_EINVAL, "%s: out is NULL", fn);
  if (misaligned(out, 8)) return fail(NFS_EINVAL, "%s: out not 8-byte aligned", fn);
  const size_t need = ssim_workspace_bytes(n_img, nx, ny, nz);
  if (!ws) return fail(NFS_EWORKSPACE, "%s: workspace is NULL", fn);
  if ((uintptr_t)ws % 256) return fail(NFS_EWORKSPACE, "%s: workspace not 256-byte aligned", fn);
  if (ws_bytes < need) return fail(NFS_EWORKSPACE, "%s: workspace has %zu bytes, needs %zu", fn, ws_bytes, need);
  NFS_TRY(launch_ssim(reinterpret_cast<const float2*>(imgs), n_img, reinterpret_cast<const float2*>(ref), nx, ny, nz,
                      out, ws, (hipStream_t)stream),
          "ssim");
  return NFS_OK;
}

extern "C" int nfs_lcurve_corner(const double* hist, int n_rows, int* corner, double* kappa) {
  const char* fn = "nfs_lcurve_corner";
  if (n_rows < 0) return fail(NFS_EINVAL, "%s: n_rows %d < 0", fn, n_rows);
  if ((n_rows > 0 && !hist) || !corner) return fail(NFS_EINVAL, "%s: NULL argument", fn);
  // usable rows: ||rho_n|| and ||d_n||^2 positive and finite
  std::vector<int> rows;
  for (int n = 0; n < n_rows; ++n) {
    const double xr = hist[3 * n + 1], d2 = hist[3 * n + 2];
    if (std::isfinite(xr) && std::isfinite(d2) && xr > 0.0 && d2 > 0.0) rows.push_back(n);
  }
  if (kappa)
    for (int n = 0; n < n_rows; ++n) kappa[n] = std::nan("");
  *corner = -1;
  double best = 0.0;
  for (size_t j = 1; j + 1 < rows.size(); ++j) {
    double px[3], py[3];
    for (int t = 0; t < 3; ++t) {
      const int n = rows[j - 1 + t];
      px[t] = std::log(hist[3 * n + 1]);
      py[t] = 0.5 * std::log(hist[3 * n + 2]);
    }
    const double ax = px[1] - px[0], ay = py[1] - py[0];
    const double bx = px[2] - px[1], by = py[2] - py[1];
    const double cx = px[2] - px[0], cy = py[2] - py[0];
    const double cross = ax * by - ay * bx;
    const double den = std::hypot(ax, ay) * std::hypot(bx, by) * std::hypot(cx, cy);
    if (!(den > 0.0)) continue;
    const double k = 2.0 * cross / den;
    if (kappa) kappa[rows[j]] = k;
    if (*corner < 0 || k > best) {
      best = k;
      *corner = rows[j];
    }
  }
  return NFS_OK;
}

// ---------------------------------------------------------------------------
// k-space filter: rho_f = IFFT(FFT(rho) o f), one DFT pass per axis and
// direction (axes of length 1 skipped), the filter and 1/L applied with the
// last forward pass; the passes alternate between the workspace ([L]
// complex) and `out`, so that the last one writes `out`.
static int check_filter_dims(int nx, int ny, int nz, const char* fn) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(NFS_ESHAPE, "%s: grid %d x %d x %d", fn, nx, ny, nz);
  if (nx > kMaxDftAxis || ny > kMaxDftAxis || nz > kMaxDftAxis)
    return fail(NFS_ESHAPE, "%s: grid %d x %d x %d has an axis longer than %d", fn, nx, ny, nz, kMaxDftAxis);
  if ((int64_t)nx * ny * nz > ((int64_t)1 << 26)) return fail(NFS_ESHAPE, "%s: grid too large", fn);
  return NFS_OK;
}

extern "C" int nfs_kspace_filter_workspace_bytes(const nfs_ctx* ctx, int nx, int ny, int nz, size_t* bytes) {
  const char* fn = "nfs_kspace_filter_workspace_bytes";
  (void)ctx;
  if (!bytes) return fail(NFS_EINVAL, "%s: bytes is NULL", fn);
  int rc = check_filter_dims(nx, ny, nz, fn);
  if (rc) return rc;
  *bytes = al((size_t)nx * ny * nz * 8);
  return NFS_OK;
}

extern "C" int nfs_apply_kspace_filter(nfs_ctx* ctx, const float* rho, float* out, int nx, int ny, int nz,
                                       const float* f, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nfs_apply_kspace_filter";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  int rc = check_filter_dims(nx, ny, nz, fn);
  if (rc) return rc;
  const int64_t L = (int64_t)nx * ny * nz;
  if ((rc = check_vec(rho, L, fn, "rho"))) return rc;
  if ((rc = check_vec(out, L, fn, "out"))) return rc;
  if (!f) return fail(NFS_EINVAL, "%s: f is NULL", fn);
  if (misaligned(f, 4)) return fail(NFS_EINVAL, "%s: f not 4-byte aligned", fn);
  if (!ws) return fail(NFS_EWORKSPACE, "%s: workspace is NULL", fn);
  if ((uintptr_t)ws % 256) return fail(NFS_EWORKSPACE, "%s: workspace not 256-byte aligned", fn);
  if (ws_bytes < al((size_t)L * 8))
    return fail(NFS_EWORKSPACE, "%s: workspace has %zu bytes, needs %zu", fn, ws_bytes, al((size_t)L * 8));
  hipStream_t s = (hipStream_t)stream;
  // axes as [outer][n][inner] views: x (contiguous), y, z
  struct Axis {
    int n;
    int64_t outer, inner;
  };
  std::vector<Axis> axes;
  if (nx > 1) axes.push_back({nx, (int64_t)ny * nz, 1});
  if (ny > 1) axes.push_back({ny, (int64_t)nz, (int64_t)nx});
  if (nz > 1) axes.push_back({nz, 1, (int64_t)nx * ny});
  const float inv_l = (float)(1.0 / (double)L);
  const float2* src = reinterpret_cast<const float2*>(rho);
  float2* dst_out = reinterpret_cast<float2*>(out);
  float2* dst_ws = static_cast<float2*>(ws);
  if (axes.empty()) {
    NFS_TRY(launch_filter_scale(src, dst_out, f, inv_l, L, s), "filter_scale");
    return NFS_OK;
  }
  const int passes = 2 * (int)axes.size();
  for (int i = 0; i < passes; ++i) {
    const bool fwd = i < (int)axes.size();
    const Axis& ax = fwd ? axes[i] : axes[passes - 1 - i];
    const bool last_fwd = i + 1 == (int)axes.size();
    float2* dst = (passes - 1 - i) % 2 == 0 ? dst_out : dst_ws;
    NFS_TRY(launch_dft_axis(src, dst, ax.outer, ax.n, ax.inner, fwd ? -1 : +1, last_fwd ? inv_l : 1.f,
                            last_fwd ? f : nullptr, s),
            "dft_axis");
    src = dst;
  }
  return NFS_OK;
}

// Filter mask from the first-order k-space positions (host arithmetic):
// Andrew's monotone chain builds the convex hull; a bin is inside when it is
// on the inner side of (or on) every hull edge, up to a relative tolerance.
// ---------------------------------------------------------------------------
// 3D convex hull (quickhull): the face planes n.x <= d (unit n) of the hull
// of pts [n][3].  Points are assigned to a face they lie above (conflict
// lists); the farthest point of a face is added by deleting the faces it
// sees and joining the horizon edges to it.  Returns false for point sets
// without volume (all points on a plane).
namespace {

struct HullFace {
  int v[3];       // counter-clockwise seen from outside
  int nb[3];      // face across edge v[i] -> v[(i + 1) % 3]
  double n[3], d;
  bool alive;
  std::vector<int> pts;
};

struct Hull3 {
  const double* P;
  double eps;
  std::vector<HullFace> F;
  std::vector<int64_t> mark;  // visit stamps of the current step (2 r: visible, 2 r + 1: not)
  int64_t round = 0;

  const double* pt(int i) const { return P + 3 * (size_t)i; }
  double dist(const HullFace& f, int i) const {
    const double* q = pt(i);
    return f.n[0] * q[0] + f.n[1] * q[1] + f.n[2] * q[2] - f.d;
  }
  int add_face(int a, int b, int c) {
    HullFace f;
    f.v[0] = a;
    f.v[1] = b;
    f.v[2] = c;
    f.nb[0] = f.nb[1] = f.nb[2] = -1;
    const double *A = pt(a), *B = pt(b), *C = pt(c);
    const double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    const double w[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int k = 0; k < 3; ++k) f.n[k] = len > 0 ? n[k] / len : 0.0;
    f.d = f.n[0] * A[0] + f.n[1] * A[1] + f.n[2] * A[2];
    f.alive = true;
    F.push_back(std::move(f));
    return (int)F.size() - 1;
  }
  // link faces sharing an edge (a -> b in one, b -> a in the other)
  void link_all(const std::vector<int>& ids) {
    std::map<std::pair<int, int>, std::pair<int, int>> edge;  // (a, b) -> (face, edge index)
    for (int f : ids)
      for (int e = 0; e < 3; ++e) edge[{F[f].v[e], F[f].v[(e + 1) % 3]}] = {f, e};
    for (int f : ids)
      for (int e = 0; e < 3; ++e) {
        auto it = edge.find({F[f].v[(e + 1) % 3], F[f].v[e]});
        if (it != edge.end()) F[f].nb[e] = it->second.first;
      }
  }

  // Four points spanning a tetrahedron thicker than eps in every sense:
  // the extremes along the axis of largest extent, the point farthest from
  // their line, the point farthest from that plane; false if none exist.
  bool simplex(int64_t n, int tv[4]) {
    if (n < 4) return false;
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int64_t i = 1; i < n; ++i)
      for (int k = 0; k < 3; ++k) {
        if (pt((int)i)[k] < pt(lo[k])[k]) lo[k] = (int)i;
        if (pt((int)i)[k] > pt(hi[k])[k]) hi[k] = (int)i;
      }
    int ax = 0;
    for (int k = 1; k < 3; ++k)
      if (pt(hi[k])[k] - pt(lo[k])[k] > pt(hi[ax])[ax] - pt(lo[ax])[ax]) ax = k;
    const int i0 = lo[ax], i1 = hi[ax];
    if (!(pt(i1)[ax] - pt(i0)[ax] > eps)) return false;
    const double* a = pt(i0);
    const double* b = pt(i1);
    const double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    int i2 = -1;
    double best = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double* q = pt((int)i);
      const double aq[3] = {q[0] - a[0], q[1] - a[1], q[2] - a[2]};
      const double c[3] = {ab[1] * aq[2] - ab[2] * aq[1], ab[2] * aq[0] - ab[0] * aq[2], ab[0] * aq[1] - ab[1] * aq[0]};
      const double d2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
      if (d2 > best) {
        best = d2;
        i2 = (int)i;
      }
    }
    const double lab = std::sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
    if (i2 < 0 || !(std::sqrt(best) / lab > eps)) return false;
    const int t = add_face(i0, i1, i2);
    int i3 = -1;
    best = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double dd = std::fabs(dist(F[t], (int)i));
      if (dd > best) {
        best = dd;
        i3 = (int)i;
      }
    }
    F.clear();
    if (i3 < 0 || !(best > eps)) return false;
    tv[0] = i0;
    tv[1] = i1;
    tv[2] = i2;
    tv[3] = i3;
    return true;
  }

  bool build(int64_t n) {
    int tv[4];
    if (!simplex(n, tv)) return false;
    const int i0 = tv[0], i1 = tv[1], i2 = tv[2], i3 = tv[3];
    // the tetrahedron, every face oriented away from its centroid
    double cen[3] = {0, 0, 0};
    for (int q : tv)
      for (int k = 0; k < 3; ++k) cen[k] += 0.25 * pt(q)[k];
    const int fv[4][3] = {{0, 1, 2}, {0, 3, 1}, {1, 3, 2}, {2, 3, 0}};
    std::vector<int> ids;
    for (auto& f3 : fv) {
      int id = add_face(tv[f3[0]], tv[f3[1]], tv[f3[2]]);
      const HullFace& f = F[id];
      if (f.n[0] * cen[0] + f.n[1] * cen[1] + f.n[2] * cen[2] - f.d > 0) {
        F.pop_back();
        id = add_face(tv[f3[0]], tv[f3[2]], tv[f3[1]]);
      }
      ids.push_back(id);
    }
    link_all(ids);
    for (int64_t i = 0; i < n; ++i) {
      if (i == i0 || i == i1 || i == i2 || i == i3) continue;
      for (int f : ids)
        if (dist(F[f], (int)i) > eps) {
          F[f].pts.push_back((int)i);
          break;
        }
    }
    std::vector<int> work(ids);
    while (!work.empty()) {
      const int f0 = work.back();
      work.pop_back();
      if (!F[f0].alive || F[f0].pts.empty()) continue;
      // farthest conflict point
      int p = -1;
      double far = -1.0;
      for (int q : F[f0].pts) {
        const double dd = dist(F[f0], q);
        if (dd > far) {
          far = dd;
          p = q;
        }
      }
      // faces visible from p (connected region around f0) and its horizon
      std::vector<int> vis{f0}, stack{f0};
      ++round;
      if (mark.size() < F.size()) mark.resize(F.size() + F.size() / 2, 0);
      auto seen = [&](int g) { return mark[g] == 2 * round ? 1 : mark[g] == 2 * round + 1 ? 2 : 0; };
      mark[f0] = 2 * round;
      std::vector<std::pair<int, int>> horizon;  // (visible face, edge index)
      while (!stack.empty()) {
        const int f = stack.back();
        stack.pop_back();
        for (int e = 0; e < 3; ++e) {
          const int g = F[f].nb[e];
          if (g < 0) return false;  // broken adjacency (degenerate input)
          const int sg = seen(g);
          if (sg == 1) continue;
          if (sg == 2) {
            horizon.push_back({f, e});
            continue;
          }
          if (dist(F[g], p) > eps) {
            mark[g] = 2 * round;
            vis.push_back(g);
            stack.push_back(g);
          } else {
            mark[g] = 2 * round + 1;
            horizon.push_back({f, e});
          }
        }
      }
      // new faces (a, b, p) on the horizon edges a -> b
      std::map<int, int> start, end;  // horizon vertex -> new face starting / ending there
      std::vector<int> fresh;
      for (auto& he : horizon) {
        const int a = F[he.first].v[he.second], b = F[he.first].v[(he.second + 1) % 3];
        const int g = F[he.first].nb[he.second];
        const int nf = add_face(a, b, p);
        F[nf].nb[0] = g;
        for (int e = 0; e < 3; ++e)
          if (F[g].v[e] == b && F[g].v[(e + 1) % 3] == a) F[g].nb[e] = nf;
        if (start.count(a) || end.count(b)) return false;  // the horizon is not a simple cycle
        start[a] = nf;
        end[b] = nf;
        fresh.push_back(nf);
      }
      for (int nf : fresh) {
        const int a = F[nf].v[0], b = F[nf].v[1];
        if (!start.count(b) || !end.count(a)) return false;
        F[nf].nb[1] = start[b];  // across b -> p
        F[nf].nb[2] = end[a];    // across p -> a
      }
      // hand the orphaned conflict points to the new faces
      for (int f : vis) {
        F[f].alive = false;
        for (int q : F[f].pts) {
          if (q == p) continue;
          for (int nf : fresh)
            if (dist(F[nf], q) > eps) {
              F[nf].pts.push_back(q);
              break;
            }
        }
        std::vector<int>().swap(F[f].pts);
      }
      for (int nf : fresh) work.push_back(nf);
    }
    return true;
  }
};

}  // namespace

// Unit-normal face planes (n0, n1, n2, d) of the hull of pts [n][3]; false
// if the points do not span a volume.  The points are first joggled by a
// fixed pseudo-random offset of at most 5e-10 of their largest coordinate
// (trajectory samples lie on smooth curves, many nearly coplanar with hull
// faces, where the region a new point sees is otherwise not a disk); the
// faces therefore move by at most that much.
static bool convex_hull_3d(const double* pts, int64_t n, double scale, std::vector<std::array<double, 4>>* planes) {
  const double s = scale > 1.0 ? scale : 1.0;
  {
    // the unjoggled points must span a volume well above the joggle
    Hull3 h0;
    h0.P = pts;
    h0.eps = 1e-7 * s;
    int tv[4];
    if (!h0.simplex(n, tv)) return false;
  }
  std::vector<double> q(pts, pts + 3 * n);
  uint64_t st = 88172645463325252ULL;  // xorshift64
  for (double& x : q) {
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    x += 1e-9 * s * ((double)(st >> 11) / 9007199254740992.0 - 0.5);
  }
  Hull3 h;
  h.P = q.data();
  h.eps = 1e-12 * s;
  if (!h.build(n)) return false;
  planes->clear();
  for (const HullFace& f : h.F)
    if (f.alive) planes->push_back({f.n[0], f.n[1], f.n[2], f.d});
  return !planes->empty();
}

// Mask of the bins of an nx x ny x nz grid inside the hull planes: per
// (x, y) column the planes bound z to one interval (tol: slack in the
// plane distance, so that bins on the hull count as inside).
static int64_t mask_from_planes(const std::vector<std::array<double, 4>>& planes, int nx, int ny, int nz, double tol,
                                unsigned char* mask) {
  auto freq = [](int i, int n) { return (double)(i < (n + 1) / 2 ? i : i - n); };
  int64_t count = 0;
  for (int iy = 0; iy < ny; ++iy)
    for (int ix = 0; ix < nx; ++ix) {
      const double u = freq(ix, nx), v = freq(iy, ny);
      double zlo = -HUGE_VAL, zhi = HUGE_VAL;
      bool ok = true;
      for (const auto& pl : planes) {
        const double rhs = pl[3] + tol - pl[0] * u - pl[1] * v;
        if (pl[2] > 1e-12) zhi = std::min(zhi, rhs / pl[2]);
        else if (pl[2] < -1e-12) zlo = std::max(zlo, rhs / pl[2]);
        else if (rhs < 0) ok = false;
      }
      for (int iz = 0; iz < nz; ++iz) {
        const double w = freq(iz, nz);
        const bool in = ok && w >= zlo && w <= zhi;
        mask[ix + (int64_t)nx * (iy + (int64_t)ny * iz)] = in ? 1 : 0;
        count += in;
      }
    }
  return count;
}

extern "C" int nfs_kspace_filter_mask(const double* kpos, int64_t K, int dim, int nx, int ny, int nz,
                                      unsigned char* mask, int64_t* n_inside) {
  const char* fn = "nfs_kspace_filter_mask";
  if (!(dim == 3 || (dim == 2 && nz == 1)))
    return fail(NFS_EUNSUPPORTED, "%s: dim must be 3, or 2 with nz 1", fn);
  int rc = check_filter_dims(nx, ny, nz, fn);
  if (rc) return rc;
  if (K < 0 || (K > 0 && !kpos) || !mask) return fail(NFS_EINVAL, "%s: NULL or negative argument", fn);
  if (dim == 3) {
    double scale = 0.0;
    for (int64_t k = 0; k < 3 * K; ++k) {
      if (!std::isfinite(kpos[k])) return fail(NFS_EINVAL, "%s: non-finite position %lld", fn, (long long)(k / 3));
      scale = std::max(scale, std::fabs(kpos[k]));
    }
    std::vector<std::array<double, 4>> planes;
    if (!convex_hull_3d(kpos, K, scale, &planes))
      return fail(NFS_EINVAL, "%s: the %lld positions span no volume (fewer than 4 or all on a plane)", fn,
                  (long long)K);
    const int64_t cnt = mask_from_planes(planes, nx, ny, nz, 1e-9 * (scale > 1.0 ? scale : 1.0), mask);
    if (n_inside) *n_inside = cnt;
    return NFS_OK;
  }
  const int64_t L = (int64_t)nx * ny;
  std::vector<std::pair<double, double>> pts;
  pts.reserve((size_t)K);
  double scale = 0.0;
  for (int64_t k = 0; k < K; ++k) {
    const double x = kpos[2 * k], y = kpos[2 * k + 1];
    if (!std::isfinite(x) || !std::isfinite(y)) return fail(NFS_EINVAL, "%s: non-finite position %lld", fn, (long long)k);
    pts.emplace_back(x, y);
    scale = std::max(scale, std::max(std::fabs(x), std::fabs(y)));
  }
  std::sort(pts.begin(), pts.end());
  pts.erase(std::unique(pts.begin(), pts.end()), pts.end());
  auto cross = [](const std::pair<double, double>& o, const std::pair<double, double>& a,
                  const std::pair<double, double>& b) {
    return (a.first - o.first) * (b.second - o.second) - (a.second - o.second) * (b.first - o.first);
  };
  std::vector<std::pair<double, double>> hull;
  if (pts.size() >= 3) {
    std::vector<std::pair<double, double>> h(2 * pts.size());
    size_t k = 0;
    for (size_t i = 0; i < pts.size(); ++i) {
      while (k >= 2 && cross(h[k - 2], h[k - 1], pts[i]) <= 0) --k;
      h[k++] = pts[i];
    }
    for (size_t i = pts.size() - 1, t = k + 1; i-- > 0;) {
      while (k >= t && cross(h[k - 2], h[k - 1], pts[i]) <= 0) --k;
      h[k++] = pts[i];
    }
    h.resize(k - 1);  // counter-clockwise, first point not repeated
    hull = h;
  }
  const double eps = 1e-12 * (scale > 1.0 ? scale * scale : 1.0);
  int64_t count = 0;
  for (int64_t l = 0; l < L; ++l) {
    const int ix = (int)(l % nx), iy = (int)(l / nx);
    const std::pair<double, double> p((double)(ix < (nx + 1) / 2 ? ix : ix - nx),
                                      (double)(iy < (ny + 1) / 2 ? iy : iy - ny));
    bool in = hull.size() >= 3;
    for (size_t e = 0; in && e < hull.size(); ++e)
      if (cross(hull[e], hull[(e + 1) % hull.size()], p) < -eps) in = false;
    mask[l] = in ? 1 : 0;
    count += in;
  }
  if (n_inside) *n_inside = count;
  return NFS_OK;
}

// ---------------------------------------------------------------------------
// Batched solves: independent slices, forked from the caller's stream onto
// the context's streams (longest-processing-time assignment by L*K*G) and
// joined back.
constexpr int kBatchStreams = 8;

static int ensure_batch_streams(nfs_ctx* ctx) {
  if ((int)ctx->bstreams.size() == kBatchStreams) return NFS_OK;
  int cur = 0;
  NFS_TRY(hipGetDevice(&cur), "hipGetDevice");
  NFS_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  while ((int)ctx->bstreams.size() < kBatchStreams) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    NFS_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    NFS_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreateWithFlags");
    ctx->bstreams.push_back(st);
    ctx->bevents.push_back(ev);
  }
  if (!ctx->fork_event) NFS_TRY(hipEventCreateWithFlags(&ctx->fork_event, hipEventDisableTiming), "hipEventCreate");
  NFS_TRY(hipSetDevice(cur), "hipSetDevice");
  return NFS_OK;
}

// longest-processing-time assignment of slices (by L*K*G) to at most
// kBatchStreams lanes
static std::vector<std::vector<int>> assign_lanes(int n_slices, const nfs_problem* probs) {
  std::vector<int> order(n_slices);
  for (int i = 0; i < n_slices; ++i) order[i] = i;
  auto work = [&](int i) { return (double)probs[i].n_vox * probs[i].n_samp * probs[i].n_coil; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  const int ns = n_slices < kBatchStreams ? n_slices : kBatchStreams;
  std::vector<std::vector<int>> lanes(ns);
  std::vector<double> load(ns, 0.0);
  for (int i : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lanes[k].push_back(i);
    load[k] += work(i);
  }
  return lanes;
}

// Slices' layouts one after another, then kBatchCounters work-list counters
// of the persistent launches (the last offset in offs).
constexpr int kBatchCounters = 256;
// and the per-slice arguments of the lock-step form's batched vector and
// packing launches (CgSlice[n], then two PackSlice[n])
static size_t slice_args_bytes(int n) { return al(n * sizeof(CgSlice)) + 2 * al(n * sizeof(PackSlice)); }
static size_t batch_layouts(const nfs_ctx* ctx, int n, const nfs_problem* probs, int precision, int n_iter, int reorth,
                            std::vector<Layout>* ys, std::vector<size_t>* offs) {
  size_t tot = 0;
  for (int i = 0; i < n; ++i) {
    Layout y = make_layout(ctx, &probs[i], NFS_OP_CG, precision, n_iter, reorth);
    if (offs) offs->push_back(tot);
    tot += al(y.total);
    if (ys) ys->push_back(y);
  }
  if (offs) offs->push_back(tot);
  return n ? tot + al(kBatchCounters * sizeof(int)) + slice_args_bytes(n) : 0;
}

extern "C" int nfs_workspace_bytes_batched(const nfs_ctx* ctx, int n_slices, const nfs_problem* probs, int precision,
                                           int n_iter, int reorth, size_t* bytes) {
  const char* fn = "nfs_workspace_bytes_batched";
  if (!bytes) return fail(NFS_EINVAL, "%s: bytes is NULL", fn);
  if (n_slices < 0 || (n_slices > 0 && !probs)) return fail(NFS_EINVAL, "%s: bad slice list", fn);
  int rc;
  if ((rc = check_prec(precision, fn))) return rc;
  if (n_iter < 0) return fail(NFS_EINVAL, "%s: n_iter %d < 0", fn, n_iter);
  if (reorth && n_iter > kMaxReorth) return fail(NFS_EINVAL, "%s: reorth needs n_iter <= %d", fn, kMaxReorth);
  for (int i = 0; i < n_slices; ++i)
    if ((rc = check_sizes(&probs[i], fn))) return rc;
  *bytes = batch_layouts(ctx, n_slices, probs, precision, n_iter, reorth != 0, nullptr, nullptr);
  return NFS_OK;
}

// ---------------------------------------------------------------------------
// Lock-step batched CG: every slice runs the nfs_cg_solve sequence, but the
// E and E^H contractions of all slices go into one persistent encode launch
// each (launch_encode_persistent), and between them the operand packing and
// the CG vector steps of all slices are one batched launch per step (the
// setup and the residual replacements fork per-slice kernels over the
// library streams instead).
struct SliceRun {
  const nfs_problem* pr;
  const Layout* y;
  void* ws;
  CgState st;
  const float2* sens;
  float2* x;
  const float* m;
  double* hist;
  int* info;
};

static EncodeItem encode_item(const SliceRun& r, int op) {
  const Layout& y = *r.y;
  const EncodeShape& sh = op == OP_E ? y.shE : y.shH;
  EncodeItem e{};
  e.heldcoef = at<void>(r.ws, op == OP_E ? y.o_sB : y.o_vB);
  e.strmcoef = at<void>(r.ws, op == OP_E ? y.o_vA : y.o_sA);
  e.sdata = at<void>(r.ws, op == OP_E ? y.o_dataE : y.o_dataH);
  e.HC = sh.HC;
  e.SC = sh.SC;
  e.cps = sh.cps;
  e.out_part = at<float>(r.ws, op == OP_E ? y.o_epart : y.o_hpart);
  e.sens = r.sens;
  e.L = y.L;
  e.tmax = at<unsigned>(r.ws, y.o_tmax);
  e.stop = r.st.stop;
  e.G = y.G;
  e.T = y.P + 1;
  e.NB = sh.NB;
  e.gx = (int)cdiv(sh.HC, (int64_t)kWaves * sh.MT);
  return e;
}

// Whether the batch can run in lock-step with persistent launches: every
// slice's shapes are ones the persistent kernel is built for.
static bool lockstep_ok(int n, const std::vector<Layout>& ys) {
  if (n < 1) return false;
  for (int i = 0; i < n; ++i) {
    const Layout& y = ys[i];
    if (y.L == 0 || y.K == 0) return false;
    for (const EncodeShape* sh : {&y.shE, &y.shH})
      if (!persistent_supported(sh->prec, sh->NQ, sh->NB, sh->MT)) return false;
  }
  return true;
}

// The persistent encode launches of one direction (op OP_E or OP_EH) over
// all slices: one launch per shape class (phase instructions, column
// blocks, held tiles), at most kMaxBatchItems slices each.  The classes are
// independent, so their launches go onto the library streams and run side
// by side; each gets a grid of its resident workgroups (the encode kernel's
// registers allow four per CU up to two column blocks or with two held
// tiles, three for four column blocks with four held tiles).
static int persistent_encode(nfs_ctx* ctx, const std::vector<SliceRun>& runs, int op, int* counters,
                             hipStream_t s) {
  std::map<int, std::vector<int>> groups;  // (NQ * 8 + NB) * 8 + MT -> slices
  for (size_t i = 0; i < runs.size(); ++i) {
    const EncodeShape& sh = op == OP_E ? runs[i].y->shE : runs[i].y->shH;
    groups[(sh.NQ * 8 + sh.NB) * 8 + sh.MT].push_back((int)i);
  }
  // longest items first: slices by streamed chunks per item, descending
  for (auto& g : groups)
    std::stable_sort(g.second.begin(), g.second.end(), [&](int a, int b) {
      const EncodeShape& sa = op == OP_E ? runs[a].y->shE : runs[a].y->shH;
      const EncodeShape& sb = op == OP_E ? runs[b].y->shE : runs[b].y->shH;
      return sa.cps > sb.cps;
    });
  std::vector<EncodeBatch> batches;
  std::vector<int> keys;
  for (const auto& g : groups)
    for (size_t b0 = 0; b0 < g.second.size(); b0 += kMaxBatchItems) {
      EncodeBatch b{};
      int64_t first = 0;
      for (size_t j = b0; j < g.second.size() && j < b0 + kMaxBatchItems; ++j) {
        const SliceRun& r = runs[g.second[j]];
        const EncodeShape& sh = op == OP_E ? r.y->shE : r.y->shH;
        EncodeItem& e = b.it[b.n++];
        e = encode_item(r, op);
        e.first = first;
        first += (int64_t)e.gx * sh.nsplit;
      }
      b.total = first;
      batches.push_back(b);
      keys.push_back(g.first);
    }
  const int nb = (int)batches.size();
  const bool fork = nb > 1;
  if (fork) NFS_TRY(hipEventRecord(ctx->fork_event, s), "hipEventRecord");
  for (int k = 0; k < nb; ++k) {
    const int key = keys[k];
    const int MT = key % 8, NB = (key / 8) % 8, NQ = key / 64;
    hipStream_t sk = fork ? ctx->bstreams[k % kBatchStreams] : s;
    if (fork) NFS_TRY(hipStreamWaitEvent(sk, ctx->fork_event, 0), "hipStreamWaitEvent");
    const int per_cu = NB <= 2 || MT == 2 ? 4 : 3;
    if (k >= kBatchCounters / 2) return fail(NFS_EINVAL, "encode_persistent: too many shape classes");
    batches[k].counter = counters + (op == OP_E ? 0 : kBatchCounters / 2) + k;
    NFS_TRY(launch_fill_zero(reinterpret_cast<float*>(batches[k].counter), 1, sk), "fill_zero(counter)");
    NFS_TRY(launch_encode_persistent(op, runs[0].y->prec, NQ, NB, MT, batches[k], per_cu * ctx->n_cu, sk),
            "encode_persistent");
  }
  if (fork)
    for (int k = 0; k < nb && k < kBatchStreams; ++k) {  // after every launch on that stream
      NFS_TRY(hipEventRecord(ctx->bevents[k], ctx->bstreams[k]), "hipEventRecord");
      NFS_TRY(hipStreamWaitEvent(s, ctx->bevents[k], 0), "hipStreamWaitEvent");
    }
  return NFS_OK;
}

// Run f(run, stream) for every slice, slices forked over the library
// streams (lanes) and joined back into s.
template <class F>
static int fork_join(nfs_ctx* ctx, const std::vector<std::vector<int>>& lanes, std::vector<SliceRun>& runs,
                     hipStream_t s, F&& f) {
  NFS_TRY(hipEventRecord(ctx->fork_event, s), "hipEventRecord");
  for (size_t k = 0; k < lanes.size(); ++k) {
    hipStream_t sk = ctx->bstreams[k];
    NFS_TRY(hipStreamWaitEvent(sk, ctx->fork_event, 0), "hipStreamWaitEvent");
    for (int i : lanes[k]) {
      const int rc = f(runs[i], sk);
      if (rc) return rc;
    }
    NFS_TRY(hipEventRecord(ctx->bevents[k], sk), "hipEventRecord");
    NFS_TRY(hipStreamWaitEvent(s, ctx->bevents[k], 0), "hipStreamWaitEvent");
  }
  return NFS_OK;
}

static int run_cg_lockstep(nfs_ctx* ctx, int n, const nfs_problem* probs, const std::vector<Layout>& ys,
                           const std::vector<size_t>& offs, const float* const* m, float* const* rho, int n_iter,
                           double tol, int replace_every, int reorth, double* const* hist, int* const* info, void* ws,
                           const std::vector<std::vector<int>>& lanes, hipStream_t s) {
  int* counters = at<int>(ws, offs[n]);
  std::vector<SliceRun> runs(n);
  for (int i = 0; i < n; ++i) {
    SliceRun& r = runs[i];
    const Layout& y = ys[i];
    r.pr = &probs[i];
    r.y = &ys[i];
    r.ws = static_cast<char*>(ws) + offs[i];
    r.x = reinterpret_cast<float2*>(rho[i]);
    r.m = m[i];
    r.hist = hist ? hist[i] : nullptr;
    r.info = info ? info[i] : nullptr;
    CgState& st = r.st;
    st.r = at<float2>(r.ws, y.o_r);
    st.p = at<float2>(r.ws, y.o_p);
    st.q = at<float2>(r.ws, y.o_q);
    st.b = at<float2>(r.ws, y.o_b);
    st.part = at<double>(r.ws, y.o_part);
    st.alpha = at<double>(r.ws, y.o_alpha);
    st.scal = at<double>(r.ws, y.o_scal);
    st.hist = r.hist ? r.hist : at<double>(r.ws, y.o_hist);
    st.info = r.info ? r.info : at<int>(r.ws, y.o_info);
    st.stop = at<int>(r.ws, y.o_stop);
    st.V = reorth ? at<float2>(r.ws, y.o_V) : nullptr;
    st.rn = reorth ? at<float2>(r.ws, y.o_rn) : nullptr;
    st.iters = nullptr;
    st.icorr = probs[i].icorr;
    st.rpart = reorth ? at<double>(r.ws, y.o_rpart) : nullptr;
    const bool f16ops = scaled_prec(y.prec);
    st.smax = f16ops ? at<float>(r.ws, y.o_smax) : nullptr;
    st.bmax = f16ops ? at<float>(r.ws, y.o_bmax) : nullptr;
    st.L = y.L;
    const int64_t nb = cdiv(y.L, 256);
    st.nblk = (int)(nb < 1 ? 1 : (nb > kCgBlocks ? kCgBlocks : nb));
    r.sens = probs[i].icorr ? at<float2>(r.ws, y.o_sensj) : reinterpret_cast<const float2*>(probs[i].sens);
  }
  auto ctx_of = [&](SliceRun& r, hipStream_t sk) {
    return Ctx{ctx, *r.y, r.pr, r.sens, r.ws, sk, r.st.stop};
  };
  auto hs = [](const SliceRun& r) { return r.y->LC * 16; };
  // the batched launches' per-slice arguments (the single-slice launches'
  // arguments of pre_E for the direction, mid_EHE, cg_beta ... cg_direction)
  char* argbase = static_cast<char*>(ws) + offs[n] + al(kBatchCounters * sizeof(int));
  CgSlice* d_cg = reinterpret_cast<CgSlice*>(argbase);
  PackSlice* d_pe = reinterpret_cast<PackSlice*>(argbase + al(n * sizeof(CgSlice)));
  PackSlice* d_ph = reinterpret_cast<PackSlice*>(argbase + al(n * sizeof(CgSlice)) + al(n * sizeof(PackSlice)));
  std::vector<CgSlice> h_cg(n);
  std::vector<PackSlice> h_pe(n), h_ph(n);
  int max_nblk = 1;
  int64_t max_pe = 0, max_ph = 0;
  for (int i = 0; i < n; ++i) {
    const SliceRun& r = runs[i];
    const Layout& y = *r.y;
    float* us = scaled_prec(y.prec) ? at<float>(r.ws, y.o_unscale) : nullptr;
    CgSlice& cg = h_cg[i];
    cg = CgSlice{};
    cg.st = r.st;
    cg.hpart = at<float2>(r.ws, y.o_hpart);
    cg.unscale = us ? us + 1 : nullptr;
    cg.rho = r.x;
    cg.stride = hs(r);
    cg.nsplit = y.shH.nsplit;
    max_nblk = std::max(max_nblk, r.st.nblk);
    PackSlice& pe = h_pe[i];  // pre_E of the direction (bound already formed by the CG step)
    pe = PackSlice{};
    pe.src = r.st.p;
    pe.mul = r.sens;
    pe.out = at<void>(r.ws, y.o_dataE);
    pe.bmax = at<float>(r.ws, y.o_bmax);
    pe.unscale = at<float>(r.ws, y.o_unscale);
    pe.stop = r.st.stop;
    pe.n_items = y.L;
    pe.is = 1;
    pe.cs = 0;
    pe.nchunks = y.LC;
    pe.G = y.G;
    pe.NB = y.NB;
    max_pe = std::max(max_pe, cdiv(y.LC * y.NB * 64, 256));
    PackSlice& ph = h_ph[i];  // mid_EHE
    ph = PackSlice{};
    ph.src = at<float>(r.ws, y.o_epart);
    ph.out = at<void>(r.ws, y.o_dataH);
    ph.unscale_in = at<float>(r.ws, y.o_unscale);
    ph.unscale = at<float>(r.ws, y.o_unscale) + 1;
    ph.stop = r.st.stop;
    ph.n_items = y.K;
    ph.nchunks = y.KC;
    ph.HC16 = y.KC * 16;
    ph.scale = epart_pack_scale(y.prec, y.L);
    ph.wmul = 1.f;
    ph.G = y.G;
    ph.NB = y.NB;
    ph.nsplit = y.shE.nsplit;
    max_ph = std::max(max_ph, cdiv(y.KC * y.NB * 64, 256));
  }
  int rc;
  // setup and the E^H packing of the data
  rc = fork_join(ctx, lanes, runs, s, [&](SliceRun& r, hipStream_t sk) -> int {
    const Layout& y = *r.y;
    const int i = (int)(&r - runs.data());
    NFS_TRY(launch_store_slice_args(h_cg[i], h_pe[i], h_ph[i], d_cg + i, d_pe + i, d_ph + i, sk), "store_slice_args");
    if (r.pr->icorr)
      NFS_TRY(launch_scale_sens(reinterpret_cast<const float2*>(r.pr->sens), r.pr->icorr, y.G, y.L,
                                const_cast<float2*>(r.sens), sk),
              "scale_sens");
    if (scaled_prec(y.prec)) NFS_TRY(launch_sens_absmax(r.sens, y.G, y.L, at<float>(r.ws, y.o_smax), sk), "sens_absmax");
    NFS_TRY(launch_cg_reset(r.st, sk), "cg_reset");
    Ctx c = ctx_of(r, sk);
    int e = seq_pack_coefs(c, true, true);
    if (e) return e;
    NFS_TRY(launch_cg_norm_m(r.st, reinterpret_cast<const float2*>(r.m), (int64_t)y.G * y.K, sk), "cg_norm_m");
    return pre_EH(c, reinterpret_cast<const float2*>(r.m), 1, y.K);
  });
  if (rc) return rc;
  if ((rc = persistent_encode(ctx, runs, OP_EH, counters, s))) return rc;
  // Per iteration two fork-joins: the E^H packing between the persistent E
  // and E^H launches, and the CG vector updates together with the packing
  // of the next iteration's E operand (a residual replacement adds one
  // more E^H E of the iterate).
  auto pre_E_dir = [&](SliceRun& r, hipStream_t sk) -> int {
    return pre_E(ctx_of(r, sk), r.st.p, scaled_prec(r.y->prec));
  };
  rc = fork_join(ctx, lanes, runs, s, [&](SliceRun& r, hipStream_t sk) -> int {
    Ctx c = ctx_of(r, sk);
    NFS_TRY(launch_cg_init(r.st, at<float2>(r.ws, r.y->o_hpart), r.y->shH.nsplit, hs(r), unscale_slot(c, 1), r.x,
                           r.y->L, sk),
            "cg_init");
    NFS_TRY(launch_cg_start(r.st, n_iter, sk), "cg_start");
    if (reorth) NFS_TRY(launch_cg_store_v(r.st, 0, sk), "cg_store_v");
    return n_iter > 0 ? pre_E_dir(r, sk) : NFS_OK;
  });
  if (rc) return rc;
  // E (operand already packed), E^H packing, E^H
  const int prec = ys[0].prec;
  auto ehe_rest = [&]() -> int {
    int e = persistent_encode(ctx, runs, OP_E, counters, s);
    if (e) return e;
    NFS_TRY(launch_pack_EH_from_epart_batched(prec, d_ph, n, max_ph, s), "pack_EH_from_epart(batched)");
    return persistent_encode(ctx, runs, OP_EH, counters, s);
  };
  for (int it = 0; it < n_iter; ++it) {
    if ((rc = ehe_rest())) return rc;
    const bool replace = replace_every > 0 && (it + 1) % replace_every == 0 && it + 1 < n_iter;
    const bool more = it + 1 < n_iter;
    const int nv = reorth ? it + 1 : 0;
    auto beta_update = [&](SliceRun& r, hipStream_t sk) -> int {
      Ctx c = ctx_of(r, sk);
      NFS_TRY(launch_cg_beta(r.st, at<float2>(r.ws, r.y->o_hpart), r.y->shH.nsplit, hs(r), unscale_slot(c, 1),
                             r.y->L, sk),
              "cg_beta");
      NFS_TRY(launch_cg_update(r.st, r.x, r.y->L, it, replace ? 0 : nv, sk), "cg_update");
      return NFS_OK;
    };
    auto finish_iteration = [&](SliceRun& r, hipStream_t sk) -> int {
      if (reorth) NFS_TRY(launch_cg_reorth_apply(r.st, nv, !replace, sk), "cg_reorth_apply");
      NFS_TRY(launch_cg_direction(r.st, r.y->L, it, n_iter, tol, sk), "cg_direction");
      return more ? pre_E_dir(r, sk) : NFS_OK;
    };
    if (!replace) {
      NFS_TRY(launch_cg_beta_batched(d_cg, n, max_nblk, s), "cg_beta(batched)");
      NFS_TRY(launch_cg_update_batched(d_cg, n, max_nblk, it, nv, s), "cg_update(batched)");
      if (reorth) NFS_TRY(launch_cg_reorth_apply_batched(d_cg, n, max_nblk, nv, true, s), "cg_reorth_apply(batched)");
      NFS_TRY(launch_cg_direction_batched(d_cg, n, max_nblk, it, n_iter, tol, s), "cg_direction(batched)");
      if (more) NFS_TRY(launch_pack_data_E_batched(prec, d_pe, n, max_pe, s), "pack_data(E, batched)");
      continue;
    }
    rc = fork_join(ctx, lanes, runs, s, [&](SliceRun& r, hipStream_t sk) -> int {
      const int e = beta_update(r, sk);
      return e ? e : pre_E(ctx_of(r, sk), r.x, false);
    });
    if (rc) return rc;
    if ((rc = ehe_rest())) return rc;
    rc = fork_join(ctx, lanes, runs, s, [&](SliceRun& r, hipStream_t sk) -> int {
      Ctx c = ctx_of(r, sk);
      NFS_TRY(launch_cg_replace(r.st, at<float2>(r.ws, r.y->o_hpart), r.y->shH.nsplit, hs(r), unscale_slot(c, 1),
                                r.y->L, nv, sk),
              "cg_replace");
      return finish_iteration(r, sk);
    });
    if (rc) return rc;
  }
  return fork_join(ctx, lanes, runs, s, [&](SliceRun& r, hipStream_t sk) -> int {
    NFS_TRY(launch_cg_finish(r.st, r.x, r.pr->icorr, r.y->L, sk), "cg_finish");
    return NFS_OK;
  });
}

extern "C" int nfs_set_batch_mode(nfs_ctx* ctx, int mode) {
  if (!ctx) return fail(NFS_EINVAL, "nfs_set_batch_mode: ctx is NULL");
  if (mode != NFS_BATCH_STREAMS && mode != NFS_BATCH_PERSISTENT)
    return fail(NFS_EINVAL, "nfs_set_batch_mode: unknown mode %d", mode);
  ctx->batch_mode = mode;
  return NFS_OK;
}

extern "C" int nfs_cg_solve_batched(nfs_ctx* ctx, int n_slices, const nfs_problem* probs, const float* const* m,
                                    float* const* rho, int n_iter, double tol, int replace_every, int reorth,
                                    int precision, double* const* hist, int* const* info, void* ws, size_t ws_bytes,
                                    void* stream) {
  const char* fn = "nfs_cg_solve_batched";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  if (n_slices < 0 || (n_slices > 0 && (!probs || !m || !rho))) return fail(NFS_EINVAL, "%s: bad slice list", fn);
  int rc;
  for (int i = 0; i < n_slices; ++i) {
    rc = check_cg_args(ctx, &probs[i], m[i], rho[i], n_iter, tol, replace_every, reorth, precision,
                       hist ? hist[i] : nullptr, info ? info[i] : nullptr, fn);
    if (rc) return rc;
  }
  std::vector<Layout> ys;
  std::vector<size_t> offs;
  if (n_slices == 0) return NFS_OK;
  const size_t need = batch_layouts(ctx, n_slices, probs, precision, n_iter, reorth, &ys, &offs);
  if (!ws) return fail(NFS_EWORKSPACE, "%s: workspace is NULL", fn);
  if ((uintptr_t)ws % 256) return fail(NFS_EWORKSPACE, "%s: workspace not 256-byte aligned", fn);
  if (ws_bytes < need) return fail(NFS_EWORKSPACE, "%s: workspace has %zu bytes, needs %zu", fn, ws_bytes, need);
  if ((rc = ensure_batch_streams(ctx))) return rc;
  const std::vector<std::vector<int>> lanes = assign_lanes(n_slices, probs);
  const int ns = (int)lanes.size();
  std::vector<const void*> ptrs;
  for (int i = 0; i < n_slices; ++i) {
    ptrs.push_back(m[i]);
    ptrs.push_back(rho[i]);
    ptrs.push_back(hist ? hist[i] : nullptr);
    ptrs.push_back(info ? info[i] : nullptr);
  }
  const bool lockstep = ctx->batch_mode == NFS_BATCH_PERSISTENT && lockstep_ok(n_slices, ys);
  const std::string key = graph_key(ctx, lockstep ? "cgbp" : "cgb", probs, n_slices, ptrs.data(), (int)ptrs.size(),
                                    n_iter, tol, replace_every, reorth, precision, ws, ws_bytes, stream);
  if (lockstep)
    return run_maybe_graph(ctx, key, (hipStream_t)stream, [&](hipStream_t s) -> int {
      return run_cg_lockstep(ctx, n_slices, probs, ys, offs, m, rho, n_iter, tol, replace_every, reorth, hist, info,
                             ws, lanes, s);
    });
  return run_maybe_graph(ctx, key, (hipStream_t)stream, [&](hipStream_t s) -> int {
    NFS_TRY(hipEventRecord(ctx->fork_event, s), "hipEventRecord");
    for (int k = 0; k < ns; ++k) {
      hipStream_t sk = ctx->bstreams[k];
      NFS_TRY(hipStreamWaitEvent(sk, ctx->fork_event, 0), "hipStreamWaitEvent");
      for (int i : lanes[k]) {
        const int r2 = run_cg(ctx, &probs[i], ys[i], m[i], rho[i], n_iter, tol, replace_every, reorth,
                              hist ? hist[i] : nullptr, info ? info[i] : nullptr,
                              static_cast<char*>(ws) + offs[i], sk);
        if (r2) return r2;
      }
      NFS_TRY(hipEventRecord(ctx->bevents[k], sk), "hipEventRecord");
      NFS_TRY(hipStreamWaitEvent(s, ctx->bevents[k], 0), "hipStreamWaitEvent");
    }
    return NFS_OK;
  });
}

extern "C" int nfs_encode_backward(nfs_ctx* ctx, const nfs_problem* prob, const float* rho, const float* grad_m,
                                   float* grad_rho, float* grad_b0, float* grad_kcoef, int precision, void* ws,
                                   size_t ws_bytes, void* stream) {
  const char* fn = "nfs_encode_backward";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  int rc = check_problem(prob, fn);
  if (rc) return rc;
  if ((rc = check_prec(precision, fn))) return rc;
  if ((rc = check_vec(grad_m, prob->n_samp, fn, "grad_m"))) return rc;
  if ((grad_b0 || grad_kcoef) && (rc = check_vec(rho, prob->n_vox, fn, "rho"))) return rc;
  if ((rc = check_vec(grad_rho, 0, fn, "grad_rho"))) return rc;
  if (misaligned(grad_b0, 4) || misaligned(grad_kcoef, 4))
    return fail(NFS_EINVAL, "%s: gradient array not 4-byte aligned", fn);
  const Layout y = make_layout(ctx, prob, NFS_OP_EHE, precision, 0, 0);
  if ((rc = check_ws(y, ws, ws_bytes, fn))) return rc;
  Ctx c{ctx, y, prob, reinterpret_cast<const float2*>(prob->sens), ws, (hipStream_t)stream, nullptr};
  const float2* G = reinterpret_cast<const float2*>(grad_m);
  const float2* r = reinterpret_cast<const float2*>(rho);
  if ((rc = seq_pack_coefs(c, grad_kcoef != nullptr && y.P > 0, grad_rho != nullptr || grad_b0 != nullptr))) return rc;
  if (grad_rho && y.L > 0) {
    if ((rc = seq_EH(c, G, 1, y.K))) return rc;
    NFS_TRY(launch_finish_EH(at<float2>(ws, y.o_hpart), y.shH.nsplit, y.LC * 16, y.L, unscale_slot(c, 1),
                             reinterpret_cast<float2*>(grad_rho), c.s),
            "finish_EH");
  }
  if (grad_b0 && y.L > 0) {
    if ((rc = seq_EH(c, G, 1, y.K, prob->t))) return rc;
    NFS_TRY(launch_grad_b0(at<float2>(ws, y.o_hpart), y.shH.nsplit, y.LC * 16, y.L, unscale_slot(c, 1), r, grad_b0,
                           c.s),
            "grad_b0");
  }
  if (grad_kcoef && y.K > 0 && y.P > 0) {
    for (int b = 0; b < y.P; ++b) {
      if ((rc = seq_E(c, r, prob->fields + (int64_t)b * y.L))) return rc;
      NFS_TRY(launch_grad_kcoef(at<float>(ws, y.o_epart), y.shE.nsplit, y.KC * 16, y.NB, unscale_slot(c, 0), G, y.K,
                                y.G, y.P, b, grad_kcoef, c.s),
              "grad_kcoef");
    }
  }
  return NFS_OK;
}

// ---------------------------------------------------------------------------
// Autotuning of the encode shapes: held tiles per wave (MT) and the split
// count of the streamed range, per direction, measured on the problem's own
// phase coefficients with realistic operands (E of rho = 1 + i, then E^H of
// that E output).  The objective of a shape includes the kernel that
// consumes its split partials (the E^H operand pack after E, the E^H finish
// after E^H), since more splits mean more partials to sum.  The fastest
// shape is kept in the context under the shape class (direction, precision,
// L, K, G, P) and used by every later call.
struct TuneCand {
  int MT, ns;
};

static std::vector<TuneCand> tune_candidates(const nfs_ctx* ctx, int NB, int64_t HC, int64_t SC) {
  std::vector<TuneCand> v;
  const int64_t maxs = std::max<int64_t>(1, std::min<int64_t>(64, SC / 8));
  for (int MT : {2, 4}) {
    if (!valid_held_tiles(NB, MT)) continue;
    const int64_t gx = std::max<int64_t>(1, cdiv(HC, (int64_t)kWaves * MT));
    std::vector<int> seen;
    // target workgroups per CU; the large targets give problems with many
    // held blocks (the 3D workload's 1728-2235 per split) split counts of
    // 3-8, where the last partial round of resident workgroups is small
    for (int per_cu : {1, 2, 3, 4, 5, 6, 8, 12, 16, 24, 32, 48}) {
      const int ns = (int)std::min(std::max<int64_t>(cdiv((int64_t)per_cu * ctx->n_cu, gx), 1), maxs);
      if (std::find(seen.begin(), seen.end(), ns) == seen.end()) {
        seen.push_back(ns);
        v.push_back({MT, ns});
      }
    }
  }
  return v;
}

// split count for a target of quarter_wg_per_cu / 4 workgroups per CU (batches)
static int split_for_target(const nfs_ctx* ctx, int MT, int64_t HC, int64_t SC, int quarter_wg_per_cu) {
  const int64_t maxs = std::max<int64_t>(1, std::min<int64_t>(64, SC / 8));
  const int64_t gx = std::max<int64_t>(1, cdiv(HC, (int64_t)kWaves * MT));
  return (int)std::min(std::max<int64_t>(cdiv((int64_t)quarter_wg_per_cu * ctx->n_cu, 4 * gx), 1), maxs);
}

struct TuneLayout {
  Layout y;  // E^H E layout with the default shapes (phase parts, operands)
  std::vector<TuneCand> cE, cH;
  size_t o_epart, o_hpart, o_ones, total;
};

static TuneLayout tune_layout(const nfs_ctx* ctx, const nfs_problem* prob, int prec) {
  TuneLayout t;
  t.y = make_layout(ctx, prob, NFS_OP_EHE, prec, 0, 0);
  const Layout& y = t.y;
  t.cE = tune_candidates(ctx, y.NB, y.KC, y.LC);
  t.cH = tune_candidates(ctx, y.NB, y.LC, y.KC);
  size_t maxE = 0, maxH = 0;
  for (const TuneCand& c : t.cE) {
    const int ov[2] = {c.MT, c.ns};
    maxE = std::max(maxE, epart_bytes(encode_shape(ctx, prob, OP_E, prec, y.NQ, y.NB, y.KC, y.LC, ov), y.NB));
  }
  for (const TuneCand& c : t.cH) {
    const int ov[2] = {c.MT, c.ns};
    maxH = std::max(maxH, hpart_bytes(encode_shape(ctx, prob, OP_EH, prec, y.NQ, y.NB, y.LC, y.KC, ov)));
  }
  t.o_epart = y.o_epart;  // the split partials come last in the layout
  t.o_hpart = al(t.o_epart + maxE);
  t.o_ones = al(t.o_hpart + maxH);
  t.total = al(t.o_ones + (size_t)y.L * 8);
  return t;
}

// One problem under tuning: its layout, workspace and launch context.
struct TuneSlice {
  const nfs_problem* pr;
  TuneLayout tl;
  void* ws;
};

// phase coefficients and the E operand of rho = 1 + i
static int tune_prepare(nfs_ctx* ctx, const TuneSlice& t, hipStream_t s) {
  const Layout& y = t.tl.y;
  Ctx c{ctx, y, t.pr, reinterpret_cast<const float2*>(t.pr->sens), t.ws, s, nullptr};
  int rc = seq_pack_coefs(c, true, true);
  if (rc) return rc;
  float2* ones = at<float2>(t.ws, t.tl.o_ones);
  NFS_TRY(launch_fill(reinterpret_cast<float*>(ones), 2 * y.L, 1.f, s), "fill");
  float* bmax = at<float>(t.ws, y.o_bmax);
  if (scaled_prec(y.prec))
    NFS_TRY(launch_absmax(ones, c.sens, nullptr, y.L, 1, 0, y.G, bmax, nullptr, s), "absmax");
  NFS_TRY(launch_pack_data(OP_E, y.prec, ones, c.sens, nullptr, y.L, 1, 0, y.G, y.NB, y.LC, at<void>(t.ws, y.o_dataE),
                           bmax, at<float>(t.ws, y.o_unscale), nullptr, s),
          "pack_data(E)");
  return NFS_OK;
}

// E with shape ovE then the E^H operand pack (ovE non-null), and/or E^H with
// shape ovH then the E^H finish (ovH non-null)
static int tune_pass(const nfs_ctx* ctx, const TuneSlice& t, const int* ovE, const int* ovH, hipStream_t s) {
  const Layout& y = t.tl.y;
  void* ws = t.ws;
  const float2* sens = reinterpret_cast<const float2*>(t.pr->sens);
  const unsigned* tmax = at<unsigned>(ws, y.o_tmax);
  float* us = at<float>(ws, y.o_unscale);
  if (ovE) {
    const EncodeShape sh = encode_shape(ctx, t.pr, OP_E, y.prec, y.NQ, y.NB, y.KC, y.LC, ovE);
    float* epart = at<float>(ws, t.tl.o_epart);
    NFS_TRY(launch_encode(sh, at<void>(ws, y.o_sB), at<void>(ws, y.o_vA), at<void>(ws, y.o_dataE), epart, sens, y.L,
                          y.G, tmax, y.P + 1, nullptr, s),
            "encode E (tuning)");
    NFS_TRY(launch_pack_EH_from_epart(y.prec, epart, sh.nsplit, y.KC * 16, y.NB, y.K, y.G, y.L, nullptr, 1.f, us,
                                      us + 1, y.KC, at<void>(ws, y.o_dataH), nullptr, s),
            "pack_EH_from_epart (tuning)");
  }
  if (ovH) {
    const EncodeShape sh = encode_shape(ctx, t.pr, OP_EH, y.prec, y.NQ, y.NB, y.LC, y.KC, ovH);
    float2* hpart = at<float2>(ws, t.tl.o_hpart);
    NFS_TRY(launch_encode(sh, at<void>(ws, y.o_vB), at<void>(ws, y.o_sA), at<void>(ws, y.o_dataH), (float*)hpart,
                          sens, y.L, y.G, tmax, y.P + 1, nullptr, s),
            "encode EH (tuning)");
    // the E operand has been packed already, so the ones vector is free
    NFS_TRY(launch_finish_EH(hpart, sh.nsplit, y.LC * 16, y.L, scaled_prec(y.prec) ? us + 1 : nullptr,
                             at<float2>(ws, t.tl.o_ones), s),
            "finish_EH (tuning)");
  }
  return NFS_OK;
}

// Mean duration of `enqueue` on stream s: one untimed run, then 1 timed run,
// or 3 when that one took under 5 ms.
struct TuneTimer {
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~TuneTimer() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  int init() {
    for (hipEvent_t& e : ev) NFS_TRY(hipEventCreate(&e), "hipEventCreate");
    return NFS_OK;
  }
  template <class F>
  int time(hipStream_t s, F&& enqueue, float* ms) {
    int rc = enqueue();
    if (rc) return rc;
    NFS_TRY(hipEventRecord(ev[0], s), "hipEventRecord");
    if ((rc = enqueue())) return rc;
    NFS_TRY(hipEventRecord(ev[1], s), "hipEventRecord");
    NFS_TRY(hipEventSynchronize(ev[1]), "hipEventSynchronize");
    float first = 0.f;
    NFS_TRY(hipEventElapsedTime(&first, ev[0], ev[1]), "hipEventElapsedTime");
    if (first > 5.f) {
      *ms = first;
      return NFS_OK;
    }
    NFS_TRY(hipEventRecord(ev[0], s), "hipEventRecord");
    for (int r = 0; r < 3; ++r)
      if ((rc = enqueue())) return rc;
    NFS_TRY(hipEventRecord(ev[1], s), "hipEventRecord");
    NFS_TRY(hipEventSynchronize(ev[1]), "hipEventSynchronize");
    float tot = 0.f;
    NFS_TRY(hipEventElapsedTime(&tot, ev[0], ev[1]), "hipEventElapsedTime");
    *ms = tot / 3;
    return NFS_OK;
  }
};

static int check_tune_stream(hipStream_t s, const char* fn) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (s) NFS_TRY(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone) return fail(NFS_EINVAL, "%s: the stream is being captured", fn);
  return NFS_OK;
}

extern "C" int nfs_tune_workspace_bytes(const nfs_ctx* ctx, const nfs_problem* prob, int precision, size_t* bytes) {
  const char* fn = "nfs_tune_workspace_bytes";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  if (!bytes) return fail(NFS_EINVAL, "%s: bytes is NULL", fn);
  int rc = check_sizes(prob, fn);
  if (rc) return rc;
  if ((rc = check_prec(precision, fn))) return rc;
  *bytes = tune_layout(ctx, prob, precision).total;
  return NFS_OK;
}

extern "C" int nfs_autotune(nfs_ctx* ctx, const nfs_problem* prob, int precision, void* ws, size_t ws_bytes,
                            void* stream) {
  const char* fn = "nfs_autotune";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  int rc = check_problem(prob, fn);
  if (rc) return rc;
  if ((rc = check_prec(precision, fn))) return rc;
  TuneSlice t{prob, tune_layout(ctx, prob, precision), ws};
  if (!ws) return fail(NFS_EWORKSPACE, "%s: workspace is NULL", fn);
  if ((uintptr_t)ws % 256) return fail(NFS_EWORKSPACE, "%s: workspace not 256-byte aligned", fn);
  if (ws_bytes < t.tl.total)
    return fail(NFS_EWORKSPACE, "%s: workspace has %zu bytes, needs %zu", fn, ws_bytes, t.tl.total);
  hipStream_t s = (hipStream_t)stream;
  if ((rc = check_tune_stream(s, fn))) return rc;
  if (t.tl.y.L == 0 || t.tl.y.K == 0) return NFS_OK;
  if ((rc = tune_prepare(ctx, t, s))) return rc;
  TuneTimer tm;
  if ((rc = tm.init())) return rc;
  TuneCand bE{}, bH{};
  float best = 0.f;
  for (size_t i = 0; i < t.tl.cE.size(); ++i) {
    const int ov[2] = {t.tl.cE[i].MT, t.tl.cE[i].ns};
    float ms = 0.f;
    if ((rc = tm.time(s, [&] { return tune_pass(ctx, t, ov, nullptr, s); }, &ms))) return rc;
    if (i == 0 || ms < best) {
      best = ms;
      bE = t.tl.cE[i];
    }
  }
  const int ovE[2] = {bE.MT, bE.ns};
  if ((rc = tune_pass(ctx, t, ovE, nullptr, s))) return rc;  // E^H operand of the chosen E shape
  for (size_t i = 0; i < t.tl.cH.size(); ++i) {
    const int ov[2] = {t.tl.cH[i].MT, t.tl.cH[i].ns};
    float ms = 0.f;
    if ((rc = tm.time(s, [&] { return tune_pass(ctx, t, nullptr, ov, s); }, &ms))) return rc;
    if (i == 0 || ms < best) {
      best = ms;
      bH = t.tl.cH[i];
    }
  }
  ctx->tune[tune_key(OP_E, precision, prob)] = {bE.MT, bE.ns};
  ctx->tune[tune_key(OP_EH, precision, prob)] = {bH.MT, bH.ns};
  ++ctx->tune_generation;
  return NFS_OK;
}

// Batched tuning: the slices of a batch run concurrently on the context's
// streams, so the shape that is fastest for a slice alone (one that fills
// the GPU by itself) is not the fastest inside the batch.  Candidates here
// are batch-wide: a held-tile count (2 or 4, where the slice allows it) and
// a target of 1/4, 1/2, 1, 2 or 4 workgroups per CU per slice, from which
// every slice derives its split counts; each candidate is timed as one
// concurrent E^H E pass over all slices (with the kernels that consume the
// split partials), forked and joined exactly as the batched solve does.
extern "C" int nfs_tune_workspace_bytes_batched(const nfs_ctx* ctx, int n_slices, const nfs_problem* probs,
                                                int precision, size_t* bytes) {
  const char* fn = "nfs_tune_workspace_bytes_batched";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  if (!bytes) return fail(NFS_EINVAL, "%s: bytes is NULL", fn);
  if (n_slices < 0 || (n_slices > 0 && !probs)) return fail(NFS_EINVAL, "%s: bad slice list", fn);
  int rc;
  if ((rc = check_prec(precision, fn))) return rc;
  size_t tot = 0;
  for (int i = 0; i < n_slices; ++i) {
    if ((rc = check_sizes(&probs[i], fn))) return rc;
    tot += al(tune_layout(ctx, &probs[i], precision).total);
  }
  *bytes = tot;
  return NFS_OK;
}

extern "C" int nfs_autotune_batched(nfs_ctx* ctx, int n_slices, const nfs_problem* probs, int precision, void* ws,
                                    size_t ws_bytes, void* stream) {
  const char* fn = "nfs_autotune_batched";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  if (n_slices < 0 || (n_slices > 0 && !probs)) return fail(NFS_EINVAL, "%s: bad slice list", fn);
  int rc;
  if ((rc = check_prec(precision, fn))) return rc;
  std::vector<TuneSlice> ts;
  size_t off = 0;
  for (int i = 0; i < n_slices; ++i) {
    if ((rc = check_problem(&probs[i], fn))) return rc;
    ts.push_back(TuneSlice{&probs[i], tune_layout(ctx, &probs[i], precision), nullptr});
    off += al(ts.back().tl.total);
  }
  if (!ws) return fail(NFS_EWORKSPACE, "%s: workspace is NULL", fn);
  if ((uintptr_t)ws % 256) return fail(NFS_EWORKSPACE, "%s: workspace not 256-byte aligned", fn);
  if (ws_bytes < off) return fail(NFS_EWORKSPACE, "%s: workspace has %zu bytes, needs %zu", fn, ws_bytes, off);
  hipStream_t s = (hipStream_t)stream;
  if ((rc = check_tune_stream(s, fn))) return rc;
  off = 0;
  std::vector<int> live;  // slices with work
  for (int i = 0; i < n_slices; ++i) {
    ts[i].ws = static_cast<char*>(ws) + off;
    off += al(ts[i].tl.total);
    if (ts[i].tl.y.L > 0 && ts[i].tl.y.K > 0) live.push_back(i);
  }
  if (live.empty()) return NFS_OK;
  if ((rc = ensure_batch_streams(ctx))) return rc;
  for (int i : live)
    if ((rc = tune_prepare(ctx, ts[i], s))) return rc;
  const std::vector<std::vector<int>> lanes = assign_lanes(n_slices, probs);
  // per-slice shapes of a batch candidate
  auto shapes = [&](int i, int MT, int q, int* ovE, int* ovH) {
    const Layout& y = ts[i].tl.y;
    const int mt = valid_held_tiles(y.NB, MT) ? MT : 2;
    ovE[0] = ovH[0] = mt;
    ovE[1] = split_for_target(ctx, mt, y.KC, y.LC, q);
    ovH[1] = split_for_target(ctx, mt, y.LC, y.KC, q);
  };
  TuneTimer tm;
  if ((rc = tm.init())) return rc;
  int bestMT = 2, bestQ = 4;
  float best = 0.f;
  bool first = true;
  for (int MT : {2, 4}) {
    for (int q : {1, 2, 4, 8, 16}) {
      auto enqueue = [&]() -> int {
        NFS_TRY(hipEventRecord(ctx->fork_event, s), "hipEventRecord");
        for (size_t k = 0; k < lanes.size(); ++k) {
          hipStream_t sk = ctx->bstreams[k];
          NFS_TRY(hipStreamWaitEvent(sk, ctx->fork_event, 0), "hipStreamWaitEvent");
          for (int i : lanes[k]) {
            if (ts[i].tl.y.L == 0 || ts[i].tl.y.K == 0) continue;
            int ovE[2], ovH[2];
            shapes(i, MT, q, ovE, ovH);
            const int r2 = tune_pass(ctx, ts[i], ovE, ovH, sk);
            if (r2) return r2;
          }
          NFS_TRY(hipEventRecord(ctx->bevents[k], sk), "hipEventRecord");
          NFS_TRY(hipStreamWaitEvent(s, ctx->bevents[k], 0), "hipStreamWaitEvent");
        }
        return NFS_OK;
      };
      float ms = 0.f;
      if ((rc = tm.time(s, enqueue, &ms))) return rc;
      if (first || ms < best) {
        best = ms;
        bestMT = MT;
        bestQ = q;
        first = false;
      }
    }
  }
  for (int i : live) {
    int ovE[2], ovH[2];
    shapes(i, bestMT, bestQ, ovE, ovH);
    ctx->tune[tune_key(OP_E, precision, &probs[i])] = {ovE[0], ovE[1]};
    ctx->tune[tune_key(OP_EH, precision, &probs[i])] = {ovH[0], ovH[1]};
  }
  ++ctx->tune_generation;
  return NFS_OK;
}

extern "C" int nfs_tuned_shape(const nfs_ctx* ctx, const nfs_problem* prob, int precision, int op, int* held_tiles_out,
                               int* nsplit_out) {
  const char* fn = "nfs_tuned_shape";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  if (!held_tiles_out || !nsplit_out) return fail(NFS_EINVAL, "%s: output pointer is NULL", fn);
  int rc = check_sizes(prob, fn);
  if (rc) return rc;
  if ((rc = check_prec(precision, fn))) return rc;
  if (op != NFS_OP_E && op != NFS_OP_EH) return fail(NFS_EINVAL, "%s: op must be NFS_OP_E or NFS_OP_EH", fn);
  const Layout y = make_layout(ctx, prob, NFS_OP_EHE, precision, 0, 0);
  const EncodeShape& sh = op == NFS_OP_E ? y.shE : y.shH;
  *held_tiles_out = sh.MT;
  *nsplit_out = sh.nsplit;
  return NFS_OK;
}

extern "C" int nfs_set_shape(nfs_ctx* ctx, const nfs_problem* prob, int precision, int op, int held_tiles,
                             int nsplit) {
  const char* fn = "nfs_set_shape";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  int rc = check_sizes(prob, fn);
  if (rc) return rc;
  if ((rc = check_prec(precision, fn))) return rc;
  if (op != NFS_OP_E && op != NFS_OP_EH) return fail(NFS_EINVAL, "%s: op must be NFS_OP_E or NFS_OP_EH", fn);
  const int nb = col_blocks(prob->n_coil);
  if (!valid_held_tiles(nb, held_tiles))
    return fail(NFS_EINVAL, "%s: %d held tiles not built for %d column blocks", fn, held_tiles, nb);
  if (nsplit < 1 || nsplit > 64) return fail(NFS_EINVAL, "%s: nsplit %d outside [1, 64]", fn, nsplit);
  ctx->tune[tune_key(op == NFS_OP_E ? OP_E : OP_EH, precision, prob)] = {held_tiles, nsplit};
  ++ctx->tune_generation;
  return NFS_OK;
}

// ---------------------------------------------------------------------------
// map estimation (sensitivity and B0 maps from multi-echo prescan data)

namespace {

constexpr int kMaxMapEchoes = 1024;

struct MapLayout {
  size_t shat = 0, b = 0, t = 0, w = 0, fit = 0, pcg = 0, mg = 0, total = 0;
};

MapLayout map_layout(int kind, int G, int nx, int ny, int nz, int precond) {
  const int64_t L = (int64_t)nx * ny * nz;
  const bool mg = precond == NFS_PRECOND_MG;
  const int nrhs = kind == NFS_MAP_SENS ? 3 * G : 1;
  MapLayout m;
  const int64_t Lp = (L + 63) & ~(int64_t)63;
  size_t off = 0;
  auto take = [&](size_t n) {
    const size_t o = off;
    off += al(n);
    return o;
  };
  if (kind == NFS_MAP_SENS) {
    m.shat = take((size_t)G * L * 16);
    m.b = take((size_t)3 * G * Lp * 8);
    m.t = take((size_t)Lp * 8);
    m.w = take((size_t)Lp * 8);
  } else {
    m.fit = take((size_t)3 * Lp * 8);  // B0^, beta, eps
    m.w = take((size_t)Lp * 8);
  }
  m.pcg = take(pcg_state_bytes(nrhs, nx, ny, nz, mg));
  if (mg) m.mg = take(mg_bytes(nrhs, nx, ny, nz));
  m.total = off;
  return m;
}

int check_map_grid(int nx, int ny, int nz, const char* fn, int64_t* L) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(NFS_ESHAPE, "%s: grid %d x %d x %d has an empty axis", fn, nx, ny, nz);
  const int64_t n = (int64_t)nx * ny * nz;
  if (n > ((int64_t)1 << 26)) return fail(NFS_ESHAPE, "%s: %lld voxels exceed 2^26", fn, (long long)n);
  *L = n;
  return NFS_OK;
}

int check_solver_args(double alpha, double tol, int max_iter, int precond, const char* fn) {
  if (precond != NFS_PRECOND_JACOBI && precond != NFS_PRECOND_MG)
    return fail(NFS_EINVAL, "%s: unknown preconditioner %d", fn, precond);
  if (!std::isfinite(alpha) || alpha < 0.0) return fail(NFS_EINVAL, "%s: alpha %g not finite and >= 0", fn, alpha);
  if (!std::isfinite(tol) || tol < 0.0) return fail(NFS_EINVAL, "%s: tol %g not finite and >= 0", fn, tol);
  if (max_iter < 0) return fail(NFS_EINVAL, "%s: max_iter %d < 0", fn, max_iter);
  return NFS_OK;
}

int check_map_ws(const MapLayout& m, void* ws, size_t ws_bytes, const char* fn) {
  if (!ws) return fail(NFS_EWORKSPACE, "%s: workspace is NULL", fn);
  if ((uintptr_t)ws % 256) return fail(NFS_EWORKSPACE, "%s: workspace not 256-byte aligned", fn);
  if (ws_bytes < m.total) return fail(NFS_EWORKSPACE, "%s: workspace has %zu bytes, needs %zu", fn, ws_bytes, m.total);
  return NFS_OK;
}

// Solve, then info (host, may be NULL) = (largest iteration count, status).
int run_pcg(int op, int precond, const PcgState& st, void* mg_ws, const double* b, int nx, int ny, int nz,
            const double* t, const double* w, double alpha, double tol, int max_iter, int* info, hipStream_t s,
            const char* fn) {
  std::vector<int> status(st.nrhs), iters(st.nrhs);
  NFS_TRY(pcg_solve(op, precond, st, mg_ws, b, nx, ny, nz, t, w, alpha, tol, max_iter, status.data(), iters.data(), s),
          fn);
  if (info) {
    int most = 0, worst = NFS_CG_EXACT;
    bool any_running = false, any_break = false, any_tol = false;
    for (int i = 0; i < st.nrhs; ++i) {
      most = std::max(most, iters[i]);
      any_running |= status[i] == 0;
      any_break |= status[i] == PCG_BREAKDOWN;
      any_tol |= status[i] == PCG_TOL;
    }
    if (any_break) worst = NFS_CG_BREAKDOWN;
    else if (any_running) worst = NFS_CG_MAXITER;
    else if (any_tol) worst = NFS_CG_TOL;
    info[0] = most;
    info[1] = worst;
  }
  return NFS_OK;
}

}  // namespace

extern "C" int nfs_maps_workspace_bytes(int kind, int n_coil, int nx, int ny, int nz, int precond, size_t* bytes) {
  const char* fn = "nfs_maps_workspace_bytes";
  if (!bytes) return fail(NFS_EINVAL, "%s: bytes is NULL", fn);
  if (kind != NFS_MAP_SENS && kind != NFS_MAP_B0) return fail(NFS_EINVAL, "%s: unknown kind %d", fn, kind);
  if (n_coil < 1 || n_coil > (kind == NFS_MAP_SENS ? kMaxSvdCoils : 64))
    return fail(NFS_ESHAPE, "%s: n_coil %d outside the supported range", fn, n_coil);
  int64_t L;
  int rc = check_map_grid(nx, ny, nz, fn, &L);
  if (rc) return rc;
  if (precond != NFS_PRECOND_JACOBI && precond != NFS_PRECOND_MG)
    return fail(NFS_EINVAL, "%s: unknown preconditioner %d", fn, precond);
  *bytes = map_layout(kind, n_coil, nx, ny, nz, precond).total;
  return NFS_OK;
}

extern "C" int nfs_sens_initial(nfs_ctx* ctx, const float* imgs, int n_coil, int n_echo, int64_t n_vox, double* shat,
                                void* stream) {
  const char* fn = "nfs_sens_initial";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  if (n_coil < 1 || n_coil > kMaxSvdCoils) return fail(NFS_ESHAPE, "%s: n_coil %d outside [1, %d]", fn, n_coil, kMaxSvdCoils);
  if (n_echo < 1 || n_echo > kMaxMapEchoes) return fail(NFS_ESHAPE, "%s: n_echo %d outside [1, %d]", fn, n_echo, kMaxMapEchoes);
  if (n_vox < 0 || n_vox > ((int64_t)1 << 26)) return fail(NFS_ESHAPE, "%s: n_vox %lld outside [0, 2^26]", fn, (long long)n_vox);
  int rc;
  if ((rc = check_vec(imgs, (int64_t)n_coil * n_echo * n_vox, fn, "imgs"))) return rc;
  if ((rc = check_vec(shat, n_vox, fn, "shat"))) return rc;
  NFS_TRY(launch_sens_initial(reinterpret_cast<const float2*>(imgs), n_coil, n_echo, n_vox,
                              reinterpret_cast<double2*>(shat), (hipStream_t)stream),
          fn);
  return NFS_OK;
}

extern "C" int nfs_sens_maps(nfs_ctx* ctx, const float* imgs, int n_coil, int n_echo, const float* mask_T,
                             const float* mask_R, int nx, int ny, int nz, double alpha, double tol, int max_iter,
                             int precond, float* sens, double* sens64, double* shat, double* parts, int* info,
                             void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nfs_sens_maps";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  if (n_coil < 1 || n_coil > kMaxSvdCoils) return fail(NFS_ESHAPE, "%s: n_coil %d outside [1, %d]", fn, n_coil, kMaxSvdCoils);
  if (n_echo < 1 || n_echo > kMaxMapEchoes) return fail(NFS_ESHAPE, "%s: n_echo %d outside [1, %d]", fn, n_echo, kMaxMapEchoes);
  int64_t L;
  int rc = check_map_grid(nx, ny, nz, fn, &L);
  if (rc) return rc;
  if ((rc = check_solver_args(alpha, tol, max_iter, precond, fn))) return rc;
  if ((rc = check_vec(imgs, (int64_t)n_coil * n_echo * L, fn, "imgs"))) return rc;
  if (!mask_T || !mask_R) return fail(NFS_EINVAL, "%s: mask is NULL", fn);
  if (misaligned(mask_T, 4) || misaligned(mask_R, 4)) return fail(NFS_EINVAL, "%s: mask not 4-byte aligned", fn);
  if (!sens && !sens64) return fail(NFS_EINVAL, "%s: both outputs are NULL", fn);
  if (misaligned(sens, 8) || misaligned(sens64, 16) || misaligned(shat, 16) || misaligned(parts, 8))
    return fail(NFS_EINVAL, "%s: output misaligned", fn);
  const MapLayout m = map_layout(NFS_MAP_SENS, n_coil, nx, ny, nz, precond);
  if ((rc = check_map_ws(m, ws, ws_bytes, fn))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const bool mg = precond == NFS_PRECOND_MG;
  const PcgState st = pcg_state(at<char>(ws, m.pcg), 3 * n_coil, nx, ny, nz, mg);
  double2* sh = shat ? reinterpret_cast<double2*>(shat) : at<double2>(ws, m.shat);
  double* b = at<double>(ws, m.b);
  double* t = at<double>(ws, m.t);
  double* w = at<double>(ws, m.w);
  NFS_TRY(launch_sens_initial(reinterpret_cast<const float2*>(imgs), n_coil, n_echo, L, sh, s), fn);
  NFS_TRY(launch_sens_rhs(sh, mask_T, n_coil, L, st.Lp, b, s), fn);
  NFS_TRY(launch_smooth_setup(MAP_SENS, nx, ny, nz, mask_T, mask_R, nullptr, alpha, t, w, st, s), fn);
  if ((rc = run_pcg(MAP_SENS, precond, st, mg ? at<char>(ws, m.mg) : nullptr, b, nx, ny, nz, t, w, alpha, tol,
                    max_iter, info, s, fn)))
    return rc;
  NFS_TRY(launch_sens_combine(st.x, n_coil, L, st.Lp, reinterpret_cast<float2*>(sens),
                              reinterpret_cast<double2*>(sens64), s),
          fn);
  if (parts && L > 0)
    NFS_TRY(hipMemcpy2DAsync(parts, L * 8, st.x, st.Lp * 8, L * 8, 3 * n_coil, hipMemcpyDeviceToDevice, s), fn);
  return NFS_OK;
}

extern "C" int nfs_b0_map(nfs_ctx* ctx, const float* imgs, int n_coil, int n_echo, const float* sens, int nx, int ny,
                          int nz, double delta_te, double alpha, double tol, int max_iter, int precond, float* b0,
                          double* b064, double* fit, int* info, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "nfs_b0_map";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  if (n_coil < 1 || n_coil > 64) return fail(NFS_ESHAPE, "%s: n_coil %d outside [1, 64]", fn, n_coil);
  if (n_echo < 3 || n_echo > kMaxFitEchoes)
    return fail(NFS_ESHAPE, "%s: n_echo %d outside [3, %d] (the fit has two parameters)", fn, n_echo, kMaxFitEchoes);
  int64_t L;
  int rc = check_map_grid(nx, ny, nz, fn, &L);
  if (rc) return rc;
  if ((rc = check_solver_args(alpha, tol, max_iter, precond, fn))) return rc;
  if (!std::isfinite(delta_te) || !(delta_te > 0.0)) return fail(NFS_EINVAL, "%s: delta_te %g not > 0", fn, delta_te);
  if ((rc = check_vec(imgs, (int64_t)n_coil * n_echo * L, fn, "imgs"))) return rc;
  if ((rc = check_vec(sens, (int64_t)n_coil * L, fn, "sens"))) return rc;
  if (!b0 && !b064 && !fit) return fail(NFS_EINVAL, "%s: every output is NULL", fn);
  if (misaligned(b0, 4) || misaligned(b064, 8) || misaligned(fit, 8)) return fail(NFS_EINVAL, "%s: output misaligned", fn);
  const MapLayout m = map_layout(NFS_MAP_B0, n_coil, nx, ny, nz, precond);
  if ((rc = check_map_ws(m, ws, ws_bytes, fn))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const bool mg = precond == NFS_PRECOND_MG;
  const PcgState st = pcg_state(at<char>(ws, m.pcg), 1, nx, ny, nz, mg);
  double* f = at<double>(ws, m.fit);
  double *b0hat = f, *beta = f + st.Lp, *eps = f + 2 * st.Lp;
  double* w = at<double>(ws, m.w);
  NFS_TRY(launch_b0_fit(reinterpret_cast<const float2*>(imgs), reinterpret_cast<const float2*>(sens), n_coil, n_echo,
                        L, delta_te, b0hat, beta, eps, s),
          fn);
  if (fit && L > 0) {
    NFS_TRY(hipMemcpyAsync(fit, b0hat, L * 8, hipMemcpyDeviceToDevice, s), fn);
    NFS_TRY(hipMemcpyAsync(fit + L, beta, L * 8, hipMemcpyDeviceToDevice, s), fn);
    NFS_TRY(hipMemcpyAsync(fit + 2 * L, eps, L * 8, hipMemcpyDeviceToDevice, s), fn);
  }
  if (!b0 && !b064) {
    if (info) info[0] = info[1] = 0;
    return NFS_OK;
  }
  NFS_TRY(launch_smooth_setup(MAP_B0, nx, ny, nz, nullptr, nullptr, eps, alpha, nullptr, w, st, s), fn);
  if ((rc = run_pcg(MAP_B0, precond, st, mg ? at<char>(ws, m.mg) : nullptr, b0hat, nx, ny, nz, nullptr, w, alpha, tol,
                    max_iter, info, s, fn)))
    return rc;
  NFS_TRY(launch_b0_store(st.x, L, b0, b064, s), fn);
  return NFS_OK;
}

// ---------------------------------------------------------------------------
// Phase-basis compression (host).  phi(k, l) = sum_b a_b(k) h_b(l) over the
// T = P + 1 terms (a_0 = t, h_0 = b0; a_{b+1} = kcoef[.][b], h_{b+1} =
// fields[b]).  With s_b = max_k |a_b| and the scaled rows h^_b = s_b h_b,
// mu_b = mean_l h^_b and A_b = h^_b - mu_b, the phase is exactly
//   phi = theta(k) + sum_b (a_b / s_b)(k) A_b(l),  theta = sum_b (a_b / s_b) mu_b.
// The rows A_b span a space of some numerical rank r <= T; with U the
// eigenvectors of the Gram matrix A A^T (cyclic Jacobi, largest eigenvalue
// first), direction j has voxel side h'_j = sum_b U_bj A_b and sample side
// a'_j = sum_b (a_b / s_b) U_bj.  Directions are added in that order until
// the residual E_b = A_b - sum_{j <= r} U_bj h'_j satisfies
//   max_l sum_b |E_b(l)| <= rel_tol * sum_b max|a_b| max|h_b|,
// which bounds the phase change at every (k, l), since |a_b / s_b| <= 1.
// Everything runs in double precision; the outputs are rounded once.

// eigenvalues (descending) and eigenvectors (columns of U, row-major T x T)
// of the symmetric matrix S (row-major, overwritten), by cyclic Jacobi
// rotations
static void jacobi_eigen(std::vector<double>& S, int T, std::vector<double>* lam, std::vector<double>* U) {
  std::vector<double> V((size_t)T * T, 0.0);
  for (int i = 0; i < T; ++i) V[(size_t)i * T + i] = 1.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < T; ++p) {
      diag += S[(size_t)p * T + p] * S[(size_t)p * T + p];
      for (int q = p + 1; q < T; ++q) off += S[(size_t)p * T + q] * S[(size_t)p * T + q];
    }
    if (off <= 1e-34 * diag || off == 0.0) break;
    for (int p = 0; p < T; ++p)
      for (int q = p + 1; q < T; ++q) {
        const double apq = S[(size_t)p * T + q];
        if (apq == 0.0) continue;
        const double app = S[(size_t)p * T + p], aqq = S[(size_t)q * T + q];
        // rotation angle that zeroes S[p][q]: tan(theta) = t, the smaller root
        const double zeta = (aqq - app) / (2.0 * apq);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < T; ++k) {  // columns p, q
          const double skp = S[(size_t)k * T + p], skq = S[(size_t)k * T + q];
          S[(size_t)k * T + p] = c * skp - s * skq;
          S[(size_t)k * T + q] = s * skp + c * skq;
        }
        for (int k = 0; k < T; ++k) {  // rows p, q
          const double spk = S[(size_t)p * T + k], sqk = S[(size_t)q * T + k];
          S[(size_t)p * T + k] = c * spk - s * sqk;
          S[(size_t)q * T + k] = s * spk + c * sqk;
        }
        for (int k = 0; k < T; ++k) {
          const double vkp = V[(size_t)k * T + p], vkq = V[(size_t)k * T + q];
          V[(size_t)k * T + p] = c * vkp - s * vkq;
          V[(size_t)k * T + q] = s * vkp + c * vkq;
        }
      }
  }
  std::vector<int> order(T);
  for (int i = 0; i < T; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return S[(size_t)x * T + x] > S[(size_t)y * T + y]; });
  lam->assign(T, 0.0);
  U->assign((size_t)T * T, 0.0);
  for (int j = 0; j < T; ++j) {
    (*lam)[j] = S[(size_t)order[j] * T + order[j]];
    for (int b = 0; b < T; ++b) (*U)[(size_t)b * T + j] = V[(size_t)b * T + order[j]];
  }
}

extern "C" int nfs_compress_basis(const float* fields, const float* b0, const float* kcoef, const float* t,
                                  int64_t L, int64_t K, int P, double rel_tol, float* fields_out, float* b0_out,
                                  float* kcoef_out, float* t_out, double* theta, int* n_basis_out,
                                  double* err_bound) {
  const char* fn = "nfs_compress_basis";
  const int64_t lim = (int64_t)1 << 26;
  if (L < 0 || L > lim || K < 0 || K > lim) return fail(NFS_ESHAPE, "%s: L or K outside [0, 2^26]", fn);
  if (P < 0 || P > 31) return fail(NFS_ESHAPE, "%s: n_basis %d outside [0, 31]", fn, P);
  if (!(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return fail(NFS_EINVAL, "%s: rel_tol must be finite and >= 0", fn);
  if ((L > 0 && (!b0 || !b0_out)) || (K > 0 && (!t || !t_out || !theta)) || !n_basis_out ||
      (P > 0 && L > 0 && (!fields || !fields_out)) || (P > 0 && K > 0 && (!kcoef || !kcoef_out)))
    return fail(NFS_EINVAL, "%s: NULL array", fn);
  const double tol_rel = rel_tol > 0.0 ? rel_tol : std::ldexp(1.0, -24);
  const int T = P + 1;
  auto a_at = [&](int b, int64_t k) -> double { return b == 0 ? (double)t[k] : (double)kcoef[k * P + (b - 1)]; };
  auto h_at = [&](int b, int64_t l) -> double { return b == 0 ? (double)b0[l] : (double)fields[(b - 1) * L + l]; };
  std::vector<double> s(T, 0.0), hmax(T, 0.0);
  for (int b = 0; b < T; ++b) {
    for (int64_t k = 0; k < K; ++k) {
      const double v = a_at(b, k);
      if (!std::isfinite(v)) return fail(NFS_EINVAL, "%s: non-finite sample coefficient (term %d)", fn, b);
      s[b] = std::max(s[b], std::fabs(v));
    }
    for (int64_t l = 0; l < L; ++l) {
      const double v = h_at(b, l);
      if (!std::isfinite(v)) return fail(NFS_EINVAL, "%s: non-finite voxel coefficient (term %d)", fn, b);
      hmax[b] = std::max(hmax[b], std::fabs(v));
    }
  }
  double bound = 0.0;
  for (int b = 0; b < T; ++b) bound += s[b] * hmax[b];
  const double tol = tol_rel * bound;
  // scaled, centred voxel rows A_b and their means
  std::vector<double> A((size_t)T * L), mu(T, 0.0);
  for (int b = 0; b < T; ++b) {
    double sum = 0.0;
    for (int64_t l = 0; l < L; ++l) {
      const double v = s[b] * h_at(b, l);
      A[(size_t)b * L + l] = v;
      sum += v;
    }
    mu[b] = L > 0 ? sum / (double)L : 0.0;
    for (int64_t l = 0; l < L; ++l) A[(size_t)b * L + l] -= mu[b];
  }
  std::vector<double> S((size_t)T * T, 0.0);
  for (int p = 0; p < T; ++p)
    for (int q = p; q < T; ++q) {
      double acc = 0.0;
      for (int64_t l = 0; l < L; ++l) acc += A[(size_t)p * L + l] * A[(size_t)q * L + l];
      S[(size_t)p * T + q] = S[(size_t)q * T + p] = acc;
    }
  std::vector<double> lam, U;
  jacobi_eigen(S, T, &lam, &U);
  // add directions until the residual bound holds
  std::vector<double> E(A), H;  // E: residual rows; H: kept voxel sides, row j
  auto resid = [&]() {
    double worst = 0.0;
    for (int64_t l = 0; l < L; ++l) {
      double acc = 0.0;
      for (int b = 0; b < T; ++b) acc += std::fabs(E[(size_t)b * L + l]);
      worst = std::max(worst, acc);
    }
    return worst;
  };
  int r = 0;
  double err = resid();
  while (err > tol && r < T) {
    std::vector<double> h(L, 0.0);
    for (int b = 0; b < T; ++b) {
      const double u = U[(size_t)b * T + r];
      if (u != 0.0)
        for (int64_t l = 0; l < L; ++l) h[l] += u * A[(size_t)b * L + l];
    }
    for (int b = 0; b < T; ++b) {
      const double u = U[(size_t)b * T + r];
      if (u != 0.0)
        for (int64_t l = 0; l < L; ++l) E[(size_t)b * L + l] -= u * h[l];
    }
    H.insert(H.end(), h.begin(), h.end());
    ++r;
    err = resid();
  }
  // outputs: direction 0 in the (t, b0) slot, directions 1.. as field terms
  const int Pn = r > 0 ? r - 1 : 0;
  for (int64_t k = 0; k < K; ++k) {
    double th = 0.0;
    double as[32];
    for (int b = 0; b < T; ++b) {
      as[b] = s[b] > 0.0 ? a_at(b, k) / s[b] : 0.0;
      th += as[b] * mu[b];
    }
    theta[k] = th;
    for (int j = 0; j < std::max(r, 1); ++j) {
      double v = 0.0;
      if (j < r)
        for (int b = 0; b < T; ++b) v += as[b] * U[(size_t)b * T + j];
      if (j == 0)
        t_out[k] = (float)v;
      else
        kcoef_out[k * Pn + (j - 1)] = (float)v;
    }
  }
  for (int64_t l = 0; l < L; ++l) {
    b0_out[l] = r > 0 ? (float)H[l] : 0.f;
    for (int j = 1; j < r; ++j) fields_out[(j - 1) * L + l] = (float)H[(size_t)j * L + l];
  }
  *n_basis_out = Pn;
  if (err_bound) *err_bound = err;
  return NFS_OK;
}

// The same compression on the device (compress_kernels.hip): term maxima,
// then the launches of launch_compress_basis; the workspace holds the term
// maxima and the double-precision scratch.
static size_t compress_ws_bytes(int64_t L, int P) {
  return al(2 * kMaxTerms * 4) + al(compress_workspace_doubles(L, P) * 8);
}

extern "C" int nfs_compress_workspace_bytes(const nfs_problem* prob, size_t* bytes) {
  const char* fn = "nfs_compress_workspace_bytes";
  if (!bytes) return fail(NFS_EINVAL, "%s: bytes is NULL", fn);
  int rc = check_sizes(prob, fn);
  if (rc) return rc;
  *bytes = compress_ws_bytes(prob->n_vox, prob->n_basis);
  return NFS_OK;
}

extern "C" int nfs_compress_basis_device(nfs_ctx* ctx, const nfs_problem* prob, double rel_tol, float* fields_out,
                                         float* b0_out, float* kcoef_out, float* t_out, double* theta,
                                         int* n_basis_out, double* err_bound, void* ws, size_t ws_bytes,
                                         void* stream) {
  const char* fn = "nfs_compress_basis_device";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  int rc = check_sizes(prob, fn);
  if (rc) return rc;
  if (!(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return fail(NFS_EINVAL, "%s: rel_tol must be finite and >= 0", fn);
  const int64_t L = prob->n_vox, K = prob->n_samp;
  const int P = prob->n_basis;
  if ((L > 0 && (!prob->b0 || !b0_out)) || (K > 0 && (!prob->t || !t_out || !theta)) || !n_basis_out ||
      (P > 0 && L > 0 && (!prob->fields || !fields_out)) || (P > 0 && K > 0 && (!prob->kcoef || !kcoef_out)))
    return fail(NFS_EINVAL, "%s: NULL array", fn);
  if (misaligned(prob->fields, 4) || misaligned(prob->b0, 4) || misaligned(prob->kcoef, 4) || misaligned(prob->t, 4) ||
      misaligned(fields_out, 4) || misaligned(b0_out, 4) || misaligned(kcoef_out, 4) || misaligned(t_out, 4) ||
      misaligned(theta, 8) || misaligned(n_basis_out, 4) || misaligned(err_bound, 8))
    return fail(NFS_EINVAL, "%s: array misaligned", fn);
  if (!ws) return fail(NFS_EWORKSPACE, "%s: workspace is NULL", fn);
  if ((uintptr_t)ws % 256) return fail(NFS_EWORKSPACE, "%s: workspace not 256-byte aligned", fn);
  const size_t need = compress_ws_bytes(L, P);
  if (ws_bytes < need) return fail(NFS_EWORKSPACE, "%s: workspace has %zu bytes, needs %zu", fn, ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  unsigned* tmax = static_cast<unsigned*>(ws);
  double* dws = reinterpret_cast<double*>(static_cast<char*>(ws) + al(2 * kMaxTerms * 4));
  NFS_TRY(launch_term_absmax(prob->t, prob->kcoef, K, prob->b0, prob->fields, L, P, tmax, s), "term_absmax");
  NFS_TRY(launch_compress_basis(prob->fields, prob->b0, prob->kcoef, prob->t, L, K, P,
                                rel_tol > 0.0 ? rel_tol : std::ldexp(1.0, -24), tmax, dws, fields_out, b0_out,
                                kcoef_out, t_out, theta, n_basis_out, err_bound, s),
          "compress_basis");
  return NFS_OK;
}

extern "C" int nfs_phase_shift(nfs_ctx* ctx, const float* m, float* out, int n_coil, int64_t K, const double* theta,
                               int sign, void* stream) {
  const char* fn = "nfs_phase_shift";
  if (!ctx) return fail(NFS_EINVAL, "%s: ctx is NULL", fn);
  if (n_coil < 1 || n_coil > 64 || K < 0 || K > ((int64_t)1 << 26))
    return fail(NFS_ESHAPE, "%s: n_coil %d or K %lld out of range", fn, n_coil, (long long)K);
  if (sign != 1 && sign != -1) return fail(NFS_EINVAL, "%s: sign must be +1 or -1", fn);
  if (K > 0 && (!m || !out || !theta)) return fail(NFS_EINVAL, "%s: NULL array", fn);
  if (misaligned(m, 8) || misaligned(out, 8) || misaligned(theta, 8)) return fail(NFS_EINVAL, "%s: array misaligned", fn);
  NFS_TRY(launch_phase_shift(reinterpret_cast<const float2*>(m), reinterpret_cast<float2*>(out), theta, n_coil, K,
                             sign, (hipStream_t)stream),
          fn);
  return NFS_OK;
}
