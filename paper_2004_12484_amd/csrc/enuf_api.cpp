// enuf_api.cpp -- host side of the ENUF C ABI (include/enuf.h): parameter
// validation, the workspace layout, stream binding, HIP graph replay and the
// launch sequences.  The library allocates no device memory unless asked to
// (enuf_alloc_workspace).
#include "enuf.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "enuf_internal.h"

using enuf::Geom;
using enuf::Work;

// Device scratch of enuf_energy_forces_noalloc: one block per GPU, part of the
// library's code object (no allocation call creates it), held until the
// process ends.  In host code `scratch` only names the symbol; its device
// address on the current GPU comes from hipGetSymbolAddress, taken once per
// device (scratch_address) and used wherever host code needs the memory.
static __device__ __align__(256) unsigned char scratch[ENUF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kAlign = 256;

// The captured launch sequence of one evaluation and the arguments and
// options it was captured with (a call with other ones captures again).
struct GraphCache {
  hipGraphExec_t exec = nullptr;
  const void *x = nullptr, *q = nullptr;
  double *E = nullptr;
  void *F = nullptr, *phi = nullptr, *ws = nullptr;
  bool analytic = false;
  double ke = 0.0, slater = 0.0;
  int win = 0;
  double sigma = 1.0;
  int spread16 = 0;
  int det = 0;
};

constexpr size_t kScratchBytes = ENUF_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on GPU `dev`, which must be the current device.
hipError_t scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

struct enuf_ctx_s {
  Geom g{};                    // parameters of the next evaluation
  Work w{};                    // workspace pointers (valid when have_ws)
  int nruns = 0;               // spread run-table entries
  int prec = ENUF_FP64;
  hipStream_t st = nullptr;
  int device = 0;
  bool have_ws = false;
  void *owned_ws = nullptr;    // workspace from enuf_alloc_workspace
  void *ws = nullptr;          // the workspace block given (before alignment)
  size_t ws_bytes = 0;
  // the last evaluation on the context workspace, read by the adjoint
  bool have_forward = false;
  bool last_all_active = false;
  bool last_analytic = false;  // it left psi as a plain real grid
  Geom gf{};                   // its parameters (ke, Slater length)
  uint64_t token = 0;          // evaluations on the context workspace so far
  bool check = false;
  bool analytic = false;       // ENUF_OPT_FORCE_MODE = 1
  // graph replay (ENUF_OPT_GRAPH)
  bool graph = false;
  hipStream_t gst = nullptr;
  hipEvent_t gev[2] = {nullptr, nullptr};
  GraphCache gc;
  // timing ring: `slots` evaluations x (kPhases + 1) events
  std::vector<hipEvent_t> ring;
  int slots = 0, next = 0, recorded = 0;
  std::string err;
};

static thread_local std::string g_create_err;

static enuf_status fail(enuf_ctx c, enuf_status s, const std::string &msg) {
  if (c) c->err = msg; else g_create_err = msg;
  return s;
}

static enuf_status hip_fail(enuf_ctx c, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(c, ENUF_EDEVICE, m);
}

static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Real-space cells of side > r_c + skin (at most 2^22 of them) and the spill
// margin of the tile classes, ceil(skin/2 in grid points) per axis, for
// persistent binning with that skin (0: none).
static void set_cells(Geom &g, double skin) {
  const double side = g.rc + skin;
  for (int d = 0; d < 3; ++d) {
    int nc = (int)std::floor(g.L[d] / (side * (1.0 + 1e-5)));
    g.nc[d] = std::max(1, std::min(nc, 1024));
  }
  while ((int64_t)g.nc[0] * g.nc[1] * g.nc[2] > (int64_t(1) << 22)) {
    int dm = 0;
    for (int d = 1; d < 3; ++d) if (g.nc[d] > g.nc[dm]) dm = d;
    g.nc[dm] = std::max(1, g.nc[dm] / 2);
  }
  for (int d = 0; d < 3; ++d) {
    g.cL[d] = g.nc[d] / g.L[d];
    g.sdig[d] = skin > 0.0 ? (int)std::ceil(0.5 * skin * g.mL[d] - 1e-12) : 0;
    if (skin > 0.0) g.sdig[d] = std::max(1, g.sdig[d]);
  }
  g.ncells = g.nc[0] * g.nc[1] * g.nc[2];
  g.skin = skin;
}

static size_t real_bytes(enuf_ctx c) { return c->prec == ENUF_FP64 ? 8 : 4; }

// Workspace layout: every buffer starts on a 256-byte boundary of one block.
// With base == nullptr only the size is computed.  The size returned includes
// 256 bytes of slack so that any caller pointer can be aligned up.
static size_t layout(const Geom &g, size_t rs, char *base, Work *w) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void * {
    off = (off + kAlign - 1) / kAlign * kAlign;
    void *p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const size_t n = (size_t)g.n;
  const size_t G = (size_t)g.M[0] * g.M[1] * g.M[2];
  const enuf::SortPlan sp = enuf::sort_plan(g, (int)rs);
  const size_t nbk = (size_t)sp.nb[0] + sp.nb[1];
  Work t;
  t.part_t = take(n * 4 * rs);
  t.part_c = take(n * 4 * rs);
  t.perm_t = (int *)take(n * 4);
  t.perm_c = (int *)take(n * 4);
  t.key_t = (int *)take(n * 4);
  t.key_c = (int *)take(n * 4);
  t.off_t = (int *)take(((size_t)sp.nbins[0] + 1) * 4);
  t.off_c = (int *)take(((size_t)sp.nbins[1] + 1) * 4);
  t.hist = (int *)take((size_t)sp.nblk * nbk * 4);
  t.bbase = (int *)take((nbk + 2) * 4);
  t.stg_t = take(n * 4 * rs);
  t.stg_c = take(n * 4 * rs);
  t.ik_t = (int2 *)take(n * sizeof(int2));
  t.ik_c = (int2 *)take(n * sizeof(int2));
  t.runs = (int *)take((size_t)5 * enuf::kMaxRuns * 4);
  t.counts = (int *)take(8 * 4);
  t.x_ref = take(n * 3 * rs);
  t.q_ref = take(n * rs);
  t.act = (int *)take(n * 4);
  t.scal = (double *)take(4 * 8);
  t.qpart = (double *)take((size_t)4 * sp.nblk * 8);
  t.eslot = (double *)take(enuf::eslot_len(g) * 8);
  t.grid = take(G * rs);
  t.spec = take(G / 2 * 2 * rs);
  t.fspec = take(4 * (G / 2) * 2 * rs);
  t.field = take(G * 4 * rs);
  const size_t ntab = enuf::table_size(g, t.tab_off);
  t.tables = take(ntab * rs);
  if (w) *w = t;
  return (off + kAlign - 1) / kAlign * kAlign + kAlign;
}

static void drop_graph(enuf_ctx c) {
  if (c->gc.exec) (void)hipGraphExecDestroy(c->gc.exec);
  c->gc = GraphCache{};
}

static void release(enuf_ctx c) {
  drop_graph(c);
  if (c->owned_ws) (void)hipFree(c->owned_ws);
  c->owned_ws = nullptr;
  for (auto &e : c->ring) (void)hipEventDestroy(e);
  c->ring.clear();
  c->slots = c->next = c->recorded = 0;
  for (auto &e : c->gev)
    if (e) (void)hipEventDestroy(e);
  c->gev[0] = c->gev[1] = nullptr;
  if (c->gst) (void)hipStreamDestroy(c->gst);
  c->gst = nullptr;
}

// Window and kept modes from the options: kept_d = 2 floor(M_d / (2 sigma)),
// and for the Gaussian the NFFT shape b = 2 sigma m / ((2 sigma - 1) pi) of
// cutoff m = p/2 - 1.  The tables depend on them: a context with a workspace
// initialises it again (which also forgets the last evaluation).
static enuf_status apply_window(enuf_ctx c, int win, double sigma);

static hipError_t sync_stream(enuf_ctx c) { return c->st ? hipStreamSynchronize(c->st) : hipDeviceSynchronize(); }

// Point the context at a workspace block (aligned up) and enqueue its
// initialisation on the context stream.
static enuf_status attach(enuf_ctx c, void *ws) {
  char *b = (char *)(((uintptr_t)ws + kAlign - 1) & ~(uintptr_t)(kAlign - 1));
  Work w;
  layout(c->g, real_bytes(c), b, &w);
  w.nruns = c->nruns;
  hipError_t e = enuf::launch_init_ws(c->g, w, c->st, c->prec == ENUF_FP64);
  if (e != hipSuccess) return hip_fail(c, e, "workspace initialisation");
  c->w = w;
  c->have_ws = true;
  c->have_forward = false;
  return ENUF_OK;
}

static hipError_t forward(enuf_ctx c, const Work &w, hipStream_t st, const void *x, const void *q, double *E,
                          void *F, void *phi, bool all, bool an, hipEvent_t *ev) {
  if (c->prec == ENUF_FP64)
    return enuf::launch_forward<double>(c->g, w, st, (const double *)x, (const double *)q, E, (double *)F,
                                        (double *)phi, all, all, an, ev);
  return enuf::launch_forward<float>(c->g, w, st, (const float *)x, (const float *)q, E, (float *)F, (float *)phi,
                                     all, all, an, ev);
}

// One evaluation replayed as a HIP graph on the context's own stream, joined
// to the caller's stream by events on both sides.  The graph is captured on
// the first call and again whenever the pointers or options change.
static hipError_t run_graph(enuf_ctx c, const void *x, const void *q, double *E, void *F, void *phi, bool all,
                            bool an) {
  GraphCache &gc = c->gc;
  const bool hit = gc.exec && gc.x == x && gc.q == q && gc.E == E && gc.F == F && gc.phi == phi &&
                   gc.ws == c->w.grid && gc.analytic == an && gc.ke == c->g.ke && gc.slater == c->g.slater &&
                   gc.win == c->g.win && gc.sigma == c->g.sigma && gc.spread16 == c->g.spread16 &&
                   gc.det == c->g.det;
  if (!hit) {
    drop_graph(c);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(c->gst, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t el = forward(c, c->w, c->gst, x, q, E, F, phi, all, an, nullptr);
    e = hipStreamEndCapture(c->gst, &graph);
    if (el != hipSuccess || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return el != hipSuccess ? el : e;
    }
    e = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      gc.exec = nullptr;
      return e;
    }
    gc.x = x;
    gc.q = q;
    gc.E = E;
    gc.F = F;
    gc.phi = phi;
    gc.ws = c->w.grid;
    gc.analytic = an;
    gc.ke = c->g.ke;
    gc.slater = c->g.slater;
    gc.win = c->g.win;
    gc.sigma = c->g.sigma;
    gc.spread16 = c->g.spread16;
    gc.det = c->g.det;
  }
  hipError_t e = hipEventRecord(c->gev[0], c->st);
  if (e == hipSuccess) e = hipStreamWaitEvent(c->gst, c->gev[0], 0);
  if (e == hipSuccess) e = hipGraphLaunch(gc.exec, c->gst);
  if (e == hipSuccess) e = hipEventRecord(c->gev[1], c->gst);
  if (e == hipSuccess) e = hipStreamWaitEvent(c->st, c->gev[1], 0);
  return e;
}

extern "C" {

enuf_status enuf_copy_probe(const void *src, void *dst, size_t bytes, void *stream) {
  if (!src || !dst) return fail(nullptr, ENUF_EINVAL, "src or dst is NULL");
  if (bytes == 0 || bytes % 16 != 0) return fail(nullptr, ENUF_EINVAL, "bytes must be a positive multiple of 16");
  if ((uintptr_t)src % 16 != 0 || (uintptr_t)dst % 16 != 0)
    return fail(nullptr, ENUF_EINVAL, "src and dst must be 16-byte aligned");
  const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
  if (a < b + bytes && b < a + bytes) return fail(nullptr, ENUF_EINVAL, "src and dst overlap");
  hipError_t e = enuf::launch_copy16(src, dst, bytes / 16, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(nullptr, e, "copy probe launch");
  return ENUF_OK;
}

int32_t enuf_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

const char *enuf_status_string(enuf_status s) {
  switch (s) {
    case ENUF_OK: return "ok";
    case ENUF_EINVAL: return "invalid argument";
    case ENUF_ENOMEM: return "out of memory";
    case ENUF_EDEVICE: return "device error";
    case ENUF_ENONFINITE: return "non-finite input";
    case ENUF_ESTATE: return "invalid call sequence";
    case ENUF_EUNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

const char *enuf_last_error(enuf_ctx ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

enuf_status enuf_create(enuf_ctx *out, const double box[3], int64_t n, double alpha, double r_c,
                        const int32_t M[3], int32_t p, int32_t precision, void *stream) {
  if (!out) return fail(nullptr, ENUF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!box || !M) return fail(nullptr, ENUF_EINVAL, "box or M is NULL");
  if (n <= 0 || n > (int64_t(1) << 28)) return fail(nullptr, ENUF_EINVAL, "n must be in [1, 2^28]");
  for (int d = 0; d < 3; ++d)
    if (!(box[d] > 0.0) || !std::isfinite(box[d])) return fail(nullptr, ENUF_EINVAL, "box lengths must be > 0");
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(nullptr, ENUF_EINVAL, "alpha must be > 0");
  if (!(r_c > 0.0) || !std::isfinite(r_c)) return fail(nullptr, ENUF_EINVAL, "r_c must be > 0");
  if (precision != ENUF_FP64 && precision != ENUF_FP32) return fail(nullptr, ENUF_EINVAL, "bad precision");
  if (p != 2 && p != 4 && p != 6 && p != 8) return fail(nullptr, ENUF_EINVAL, "p must be 2, 4, 6 or 8");
  for (int d = 0; d < 3; ++d) {
    if (!pow2(M[d]) || M[d] < 8 || M[d] > 1024) return fail(nullptr, ENUF_EINVAL, "M must be powers of two in [8, 1024]");
    if (2 * p > M[d]) return fail(nullptr, ENUF_EINVAL, "need 2p <= M on every axis");
  }
  const double lmin = std::fmin(box[0], std::fmin(box[1], box[2]));
  if (r_c > 0.5 * lmin * (1.0 + 1e-12))
    return fail(nullptr, ENUF_EUNSUPPORTED, "r_c > min(L)/2 (minimum image) is not supported");

  Geom g{};
  const int tdef[3] = {enuf::kTileX, enuf::kTileY, enuf::kTileZ};
  for (int d = 0; d < 3; ++d) {
    g.M[d] = M[d];
    g.T[d] = std::min(tdef[d], M[d] / 2);
    g.nt[d] = M[d] / g.T[d];
    g.L[d] = box[d];
    g.iL[d] = 1.0 / g.L[d];
    g.mL[d] = g.M[d] / g.L[d];
  }
  g.ntiles = g.nt[0] * g.nt[1] * g.nt[2];
  g.p = p;
  g.n = (int)n;
  g.alpha = alpha;
  g.rc = r_c;
  set_cells(g, 0.0);
  g.ke = 1.0;
  g.slater = 0.0;
  g.win = 0;
  g.gb = g.gib = 0.0;
  g.sigma = 1.0;
  for (int d = 0; d < 3; ++d) g.kept[d] = g.M[d];
  g.spread16 = 0;
  g.det = 0;

  const size_t rs = precision == ENUF_FP64 ? 8 : 4;
  if (!enuf::fft_plans_fit(g, precision == ENUF_FP64))
    return fail(nullptr, ENUF_EUNSUPPORTED, "grid transform does not fit one workgroup's LDS");
  const enuf::SortPlan sp = enuf::sort_plan(g, (int)rs);
  const size_t nbk = (size_t)sp.nb[0] + sp.nb[1];
  if (nbk * sizeof(int) > 65536 || enuf::sort_stage_lds(sp, (int)rs) > 65536 || enuf::sort_fine_lds(sp) > 65536)
    return fail(nullptr, ENUF_EUNSUPPORTED, "too many sort buckets for one workgroup's LDS");
  int runs[5 * enuf::kMaxRuns];
  const int nruns = enuf::build_runs(g, runs);
  if (nruns <= 0) return fail(nullptr, ENUF_EUNSUPPORTED, "spread run table overflow");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");

  enuf_ctx c = new (std::nothrow) enuf_ctx_s();
  if (!c) return fail(nullptr, ENUF_ENOMEM, "host allocation failed");
  c->g = g;
  c->nruns = nruns;
  c->prec = precision;
  c->st = reinterpret_cast<hipStream_t>(stream);
  c->device = dev;
  *out = c;
  return ENUF_OK;
}

enuf_status enuf_workspace_bytes(enuf_ctx ctx, size_t *bytes) {
  if (!ctx || !bytes) return fail(ctx, ENUF_EINVAL, "ctx or bytes is NULL");
  *bytes = layout(ctx->g, real_bytes(ctx), nullptr, nullptr);
  return ENUF_OK;
}

enuf_status enuf_set_workspace(enuf_ctx ctx, void *ws, size_t bytes) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  if (!ws) return fail(ctx, ENUF_EINVAL, "workspace pointer is NULL");
  const size_t need = layout(ctx->g, real_bytes(ctx), nullptr, nullptr);
  if (bytes < need)
    return fail(ctx, ENUF_EINVAL, "workspace too small: " + std::to_string(bytes) + " bytes given, " +
                                      std::to_string(need) + " needed (enuf_workspace_bytes)");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  if (ctx->owned_ws) {
    // the library's own block may still be in use by enqueued work
    e = sync_stream(ctx);
    if (e != hipSuccess) return hip_fail(ctx, e, "synchronize");
    (void)hipFree(ctx->owned_ws);
    ctx->owned_ws = nullptr;
  }
  drop_graph(ctx);
  ctx->have_ws = false;
  ctx->ws = ws;
  ctx->ws_bytes = bytes;
  return attach(ctx, ws);
}

enuf_status enuf_alloc_workspace(enuf_ctx ctx) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  const size_t need = layout(ctx->g, real_bytes(ctx), nullptr, nullptr);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  void *p = nullptr;
  if (std::getenv("ENUF_FAIL_ALLOC") || hipMalloc(&p, need) != hipSuccess)
    return fail(ctx, ENUF_ENOMEM, "device workspace allocation of " + std::to_string(need) + " bytes failed");
  enuf_status s = enuf_set_workspace(ctx, p, need);
  if (s != ENUF_OK) {
    (void)hipFree(p);
    return s;
  }
  ctx->owned_ws = p;
  return ENUF_OK;
}

enuf_status enuf_destroy(enuf_ctx ctx) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  (void)hipSetDevice(ctx->device);
  (void)sync_stream(ctx);
  if (ctx->gst) (void)hipStreamSynchronize(ctx->gst);
  release(ctx);
  delete ctx;
  return ENUF_OK;
}

enuf_status enuf_set_option(enuf_ctx ctx, int32_t option, double value) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  switch (option) {
    case ENUF_OPT_KE:
      if (!(value > 0.0) || !std::isfinite(value)) return fail(ctx, ENUF_EINVAL, "ke must be > 0");
      ctx->g.ke = value;
      return ENUF_OK;
    case ENUF_OPT_TIMING: {
      if (!(value >= 0.0 && value <= 4096.0) || value != std::floor(value))
        return fail(ctx, ENUF_EINVAL, "timing slots must be an integer in [0, 4096]");
      for (auto &e : ctx->ring) (void)hipEventDestroy(e);
      ctx->ring.clear();
      ctx->slots = ctx->next = ctx->recorded = 0;
      const int slots = (int)value;
      if (slots > 0) {
        ctx->ring.resize((size_t)slots * (enuf::kPhases + 1));
        for (auto &e : ctx->ring) {
          hipError_t r = hipEventCreate(&e);
          if (r != hipSuccess) {
            e = nullptr;
            return hip_fail(ctx, r, "hipEventCreate");
          }
        }
        ctx->slots = slots;
      }
      return ENUF_OK;
    }
    case ENUF_OPT_GRAPH: {
      if (value != 0.0 && value != 1.0) return fail(ctx, ENUF_EINVAL, "graph is 0 or 1");
      drop_graph(ctx);
      ctx->graph = value == 1.0;
      if (ctx->graph && !ctx->gst) {
        hipError_t e = hipSetDevice(ctx->device);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->gst, hipStreamNonBlocking);
        for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&ctx->gev[k], hipEventDisableTiming);
        if (e != hipSuccess) {
          ctx->graph = false;
          return hip_fail(ctx, e, "graph stream set-up");
        }
      }
      return ENUF_OK;
    }
    case ENUF_OPT_CHECK:
      if (value != 0.0 && value != 1.0) return fail(ctx, ENUF_EINVAL, "check is 0 or 1");
      ctx->check = value == 1.0;
      return ENUF_OK;
    case ENUF_OPT_FORCE_MODE:
      if (value != 0.0 && value != 1.0) return fail(ctx, ENUF_EINVAL, "force mode is 0 (ik) or 1 (analytic)");
      ctx->analytic = value == 1.0;
      return ENUF_OK;
    case ENUF_OPT_SLATER:
      if (!(value >= 0.0) || !std::isfinite(value)) return fail(ctx, ENUF_EINVAL, "lambda_e must be >= 0 and finite");
      ctx->g.slater = value;
      return ENUF_OK;
    case ENUF_OPT_SKIN: {
      if (!(value >= 0.0) || !std::isfinite(value)) return fail(ctx, ENUF_EINVAL, "skin must be >= 0 and finite");
      Geom g2 = ctx->g;
      set_cells(g2, value);
      for (int d = 0; d < 3; ++d)
        if (g2.p + 2 * g2.sdig[d] > g2.T[d] + 1)
          return fail(ctx, ENUF_EUNSUPPORTED,
                      "skin too large for the window and grid: p + 2 ceil(skin/2 M/L) must not exceed the spread "
                      "tile (" + std::to_string(g2.T[d]) + " points on axis " + std::to_string(d) + ") plus 1");
      const size_t rs = real_bytes(ctx);
      const enuf::SortPlan sp = enuf::sort_plan(g2, (int)rs);
      const size_t nbk = (size_t)sp.nb[0] + sp.nb[1];
      if (nbk * sizeof(int) > 65536 || enuf::sort_stage_lds(sp, (int)rs) > 65536 || enuf::sort_fine_lds(sp) > 65536)
        return fail(ctx, ENUF_EUNSUPPORTED, "too many sort buckets for one workgroup's LDS");
      if (ctx->have_ws && layout(g2, rs, nullptr, nullptr) > ctx->ws_bytes)
        return fail(ctx, ENUF_ESTATE, "the workspace is too small for this skin: set a new one of "
                                      "enuf_workspace_bytes() bytes");
      ctx->g = g2;
      drop_graph(ctx);
      if (ctx->have_ws) {
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
        return attach(ctx, ctx->ws);
      }
      return ENUF_OK;
    }
    case ENUF_OPT_DETERMINISTIC:
      if (value != 0.0 && value != 1.0) return fail(ctx, ENUF_EINVAL, "deterministic is 0 or 1");
      ctx->g.det = (int)value;
      drop_graph(ctx);
      return ENUF_OK;
    case ENUF_OPT_SPREAD_F16:
      if (value != 0.0 && value != 1.0) return fail(ctx, ENUF_EINVAL, "spread product mode is 0 or 1");
      ctx->g.spread16 = (int)value;
      drop_graph(ctx);
      return ENUF_OK;
    case ENUF_OPT_WINDOW:
      if (value != 0.0 && value != 1.0) return fail(ctx, ENUF_EINVAL, "window is 0 (B-spline) or 1 (Gaussian)");
      if (value == 1.0 && ctx->g.p < 4) return fail(ctx, ENUF_EINVAL, "the Gaussian window needs p >= 4 (cutoff m = p/2 - 1 >= 1)");
      return apply_window(ctx, (int)value, ctx->g.sigma);
    case ENUF_OPT_OVERSAMPLING:
      if (!(value >= 1.0) || !std::isfinite(value)) return fail(ctx, ENUF_EINVAL, "oversampling factor must be >= 1");
      for (int d = 0; d < 3; ++d)
        if (2 * (int)std::floor(ctx->g.M[d] / (2.0 * value) + 1e-9) < 2)
          return fail(ctx, ENUF_EINVAL, "oversampling leaves no mode on some axis");
      return apply_window(ctx, ctx->g.win, value);
  }
  return fail(ctx, ENUF_EINVAL, "unknown option");
}

static enuf_status apply_window(enuf_ctx c, int win, double sigma) {
  Geom &g = c->g;
  g.win = win;
  g.sigma = sigma;
  for (int d = 0; d < 3; ++d) g.kept[d] = 2 * (int)std::floor(g.M[d] / (2.0 * sigma) + 1e-9);
  if (win == 1) {
    const int m = g.p / 2 - 1;
    g.gb = 2.0 * sigma * m / ((2.0 * sigma - 1.0) * 3.14159265358979323846);
    g.gib = 1.0 / g.gb;
  } else {
    g.gb = g.gib = 0.0;
  }
  drop_graph(c);
  if (!c->have_ws) return ENUF_OK;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  c->w.nruns = c->nruns;
  e = enuf::launch_init_ws(g, c->w, c->st, c->prec == ENUF_FP64);
  if (e != hipSuccess) return hip_fail(c, e, "workspace initialisation");
  c->have_forward = false;
  return ENUF_OK;
}

enuf_status enuf_set_stream(enuf_ctx ctx, void *stream) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  ctx->st = reinterpret_cast<hipStream_t>(stream);
  return ENUF_OK;
}

static enuf_status read_flags_at(enuf_ctx ctx, int *counts, int32_t *flags, bool clear) {
  hipError_t e = sync_stream(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "synchronize");
  int h[4];
  e = hipMemcpy(h, counts, sizeof(h), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "flag read");
  *flags = h[2];
  if (clear && h[2]) {
    const int zero = 0;
    e = hipMemcpy(counts + 2, &zero, sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "flag clear");
  }
  return ENUF_OK;
}

enuf_status enuf_energy_forces(enuf_ctx ctx, const void *x, const void *q, double *E, void *F, void *phi) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  if (!x || !q || !E) return fail(ctx, ENUF_EINVAL, "x, q and E must not be NULL");
  if (!ctx->have_ws)
    return fail(ctx, ENUF_ESTATE, "no workspace: call enuf_set_workspace or enuf_alloc_workspace first");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  const bool all = phi != nullptr;
  const bool an = ctx->analytic;
  if (ctx->graph) {
    e = run_graph(ctx, x, q, E, F, phi, all, an);
  } else {
    hipEvent_t *ev = nullptr;
    if (ctx->slots > 0) {
      ev = &ctx->ring[(size_t)ctx->next * (enuf::kPhases + 1)];
      ctx->next = (ctx->next + 1) % ctx->slots;
      ctx->recorded = std::min(ctx->recorded + 1, ctx->slots);
    }
    e = forward(ctx, ctx->w, ctx->st, x, q, E, F, phi, all, an, ev);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
  ctx->have_forward = true;
  ctx->last_all_active = all;
  ctx->last_analytic = an;
  ctx->gf = ctx->g;
  ++ctx->token;
  if (ctx->check) {
    int32_t f = 0;
    enuf_status s = read_flags_at(ctx, ctx->w.counts, &f, true);
    if (s != ENUF_OK) return s;
    if (f & 1) return fail(ctx, ENUF_ENONFINITE, "non-finite position or charge (excluded from the sums)");
  }
  return ENUF_OK;
}

enuf_status enuf_energy_forces_noalloc(enuf_ctx ctx, const void *x, const void *q, double *E, void *F,
                                       void *phi) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  if (!x || !q || !E) return fail(ctx, ENUF_EINVAL, "x, q and E must not be NULL");
  const size_t need = layout(ctx->g, real_bytes(ctx), nullptr, nullptr);
  if (need > kScratchBytes)
    return fail(ctx, ENUF_EUNSUPPORTED, "enuf_energy_forces_noalloc: this context needs " + std::to_string(need) +
                                            " bytes of working memory, more than the library's static scratch of " +
                                            std::to_string(kScratchBytes) + " bytes");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  void *base = nullptr;
  e = scratch_address(ctx->device, &base);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipGetSymbolAddress(scratch)");
  // The scratch holds whatever the last call on this GPU left: lay this
  // context's buffers over it and initialise them (tables, run table, cleared
  // counters, flags and energy slots) before the evaluation, on the stream.
  Work w;
  layout(ctx->g, real_bytes(ctx), (char *)base, &w);
  w.nruns = ctx->nruns;
  e = enuf::launch_init_ws(ctx->g, w, ctx->st, ctx->prec == ENUF_FP64);
  if (e != hipSuccess) return hip_fail(ctx, e, "scratch initialisation");
  e = forward(ctx, w, ctx->st, x, q, E, F, phi, phi != nullptr, ctx->analytic, nullptr);
  if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
  if (ctx->check) {
    int32_t f = 0;
    enuf_status s = read_flags_at(ctx, w.counts, &f, true);
    if (s != ENUF_OK) return s;
    if (f & 1) return fail(ctx, ENUF_ENONFINITE, "non-finite position or charge (excluded from the sums)");
  }
  return ENUF_OK;
}

static enuf_status adjoint(enuf_ctx ctx, double grad_E, const double *gdev, void *dEdx, void *dEdq) {
  if (!ctx->have_forward) return fail(ctx, ENUF_ESTATE, "no forward evaluation on this context");
  if (!ctx->last_all_active)
    return fail(ctx, ENUF_ESTATE, "the adjoint needs the forward call made with phi != NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  if (ctx->prec == ENUF_FP64)
    e = enuf::launch_adjoint<double>(ctx->gf, ctx->w, ctx->st, grad_E, (double *)dEdx, (double *)dEdq,
                                     ctx->last_analytic, gdev);
  else
    e = enuf::launch_adjoint<float>(ctx->gf, ctx->w, ctx->st, grad_E, (float *)dEdx, (float *)dEdq,
                                    ctx->last_analytic, gdev);
  if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
  return ENUF_OK;
}

enuf_status enuf_energy_grad(enuf_ctx ctx, double grad_E, void *dEdx, void *dEdq) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  if (!std::isfinite(grad_E)) return fail(ctx, ENUF_EINVAL, "grad_E must be finite");
  return adjoint(ctx, grad_E, nullptr, dEdx, dEdq);
}

enuf_status enuf_eval_token(enuf_ctx ctx, uint64_t *token) {
  if (!ctx || !token) return fail(ctx, ENUF_EINVAL, "ctx or token is NULL");
  *token = ctx->token;
  return ENUF_OK;
}

enuf_status enuf_energy_grad_dev(enuf_ctx ctx, uint64_t token, const double *grad_E, void *dEdx, void *dEdq) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  if (!grad_E) return fail(ctx, ENUF_EINVAL, "grad_E is NULL");
  if (!ctx->have_forward || token != ctx->token)
    return fail(ctx, ENUF_ESTATE, "the evaluation this gradient belongs to is no longer the context's last one");
  return adjoint(ctx, 1.0, grad_E, dEdx, dEdq);
}

enuf_status enuf_get_flags(enuf_ctx ctx, int32_t *flags) {
  if (!ctx || !flags) return fail(ctx, ENUF_EINVAL, "ctx or flags is NULL");
  if (!ctx->have_ws) return fail(ctx, ENUF_ESTATE, "no workspace");
  return read_flags_at(ctx, ctx->w.counts, flags, true);
}

enuf_status enuf_stage_bytes(enuf_ctx ctx, int32_t stage, size_t *bytes) {
  if (!ctx || !bytes) return fail(ctx, ENUF_EINVAL, "ctx or bytes is NULL");
  const size_t rs = real_bytes(ctx);
  const size_t G = (size_t)ctx->g.M[0] * ctx->g.M[1] * ctx->g.M[2];
  switch (stage) {
    case ENUF_STAGE_GRID: *bytes = G * rs; return ENUF_OK;
    case ENUF_STAGE_SPECTRUM: *bytes = G / 2 * 2 * rs; return ENUF_OK;
    case ENUF_STAGE_FIELDS: *bytes = G * (ctx->last_analytic ? 1 : 4) * rs; return ENUF_OK;
    case ENUF_STAGE_SORTED: *bytes = (size_t)ctx->g.n * 4; return ENUF_OK;
    case ENUF_STAGE_COUNTS: *bytes = 8 * 4; return ENUF_OK;
    case ENUF_STAGE_CELLS: *bytes = (size_t)ctx->g.n * 4; return ENUF_OK;
  }
  return fail(ctx, ENUF_EINVAL, "unknown stage");
}

enuf_status enuf_stage_copy(enuf_ctx ctx, int32_t stage, void *dst, size_t bytes) {
  if (!ctx || !dst) return fail(ctx, ENUF_EINVAL, "ctx or dst is NULL");
  size_t need = 0;
  enuf_status s = enuf_stage_bytes(ctx, stage, &need);
  if (s != ENUF_OK) return s;
  if (bytes < need) return fail(ctx, ENUF_EINVAL, "destination too small");
  if (!ctx->have_forward) return fail(ctx, ENUF_ESTATE, "no forward evaluation on this context");
  const void *src = nullptr;
  switch (stage) {
    case ENUF_STAGE_GRID: src = ctx->w.grid; break;
    case ENUF_STAGE_SPECTRUM: src = ctx->w.spec; break;
    case ENUF_STAGE_FIELDS: src = ctx->w.field; break;
    case ENUF_STAGE_SORTED: src = ctx->w.perm_t; break;
    case ENUF_STAGE_COUNTS: src = ctx->w.counts; break;
    case ENUF_STAGE_CELLS: src = ctx->w.perm_c; break;
  }
  hipError_t e = sync_stream(ctx);
  if (e == hipSuccess) e = hipMemcpy(dst, src, need, hipMemcpyDeviceToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "stage copy");
  return ENUF_OK;
}

enuf_status enuf_get_timings(enuf_ctx ctx, double *ms, int32_t n, int32_t *count) {
  if (!ctx || !ms || !count) return fail(ctx, ENUF_EINVAL, "NULL argument");
  if (ctx->graph) return fail(ctx, ENUF_ESTATE, "per-phase timing is not recorded in graph mode");
  if (ctx->slots == 0 || ctx->recorded == 0) return fail(ctx, ENUF_ESTATE, "timing is off or nothing ran");
  hipError_t e = sync_stream(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "synchronize");
  double acc[enuf::kPhases] = {0};
  for (int k = 0; k < ctx->recorded; ++k) {
    const int slot = (ctx->next - 1 - k + 2 * ctx->slots) % ctx->slots;
    hipEvent_t *ev = &ctx->ring[(size_t)slot * (enuf::kPhases + 1)];
    for (int i = 0; i < enuf::kPhases; ++i) {
      float t = 0.f;
      e = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
      if (e != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
      acc[i] += t;
    }
  }
  *count = enuf::kPhases;
  for (int i = 0; i < enuf::kPhases && i < n; ++i) ms[i] = acc[i] / ctx->recorded;
  ctx->recorded = 0;
  return ENUF_OK;
}

enuf_status enuf_get_step_timings(enuf_ctx ctx, double *ms, int32_t cap, int32_t *count) {
  if (!ctx || !ms || !count) return fail(ctx, ENUF_EINVAL, "NULL argument");
  if (ctx->graph) return fail(ctx, ENUF_ESTATE, "per-phase timing is not recorded in graph mode");
  if (ctx->slots == 0 || ctx->recorded == 0) return fail(ctx, ENUF_ESTATE, "timing is off or nothing ran");
  hipError_t e = sync_stream(ctx);
  if (e != hipSuccess) return hip_fail(ctx, e, "synchronize");
  const int nrec = std::min(ctx->recorded, (int)std::max(0, cap));
  // oldest first
  for (int k = 0; k < nrec; ++k) {
    const int slot = (ctx->next - ctx->recorded + k + 2 * ctx->slots) % ctx->slots;
    hipEvent_t *ev = &ctx->ring[(size_t)slot * (enuf::kPhases + 1)];
    for (int i = 0; i < enuf::kPhases; ++i) {
      float t = 0.f;
      e = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
      if (e != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
      ms[(size_t)k * enuf::kPhases + i] = t;
    }
  }
  *count = nrec;
  ctx->recorded = 0;
  return ENUF_OK;
}

}  // extern "C"
