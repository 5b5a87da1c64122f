// enuf_api.cpp -- host side of the ENUF C ABI (include/enuf.h): parameter
// validation, workspace ownership, stream binding and the launch sequences.
#include "enuf.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "enuf_internal.h"

using enuf::Geom;
using enuf::Work;

struct enuf_ctx_s {
  Geom g{};
  Work w{};
  int prec = ENUF_FP64;
  hipStream_t st = nullptr;
  int device = 0;
  bool have_forward = false;
  bool last_all_active = false;
  bool check = false;
  bool analytic = false;       // ENUF_OPT_FORCE_MODE = 1
  bool last_analytic = false;  // the last forward left psi as a plain real grid
  // timing ring: `slots` evaluations x (kPhases + 1) events
  std::vector<hipEvent_t> ring;
  int slots = 0, next = 0, recorded = 0;
  std::string err;
  std::vector<void *> allocs;
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

static void free_all(enuf_ctx c) {
  for (void *p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  for (auto &e : c->ring) (void)hipEventDestroy(e);
  c->ring.clear();
  c->slots = c->next = c->recorded = 0;
}

template <typename T>
static hipError_t dalloc(enuf_ctx c, T **p, size_t count) {
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T) + 256);
  if (e != hipSuccess) return e;
  c->allocs.push_back(q);
  *p = reinterpret_cast<T *>(q);
  return hipSuccess;
}

extern "C" {

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

  enuf_ctx c = new (std::nothrow) enuf_ctx_s();
  if (!c) return fail(nullptr, ENUF_ENOMEM, "host allocation failed");
  Geom &g = c->g;
  const int tdef[3] = {enuf::kTileX, enuf::kTileY, enuf::kTileZ};
  for (int d = 0; d < 3; ++d) {
    g.M[d] = M[d];
    g.T[d] = std::min(tdef[d], M[d] / 2);
    g.nt[d] = M[d] / g.T[d];
    g.L[d] = box[d];
    int nc = (int)std::floor(box[d] / (r_c * (1.0 + 1e-5)));
    g.nc[d] = std::max(1, std::min(nc, 1024));
  }
  while ((int64_t)g.nc[0] * g.nc[1] * g.nc[2] > (int64_t(1) << 22)) {
    int dm = 0;
    for (int d = 1; d < 3; ++d) if (g.nc[d] > g.nc[dm]) dm = d;
    g.nc[dm] = std::max(1, g.nc[dm] / 2);
  }
  for (int d = 0; d < 3; ++d) {
    g.iL[d] = 1.0 / g.L[d];
    g.mL[d] = g.M[d] / g.L[d];
    g.cL[d] = g.nc[d] / g.L[d];
  }
  g.ntiles = g.nt[0] * g.nt[1] * g.nt[2];
  g.ncells = g.nc[0] * g.nc[1] * g.nc[2];
  g.p = p;
  g.n = (int)n;
  g.alpha = alpha;
  g.rc = r_c;
  g.ke = 1.0;
  g.slater = 0.0;
  c->prec = precision;
  c->st = reinterpret_cast<hipStream_t>(stream);

  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    enuf_status s = hip_fail(nullptr, e, "hipGetDevice");
    delete c;
    return s;
  }
  const size_t rs = precision == ENUF_FP64 ? 8 : 4;
  const size_t G = (size_t)M[0] * M[1] * M[2];
  Work &w = c->w;
  unsigned char *bytes = nullptr;
  auto need = [&](hipError_t err) -> bool { return err == hipSuccess; };
  bool ok = true;
  ok = ok && need(dalloc(c, (unsigned char **)&w.part_t, (size_t)n * 4 * rs));
  ok = ok && need(dalloc(c, (unsigned char **)&w.part_c, (size_t)n * 4 * rs));
  ok = ok && need(dalloc(c, &w.perm_t, (size_t)n));
  ok = ok && need(dalloc(c, &w.perm_c, (size_t)n));
  const enuf::SortPlan sp = enuf::sort_plan(g, (int)rs);
  const size_t nbk = (size_t)sp.nb[0] + sp.nb[1];
  if (!enuf::fft_plans_fit(g, precision == ENUF_FP64)) {
    delete c;
    return fail(nullptr, ENUF_EUNSUPPORTED, "grid transform does not fit one workgroup's LDS");
  }
  if (nbk * sizeof(int) > 65536 || enuf::sort_stage_lds(sp, (int)rs) > 65536 || enuf::sort_fine_lds(sp) > 65536) {
    delete c;
    return fail(nullptr, ENUF_EUNSUPPORTED, "too many sort buckets for one workgroup's LDS");
  }
  ok = ok && need(dalloc(c, &w.key_t, (size_t)n));
  ok = ok && need(dalloc(c, &w.key_c, (size_t)n));
  ok = ok && need(dalloc(c, &w.off_t, (size_t)sp.nbins[0] + 1));
  ok = ok && need(dalloc(c, &w.off_c, (size_t)sp.nbins[1] + 1));
  ok = ok && need(dalloc(c, &w.hist, (size_t)sp.nblk * nbk));
  ok = ok && need(dalloc(c, &w.bbase, nbk + 2));
  ok = ok && need(dalloc(c, (unsigned char **)&w.stg_t, (size_t)n * 4 * rs));
  ok = ok && need(dalloc(c, (unsigned char **)&w.stg_c, (size_t)n * 4 * rs));
  ok = ok && need(dalloc(c, &w.ik_t, (size_t)n));
  ok = ok && need(dalloc(c, &w.ik_c, (size_t)n));
  ok = ok && need(dalloc(c, &w.runs, (size_t)5 * enuf::kMaxRuns));
  ok = ok && need(dalloc(c, &w.counts, 4));
  ok = ok && need(dalloc(c, &w.scal, 4));
  ok = ok && need(dalloc(c, &w.qpart, (size_t)4 * sp.nblk));
  ok = ok && need(dalloc(c, &w.eslot, (size_t)2 * enuf::kESlots));
  ok = ok && need(dalloc(c, (unsigned char **)&w.grid, G * rs));
  ok = ok && need(dalloc(c, (unsigned char **)&w.spec, G / 2 * 2 * rs));
  ok = ok && need(dalloc(c, (unsigned char **)&w.fspec, 4 * (G / 2) * 2 * rs));
  ok = ok && need(dalloc(c, (unsigned char **)&w.field, G * 4 * rs));
  size_t ntab = enuf::table_size(g, w.tab_off);
  ok = ok && need(dalloc(c, (unsigned char **)&w.tables, ntab * rs));
  (void)bytes;
  if (!ok || std::getenv("ENUF_FAIL_ALLOC")) {
    free_all(c);
    delete c;
    return fail(nullptr, ENUF_ENOMEM, "device workspace allocation failed");
  }
  // tables
  std::vector<unsigned char> host(ntab * rs);
  if (precision == ENUF_FP64) enuf::fill_tables<double>(g, w.tab_off, (double *)host.data());
  else enuf::fill_tables<float>(g, w.tab_off, (float *)host.data());
  int runs[5 * enuf::kMaxRuns];
  w.nruns = enuf::build_runs(g, runs);
  if (w.nruns <= 0) {
    free_all(c);
    delete c;
    return fail(nullptr, ENUF_EUNSUPPORTED, "spread run table overflow");
  }
  e = hipMemcpy(w.tables, host.data(), ntab * rs, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(w.runs, runs, sizeof(int) * 5 * w.nruns, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(w.counts, 0, 4 * sizeof(int));
  if (e == hipSuccess) e = hipMemset(w.eslot, 0, 2 * enuf::kESlots * sizeof(double));
  if (e != hipSuccess) {
    enuf_status s = hip_fail(nullptr, e, "workspace initialisation");
    free_all(c);
    delete c;
    return s;
  }
  *out = c;
  return ENUF_OK;
}

enuf_status enuf_destroy(enuf_ctx ctx) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  (void)hipSetDevice(ctx->device);
  if (ctx->st) (void)hipStreamSynchronize(ctx->st);
  else (void)hipDeviceSynchronize();
  free_all(ctx);
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
    case ENUF_OPT_GRAPH:
      if (value != 0.0 && value != 1.0) return fail(ctx, ENUF_EINVAL, "graph is 0 or 1");
      if (value == 1.0) return fail(ctx, ENUF_EUNSUPPORTED, "graph replay is not available in this library");
      return ENUF_OK;
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
  }
  return fail(ctx, ENUF_EINVAL, "unknown option");
}

enuf_status enuf_set_stream(enuf_ctx ctx, void *stream) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  ctx->st = reinterpret_cast<hipStream_t>(stream);
  return ENUF_OK;
}

static enuf_status read_flags(enuf_ctx ctx, int32_t *flags, bool clear) {
  hipError_t e = ctx->st ? hipStreamSynchronize(ctx->st) : hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(ctx, e, "synchronize");
  int h[4];
  e = hipMemcpy(h, ctx->w.counts, sizeof(h), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "flag read");
  *flags = h[2];
  if (clear && h[2]) {
    e = hipMemset(ctx->w.counts + 2, 0, sizeof(int));
    if (e != hipSuccess) return hip_fail(ctx, e, "flag clear");
  }
  return ENUF_OK;
}

enuf_status enuf_energy_forces(enuf_ctx ctx, const void *x, const void *q, double *E, void *F, void *phi) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  if (!x || !q || !E) return fail(ctx, ENUF_EINVAL, "x, q and E must not be NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  const bool all = phi != nullptr;
  hipEvent_t *ev = nullptr;
  if (ctx->slots > 0) {
    ev = &ctx->ring[(size_t)ctx->next * (enuf::kPhases + 1)];
    ctx->next = (ctx->next + 1) % ctx->slots;
    ctx->recorded = std::min(ctx->recorded + 1, ctx->slots);
  }
  const bool an = ctx->analytic;
  if (ctx->prec == ENUF_FP64)
    e = enuf::launch_forward<double>(ctx->g, ctx->w, ctx->st, (const double *)x, (const double *)q, E,
                                     (double *)F, (double *)phi, all, all, an, ev);
  else
    e = enuf::launch_forward<float>(ctx->g, ctx->w, ctx->st, (const float *)x, (const float *)q, E,
                                    (float *)F, (float *)phi, all, all, an, ev);
  if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
  ctx->have_forward = true;
  ctx->last_all_active = all;
  ctx->last_analytic = an;
  if (ctx->check) {
    int32_t f = 0;
    enuf_status s = read_flags(ctx, &f, true);
    if (s != ENUF_OK) return s;
    if (f & 1) return fail(ctx, ENUF_ENONFINITE, "non-finite position or charge (excluded from the sums)");
  }
  return ENUF_OK;
}

enuf_status enuf_energy_grad(enuf_ctx ctx, double grad_E, void *dEdx, void *dEdq) {
  if (!ctx) return fail(nullptr, ENUF_EINVAL, "ctx is NULL");
  if (!std::isfinite(grad_E)) return fail(ctx, ENUF_EINVAL, "grad_E must be finite");
  if (!ctx->have_forward) return fail(ctx, ENUF_ESTATE, "no forward evaluation on this context");
  if (!ctx->last_all_active)
    return fail(ctx, ENUF_ESTATE, "the adjoint needs the forward call made with phi != NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  if (ctx->prec == ENUF_FP64)
    e = enuf::launch_adjoint<double>(ctx->g, ctx->w, ctx->st, grad_E, (double *)dEdx, (double *)dEdq,
                                     ctx->last_analytic);
  else
    e = enuf::launch_adjoint<float>(ctx->g, ctx->w, ctx->st, grad_E, (float *)dEdx, (float *)dEdq,
                                    ctx->last_analytic);
  if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
  return ENUF_OK;
}

enuf_status enuf_get_flags(enuf_ctx ctx, int32_t *flags) {
  if (!ctx || !flags) return fail(ctx, ENUF_EINVAL, "ctx or flags is NULL");
  return read_flags(ctx, flags, true);
}

enuf_status enuf_stage_bytes(enuf_ctx ctx, int32_t stage, size_t *bytes) {
  if (!ctx || !bytes) return fail(ctx, ENUF_EINVAL, "ctx or bytes is NULL");
  const size_t rs = ctx->prec == ENUF_FP64 ? 8 : 4;
  const size_t G = (size_t)ctx->g.M[0] * ctx->g.M[1] * ctx->g.M[2];
  switch (stage) {
    case ENUF_STAGE_GRID: *bytes = G * rs; return ENUF_OK;
    case ENUF_STAGE_SPECTRUM: *bytes = G / 2 * 2 * rs; return ENUF_OK;
    case ENUF_STAGE_FIELDS: *bytes = G * (ctx->last_analytic ? 1 : 4) * rs; return ENUF_OK;
    case ENUF_STAGE_SORTED: *bytes = (size_t)ctx->g.n * 4; return ENUF_OK;
    case ENUF_STAGE_COUNTS: *bytes = 2 * 4; return ENUF_OK;
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
  hipError_t e = ctx->st ? hipStreamSynchronize(ctx->st) : hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(dst, src, need, hipMemcpyDeviceToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "stage copy");
  return ENUF_OK;
}

enuf_status enuf_get_timings(enuf_ctx ctx, double *ms, int32_t n, int32_t *count) {
  if (!ctx || !ms || !count) return fail(ctx, ENUF_EINVAL, "NULL argument");
  if (ctx->slots == 0 || ctx->recorded == 0) return fail(ctx, ENUF_ESTATE, "timing is off or nothing ran");
  hipError_t e = ctx->st ? hipStreamSynchronize(ctx->st) : hipDeviceSynchronize();
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

}  // extern "C"
