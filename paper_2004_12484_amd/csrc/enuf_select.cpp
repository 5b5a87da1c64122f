// enuf_select.cpp -- enuf_select_params (include/enuf.h): ENUF parameters for
// a target RMS force error, from the paper's error relations (Eq. 31-32 with
// the reciprocal-cutoff iteration of Sec. 2.3.2) or from the trained
// parameter network evaluated by the MLP forward kernel (enuf_mlp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "enuf.h"
#include "enuf_mlp.h"

namespace {

constexpr int kMMin = 8, kMMax = 512;

thread_local std::string g_select_err;

enuf_status sel_fail(enuf_status s, const std::string &m) {
  g_select_err = m;
  return s;
}

int pow2_ceil_exp(double v) { return (int)std::ceil(v - 1e-6); }

int clamp_grid(double log2m) {
  const double m = std::ldexp(1.0, pow2_ceil_exp(log2m));
  return (int)std::min<double>(kMMax, std::max<double>(kMMin, m));
}

// largest of 8, 6, 4, 2 not above p0 with 2p <= M on every axis
int fit_window(int p0, const int32_t M[3]) {
  int p = p0;
  while (p > 2 && (2 * p > M[0] || 2 * p > M[1] || 2 * p > M[2])) p -= 2;
  return p;
}

// The paper's relations at equality for the target delta (Sec. 2.3.2):
// Eq. 31, exp(-pi^2 n_c^2 / (alpha L)^2) = delta, gives alpha from the
// reciprocal cutoff n_c; Eq. 32, exp(-alpha^2 r_c^2) = delta (the leading
// behaviour of erfc), gives r_c.  n_c is raised from 2 until r_c fits the
// short-range cutoff of 3 mean spacings (and the minimum-image bound); the
// grid keeps every mode up to n_c on each axis, p = 6.
void heuristic(const double box[3], int64_t n, double target, double *alpha, double *rc, int32_t M[3],
               int32_t *p) {
  const double V = box[0] * box[1] * box[2];
  const double a = std::cbrt(V / (double)n);
  const double L = box[0];
  const double s = std::sqrt(-std::log(target));
  const double lmin = std::min(box[0], std::min(box[1], box[2]));
  double al = 0.0, r = 0.0;
  int nc = 2;
  for (; nc < 512; ++nc) {
    al = M_PI * nc / (L * s);
    r = s / al;
    if (r <= std::min(3.0 * a, 0.5 * lmin)) break;
  }
  if (nc == 512) nc = 511;
  for (int d = 0; d < 3; ++d) {
    const double m = std::ldexp(1.0, (int)std::ceil(std::log2(2.0 * nc * box[d] / L + 2.0)));
    M[d] = (int)std::min<double>(kMMax, std::max<double>(kMMin, m));
  }
  *alpha = al;
  *rc = r;
  *p = fit_window(6, M);
}

// The network file: the little-endian binary the training script writes.
//   char[8] "ENUFMLP1"; int32 n_in, n_hidden, n_layers, n_out;
//   double x_mean[n_in], x_std[n_in], y_mean[n_out], y_std[n_out];
//   double range[8] = N lo/hi, density lo/hi, charged fraction lo/hi,
//                     target lo/hi of the training systems;
//   int32 n_shapes; double shapes[n_shapes][2] = (Ly/Lx, Lz/Lx) trained on;
//   int64 n_params; float params[n_params] (enuf_mlp.h layout).
struct Net {
  enuf_mlp_shape shape{};
  std::vector<double> xm, xs, ym, ys, shapes;
  double range[8] = {0};
  std::vector<float> params;
};

enuf_status read_net(const char *path, Net *net) {
  FILE *f = std::fopen(path, "rb");
  if (!f) return sel_fail(ENUF_EINVAL, std::string("cannot open network file ") + path);
  bool ok = true;
  auto rd = [&](void *dst, size_t bytes) {
    if (ok && std::fread(dst, 1, bytes, f) != bytes) ok = false;
  };
  char magic[8] = {0};
  rd(magic, 8);
  ok = ok && std::memcmp(magic, "ENUFMLP1", 8) == 0;
  int32_t dims[4] = {0, 0, 0, 0};
  rd(dims, sizeof(dims));
  net->shape = enuf_mlp_shape{dims[0], dims[1], dims[2], dims[3]};
  const int64_t count = ok ? enuf_mlp_param_count(&net->shape) : -1;
  ok = ok && count > 0 && dims[0] == 5 && dims[3] == 6;
  if (ok) {
    net->xm.resize(5);
    net->xs.resize(5);
    net->ym.resize(6);
    net->ys.resize(6);
  }
  rd(net->xm.data(), 5 * sizeof(double));
  rd(net->xs.data(), 5 * sizeof(double));
  rd(net->ym.data(), 6 * sizeof(double));
  rd(net->ys.data(), 6 * sizeof(double));
  rd(net->range, sizeof(net->range));
  int32_t ns = 0;
  rd(&ns, sizeof(ns));
  ok = ok && ns >= 0 && ns <= 64;
  if (ok) net->shapes.resize(2 * (size_t)ns);
  rd(net->shapes.data(), net->shapes.size() * sizeof(double));
  int64_t np = 0;
  rd(&np, sizeof(np));
  ok = ok && np == count;
  if (ok) net->params.resize((size_t)np);
  rd(net->params.data(), net->params.size() * sizeof(float));
  std::fclose(f);
  if (!ok) return sel_fail(ENUF_EINVAL, std::string("malformed network file ") + path);
  return ENUF_OK;
}

bool in_range(const Net &net, const double box[3], int64_t n, double fq, double target) {
  const double rho = (double)n / (box[0] * box[1] * box[2]);
  const double *r = net.range;
  if (!(n >= r[0] && n <= r[1] && rho >= r[2] && rho <= r[3] && fq >= r[4] && fq <= r[5] && target >= r[6] &&
        target <= r[7]))
    return false;
  for (size_t k = 0; k + 1 < net.shapes.size(); k += 2)
    if (std::fabs(box[1] / box[0] - net.shapes[k]) < 1e-6 && std::fabs(box[2] / box[0] - net.shapes[k + 1]) < 1e-6)
      return true;
  return false;
}

// Network prediction, (alpha a, log2 M per axis, p, r_c / a) with a the mean
// spacing, evaluated by the MLP forward kernel, then snapped to a valid
// setting: M a power of two in [8, 512] (rounded up), p the nearest of 4, 6,
// 8 that fits, r_c within the minimum-image bound.
enuf_status predict(const Net &net, const double box[3], int64_t n, double fq, double target, double *alpha,
                    double *rc, int32_t M[3], int32_t *p) {
  const double feat[5] = {std::log10((double)n), box[1] / box[0], box[2] / box[0], fq, std::log10(target)};
  float xin[5];
  for (int k = 0; k < 5; ++k) xin[k] = (float)((feat[k] - net.xm[k]) / net.xs[k]);
  const size_t pbytes = net.params.size() * sizeof(float);
  char *dev = nullptr;
  hipError_t e = hipMalloc((void **)&dev, pbytes + 256 + 64);
  if (e != hipSuccess)
    return sel_fail(e == hipErrorOutOfMemory ? ENUF_ENOMEM : ENUF_EDEVICE,
                    std::string("device buffer for the network: ") + hipGetErrorString(e));
  float *dp = (float *)dev;
  float *dx = (float *)(dev + ((pbytes + 255) / 256) * 256);
  float *dy = dx + 8;
  float yout[6];
  enuf_status st = ENUF_OK;
  e = hipMemcpy(dp, net.params.data(), pbytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dx, xin, sizeof(xin), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    st = enuf_mlp_forward(&net.shape, dp, 1, dx, dy, nullptr, nullptr);
    if (st == ENUF_OK) e = hipMemcpy(yout, dy, sizeof(yout), hipMemcpyDeviceToHost);
  }
  (void)hipFree(dev);
  if (st != ENUF_OK) return sel_fail(st, "network forward pass");
  if (e != hipSuccess) return sel_fail(ENUF_EDEVICE, std::string("network evaluation: ") + hipGetErrorString(e));
  double y[6];
  for (int k = 0; k < 6; ++k) y[k] = (double)yout[k] * net.ys[k] + net.ym[k];
  const double a = std::cbrt(box[0] * box[1] * box[2] / (double)n);
  const double lmin = std::min(box[0], std::min(box[1], box[2]));
  for (int d = 0; d < 3; ++d) M[d] = clamp_grid(y[1 + d]);
  int pp = 4;
  for (int c : {6, 8})
    if (std::fabs(c - y[4]) < std::fabs(pp - y[4])) pp = c;
  *p = fit_window(pp, M);
  *alpha = y[0] / a;
  *rc = std::min(y[5] * a, 0.5 * lmin);
  return ENUF_OK;
}

}  // namespace

extern "C" {

enuf_status enuf_select_params(const double box[3], int64_t n, double charged_frac, double target_rms_err,
                               const char *model_path, double *alpha, double *r_c, int32_t M[3], int32_t *p,
                               int32_t *method) {
  if (!box || !alpha || !r_c || !M || !p) return sel_fail(ENUF_EINVAL, "NULL argument");
  for (int d = 0; d < 3; ++d)
    if (!(box[d] > 0.0) || !std::isfinite(box[d])) return sel_fail(ENUF_EINVAL, "box lengths must be > 0");
  if (n < 2) return sel_fail(ENUF_EINVAL, "n must be >= 2");
  if (!(charged_frac > 0.0 && charged_frac <= 1.0)) return sel_fail(ENUF_EINVAL, "charged_frac must be in (0, 1]");
  if (!(target_rms_err > 0.0 && target_rms_err < 1.0)) return sel_fail(ENUF_EINVAL, "target must be in (0, 1)");
  if (model_path) {
    Net net;
    enuf_status st = read_net(model_path, &net);
    if (st != ENUF_OK) return st;
    if (in_range(net, box, n, charged_frac, target_rms_err)) {
      st = predict(net, box, n, charged_frac, target_rms_err, alpha, r_c, M, p);
      if (st != ENUF_OK) return st;
      if (method) *method = ENUF_SELECT_NETWORK;
      return ENUF_OK;
    }
  }
  heuristic(box, n, target_rms_err, alpha, r_c, M, p);
  if (method) *method = ENUF_SELECT_HEURISTIC;
  return ENUF_OK;
}

const char *enuf_select_last_error(void) { return g_select_err.c_str(); }

}  // extern "C"
