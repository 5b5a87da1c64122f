// enuf_mlp.hip -- forward, loss, backward and Adam kernels of the parameter
// predictor (include/enuf_mlp.h).  The network is tiny (~9k parameters), so
// plain VALU dot products with activations staged in LDS are used; the
// per-block partial gradients are summed by a second kernel (no atomics).
#include <hip/hip_runtime.h>

#include <cmath>

#include "enuf_mlp.h"

namespace {

constexpr int kMlpBlock = 256;
constexpr int kMlpSamples = 32;   // samples per block
constexpr int kMlpMaxWidth = 128; // max(n_in, n_hidden, n_out)

bool shape_ok(const enuf_mlp_shape *s) {
  return s && s->n_in >= 1 && s->n_in <= 64 && s->n_out >= 1 && s->n_out <= 64 && s->n_hidden >= 1 &&
         s->n_hidden <= kMlpMaxWidth && s->n_layers >= 1 && s->n_layers <= 8;
}

struct Shape {
  int n_in, H, nl, n_out;
  __host__ __device__ int in_of(int l) const { return l == 0 ? n_in : H; }
  __host__ __device__ int out_of(int l) const { return l == nl ? n_out : H; }
  // float offset of layer l's weights in the parameter array
  __host__ __device__ long off(int l) const {
    long o = 0;
    for (int k = 0; k < l; ++k) o += (long)out_of(k) * in_of(k) + out_of(k);
    return o;
  }
  __host__ __device__ long count() const { return off(nl + 1); }
  __host__ __device__ int cache() const { return nl * H; }
};

Shape mk(const enuf_mlp_shape *s) { return Shape{s->n_in, s->n_hidden, s->n_layers, s->n_out}; }

__global__ __launch_bounds__(kMlpBlock) void k_mlp_fwd(Shape sh, const float *__restrict__ P, long B,
                                                       const float *__restrict__ x, float *__restrict__ y,
                                                       float *__restrict__ cache) {
  __shared__ float buf[2][kMlpSamples][kMlpMaxWidth];
  const long s0 = (long)blockIdx.x * kMlpSamples;
  for (int e = threadIdx.x; e < kMlpSamples * sh.n_in; e += blockDim.x) {
    const int s = e / sh.n_in, k = e % sh.n_in;
    buf[0][s][k] = (s0 + s < B) ? x[(s0 + s) * sh.n_in + k] : 0.f;
  }
  __syncthreads();
  int cur = 0;
  for (int l = 0; l <= sh.nl; ++l) {
    const int in = sh.in_of(l), out = sh.out_of(l);
    const float *W = P + sh.off(l);
    const float *b = W + (long)out * in;
    for (int e = threadIdx.x; e < kMlpSamples * out; e += blockDim.x) {
      const int s = e / out, j = e % out;
      float z = b[j];
      const float *wr = W + (long)j * in;
      for (int k = 0; k < in; ++k) z += wr[k] * buf[cur][s][k];
      const float a = (l < sh.nl) ? tanhf(z) : z;
      buf[cur ^ 1][s][j] = a;
      if (s0 + s < B) {
        if (l < sh.nl) {
          if (cache) cache[(s0 + s) * sh.cache() + l * sh.H + j] = a;
        } else {
          y[(s0 + s) * sh.n_out + j] = a;
        }
      }
    }
    __syncthreads();
    cur ^= 1;
  }
}

__global__ __launch_bounds__(kMlpBlock) void k_mlp_bwd(Shape sh, const float *__restrict__ P, long B,
                                                       const float *__restrict__ x,
                                                       const float *__restrict__ cache,
                                                       const float *__restrict__ dy, float *__restrict__ gpart) {
  __shared__ float dz[2][kMlpSamples][kMlpMaxWidth];
  __shared__ float ain[kMlpSamples][kMlpMaxWidth];
  const long s0 = (long)blockIdx.x * kMlpSamples;
  float *gp = gpart + (long)blockIdx.x * sh.count();
  for (int e = threadIdx.x; e < kMlpSamples * sh.n_out; e += blockDim.x) {
    const int s = e / sh.n_out, j = e % sh.n_out;
    dz[0][s][j] = (s0 + s < B) ? dy[(s0 + s) * sh.n_out + j] : 0.f;
  }
  int cur = 0;
  for (int l = sh.nl; l >= 0; --l) {
    const int in = sh.in_of(l), out = sh.out_of(l);
    const float *W = P + sh.off(l);
    // inputs of layer l: x for l == 0, else the activations of hidden layer l-1
    for (int e = threadIdx.x; e < kMlpSamples * in; e += blockDim.x) {
      const int s = e / in, k = e % in;
      float a = 0.f;
      if (s0 + s < B) a = (l == 0) ? x[(s0 + s) * sh.n_in + k] : cache[(s0 + s) * sh.cache() + (l - 1) * sh.H + k];
      ain[s][k] = a;
    }
    __syncthreads();
    // weight and bias gradients of this block's samples
    float *gW = gp + sh.off(l);
    for (int e = threadIdx.x; e < out * in; e += blockDim.x) {
      const int j = e / in, k = e % in;
      float acc = 0.f;
      for (int s = 0; s < kMlpSamples; ++s) acc += dz[cur][s][j] * ain[s][k];
      gW[e] = acc;
    }
    for (int j = threadIdx.x; j < out; j += blockDim.x) {
      float acc = 0.f;
      for (int s = 0; s < kMlpSamples; ++s) acc += dz[cur][s][j];
      gW[(long)out * in + j] = acc;
    }
    // back through W and the tanh of the previous layer
    if (l > 0) {
      for (int e = threadIdx.x; e < kMlpSamples * in; e += blockDim.x) {
        const int s = e / in, k = e % in;
        float acc = 0.f;
        for (int j = 0; j < out; ++j) acc += W[(long)j * in + k] * dz[cur][s][j];
        const float a = ain[s][k];
        dz[cur ^ 1][s][k] = acc * (1.f - a * a);
      }
    }
    __syncthreads();
    cur ^= 1;
  }
}

__global__ __launch_bounds__(kMlpBlock) void k_mlp_reduce(const float *__restrict__ gpart, long nblk, long np,
                                                          float *__restrict__ grad) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  float acc = 0.f;
  for (long b = 0; b < nblk; ++b) acc += gpart[b * np + p];
  grad[p] = acc;
}

__global__ __launch_bounds__(1024) void k_mlp_loss(long n, int n_out, long B, const float *__restrict__ y,
                                                   const float *__restrict__ t, const float *__restrict__ w,
                                                   float *__restrict__ dy, double *loss) {
  __shared__ double red[16];
  double acc = 0.0;
  for (long e = threadIdx.x; e < n; e += blockDim.x) {
    const int o = (int)(e % n_out);
    const float d = y[e] - t[e];
    dy[e] = 2.f * w[o] * d / (float)B;
    acc += (double)w[o] * (double)d * (double)d;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    *loss = s / (double)B;
  }
}

__global__ __launch_bounds__(kMlpBlock) void k_mlp_adam(long n, float *__restrict__ p, const float *__restrict__ g,
                                                        float *__restrict__ m, float *__restrict__ v, float lr,
                                                        float b1, float b2, float eps, float c1, float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

enuf_status launched() { return hipGetLastError() == hipSuccess ? ENUF_OK : ENUF_EDEVICE; }

}  // namespace

extern "C" {

int64_t enuf_mlp_param_count(const enuf_mlp_shape *shape) {
  if (!shape_ok(shape)) return -1;
  return mk(shape).count();
}

int64_t enuf_mlp_cache_count(const enuf_mlp_shape *shape) {
  if (!shape_ok(shape)) return -1;
  return mk(shape).cache();
}

enuf_status enuf_mlp_forward(const enuf_mlp_shape *shape, const float *params, int64_t batch, const float *x,
                             float *y, float *cache, void *stream) {
  if (!shape_ok(shape) || !params || batch < 1 || !x || !y) return ENUF_EINVAL;
  const long nblk = (batch + kMlpSamples - 1) / kMlpSamples;
  hipLaunchKernelGGL(k_mlp_fwd, dim3(nblk), dim3(kMlpBlock), 0, (hipStream_t)stream, mk(shape), params,
                     (long)batch, x, y, cache);
  return launched();
}

enuf_status enuf_mlp_loss(const enuf_mlp_shape *shape, int64_t batch, const float *y, const float *target,
                          const float *w, float *dy, double *loss, void *stream) {
  if (!shape_ok(shape) || batch < 1 || !y || !target || !w || !dy || !loss) return ENUF_EINVAL;
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(1024), 0, (hipStream_t)stream, (long)batch * shape->n_out,
                     shape->n_out, (long)batch, y, target, w, dy, loss);
  return launched();
}

size_t enuf_mlp_workspace_bytes(const enuf_mlp_shape *shape, int64_t batch) {
  if (!shape_ok(shape) || batch < 1) return 0;
  const long nblk = (batch + kMlpSamples - 1) / kMlpSamples;
  return (size_t)nblk * (size_t)mk(shape).count() * sizeof(float);
}

enuf_status enuf_mlp_backward(const enuf_mlp_shape *shape, const float *params, int64_t batch, const float *x,
                              const float *cache, const float *dy, float *grad, void *workspace,
                              size_t workspace_bytes, void *stream) {
  if (!shape_ok(shape) || !params || batch < 1 || !x || !cache || !dy || !grad || !workspace) return ENUF_EINVAL;
  if (workspace_bytes < enuf_mlp_workspace_bytes(shape, batch)) return ENUF_EINVAL;
  const Shape sh = mk(shape);
  const long nblk = (batch + kMlpSamples - 1) / kMlpSamples;
  float *gpart = (float *)workspace;
  hipLaunchKernelGGL(k_mlp_bwd, dim3(nblk), dim3(kMlpBlock), 0, (hipStream_t)stream, sh, params, (long)batch, x,
                     cache, dy, gpart);
  const long np = sh.count();
  hipLaunchKernelGGL(k_mlp_reduce, dim3((np + kMlpBlock - 1) / kMlpBlock), dim3(kMlpBlock), 0,
                     (hipStream_t)stream, (const float *)gpart, nblk, np, grad);
  return launched();
}

enuf_status enuf_mlp_adam(int64_t n, float *params, const float *grad, float *m, float *v, float lr, float beta1,
                          float beta2, float eps, int32_t t, void *stream) {
  if (n < 1 || !params || !grad || !m || !v || t < 1) return ENUF_EINVAL;
  const float c1 = 1.f - std::pow(beta1, (float)t), c2 = 1.f - std::pow(beta2, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((n + kMlpBlock - 1) / kMlpBlock), dim3(kMlpBlock), 0, (hipStream_t)stream,
                     (long)n, params, grad, m, v, lr, beta1, beta2, eps, c1, c2);
  return launched();
}

}  // extern "C"
