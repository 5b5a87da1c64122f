// enuf_kernels.hip -- HIP kernels of the ENUF hot path for gfx950 (CDNA4).
//
// One evaluation (paper Sec. 3.1-3.2) runs these phases on one stream:
//   prep      wrap positions, bin keys, per-block bucket counts, charge sums
//   sort      bucket slots, staging into buckets, per-bucket counting sort
//             into tile / cell order (no global atomics)
//   spread    type-1 NFFT gridding step (Eq. 36): B-spline window, one
//             workgroup per grid tile accumulating in LDS (no global atomics)
//   fft_fwd   real-to-complex transform along x, complex along y (LDS pencils)
//   z fused   forward z transform, scaling by the window transform (Eq. 37),
//             influence function and FP64 energy (Eq. 38), the three ik field
//             spectra of Eq. 41 plus the potential spectrum, inverse z
//             transforms -- the spectrum never returns to HBM in between
//   fft_inv   inverse y transforms, complex-to-real x transforms writing the
//             four real fields interleaved (E_x, E_y, E_z, psi) per grid point
//   gather    type-2 NFFT interpolation (Eq. 35, 42): all three force
//             components and the potential in one pass
//   pair      erfc real-space sum on a linked-cell list (Eq. 17, 29)
//   finalize  energy parts in FP64, self (Eq. 24) and background terms
#include "enuf_internal.h"

#include <cmath>
#include <cstring>
#include <algorithm>

namespace enuf {

// --------------------------------------------------------------------------
// small types and helpers
// --------------------------------------------------------------------------
template <typename R> struct V4;
template <> struct V4<float> { using T = float4; };
template <> struct V4<double> { using T = double4; };
template <typename R> using real4 = typename V4<R>::T;

template <typename R> struct Cx { R x, y; };

// 1/x: the hardware reciprocal (1 ulp) in single precision, a division in double
__device__ __forceinline__ float recip_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip_r(double x) { return 1.0 / x; }

// plain register types for staging copies (no constructors, so arrays of
// them stay in registers)
template <typename T> struct PodOf { using type = T; };
template <> struct PodOf<float4> { using type = float __attribute__((ext_vector_type(4))); };
template <> struct PodOf<double4> { using type = double __attribute__((ext_vector_type(4))); };
template <> struct PodOf<Cx<float>> { using type = float __attribute__((ext_vector_type(2))); };
template <> struct PodOf<Cx<double>> { using type = double __attribute__((ext_vector_type(2))); };
template <typename T> using pod_t = typename PodOf<T>::type;

// the potential component of a field grid point: .w of the interleaved
// (E_x, E_y, E_z, psi) layout, or the value itself on a potential-only grid
template <typename R> __device__ __forceinline__ R psi_of(const real4<R> &f) { return f.w; }
template <typename R> __device__ __forceinline__ R psi_of(R f) { return f; }

template <typename R> __device__ __forceinline__ Cx<R> cadd(Cx<R> a, Cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R> __device__ __forceinline__ Cx<R> csub(Cx<R> a, Cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R> __device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R> __device__ __forceinline__ Cx<R> cconj(Cx<R> a) { return {a.x, -a.y}; }
// multiply by s*i (s = +1 or -1)
template <typename R, int S> __device__ __forceinline__ Cx<R> cmuli(Cx<R> a) {
  return S > 0 ? Cx<R>{-a.y, a.x} : Cx<R>{a.y, -a.x};
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Sum over the block (blockDim.x a multiple of 64, <= 1024); result in thread 0.
__device__ double block_sum(double v) {
  __shared__ double red[16];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  __syncthreads();
  return s;
}

__device__ double block_max(double v) {
  __shared__ double red[16];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) s = fmax(s, red[i]);
  }
  __syncthreads();
  return s;
}

// Periodic wrap of one coordinate into [0, L).  Positions already inside the
// box pass through unchanged (bit for bit), so pair distances between them
// carry no wrap rounding.
template <typename R>
__device__ __forceinline__ R wrap_pos(R x, R L, R invL) {
  R xw = x;
  if (!(xw >= R(0) && xw < L)) {
    xw = x - L * floor(x * invL);
    if (xw >= L) xw -= L;
    if (xw < R(0)) xw += L;
    if (!(xw >= R(0) && xw < L)) xw = R(0);
  }
  return xw;
}

// Grid coordinate s = x_w * M / L in [0, M) of a wrapped coordinate.
template <typename R>
__device__ __forceinline__ R grid_coord(R xw, R scale, int M) {
  R s = xw * scale;
  if (!(s < R(M))) s = R(0);  // x_w just below L rounding up to M is the point 0
  return s;
}

__device__ __forceinline__ int wrapi(int i, int m) { return i < 0 ? i + m : (i >= m ? i - m : i); }

// Cardinal B-spline of order P evaluated on a particle's P stencil points:
// with f the fractional part of the grid coordinate, the stencil points are
// floor(s) - P/2 + 1 + j and their weights w[j] = M_P(f + P - 1 - j), using
// M_1 = 1 on [0,1) and M_n(y) = (y M_{n-1}(y) + (n - y) M_{n-1}(y - 1))/(n-1).
//
// Each weight is one polynomial piece of M_P, a polynomial of degree P - 1 in
// f.  BsplinePoly runs the recursion at compile time on those pieces:
// V_k(f) = (n-1)! M_n(f + k) has integer coefficients, with
//   V^n_k = (f + k) V^{n-1}_k + (n - k - f) V^{n-1}_{k-1},
// and c[j][m] = V^P_{P-1-j}[m] / (P-1)! is the coefficient of f^m in w[j].
template <int P>
struct BsplinePoly {
  double c[P][P];
  constexpr BsplinePoly() : c() {
    long long v[P][P] = {};
    v[0][0] = 1;
    for (int n = 2; n <= P; ++n) {
      long long u[P][P] = {};
      for (int k = 0; k < n; ++k)
        for (int m = 0; m < n; ++m) {
          long long t = k * v[k][m] + (m > 0 ? v[k][m - 1] : 0);
          if (k > 0) t += (n - k) * v[k - 1][m] - (m > 0 ? v[k - 1][m - 1] : 0);
          u[k][m] = t;
        }
      for (int k = 0; k < P; ++k)
        for (int m = 0; m < P; ++m) v[k][m] = u[k][m];
    }
    double fact = 1.0;
    for (int i = 2; i < P; ++i) fact *= i;
    for (int j = 0; j < P; ++j)
      for (int m = 0; m < P; ++m) c[j][m] = (double)v[P - 1 - j][m] / fact;
  }
};

// Weights by Horner's rule.  M_P(y) = M_P(P - y) gives w[P-1-j](f) =
// w[j](1 - f), so only the pieces j >= P/2 are used, each in the variable in
// which it vanishes at 0 (f for w[j], 1 - f for w[P-1-j]): the small weights
// at the stencil's ends keep their relative accuracy.
template <typename R, int P>
__device__ __forceinline__ void bspline(R f, R (&w)[P]) {
  constexpr BsplinePoly<P> C{};
  const R u = R(1) - f;
#pragma unroll
  for (int j = P / 2; j < P; ++j) {
    R a = R(C.c[j][P - 1]), b = a;
#pragma unroll
    for (int m = P - 2; m >= 0; --m) {
      a = fma(a, f, R(C.c[j][m]));
      b = fma(b, u, R(C.c[j][m]));
    }
    w[j] = a;
    w[P - 1 - j] = b;
  }
}

// Same, plus the derivative of each weight with respect to s (= d/df), from
// the differentiated pieces (d/df of w[j](1 - f) is -w[j]'(1 - f)).
template <typename R, int P>
__device__ __forceinline__ void bspline_d(R f, R (&w)[P], R (&dw)[P]) {
  constexpr BsplinePoly<P> C{};
  const R u = R(1) - f;
#pragma unroll
  for (int j = P / 2; j < P; ++j) {
    R a = R(C.c[j][P - 1]), b = a;
    R da = R((P - 1) * C.c[j][P - 1]), db = da;
#pragma unroll
    for (int m = P - 2; m >= 0; --m) {
      a = fma(a, f, R(C.c[j][m]));
      b = fma(b, u, R(C.c[j][m]));
      if (m >= 1) {
        da = fma(da, f, R(m * C.c[j][m]));
        db = fma(db, u, R(m * C.c[j][m]));
      }
    }
    w[j] = a;
    w[P - 1 - j] = b;
    dw[j] = da;
    dw[P - 1 - j] = -db;
  }
}

__device__ __forceinline__ float exp_win(float v) { return __expf(v); }
__device__ __forceinline__ double exp_win(double v) { return exp(v); }

// The window the context uses on a particle's P stencil points (the same
// points for both windows: floor(s) - P/2 + 1 + j): the cardinal B-spline
// above, or the Gaussian exp(-d^2/b) of the paper's NFFT form, d = s - l =
// f + P/2 - 1 - j (for P = 2m + 2 the points floor(s) - m .. floor(s) + m + 1
// of an NFFT of cutoff m).  The branch is uniform across a launch.
template <typename R, int P>
__device__ __forceinline__ void window_w(R f, R (&w)[P], const Geom &g) {
  if (g.win == 0) {
    bspline<R, P>(f, w);
    return;
  }
  const R ib = (R)g.gib;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const R d = f + R(P / 2 - 1 - j);
    w[j] = exp_win(-d * d * ib);
  }
}

// Weights and their derivatives with respect to s.
template <typename R, int P>
__device__ __forceinline__ void window_wd(R f, R (&w)[P], R (&dw)[P], const Geom &g) {
  if (g.win == 0) {
    bspline_d<R, P>(f, w, dw);
    return;
  }
  const R ib = (R)g.gib;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const R d = f + R(P / 2 - 1 - j);
    w[j] = exp_win(-d * d * ib);
    dw[j] = R(-2) * d * ib * w[j];
  }
}

// --------------------------------------------------------------------------
// fills
// --------------------------------------------------------------------------
__global__ void k_fill_i32(int *p, int n, int v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}
template <typename R>
__global__ void k_fill_real(R *p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = R(0);
}

// Exclusive scan of one int per thread over the block (blockDim.x a multiple
// of 64, <= 1024); the block total goes to *total.
__device__ int block_exscan_int(int v, int *total) {
  __shared__ int wsum[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int before = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    const int t = wsum[k];
    if (k < wv) before += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return before + inc - v;
}

// Block order for kernels whose neighbouring blocks read overlapping data:
// workgroups are dealt to the eight XCDs in turn (block b to XCD b mod 8),
// each XCD with its own L2.  Mapping hardware block b to logical block
// (b mod 8) n/8 + b/8 gives each XCD one contiguous eighth of the logical
// order (a slab of the grid), so the overlap between neighbours is fetched
// into one L2 instead of several.  A bijection when n is a multiple of 8;
// other counts keep the plain order.
__device__ __forceinline__ int xcd_slab(int b, int n) {
  return (n & 7) == 0 ? (b & 7) * (n >> 3) + (b >> 3) : b;
}

// block-wide exclusive count of a flag: the wave's ballot and a masked bit
// count give the rank inside the wave, one LDS word per wave the rest
// (NW: the block's wave count when known at compile time, else 0)
template <int NW = 0>
__device__ int block_exscan_flag(bool f, int *total) {
  __shared__ int wcnt[16];
  const int wv = threadIdx.x >> 6, nw = NW > 0 ? NW : (int)(blockDim.x >> 6);
  const unsigned long long m = __ballot(f);
  const int inwave = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
  if ((threadIdx.x & 63) == 0) wcnt[wv] = __popcll(m);
  __syncthreads();
  int before = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    const int t = wcnt[k];
    if (k < wv) before += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return before + inwave;
}

// --------------------------------------------------------------------------
// prep and sort: wrap, bin keys, two-level counting sort, charge sums
//
// Reciprocal-path key: (tile, charged/neutral, spill class).  Along each axis
// a particle's stencil either stays inside its tile (digit 1), crosses the low
// face (digit 0) or the high face (digit 2); the class is the three digits.
// With that order a tile can read, from each neighbouring tile, exactly the
// particles whose stencils reach it, as a few contiguous runs.
// Real-space key: (cell, charged/neutral).
//
// Both orders are built without global atomics.  Each key range is cut into
// buckets of 2^sh consecutive keys.  Pass 1 counts, per block of particles,
// the particles of each bucket in LDS; a column scan and a bucket scan turn the
// per-block counts into each block's first slot in every bucket; pass 2 moves
// every particle to its bucket (slots taken with LDS atomics); pass 3 sorts
// one bucket per workgroup by its fine key in LDS and writes the final order
// and the bin offsets.
// --------------------------------------------------------------------------
// D: margin in grid points for particles that may move (persistent binning):
// the digit then says whether the stencil can cross a face after moving D
// points (P + 2D <= T + 1 keeps the two faces exclusive).
__device__ __forceinline__ int spill_digit(int local, int T, int P, int D) {
  if (local < P / 2 - 1 + D) return 0;
  if (local > T - 1 - P / 2 - D) return 2;
  return 1;
}

// Wrapped position and grid coordinate of one particle (shared by the key
// pass and the staging pass, so both see the same values).
template <typename R>
__device__ __forceinline__ void particle_coords(const R (&p3)[3], const Geom &g, R (&xw)[3], R (&sg)[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    xw[d] = wrap_pos(p3[d], R(g.L[d]), R(g.iL[d]));
    sg[d] = grid_coord(xw[d], R(g.mL[d]), g.M[d]);
  }
}

template <typename R>
__device__ __forceinline__ void particle_keys(const R (&xw)[3], const R (&sg)[3], bool neutral, const Geom &g,
                                              int &kt, int &kc) {
  int tix[3], cix[3], dig[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int gi = (int)sg[d];
    tix[d] = gi / g.T[d];
    dig[d] = spill_digit(gi - tix[d] * g.T[d], g.T[d], g.p, g.sdig[d]);
    const int ci = (int)(xw[d] * R(g.cL[d]));
    cix[d] = ci < g.nc[d] ? ci : g.nc[d] - 1;
  }
  const int nt = neutral ? 1 : 0;
  const int tile = (tix[2] * g.nt[1] + tix[1]) * g.nt[0] + tix[0];
  kt = tile * kTileBins + nt * kClasses + (dig[0] * 9 + dig[1] * 3 + dig[2]);
  kc = 2 * ((cix[2] * g.nc[1] + cix[1]) * g.nc[0] + cix[0]) + nt;
}

// Pass 1: keys of every particle (-1 for inactive ones, whose outputs are
// zeroed here), per-block bucket counts hist[blk][bucket] (tile buckets, then
// cell buckets), per-block sums of q, q^2, max |q| and the charged count.
template <typename R>
__global__ __launch_bounds__(kSortBlock) void k_sort_count(const R *__restrict__ x, const R *__restrict__ q, Geom g,
                                                           SortPlan sp, int all_active, int *__restrict__ key_t,
                                                           int *__restrict__ key_c, int *__restrict__ hist,
                                                           R *F, R *phi, double *qpart, int *counts, int persist,
                                                           R *__restrict__ x_ref, R *__restrict__ q_ref,
                                                           int *__restrict__ act) {
  // persistent binning: this evaluation keeps the last sort (k_refresh runs)
  if (persist && counts[3] == 0) return;
  if (persist && blockIdx.x == 0 && threadIdx.x == 0) counts[4] = all_active;
  extern __shared__ int cnt[];
  const int nbk = sp.nb[0] + sp.nb[1];
  for (int b = threadIdx.x; b < nbk; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  const long long i0 = (long long)blockIdx.x * sp.per;
  const int i1 = (int)min((long long)g.n, i0 + sp.per);
  double qs = 0.0, q2 = 0.0, qa = 0.0, nq = 0.0;
  // four particles per thread per step: their loads are issued together
  constexpr int U = 4;
  for (int ib = (int)i0 + threadIdx.x; ib < i1; ib += U * blockDim.x) {
    R px[U][3], pq[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = ib + u * blockDim.x;
      if (i < i1) {
        px[u][0] = x[3 * i];
        px[u][1] = x[3 * i + 1];
        px[u][2] = x[3 * i + 2];
        pq[u] = q[i];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = ib + u * blockDim.x;
      if (i >= i1) break;
      const R p3[3] = {px[u][0], px[u][1], px[u][2]};
      const R qi = pq[u];
      const bool fin = isfinite(p3[0]) && isfinite(p3[1]) && isfinite(p3[2]) && isfinite(qi);
      if (!fin) atomicOr(&counts[2], 1);
      const bool active = fin && (qi != R(0) || all_active);
      if (persist) {
        x_ref[3 * i] = p3[0];
        x_ref[3 * i + 1] = p3[1];
        x_ref[3 * i + 2] = p3[2];
        q_ref[i] = qi;
        act[i] = active ? 1 : 0;
      }
      if (fin) {
        qs += (double)qi;
        q2 += (double)qi * (double)qi;
        qa = fmax(qa, fabs((double)qi));
      }
      if (active) {
        R xw[3], sg[3];
        particle_coords(p3, g, xw, sg);
        int kt, kc;
        particle_keys(xw, sg, qi == R(0), g, kt, kc);
        key_t[i] = kt;
        key_c[i] = kc;
        atomicAdd(&cnt[kt >> sp.sh[0]], 1);
        atomicAdd(&cnt[sp.nb[0] + (kc >> sp.sh[1])], 1);
        if (qi != R(0)) nq += 1.0;
      } else {
        key_t[i] = -1;
        key_c[i] = -1;
        if (F) { F[3 * i] = R(0); F[3 * i + 1] = R(0); F[3 * i + 2] = R(0); }
        if (phi) phi[i] = R(0);
      }
    }
  }
  __syncthreads();
  int *row = hist + (size_t)blockIdx.x * nbk;
  for (int b = threadIdx.x; b < nbk; b += blockDim.x) row[b] = cnt[b];
  const double a = block_sum(qs);
  const double b2 = block_sum(q2);
  const double m = block_max(qa);
  const double c = block_sum(nq);
  if (threadIdx.x == 0) {
    qpart[4 * blockIdx.x] = a;
    qpart[4 * blockIdx.x + 1] = b2;
    qpart[4 * blockIdx.x + 2] = m;
    qpart[4 * blockIdx.x + 3] = c;
  }
}

// Persistent binning, step 1: does this evaluation sort?  counts[3] is 1
// after a workspace initialisation; otherwise it is set here when some
// particle has moved more than skin/2 (minimum image) since the last sort, a
// charge differs from its value then, an input is not finite, or the
// all-active flag differs.  k_finalize clears it at the end of each
// evaluation.
template <typename R>
__global__ __launch_bounds__(kSortBlock) void k_persist_check(const R *__restrict__ x, const R *__restrict__ q, Geom g,
                                                              const R *__restrict__ x_ref,
                                                              const R *__restrict__ q_ref, int all_active,
                                                              int *counts) {
  const R lim2 = (R)(0.25 * g.skin * g.skin);
  const R L0 = (R)g.L[0], L1 = (R)g.L[1], L2 = (R)g.L[2];
  const R i0 = (R)g.iL[0], i1 = (R)g.iL[1], i2 = (R)g.iL[2];
  bool bad = blockIdx.x == 0 && threadIdx.x == 0 && counts[4] != all_active;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += gridDim.x * blockDim.x) {
    const R px = x[3 * i], py = x[3 * i + 1], pz = x[3 * i + 2], qi = q[i];
    R dx = px - x_ref[3 * i], dy = py - x_ref[3 * i + 1], dz = pz - x_ref[3 * i + 2];
    dx -= L0 * rint(dx * i0);
    dy -= L1 * rint(dy * i1);
    dz -= L2 * rint(dz * i2);
    const R d2 = dx * dx + dy * dy + dz * dz;
    // written so that NaN anywhere reads as a violation
    const bool ok = d2 <= lim2 && qi == q_ref[i] && isfinite(px) && isfinite(py) && isfinite(pz);
    bad = bad || !ok;
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&counts[3], 1);
}

// Persistent binning, step 2 (when no sort is needed): the sorted copies of
// the particles in the kept order, from the current positions and charges:
// grid coordinates of the wrapped position for the tile order; for the cell
// order, the position at the last sort (wrapped as the sort wrapped it) plus
// the minimum-image displacement since, so every particle stays beside the
// cell it is binned in.  Also the per-block charge sums of k_sort_count and
// zero outputs for inactive particles.
template <typename R>
__global__ __launch_bounds__(kSortBlock) void k_refresh(const R *__restrict__ x, const R *__restrict__ q, Geom g,
                                                        SortPlan sp, const R *__restrict__ x_ref,
                                                        const int *__restrict__ act, const int *__restrict__ perm_t,
                                                        const int *__restrict__ perm_c, real4<R> *__restrict__ part_t,
                                                        real4<R> *__restrict__ part_c, R *F, R *phi, double *qpart,
                                                        const int *counts) {
  if (counts[3] != 0) return;
  const long long i0 = (long long)blockIdx.x * sp.per;
  const int i1 = (int)min((long long)g.n, i0 + sp.per);
  double qs = 0.0, q2 = 0.0, qa = 0.0, nq = 0.0;
  for (int i = (int)i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const R qi = q[i];
    qs += (double)qi;
    q2 += (double)qi * (double)qi;
    qa = fmax(qa, fabs((double)qi));
    if (act[i]) {
      if (qi != R(0)) nq += 1.0;
    } else {
      if (F) { F[3 * i] = R(0); F[3 * i + 1] = R(0); F[3 * i + 2] = R(0); }
      if (phi) phi[i] = R(0);
    }
  }
  // the kept orders gather from the caller's arrays at random: four slots
  // per thread, their loads issued together
  const int ke = min(i1, counts[0]);
  constexpr int U = 4;
  for (int kb = (int)i0 + threadIdx.x; kb < ke; kb += U * blockDim.x) {
    int it[U], ic[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = kb + u * blockDim.x;
      it[u] = k < ke ? perm_t[k] : 0;
      ic[u] = k < ke ? perm_c[k] : 0;
    }
    R pt[U][4], pc[U][4], pr[U][3];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      pt[u][0] = x[3 * it[u]];
      pt[u][1] = x[3 * it[u] + 1];
      pt[u][2] = x[3 * it[u] + 2];
      pt[u][3] = q[it[u]];
      pc[u][0] = x[3 * ic[u]];
      pc[u][1] = x[3 * ic[u] + 1];
      pc[u][2] = x[3 * ic[u] + 2];
      pc[u][3] = q[ic[u]];
      pr[u][0] = x_ref[3 * ic[u]];
      pr[u][1] = x_ref[3 * ic[u] + 1];
      pr[u][2] = x_ref[3 * ic[u] + 2];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = kb + u * blockDim.x;
      if (k >= ke) break;
      {
        const R p3[3] = {pt[u][0], pt[u][1], pt[u][2]};
        R xw[3], sg[3];
        particle_coords(p3, g, xw, sg);
        real4<R> a;
        a.x = sg[0];
        a.y = sg[1];
        a.z = sg[2];
        a.w = pt[u][3];
        part_t[k] = a;
      }
      {
        // the position at the last sort, wrapped as the sort wrapped it, plus
        // the minimum-image displacement since
        const R r3[3] = {pr[u][0], pr[u][1], pr[u][2]};
        R xw[3], sg[3];
        particle_coords(r3, g, xw, sg);
        R d[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          d[e] = pc[u][e] - r3[e];
          d[e] -= R(g.L[e]) * rint(d[e] * R(g.iL[e]));
        }
        real4<R> a;
        a.x = xw[0] + d[0];
        a.y = xw[1] + d[1];
        a.z = xw[2] + d[2];
        a.w = pc[u][3];
        part_c[k] = a;
      }
    }
  }
  const double a = block_sum(qs);
  const double b2 = block_sum(q2);
  const double m = block_max(qa);
  const double c = block_sum(nq);
  if (threadIdx.x == 0) {
    qpart[4 * blockIdx.x] = a;
    qpart[4 * blockIdx.x + 1] = b2;
    qpart[4 * blockIdx.x + 2] = m;
    qpart[4 * blockIdx.x + 3] = c;
  }
}

// Exclusive scan over the blocks of each bucket column of hist (in place);
// the column total goes to the bucket's slot of bbase.  16 columns per
// workgroup (64-byte row segments), 64 row groups of up to a few rows each,
// the row group's values held in registers between the two passes.
__device__ __forceinline__ int bucket_slot(const SortPlan &sp, int b) { return b < sp.nb[0] ? b : b + 1; }

constexpr int kColW = 16, kColG = 64, kColR = 16;  // columns, row groups, rows per group held

__global__ __launch_bounds__(kColW * kColG) void k_sort_colscan(int *__restrict__ hist, SortPlan sp,
                                                                int *__restrict__ bbase, const int *need) {
  if (need && *need == 0) return;
  __shared__ int part[kColG][kColW];
  const int nbk = sp.nb[0] + sp.nb[1];
  const int lane = threadIdx.x % kColW, rg = threadIdx.x / kColW;
  const int col = blockIdx.x * kColW + lane;
  const int rows = (sp.nblk + kColG - 1) / kColG;  // <= kColR: nblk <= kSortMaxBlocks
  const int r0 = rg * rows, r1 = min(sp.nblk, r0 + rows);
  int v[kColR];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kColR; ++k) {
    v[k] = (col < nbk && r0 + k < r1) ? hist[(size_t)(r0 + k) * nbk + col] : 0;
    s += v[k];
  }
  part[rg][lane] = s;
  __syncthreads();
  int run = 0;
  for (int k = 0; k < rg; ++k) run += part[k][lane];
  if (col < nbk) {
    if (rg == kColG - 1) bbase[bucket_slot(sp, col)] = run + s;
#pragma unroll
    for (int k = 0; k < kColR; ++k) {
      if (r0 + k < r1) hist[(size_t)(r0 + k) * nbk + col] = run;
      run += v[k];
    }
  }
}

// Exclusive scan of the bucket totals of each order (in place in bbase, the
// grand total after the last bucket), the bin-offset terminators, the active
// and charged counts and the charge sums.
__global__ __launch_bounds__(1024) void k_sort_base(int *__restrict__ bbase, SortPlan sp, int *off_t, int *off_c,
                                                    const double *__restrict__ qpart, double *scal, int *counts,
                                                    double *eslot, size_t eoff, int persist) {
  // the energy slots the transform and pair kernels add into
  for (int i = threadIdx.x; i < kESlots; i += blockDim.x) {
    eslot[i] = 0.0;
    eslot[eoff + i] = 0.0;
  }
  // with persistent binning an evaluation that keeps the last sort only
  // reduces the charge sums (from k_refresh's partials)
  const bool sorting = !persist || counts[3] != 0;
  // per-block charge sums, loaded first so their latency overlaps the scans
  double a = 0.0, b = 0.0, m = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < sp.nblk; i += blockDim.x) {
    a += qpart[4 * i];
    b += qpart[4 * i + 1];
    m = fmax(m, qpart[4 * i + 2]);
    c += qpart[4 * i + 3];
  }
  __shared__ int carry;
  for (int seg = 0; seg < (sorting ? 2 : 0); ++seg) {
    const int lo = seg == 0 ? 0 : sp.nb[0] + 1, n = sp.nb[seg];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < n; c0 += blockDim.x) {
      const int i = c0 + threadIdx.x;
      const int v = i < n ? bbase[lo + i] : 0;
      int tot;
      const int ex = block_exscan_int(v, &tot);
      const int cy = carry;
      if (i < n) bbase[lo + i] = cy + ex;
      __syncthreads();
      if (threadIdx.x == 0) carry = cy + tot;
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      bbase[lo + n] = carry;
      if (seg == 0) { off_t[sp.nbins[0]] = carry; counts[0] = carry; }
      else off_c[sp.nbins[1]] = carry;
    }
    __syncthreads();
  }
  // the four reductions in one exchange
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    b += __shfl_down(b, o, 64);
    m = fmax(m, __shfl_down(m, o, 64));
    c += __shfl_down(c, o, 64);
  }
  __shared__ double red4[16][4];
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red4[wv][0] = a;
    red4[wv][1] = b;
    red4[wv][2] = m;
    red4[wv][3] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0, sm = 0.0, sc = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      sa += red4[k][0];
      sb += red4[k][1];
      sm = fmax(sm, red4[k][2]);
      sc += red4[k][3];
    }
    counts[1] = (int)sc;
    if (sorting) counts[5] += 1;
    scal[0] = sa;
    scal[1] = sb;
    scal[2] = sm;
  }
}

// Pass 2: each active particle to the next free slot of its bucket, one order
// after the other, in chunks of sp.chunk particles: the chunk is grouped by
// bucket in LDS first, so each bucket's particles leave as one contiguous run.
// Staged records: (s_x, s_y, s_z, q) for the tile order, (x_w, y_w, z_w, q)
// for the cell order, each with (source index, key).
template <typename R>
__global__ __launch_bounds__(kSortStageBlock) void k_sort_stage(const R *__restrict__ x, const R *__restrict__ q, Geom g,
                                                           SortPlan sp, const int *__restrict__ key_t,
                                                           const int *__restrict__ key_c,
                                                           const int *__restrict__ hist,
                                                           const int *__restrict__ bbase, real4<R> *stg_t,
                                                           int2 *ik_t, real4<R> *stg_c, int2 *ik_c,
                                                           const int *need) {
  if (need && *need == 0) return;
  constexpr int U = kSortChunkMax / kSortStageBlock;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int nbk = sp.nb[0] + sp.nb[1];
  const int nbm = max(sp.nb[0], sp.nb[1]);
  real4<R> *rec = reinterpret_cast<real4<R> *>(lds_raw);  // [chunk]
  int2 *rik = reinterpret_cast<int2 *>(rec + sp.chunk);    // [chunk]
  int *slot = reinterpret_cast<int *>(rik + sp.chunk);     // [nbm] the block's next free slot per bucket
  int *cnt = slot + nbm;                                   // [nbm] chunk counts, then chunk starts
  const int tid = threadIdx.x;
  const int *row = hist + (size_t)blockIdx.x * nbk;
  const long long i0 = (long long)blockIdx.x * sp.per;
  const int i1 = (int)min((long long)g.n, i0 + sp.per);
  for (int o = 0; o < 2; ++o) {
    const int nb = sp.nb[o], sh = sp.sh[o];
    const int *key = o == 0 ? key_t : key_c;
    real4<R> *stg = o == 0 ? stg_t : stg_c;
    int2 *ik = o == 0 ? ik_t : ik_c;
    const int cb = o == 0 ? 0 : sp.nb[0];
    const int sb = o == 0 ? 0 : sp.nb[0] + 1;
    for (int b = tid; b < nb; b += blockDim.x) slot[b] = bbase[sb + b] + row[cb + b];
    if (sp.chunk == 0) {
      // ungrouped: every particle straight to its slot
      __syncthreads();
      for (int i = (int)i0 + tid; i < i1; i += blockDim.x) {
        const int k = key[i];
        if (k < 0) continue;
        const R p3[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
        R xw[3], sg[3];
        particle_coords(p3, g, xw, sg);
        real4<R> a;
        a.x = o == 0 ? sg[0] : xw[0];
        a.y = o == 0 ? sg[1] : xw[1];
        a.z = o == 0 ? sg[2] : xw[2];
        a.w = q[i];
        const int p = atomicAdd(&slot[k >> sh], 1);
        stg[p] = a;
        ik[p] = make_int2(i, k);
      }
      __syncthreads();
      continue;
    }
    for (int c0 = (int)i0; c0 < i1; c0 += sp.chunk) {
      for (int b = tid; b < nb; b += blockDim.x) cnt[b] = 0;
      __syncthreads();
      int kk[U], rr[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = c0 + u * kSortStageBlock + tid;
        kk[u] = (u * kSortStageBlock + tid < sp.chunk && i < i1) ? key[i] : -1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) rr[u] = kk[u] >= 0 ? atomicAdd(&cnt[kk[u] >> sh], 1) : 0;
      __syncthreads();
      // chunk starts per bucket: exclusive scan, each thread a run of buckets
      const int per = (nb + blockDim.x - 1) / blockDim.x;
      const int b0 = tid * per, b1 = min(nb, b0 + per);
      int sum = 0;
      for (int b = b0; b < b1; ++b) sum += cnt[b];
      int m;
      int run = block_exscan_int(sum, &m);
      for (int b = b0; b < b1; ++b) {
        const int v = cnt[b];
        cnt[b] = run;
        run += v;
      }
      __syncthreads();
      // positions and charges of the U particles, loaded together (a lane
      // without a particle rereads the chunk's first one)
      R px[U][3], pq[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = kk[u] >= 0 ? c0 + u * kSortStageBlock + tid : c0;
        px[u][0] = x[3 * i];
        px[u][1] = x[3 * i + 1];
        px[u][2] = x[3 * i + 2];
        pq[u] = q[i];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (kk[u] < 0) continue;
        const int i = c0 + u * kSortStageBlock + tid;
        R xw[3], sg[3];
        particle_coords(px[u], g, xw, sg);
        real4<R> a;
        a.x = o == 0 ? sg[0] : xw[0];
        a.y = o == 0 ? sg[1] : xw[1];
        a.z = o == 0 ? sg[2] : xw[2];
        a.w = pq[u];
        const int p = cnt[kk[u] >> sh] + rr[u];
        rec[p] = a;
        rik[p] = make_int2(i, kk[u]);
      }
      __syncthreads();
      for (int t = tid; t < m; t += blockDim.x) {
        const int2 v = rik[t];
        const int b = v.y >> sh;
        const int pos = slot[b] + (t - cnt[b]);
        stg[pos] = rec[t];
        ik[pos] = v;
      }
      __syncthreads();
      // advance the slots by the chunk's counts
      for (int b = tid; b < nb; b += blockDim.x) slot[b] += (b + 1 < nb ? cnt[b + 1] : m) - cnt[b];
      __syncthreads();
    }
  }
}

// Pass 3: one workgroup per bucket (tile buckets, then cell buckets): counting
// sort of the bucket's particles by fine key in LDS, bin offsets of the
// bucket's keys, particles and source indices in final order.  A bucket of at
// most kSortFineRegs*blockDim particles keeps keys and ranks in registers,
// then (WIN) also its records and source indices, read once and
// coalesced, and writes them out through an LDS window of kFineOutBytes: each
// pass places the records whose final slot falls in the window, then the
// window goes to memory contiguously, so the permutation happens in LDS.
// Otherwise it builds the inverse permutation in LDS and writes the final
// order contiguously while the reads gather from the staged bucket (64 cache
// lines per wave instruction: slow when every bucket's block is resident at
// once and that latency is all there is, or when the buckets are full; for
// many sparse buckets the lighter first read wins).  A larger bucket goes
// through global ranks and scattered writes.
template <typename R, bool WIN>
__device__ __forceinline__ void sort_fine(const SortPlan &sp, const int *__restrict__ bbase,
                                          const real4<R> *__restrict__ stg_t, const int2 *__restrict__ ik_t,
                                          int *srank_t, const real4<R> *__restrict__ stg_c,
                                          const int2 *__restrict__ ik_c, int *srank_c, real4<R> *part_t,
                                          int *perm_t, int *off_t, real4<R> *part_c, int *perm_c, int *off_c,
                                          const int *need) {
  if (need && *need == 0) return;
  constexpr int U = kSortFineRegs;
  extern __shared__ int lds_fine[];
  const bool tiles = (int)blockIdx.x < sp.nb[0];
  const int b = tiles ? blockIdx.x : blockIdx.x - sp.nb[0];
  const int o = tiles ? 0 : 1;
  const int slot = tiles ? b : sp.nb[0] + 1 + b;
  const int s = bbase[slot], e = bbase[slot + 1];
  const int k0 = b << sp.sh[o];
  const int nf = min(1 << sp.sh[o], sp.nbins[o] - k0);
  const real4<R> *stg = tiles ? stg_t : stg_c;
  const int2 *ik = tiles ? ik_t : ik_c;
  int *srank = tiles ? srank_t : srank_c;
  real4<R> *part = tiles ? part_t : part_c;
  int *perm = tiles ? perm_t : perm_c;
  int *off = tiles ? off_t : off_c;
  const int nt = blockDim.x, tid = threadIdx.x;
  int *bin = lds_fine;  // [2^max sh] counts, then starts
  // after the bins either the output window (WN records, then their source
  // indices) or the inverse permutation ([U*nt] bucket position -> staged index)
  constexpr int WN = kFineOutBytes / (int)sizeof(real4<R>);
  real4<R> *wrec = reinterpret_cast<real4<R> *>(lds_fine + (1 << max(sp.sh[0], sp.sh[1])));
  int *wsrc = reinterpret_cast<int *>(wrec + WN);
  int *inv = lds_fine + (1 << max(sp.sh[0], sp.sh[1]));
  const bool small = e - s <= U * nt;

  for (int f = tid; f < nf; f += nt) bin[f] = 0;
  __syncthreads();
  int kk[U], rr[U], src[U];
  int kr[U];  // window form: key << 16 | rank (key < 2^12, rank < 2^13), or -1
  pod_t<real4<R>> rec[U];
  if (small) {
    // every lane loads U (key, source index, record) triples (past the end:
    // the bucket's last one again), so the loads go out together instead of
    // one per branch
    int raw[U];
    if (WIN) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int jc = e > s ? min(s + u * nt + tid, e - 1) : 0;
        const int2 v = ik[jc];
        raw[u] = v.y;
        src[u] = v.x;
        rec[u] = *reinterpret_cast<const pod_t<real4<R>> *>(stg + jc);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) raw[u] = e > s ? ik[min(s + u * nt + tid, e - 1)].y : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = s + u * nt + tid;
      kk[u] = j < e ? raw[u] - k0 : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) rr[u] = (unsigned)kk[u] < (unsigned)nf ? atomicAdd(&bin[kk[u]], 1) : 0;
    if (WIN) {
#pragma unroll
      for (int u = 0; u < U; ++u) kr[u] = (unsigned)kk[u] < (unsigned)nf ? (kk[u] << 16) | rr[u] : -1;
    }
  } else {
    for (int j0 = s + tid; j0 < e; j0 += U * nt) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * nt;
        kk[u] = j < e ? ik[j].y - k0 : -1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * nt;
        if (j < e) srank[j] = (unsigned)kk[u] < (unsigned)nf ? atomicAdd(&bin[kk[u]], 1) : 0;
      }
    }
  }
  __syncthreads();
  // exclusive scan of the nf counts: each thread owns a run of consecutive bins
  const int per = (nf + nt - 1) / nt;
  const int f0 = tid * per, f1 = min(nf, f0 + per);
  int sum = 0;
  for (int f = f0; f < f1; ++f) sum += bin[f];
  int tot;
  int run = block_exscan_int(sum, &tot);
  for (int f = f0; f < f1; ++f) {
    const int v = bin[f];
    bin[f] = run;
    off[k0 + f] = s + run;
    run += v;
  }
  __syncthreads();
  if (small && !WIN) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if ((unsigned)kk[u] < (unsigned)nf) inv[bin[kk[u]] + rr[u]] = u * nt + tid;
    __syncthreads();
    for (int t0 = tid; t0 < e - s; t0 += 4 * nt) {
      int jj[4];
      pod_t<real4<R>> a[4];
      int pv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int v = t0 + u * nt < e - s ? inv[t0 + u * nt] : -1;
        jj[u] = (unsigned)v < (unsigned)(e - s) ? s + v : -1;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        // unconditional loads (a lane past the end rereads the bucket's
        // first record), all in flight together
        const int jc = jj[u] >= 0 ? jj[u] : s;
        a[u] = *reinterpret_cast<const pod_t<real4<R>> *>(stg + jc);
        pv[u] = ik[jc].x;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (jj[u] >= 0) {
          *reinterpret_cast<pod_t<real4<R>> *>(part + s + t0 + u * nt) = a[u];
          perm[s + t0 + u * nt] = pv[u];
        }
    }
  } else if (small) {
    int pos[U];
#pragma unroll
    for (int u = 0; u < U; ++u) pos[u] = kr[u] >= 0 ? bin[kr[u] >> 16] + (kr[u] & 0xFFFF) : -1;
    for (int w0 = 0; w0 < e - s; w0 += WN) {
      const int wn = min(WN, e - s - w0);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if ((unsigned)(pos[u] - w0) < (unsigned)wn) {
          *reinterpret_cast<pod_t<real4<R>> *>(wrec + pos[u] - w0) = rec[u];
          wsrc[pos[u] - w0] = src[u];
        }
      __syncthreads();
      for (int t = tid; t < wn; t += nt) {
        *reinterpret_cast<pod_t<real4<R>> *>(part + s + w0 + t) =
            *reinterpret_cast<const pod_t<real4<R>> *>(wrec + t);
        perm[s + w0 + t] = wsrc[t];
      }
      __syncthreads();
    }
  } else {
    for (int j0 = s + tid; j0 < e; j0 += U * nt) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * nt;
        if (j >= e) continue;
        const int2 v = ik[j];
        const int k = v.y - k0;
        if ((unsigned)k >= (unsigned)nf) continue;
        const int pos = s + bin[k] + srank[j];
        part[pos] = stg[j];
        perm[pos] = v.x;
      }
    }
  }
}

// The two forms as kernels: the gather form keeps few registers (two blocks
// per CU with room to spare), the window form (FP32 only) is held to 64
// registers (eight waves per SIMD: two 1024-thread blocks per CU).
template <typename R>
__global__ __launch_bounds__(kSortFineBlock) void k_sort_fine(SortPlan sp, const int *__restrict__ bbase,
                                                              const real4<R> *__restrict__ stg_t,
                                                              const int2 *__restrict__ ik_t, int *srank_t,
                                                              const real4<R> *__restrict__ stg_c,
                                                              const int2 *__restrict__ ik_c, int *srank_c,
                                                              real4<R> *part_t, int *perm_t, int *off_t,
                                                              real4<R> *part_c, int *perm_c, int *off_c,
                                                              const int *need) {
  sort_fine<R, false>(sp, bbase, stg_t, ik_t, srank_t, stg_c, ik_c, srank_c, part_t, perm_t, off_t, part_c, perm_c,
                      off_c, need);
}
template <typename R>
__global__ __launch_bounds__(kSortFineBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_sort_fine_win(
    SortPlan sp, const int *__restrict__ bbase, const real4<R> *__restrict__ stg_t, const int2 *__restrict__ ik_t,
    int *srank_t, const real4<R> *__restrict__ stg_c, const int2 *__restrict__ ik_c, int *srank_c,
    real4<R> *part_t, int *perm_t, int *off_t, real4<R> *part_c, int *perm_c, int *off_c, const int *need) {
  sort_fine<R, true>(sp, bbase, stg_t, ik_t, srank_t, stg_c, ik_c, srank_c, part_t, perm_t, off_t, part_c, perm_c,
                     off_c, need);
}

// --------------------------------------------------------------------------
// Deterministic mode: the particles of every bin in caller-index order, so
// that every later sum (spread columns, pair candidates, energy partials)
// runs in one order from run to run.  Bins of up to kDetSmall particles are
// ordered by one thread (insertion sort in place); larger ones are listed
// (in the dead key array of the order) and ordered by one workgroup each
// (bitonic sort of (index, position) pairs in LDS, records moved through the
// dead staging array); a bin above kDetBig sets flag bit 1.
// --------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kBlock) void k_det_small(int nbins, const int *__restrict__ off, int *perm,
                                                      real4<R> *part, int *big, int *nbig, const int *need) {
  if (need && *need == 0) return;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nbins; b += gridDim.x * blockDim.x) {
    const int s0 = off[b], n = off[b + 1] - s0;
    if (n < 2) continue;
    if (n > kDetSmall) {
      big[atomicAdd(nbig, 1)] = b;
      continue;
    }
    for (int i = 1; i < n; ++i) {
      const int key = perm[s0 + i];
      const real4<R> rec = part[s0 + i];
      int j = i - 1;
      while (j >= 0 && perm[s0 + j] > key) {
        perm[s0 + j + 1] = perm[s0 + j];
        part[s0 + j + 1] = part[s0 + j];
        --j;
      }
      perm[s0 + j + 1] = key;
      part[s0 + j + 1] = rec;
    }
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_det_big(const int *__restrict__ off, int *perm, real4<R> *part,
                                                    real4<R> *tmp, const int *__restrict__ big,
                                                    const int *__restrict__ nbig, int *counts, const int *need) {
  if (need && *need == 0) return;
  __shared__ int key[kDetBig], pos[kDetBig];
  const int nb = *nbig;
  for (int k = blockIdx.x; k < nb; k += gridDim.x) {
    const int b = big[k];
    const int s0 = off[b], n = off[b + 1] - s0;
    if (n > kDetBig) {
      if (threadIdx.x == 0) atomicOr(&counts[2], 2);
      continue;
    }
    int m = 1;
    while (m < n) m <<= 1;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      key[i] = i < n ? perm[s0 + i] : 0x7fffffff;
      pos[i] = i;
      if (i < n) tmp[s0 + i] = part[s0 + i];
    }
    __syncthreads();
    for (int size = 2; size <= m; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
          const int j = i ^ stride;
          if (j > i) {
            const bool up = (i & size) == 0;
            const int ki = key[i], kj = key[j];
            if ((ki > kj) == up) {
              key[i] = kj;
              key[j] = ki;
              const int t = pos[i];
              pos[i] = pos[j];
              pos[j] = t;
            }
          }
        }
        __syncthreads();
      }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      perm[s0 + i] = key[i];
      part[s0 + i] = tmp[s0 + pos[i]];
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------------------
// spread: rho_l = sum_i q_i B(s_i - l)   (type-1 gridding, Eq. 36)
//
// One workgroup owns one grid tile of T_x*T_y*T_z points and accumulates it in
// LDS, so each grid point is written exactly once and no global atomics are
// used.  It pulls exactly the charged particles whose stencils reach the tile:
// its own, plus, from each neighbouring tile, the spill classes facing it (a
// host-built table of runs: neighbour offset and class range).  Staging:
// threads compute, for a batch of particles, the box of stencil points inside
// the tile and the 3*P window weights (charge folded into z) into LDS; then
// each wavefront takes one staged particle at a time and its 64 lanes sweep
// that particle's box with LDS atomic adds.
// --------------------------------------------------------------------------
template <typename R>
constexpr int spread_block() { return sizeof(R) == 8 ? 128 : 256; }

template <typename R, int P>
__global__ __launch_bounds__(spread_block<R>()) void k_spread(const real4<R> *__restrict__ part,
                                                              const int *__restrict__ off_t,
                                                              const int *__restrict__ runs, int nruns, Geom g,
                                                              R *__restrict__ grid) {
  // One private accumulator per wavefront: a wave only ever adds the distinct
  // box points of one particle per step, so plain LDS read-modify-write is
  // race free (LDS float atomics are several times slower).
  constexpr int NB = spread_block<R>();
  __shared__ R acc[NB / 64][kMaxTilePts];
  // Per staged particle: its box in the tile as two "lane" axes A (outer),
  // B (inner) and one "loop" axis C, the window weights along each (charge
  // folded into C, entry 0 = first point inside the tile), and a descriptor
  // {corner offset, nA | nB << 8 | nC << 16, strideA | strideB << 16, strideC}.
  __shared__ R wA[NB][P], wB[NB][P], wC[NB][P];
  __shared__ int4 desc[NB];
  __shared__ int rstart[kMaxRuns], rpre[kMaxRuns + 1];
  __shared__ int nstaged;

  const int tid = threadIdx.x;
  int t = blockIdx.x;
  const int tx = t % g.nt[0];
  t /= g.nt[0];
  const int ty = t % g.nt[1];
  const int tz = t / g.nt[1];
  const int t0[3] = {tx * g.T[0], ty * g.T[1], tz * g.T[2]};
  const int tpts = g.T[0] * g.T[1] * g.T[2];
  const int sy = g.T[0], sz = g.T[0] * g.T[1];
  for (int e = tid; e < tpts; e += blockDim.x)
#pragma unroll
    for (int k = 0; k < NB / 64; ++k) acc[k][e] = R(0);

  // runs -> particle ranges, then an exclusive prefix over their lengths
  for (int k = tid; k < nruns; k += blockDim.x) {
    const int *rr = runs + 5 * k;
    const int nx = wrapi(tx + rr[0], g.nt[0]);
    const int ny = wrapi(ty + rr[1], g.nt[1]);
    const int nz = wrapi(tz + rr[2], g.nt[2]);
    const int tt = (nz * g.nt[1] + ny) * g.nt[0] + nx;
    const int s0 = off_t[tt * kTileBins + rr[3]];
    const int s1 = off_t[tt * kTileBins + rr[4] + 1];
    rstart[k] = s0;
    rpre[k + 1] = s1 - s0;
  }
  __syncthreads();
  if (tid < 64) {
    int carry = 0;
    for (int c0 = 0; c0 < nruns; c0 += 64) {
      const int k = c0 + tid;
      const int v = k < nruns ? rpre[k + 1] : 0;
      int inc = v;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(inc, o, 64);
        if (tid >= o) inc += u;
      }
      if (k < nruns) rpre[k + 1] = carry + inc;
      carry += __shfl(inc, 63, 64);
    }
    if (tid == 0) rpre[0] = 0;
  }
  __syncthreads();
  const int total = rpre[nruns];
  const int lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
  R *my = acc[wv];

  for (int base = 0; base < total; base += blockDim.x) {
    const int c = base + tid;
    real4<R> v{};
    int ls[3] = {0, 0, 0}, cnt[3] = {0, 0, 0}, js[3] = {0, 0, 0};
    R fr[3] = {R(0), R(0), R(0)};
    bool hit = false;
    if (c < total) {
      int lo = 0, hi = nruns;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rpre[mid] <= c) lo = mid; else hi = mid;
      }
      v = part[rstart[lo] + (c - rpre[lo])];
      const R s[3] = {v.x, v.y, v.z};
      hit = true;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const R fl = floor(s[d]);
        fr[d] = s[d] - fl;
        // stencil start relative to the tile, brought into [0, M)
        int rel = (int)fl - P / 2 + 1 - t0[d];
        if (rel < 0) rel += g.M[d];
        if (rel < 0) rel += g.M[d];
        if (rel >= g.M[d]) rel -= g.M[d];
        if (rel < g.T[d]) {
          ls[d] = rel;
          js[d] = 0;
          cnt[d] = min(P, g.T[d] - rel);
        } else {
          ls[d] = 0;
          js[d] = g.M[d] - rel;
          cnt[d] = P - js[d];
        }
        hit = hit && cnt[d] > 0;
      }
    }
    {
      // staging slots in candidate order (a block scan, so the order of the
      // sums is the same from run to run)
      int ns;
      const int slot = block_exscan_flag(hit, &ns);
      if (tid == 0) nstaged = ns;
      if (hit) {
        // loop over the shorter of z and x; lanes cover the other two axes
        const bool loopz = cnt[2] <= cnt[0];
        const int aA = loopz ? 1 : 2, aB = loopz ? 0 : 1, aC = loopz ? 2 : 0;
        const int strd[3] = {1, sy, sz};
        R w[P];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          window_w<R, P>(fr[d], w, g);
          const R sc = (d == aC) ? v.w : R(1);
          R *dst = (d == aA) ? wA[slot] : ((d == aB) ? wB[slot] : wC[slot]);
#pragma unroll
          for (int j = 0; j < P; ++j)
            if (j >= js[d] && j - js[d] < cnt[d]) dst[j - js[d]] = w[j] * sc;
        }
        desc[slot] = make_int4(ls[2] * sz + ls[1] * sy + ls[0],
                               cnt[aA] | (cnt[aB] << 8) | (cnt[aC] << 16),
                               strd[aA] | (strd[aB] << 16), strd[aC]);
      }
    }
    __syncthreads();
    const int ns = nstaged;
    for (int sp = wv; sp < ns; sp += nwv) {
      // descriptor fields are the same for the whole wave: keep them scalar
      const int4 dd = desc[sp];
      const int corner = __builtin_amdgcn_readfirstlane(dd.x);
      const int dims = __builtin_amdgcn_readfirstlane(dd.y);
      const int st2 = __builtin_amdgcn_readfirstlane(dd.z);
      const int sC = __builtin_amdgcn_readfirstlane(dd.w);
      const int nA = dims & 255, nB = (dims >> 8) & 255, nC = dims >> 16;
      const int sA = st2 & 0xffff, sB = st2 >> 16;
      if (lane < nA * nB) {
        const int a = (int)(((float)lane + 0.5f) * __builtin_amdgcn_rcpf((float)nB));
        const int b = lane - __umul24(a, nB);
        const R w2 = wA[sp][a] * wB[sp][b];
        R *pa = my + corner + __umul24(a, sA) + __umul24(b, sB);
        const R *wc = wC[sp];
        // the nC points of this lane are distinct: read them all, then write
        R vv[P];
#pragma unroll
        for (int k = 0; k < P; ++k)
          if (k < nC) vv[k] = pa[k * sC];
#pragma unroll
        for (int k = 0; k < P; ++k)
          if (k < nC) pa[k * sC] = vv[k] + w2 * wc[k];
      }
    }
    __syncthreads();
  }
  // write the tile (rows of T_x contiguous points)
  for (int e = tid; e < tpts; e += blockDim.x) {
    const int ix = e % g.T[0];
    const int r = e / g.T[0];
    const int iy = r % g.T[1];
    const int iz = r / g.T[1];
    R v = R(0);
#pragma unroll
    for (int k = 0; k < NB / 64; ++k) v += acc[k][e];
    grid[((size_t)(t0[2] + iz) * g.M[1] + (t0[1] + iy)) * g.M[0] + t0[0] + ix] = v;
  }
}

// --------------------------------------------------------------------------
// spread on the matrix cores (FP32 path), same tiles and particle runs as
// k_spread.  With the window weights of particle k embedded in tile
// coordinates (e^x_k: 16 values, e^y_k, e^z_k: 8 values, zero outside the
// stencil and outside the tile),
//   rho[x][y, z] = sum_k e^x_k[x] * e^y_k[y] * (q_k e^z_k[z])
// is the product of a 16 x K and a K x 64 matrix over the K particles that
// reach the tile.  Each wavefront accumulates all 16 x 64 outputs in MFMA
// registers (16x16x16 f16 blocks, four column blocks) over its share of the
// 16-particle steps; the four partial tiles are summed through LDS at the end.
// Operands are split into f16 high and low parts, a = a_h + a_l, and each
// product is taken as a_h b_h + a_h b_l + a_l b_h (about 21 significant bits;
// the accumulation is FP32).  Charges are scaled by 2^-e, 2^e > max|q|, so
// that every operand is at most 1 in magnitude; the tile is scaled back on
// output.
// --------------------------------------------------------------------------
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kSpreadK = 256;             // particles staged per round (one per thread)
constexpr int kSpreadLd = kSpreadK + 4;   // LDS row pitch of the staged columns (floats)

__device__ __forceinline__ void split_f16(float4_t v, half4_t &hi, half4_t &lo) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const _Float16 h = (_Float16)v[r];
    hi[r] = h;
    lo[r] = (_Float16)(v[r] - (float)h);  // v - h is exact in FP32
  }
}

// Particle ranges of the runs that reach tile (tx, ty, tz) and the exclusive
// prefix of their lengths: rpre[nruns] is the candidate count.
__device__ void tile_runs(const int *__restrict__ off_t, const int *__restrict__ runs, int nruns, const Geom &g,
                          int tx, int ty, int tz, int *rstart, int *rpre) {
  const int tid = threadIdx.x;
  for (int k = tid; k < nruns; k += blockDim.x) {
    const int *rr = runs + 5 * k;
    const int nx = wrapi(tx + rr[0], g.nt[0]);
    const int ny = wrapi(ty + rr[1], g.nt[1]);
    const int nz = wrapi(tz + rr[2], g.nt[2]);
    const int tt = (nz * g.nt[1] + ny) * g.nt[0] + nx;
    const int s0 = off_t[tt * kTileBins + rr[3]];
    const int s1 = off_t[tt * kTileBins + rr[4] + 1];
    rstart[k] = s0;
    rpre[k + 1] = s1 - s0;
  }
  __syncthreads();
  if (tid < 64) {
    int carry = 0;
    for (int c0 = 0; c0 < nruns; c0 += 64) {
      const int k = c0 + tid;
      const int v = k < nruns ? rpre[k + 1] : 0;
      int inc = v;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(inc, o, 64);
        if (tid >= o) inc += u;
      }
      if (k < nruns) rpre[k + 1] = carry + inc;
      carry += __shfl(inc, 63, 64);
    }
    if (tid == 0) rpre[0] = 0;
  }
  __syncthreads();
}

template <int P, bool F32MAC>
__global__ __launch_bounds__(256) void k_spread_mfma(const float4 *__restrict__ part, const int *__restrict__ off_t,
                                                     const int *__restrict__ runs, int nruns, Geom g,
                                                     const double *__restrict__ scal, float *__restrict__ grid) {
  // rows 0..15: e^x, 16..23: e^y, 24..31: q e^z, one column per staged
  // particle; row 32 takes the weights that fall outside the tile
  __shared__ __align__(16) float E[33][kSpreadLd];
  __shared__ int rstart[kMaxRuns], rpre[kMaxRuns + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int t = blockIdx.x;
  const int tx = t % g.nt[0];
  t /= g.nt[0];
  const int ty = t % g.nt[1];
  const int tz = t / g.nt[1];
  const int t0[3] = {tx * g.T[0], ty * g.T[1], tz * g.T[2]};
  tile_runs(off_t, runs, nruns, g, tx, ty, tz, rstart, rpre);
  const int total = rpre[nruns];
  int qe;
  (void)frexp(scal[2], &qe);  // 2^qe > max|q| (qe = 0 when there are no charges)
  const float qscale = ldexpf(1.0f, -qe);
  const int row0[3] = {0, 16, 24};

  float4_t acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = float4_t{0.0f, 0.0f, 0.0f, 0.0f};

  for (int base = 0; base < total; base += kSpreadK) {
    // clear rows 0..31 (every column the products read), 16 bytes per store;
    // the scan's barriers below order these stores before the weights'
    for (int e = tid; e < 32 * kSpreadLd / 4; e += blockDim.x)
      reinterpret_cast<float4_t *>(&E[0][0])[e] = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
    const int c = base + tid;
    int start[3] = {0, 0, 0};
    float fr[3] = {0.0f, 0.0f, 0.0f}, qv = 0.0f;
    bool hit = false;
    if (c < total) {
      int lo = 0, hi = nruns;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rpre[mid] <= c) lo = mid; else hi = mid;
      }
      const float4 v = part[rstart[lo] + (c - rpre[lo])];
      const float s[3] = {v.x, v.y, v.z};
      hit = true;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float fl = floorf(s[d]);
        fr[d] = s[d] - fl;
        // stencil start relative to the tile, wrapped into [T - M, T)
        int rel = (int)fl - P / 2 + 1 - t0[d];
        if (rel < 0) rel += g.M[d];
        if (rel < 0) rel += g.M[d];
        if (rel >= g.M[d]) rel -= g.M[d];
        start[d] = rel < g.T[d] ? rel : rel - g.M[d];
        hit = hit && start[d] + P > 0;
      }
      qv = v.w * qscale;
    }
    // deterministic compaction of the hits into columns 0 .. ns-1; the
    // columns up to the next multiple of 16 (read by the last k-step) are
    // zeroed, so no stale LDS word ever enters a product
    int ns;
    const int slot = block_exscan_flag<4>(hit, &ns);
    if (hit) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        float w[P];
        window_w<float, P>(fr[d], w, g);
        const float sc = d == 2 ? qv : 1.0f;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const int idx = start[d] + j;
          const int row = (unsigned)idx < (unsigned)g.T[d] ? row0[d] + idx : 32;
          (&E[0][0])[__umul24((unsigned)row, (unsigned)kSpreadLd) + slot] = w[j] * sc;
        }
      }
    }
    __syncthreads();
    const int nsteps = (ns + 15) >> 4;
    for (int ks = wv; ks < nsteps; ks += 4) {
      const int k0 = 16 * ks + 4 * (lane >> 4);
      // columns ns .. 16 nsteps - 1 hold the zeros stored above
      const float4_t a = *reinterpret_cast<const float4_t *>(&E[lane & 15][k0]);
      const float4_t by = *reinterpret_cast<const float4_t *>(&E[16 + (lane & 7)][k0]);
      if constexpr (F32MAC) {
        // FP32 products: four 16x16x4 FP32 MFMAs per column block, the j-th
        // taking element j of every lane's four staged particles (so the
        // four cover the step's 16 particles; A and B use the same order)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const float4_t bz = *reinterpret_cast<const float4_t *>(&E[24 + 2 * nb + ((lane >> 3) & 1)][k0]);
          const float4_t b = by * bz;
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[j], acc[nb], 0, 0, 0);
        }
      } else {
        half4_t ah, al;
        split_f16(a, ah, al);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const float4_t bz = *reinterpret_cast<const float4_t *>(&E[24 + 2 * nb + ((lane >> 3) & 1)][k0]);
          half4_t bh, bl;
          split_f16(by * bz, bh, bl);
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bh, acc[nb], 0, 0, 0);
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bl, acc[nb], 0, 0, 0);
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16f16(al, bh, acc[nb], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // partial tiles of the four waves -> LDS [wave][z][y][x], summed and written
  float *red = &E[0][0];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int y = lane & 7, z = 2 * nb + ((lane >> 3) & 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x = 4 * (lane >> 4) + r;
      red[wv * 1024 + (z * 8 + y) * 16 + x] = acc[nb][r];
    }
  }
  __syncthreads();
  const float out_scale = ldexpf(1.0f, qe);
  for (int e = tid; e < 1024; e += blockDim.x) {
    const int x = e & 15, y = (e >> 4) & 7, z = e >> 7;
    if (x < g.T[0] && y < g.T[1] && z < g.T[2]) {
      const float v = (red[e] + red[1024 + e]) + (red[2048 + e] + red[3072 + e]);
      grid[((size_t)(t0[2] + z) * g.M[1] + (t0[1] + y)) * g.M[0] + t0[0] + x] = v * out_scale;
    }
  }
}

// --------------------------------------------------------------------------
// FFT pencils.  A pencil of length n = 2^ln is transformed by one to three
// Stockham autosort stages of radix 16, 8 or 4 whose butterflies keep their
// RAD inputs in registers: a stage reads and writes each element once.
// Stage (radix RAD, span Ns = product of the earlier radices): butterfly j,
// k = j mod Ns, takes elements j + r n/RAD (r < RAD), multiplies element r
// by exp(DIR 2 pi i r k / (Ns RAD)), applies the RAD-point DFT and writes
// output r to (j - k) RAD + k + r Ns.  The first stage reads through a
// caller-supplied loader and the last writes through a storer (global memory
// or LDS); intermediate stages go through LDS, element i of pencil f of
// batch o at buf[(o n + i) ld + f] so neighbouring lanes (consecutive f)
// touch neighbouring words.  tw[m] = exp(-2 pi i m / n).  DIR = -1 forward,
// +1 inverse (unnormalised).
// --------------------------------------------------------------------------
constexpr double kCos16[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                              0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
constexpr double kSin16[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                              1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};

// a * exp(DIR 2 pi i E / 16)
template <typename R, int DIR, int E>
__device__ __forceinline__ Cx<R> wmul16(Cx<R> a) {
  constexpr int e = ((E % 16) + 16) % 16;
  if constexpr (e == 0) {
    return a;
  } else if constexpr (e == 4) {
    return cmuli<R, DIR>(a);
  } else if constexpr (e == 8) {
    return Cx<R>{-a.x, -a.y};
  } else if constexpr (e == 12) {
    return cmuli<R, -DIR>(a);
  } else if constexpr (e > 8) {
    const Cx<R> b = wmul16<R, DIR, e - 8>(a);
    return Cx<R>{-b.x, -b.y};
  } else {
    const R c = (R)kCos16[e], s = (R)(DIR * kSin16[e]);
    return Cx<R>{a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

template <typename R, int DIR>
__device__ __forceinline__ void dft4(Cx<R> &a0, Cx<R> &a1, Cx<R> &a2, Cx<R> &a3) {
  const Cx<R> s02 = cadd(a0, a2), d02 = csub(a0, a2), s13 = cadd(a1, a3);
  const Cx<R> id13 = cmuli<R, DIR>(csub(a1, a3));
  a0 = cadd(s02, s13);
  a1 = cadd(d02, id13);
  a2 = csub(s02, s13);
  a3 = csub(d02, id13);
}

// RAD-point DFT in place, natural order in and out
template <typename R, int RAD, int DIR>
__device__ __forceinline__ void dft(Cx<R> (&v)[RAD]) {
  if constexpr (RAD == 4) {
    dft4<R, DIR>(v[0], v[1], v[2], v[3]);
  } else if constexpr (RAD == 8) {
    // even / odd halves, then X_k = E_k + W8^k O_k, X_{k+4} = E_k - W8^k O_k
    Cx<R> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    Cx<R> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<R, DIR>(e0, e1, e2, e3);
    dft4<R, DIR>(o0, o1, o2, o3);
    o1 = wmul16<R, DIR, 2>(o1);
    o2 = wmul16<R, DIR, 4>(o2);
    o3 = wmul16<R, DIR, 6>(o3);
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
  } else {
    static_assert(RAD == 16, "radix 4, 8 or 16");
    // 4 x 4: index n = n2 + 4 n1, k = k1 + 4 k2.  Columns (fixed n2) first,
    // twiddle W16^(n2 k1), then rows (fixed k1); row k1 output k2 is X_{k1+4k2}.
    dft4<R, DIR>(v[0], v[4], v[8], v[12]);
    dft4<R, DIR>(v[1], v[5], v[9], v[13]);
    dft4<R, DIR>(v[2], v[6], v[10], v[14]);
    dft4<R, DIR>(v[3], v[7], v[11], v[15]);
    v[5] = wmul16<R, DIR, 1>(v[5]);
    v[9] = wmul16<R, DIR, 2>(v[9]);
    v[13] = wmul16<R, DIR, 3>(v[13]);
    v[6] = wmul16<R, DIR, 2>(v[6]);
    v[10] = wmul16<R, DIR, 4>(v[10]);
    v[14] = wmul16<R, DIR, 6>(v[14]);
    v[7] = wmul16<R, DIR, 3>(v[7]);
    v[11] = wmul16<R, DIR, 6>(v[11]);
    v[15] = wmul16<R, DIR, 9>(v[15]);
    Cx<R> t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      Cx<R> a0 = v[4 * k1], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
      dft4<R, DIR>(a0, a1, a2, a3);
      t[k1] = a0;
      t[k1 + 4] = a1;
      t[k1 + 8] = a2;
      t[k1 + 12] = a3;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = t[i];
  }
}

template <typename R, int RAD, int DIR, class LD, class ST>
__device__ __forceinline__ void fft_stage(int ln, int lns, int lnb, int nrep, const Cx<R> *__restrict__ tw, LD ld,
                                          ST st) {
  constexpr int LR = RAD == 16 ? 4 : (RAD == 8 ? 3 : 2);
  const int lq = ln - LR;  // log2 of butterflies per pencil
  const int lt = ln - lns - LR;
  const int total = nrep << (lq + lnb);
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    const int f = w & ((1 << lnb) - 1);
    const int t = w >> lnb;
    const int j = t & ((1 << lq) - 1);
    const int o = t >> lq;
    const int k = j & ((1 << lns) - 1);
    Cx<R> v[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) v[r] = ld(o, j + (r << lq), f);
    if (lns > 0) {
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        Cx<R> wr = tw[(r * k) << lt];
        if (DIR > 0) wr = cconj(wr);
        v[r] = cmul(v[r], wr);
      }
    }
    dft<R, RAD, DIR>(v);
    const int ob = ((j - k) << LR) + k;
#pragma unroll
    for (int r = 0; r < RAD; ++r) st(o, ob + (r << lns), f, v[r]);
  }
}

__host__ __device__ constexpr int fft_nstages(int ln) { return ln <= 4 ? 1 : (ln <= 8 ? 2 : 3); }

// Runs the stages for length 2^ln (ln in 2..10) over nrep batches of 2^lnb
// pencils.  Stage 0 reads through `first`, the last stage writes through
// `last`; stage 0 / stage 1 outputs (when not last) go to LDS X / Y with
// pencil stride ldp.  Barriers separate the stages; the caller synchronises
// before the first and after the last.
template <typename R, int DIR, class LD, class ST>
__device__ void fft_run(int ln, int lnb, int nrep, const Cx<R> *__restrict__ tw, Cx<R> *X, Cx<R> *Y, int ldp,
                        LD first, ST last) {
  auto ldX = [=](int o, int i, int f) { return X[((o << ln) + i) * ldp + f]; };
  auto stX = [=](int o, int i, int f, Cx<R> v) { X[((o << ln) + i) * ldp + f] = v; };
  auto ldY = [=](int o, int i, int f) { return Y[((o << ln) + i) * ldp + f]; };
  auto stY = [=](int o, int i, int f, Cx<R> v) { Y[((o << ln) + i) * ldp + f] = v; };
  switch (ln) {
    case 2: fft_stage<R, 4, DIR>(ln, 0, lnb, nrep, tw, first, last); break;
    case 3: fft_stage<R, 8, DIR>(ln, 0, lnb, nrep, tw, first, last); break;
    case 4: fft_stage<R, 16, DIR>(ln, 0, lnb, nrep, tw, first, last); break;
    case 5:
      fft_stage<R, 8, DIR>(ln, 0, lnb, nrep, tw, first, stX);
      __syncthreads();
      fft_stage<R, 4, DIR>(ln, 3, lnb, nrep, tw, ldX, last);
      break;
    case 6:
      fft_stage<R, 8, DIR>(ln, 0, lnb, nrep, tw, first, stX);
      __syncthreads();
      fft_stage<R, 8, DIR>(ln, 3, lnb, nrep, tw, ldX, last);
      break;
    case 7:
      fft_stage<R, 16, DIR>(ln, 0, lnb, nrep, tw, first, stX);
      __syncthreads();
      fft_stage<R, 8, DIR>(ln, 4, lnb, nrep, tw, ldX, last);
      break;
    case 8:
      fft_stage<R, 16, DIR>(ln, 0, lnb, nrep, tw, first, stX);
      __syncthreads();
      fft_stage<R, 16, DIR>(ln, 4, lnb, nrep, tw, ldX, last);
      break;
    case 9:
      fft_stage<R, 8, DIR>(ln, 0, lnb, nrep, tw, first, stX);
      __syncthreads();
      fft_stage<R, 8, DIR>(ln, 3, lnb, nrep, tw, ldX, stY);
      __syncthreads();
      fft_stage<R, 8, DIR>(ln, 6, lnb, nrep, tw, ldY, last);
      break;
    default:
      fft_stage<R, 16, DIR>(ln, 0, lnb, nrep, tw, first, stX);
      __syncthreads();
      fft_stage<R, 8, DIR>(ln, 4, lnb, nrep, tw, ldX, stY);
      __syncthreads();
      fft_stage<R, 8, DIR>(ln, 7, lnb, nrep, tw, ldY, last);
      break;
  }
}

// x pass, forward: each row of Mx reals -> bins 0 .. Mx/2-1 (the Nyquist bin
// is not kept: those modes are outside the k-set).  The row is packed as
// z_j = x_{2j} + i x_{2j+1}, transformed at length n = Mx/2 and untangled:
// X_k = (Z_k + conj Z_{n-k})/2 - (i/2) e^{-2 pi i k/Mx} (Z_k - conj Z_{n-k}).
// A block takes 2^lnb rows; LDS pencil stride ldp (odd when > 1) keeps the
// row <-> pencil transposes free of bank conflicts.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_fft_x_r2c(const R *__restrict__ grid, Cx<R> *__restrict__ spec,
                                                      int lnh, int lnb, const Cx<R> *__restrict__ tw_n,
                                                      const Cx<R> *__restrict__ tw_2n) {
  extern __shared__ unsigned char smem_raw[];
  const int n = 1 << lnh, nb = 1 << lnb;
  const int ldp = nb == 1 ? 1 : nb + 1;
  Cx<R> *B0 = reinterpret_cast<Cx<R> *>(smem_raw);
  Cx<R> *B1 = B0 + n * ldp;
  const size_t row0 = (size_t)blockIdx.x * nb;
  const Cx<R> *src = reinterpret_cast<const Cx<R> *>(grid) + (row0 << lnh);
  for (int e0 = threadIdx.x; e0 < (n << lnb); e0 += 4 * blockDim.x) {
    using V = pod_t<Cx<R>>;
    V v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = e0 + k * blockDim.x;
      v[k] = V{};
      if (e < (n << lnb)) v[k] = reinterpret_cast<const V *>(src)[e];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = e0 + k * blockDim.x;
      if (e < (n << lnb)) reinterpret_cast<V *>(B0)[(e & (n - 1)) * ldp + (e >> lnh)] = v[k];
    }
  }
  __syncthreads();
  Cx<R> *res = (fft_nstages(lnh) & 1) ? B1 : B0;
  fft_run<R, -1>(lnh, lnb, 1, tw_n, B1, B0, ldp, [=](int, int i, int f) { return B0[i * ldp + f]; },
                 [=](int, int i, int f, Cx<R> v) { res[i * ldp + f] = v; });
  __syncthreads();
  Cx<R> *dst = spec + (row0 << lnh);
  for (int e = threadIdx.x; e < (n << lnb); e += blockDim.x) {
    const int f = e >> lnh, k = e & (n - 1);
    const Cx<R> zk = res[k * ldp + f];
    const Cx<R> zm = cconj(res[((n - k) & (n - 1)) * ldp + f]);
    const Cx<R> s = cadd(zk, zm), d = csub(zk, zm);
    const Cx<R> wd = cmul(tw_2n[k], d);
    // X = s/2 - (i/2) w d
    dst[e] = Cx<R>{R(0.5) * (s.x + wd.y), R(0.5) * (s.y - wd.x)};
  }
}

// Complex pencils along y (length 2^ln, element stride 2^linner: x is the
// contiguous dimension), in place; a block takes 2^lnb consecutive pencils.
// blockIdx.x: pencil block, blockIdx.y: z plane, blockIdx.z: component.
template <typename R, int DIR>
__global__ __launch_bounds__(kBlock) void k_fft_y(Cx<R> *data, int ln, int linner, size_t plane_stride,
                                                  size_t comp_stride, const Cx<R> *__restrict__ tw, int lnb) {
  extern __shared__ unsigned char smem_raw[];
  const int nb = 1 << lnb;
  Cx<R> *X = reinterpret_cast<Cx<R> *>(smem_raw);
  Cx<R> *Y = X + (nb << ln);
  Cx<R> *base = data + blockIdx.z * comp_stride + blockIdx.y * plane_stride + ((size_t)blockIdx.x << lnb);
  fft_run<R, DIR>(ln, lnb, 1, tw, X, Y, nb, [=](int, int i, int f) { return base[((size_t)i << linner) + f]; },
                  [=](int, int i, int f, Cx<R> v) { base[((size_t)i << linner) + f] = v; });
}

// One Stockham stage in place in LDS (element i of pencil f at X[i nb + f]):
// every butterfly of the stage has its own thread (n / RAD * nb <= blockDim),
// which reads its inputs, waits for the whole block, then writes its outputs.
// Every thread of the block must call it.
template <typename R, int RAD, int DIR>
__device__ __forceinline__ void fft_stage_ip(int ln, int lns, int lnb, const Cx<R> *__restrict__ tw, Cx<R> *X) {
  constexpr int LR = RAD == 16 ? 4 : (RAD == 8 ? 3 : 2);
  const int lq = ln - LR;
  const int lt = ln - lns - LR;
  const int w = threadIdx.x;
  const bool act = w < (1 << (lq + lnb));
  const int f = w & ((1 << lnb) - 1);
  const int j = (w >> lnb) & ((1 << lq) - 1);
  const int k = j & ((1 << lns) - 1);
  Cx<R> v[RAD];
  if (act) {
#pragma unroll
    for (int r = 0; r < RAD; ++r) v[r] = X[((j + (r << lq)) << lnb) + f];
    if (lns > 0) {
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        Cx<R> wr = tw[(r * k) << lt];
        if (DIR > 0) wr = cconj(wr);
        v[r] = cmul(v[r], wr);
      }
    }
    dft<R, RAD, DIR>(v);
  }
  __syncthreads();
  if (act) {
    const int ob = ((j - k) << LR) + k;
#pragma unroll
    for (int r = 0; r < RAD; ++r) X[((ob + (r << lns)) << lnb) + f] = v[r];
  }
}

// The same stage with post(v, ob) applied to the butterfly's outputs (in
// registers, before they are written back): output r goes to element
// ob + (r << lns).
template <typename R, int RAD, int DIR, typename Post>
__device__ __forceinline__ void fft_stage_ip_post(int ln, int lns, int lnb, const Cx<R> *__restrict__ tw, Cx<R> *X,
                                                  Post post) {
  constexpr int LR = RAD == 16 ? 4 : (RAD == 8 ? 3 : 2);
  const int lq = ln - LR;
  const int lt = ln - lns - LR;
  const int w = threadIdx.x;
  const bool act = w < (1 << (lq + lnb));
  const int f = w & ((1 << lnb) - 1);
  const int j = (w >> lnb) & ((1 << lq) - 1);
  const int k = j & ((1 << lns) - 1);
  const int ob = ((j - k) << LR) + k;
  Cx<R> v[RAD];
  if (act) {
#pragma unroll
    for (int r = 0; r < RAD; ++r) v[r] = X[((j + (r << lq)) << lnb) + f];
    if (lns > 0) {
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        Cx<R> wr = tw[(r * k) << lt];
        if (DIR > 0) wr = cconj(wr);
        v[r] = cmul(v[r], wr);
      }
    }
    dft<R, RAD, DIR>(v);
    post(v, ob);
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < RAD; ++r) X[((ob + (r << lns)) << lnb) + f] = v[r];
  }
}

// z pass for a single field from the potential spectrum (analytic forces),
// lengths 128 and 256 (two stages): one LDS buffer of n x 16 pencils holds
// the spectrum throughout (stages in place), so a block reads and writes
// 128-byte rows and every thread owns a butterfly.  Same results as
// k_z_fused with nf = 1, fbase = 3.
// One in-place Stockham stage (radix RAD, span 2^lns) over a 2^ln-point
// transform of 2^lnb pencils held in X, with PER butterflies per thread: all
// of a thread's inputs are read, the block waits, then the outputs are
// written.
template <typename R, int RAD, int DIR, int PER>
__device__ __forceinline__ void fft_stage_ip_n(int ln, int lns, int lnb, const Cx<R> *__restrict__ tw, Cx<R> *X) {
  constexpr int LR = RAD == 16 ? 4 : (RAD == 8 ? 3 : (RAD == 4 ? 2 : 1));
  const int lq = ln - LR;
  const int lt = ln - lns - LR;
  Cx<R> v[PER][RAD];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int w = threadIdx.x + i * blockDim.x;
    const int f = w & ((1 << lnb) - 1);
    const int j = (w >> lnb) & ((1 << lq) - 1);
    const int k = j & ((1 << lns) - 1);
#pragma unroll
    for (int r = 0; r < RAD; ++r) v[i][r] = X[((j + (r << lq)) << lnb) + f];
    if (lns > 0) {
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        Cx<R> wr = tw[(r * k) << lt];
        if (DIR > 0) wr = cconj(wr);
        v[i][r] = cmul(v[i][r], wr);
      }
    }
    if constexpr (RAD == 2) {
      const Cx<R> a = v[i][0], b = v[i][1];
      v[i][0] = cadd(a, b);
      v[i][1] = csub(a, b);
    } else {
      dft<R, RAD, DIR>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int w = threadIdx.x + i * blockDim.x;
    const int f = w & ((1 << lnb) - 1);
    const int j = (w >> lnb) & ((1 << lq) - 1);
    const int k = j & ((1 << lns) - 1);
    const int ob = ((j - k) << LR) + k;
#pragma unroll
    for (int r = 0; r < RAD; ++r) X[((ob + (r << lns)) << lnb) + f] = v[i][r];
  }
}

// The z pass of the potential spectrum alone for 512-point z axes (FP32,
// analytic forces): 16 pencils per block in one 64 KB LDS buffer, 512
// threads; forward stages of radix 16, 16, 2 (the first reads global memory
// in rows of 16 pencils), the influence multiply and the energy partial, and
// inverse stages of radix 2, 16, 16 (the last writes global memory).  The
// block's energy partial is reduced through the same buffer once it is
// free, so the block needs no other LDS.
template <typename R>
__global__ __launch_bounds__(512) void k_z_psi512(const Cx<R> *__restrict__ spec, Cx<R> *__restrict__ fspec,
                                                  Geom g, int lhx, const Cx<R> *__restrict__ tw_z,
                                                  const R *__restrict__ sx, const R *__restrict__ sy,
                                                  const R *__restrict__ sz, const R *__restrict__ kvx,
                                                  const R *__restrict__ kvy, const R *__restrict__ kvz,
                                                  double *eslot) {
  constexpr int lnz = 9, n = 512, lnb = 4, nb = 16;
  extern __shared__ unsigned char smem_raw[];
  Cx<R> *X = reinterpret_cast<Cx<R> *>(smem_raw);
  const int hx = 1 << lhx;
  const size_t inner = (size_t)hx * g.M[1];
  const size_t p0 = (size_t)blockIdx.x << lnb;
  const int tid = threadIdx.x;
  const int f = tid & (nb - 1), j = tid >> lnb;  // pencil, butterfly (0..31) of a radix-16 stage
  // forward: radix 16 (span 1) from global memory
  {
    Cx<R> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = spec[(size_t)(j + (r << 5)) * inner + p0 + f];
    dft<R, 16, -1>(v);
#pragma unroll
    for (int r = 0; r < 16; ++r) X[((j * 16 + r) << lnb) + f] = v[r];
  }
  __syncthreads();
  fft_stage_ip_n<R, 16, -1, 1>(lnz, 4, lnb, tw_z, X);
  __syncthreads();
  // last forward stage (radix 2, span 256), influence and energy, first
  // inverse stage (radix 2, span 1) on the same registers: forward
  // butterfly jb leaves elements jb and jb + 256 in natural order, which
  // are the inverse butterfly jb's inputs; it writes elements 2 jb, 2 jb + 1
  double en = 0.0;
  {
    const int pidx = (int)p0 + f;
    const int kx = pidx & (hx - 1), ky = pidx >> lhx;
    const R kxy2 = kvx[kx] * kvx[kx] + kvy[ky] * kvy[ky];
    const R sxy = sx[kx] * sy[ky];
    const R wk = kx > 0 ? R(2) : R(1);
    Cx<R> a[8], b[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int jb = (tid >> lnb) + 32 * t;  // butterfly 0..255 of pencil f
      a[t] = X[(jb << lnb) + f];
      b[t] = cmul(X[((jb + 256) << lnb) + f], tw_z[jb]);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int jb = (tid >> lnb) + 32 * t;
      Cx<R> u0 = cadd(a[t], b[t]), u1 = csub(a[t], b[t]);  // kz = jb, jb + 256
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        Cx<R> &u = r == 0 ? u0 : u1;
        const int kz = jb + 256 * r;
        const R k2 = kxy2 + kvz[kz] * kvz[kz];
        const R gv = k2 > R(0) ? sxy * sz[kz] * recip_r(k2) : R(0);
        en += (double)(wk * gv * (u.x * u.x + u.y * u.y));
        u = Cx<R>{gv * u.x, gv * u.y};
      }
      a[t] = cadd(u0, u1);
      b[t] = csub(u0, u1);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int jb = (tid >> lnb) + 32 * t;
      X[((2 * jb) << lnb) + f] = a[t];
      X[((2 * jb + 1) << lnb) + f] = b[t];
    }
  }
  __syncthreads();
  // inverse: radix 16 (span 2) in place
  fft_stage_ip_n<R, 16, 1, 1>(lnz, 1, lnb, tw_z, X);
  __syncthreads();
  // last stage: radix 16, span 32, to global memory
  {
    const int k = j & 31;
    const int ob = ((j - k) << 4) + k;
    Cx<R> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = X[((j + (r << 5)) << lnb) + f];
#pragma unroll
    for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], cconj(tw_z[r * k]));
    dft<R, 16, 1>(v);
#pragma unroll
    for (int r = 0; r < 16; ++r) fspec[(size_t)(ob + (r << 5)) * inner + p0 + f] = v[r];
  }
  // energy partial: wave sums, then the waves' sums through the freed buffer
  en = wave_sum(en);
  __syncthreads();  // every thread has read X
  double *red = reinterpret_cast<double *>(smem_raw);
  if ((tid & 63) == 0) red[tid >> 6] = en;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) tot += red[k];
    // deterministic mode: one slot per block, summed in a fixed order
    if (g.det) eslot[blockIdx.x] = tot;
    else atomicAdd(&eslot[blockIdx.x % kESlots], tot);
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_z_psi(const Cx<R> *__restrict__ spec, Cx<R> *__restrict__ fspec, Geom g,
                                                  int lnz, int lhx, const Cx<R> *__restrict__ tw_z,
                                                  const R *__restrict__ sx, const R *__restrict__ sy,
                                                  const R *__restrict__ sz, const R *__restrict__ kvx,
                                                  const R *__restrict__ kvy, const R *__restrict__ kvz,
                                                  double *eslot) {
  constexpr int lnb = 4, nb = 16;
  extern __shared__ unsigned char smem_raw[];
  Cx<R> *X = reinterpret_cast<Cx<R> *>(smem_raw);
  const int n = 1 << lnz, hx = 1 << lhx;
  const size_t inner = (size_t)hx * g.M[1];
  const size_t p0 = (size_t)blockIdx.x << lnb;
  const int L1 = lnz == 8 ? 4 : 3;  // second stage radix 16 (n = 256) or 8 (n = 128)
  // forward: radix-16 stage from global memory into X, then the second stage in place
  {
    constexpr int LR = 4;
    const int lq = lnz - LR;
    const int w = threadIdx.x;
    const bool act = w < (1 << (lq + lnb));
    const int f = w & (nb - 1), j = (w >> lnb) & ((1 << lq) - 1);
    Cx<R> v[16];
    if (act) {
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = spec[(size_t)(j + (r << lq)) * inner + p0 + f];
      dft<R, 16, -1>(v);
#pragma unroll
      for (int r = 0; r < 16; ++r) X[((j * 16 + r) << lnb) + f] = v[r];
    }
  }
  __syncthreads();
  // second forward stage; its outputs (element kz = ob + 16 r of pencil f,
  // in natural order) take the influence factor and give their energy
  // before they are written back
  double en = 0.0;
  {
    const int f = threadIdx.x & (nb - 1);
    const int pidx = (int)p0 + f;
    const int kx = pidx & (hx - 1), ky = pidx >> lhx;
    const R kxy2 = kvx[kx] * kvx[kx] + kvy[ky] * kvy[ky];
    const R sxy = sx[kx] * sy[ky];
    const R wk = kx > 0 ? R(2) : R(1);
    auto scale = [&](auto &v, int ob) {
      constexpr int RAD = sizeof(v) / sizeof(v[0]);
#pragma unroll
      for (int r = 0; r < RAD; ++r) {
        const int kz = ob + (r << 4);
        const R k2 = kxy2 + kvz[kz] * kvz[kz];
        const R gv = k2 > R(0) ? sxy * sz[kz] * recip_r(k2) : R(0);
        en += (double)(wk * gv * (v[r].x * v[r].x + v[r].y * v[r].y));
        v[r] = Cx<R>{gv * v[r].x, gv * v[r].y};
      }
    };
    if (L1 == 4) {
      // n = 256: the second forward stage leaves a thread elements j + 16 r,
      // exactly the inputs of the first inverse (radix-16, span-1) stage's
      // butterfly j, so both run on the same registers: read, twiddle,
      // forward DFT, influence, inverse DFT, then write elements 16 j + r
      const int w = threadIdx.x;
      const int f = w & (nb - 1), j = (w >> lnb) & 15;
      Cx<R> v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = X[((j + (r << 4)) << lnb) + f];
#pragma unroll
      for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], tw_z[r * j]);
      dft<R, 16, -1>(v);
      scale(v, j);
      dft<R, 16, 1>(v);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) X[(((j << 4) + r) << lnb) + f] = v[r];
    } else {
      fft_stage_ip_post<R, 8, -1>(lnz, 4, lnb, tw_z, X, scale);
      __syncthreads();
      // inverse: first stage in place
      fft_stage_ip<R, 16, 1>(lnz, 0, lnb, tw_z, X);
    }
  }
  __syncthreads();
  // inverse: the second stage writes global memory
  {
    const int LR = L1;
    const int lq = lnz - LR;
    const int lt = lnz - 4 - LR;
    const int w = threadIdx.x;
    const bool act = w < (1 << (lq + lnb));
    const int f = w & (nb - 1), j = (w >> lnb) & ((1 << lq) - 1);
    const int k = j & 15;
    if (act) {
      const int ob = ((j - k) << LR) + k;
      if (L1 == 4) {
        Cx<R> v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = X[((j + (r << lq)) << lnb) + f];
#pragma unroll
        for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], cconj(tw_z[(r * k) << lt]));
        dft<R, 16, 1>(v);
#pragma unroll
        for (int r = 0; r < 16; ++r) fspec[(size_t)(ob + (r << 4)) * inner + p0 + f] = v[r];
      } else {
        Cx<R> v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = X[((j + (r << lq)) << lnb) + f];
#pragma unroll
        for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], cconj(tw_z[(r * k) << lt]));
        dft<R, 8, 1>(v);
#pragma unroll
        for (int r = 0; r < 8; ++r) fspec[(size_t)(ob + (r << 4)) * inner + p0 + f] = v[r];
      }
    }
  }
  const double tot = block_sum(en);
  // deterministic mode: one slot per block, summed in a fixed order
  if (threadIdx.x == 0) {
    if (g.det) eslot[blockIdx.x] = tot;
    else atomicAdd(&eslot[blockIdx.x % kESlots], tot);
  }
}

// z pass fused with the scaling and influence steps.  For each pencil
// (kx, ky): forward transform along z; then for every mode n in the k-set
//   g(n) = A(k) / c(n)^2,  A = exp(-k^2/4a^2)/k^2,  c = window transform,
// which factorises as s_x(kx) s_y(ky) s_z(kz) / k^2 with
// s_d = exp(-k_d^2/4a^2) / c_d^2 (zero at the Nyquist index);
// energy += w_x g |rho^|^2 (w_x = 2 for kx > 0: the mirrored half),
// field spectra E^_d = -i k_d g rho^ (d = x,y,z) and psi^ = g rho^, each
// transformed back along z and written to fspec[d].  The nf field pencils
// (field ids fbase .. fbase+nf-1, id 3 = psi) are transformed as batches of
// nfp (nf or 1) at a time.
// tab: s_x (Mx/2), s_y (My), s_z (Mz), k_x (Mx/2), k_y (My), k_z (Mz).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_z_fused(const Cx<R> *__restrict__ spec, Cx<R> *__restrict__ fspec,
                                                    Geom g, int lnz, int lhx, int lnb, int nf, int nfp, int fbase,
                                                    const Cx<R> *__restrict__ tw_z, const R *__restrict__ sx,
                                                    const R *__restrict__ sy, const R *__restrict__ sz,
                                                    const R *__restrict__ kvx, const R *__restrict__ kvy,
                                                    const R *__restrict__ kvz, double *eslot) {
  extern __shared__ unsigned char smem_raw[];
  const int n = 1 << lnz, nb = 1 << lnb, hx = 1 << lhx;
  const size_t inner = (size_t)hx * g.M[1];
  const size_t half = inner << lnz;
  const int nst = fft_nstages(lnz);
  Cx<R> *S = reinterpret_cast<Cx<R> *>(smem_raw);  // n x nb, the (scaled) spectrum
  Cx<R> *X = S + (n << lnb);                        // nfp x n x nb when nst >= 2
  Cx<R> *Y = X + (nst >= 2 ? (nfp << (lnz + lnb)) : 0);
  const size_t p0 = (size_t)blockIdx.x << lnb;
  fft_run<R, -1>(lnz, lnb, 1, tw_z, X, Y, nb, [=](int, int i, int f) { return spec[i * inner + p0 + f]; },
                 [=](int, int i, int f, Cx<R> v) { S[i * nb + f] = v; });
  __syncthreads();
  double en = 0.0;
  {
    // a thread keeps one pencil f (blockDim is a multiple of nb), so its x
    // and y factors are loaded once
    const int f = threadIdx.x & (nb - 1);
    const int pidx = (int)p0 + f;
    const int kx = pidx & (hx - 1), ky = pidx >> lhx;
    const R kxy2 = kvx[kx] * kvx[kx] + kvy[ky] * kvy[ky];
    const R sxy = sx[kx] * sy[ky];
    const R wk = kx > 0 ? R(2) : R(1);  // the x half spectrum counts the other half too
    for (int kz = threadIdx.x >> lnb; kz < n; kz += blockDim.x >> lnb) {
      const int e = (kz << lnb) + f;
      const R k2 = kxy2 + kvz[kz] * kvz[kz];
      const R gv = k2 > R(0) ? sxy * sz[kz] * recip_r(k2) : R(0);
      const Cx<R> r = S[e];
      en += (double)(wk * gv * (r.x * r.x + r.y * r.y));
      S[e] = Cx<R>{gv * r.x, gv * r.y};
    }
  }
  __syncthreads();
  for (int o0 = 0; o0 < nf; o0 += nfp) {
    fft_run<R, 1>(
        lnz, lnb, nfp, tw_z, X, Y, nb,
        [=](int o, int i, int f) {
          const Cx<R> v = S[i * nb + f];
          const int c = fbase + o0 + o;
          if (c == 3) return v;
          const int pidx = (int)p0 + f;
          const R kd = c == 0 ? kvx[pidx & (hx - 1)] : (c == 1 ? kvy[pidx >> lhx] : kvz[i]);
          return Cx<R>{kd * v.y, -kd * v.x};  // -i k_d v
        },
        [=](int o, int i, int f, Cx<R> v) { fspec[(o0 + o) * half + i * inner + p0 + f] = v; });
    __syncthreads();
  }
  const double tot = block_sum(en);
  // deterministic mode: one slot per block, summed in a fixed order
  if (threadIdx.x == 0) {
    if (g.det) eslot[blockIdx.x] = tot;
    else atomicAdd(&eslot[blockIdx.x % kESlots], tot);
  }
}

// x pass, inverse, nf components: bins 0 .. Mx/2-1 of each field (Nyquist
// bin zero) -> Mx reals, written interleaved as real4 (E_x, E_y, E_z, psi),
// or, for a single field (SCALAR), as a plain real grid.
// Z_k = (X_k + conj X_{n-k}) + i e^{+2 pi i k/Mx} (X_k - conj X_{n-k}),
// z = inverse transform (length n), x_{2j} = Re z_j, x_{2j+1} = Im z_j.
// The untangling is folded into the first stage's loads.
template <typename R, bool SCALAR>
__global__ __launch_bounds__(kBlock) void k_fft_x_c2r4(const Cx<R> *__restrict__ fspec, void *__restrict__ field_out,
                                                       Geom g, int lnh, int lnb, int nf,
                                                       const Cx<R> *__restrict__ tw_n,
                                                       const Cx<R> *__restrict__ tw_2n) {
  extern __shared__ unsigned char smem_raw[];
  const int n = 1 << lnh, nb = 1 << lnb, Mx = 2 * n;
  const int ldp = nb == 1 ? 1 : nb + 1;
  const size_t half = ((size_t)g.M[1] * g.M[2]) << lnh;
  Cx<R> *B0 = reinterpret_cast<Cx<R> *>(smem_raw);
  Cx<R> *B1 = B0 + nf * n * ldp;
  const size_t row0 = (size_t)blockIdx.x * nb;
  for (int e0 = threadIdx.x; e0 < ((nf * n) << lnb); e0 += 4 * blockDim.x) {
    using V = pod_t<Cx<R>>;
    V v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * blockDim.x;
      v[u] = V{};
      if (e < ((nf * n) << lnb)) {
        const int k = e & (n - 1), t = e >> lnh;
        const int f = t & (nb - 1), o = t >> lnb;
        v[u] = reinterpret_cast<const V *>(fspec)[o * half + ((row0 + f) << lnh) + k];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * blockDim.x;
      if (e < ((nf * n) << lnb)) {
        const int k = e & (n - 1), t = e >> lnh;
        const int f = t & (nb - 1), o = t >> lnb;
        reinterpret_cast<V *>(B0)[(o * n + k) * ldp + f] = v[u];
      }
    }
  }
  __syncthreads();
  Cx<R> *res = (fft_nstages(lnh) & 1) ? B1 : B0;
  fft_run<R, 1>(
      lnh, lnb, nf, tw_n, B1, B0, ldp,
      [=](int o, int k, int f) {
        const Cx<R> xk = B0[(o * n + k) * ldp + f];
        const Cx<R> xm = k == 0 ? Cx<R>{R(0), R(0)} : cconj(B0[(o * n + n - k) * ldp + f]);
        const Cx<R> s = cadd(xk, xm), d = csub(xk, xm);
        const Cx<R> wd = cmul(cconj(tw_2n[k]), d);
        return Cx<R>{s.x - wd.y, s.y + wd.x};  // s + i wd
      },
      [=](int o, int i, int f, Cx<R> v) { res[(o * n + i) * ldp + f] = v; });
  __syncthreads();
  if constexpr (SCALAR) {
    // one field: a plain real grid; z_j holds the reals x_{2j}, x_{2j+1}
    Cx<R> *dst = reinterpret_cast<Cx<R> *>(reinterpret_cast<R *>(field_out) + row0 * Mx);
    for (int e = threadIdx.x; e < (nb << lnh); e += blockDim.x) {
      const int j = e & (n - 1), f = e >> lnh;
      dst[e] = res[j * ldp + f];
    }
    return;
  }
  real4<R> *dst = reinterpret_cast<real4<R> *>(field_out) + row0 * Mx;
  for (int e = threadIdx.x; e < (nb * Mx); e += blockDim.x) {
    const int xi = e & (Mx - 1), f = e >> (lnh + 1);
    const int j = xi >> 1;
    const bool odd = xi & 1;
    R c[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      if (o < nf) {
        const Cx<R> v = res[(o * n + j) * ldp + f];
        c[o] = odd ? v.y : v.x;
      } else {
        c[o] = R(0);
      }
    }
    real4<R> v;
    v.x = c[0];
    v.y = c[1];
    v.z = c[2];
    v.w = c[3];
    dst[e] = v;
  }
}
// --------------------------------------------------------------------------
// gather: type-2 interpolation of the four fields (Eq. 35, 42), one thread per
// active particle in tile order; results scattered to the caller's order.
//   F_i   = pref q_i sum_l B(s_i - l) (E_x, E_y, E_z)_l,  pref = ke 4 pi / V
//   phi_i = pref     sum_l B(s_i - l) psi_l
// GRAD: exact gradient of the discrete energy instead,
//   dE/dr_i,d = pref q_i (M_d/L_d) sum_l dB/ds_d psi_l,  dE/dq_i = phi_i.
// --------------------------------------------------------------------------
template <typename R, int P, bool GRAD, typename FT>
__global__ __launch_bounds__(kGatherBlock) void k_gather(const real4<R> *__restrict__ part,
                                                         const int *__restrict__ perm,
                                                         const int *__restrict__ counts, Geom g,
                                                         const FT *__restrict__ field, R pref, R gscale,
                                                         R sscale, R *__restrict__ vec_out,
                                                         R *__restrict__ sca_out) {
  // per-thread y/z weights live in LDS so the (z, y) row loop can stay rolled
  // without indexing registers dynamically; only the x sweep is unrolled
  __shared__ R wsh[kGatherBlock][GRAD ? 4 : 2][P];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= counts[0]) return;
  R(*ws)[P] = wsh[threadIdx.x];
  const real4<R> v = part[j];
  const R s[3] = {v.x, v.y, v.z};
  int b[3];
  R wx[P], dx[P];
  {
    R wy[P], wz[P], dy[P], dz[P];
    R fl = floor(s[0]);
    b[0] = (int)fl - P / 2 + 1;
    if (GRAD) window_wd<R, P>(s[0] - fl, wx, dx, g); else window_w<R, P>(s[0] - fl, wx, g);
    fl = floor(s[1]);
    b[1] = (int)fl - P / 2 + 1;
    if (GRAD) window_wd<R, P>(s[1] - fl, wy, dy, g); else window_w<R, P>(s[1] - fl, wy, g);
    fl = floor(s[2]);
    b[2] = (int)fl - P / 2 + 1;
    if (GRAD) window_wd<R, P>(s[2] - fl, wz, dz, g); else window_w<R, P>(s[2] - fl, wz, g);
#pragma unroll
    for (int k = 0; k < P; ++k) {
      ws[0][k] = wy[k];
      ws[1][k] = wz[k];
      if (GRAD) {
        ws[2][k] = dy[k];
        ws[3][k] = dz[k];
      }
    }
  }
  int gx[P];
#pragma unroll
  for (int jx = 0; jx < P; ++jx) gx[jx] = wrapi(b[0] + jx, g.M[0]);
  R a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll 2
  for (int r = 0; r < P * P; ++r) {
    const int jz = r / P, jy = r - jz * P;
    const int gz = wrapi(b[2] + jz, g.M[2]);
    const int gy = wrapi(b[1] + jy, g.M[1]);
    const FT *row = field + ((size_t)gz * g.M[1] + gy) * g.M[0];
    if constexpr (!GRAD) {
      const R wzy = ws[1][jz] * ws[0][jy];
#pragma unroll
      for (int jx = 0; jx < P; ++jx) {
        const real4<R> f = row[gx[jx]];
        const R w = wzy * wx[jx];
        a0 += w * f.x;
        a1 += w * f.y;
        a2 += w * f.z;
        a3 += w * f.w;
      }
    } else {
      const R wz_ = ws[1][jz], wy_ = ws[0][jy], dz_ = ws[3][jz], dy_ = ws[2][jy];
      const R wzy = wz_ * wy_, dzy = dz_ * wy_, wzdy = wz_ * dy_;
#pragma unroll
      for (int jx = 0; jx < P; ++jx) {
        const R psi = psi_of<R>(row[gx[jx]]);
        a0 += wzy * dx[jx] * psi;
        a1 += wzdy * wx[jx] * psi;
        a2 += dzy * wx[jx] * psi;
        a3 += wzy * wx[jx] * psi;
      }
    }
  }
  const int i = perm[j];
  const R qi = v.w;
  if (!GRAD) {
    if (vec_out) {
      vec_out[3 * i] = pref * qi * a0;
      vec_out[3 * i + 1] = pref * qi * a1;
      vec_out[3 * i + 2] = pref * qi * a2;
    }
    if (sca_out) sca_out[i] = pref * a3;
  } else {
    if (vec_out) {
      const R c = gscale * pref * qi;
      vec_out[3 * i] = c * R(g.mL[0]) * a0;
      vec_out[3 * i + 1] = c * R(g.mL[1]) * a1;
      vec_out[3 * i + 2] = c * R(g.mL[2]) * a2;
    }
    if (sca_out) sca_out[i] = sscale * pref * a3;
  }
}

// Staged rows of the tile gather start at the 16-byte boundary at or below
// the region's first point: xoff points before it (tiles start at multiples
// of 4 points, so xoff is the same for every block), and the row pitch W is
// the region's width T_x + P - 1 + 2 D plus xoff, rounded up to whole chunks.
template <typename FT, int P>
__host__ __device__ __forceinline__ int gather_xoff(int D0) {
  constexpr int PC = sizeof(FT) <= 16 ? 16 / (int)sizeof(FT) : 1;
  return (PC - (P / 2 - 1 + D0) % PC) % PC;
}
template <typename FT, int P>
__host__ __device__ __forceinline__ int gather_pitch(const Geom &g) {
  constexpr int PC = sizeof(FT) <= 16 ? 16 / (int)sizeof(FT) : 1;
  const int e = gather_xoff<FT, P>(g.sdig[0]) + g.T[0] + P - 1 + 2 * g.sdig[0];
  return (e + PC - 1) / PC * PC;
}

// Tile form of the gather: one workgroup per SY x SZ spread tiles stages
// their fields plus the (P-1)-point halo in LDS, then interpolates every
// active particle of those tiles from LDS.  Four lanes share a particle: each sums the (z, y) rows of
// one parity pair (z even/odd x y even/odd; P is even) and the four partial
// sums are combined with lane shuffles, so a tile of 64 particles keeps all
// 256 lanes busy.  Used when
// the staged tile fits the LDS budget; same outputs as k_gather.
constexpr int kGatherLanes = 4;     // lanes per particle, one spread tile per workgroup
constexpr int kGatherLanesBig = 2;  // lanes per particle, 2 x 2 spread tiles per workgroup

// b ? y : x as a bit blend, so that picking between two register values is
// never turned into an indexed load from a stack copy of the array
__device__ __forceinline__ float pick(int b, float x, float y) {
  const unsigned m = 0u - (unsigned)b;
  return __uint_as_float((__float_as_uint(x) & ~m) | (__float_as_uint(y) & m));
}
__device__ __forceinline__ double pick(int b, double x, double y) {
  const unsigned long long m = 0ull - (unsigned long long)b;
  return __longlong_as_double((long long)(((unsigned long long)__double_as_longlong(x) & ~m) |
                                          ((unsigned long long)__double_as_longlong(y) & m)));
}

template <typename R, int P, bool GRAD, typename FT, int SY, int SZ, int KL>
__global__ __launch_bounds__(SY * SZ > 1 ? kGatherTileBlockBig : kGatherTileBlock) void k_gather_tile(const real4<R> *__restrict__ part,
                                                                  const int *__restrict__ perm,
                                                                  const int *__restrict__ off_t, Geom g,
                                                                  const FT *__restrict__ field, R pref,
                                                                  R gscale, R sscale, R *__restrict__ vec_out,
                                                                  R *__restrict__ sca_out) {
  extern __shared__ unsigned char smem_raw[];
  FT *ext = reinterpret_cast<FT *>(smem_raw);
  const int tid = threadIdx.x;
  // block = SY x SZ spread tiles along y and z (fewer at the top of an axis
  // with an odd tile count)
  const int nsy = (g.nt[1] + SY - 1) / SY;
  int t = xcd_slab(blockIdx.x, gridDim.x);
  const int tx = t % g.nt[0];
  t /= g.nt[0];
  const int ty0 = SY * (t % nsy);
  const int tz0 = SZ * (t / nsy);
  const int nys = min(SY, g.nt[1] - ty0), nzs = min(SZ, g.nt[2] - tz0);
  const int t0[3] = {tx * g.T[0], ty0 * g.T[1], tz0 * g.T[2]};
  // with persistent binning a particle may sit up to sdig points outside its
  // tile: the region grows by that margin on each side
  const int D0 = g.sdig[0], D1 = g.sdig[1], D2 = g.sdig[2];
  const int E1 = nys * g.T[1] + P - 1 + 2 * D1, E2 = nzs * g.T[2] + P - 1 + 2 * D2;
  const int e0x = t0[0] - P / 2 + 1 - D0, e0y = t0[1] - P / 2 + 1 - D1, e0z = t0[2] - P / 2 + 1 - D2;
  const int span[3] = {g.T[0], nys * g.T[1], nzs * g.T[2]};
  const int marg[3] = {D0, D1, D2};
  // The block's region plus halo goes to LDS by direct loads (global memory
  // to LDS, no registers): rows of W points starting at the 16-byte boundary
  // at or below the region's first x (xoff points before it), so that every
  // 16-byte chunk of a row is one aligned load; all of a lane's loads are in
  // flight at once.  A wave's loads land in 64 consecutive chunks, chunk c of
  // the block at byte 16 c.
  // grid points per chunk, chunks per grid point (one of them is 1)
  constexpr int PC = sizeof(FT) <= 16 ? 16 / (int)sizeof(FT) : 1;
  constexpr int CPP = sizeof(FT) <= 16 ? 1 : (int)sizeof(FT) / 16;
  const int xoff = gather_xoff<FT, P>(D0), W = gather_pitch<FT, P>(g);
  {
    const int WC = W * CPP / PC, nch = WC * E1 * E2;
    const int xa = e0x - xoff;  // a multiple of PC: tiles start at multiples of 4 points
    const bool inner = xa >= 0 && e0y >= 0 && e0z >= 0 && xa + W <= g.M[0] && e0y + E1 <= g.M[1] &&
                       e0z + E2 <= g.M[2];
    const float iwc = 1.0f / (float)WC, ie1 = 1.0f / (float)E1;
    unsigned char *lds = smem_raw;
    for (int c0 = 0; c0 < nch; c0 += blockDim.x) {
      const int wbase = c0 + (tid & ~63);
      const int c = wbase + (tid & 63);
      if (c < nch) {
        const int row = (int)(((float)c + 0.5f) * iwc);
        const int cx = c - row * WC;
        const int iz = (int)(((float)row + 0.5f) * ie1);
        const int iy = row - iz * E1;
        int gx = xa + cx * PC / CPP, gy = e0y + iy, gz = e0z + iz;
        if (!inner) {
          gx = wrapi(gx, g.M[0]);
          gy = wrapi(gy, g.M[1]);
          gz = wrapi(gz, g.M[2]);
        }
        const unsigned char *src = reinterpret_cast<const unsigned char *>(
                                       field + ((size_t)gz * g.M[1] + gy) * g.M[0] + gx) + 16 * (cx % CPP);
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                         (__attribute__((address_space(3))) void *)(lds + 16 * wbase), 16, 0, 0);
      }
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): every chunk has landed
  }
  __syncthreads();
  // the block's particles: the sorted ranges of its spread tiles, end to end
  int rs[SY * SZ], rc[SY * SZ + 1];
  rc[0] = 0;
#pragma unroll
  for (int sb = 0; sb < SY * SZ; ++sb) {
    const int ya = sb % SY, zb = sb / SY;
    int n = 0;
    rs[sb] = 0;
    if (ya < nys && zb < nzs) {
      const int tile = ((tz0 + zb) * g.nt[1] + ty0 + ya) * g.nt[0] + tx;
      rs[sb] = off_t[tile * kTileBins];
      n = off_t[tile * kTileBins + kTileBins] - rs[sb];
    }
    rc[sb + 1] = rc[sb] + n;
  }
  const int ntot = rc[SY * SZ];
  const int sub = tid & (KL - 1);
  // every lane of a wave runs the same number of iterations (the shuffles
  // below need all KL lanes of a particle); lanes past the end idle, waves
  // past the end skip
  const int npass = (ntot + (blockDim.x / KL) - 1) / (blockDim.x / KL);
  for (int it = 0; it < npass; ++it) {
    const int jv = it * (blockDim.x / KL) + (tid / KL);
    const bool live = jv < ntot;
    if (!__any(live)) continue;
    int sb = 0;
#pragma unroll
    for (int k = 1; k < SY * SZ; ++k) sb += jv >= rc[k] ? 1 : 0;
    const int j = live ? rs[sb] + (jv - rc[sb]) : rs[0];
    const real4<R> v = part[live ? j : 0];
    int l[3];
    R wx[P], wy[P], wz[P], dx[P], dy[P], dz[P];
    {
      R fl = floor(v.x);
      l[0] = (int)fl - t0[0];
      if (GRAD) window_wd<R, P>(v.x - fl, wx, dx, g); else window_w<R, P>(v.x - fl, wx, g);
      fl = floor(v.y);
      l[1] = (int)fl - t0[1];
      if (GRAD) window_wd<R, P>(v.y - fl, wy, dy, g); else window_w<R, P>(v.y - fl, wy, g);
      fl = floor(v.z);
      l[2] = (int)fl - t0[2];
      if (GRAD) window_wd<R, P>(v.z - fl, wz, dz, g); else window_w<R, P>(v.z - fl, wz, g);
      // a particle that moved across the periodic boundary (persistent
      // binning) comes back within the margin of its tile; offset into the
      // region past the margin
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (l[d] >= span[d] + marg[d]) l[d] -= g.M[d];
        else if (l[d] < -marg[d]) l[d] += g.M[d];
        l[d] += marg[d];
      }
    }
    R a0s = 0, a1s = 0, a2s = 0, a3s = 0;
    // this lane's (z, y) rows: with four lanes z = za + 2m, y = yb + 2n (za,
    // yb = the lane's bits), with two z = za + 2m and every y, with one every
    // row; its z and y weights are picked once so the row loop indexes them
    // statically
    constexpr int ZS = KL >= 2 ? 2 : 1, YS = KL == 4 ? 2 : 1;
    constexpr int ZN = P / ZS, YN = P / YS;
    const int za = KL == 4 ? sub >> 1 : (KL == 2 ? sub : 0), yb = KL == 4 ? sub & 1 : 0;
    R mwz[ZN], mdz[ZN], mwy[YN], mdy[YN];
#pragma unroll
    for (int m = 0; m < ZN; ++m) {
      mwz[m] = ZS == 2 ? pick(za, wz[2 * m], wz[2 * m + 1]) : wz[m];
      if (GRAD) mdz[m] = ZS == 2 ? pick(za, dz[2 * m], dz[2 * m + 1]) : dz[m];
    }
#pragma unroll
    for (int m = 0; m < YN; ++m) {
      mwy[m] = YS == 2 ? pick(yb, wy[2 * m], wy[2 * m + 1]) : wy[m];
      if (GRAD) mdy[m] = YS == 2 ? pick(yb, dy[2 * m], dy[2 * m + 1]) : dy[m];
    }
    const FT *base = ext + ((l[2] + za) * E1 + l[1] + yb) * W + l[0] + xoff;
#pragma unroll
    for (int mz = 0; mz < ZN; ++mz) {
      // gradient form: per z plane, y sums of the row sums (sum_y w_y sw,
      // sum_y w'_y sw, sum_y w_y sd), then the plane's z weights
      R tw = 0, tdy = 0, td = 0;
#pragma unroll
      for (int my = 0; my < YN; ++my) {
        const FT *row = base + (ZS * mz * E1 + YS * my) * W;
        // x sums of the row first, then the row's z-y weight
        if constexpr (!GRAD) {
          R s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
          for (int jx = 0; jx < P; ++jx) {
            const real4<R> f = row[jx];
            s0 += wx[jx] * f.x;
            s1 += wx[jx] * f.y;
            s2 += wx[jx] * f.z;
            s3 += wx[jx] * f.w;
          }
          const R wzy = mwz[mz] * mwy[my];
          a0s += wzy * s0;
          a1s += wzy * s1;
          a2s += wzy * s2;
          a3s += wzy * s3;
        } else {
          R sw = 0, sd = 0;
#pragma unroll
          for (int jx = 0; jx < P; ++jx) {
            const R psi = psi_of<R>(row[jx]);
            sw += wx[jx] * psi;
            sd += dx[jx] * psi;
          }
          tw += mwy[my] * sw;
          tdy += mdy[my] * sw;
          td += mwy[my] * sd;
        }
      }
      if constexpr (GRAD) {
        a0s += mwz[mz] * td;
        a1s += mwz[mz] * tdy;
        a2s += mdz[mz] * tw;
        a3s += mwz[mz] * tw;
      }
    }
#pragma unroll
    for (int o = 1; o < KL; o <<= 1) {
      a0s += __shfl_xor(a0s, o, 64);
      a1s += __shfl_xor(a1s, o, 64);
      a2s += __shfl_xor(a2s, o, 64);
      a3s += __shfl_xor(a3s, o, 64);
    }
    if (!live || sub != 0) continue;
    const int i = perm[j];
    const R qi = v.w;
    if (!GRAD) {
      if (vec_out) {
        vec_out[3 * i] = pref * qi * a0s;
        vec_out[3 * i + 1] = pref * qi * a1s;
        vec_out[3 * i + 2] = pref * qi * a2s;
      }
      if (sca_out) sca_out[i] = pref * a3s;
    } else {
      if (vec_out) {
        const R c = gscale * pref * qi;
        vec_out[3 * i] = c * R(g.mL[0]) * a0s;
        vec_out[3 * i + 1] = c * R(g.mL[1]) * a1s;
        vec_out[3 * i + 2] = c * R(g.mL[2]) * a2s;
      }
      if (sca_out) sca_out[i] = sscale * pref * a3s;
    }
  }
}

// --------------------------------------------------------------------------
// real-space pair sum on a linked-cell list (Eq. 17; gradient form of Eq. 29)
//
// One workgroup per cell (cell side > r_c).  The charged particles of the
// (up to) 27 neighbouring cells are staged through LDS in chunks; the cell's
// own active particles are spread over the lanes, and when there are fewer of
// them than lanes, several lane groups split each chunk and their partial sums
// are combined in LDS.  Both orderings of a pair are evaluated (no atomics).
//   MODE 0: out_vec (forces) += ke q_i f_i, out_sca (potential) += ke phi_i +
//           self + background terms, energy partial per cell.
//   MODE 1: adjoint, out_vec (dE/dr) -= gscale ke q_i f_i, out_sca (dE/dq) +=
//           gscale (ke phi_i + self + background).
// --------------------------------------------------------------------------

// erfc(x) given e = exp(-x^2).  Single precision uses the five-term rational
// approximation of Abramowitz & Stegun, Handbook of Mathematical Functions,
// eq. 7.1.26 (absolute error <= 1.5e-7, below FP32 resolution of the force
// sums), which reuses the exponential the force needs anyway; double precision
// calls the device library's erfc.
__device__ __forceinline__ float erfc_with_exp(float x, float e) {
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * x);
  const float poly = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f +
                                                                                     t * 1.061405429f))));
  return poly * e;
}
__device__ __forceinline__ double erfc_with_exp(double x, double) { return erfc(x); }
__device__ __forceinline__ float exp_fast(float v) { return __expf(v); }
__device__ __forceinline__ double exp_fast(double v) { return exp(v); }
// 2^v: the hardware base-2 exponential in single precision (arguments here
// lie in [-13, 0], far from its denormal range)
__device__ __forceinline__ float exp2_r(float v) { return __builtin_amdgcn_exp2f(v); }
__device__ __forceinline__ double exp2_r(double v) { return exp2(v); }
__device__ __forceinline__ float rsqrt_r(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double rsqrt_r(double v) { return 1.0 / sqrt(v); }

// acc = 2 acc + (r2 < rc2): the compare's lane mask is the carry-in of an
// add with carry, so marking a candidate costs two instructions
__device__ __forceinline__ unsigned shift_in_lt(unsigned acc, float r2, float rc2) {
  unsigned r;
  asm("v_cmp_gt_f32 vcc, %2, %1\n\tv_addc_co_u32 %0, vcc, %3, %3, vcc" : "=v"(r) : "v"(r2), "v"(rc2), "v"(acc)
      : "vcc");
  return r;
}
__device__ __forceinline__ unsigned shift_in_lt(unsigned acc, double r2, double rc2) {
  return acc + acc + (r2 < rc2 ? 1u : 0u);
}


// Correction factors of Slater-type smeared charges (ENUF-DPD, Eq. 57-58)
// as functions of t = 2 r / lambda_e, given et = exp(-t):
//   B_F = 1 - e^-t (1 + t + t^2/2)   (the regularised incomplete gamma P(3, t))
//   B_U = 1 - e^-t (1 + t/2).
// Below t = 1 both come from their series, e^-t sum_{k>=3} t^k/k! for B_F
// (to k = 18: truncation below 1e-16 relative) and e^-t (t/2 + t^2/2 + the
// same sum) for B_U, so they keep their relative accuracy where they vanish
// (like t^3/6 and t/2) instead of cancelling against 1.
template <typename R>
__device__ __forceinline__ void slater_factors(R t, R et, R &bu, R &bf) {
  if (t < R(1)) {
    R s = R(1);
#pragma unroll
    for (int k = 18; k >= 4; --k) s = fma(s, t * R(1.0 / k), R(1));
    s *= t * t * t * R(1.0 / 6.0);
    bf = et * s;
    bu = et * (R(0.5) * t * (R(1) + t) + s);
  } else {
    bf = R(1) - et * (R(1) + t + R(0.5) * t * t);
    bu = R(1) - et * (R(1) + R(0.5) * t);
  }
}

// Constants of the pair sum, formed once on the host (double divisions are
// costly per thread).  bg times the total charge is the background
// potential; self times q_i the self potential.
template <typename R>
struct PairConst {
  R L[3], iL[3], rc2, al, c2a;
  R nal2l2e;  // -alpha^2 log2(e): exp(-alpha^2 r^2) = 2^(nal2l2e r^2)
  R isl;  // 1 / lambda_e of Slater-smeared charges (ENUF-DPD); 0 for point charges
  double bg, self;
};
template <typename R>
static PairConst<R> pair_const(const Geom &g) {
  const double pi = 3.14159265358979323846, sqpi = 1.7724538509055160272981674833411;
  PairConst<R> c;
  for (int d = 0; d < 3; ++d) {
    c.L[d] = (R)g.L[d];
    c.iL[d] = (R)g.iL[d];
  }
  c.rc2 = (R)(g.rc * g.rc);
  c.al = (R)g.alpha;
  c.c2a = (R)(2.0 * g.alpha / sqpi);
  c.nal2l2e = (R)(-g.alpha * g.alpha * 1.4426950408889634074);
  c.isl = g.slater > 0.0 ? (R)(1.0 / g.slater) : R(0);
  c.bg = -g.ke * pi / (g.L[0] * g.L[1] * g.L[2] * g.alpha * g.alpha);
  c.self = -2.0 * g.ke * g.alpha / sqpi;
  return c;
}

// candidates staged per chunk: 12 KB of LDS in either precision
template <typename R>
constexpr int pair_chunk() { return sizeof(R) == 4 ? 768 : 384; }

template <typename R, int MODE, bool MINIMG>
__global__ __launch_bounds__(kPairBlock) void k_pair(const real4<R> *__restrict__ part,
                                                     const int *__restrict__ perm,
                                                     const int *__restrict__ off_c, Geom g,
                                                     const double *__restrict__ scal, PairConst<R> pc,
                                                     R gscale, R *__restrict__ out_vec, R *__restrict__ out_sca,
                                                     double *eslot) {
  constexpr int CH = pair_chunk<R>();
  __shared__ real4<R> cand[CH];
  __shared__ R red[kPairBlock][4];
  __shared__ int rs[27], rp[28];
  __shared__ R rsh[27][3];  // periodic image shift of each neighbour cell
  __shared__ int hrange[2];
  const int tid = threadIdx.x;
  const int cell = blockIdx.x;
  const int cx = cell % g.nc[0];
  const int cy = (cell / g.nc[0]) % g.nc[1];
  const int cz = cell / (g.nc[0] * g.nc[1]);
  // with >= 3 cells on an axis the neighbour's image is fixed by the cell
  // offset and is added while staging; with fewer, the minimum image is taken
  // per pair on that axis
  // MINIMG: some axis has fewer than 3 cells; only then is rint needed
  const bool mi0 = MINIMG && g.nc[0] < 3, mi1 = MINIMG && g.nc[1] < 3, mi2 = MINIMG && g.nc[2] < 3;
  if (tid < 27) {
    const int o[3] = {tid % 3 - 1, (tid / 3) % 3 - 1, tid / 9 - 1};
    const int cc[3] = {cx, cy, cz};
    bool ok = true;
    int nb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (g.nc[d] == 1) ok = ok && o[d] == 0;
      else if (g.nc[d] == 2) ok = ok && o[d] >= 0;
      const int v = cc[d] + o[d];
      nb[d] = (v + g.nc[d]) % g.nc[d];
      R sh = R(0);
      if (g.nc[d] >= 3) sh = v < 0 ? -(R)g.L[d] : (v >= g.nc[d] ? (R)g.L[d] : R(0));
      rsh[tid][d] = sh;
    }
    int s0 = 0, len = 0;
    if (ok) {
      const int cid = (nb[2] * g.nc[1] + nb[1]) * g.nc[0] + nb[0];
      s0 = off_c[2 * cid];
      len = off_c[2 * cid + 1] - s0;  // charged particles only
    }
    rs[tid] = s0;
    rp[tid + 1] = len;
  }
  if (tid == 32) { hrange[0] = off_c[2 * cell]; hrange[1] = off_c[2 * cell + 2]; }
  __syncthreads();
  if (tid < 32) {  // inclusive prefix over the 27 lengths in one wave
    int v = (tid < 27) ? rp[tid + 1] : 0;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      const int u = __shfl_up(v, o, 64);
      if (tid >= o) v += u;
    }
    if (tid < 27) rp[tid + 1] = v;
    if (tid == 0) rp[0] = 0;
  }
  __syncthreads();
  const int ncand = rp[27];
  const int h0 = hrange[0], h1 = hrange[1];  // all active particles of the cell
  const R L0 = pc.L[0], L1 = pc.L[1], L2 = pc.L[2];
  const R iL0 = pc.iL[0], iL1 = pc.iL[1], iL2 = pc.iL[2];
  const R rc2 = pc.rc2;
  const R al = pc.al;
  const R c2a = pc.c2a;
  const double phi_bg = pc.bg * scal[0];
  const double c_self = pc.self;
  double e = 0.0;

  for (int hb = h0; hb < h1; hb += blockDim.x) {
    // lane groups: every thread works on one home particle; home hi gets Gh
    // groups (G or G+1), which split its candidates by index modulo Gh
    const int nh = min((int)blockDim.x, h1 - hb);
    const int G = blockDim.x / nh;
    const int extra = blockDim.x - G * nh;
    const int hi = tid % nh, grp = tid / nh;
    const int Gh = G + (hi < extra ? 1 : 0);
    real4<R> me;
    int iout = 0;
    R prev[4] = {R(0), R(0), R(0), R(0)};
    {
      me = part[hb + hi];
      if (grp == 0) {
        // the outputs this particle adds to, fetched now so their latency
        // hides behind the pair loop
        iout = perm[hb + hi];
        if (out_vec) {
          prev[0] = out_vec[3 * iout];
          prev[1] = out_vec[3 * iout + 1];
          prev[2] = out_vec[3 * iout + 2];
        }
        if (out_sca) prev[3] = out_sca[iout];
      }
    }
    R fx = 0, fy = 0, fz = 0, ph = 0;
    // separation to staged candidate k (image already applied where fixed)
    auto sep = [&](int k, R &ddx, R &ddy, R &ddz) {
      const real4<R> u = cand[k];
      ddx = me.x - u.x;
      ddy = me.y - u.y;
      ddz = me.z - u.z;
      if (mi0) ddx -= L0 * rint(ddx * iL0);
      if (mi1) ddy -= L1 * rint(ddy * iL1);
      if (mi2) ddz -= L2 * rint(ddz * iL2);
      return u.w;
    };
    for (int c0 = 0; c0 < ncand; c0 += CH) {
      const int nc = min(CH, ncand - c0);
      __syncthreads();
      {
        // stage candidates c0 .. c0+nc-1: a team of TS threads per neighbour
        // cell copies that cell's part of the window, TS consecutive
        // particles per step (27 teams of TS = blockDim / 27)
        constexpr int TS = kPairBlock / 27;
        const int r = tid / TS, j0 = tid - TS * (tid / TS);
        if (r < 27) {
          const int a0 = max(0, c0 - rp[r]), a1 = min(rp[r + 1] - rp[r], c0 + nc - rp[r]);
          const R sx = rsh[r][0], sy = rsh[r][1], sz = rsh[r][2];
          // four particles per member at a time, their loads issued together
          // (past the end a member rereads the first one)
          constexpr int UB = 4;
          for (int k0 = a0 + j0; k0 < a1; k0 += UB * TS) {
            pod_t<real4<R>> v[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
              const int k = k0 + u * TS;
              v[u] = *reinterpret_cast<const pod_t<real4<R>> *>(part + rs[r] + (k < a1 ? k : a0));
            }
#pragma unroll
            for (int u = 0; u < UB; ++u) {
              const int k = k0 + u * TS;
              if (k < a1) {
                real4<R> w;
                w.x = v[u][0] + sx;
                w.y = v[u][1] + sy;
                w.z = v[u][2] + sz;
                w.w = v[u][3];
                cand[rp[r] + k - c0] = w;
              }
            }
          }
        }
      }
      __syncthreads();
      {
        // lane group grp takes candidates grp, grp + Gh, ... of the chunk (an
        // interleaved share, so every lane sees a mix of near and far cells
        // and the pass-2 work stays balanced), in rounds of up to 64.  Pass 1
        // marks the candidates inside the cutoff in a 64-bit mask, four per
        // unrolled step; pass 2 does the erfc/exp work for the marked ones
        // only, so lanes that miss do not idle through it
        const int nmine = (nc - grp + Gh - 1) / Gh;
        for (int m0 = 0; m0 < nmine; m0 += 64) {
          const int n64 = min(64, nmine - m0);
          const int b0 = grp + Gh * m0;
          // each half of the round shifts its marks in from the right
          // (m = 2m + hit, an add with carry-in), then one bit reversal puts
          // candidate k at bit k
          unsigned long long mask = 0ull;
#pragma unroll
          for (int half = 0; half < 2; ++half) {
            const int s0 = 32 * half, s1 = min(n64, s0 + 32);
            if (s0 >= s1) break;
            unsigned acc = 0u;
            int k = s0;
#pragma unroll 1
            for (; k + 4 <= s1; k += 4) {
              const int a = b0 + Gh * k;
#pragma unroll
              for (int b = 0; b < 4; ++b) {
                R ddx, ddy, ddz;
                sep(a + Gh * b, ddx, ddy, ddz);
                acc = shift_in_lt(acc, ddx * ddx + ddy * ddy + ddz * ddz, rc2);
              }
            }
            for (; k < s1; ++k) {
              R ddx, ddy, ddz;
              sep(b0 + Gh * k, ddx, ddy, ddz);
              acc = shift_in_lt(acc, ddx * ddx + ddy * ddy + ddz * ddz, rc2);
            }
            acc = __builtin_bitreverse32(acc) >> (32 - (s1 - s0));
            mask |= (unsigned long long)acc << s0;
          }
          while (mask) {
            const int b = __builtin_ctzll(mask);
            mask &= mask - 1ull;
            R ddx, ddy, ddz;
            const R qj = sep(b0 + (int)__umul24((unsigned)Gh, (unsigned)b), ddx, ddy, ddz);
            const R r2 = ddx * ddx + ddy * ddy + ddz * ddz;
            const R ir = r2 > R(0) ? rsqrt_r(r2) : R(0);  // r = 0 (itself) marked above, adds nothing
            const R r = r2 * ir;
            const R ex = exp2_r(pc.nal2l2e * r2);
            R ec = erfc_with_exp(al * r, ex) * ir;
            R fs = qj * (ec + c2a * ex) * ir * ir;
            if (pc.isl > R(0)) {
              // ENUF-DPD smeared charges (Eq. 57-58), t = 2 r / lambda_e: the
              // energy and potential scaled by B_U; the force by B_F
              // (forward), or the exact gradient of B_U erfc(a r)/r
              // (adjoint), using B_U' = (1 + t) exp(-t) / lambda_e
              const R t = R(2) * r * pc.isl;
              const R et = exp_fast(-t);
              R bu, bf;
              slater_factors(t, et, bu, bf);
              if (MODE == 0) fs *= bf;
              else fs = fs * bu - qj * ec * (pc.isl * (R(1) + t) * et) * ir;
              ec *= bu;
            }
            ph += qj * ec;
            fx += fs * ddx;
            fy += fs * ddy;
            fz += fs * ddz;
          }
        }
      }
    }
    // combine the lane groups of each home particle
    __syncthreads();
    red[tid][0] = fx;
    red[tid][1] = fy;
    red[tid][2] = fz;
    red[tid][3] = ph;
    __syncthreads();
    if (grp == 0) {
      for (int k = 1; k < Gh; ++k) {
        fx += red[k * nh + hi][0];
        fy += red[k * nh + hi][1];
        fz += red[k * nh + hi][2];
        ph += red[k * nh + hi][3];
      }
      const R qi = me.w;
      e += 0.5 * (double)qi * (double)ph;
      const int i = iout;
      const double phs = g.ke * (double)ph + c_self * (double)qi + phi_bg;
      const R c = MODE == 0 ? (R)g.ke * qi : -gscale * (R)g.ke * qi;
      const R cs = MODE == 0 ? R(1) : gscale;
      if (out_vec) {
        out_vec[3 * i] = prev[0] + c * fx;
        out_vec[3 * i + 1] = prev[1] + c * fy;
        out_vec[3 * i + 2] = prev[2] + c * fz;
      }
      if (out_sca) out_sca[i] = prev[3] + cs * (R)phs;
    }
  }
  if (MODE == 0) {
    const double tot = block_sum(e);
    // deterministic mode: one slot per cell, summed in a fixed order
    if (tid == 0) {
      if (g.det) eslot[blockIdx.x] = tot;
      else atomicAdd(&eslot[blockIdx.x % kESlots], tot);
    }
  }
}

// energy parts in FP64: (total, E_R, E_K, E_self, E_bg)
__global__ __launch_bounds__(1024) void k_finalize(const double *kpart, int nk, const double *rpart, int nr,
                                                  const double *scal, Geom g, double *E, int *counts) {
  // eight independent partial sums per thread keep eight loads in flight
  auto sum = [](const double *v, int n) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int step = blockDim.x;
    int i = threadIdx.x;
    for (; i + 7 * step < n; i += 8 * step) {
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[k] += v[i + k * step];
    }
    for (; i < n; i += step) acc[0] += v[i];
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  };
  double a = sum(kpart, nk), b = sum(rpart, nr);
  a = block_sum(a);
  b = block_sum(b);
  if (threadIdx.x == 0) {
    const double pi = 3.14159265358979323846;
    const double V = g.L[0] * g.L[1] * g.L[2];
    const double ek = g.ke * 2.0 * pi / V * a;
    const double er = g.ke * b;
    const double es = -g.ke * g.alpha / 1.7724538509055160272981674833411 * scal[1];
    const double eb = -g.ke * pi * scal[0] * scal[0] / (2.0 * V * g.alpha * g.alpha);
    E[0] = er + ek + es + eb;
    E[1] = er;
    E[2] = ek;
    E[3] = es;
    E[4] = eb;
    counts[3] = 0;  // persistent binning: the next evaluation decides afresh
  }
}

// --------------------------------------------------------------------------
// host side: tables and launch sequences
// --------------------------------------------------------------------------

size_t sort_stage_lds(const SortPlan &sp, int real_bytes) {
  const size_t nbm = std::max(sp.nb[0], sp.nb[1]);
  if (sp.chunk == 0) return nbm * sizeof(int);
  return (size_t)sp.chunk * (4 * real_bytes + 8) + 2 * nbm * sizeof(int);
}

size_t sort_fine_lds(const SortPlan &sp) {
  // bins, then the output window's records and source indices (at most
  // kFineOutBytes / 16 of them) or the inverse permutation
  const size_t win = kFineOutBytes + kFineOutBytes / 16 * sizeof(int);
  const size_t inv = (size_t)kSortFineRegs * kSortFineBlock * sizeof(int);
  return (size_t)(1 << std::max(sp.sh[0], sp.sh[1])) * sizeof(int) + std::max(win, inv);
}

SortPlan sort_plan(const Geom &g, int real_bytes) {
  SortPlan sp{};
  sp.nblk = std::max(1, std::min(kSortMaxBlocks, (g.n + kSortPer - 1) / kSortPer));
  sp.per = (g.n + sp.nblk - 1) / sp.nblk;
  sp.nbins[0] = kTileBins * g.ntiles;
  sp.nbins[1] = 2 * g.ncells;
  // buckets per order: at least kSortBuckets, and enough that an average
  // bucket holds at most half of what the fine pass keeps in registers
  const int fill = kSortFineRegs * kSortFineBlock / 2;
  const int target = std::min(kSortBucketsMax, std::max(kSortBuckets, (g.n + fill - 1) / fill));
  for (int o = 0; o < 2; ++o) {
    int sh = 0;
    while (sh < kSortFineLog && ((sp.nbins[o] + (1 << sh) - 1) >> sh) > target) ++sh;
    sp.sh[o] = sh;
    sp.nb[o] = (sp.nbins[o] + (1 << sh) - 1) >> sh;
  }
  // the fine pass writes through its LDS window when every bucket's block
  // can be resident at once (two 1024-thread blocks per CU); the evaluation
  // also chooses it for well-filled buckets when it knows their fill
  sp.window = sp.nb[0] + sp.nb[1] <= kFineWindowBuckets;
  // largest staging chunk (a multiple of the block) that fits 64 KB of LDS;
  // zero (ungrouped staging) if none does
  for (sp.chunk = kSortChunkMax; sp.chunk >= kSortBlock; sp.chunk /= 2)
    if (sort_stage_lds(sp, real_bytes) <= 65536) break;
  if (sp.chunk < kSortBlock) sp.chunk = 0;
  return sp;
}

__host__ __device__ int build_runs(const Geom &g, int *out) {
  int n = 0;
  int offs[3][3], no[3];
  for (int d = 0; d < 3; ++d) {
    if (g.nt[d] >= 3) { offs[d][0] = -1; offs[d][1] = 0; offs[d][2] = 1; no[d] = 3; }
    else { offs[d][0] = 0; offs[d][1] = 1; no[d] = 2; }
  }
  // digits a particle of the neighbour at offset o must have on one axis to
  // reach the consuming tile: above it (o=+1) it must cross its low face (0),
  // below it (o=-1) its high face (2); with two tiles per axis the single
  // neighbour is on both sides
  auto allowed = [&](int d, int o, int dig) {
    if (o == 0) return true;
    if (g.nt[d] == 2) return dig != 1;
    return o > 0 ? dig == 0 : dig == 2;
  };
  for (int a = 0; a < no[2]; ++a)
    for (int b = 0; b < no[1]; ++b)
      for (int c = 0; c < no[0]; ++c) {
        const int o[3] = {offs[0][c], offs[1][b], offs[2][a]};
        int lo = -1, prev = -2;
        for (int cl = 0; cl < kClasses; ++cl) {
          const int dx = cl / 9, dy = (cl / 3) % 3, dz = cl % 3;
          const bool ok = allowed(0, o[0], dx) && allowed(1, o[1], dy) && allowed(2, o[2], dz);
          if (ok) {
            if (prev != cl - 1) lo = cl;
            prev = cl;
          }
          const bool close = lo >= 0 && prev == cl && (cl == kClasses - 1 || !(
              allowed(0, o[0], (cl + 1) / 9) && allowed(1, o[1], ((cl + 1) / 3) % 3) && allowed(2, o[2], (cl + 1) % 3)));
          if (close) {
            if (n >= kMaxRuns) return -1;
            out[5 * n] = o[0];
            out[5 * n + 1] = o[1];
            out[5 * n + 2] = o[2];
            out[5 * n + 3] = lo;
            out[5 * n + 4] = cl;
            ++n;
            lo = -1;
          }
        }
      }
  return n;
}

static int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Launch shape of the FFT passes: log2 pencils per block and dynamic LDS
// bytes, the largest batch (at most 16 pencils) that fits the LDS budget and
// divides the pencil count.
struct FftPlan {
  int lnh, lny, lnz, lhx;
  int lb_r2c, lb_y, lb_z, lb_c2r;
  int nfp;  // field pencils per inverse-z batch
  size_t lds_r2c, lds_y, lds_z, lds_c2r;
  int zblocks;
};

static size_t pad_ld(int lb) { return lb == 0 ? 1 : (1u << lb) + 1; }

static FftPlan fft_plan(const Geom &g, size_t cs, int nf) {
  FftPlan P;
  P.lnh = ilog2(g.M[0] / 2);
  P.lny = ilog2(g.M[1]);
  P.lnz = ilog2(g.M[2]);
  P.lhx = P.lnh;
  const size_t nh = (size_t)1 << P.lnh, ny = g.M[1], nz = g.M[2];
  auto pick = [](int count, auto lds_of, size_t budget) {
    int lb = 4;
    while (lb > 0 && (lds_of(lb) > budget || count % (1 << lb) != 0)) --lb;
    return lb;
  };
  auto r2c = [&](int lb) { return 2 * nh * pad_ld(lb) * cs; };
  P.lb_r2c = pick(g.M[1] * g.M[2], r2c, 32768);
  P.lds_r2c = r2c(P.lb_r2c);
  const int sty = fft_nstages(P.lny);
  auto yl = [&](int lb) { return (size_t)((sty >= 2) + (sty == 3)) * ny * ((size_t)1 << lb) * cs; };
  P.lb_y = pick((int)nh, yl, 32768);
  P.lds_y = yl(P.lb_y);
  const int stz = fft_nstages(P.lnz);
  auto zl = [&](int nfp, int lb) {
    return (size_t)(1 + (stz >= 2) * nfp + (stz == 3) * nfp) * nz * ((size_t)1 << lb) * cs;
  };
  // z: the widest pencil batch (rows of up to 16 contiguous elements) that
  // fits, batching the field pencils when there is room for them
  const int zp = (int)nh * g.M[1];
  const size_t zbudget = 65536 - 512;  // leave room for the static reduction scratch
  // (the field pencils batched when rows of 8 or more still fit, since the
  // batch saves passes over the spectrum; else one field at a time)
  P.nfp = 1;
  P.lb_z = 0;
  bool found = false;
  for (int lb = 4; lb >= 3 && !found; --lb)
    if (zp % (1 << lb) == 0 && zl(nf, lb) <= zbudget) { P.nfp = nf; P.lb_z = lb; found = true; }
  for (int lb = 4; lb >= 0 && !found; --lb)
    if (zp % (1 << lb) == 0 && zl(1, lb) <= zbudget) { P.nfp = 1; P.lb_z = lb; found = true; }
  P.lds_z = zl(P.nfp, P.lb_z);
  P.zblocks = zp >> P.lb_z;
  auto c2r = [&](int lb) { return 2 * (size_t)nf * nh * pad_ld(lb) * cs; };
  P.lb_c2r = pick(g.M[1] * g.M[2], c2r, 40960);  // 16 rows of 256 points (faster than 8 there; not for r2c)
  P.lds_c2r = c2r(P.lb_c2r);
  return P;
}

bool fft_plans_fit(const Geom &g, bool fp64) {
  const size_t cs = fp64 ? 16 : 8;
  for (int nf : {1, 3, 4}) {
    const FftPlan P = fft_plan(g, cs, nf);
    if (P.lds_r2c > 65536 || P.lds_y > 65536 || P.lds_z > 65536 - 512 || P.lds_c2r > 65536) return false;
  }
  return true;
}


// table layout (in reals): [0] tw x-half (n=Mx/2) complex, [1] tw e^{-2pi i k/Mx}
// k<Mx/2 complex, [2] tw y complex, [3] tw z complex, [4..6] influence
// factors s_x (Mx/2), s_y (My), s_z (Mz), [7..9] wave numbers k_x, k_y, k_z
size_t table_size(const Geom &g, size_t off[kTabSlots]) {
  const size_t hx = g.M[0] / 2;
  const size_t len[kTabSlots - 1] = {2 * hx, 2 * hx, 2 * (size_t)g.M[1], 2 * (size_t)g.M[2], hx,
                                     (size_t)g.M[1], (size_t)g.M[2], hx, (size_t)g.M[1], (size_t)g.M[2]};
  size_t o = 0;
  for (int i = 0; i < kTabSlots - 1; ++i) {
    off[i] = o;
    o += len[i];
  }
  off[kTabSlots - 1] = o;
  return o;
}

// Workspace initialisation, on the device so that a workspace can be set up
// by kernels alone (no host copy): every table entry in FP64, cast to the
// precision.  Twiddles e^{-2 pi i m / period}; per axis the influence factor
// s_d = exp(-k_d^2 / 4 alpha^2) / c_d^2 with the window transform
// c_d = sinc^p(pi n / M_d) of the B-spline, or sqrt(pi b) exp(-b (pi n/M_d)^2)
// of the Gaussian (n signed; zero at the Nyquist index and, when
// oversampling, at |n| >= kept_d / 2: both outside the k-set), and the wave
// number k_d = 2 pi n / L_d.  Thread 0 also
// writes the spread run table and clears the flags; block 0 clears the
// energy slots.
struct TabOff {
  size_t o[kTabSlots];
};
template <typename R>
__global__ __launch_bounds__(256) void k_init_ws(Geom g, TabOff t, R *__restrict__ tab, int *__restrict__ runs,
                                                 int *__restrict__ counts, double *__restrict__ eslot) {
  const double pi = 3.14159265358979323846;
  const size_t total = t.o[kTabSlots - 1];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    int seg = 0;
    while (seg < kTabSlots - 2 && i >= t.o[seg + 1]) ++seg;
    const int k = (int)(i - t.o[seg]);
    double v;
    if (seg < 4) {
      const int period = seg == 0 ? g.M[0] / 2 : seg == 1 ? g.M[0] : seg == 2 ? g.M[1] : g.M[2];
      double sn, cs;
      sincospi(-2.0 * (double)(k >> 1) / (double)period, &sn, &cs);
      v = (k & 1) ? sn : cs;
    } else {
      const int d = seg < 7 ? seg - 4 : seg - 7;
      const int M = g.M[d];
      const int nn = k < M / 2 ? k : k - M;
      const double kd = 2.0 * pi * (double)nn / g.L[d];
      if (seg >= 7) {
        v = kd;
      } else if (k == M / 2 || 2 * (nn < 0 ? -nn : nn) >= g.kept[d]) {
        v = 0.0;  // the Nyquist index, and modes beyond the kept set when oversampling
      } else {
        double c = 1.0;
        if (g.win == 0) {
          const double r = nn == 0 ? 1.0 : sinpi((double)nn / (double)M) / (pi * (double)nn / (double)M);
          for (int j = 0; j < g.p; ++j) c *= r;
        } else {
          const double t = pi * (double)nn / (double)M;
          c = sqrt(pi * g.gb) * exp(-g.gb * t * t);
        }
        v = exp(-kd * kd / (4.0 * g.alpha * g.alpha)) / (c * c);
      }
    }
    tab[i] = (R)v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    build_runs(g, runs);
    for (int j = 0; j < 8; ++j) counts[j] = 0;
    counts[3] = 1;   // the first evaluation on a workspace sorts
    counts[4] = -1;  // no all-active flag seen yet
  }
  if (blockIdx.x == 0)
    (void)eslot;
}

hipError_t launch_init_ws(const Geom &g, const Work &w, hipStream_t st, bool fp64) {
  TabOff t;
  for (int i = 0; i < kTabSlots; ++i) t.o[i] = w.tab_off[i];
  const int nb = (int)std::min<size_t>(64, (t.o[kTabSlots - 1] + 255) / 256);
  if (fp64)
    hipLaunchKernelGGL((k_init_ws<double>), dim3(nb), dim3(256), 0, st, g, t, (double *)w.tables, w.runs, w.counts,
                       w.eslot);
  else
    hipLaunchKernelGGL((k_init_ws<float>), dim3(nb), dim3(256), 0, st, g, t, (float *)w.tables, w.runs, w.counts,
                       w.eslot);
  return hipGetLastError();
}

// Multiply a device array by a device scalar (the adjoint's upstream
// gradient when it lives in device memory).
template <typename R>
__global__ void k_scale_dev(R *__restrict__ a, long long n, const double *__restrict__ s) {
  const R f = (R)*s;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    a[i] *= f;
}

#define ENUF_TRY(x)                   \
  do {                                \
    hipError_t e_ = (x);              \
    if (e_ != hipSuccess) return e_;  \
  } while (0)

template <typename R, int P>
static void launch_spread(const Geom &g, const Work &w, hipStream_t st) {
  if constexpr (sizeof(R) == 4) {
    if (g.spread16)
      hipLaunchKernelGGL((k_spread_mfma<P, false>), dim3(g.ntiles), dim3(256), 0, st, (const float4 *)w.part_t,
                         w.off_t, (const int *)w.runs, w.nruns, g, (const double *)w.scal, (float *)w.grid);
    else
      hipLaunchKernelGGL((k_spread_mfma<P, true>), dim3(g.ntiles), dim3(256), 0, st, (const float4 *)w.part_t,
                         w.off_t, (const int *)w.runs, w.nruns, g, (const double *)w.scal, (float *)w.grid);
  } else
    hipLaunchKernelGGL((k_spread<R, P>), dim3(g.ntiles), dim3(spread_block<R>()), 0, st,
                       (const real4<R> *)w.part_t, w.off_t, (const int *)w.runs, w.nruns, g, (R *)w.grid);
}
template <typename FT, int P>
static size_t gather_tile_lds(const Geom &g, int sy, int sz) {
  return (size_t)gather_pitch<FT, P>(g) * (sy * g.T[1] + P - 1 + 2 * g.sdig[1]) *
         (sz * g.T[2] + P - 1 + 2 * g.sdig[2]) * sizeof(FT);
}
// Gather kinds: ik forces and potentials from the interleaved (E, psi) grid;
// gradient form (forces -dE/dr or the adjoint dE/dr, scaled by gs, and the
// potential scaled by ss) from psi, read either from the interleaved grid
// (.w) or from a potential-only grid (scalar).
enum GatherKind { kGatherIk = 0, kGatherGrad4 = 1, kGatherGradScalar = 2 };
template <typename R, int P, bool GRAD, typename FT>
static void launch_gather_as(const Geom &g, const Work &w, hipStream_t st, R pref, R gs, R ss, R *vo, R *so) {
  // a potential-only grid stages 2 x 2 spread tiles (y, z) per block (less
  // halo per point, more particles per block); the interleaved fields one.
  // Under persistent binning particles may have left their tile by up to
  // sdig points: the staged region carries that margin, and the direct form
  // (grid read per particle) takes over when it no longer fits.
  const size_t lds2 = gather_tile_lds<FT, P>(g, 2, 2);
  if (sizeof(FT) == sizeof(R) && lds2 <= 65536) {
    const int nb = g.nt[0] * ((g.nt[1] + 1) / 2) * ((g.nt[2] + 1) / 2);
    hipLaunchKernelGGL((k_gather_tile<R, P, GRAD, FT, 2, 2, kGatherLanesBig>), dim3(nb), dim3(kGatherTileBlockBig), lds2, st,
                       (const real4<R> *)w.part_t, w.perm_t, w.off_t, g, (const FT *)w.field, pref, gs, ss, vo,
                       so);
    return;
  }
  const size_t lds = gather_tile_lds<FT, P>(g, 1, 1);
  if (lds <= 65536) {
    hipLaunchKernelGGL((k_gather_tile<R, P, GRAD, FT, 1, 1, kGatherLanes>), dim3(g.ntiles), dim3(kGatherTileBlock), lds, st,
                       (const real4<R> *)w.part_t, w.perm_t, w.off_t, g, (const FT *)w.field, pref, gs, ss, vo,
                       so);
    return;
  }
  const int nb = (g.n + kGatherBlock - 1) / kGatherBlock;
  hipLaunchKernelGGL((k_gather<R, P, GRAD, FT>), dim3(nb), dim3(kGatherBlock), 0, st, (const real4<R> *)w.part_t,
                     w.perm_t, w.counts, g, (const FT *)w.field, pref, gs, ss, vo, so);
}
template <typename R, int P>
static void launch_gather(const Geom &g, const Work &w, hipStream_t st, R pref, R gs, R ss, R *vo, R *so,
                          int kind) {
  if (kind == kGatherIk) launch_gather_as<R, P, false, real4<R>>(g, w, st, pref, gs, ss, vo, so);
  else if (kind == kGatherGrad4) launch_gather_as<R, P, true, real4<R>>(g, w, st, pref, gs, ss, vo, so);
  else launch_gather_as<R, P, true, R>(g, w, st, pref, gs, ss, vo, so);
}

template <typename R>
static void dispatch_spread(const Geom &g, const Work &w, hipStream_t st) {
  switch (g.p) {
    case 2: launch_spread<R, 2>(g, w, st); break;
    case 4: launch_spread<R, 4>(g, w, st); break;
    case 6: launch_spread<R, 6>(g, w, st); break;
    default: launch_spread<R, 8>(g, w, st); break;
  }
}
template <typename R>
static void dispatch_gather(const Geom &g, const Work &w, hipStream_t st, R pref, R gs, R ss, R *vo, R *so,
                            int kind) {
  switch (g.p) {
    case 2: launch_gather<R, 2>(g, w, st, pref, gs, ss, vo, so, kind); break;
    case 4: launch_gather<R, 4>(g, w, st, pref, gs, ss, vo, so, kind); break;
    case 6: launch_gather<R, 6>(g, w, st, pref, gs, ss, vo, so, kind); break;
    default: launch_gather<R, 8>(g, w, st, pref, gs, ss, vo, so, kind); break;
  }
}

template <typename R>
hipError_t launch_forward(const Geom &g, const Work &w, hipStream_t st, const R *x, const R *q, double *E,
                          R *F, R *phi, bool all_active, bool want_psi, bool analytic, hipEvent_t *ev) {
  const size_t cs = sizeof(Cx<R>);
  const R *tab = (const R *)w.tables;
  const Cx<R> *tw_xh = (const Cx<R> *)(tab + w.tab_off[0]);
  const Cx<R> *tw_x2 = (const Cx<R> *)(tab + w.tab_off[1]);
  const Cx<R> *tw_y = (const Cx<R> *)(tab + w.tab_off[2]);
  const Cx<R> *tw_z = (const Cx<R> *)(tab + w.tab_off[3]);
  const R *sx = tab + w.tab_off[4], *sy = tab + w.tab_off[5], *sz = tab + w.tab_off[6];
  const R *kvx = tab + w.tab_off[7], *kvy = tab + w.tab_off[8], *kvz = tab + w.tab_off[9];
  const int hx = g.M[0] / 2;
  const size_t halfG = (size_t)hx * g.M[1] * g.M[2];
  // ik forces use the three field spectra, and the potential field psi is
  // transformed only when potentials (or a later adjoint) need it; the
  // analytic-derivative mode transforms psi alone and differentiates the
  // window in the gather
  const int nfield = analytic ? 1 : (want_psi ? 4 : 3);
  const int fbase = analytic ? 3 : 0;
  const FftPlan P = fft_plan(g, cs, nfield);
  auto mark = [&](int k) { if (ev) (void)hipEventRecord(ev[k], st); };

  mark(0);
  // prep: keys and per-block bucket counts
  SortPlan sp = sort_plan(g, (int)sizeof(R));
  // with every particle active (potentials requested) the buckets' fill is
  // known here: well-filled buckets take the window form in any number
  if (all_active && (long long)g.n >= (long long)kFineWindowMin * (sp.nb[0] + sp.nb[1])) sp.window = 1;
  const int nbk = sp.nb[0] + sp.nb[1];
  const size_t lds_cnt = (size_t)nbk * sizeof(int);
  const size_t lds_fine = sort_fine_lds(sp);
  // persistent binning: the check decides (on the device) whether this
  // evaluation sorts; the sort passes and the refresh both launch and the
  // ones not needed return at once
  const bool persist = g.skin > 0.0;
  const int *need = persist ? w.counts + 3 : nullptr;
  if (persist)
    hipLaunchKernelGGL((k_persist_check<R>), dim3(std::min(1024, (g.n + kSortBlock - 1) / kSortBlock)),
                       dim3(kSortBlock), 0, st, x, q, g, (const R *)w.x_ref, (const R *)w.q_ref,
                       all_active ? 1 : 0, w.counts);
  hipLaunchKernelGGL((k_sort_count<R>), dim3(sp.nblk), dim3(kSortBlock), lds_cnt, st, x, q, g, sp,
                     all_active ? 1 : 0, w.key_t, w.key_c, w.hist, F, phi, w.qpart, w.counts, persist ? 1 : 0,
                     (R *)w.x_ref, (R *)w.q_ref, w.act);
  if (persist)
    hipLaunchKernelGGL((k_refresh<R>), dim3(sp.nblk), dim3(kSortBlock), 0, st, x, q, g, sp, (const R *)w.x_ref,
                       (const int *)w.act, (const int *)w.perm_t, (const int *)w.perm_c, (real4<R> *)w.part_t,
                       (real4<R> *)w.part_c, F, phi, w.qpart, (const int *)w.counts);
  ENUF_TRY(hipGetLastError());
  mark(1);
  // sort: slots, bucket staging, fine sort per bucket (the key arrays are
  // dead after staging and take the fine ranks)
  hipLaunchKernelGGL(k_sort_colscan, dim3((nbk + kColW - 1) / kColW), dim3(kColW * kColG), 0, st, w.hist, sp,
                     w.bbase, need);
  hipLaunchKernelGGL(k_sort_base, dim3(1), dim3(1024), 0, st, w.bbase, sp, w.off_t, w.off_c,
                     (const double *)w.qpart, w.scal, w.counts, w.eslot, eslot_real_off(g), persist ? 1 : 0);
  hipLaunchKernelGGL((k_sort_stage<R>), dim3(sp.nblk), dim3(kSortStageBlock), sort_stage_lds(sp, (int)sizeof(R)), st,
                     x, q, g, sp, (const int *)w.key_t, (const int *)w.key_c, (const int *)w.hist,
                     (const int *)w.bbase, (real4<R> *)w.stg_t, w.ik_t, (real4<R> *)w.stg_c, w.ik_c, need);
  bool win = false;
  if constexpr (sizeof(R) == 4) {  // the FP64 records do not fit the window form's registers
    win = sp.window != 0;
    if (win)
      hipLaunchKernelGGL((k_sort_fine_win<R>), dim3(nbk), dim3(kSortFineBlock), lds_fine, st, sp,
                         (const int *)w.bbase, (const real4<R> *)w.stg_t, (const int2 *)w.ik_t, w.key_t,
                         (const real4<R> *)w.stg_c, (const int2 *)w.ik_c, w.key_c, (real4<R> *)w.part_t,
                         w.perm_t, w.off_t, (real4<R> *)w.part_c, w.perm_c, w.off_c, need);
  }
  if (!win)
    hipLaunchKernelGGL((k_sort_fine<R>), dim3(nbk), dim3(kSortFineBlock), lds_fine, st, sp, (const int *)w.bbase,
                       (const real4<R> *)w.stg_t, (const int2 *)w.ik_t, w.key_t, (const real4<R> *)w.stg_c,
                       (const int2 *)w.ik_c, w.key_c, (real4<R> *)w.part_t, w.perm_t, w.off_t,
                       (real4<R> *)w.part_c, w.perm_c, w.off_c, need);
  if (g.det) {
    // bins in caller-index order; the key arrays (dead after the sort) hold
    // the lists of large bins, the staging arrays the moved records
    const int nbin[2] = {sp.nbins[0], sp.nbins[1]};
    int *perms[2] = {w.perm_t, w.perm_c};
    const int *offs[2] = {w.off_t, w.off_c};
    real4<R> *parts[2] = {(real4<R> *)w.part_t, (real4<R> *)w.part_c};
    real4<R> *tmps[2] = {(real4<R> *)w.stg_t, (real4<R> *)w.stg_c};
    int *bigs[2] = {w.key_t, w.key_c};
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, w.counts + 6, 2, 0);
    for (int o = 0; o < 2; ++o) {
      hipLaunchKernelGGL((k_det_small<R>), dim3(std::min(4096, (nbin[o] + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                         st, nbin[o], offs[o], perms[o], parts[o], bigs[o], w.counts + 6 + o, need);
      hipLaunchKernelGGL((k_det_big<R>), dim3(256), dim3(kBlock), 0, st, offs[o], perms[o], parts[o], tmps[o],
                         (const int *)bigs[o], (const int *)(w.counts + 6 + o), w.counts, need);
    }
  }
  ENUF_TRY(hipGetLastError());
  mark(2);
  // spread
  dispatch_spread<R>(g, w, st);
  ENUF_TRY(hipGetLastError());
  mark(3);
  // forward x (r2c), y
  hipLaunchKernelGGL((k_fft_x_r2c<R>), dim3((g.M[1] * g.M[2]) >> P.lb_r2c), dim3(kBlock), P.lds_r2c, st,
                     (const R *)w.grid, (Cx<R> *)w.spec, P.lnh, P.lb_r2c, tw_xh, tw_x2);
  hipLaunchKernelGGL((k_fft_y<R, -1>), dim3(hx >> P.lb_y, g.M[2], 1), dim3(kBlock), P.lds_y, st,
                     (Cx<R> *)w.spec, P.lny, P.lhx, (size_t)hx * g.M[1], (size_t)0, tw_y, P.lb_y);
  ENUF_TRY(hipGetLastError());
  mark(4);
  // z fused: forward z, influence, energy, inverse z of the field spectra
  const int zp = hx * g.M[1];
  const bool zpsi = analytic && sizeof(R) == 4 && (P.lnz == 7 || P.lnz == 8 || P.lnz == 9) && zp % 16 == 0;
  const int nzb = zpsi ? zp / 16 : P.zblocks;  // z-pass blocks: one energy partial each
  if (zpsi && P.lnz == 9)
    hipLaunchKernelGGL((k_z_psi512<R>), dim3(zp / 16), dim3(512), (size_t)16 * sizeof(Cx<R>) << 9, st,
                       (const Cx<R> *)w.spec, (Cx<R> *)w.fspec, g, P.lhx, tw_z, sx, sy, sz, kvx, kvy, kvz, w.eslot);
  else if (zpsi)
    hipLaunchKernelGGL((k_z_psi<R>), dim3(zp / 16), dim3(kBlock), (size_t)16 * sizeof(Cx<R>) << P.lnz, st,
                       (const Cx<R> *)w.spec, (Cx<R> *)w.fspec, g, P.lnz, P.lhx, tw_z, sx, sy, sz, kvx, kvy, kvz,
                       w.eslot);
  else
    hipLaunchKernelGGL((k_z_fused<R>), dim3(P.zblocks), dim3(kBlock), P.lds_z, st, (const Cx<R> *)w.spec,
                       (Cx<R> *)w.fspec, g, P.lnz, P.lhx, P.lb_z, nfield, P.nfp, fbase, tw_z, sx, sy, sz, kvx, kvy,
                       kvz, w.eslot);
  ENUF_TRY(hipGetLastError());
  mark(5);
  // inverse y (nfield components), inverse x c2r -> interleaved fields
  hipLaunchKernelGGL((k_fft_y<R, 1>), dim3(hx >> P.lb_y, g.M[2], nfield), dim3(kBlock), P.lds_y, st,
                     (Cx<R> *)w.fspec, P.lny, P.lhx, (size_t)hx * g.M[1], halfG, tw_y, P.lb_y);
  if (analytic)
    hipLaunchKernelGGL((k_fft_x_c2r4<R, true>), dim3((g.M[1] * g.M[2]) >> P.lb_c2r), dim3(kBlock), P.lds_c2r, st,
                       (const Cx<R> *)w.fspec, w.field, g, P.lnh, P.lb_c2r, nfield, tw_xh, tw_x2);
  else
    hipLaunchKernelGGL((k_fft_x_c2r4<R, false>), dim3((g.M[1] * g.M[2]) >> P.lb_c2r), dim3(kBlock), P.lds_c2r,
                       st, (const Cx<R> *)w.fspec, w.field, g, P.lnh, P.lb_c2r, nfield, tw_xh, tw_x2);
  ENUF_TRY(hipGetLastError());
  mark(6);
  // gather
  const double V = g.L[0] * g.L[1] * g.L[2];
  const R pref = (R)(g.ke * 4.0 * 3.14159265358979323846 / V);
  if (F || phi) {
    if (analytic) dispatch_gather<R>(g, w, st, pref, R(-1), R(1), F, phi, kGatherGradScalar);
    else dispatch_gather<R>(g, w, st, pref, R(1), R(1), F, phi, kGatherIk);
  }
  ENUF_TRY(hipGetLastError());
  mark(7);
  // pair
  if (g.nc[0] < 3 || g.nc[1] < 3 || g.nc[2] < 3)
    hipLaunchKernelGGL((k_pair<R, 0, true>), dim3(g.ncells), dim3(kPairBlock), 0, st, (const real4<R> *)w.part_c,
                       w.perm_c, w.off_c, g, w.scal, pair_const<R>(g), R(1), F, phi, w.eslot + eslot_real_off(g));
  else
    hipLaunchKernelGGL((k_pair<R, 0, false>), dim3(g.ncells), dim3(kPairBlock), 0, st, (const real4<R> *)w.part_c,
                       w.perm_c, w.off_c, g, w.scal, pair_const<R>(g), R(1), F, phi, w.eslot + eslot_real_off(g));
  ENUF_TRY(hipGetLastError());
  mark(8);
  const int nks = g.det ? nzb : kESlots, nrs = g.det ? g.ncells : kESlots;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(g.det ? 1024 : 64), 0, st, (const double *)w.eslot, nks,
                     (const double *)(w.eslot + eslot_real_off(g)), nrs, (const double *)w.scal, g, E, w.counts);
  ENUF_TRY(hipGetLastError());
  mark(9);
  return hipSuccess;
}

template <typename R>
hipError_t launch_adjoint(const Geom &g, const Work &w, hipStream_t st, double gscale, R *dEdx, R *dEdq,
                          bool psi_scalar, const double *gdev) {
  if (dEdx) hipLaunchKernelGGL((k_fill_real<R>), dim3(256), dim3(kBlock), 0, st, dEdx, 3LL * g.n);
  if (dEdq) hipLaunchKernelGGL((k_fill_real<R>), dim3(256), dim3(kBlock), 0, st, dEdq, (long long)g.n);
  ENUF_TRY(hipGetLastError());
  const double V = g.L[0] * g.L[1] * g.L[2];
  const R pref = (R)(g.ke * 4.0 * 3.14159265358979323846 / V);
  dispatch_gather<R>(g, w, st, pref, (R)gscale, (R)gscale, dEdx, dEdq,
                     psi_scalar ? kGatherGradScalar : kGatherGrad4);
  ENUF_TRY(hipGetLastError());
  if (g.nc[0] < 3 || g.nc[1] < 3 || g.nc[2] < 3)
    hipLaunchKernelGGL((k_pair<R, 1, true>), dim3(g.ncells), dim3(kPairBlock), 0, st, (const real4<R> *)w.part_c,
                       w.perm_c, w.off_c, g, w.scal, pair_const<R>(g), (R)gscale, dEdx, dEdq,
                       w.eslot + eslot_real_off(g));
  else
    hipLaunchKernelGGL((k_pair<R, 1, false>), dim3(g.ncells), dim3(kPairBlock), 0, st, (const real4<R> *)w.part_c,
                       w.perm_c, w.off_c, g, w.scal, pair_const<R>(g), (R)gscale, dEdx, dEdq,
                       w.eslot + eslot_real_off(g));
  ENUF_TRY(hipGetLastError());
  if (gdev) {
    if (dEdx) hipLaunchKernelGGL((k_scale_dev<R>), dim3(256), dim3(kBlock), 0, st, dEdx, 3LL * g.n, gdev);
    if (dEdq) hipLaunchKernelGGL((k_scale_dev<R>), dim3(256), dim3(kBlock), 0, st, dEdq, (long long)g.n, gdev);
  }
  return hipGetLastError();
}

// Plain copy, 16 bytes per lane, four non-temporal loads in flight per
// thread before any store, one workgroup per CU (the fastest of the forms
// measured for the achievable-bandwidth probe: ~6.1 TB/s over 1 GiB).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy16(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_copy16(const void *src, void *dst, size_t n16, hipStream_t st) {
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int nb = (int)std::min<size_t>((size_t)std::max(cus, 1), std::max<size_t>(1, (n16 + 255) / 256));
  hipLaunchKernelGGL(k_copy16, dim3(nb), dim3(256), 0, st, (const u32x4 *)src, (u32x4 *)dst, n16);
  return hipGetLastError();
}

template hipError_t launch_forward<float>(const Geom &, const Work &, hipStream_t, const float *, const float *,
                                          double *, float *, float *, bool, bool, bool, hipEvent_t *);
template hipError_t launch_forward<double>(const Geom &, const Work &, hipStream_t, const double *,
                                           const double *, double *, double *, double *, bool, bool, bool,
                                           hipEvent_t *);
template hipError_t launch_adjoint<float>(const Geom &, const Work &, hipStream_t, double, float *, float *, bool,
                                          const double *);
template hipError_t launch_adjoint<double>(const Geom &, const Work &, hipStream_t, double, double *, double *,
                                           bool, const double *);

}  // namespace enuf
