// enuf_internal.h -- types shared by the host API and the HIP kernels of the
// ENUF library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace enuf {

constexpr int kBlock = 256;          // threads per block for per-particle kernels
constexpr int kGatherBlock = 128;    // threads per block of the interpolation kernels
constexpr int kTileX = 16;           // spread tile (grid points) before clamping to M/2
constexpr int kTileY = 8;
constexpr int kTileZ = 8;
constexpr int kMaxTilePts = kTileX * kTileY * kTileZ;

// Geometry and parameters, passed by value to kernels.
struct Geom {
  int M[3];        // FFT grid (x, y, z)
  int T[3];        // spread tile size per axis (power of two, <= M/2)
  int nt[3];       // tiles per axis
  int ntiles;
  int nc[3];       // real-space cells per axis (side > r_c)
  int ncells;
  int p;           // window stencil width
  int n;           // particles
  double L[3];     // box
  double alpha, rc, ke;
};

// Device workspace pointers (all owned by the context).
struct Work {
  void *part_t = nullptr;   // real4 [n] grid coords (s_x, s_y, s_z) + q, tile order
  void *part_c = nullptr;   // real4 [n] wrapped positions + q, cell order
  int *perm_t = nullptr;    // [n]
  int *perm_c = nullptr;    // [n]
  int *key_t = nullptr;     // [n]
  int *rank_t = nullptr;    // [n]
  int *key_c = nullptr;     // [n]
  int *rank_c = nullptr;    // [n]
  int *off_t = nullptr;     // [2*ntiles + 1] counts, then exclusive offsets
  int *off_c = nullptr;     // [2*ncells + 1]
  int *counts = nullptr;    // [4]: active, charged, flags, spare
  double *scal = nullptr;   // [4]: Q, Q2, spare
  double *qpart = nullptr;  // [2*nblk_prep] partial sums of q, q^2
  double *kpart = nullptr;  // [nblk_z] partial reciprocal energies
  double *rpart = nullptr;  // [nblk_pair] partial real-space energies
  void *grid = nullptr;     // real [G]
  void *spec = nullptr;     // complex [G/2]
  void *fspec = nullptr;    // complex [4][G/2]
  void *field = nullptr;    // real4 [G]
  void *tables = nullptr;   // twiddles and window transforms (real)
  size_t tab_off[8] = {0};  // element offsets inside `tables`
};

// Launch-configuration numbers the host needs to size partial buffers.
int nblk_prep(const Geom &g);
int nblk_pair(const Geom &g);
int nblk_z(const Geom &g, bool fp64);

// Fill the twiddle / window tables on the host (size in reals returned by
// table_size()).  `host` must hold table_size(g) reals of the precision.
size_t table_size(const Geom &g, size_t off[8]);
template <typename R> void fill_tables(const Geom &g, const size_t off[8], R *host);

// One forward evaluation: every phase enqueued on `st`.  `ev` (optional) is
// an array of kPhases+1 events recorded between phases.
constexpr int kPhases = 9;
template <typename R>
hipError_t launch_forward(const Geom &g, const Work &w, hipStream_t st, const R *x, const R *q,
                          double *E, R *F, R *phi, bool all_active, hipEvent_t *ev);

// Adjoint of the last forward: dEdx, dEdq (either may be null).
template <typename R>
hipError_t launch_adjoint(const Geom &g, const Work &w, hipStream_t st, double gscale, R *dEdx,
                          R *dEdq);

}  // namespace enuf
