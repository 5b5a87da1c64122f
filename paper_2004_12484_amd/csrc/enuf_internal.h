// enuf_internal.h -- types shared by the host API and the HIP kernels of the
// ENUF library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace enuf {

constexpr int kBlock = 256;          // threads per block for per-particle kernels
constexpr int kGatherBlock = 128;    // threads per block of the interpolation kernels
constexpr int kGatherTileBlock = 256;  // threads per tile in the LDS-staged interpolation
constexpr int kGatherTileBlockBig = 512;  // threads per 2 x 2-tile block of the same
constexpr int kTileX = 16;           // spread tile (grid points) before clamping to M/2
constexpr int kTileY = 8;
constexpr int kTileZ = 8;
constexpr int kMaxTilePts = kTileX * kTileY * kTileZ;
constexpr int kClasses = 27;         // stencil spill classes per tile (3 digits: low/none/high)
constexpr int kTileBins = 2 * kClasses;  // sort bins per tile: charged classes, then neutral
constexpr int kMaxRuns = 256;        // neighbour (tile, class-range) runs read by one spread tile
constexpr int kPairBlock = 192;      // threads per cell in the pair kernel (27 staging teams of 7)
constexpr int kSortBlock = 256;      // threads per block of the sort passes
constexpr int kSortPer = 2048;       // particles per counting block (before the cap)
constexpr int kSortMaxBlocks = 1024; // cap on counting blocks
constexpr int kSortBuckets = 256;    // target buckets per order
constexpr int kSortBucketsMax = 4096; // cap on the target for large systems (LDS of the count pass)
constexpr int kSortFineLog = 12;     // at most 2^12 keys per bucket
constexpr int kSortChunkMax = 2048;  // particles grouped in LDS at a time by the staging pass
constexpr int kSortStageBlock = 1024;  // threads per block of the staging pass
constexpr int kSortFineBlock = 1024; // threads per bucket in the fine pass
constexpr int kSortFineRegs = 8;     // particles per thread held in registers by the fine pass
constexpr int kFineOutBytes = 32768; // LDS window through which the fine pass writes its records
constexpr int kFineWindowBuckets = 512;  // at most this many buckets (2 blocks on each of 256 CUs) use it
constexpr int kFineWindowMin = 1024;     // ... or any number of buckets this full on average
constexpr int kTabSlots = 11;  // FFT / influence table offsets (see table_size)
constexpr int kESlots = 64;    // energy partials per part outside the deterministic mode (block mod 64)
constexpr int kDetSmall = 32;  // deterministic bin order: bins up to this size sorted by one thread
constexpr int kDetBig = 4096;  // ... and up to this size by one workgroup in LDS

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
  double iL[3];    // 1 / L, M / L, nc / L (formed once on the host)
  double mL[3];
  double cL[3];
  double alpha, rc, ke;
  double slater;   // ENUF-DPD decay length lambda_e of smeared charges (0: point charges)
  // window: 0 cardinal B-spline of order p; 1 Gaussian exp(-d^2/gb) of NFFT
  // cutoff m = p/2 - 1 (gib = 1/gb, in grid units)
  int win;
  double gb, gib;
  double sigma;    // oversampling factor: modes |n_d| < kept[d]/2 are kept
  int kept[3];
  // persistent binning (skin > 0): the sorted orders are kept while no
  // particle has moved more than skin/2; cells have side >= r_c + skin and the
  // tile spill classes a margin of sdig[d] grid points
  double skin;
  int sdig[3];
  // FP32 spread products: 0 FP32 matrix products; 1 split half-precision
  // products (three f16 products per pair of operands, ~21 bits)
  int spread16;
  int det;         // deterministic mode: particles within every bin in caller-index order
};
// Work::eslot: the reciprocal partials (one per z-pass block, at most
// (Mx/2) My, and at least the kESlots atomic slots), then the real-space ones
// (one per cell, at least kESlots)
inline size_t eslot_real_off(const Geom &g) {
  const size_t n = (size_t)(g.M[0] / 2) * g.M[1];
  return n > (size_t)kESlots ? n : (size_t)kESlots;
}
inline size_t eslot_len(const Geom &g) {
  return eslot_real_off(g) + ((size_t)g.ncells > (size_t)kESlots ? (size_t)g.ncells : (size_t)kESlots);
}

// Two-level counting sort layout: particles are counted in `nblk` blocks of
// `per`; the keys of order o (0 tile, 1 cell) are cut into nb[o] buckets of
// 2^sh[o] consecutive keys; the staging pass groups `chunk` particles at a
// time in LDS (0: no grouping, for bucket counts too large for that).
struct SortPlan {
  int nblk;
  int per;
  int chunk;
  int sh[2];
  int nb[2];
  int nbins[2];  // keys per order: kTileBins*ntiles, 2*ncells
  int window;    // fine pass: write through the LDS window (else gather reads)
};
SortPlan sort_plan(const Geom &g, int real_bytes);
size_t sort_stage_lds(const SortPlan &sp, int real_bytes);
size_t sort_fine_lds(const SortPlan &sp);

// Device workspace pointers (all owned by the context).
struct Work {
  void *part_t = nullptr;   // real4 [n] grid coords (s_x, s_y, s_z) + q, tile order
  void *part_c = nullptr;   // real4 [n] wrapped positions + q, cell order
  int *perm_t = nullptr;    // [n]
  int *perm_c = nullptr;    // [n]
  int *key_t = nullptr;     // [n] tile key per input particle; later the fine ranks (bucket order)
  int *key_c = nullptr;     // [n] cell key per input particle; later the fine ranks
  int *off_t = nullptr;     // [kTileBins*ntiles + 1] exclusive bin offsets, tile order
  int *off_c = nullptr;     // [2*ncells + 1] exclusive bin offsets, cell order
  int *hist = nullptr;      // [nblk][nb0 + nb1] per-block bucket counts, then block slots
  int *bbase = nullptr;     // [nb0 + 1 + nb1 + 1] bucket starts of each order and totals
  void *stg_t = nullptr;    // real4 [n] grid coords + q, bucket order (tile)
  void *stg_c = nullptr;    // real4 [n] wrapped positions + q, bucket order (cell)
  int2 *ik_t = nullptr;     // [n] (source index, key), bucket order
  int2 *ik_c = nullptr;
  int *runs = nullptr;      // [5*nruns] spread neighbour runs (dx, dy, dz, class lo, class hi)
  int nruns = 0;
  int *counts = nullptr;    // [8]: active, charged, flags, sort needed (persistent binning), all-active
                            // flag of the last sort, sorts performed, spare, spare
  void *x_ref = nullptr;    // real [n*3] positions at the last sort (persistent binning)
  void *q_ref = nullptr;    // real [n] charges at the last sort
  int *act = nullptr;       // [n] 1 for particles active at the last sort
  double *scal = nullptr;   // [4]: Q, Q2, max abs(q), spare
  double *qpart = nullptr;  // [4*nblk] per counting block: sum q, sum q^2, max abs(q), charged count
  double *eslot = nullptr;  // energy partials: [ (Mx/2) My ] reciprocal, then [ncells] real space; blocks
                            // add into slot block mod kESlots, or in the deterministic mode each block
                            // writes its own slot (summed in a fixed order)
  void *grid = nullptr;     // real [G]
  void *spec = nullptr;     // complex [G/2]
  void *fspec = nullptr;    // complex [4][G/2]
  void *field = nullptr;    // real4 [G]
  void *tables = nullptr;   // twiddles and window transforms (real)
  size_t tab_off[kTabSlots] = {0};  // element offsets inside `tables`
};

// Runs of (neighbour tile offset, class range) a spread tile reads; returns
// the number of runs and writes 5 ints per run into out (kMaxRuns capacity).
__host__ __device__ int build_runs(const Geom &g, int *out);
// Every transform pass of the grid fits one workgroup's LDS.
bool fft_plans_fit(const Geom &g, bool fp64);

// Twiddle / window tables: offsets (in reals) of each table, total size returned.
size_t table_size(const Geom &g, size_t off[kTabSlots]);
// Enqueue the workspace initialisation on `st`: tables, spread run table,
// cleared flags and energy slots (kernels only, no host copy).
hipError_t launch_init_ws(const Geom &g, const Work &w, hipStream_t st, bool fp64);

// One forward evaluation: every phase enqueued on `st`.  `ev` (optional) is
// an array of kPhases+1 events recorded between phases.  analytic: forces
// from the window derivative on the potential grid (one inverse transform,
// psi left as a plain real grid) instead of the three ik field grids.
constexpr int kPhases = 9;
template <typename R>
hipError_t launch_forward(const Geom &g, const Work &w, hipStream_t st, const R *x, const R *q,
                          double *E, R *F, R *phi, bool all_active, bool want_psi, bool analytic,
                          hipEvent_t *ev);

// Plain device copy of n16 16-byte words (the bandwidth probe).
hipError_t launch_copy16(const void *src, void *dst, size_t n16, hipStream_t st);

// Adjoint of the last forward: dEdx, dEdq (either may be null).  psi_scalar:
// the last forward left psi as a plain real grid (analytic mode).  gdev
// (optional): device double multiplying both outputs after gscale.
template <typename R>
hipError_t launch_adjoint(const Geom &g, const Work &w, hipStream_t st, double gscale, R *dEdx,
                          R *dEdq, bool psi_scalar, const double *gdev);

}  // namespace enuf
