/*
 * enuf.h -- C ABI of the ENUF hot path on AMD Instinct MI355X (gfx950).
 *
 * ENUF is Ewald summation whose reciprocal-space part is evaluated with
 * non-uniform FFTs (paper Sec. 2.3).  For N point charges q_i at r_i in a
 * periodic orthorhombic box (tin-foil boundary, Sec. 2.1) the library
 * returns
 *
 *     E = E_R + E_K + E_self + E_bg,        F_i = -dE/dr_i
 *
 *   E_R    real-space erfc pair sum inside r_c (Eq. 17), forces from its
 *          gradient (the corrected form of Eq. 29); pairs at distance 0
 *          (coincident sites, whose Coulomb energy is infinite) are skipped;
 *   E_K    reciprocal energy from the structure factor S(n) (Eq. 37-38),
 *          S(n) computed by a type-1 ("transposed", Eq. 36) NFFT:
 *          spread -> 3D FFT -> divide by the window transform;
 *          forces from three type-2 ("conjugated", Eq. 35, 41-42) NFFTs;
 *   E_self Gaussian self energy (Eq. 24, subtracted as in Eq. 25);
 *   E_bg   neutralising-background energy -ke pi Q^2 / (2 V alpha^2), zero
 *          for neutral systems (the paper assumes neutrality).
 *
 * Readings fixed by this library: the grid M is the FFT size per axis and,
 * by default, all its modes except the Nyquist index -M/2 are kept (no
 * oversampling); the default window is the centred cardinal B-spline of
 * order p (p grid points of support per axis) and the scaling step divides
 * by its continuous Fourier transform sinc^p(pi n/M).  The paper's own NFFT
 * form (Gaussian window, oversampling) is available through
 * ENUF_OPT_WINDOW and ENUF_OPT_OVERSAMPLING.
 *
 * Conventions for every call:
 *  - Return value: ENUF_OK (0) or an error code; a failed call has no effect
 *    on the context except the text behind enuf_last_error().
 *  - Pointers named "device" must be device memory of the context's GPU
 *    (e.g. a torch tensor's data_ptr()).  The caller owns all of them; the
 *    library never frees caller memory.  The library owns its host context.
 *    Device working memory is the caller's (enuf_workspace_bytes +
 *    enuf_set_workspace), or allocated by the library only when asked
 *    (enuf_alloc_workspace, released by enuf_destroy()); enuf_create and the
 *    evaluation calls allocate no device memory.
 *  - "real" is double for ENUF_FP64 contexts and float for ENUF_FP32.
 *  - Device work is enqueued on the context's HIP stream and is NOT
 *    synchronised on return unless a call says so.  Calls on one context are
 *    stream-ordered and not re-entrant (one host thread at a time).
 */
#ifndef ENUF_H
#define ENUF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct enuf_ctx_s *enuf_ctx;

typedef enum {
    ENUF_OK = 0,
    ENUF_EINVAL = 1,        /* invalid argument (NULL, size, parameter range) */
    ENUF_ENOMEM = 2,        /* host or device allocation failed */
    ENUF_EDEVICE = 3,       /* a HIP runtime call failed */
    ENUF_ENONFINITE = 4,    /* non-finite position or charge seen on the device */
    ENUF_ESTATE = 5,        /* call sequence error (e.g. grad before forward) */
    ENUF_EUNSUPPORTED = 6   /* valid request outside what the library handles */
} enuf_status;

typedef enum { ENUF_FP64 = 0, ENUF_FP32 = 1 } enuf_precision;

/* Options for enuf_set_option(). */
typedef enum {
    ENUF_OPT_KE = 0,          /* Coulomb prefactor 1/(4 pi eps0 eps_r); default 1 */
    ENUF_OPT_TIMING = 1,      /* n > 0: record per-phase HIP events for each
                                    evaluation in a ring of n slots; 0: off
                                    (default) */
    ENUF_OPT_GRAPH = 2,       /* 1: enuf_energy_forces replays its launch
                                 sequence as a HIP graph on a stream of the
                                 context's own, joined to the context stream
                                 by events before and after (captured on the
                                 first call and again whenever x, q, E, F,
                                 phi, the workspace or an option change);
                                 per-phase timing is not recorded then.
                                 Default 0 (kernels launched one by one). */
    ENUF_OPT_CHECK = 3,       /* 1: enuf_energy_forces synchronises and reports
                                    ENUF_ENONFINITE itself; default 0 */
    ENUF_OPT_FORCE_MODE = 4,  /* reciprocal forces.  0 (default): ik
                                 differentiation as in the paper's Eq. 41-42:
                                 three field grids are transformed back and
                                 interpolated; the forces sum to zero up to
                                 rounding.  1: analytic differentiation of the
                                 window: only the potential grid psi is
                                 transformed back and the gather uses the
                                 window's derivative, so the forces are the
                                 exact negative gradient of the computed
                                 energy; their sum is zero only to the
                                 method's accuracy.  One inverse transform
                                 instead of three. */
    ENUF_OPT_SLATER = 5,      /* ENUF-DPD (paper Sec. 2.4, Eq. 51-58): value =
                                 lambda_e > 0, the decay length of Slater-type
                                 smeared charges (beta = R_c / lambda_e); 0
                                 (default): point charges.  Each real-space
                                 pair term is scaled, energy and potential by
                                 B_U(r) = 1 - (1 + r/lambda_e) exp(-2r/lambda_e)
                                 and force by B_F(r) = 1 - (1 + 2(r/lambda_e)
                                 (1 + r/lambda_e)) exp(-2r/lambda_e); the
                                 reciprocal and self terms are those of point
                                 charges (the paper's choice of a real-space
                                 cutoff past which both factors are ~1).  The
                                 adjoint (enuf_energy_grad) differentiates the
                                 scaled energy exactly; for the erfc-screened
                                 pair term that differs from the B_F-scaled
                                 force, which follows the paper. */
    ENUF_OPT_WINDOW = 6,      /* NFFT window (paper Sec. 2.2): 0 (default)
                                 cardinal B-spline of order p; 1 the
                                 Gaussian exp(-d^2/b) of the paper's NFFT
                                 (Sec. 3.1), cutoff m = p/2 - 1 on the same
                                 p = 2m + 2 stencil points floor(s) - m ..
                                 floor(s) + m + 1, shape
                                 b = 2 sigma m / ((2 sigma - 1) pi), scaling
                                 by its transform sqrt(pi b) exp(-b (pi n/M)^2);
                                 needs p >= 4. */
    ENUF_OPT_OVERSAMPLING = 7,/* oversampling factor sigma >= 1 (Sec. 2.2,
                                 2.3.2): of the M_d-point grid only the modes
                                 |n_d| < K_d/2, K_d = 2 floor(M_d/(2 sigma)),
                                 enter the k-space sums (default 1: every
                                 mode but the Nyquist index).  Setting either
                                 option re-initialises the workspace tables
                                 on the stream and forgets the last
                                 evaluation (a following enuf_energy_grad
                                 reports ENUF_ESTATE). */
    ENUF_OPT_SKIN = 8,        /* persistent binning for MD (skin length
                                 >= 0; default 0: every evaluation sorts).
                                 With skin s > 0 the particle orders of the
                                 last sort are kept while no particle has
                                 moved more than s/2 (minimum image) since
                                 it, every charge is unchanged and the phi
                                 request matches; the check runs on the
                                 device (no host synchronisation) and an
                                 evaluation that keeps the orders only
                                 refreshes the sorted positions.  Real-space
                                 cells then have side > r_c + s, the spread's
                                 tile classes a margin of ceil(s/2 M/L) grid
                                 points (ENUF_EUNSUPPORTED when p plus twice
                                 that exceeds the spread tile plus one), and
                                 the interpolation reads the grid per
                                 particle.  Results equal those of a sorting
                                 evaluation up to summation order.  The
                                 cell geometry changes, so a context with a
                                 workspace lays it out again (ENUF_ESTATE if
                                 it is too small) and forgets the last
                                 evaluation. */
    ENUF_OPT_SPREAD_F16 = 9,  /* FP32 contexts: products of the spread's
                                 tile contraction.  0 (default): FP32 matrix
                                 products with FP32 accumulation.  1: each
                                 operand split into two half-precision parts
                                 and the product taken as three
                                 half-precision matrix products (hi*hi +
                                 hi*lo + lo*hi, ~21 significant bits per
                                 product, FP32 accumulation): faster, not
                                 FP32 arithmetic.  No effect in FP64. */
    ENUF_OPT_DETERMINISTIC = 10 /* 1: run-to-run bitwise reproducible
                                 results for the same inputs and options on
                                 the same device: after each sort the
                                 particles of every bin are put in caller-index
                                 order (so spread, pair and energy sums run in
                                 one order).  A bin of more than 4096
                                 particles cannot be ordered: flag bit 1
                                 (enuf_get_flags) is set.  Default 0.  The
                                 energy partials are summed in a fixed order
                                 in either mode. */
} enuf_option;

/* Internal buffers enuf_stage_copy() can read (for tests of single steps). */
typedef enum {
    ENUF_STAGE_GRID = 0,      /* spread output rho, real [Mz][My][Mx] */
    ENUF_STAGE_SPECTRUM = 1,  /* forward 3D FFT of rho over (kx<Mx/2): complex
                                 [Mz][My][Mx/2], the z transform not applied
                                 (it happens fused with the influence step) */
    ENUF_STAGE_FIELDS = 2,    /* real-space fields after the inverse FFTs, real
                                 [Mz][My][Mx][4] = (E_x, E_y, E_z, psi); psi is
                                 0 unless the evaluation requested phi.  After
                                 an evaluation in force mode 1: psi alone,
                                 real [Mz][My][Mx] */
    ENUF_STAGE_SORTED = 3,    /* int32 [N] permutation, grid-tile order
                                 (entries past the active count are unused) */
    ENUF_STAGE_COUNTS = 4,    /* int32 [8]: active particles, charged particles,
                                 non-finite flag, (internal), (internal),
                                 sorts performed since the workspace was
                                 set, (spare), (spare) */
    ENUF_STAGE_CELLS = 5      /* int32 [N] permutation, pair-cell order */
} enuf_stage;

/*
 * enuf_create -- validate parameters and set up a context (paper Sec. 2.3:
 * box, N, Ewald alpha, real-space cutoff r_c; Sec. 2.2: grid M and window).
 *   out      receives the context (set to NULL on failure)
 *   box      host double[3] box lengths (Lx, Ly, Lz) > 0
 *   n        number of particles, 1 .. 2^28
 *   alpha    Ewald splitting parameter > 0 (alpha = 1/(sqrt 2 sigma), Sec. 2.1)
 *   r_c      real-space cutoff, 0 < r_c <= min(L)/2 (minimum image)
 *   M        host int32[3] FFT grid (Mx, My, Mz); powers of two in [8, 1024]
 *   p        window stencil width: 2, 4, 6 or 8, with 2p <= M_d for every axis
 *   precision ENUF_FP64 or ENUF_FP32 (spread/FFT/gather/pair arithmetic;
 *            energies are always reduced in double)
 *   stream   hipStream_t to enqueue on (NULL = default stream)
 * Allocates no device memory: give the context a workspace with
 * enuf_set_workspace() (or enuf_alloc_workspace()) before evaluating.  Selects the current HIP device as the
 * context's device.
 */
enuf_status enuf_create(enuf_ctx *out, const double box[3], int64_t n, double alpha,
                        double r_c, const int32_t M[3], int32_t p, int32_t precision,
                        void *stream);

/* enuf_workspace_bytes -- device bytes the context's workspace needs
 * (particle copies and sort buffers, about 16 reals + 40 bytes per
 * particle; grid, half spectrum, four field spectra and four field grids,
 * 10 reals per grid point; tables).  Any alignment of the block is accepted:
 * the figure includes 256 bytes of slack. */
enuf_status enuf_workspace_bytes(enuf_ctx ctx, size_t *bytes);

/* enuf_set_workspace -- use caller-owned device memory ws (at least
 * enuf_workspace_bytes() bytes, e.g. a torch uint8 tensor) as the context's
 * workspace.  Enqueues its initialisation (FFT twiddles, influence factors,
 * cleared flags) on the context stream; the memory must stay valid until the
 * context is destroyed or another workspace is set, and must not be used by
 * anything else meanwhile.  Forgets the previous evaluation (a following
 * enuf_energy_grad reports ENUF_ESTATE).  ENUF_EINVAL when ws is NULL or too
 * small. */
enuf_status enuf_set_workspace(enuf_ctx ctx, void *ws, size_t bytes);

/* enuf_alloc_workspace -- allocate the workspace with hipMalloc and set it
 * (owned by the library, freed by enuf_destroy); ENUF_ENOMEM on failure. */
enuf_status enuf_alloc_workspace(enuf_ctx ctx);

/* enuf_destroy -- free the context and a workspace the library allocated.
 * NULL -> ENUF_EINVAL. */
enuf_status enuf_destroy(enuf_ctx ctx);

/* enuf_set_option -- set one enuf_option (value range checked). */
enuf_status enuf_set_option(enuf_ctx ctx, int32_t option, double value);

/* enuf_set_stream -- enqueue later calls on another hipStream_t. */
enuf_status enuf_set_stream(enuf_ctx ctx, void *stream);

/*
 * enuf_energy_forces -- one full evaluation (Sec. 3.2: real and reciprocal
 * space on the GPU; forward NFFT for S(n) and the energy, Eq. 37-38; three
 * inverse NFFTs packed into one pass for the forces, Eq. 41-42).
 *   x    device real[N*3] positions, row-major (x,y,z); any values, wrapped
 *        into the box; non-finite rows are excluded and flagged
 *   q    device real[N] charges
 *   E    device double[5] out: (total, E_R, E_K, E_self, E_bg)
 *   F    device real[N*3] out forces, or NULL for energy only
 *   phi  device real[N] out potentials phi_i = dE/dq_i, or NULL.  When
 *        given, every particle (neutral ones too) gets its potential and the
 *        potential field is transformed as a fourth inverse FFT; without it
 *        only the three force fields are.
 * The reciprocal forces are the ik-differentiated ones of Eq. 41-42, which
 * sum to zero exactly; they approximate -dE/dr.  The exact gradient of the
 * computed energy is available from enuf_energy_grad().  Non-finite input is
 * recorded in a device flag read by enuf_get_flags() (or reported directly
 * with ENUF_OPT_CHECK).  ENUF_ESTATE when the context has no workspace.
 */
enuf_status enuf_energy_forces(enuf_ctx ctx, const void *x, const void *q, double *E,
                               void *F, void *phi);

/*
 * enuf_energy_grad -- adjoint of the last enuf_energy_forces() on this
 * context: the exact gradient of the energy E it computed, scaled by
 * grad_E.  Uses the sorted particles and the potential grid kept from that
 * call (x and q are not read again); that call must have requested phi
 * (which makes every particle active and transforms the potential field),
 * otherwise ENUF_ESTATE.
 *   dEdx  device real[N*3] out: grad_E * dE/dr_i (window-derivative gather on
 *         the potential grid, plus the real-space gradient), or NULL
 *   dEdq  device real[N] out: grad_E * dE/dq_i, or NULL
 * The gradient is that of the energy with the parameters (ke, Slater length)
 * the forward call used, whatever enuf_set_option() changed since.
 * ENUF_ESTATE when no forward evaluation preceded it.
 */
enuf_status enuf_energy_grad(enuf_ctx ctx, double grad_E, void *dEdx, void *dEdq);

/* enuf_eval_token -- identifier of the context's last enuf_energy_forces()
 * (a count of evaluations; 0 before the first). */
enuf_status enuf_eval_token(enuf_ctx ctx, uint64_t *token);

/* enuf_energy_grad_dev -- as enuf_energy_grad(), for the evaluation whose
 * enuf_eval_token() was `token`, with the upstream gradient read from device
 * memory grad_E (one double) on the stream, so that no host
 * synchronisation is needed.  ENUF_ESTATE when the context has evaluated
 * again since (its kept state belongs to another configuration). */
enuf_status enuf_energy_grad_dev(enuf_ctx ctx, uint64_t token, const double *grad_E, void *dEdx,
                                 void *dEdq);

/* Bytes of the static device scratch enuf_energy_forces_noalloc() works in
 * (64 MiB per GPU). */
#define ENUF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * enuf_energy_forces_noalloc -- enuf_energy_forces() for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same evaluation, kernels and outputs,
 * but its working memory is a static device array of the library
 * (ENUF_NOALLOC_SCRATCH_BYTES per GPU, created when the library's code object
 * is loaded onto a GPU and held until the process ends), not the context's
 * workspace; the context needs no workspace.  The call allocates and frees
 * nothing; the caller still provides x, q, E, F and phi as for
 * enuf_energy_forces().
 *   Size limit: ENUF_EUNSUPPORTED (with the byte counts in
 *   enuf_last_error) when the context's enuf_workspace_bytes() exceeds
 *   ENUF_NOALLOC_SCRATCH_BYTES (e.g. 32768 particles on a 64^3 grid in FP64
 *   fit; a million particles on 256^3 do not).
 *   Sharing: every call on one GPU uses that GPU's one scratch array, and
 *   each call re-initialises it (tables, counters, flags, energy slots) on
 *   the context's stream before evaluating.  Calls whose device work
 *   overlaps on one GPU (different streams or host threads without ordering)
 *   race on the scratch and give wrong results; order them on one stream.
 *   It does not change the context's adjoint state: enuf_energy_grad() and
 *   enuf_eval_token() still refer to the last enuf_energy_forces() on the
 *   context.  ENUF_OPT_GRAPH and ENUF_OPT_TIMING do not apply (kernels are
 *   launched one by one, no events recorded); ENUF_OPT_CHECK does.
 */
enuf_status enuf_energy_forces_noalloc(enuf_ctx ctx, const void *x, const void *q, double *E,
                                       void *F, void *phi);

/* enuf_get_flags -- synchronise the stream and return the sticky device
 * flags (bit 0: non-finite input seen; bit 1: a bin too large for the
 * deterministic order); clears them. */
enuf_status enuf_get_flags(enuf_ctx ctx, int32_t *flags);

/* enuf_stage_copy -- synchronously copy an internal buffer (enuf_stage) of
 * the last evaluation into device memory dst of at least `bytes` bytes. */
enuf_status enuf_stage_copy(enuf_ctx ctx, int32_t stage, void *dst, size_t bytes);

/* enuf_stage_bytes -- size in bytes of an enuf_stage buffer. */
enuf_status enuf_stage_bytes(enuf_ctx ctx, int32_t stage, size_t *bytes);

/* enuf_get_timings -- per-phase milliseconds averaged over the evaluations
 * recorded since the previous read (at most the ring size set with
 * ENUF_OPT_TIMING), measured with HIP events on the context's stream;
 * synchronises, then starts a new averaging window.  Fills up to n values in
 * the order prep, sort, spread, fft_fwd, influence+z, fft_inv, gather, pair,
 * finalize; *count receives the number of phases.  ENUF_ESTATE when timing
 * is off, nothing was recorded, or graph replay is on. */
enuf_status enuf_get_timings(enuf_ctx ctx, double *ms, int32_t n, int32_t *count);

/* enuf_get_step_timings -- the same events per evaluation: ms[k * 9 + i] is
 * phase i of the k-th recorded evaluation (oldest first, at most cap of
 * them, the last ENUF_OPT_TIMING slots); *count receives the number of
 * evaluations.  Synchronises and starts a new window, like
 * enuf_get_timings(). */
enuf_status enuf_get_step_timings(enuf_ctx ctx, double *ms, int32_t cap, int32_t *count);

/* How enuf_select_params chose (its `method` output). */
enum { ENUF_SELECT_HEURISTIC = 0, ENUF_SELECT_NETWORK = 1 };

/*
 * enuf_select_params -- ENUF parameters (alpha, r_c, grid M, window p) for a
 * system and a target RMS relative force error (paper Sec. 2.3.2: the error
 * relations of Eq. 31-32 and the choice of the reciprocal cutoff n_c).
 *   box            host double[3] box lengths > 0
 *   n              number of particles >= 2
 *   charged_frac   fraction of charged particles, in (0, 1]
 *   target_rms_err target RMS relative force error, in (0, 1)
 *   model_path     NULL: the heuristic.  Else the trained parameter network
 *                  (file written by the package's training script): when
 *                  the system lies inside the ranges it was trained on (N,
 *                  density, charged fraction, target, box shape, all stored
 *                  in the file) its prediction is evaluated on the current
 *                  HIP device with enuf_mlp_forward and snapped to a valid
 *                  setting; outside them the heuristic is used.
 *   alpha, r_c     out (host): splitting parameter and real-space cutoff
 *                  (r_c <= min(L)/2)
 *   M              out (host int32[3]): grid, powers of two in [8, 512]
 *   p              out (host): window width (4, 6 or 8 with 2p <= M)
 *   method         out (host, may be NULL): ENUF_SELECT_HEURISTIC or
 *                  ENUF_SELECT_NETWORK
 * Heuristic: alpha and r_c from Eq. 31 and 32 at equality,
 * exp(-pi^2 n_c^2/(alpha L_x)^2) = exp(-alpha^2 r_c^2) = target, with n_c
 * raised from 2 until r_c <= min(3 a, min(L)/2) (a = (V/N)^(1/3), the mean
 * spacing); every mode up to n_c is kept on each axis; p = 6.
 * Network evaluation allocates (and frees) a small device buffer and
 * synchronises.  Errors: ENUF_EINVAL for bad arguments or an unreadable or
 * malformed network file, ENUF_EDEVICE/ENUF_ENOMEM for device failures; the
 * text is in enuf_select_last_error().
 */
enuf_status enuf_select_params(const double box[3], int64_t n, double charged_frac,
                               double target_rms_err, const char *model_path, double *alpha,
                               double *r_c, int32_t M[3], int32_t *p, int32_t *method);

/* enuf_select_last_error -- text of the last enuf_select_params error on
 * this host thread. */
const char *enuf_select_last_error(void);

/* enuf_status_string -- static text for a status code. */
const char *enuf_status_string(enuf_status s);

/* enuf_last_error -- text of the last error on ctx (or of the last failed
 * enuf_create when ctx is NULL); valid until the next call on ctx. */
const char *enuf_last_error(enuf_ctx ctx);

/* enuf_device_count -- number of visible HIP devices (0 without a GPU;
 * never fails). */
int32_t enuf_device_count(void);

/* enuf_copy_probe -- a plain device-to-device copy of `bytes` bytes from
 * src to dst (device pointers, 16-byte aligned, bytes a multiple of 16, the
 * ranges not overlapping) with this library's own kernel, enqueued on
 * `stream` (NULL: the null stream).  A measurement aid, not part of the
 * method: the achievable copy bandwidth it shows is the second denominator
 * the HBM-bound kernels are reported against, beside the published peak.
 * ENUF_EINVAL for a NULL pointer, misalignment or a bad size; ENUF_EDEVICE
 * if the launch fails. */
enuf_status enuf_copy_probe(const void *src, void *dst, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ENUF_H */
