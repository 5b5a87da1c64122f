/*
 * ewald_direct.c -- plain FP64 Ewald sum over explicit k-vectors.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle the ENUF hot path is checked
 * against.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline leg may load it.  It shares no code, header, table or constant
 * with the HIP library and includes nothing from it.
 *
 * What it computes (paper Sec. 2.1, Eq. 16-17, 22, 24-26, and the force
 * forms of Eq. 29 and Eq. 41 re-derived as gradients of the energy):
 *
 *   E   = E_R + E_K + E_self + E_bg
 *   E_R = ke * sum_{pairs, images, |r_ij + t| < r_c} q_i q_j erfc(a r)/r
 *   E_K = ke * (2 pi / V) * sum_{k != 0} exp(-k^2 / 4a^2) / k^2 * |S(k)|^2,
 *         S(k) = sum_j q_j exp(-i k.r_j),  k = 2 pi (nx/Lx, ny/Ly, nz/Lz)
 *   E_self = -ke * a / sqrt(pi) * sum_i q_i^2
 *   E_bg   = -ke * pi * Q^2 / (2 V a^2)     (neutralising background;
 *                                            zero for a neutral system)
 *   F_i  = -dE/dr_i,   phi_i = dE/dq_i.
 *
 * Everything is double precision, summed in plain loops; no blocking,
 * no fast-math.  OpenMP only splits independent outer loops.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Number of OpenMP threads the oracle will use (1 without OpenMP). */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Real-space pair term for one separation vector d (Eq. 17 energy, its
 * gradient for the force).  Adds into e, f[3] and phi (per unit q_j). */
static void pair_term(const double d[3], double qi, double qj, double alpha,
                      double ke, double *e, double f[3], double *phi_i) {
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double r = sqrt(r2);
    double ec = erfc(alpha * r) / r;
    /* -d/dr [erfc(a r)/r] = erfc(a r)/r^2 + 2a/sqrt(pi) exp(-a^2 r^2)/r */
    double fr = (ec + 2.0 * alpha / sqrt(M_PI) * exp(-alpha * alpha * r2)) / r2;
    *e += ke * qi * qj * ec;
    f[0] += ke * qi * qj * fr * d[0];
    f[1] += ke * qi * qj * fr * d[1];
    f[2] += ke * qi * qj * fr * d[2];
    *phi_i += ke * qj * ec;
}

/*
 * Real-space sum with explicit periodic images (Eq. 16 with the cutoff of
 * Eq. 17): every image vector t = (a Lx, b Ly, c Lz) with |r_i - r_j + t| < rc
 * is included, also i == j for t != 0.  Works for any rc; O(N^2 * images).
 * Outputs: *e (energy), f[N*3] forces, phi[N] potentials (any may be NULL).
 */
int oracle_real_images(int64_t n, const double *x, const double *q,
                       const double box[3], double alpha, double rc, double ke,
                       double *e_out, double *f, double *phi) {
    int nim[3];
    for (int d = 0; d < 3; ++d) nim[d] = (int)ceil(rc / box[d]) + 1;
    double etot = 0.0;
    double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : etot)
    for (int64_t i = 0; i < n; ++i) {
        double fi[3] = {0, 0, 0}, phii = 0.0, ei = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            for (int a = -nim[0]; a <= nim[0]; ++a)
                for (int b = -nim[1]; b <= nim[1]; ++b)
                    for (int c = -nim[2]; c <= nim[2]; ++c) {
                        if (i == j && a == 0 && b == 0 && c == 0) continue;
                        double d[3] = {x[3 * i] - x[3 * j] + a * box[0],
                                       x[3 * i + 1] - x[3 * j + 1] + b * box[1],
                                       x[3 * i + 2] - x[3 * j + 2] + c * box[2]};
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (r2 >= rc2) continue;
                        pair_term(d, q[i], q[j], alpha, ke, &ei, fi, &phii);
                    }
        }
        etot += 0.5 * ei; /* each (i, j, t) pair is visited from both ends */
        if (f) { f[3 * i] = fi[0]; f[3 * i + 1] = fi[1]; f[3 * i + 2] = fi[2]; }
        if (phi) phi[i] = phii;
    }
    if (e_out) *e_out = etot;
    return 0;
}

/*
 * Real-space sum under the minimum-image convention (valid when
 * rc <= min(L)/2, where at most one image of each pair lies inside rc).
 * Energy over all pairs i < j; forces and potentials for the particles
 * listed in `sample` (all particles when nsample < 0).  Particles with
 * q == 0 contribute nothing to the energy but still receive a potential.
 */
int oracle_real_minimage(int64_t n, const double *x, const double *q,
                         const double box[3], double alpha, double rc, double ke,
                         int64_t nsample, const int64_t *sample,
                         double *e_out, double *f, double *phi) {
    double rc2 = rc * rc;
    double etot = 0.0;
    /* only charged particles interact; list them once */
    int64_t nq = 0;
    for (int64_t i = 0; i < n; ++i) nq += (q[i] != 0.0);
    int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (nq ? nq : 1));
    if (!cid) return -1;
    nq = 0;
    for (int64_t i = 0; i < n; ++i) if (q[i] != 0.0) cid[nq++] = i;
    /* energy: all charged pairs i < j (skipped when no energy is asked for) */
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : etot)
    for (int64_t a = 0; a < (e_out ? nq : 0); ++a) {
        int64_t i = cid[a];
        double ei = 0.0;
        for (int64_t b = a + 1; b < nq; ++b) {
            int64_t j = cid[b];
            double d[3];
            for (int k = 0; k < 3; ++k) {
                double t = x[3 * i + k] - x[3 * j + k];
                d[k] = t - box[k] * nearbyint(t / box[k]);
            }
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 >= rc2) continue;
            double r = sqrt(r2);
            ei += ke * q[i] * q[j] * erfc(alpha * r) / r;
        }
        etot += ei;
    }
    if (e_out) *e_out = etot;
    /* forces and potentials on the sampled particles */
    int64_t ns = nsample < 0 ? n : nsample;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < ns; ++s) {
        int64_t i = nsample < 0 ? s : sample[s];
        double fi[3] = {0, 0, 0}, phii = 0.0, ei = 0.0;
        for (int64_t b = 0; b < nq; ++b) {
            int64_t j = cid[b];
            if (j == i) continue;
            double d[3];
            for (int k = 0; k < 3; ++k) {
                double t = x[3 * i + k] - x[3 * j + k];
                d[k] = t - box[k] * nearbyint(t / box[k]);
            }
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 >= rc2) continue;
            pair_term(d, q[i], q[j], alpha, ke, &ei, fi, &phii);
        }
        if (f) { f[3 * s] = fi[0]; f[3 * s + 1] = fi[1]; f[3 * s + 2] = fi[2]; }
        if (phi) phi[s] = phii;
    }
    free(cid);
    return 0;
}

/*
 * Real-space pair energy E_R (Eq. 17, minimum image, rc <= min(L)/2) over all
 * charged pairs, the pairs found through a cell list instead of the
 * all-pairs loop of oracle_real_minimage (same pair term, same result up to
 * the order of the sum).  The box is cut into nc_d = floor(L_d / rc) cells per
 * axis; with nc_d >= 3 every pair closer than rc lies in the same or an
 * adjacent cell, and the 27 neighbour cells of a cell are distinct.  The
 * charged particles are copied in cell order (counting sort), and each one
 * visits the particles after it in that order within its 27 neighbour
 * cells, so every pair is taken once.  Returns -2 when some axis has fewer
 * than 3 cells (use the all-pairs loop), -1 when an allocation fails.
 */
int oracle_real_cells_energy(int64_t n, const double *x, const double *q,
                             const double box[3], double alpha, double rc, double ke,
                             double *e_out) {
    int nc[3];
    for (int d = 0; d < 3; ++d) {
        double c = floor(box[d] / rc);
        if (c < 3.0) return -2;
        nc[d] = c > 512.0 ? 512 : (int)c;
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    double *xs = (double *)malloc(sizeof(double) * 4 * (size_t)(n ? n : 1));
    if (!start || !cid || !xs) {
        free(start); free(cid); free(xs);
        return -1;
    }
    /* cell of each charged particle from its wrapped position; counts */
    for (int64_t i = 0; i < n; ++i) {
        cid[i] = -1;
        if (q[i] == 0.0) continue;
        int k[3];
        for (int d = 0; d < 3; ++d) {
            double u = x[3 * i + d] / box[d];
            u -= floor(u);
            k[d] = (int)(u * nc[d]);
            if (k[d] >= nc[d]) k[d] = nc[d] - 1;
            if (k[d] < 0) k[d] = 0;
        }
        cid[i] = ((int64_t)k[2] * nc[1] + k[1]) * nc[0] + k[0];
        start[cid[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    /* copy (x, y, z, q) in cell order; fill[c] walks each cell's range */
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    if (!fill) {
        free(start); free(cid); free(xs);
        return -1;
    }
    for (int64_t c = 0; c < ncell; ++c) fill[c] = start[c];
    for (int64_t i = 0; i < n; ++i) {
        if (cid[i] < 0) continue;
        int64_t s = fill[cid[i]]++;
        xs[4 * s] = x[3 * i];
        xs[4 * s + 1] = x[3 * i + 1];
        xs[4 * s + 2] = x[3 * i + 2];
        xs[4 * s + 3] = q[i];
    }
    free(fill);
    const double rc2 = rc * rc;
    double etot = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : etot)
    for (int64_t c = 0; c < ncell; ++c) {
        const int cx0 = (int)(c % nc[0]);
        const int cy0 = (int)((c / nc[0]) % nc[1]);
        const int cz0 = (int)(c / ((int64_t)nc[0] * nc[1]));
        double ec = 0.0;
        for (int64_t s = start[c]; s < start[c + 1]; ++s) {
            const double *pi = xs + 4 * s;
            for (int a = -1; a <= 1; ++a)
                for (int b = -1; b <= 1; ++b)
                    for (int e = -1; e <= 1; ++e) {
                        int cx = (cx0 + a + nc[0]) % nc[0];
                        int cy = (cy0 + b + nc[1]) % nc[1];
                        int cz = (cz0 + e + nc[2]) % nc[2];
                        int64_t nb = ((int64_t)cz * nc[1] + cy) * nc[0] + cx;
                        int64_t t0 = start[nb] > s ? start[nb] : s + 1;
                        for (int64_t t = t0; t < start[nb + 1]; ++t) {
                            const double *pj = xs + 4 * t;
                            double dd[3];
                            for (int k = 0; k < 3; ++k) {
                                double u = pi[k] - pj[k];
                                dd[k] = u - box[k] * nearbyint(u / box[k]);
                            }
                            double r2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
                            if (r2 >= rc2) continue;
                            double r = sqrt(r2);
                            ec += ke * pi[3] * pj[3] * erfc(alpha * r) / r;
                        }
                    }
        }
        etot += ec;
    }
    *e_out = etot;
    free(start); free(cid); free(xs);
    return 0;
}

/* exp(-i * 2 pi * m * u) for m = m0 .. m0+cnt-1 (u = r/L in [0,1)); the
 * argument is reduced to a fraction of a turn before cos/sin. */
static void phase_row(double u, int m0, int cnt, double *re, double *im) {
    for (int t = 0; t < cnt; ++t) {
        double v = (double)(m0 + t) * u;
        v -= floor(v);
        double ang = -2.0 * M_PI * v;
        re[t] = cos(ang);
        im[t] = sin(ang);
    }
}

/*
 * Reciprocal-space sum over explicit k-vectors (Eq. 22/25/26; force as the
 * exact gradient, which is the form of Eq. 41 for an orthorhombic box):
 *
 *   E_K    = ke (2pi/V) sum_{k in K} A(k) |S(k)|^2,  A = exp(-k^2/4a^2)/k^2
 *   F_i    = ke (4pi q_i/V) sum_{k in K} A(k) k Im(S(k) exp(+i k.r_i))
 *   phi_i  = ke (4pi/V)     sum_{k in K} A(k)   Re(S(k) exp(+i k.r_i))
 *
 * K = { n != 0 : |n_d| <= nmax[d], and k^2 <= kcut2 when kcut2 > 0 }.  K is
 * symmetric under n -> -n and each summand is even, so the loop runs over
 * the half space (nx > 0) u (nx = 0, ny > 0) u (nx = ny = 0, nz > 0) with
 * weight 2.  Forces/potentials are produced for the particles in `sample`
 * (all when nsample < 0), neutral ones included (their potential is dE/dq).
 */
int oracle_recip(int64_t n, const double *x, const double *q, const double box[3],
                 double alpha, double ke, const int32_t nmax[3], double kcut2,
                 int64_t nsample, const int64_t *sample,
                 double *e_out, double *f, double *phi) {
    const double V = box[0] * box[1] * box[2];
    const int nx1 = nmax[0] + 1, ny1 = 2 * nmax[1] + 1, nz1 = 2 * nmax[2] + 1;
    /* charged particles only enter S(k) */
    int64_t nq = 0;
    for (int64_t i = 0; i < n; ++i) nq += (q[i] != 0.0);
    int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (nq ? nq : 1));
    nq = 0;
    for (int64_t i = 0; i < n; ++i) if (q[i] != 0.0) cid[nq++] = i;
    int64_t ns = nsample < 0 ? n : nsample;
    /* phase tables: x: m in [0, nmax_x]; y, z: m in [-nmax, nmax] */
    size_t rowlen = (size_t)nx1 + ny1 + nz1;
    double *tre = (double *)malloc(sizeof(double) * rowlen * (size_t)(nq + ns));
    double *tim = (double *)malloc(sizeof(double) * rowlen * (size_t)(nq + ns));
    if (!cid || !tre || !tim) { free(cid); free(tre); free(tim); return -1; }
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < nq + ns; ++a) {
        int64_t i = a < nq ? cid[a] : (nsample < 0 ? a - nq : sample[a - nq]);
        double *re = tre + rowlen * a, *im = tim + rowlen * a;
        double u[3];
        for (int d = 0; d < 3; ++d) {
            double v = x[3 * i + d] / box[d];
            u[d] = v - floor(v);
        }
        phase_row(u[0], 0, nx1, re, im);
        phase_row(u[1], -nmax[1], ny1, re + nx1, im + nx1);
        phase_row(u[2], -nmax[2], nz1, re + nx1 + ny1, im + nx1 + ny1);
    }
    int nthr = oracle_num_threads();
    double *facc = (double *)calloc((size_t)nthr * ns * 4, sizeof(double));
    double etot = 0.0;
    const int64_t ncol = (int64_t)nx1 * ny1;
#pragma omp parallel reduction(+ : etot)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = facc + (size_t)tid * ns * 4;
        double *sre = (double *)malloc(sizeof(double) * nz1);
        double *sim = (double *)malloc(sizeof(double) * nz1);
#pragma omp for schedule(dynamic, 1)
        for (int64_t col = 0; col < ncol; ++col) {
            int mx = (int)(col / ny1);
            int my = (int)(col % ny1) - nmax[1];
            if (mx == 0 && my < 0) continue;  /* half space */
            double kx = 2.0 * M_PI * mx / box[0], ky = 2.0 * M_PI * my / box[1];
            double kxy2 = kx * kx + ky * ky;
            if (kcut2 > 0.0 && kxy2 > kcut2) continue;
            int zlo = -nmax[2], zhi = nmax[2];
            if (mx == 0 && my == 0) zlo = 1;
            if (kcut2 > 0.0) {
                int zm = (int)floor(sqrt((kcut2 - kxy2)) * box[2] / (2.0 * M_PI));
                if (zm < zhi) zhi = zm;
                if (-zm > zlo) zlo = -zm;
            }
            if (zlo > zhi) continue;
            int cnt = zhi - zlo + 1;
            for (int t = 0; t < cnt; ++t) { sre[t] = 0.0; sim[t] = 0.0; }
            /* S(k) = sum_j q_j e^{-i kx x_j} e^{-i ky y_j} e^{-i kz z_j} */
            for (int64_t a = 0; a < nq; ++a) {
                const double *re = tre + rowlen * a, *im = tim + rowlen * a;
                double qj = q[cid[a]];
                double xr = re[mx], xi = im[mx];
                double yr = re[nx1 + my + nmax[1]], yi = im[nx1 + my + nmax[1]];
                double cr = qj * (xr * yr - xi * yi), ci = qj * (xr * yi + xi * yr);
                const double *zr = re + nx1 + ny1 + (zlo + nmax[2]);
                const double *zi = im + nx1 + ny1 + (zlo + nmax[2]);
                for (int t = 0; t < cnt; ++t) {
                    sre[t] += cr * zr[t] - ci * zi[t];
                    sim[t] += cr * zi[t] + ci * zr[t];
                }
            }
            for (int t = 0; t < cnt; ++t) {
                int mz = zlo + t;
                double kz = 2.0 * M_PI * mz / box[2];
                double k2 = kxy2 + kz * kz;
                if (kcut2 > 0.0 && k2 > kcut2) continue;
                double A = exp(-k2 / (4.0 * alpha * alpha)) / k2;
                /* weight 2: the mirrored vector -k contributes the same */
                etot += 2.0 * ke * (2.0 * M_PI / V) * A * (sre[t] * sre[t] + sim[t] * sim[t]);
                if (ns == 0) continue;
                double kv[3] = {kx, ky, kz};
                for (int64_t s = 0; s < ns; ++s) {
                    const double *re = tre + rowlen * (nq + s), *im = tim + rowlen * (nq + s);
                    /* e^{+i k.r_s} = conj(e^{-i k.r_s}) */
                    double xr = re[mx], xi = -im[mx];
                    double yr = re[nx1 + my + nmax[1]], yi = -im[nx1 + my + nmax[1]];
                    double zr = re[nx1 + ny1 + mz + nmax[2]], zi = -im[nx1 + ny1 + mz + nmax[2]];
                    double pr = xr * yr - xi * yi, pi_ = xr * yi + xi * yr;
                    double er = pr * zr - pi_ * zi, ei = pr * zi + pi_ * zr;
                    double vr = sre[t] * er - sim[t] * ei;  /* Re(S e^{ik.r}) */
                    double vi = sre[t] * ei + sim[t] * er;  /* Im(S e^{ik.r}) */
                    double cf = 2.0 * ke * (4.0 * M_PI / V) * A;
                    acc[4 * s + 0] += cf * kv[0] * vi;
                    acc[4 * s + 1] += cf * kv[1] * vi;
                    acc[4 * s + 2] += cf * kv[2] * vi;
                    acc[4 * s + 3] += cf * vr;
                }
            }
        }
        free(sre);
        free(sim);
    }
    for (int64_t s = 0; s < ns; ++s) {
        int64_t i = nsample < 0 ? s : sample[s];
        double a4[4] = {0, 0, 0, 0};
        for (int t = 0; t < nthr; ++t)
            for (int c = 0; c < 4; ++c) a4[c] += facc[((size_t)t * ns + s) * 4 + c];
        if (f) { f[3 * s] = q[i] * a4[0]; f[3 * s + 1] = q[i] * a4[1]; f[3 * s + 2] = q[i] * a4[2]; }
        if (phi) phi[s] = a4[3];
    }
    if (e_out) *e_out = etot;
    free(facc);
    free(cid);
    free(tre);
    free(tim);
    return 0;
}
