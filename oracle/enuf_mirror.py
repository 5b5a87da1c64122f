"""ENUF reciprocal-space steps in plain numpy FP64.

TEST INFRASTRUCTURE ONLY: the second half of the oracle.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import it.  It
imports nothing from the HIP library or its package; the real-space pair sum
comes from the direct oracle (``oracle/ewald.py``).

ENUF approximates the k-space part of the Ewald sum (paper Sec. 2.3.1) by
non-uniform FFTs, computed with the gridding steps of Sec. 3.1 (Fig. 4):

  forward ("transposed" NFFT, Eq. 36/37):
    spread   rho_l = sum_i q_i phi(s_i - l)        on a grid of M_d points
    FFT      rho^(n) = sum_l rho_l exp(-2 pi i n.l/M)
    scale    S~(n) = rho^(n) / c(n)                (window Fourier coefficients)
    energy   U^K = ke (2 pi / V) sum_{n in K} A(k) |S~(n)|^2       (Eq. 38)
  inverse ("conjugated" NFFT, Eq. 35/41/42), one per force component:
    subdivide  g^_d(n) = -i k_d A(k) S~(n) / c(n)
    inverse FFT  g_d(l) = sum_n g^_d(n) exp(+2 pi i n.l/M)
    interpolate  F_i,d = ke (4 pi / V) q_i sum_l phi(s_i - l) g_d(l)

with s_i = M r_i / L (grid coordinates), k_d = 2 pi n_d / L_d and
A(k) = exp(-k^2/4a^2)/k^2.  The same grid machinery gives the potential
(psi^ = A S~ / c, phi_i = dU/dq_i) and the exact gradient of this discrete
energy (interpolating psi with the window's derivative).

Readings of the paper taken here (where it is silent or ambiguous):
  * M is the FFT grid per axis and every mode of it is kept (no
    oversampling), K = {n : -M_d/2 < n_d < M_d/2} minus n = 0; the
    self-mirrored Nyquist index -M_d/2 is dropped so K is symmetric and the
    force fields are real.  (Eq. 33 writes the index set inclusively at both
    ends, which contradicts the point count M_Pi = prod M_t stated with it.)
  * The window is the centred cardinal B-spline of order p (p grid points of
    support per axis, p = 2m in the paper's NFFT cutoff m); the paper lists
    B-splines among its NFFT windows.  c(n) is the window's continuous Fourier
    transform sinc^p(pi n/M) (the NFFT scaling step) or, optionally, its
    discrete Fourier transform on the grid.
  * Boxes are orthorhombic (the paper writes the cubic case).
  * The paper's own NFFT (Sec. 2.2, 2.3.2; CU-NFFT, Sec. 3.1) oversamples
    and uses a Gaussian window: the optional form here keeps only the modes
    |n_d| < K_d/2 of the M_d-point grid, K_d = 2 floor(M_d / (2 sigma_s))
    (oversampling factor sigma_s = M_d/K_d >= 1), and weights the stencil
    points floor(s) - m .. floor(s) + m + 1 (p = 2m + 2 of them, the NFFT
    library's support for cutoff m) by exp(-(s - l)^2 / b) with that
    library's Gaussian shape b = 2 sigma_s m / ((2 sigma_s - 1) pi); its
    scaling step divides by the continuous Fourier transform
    sqrt(pi b) exp(-b (pi n / M)^2).
"""
from __future__ import annotations

import math

import numpy as np

from . import ewald as _ewald


# --------------------------------------------------------------------------
# window
# --------------------------------------------------------------------------
def bspline_stencil(frac, p):
    """Cardinal B-spline weights on the p stencil points of a particle.

    ``frac`` is the fractional part of the grid coordinate s (array).  The
    stencil points are l = floor(s) - p/2 + 1 + j, j = 0..p-1, and the weight
    of point j is B_p(s - l) = M_p(frac + p - 1 - j), where M_p is the order-p
    cardinal B-spline on [0, p] built by the recursion
        M_1 = 1 on [0,1),  M_n(y) = (y M_{n-1}(y) + (n-y) M_{n-1}(y-1))/(n-1).
    Returns (w, dw) with dw the derivative of each weight with respect to s,
    M_p'(y) = M_{p-1}(y) - M_{p-1}(y-1).
    """
    frac = np.asarray(frac, np.float64)
    # vals[k] = M_n(frac + k), k = 0..n-1
    vals = [np.ones_like(frac)]
    prev = vals
    for n in range(2, p + 1):
        cur = []
        for k in range(n):
            y = frac + k
            a = prev[k] if k < n - 1 else 0.0
            b = prev[k - 1] if k >= 1 else 0.0
            cur.append((y * a + (n - y) * b) / (n - 1))
        if n == p:
            lower = prev
        prev = cur
    w = np.stack([prev[p - 1 - j] for j in range(p)], axis=-1)
    if p == 1:
        dw = np.zeros_like(w)
    else:
        def low(k):
            return lower[k] if 0 <= k < p - 1 else np.zeros_like(frac)
        dw = np.stack([low(p - 1 - j) - low(p - 2 - j) for j in range(p)], axis=-1)
    return w, dw


def gaussian_shape(p, sigma):
    """Shape b (in grid units squared) of the Gaussian window of NFFT cutoff
    m on its p = 2m + 2 stencil points, for oversampling factor sigma:
    b = 2 sigma m / ((2 sigma - 1) pi)."""
    m = p // 2 - 1
    return 2.0 * sigma * m / ((2.0 * sigma - 1.0) * math.pi)


def gaussian_stencil(frac, p, b):
    """Gaussian window weights exp(-d^2/b) on the same p stencil points as
    bspline_stencil (l = floor(s) - p/2 + 1 + j, signed distance
    d = s - l = frac + p/2 - 1 - j, -p/2 < d < p/2: for p = 2m + 2 the
    points floor(s) - m .. floor(s) + m + 1 of an NFFT of cutoff m), and
    their derivatives with respect to s, -2 d/b exp(-d^2/b)."""
    frac = np.asarray(frac, np.float64)
    d = frac[..., None] + (p // 2 - 1) - np.arange(p)
    w = np.exp(-d * d / b)
    return w, -2.0 * d / b * w


def kept_modes(M, sigma):
    """Modes kept per axis under oversampling sigma: K = 2 floor(M/(2 sigma))."""
    return 2 * int(math.floor(M / (2.0 * sigma) + 1e-9))


def window_ft(M, p, kind="continuous"):
    """Fourier coefficients c(n) of the B-spline window along one axis, for
    n in numpy FFT order (0, 1, .., M/2-1, -M/2, .., -1).

    continuous: sinc(pi n/M)^p, the Fourier transform of B_p at n/M.
    discrete:   sum_j B_p(j) exp(-2 pi i n j/M) over the integer nodes j.
    gaussian:   the Gaussian window's transform sqrt(pi b) exp(-b (pi n/M)^2)
                (pass kind=("gaussian", b)).
    """
    n = np.fft.fftfreq(M, 1.0 / M)
    if isinstance(kind, tuple) and kind[0] == "gaussian":
        b = kind[1]
        return math.sqrt(math.pi * b) * np.exp(-b * (np.pi * n / M) ** 2)
    if kind == "continuous":
        t = np.pi * n / M
        s = np.ones_like(t)
        nz = t != 0
        s[nz] = np.sin(t[nz]) / t[nz]
        return s ** p
    if kind == "discrete":
        # B_p(j) for integer j = M_p(j + p/2)
        w, _ = bspline_stencil(np.zeros(1), p)  # weights at frac = 0
        # at frac=0 the stencil points are l = -p/2+1 .. p/2 relative to s
        js = np.arange(p) - p // 2 + 1
        c = np.zeros(M)
        for j, wj in zip(js, w[0]):
            c += wj * np.cos(2 * np.pi * n * (-j) / M)
        return c
    raise ValueError(kind)


# --------------------------------------------------------------------------
# grid geometry
# --------------------------------------------------------------------------
def grid_coords(x, box, M):
    """Wrapped grid coordinates s = M * (r/L mod 1) per axis, in [0, M)."""
    x = np.asarray(x, np.float64)
    M = np.asarray(M)
    u = x / box[None, :]
    u = u - np.floor(u)
    s = u * M[None, :]
    s = np.where(s >= M[None, :], s - M[None, :], s)
    return s


def _stencil(s, M, p, gauss_b=None):
    fl = np.floor(s)
    frac = s - fl
    base = fl.astype(np.int64) - p // 2 + 1
    ws, dws, idx = [], [], []
    for d in range(3):
        if gauss_b is None:
            w, dw = bspline_stencil(frac[:, d], p)
        else:
            w, dw = gaussian_stencil(frac[:, d], p, gauss_b)
        ws.append(w)
        dws.append(dw)
        idx.append(np.mod(base[:, d][:, None] + np.arange(p)[None, :], M[d]))
    return ws, dws, idx


def spread(x, q, box, M, p, chunk=65536, gauss_b=None):
    """rho_l = sum_i q_i B_p(s_i - l), periodic (type-1 / transposed step);
    the Gaussian window instead when gauss_b is given.  Grid layout
    [Mz, My, Mx] (x fastest)."""
    M = np.asarray(M)
    rho = np.zeros(int(np.prod(M)))
    n = len(q)
    for a in range(0, n, chunk):
        sl = slice(a, min(n, a + chunk))
        qq = np.asarray(q[sl], np.float64)
        keep = qq != 0
        if not keep.any():
            continue
        s = grid_coords(x[sl][keep], box, M)
        ws, _, idx = _stencil(s, M, p, gauss_b)
        wx, wy, wz = ws
        ix, iy, iz = idx
        val = (qq[keep][:, None, None, None] * wz[:, :, None, None] *
               wy[:, None, :, None] * wx[:, None, None, :])
        lin = (iz[:, :, None, None] * M[1] + iy[:, None, :, None]) * M[0] + ix[:, None, None, :]
        rho += np.bincount(lin.ravel(), weights=val.ravel(), minlength=rho.size)
    return rho.reshape(M[2], M[1], M[0])


def interpolate(grids, x, box, M, p, deriv=False, chunk=32768, gauss_b=None):
    """Type-2 / conjugated step: for each particle and each grid g,
    sum_l B_p(s_i - l) g_l.  With deriv=True also returns the gradient of
    that sum with respect to the grid coordinate s (shape [N, ngrid, 3])."""
    M = np.asarray(M)
    flat = [np.asarray(g).reshape(-1) for g in grids]
    n = x.shape[0]
    out = np.zeros((n, len(flat)))
    dout = np.zeros((n, len(flat), 3)) if deriv else None
    for a in range(0, n, chunk):
        sl = slice(a, min(n, a + chunk))
        s = grid_coords(x[sl], box, M)
        ws, dws, idx = _stencil(s, M, p, gauss_b)
        ix, iy, iz = idx
        lin = (iz[:, :, None, None] * M[1] + iy[:, None, :, None]) * M[0] + ix[:, None, None, :]
        w3 = ws[2][:, :, None, None] * ws[1][:, None, :, None] * ws[0][:, None, None, :]
        for gi, g in enumerate(flat):
            vals = g[lin]
            out[sl, gi] = (w3 * vals).sum(axis=(1, 2, 3))
            if deriv:
                d0 = ws[2][:, :, None, None] * ws[1][:, None, :, None] * dws[0][:, None, None, :]
                d1 = ws[2][:, :, None, None] * dws[1][:, None, :, None] * ws[0][:, None, None, :]
                d2 = dws[2][:, :, None, None] * ws[1][:, None, :, None] * ws[0][:, None, None, :]
                dout[sl, gi, 0] = (d0 * vals).sum(axis=(1, 2, 3))
                dout[sl, gi, 1] = (d1 * vals).sum(axis=(1, 2, 3))
                dout[sl, gi, 2] = (d2 * vals).sum(axis=(1, 2, 3))
    return out, dout


# --------------------------------------------------------------------------
# reciprocal space
# --------------------------------------------------------------------------
def kgrid(box, M, K=None):
    """k vectors and the mode mask on the [Mz, My, Mx] FFT layout: every
    mode but the Nyquist index and n = 0, or with K (kept modes per axis)
    only |n_d| < K_d/2."""
    M = np.asarray(M)
    ns = [np.fft.fftfreq(M[d], 1.0 / M[d]) for d in range(3)]
    nz, ny, nx = np.meshgrid(ns[2], ns[1], ns[0], indexing="ij")
    kx = 2 * np.pi * nx / box[0]
    ky = 2 * np.pi * ny / box[1]
    kz = 2 * np.pi * nz / box[2]
    mask = ((nx != -M[0] // 2) & (ny != -M[1] // 2) & (nz != -M[2] // 2) &
            ~((nx == 0) & (ny == 0) & (nz == 0)))
    if K is not None:
        mask &= (2 * np.abs(nx) < K[0]) & (2 * np.abs(ny) < K[1]) & (2 * np.abs(nz) < K[2])
    return (kx, ky, kz), mask


def reciprocal(x, q, box, alpha, M, p, ke=1.0, window="continuous", want_grad=True, sigma=1.0):
    """ENUF k-space part: energy, ik forces, potentials and the exact
    gradient of the discrete energy, all in FP64.  window="gaussian": the
    paper's NFFT form with the Gaussian window of shape gaussian_shape(p,
    sigma); sigma > 1 keeps only the modes |n_d| < K_d/2 (kept_modes) of
    either window."""
    x = np.asarray(x, np.float64)
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    M = np.asarray(M)
    V = float(np.prod(box))
    gb = gaussian_shape(p, sigma) if window == "gaussian" else None
    rho = spread(x, q, box, M, p, gauss_b=gb)
    rho_hat = np.fft.fftn(rho)                       # exp(-2 pi i n.l/M), unnormalised
    kind = ("gaussian", gb) if gb is not None else window
    c = [window_ft(int(M[d]), p, kind) for d in range(3)]
    cfull = c[2][:, None, None] * c[1][None, :, None] * c[0][None, None, :]
    K = None if sigma == 1.0 else [kept_modes(int(M[d]), sigma) for d in range(3)]
    (kx, ky, kz), mask = kgrid(box, M, K)
    k2 = kx * kx + ky * ky + kz * kz
    A = np.zeros_like(k2)
    A[mask] = np.exp(-k2[mask] / (4 * alpha * alpha)) / k2[mask]
    S = rho_hat / cfull                              # S~(n), Eq. 37
    e_k = ke * (2 * np.pi / V) * float(np.sum(A * np.abs(S) ** 2))
    G = float(np.prod(M))
    fields = []
    for kd in (kx, ky, kz):
        gh = -1j * kd * A * S / cfull
        fields.append(np.real(np.fft.ifftn(gh)) * G)
    psi = np.real(np.fft.ifftn(A * S / cfull)) * G
    vals, dvals = interpolate(fields + [psi], x, box, M, p, deriv=want_grad, gauss_b=gb)
    pref = ke * 4 * np.pi / V
    f_k = pref * q[:, None] * vals[:, :3]
    phi_k = pref * vals[:, 3]
    out = {"E_K": e_k, "F_K": f_k, "phi_K": phi_k, "rho": rho, "rho_hat": rho_hat,
           "S": S, "A": A, "fields": fields, "psi": psi}
    if want_grad:
        # dU/dr_i = pref * q_i * (M_d / L_d) * sum_l dB/ds_d(s_i - l) psi_l
        out["grad_K"] = pref * q[:, None] * dvals[:, 3, :] * (M / box)[None, :]
    return out


def enuf(x, q, box, alpha, rc, M, p, ke=1.0, window="continuous", want_grad=True, sigma=1.0):
    """Full ENUF evaluation: real space from the direct oracle (minimum image),
    reciprocal space by the gridding steps above, self and background terms."""
    x = np.asarray(x, np.float64)
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    e_r, f_r, phi_r = _ewald.real_minimage(x, q, box, alpha, rc, ke)
    rec = reciprocal(x, q, box, alpha, M, p, ke, window, want_grad, sigma)
    e_s, e_b, phi_s, phi_b = _ewald.self_terms(q, box, alpha, ke)
    out = dict(rec)
    out.update({
        "E": e_r + rec["E_K"] + e_s + e_b, "E_R": e_r, "E_self": e_s, "E_bg": e_b,
        "F": f_r + rec["F_K"], "F_R": f_r,
        "phi": phi_r + rec["phi_K"] + phi_s + phi_b, "phi_R": phi_r,
    })
    if want_grad:
        out["grad_x"] = -f_r + rec["grad_K"]
    return out


def rms_rel(a, b):
    """||a - b||_2 / ||b||_2 over all components."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
