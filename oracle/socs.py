"""Oracle imaging: mask spectrum, SOCS image, Abbe sum, resist, loss, adjoint (FP64).

Test infrastructure only (see the package docstring).

Transforms follow one convention throughout (reading of Eq. 1, whose printed
exponent lacks the imaginary unit): the mask spectrum uses exp(-2 pi i f.r / N)
and the field synthesis exp(+2 pi i f.r / N) with a 1/N^2 factor.
"""
from __future__ import annotations

import numpy as np

from .optics import band_geometry, pupil_values, source_points


def dft_matrix(n, freqs, sign):
    """W[u, x] = exp(sign * 2 pi i * u * x / n) for u in freqs, x in [0, n)."""
    u = np.asarray(freqs, dtype=np.float64)[:, None]
    x = np.arange(n, dtype=np.float64)[None, :]
    # reduce u*x mod n in integers before the float multiply (exact phases)
    ui = np.asarray(freqs, dtype=np.int64)[:, None]
    xi = np.arange(n, dtype=np.int64)[None, :]
    r = np.mod(ui * xi, n).astype(np.float64)
    del u, x
    return np.exp(sign * 2j * np.pi * r / n)


def mask_spectrum(m, b, method="direct"):
    """Band of the thin-mask spectrum O = DFT(m) (Eq. 1's O(f), Kirchhoff reading).

    Returns Mhat[ky + b, kx + b] = sum_r m(y, x) exp(-2 pi i (ky y + kx x) / N)
    for |kx|, |ky| <= b.  method="direct" multiplies dense DFT matrices;
    method="fft" crops numpy.fft.fft2 (pinned equal to "direct" by a test).
    """
    n = m.shape[0]
    k = np.arange(-b, b + 1)
    if method == "direct":
        W = dft_matrix(n, k, -1.0)
        return W @ m @ W.T
    if method == "fft":
        F = np.fft.fft2(m)
        idx = np.mod(k, n)
        return F[np.ix_(idx, idx)]
    raise ValueError(method)


def _embed(band, n):
    """Place a centred (2b+1)^2 band into an n x n FFT-ordered array."""
    B = band.shape[-1]
    b = (B - 1) // 2
    idx = np.mod(np.arange(-b, b + 1), n)
    out = np.zeros(band.shape[:-2] + (n, n), dtype=np.complex128)
    out[..., idx[:, None], idx[None, :]] = band
    return out


def fields(mhat, phi, n, method="direct"):
    """Coherent fields of Eq. 4: E_k = IDFT(Phi_k * O) on the n x n grid.

    E_k(y, x) = n^-2 sum_f Phi_k(f) Mhat(f) exp(+2 pi i (ky y + kx x) / n).
    Returns [K, n, n] complex.
    """
    B = phi.shape[-1]
    b = (B - 1) // 2
    X = phi * mhat[None]
    if method == "direct":
        V = dft_matrix(n, np.arange(-b, b + 1), +1.0)          # [B, n]
        return np.einsum("uy,kuv,vx->kyx", V, X, V, optimize=True) / (n * n)
    if method == "fft":
        return np.fft.ifft2(_embed(X, n))
    raise ValueError(method)


def image(m, lam, phi, method="direct", dose=1.0):
    """SOCS aerial image of Eq. 4: I = D * sum_k lambda_k |E_k|^2 (real, [n, n])."""
    n = m.shape[0]
    b = (phi.shape[-1] - 1) // 2
    mhat = mask_spectrum(m, b, method)
    E = fields(mhat, phi, n, method)
    return dose * np.einsum("k,kyx->yx", lam, np.abs(E) ** 2)


def image_at(mhat, lam, phi, n, ys, xs):
    """SOCS image (Eq. 4) at the listed pixels only, by direct summation.

    For sampled parity at sizes where the full image is too costly.
    """
    b = (phi.shape[-1] - 1) // 2
    k = np.arange(-b, b + 1)
    ys = np.asarray(ys)
    xs = np.asarray(xs)
    Vy = np.exp(2j * np.pi * np.mod(np.outer(k, ys), n) / n)   # [B, P]
    Vx = np.exp(2j * np.pi * np.mod(np.outer(k, xs), n) / n)   # [B, P]
    out = np.zeros(ys.size)
    for kk in range(lam.size):
        X = phi[kk] * mhat
        E = np.einsum("up,uv,vp->p", Vy, X, Vx, optimize=True) / (n * n)
        out += lam[kk] * np.abs(E) ** 2
    return out


def image_window(mhat, lam, phi, n, y0, x0, h, w):
    """SOCS image (Eq. 4) on the window rows y0..y0+h, columns x0..x0+w.

    E_k on the window is Vy^T (Phi_k * Mhat) Vx / n^2 with the synthesis DFT
    matrices restricted to the window rows and columns.
    """
    b = (phi.shape[-1] - 1) // 2
    k = np.arange(-b, b + 1)
    Vy = dft_matrix(n, k, +1.0)[:, y0:y0 + h]
    Vx = dft_matrix(n, k, +1.0)[:, x0:x0 + w]
    out = np.zeros((h, w))
    for kk in range(lam.size):
        E = Vy.T @ (phi[kk] * mhat) @ Vx / (n * n)
        out += lam[kk] * np.abs(E) ** 2
    return out


def abbe_image(m, spec, focus_nm=0.0, dose=1.0):
    """Brute-force Abbe image: sum over source points of coherent images.

    I(r) = D sum_s S_s |IDFT_N( P(f + sigma_s) * DFT_N(m) )|^2 over the full
    n x n frequency grid (numpy.fft).  Substituting Eq. 2 into Eq. 1 gives
    this; it equals Eq. 4 when all nonzero eigenpairs are kept.
    """
    n = m.shape[0]
    _, _, R = band_geometry(spec)
    sx, sy, w = source_points(spec)
    f = np.fft.fftfreq(n, d=1.0 / n)          # integer frequencies, FFT order
    fx, fy = np.meshgrid(f, f)
    M = np.fft.fft2(m)
    out = np.zeros((n, n))
    for s in range(sx.size):
        P = pupil_values(fx + sx[s] * R, fy + sy[s] * R, R, spec.wavelength_nm,
                         spec.na, focus_nm)
        out += w[s] * np.abs(np.fft.ifft2(P * M)) ** 2
    return dose * out


def resist(I, slope, threshold):
    """Sigmoid relaxation of the threshold resist of Eqs. 5 and 17.

    Z = 1 / (1 + exp(-slope (I - threshold))), resist kernel = delta.
    """
    return 1.0 / (1.0 + np.exp(-slope * (I - threshold)))


def loss_and_residual(I, T, slope, threshold):
    """L = sum_r (Z - T)^2 and G = dL/dI = 2 (Z - T) slope Z (1 - Z)."""
    Z = resist(I, slope, threshold)
    d = Z - T
    return float(np.sum(d * d)), 2.0 * d * slope * Z * (1.0 - Z)


def loss_value(m, T, banks, slope, threshold, method="direct", weights=None):
    """Through-focus loss: sum over planes p of w_p sum_r (Z_p - T)^2.

    ``banks`` is a list of (lam, phi), one per focus plane; ``weights`` the
    plane weights w_p (default 1 each).
    """
    total = 0.0
    for p, (lam, phi) in enumerate(banks):
        I = image(m, lam, phi, method)
        L, _ = loss_and_residual(I, T, slope, threshold)
        total += (1.0 if weights is None else weights[p]) * L
    return total


def gradient(m, T, banks, slope, threshold, method="direct", G_override=None, weights=None):
    """ILT adjoint: dL/dm for the SOCS image (pixel-based ILT gradient).

    The paper names the mask gradient (Sec. III-B, Eq. 9's dI/dM channel) but
    prints no formula; differentiating Eq. 4 with E_k = IDFT(Phi_k DFT(m)) gives

        dL/dm(r) = sum_p sum_k 2 lambda_k Re[ n^-2 sum_f conj(Phi_k(f))
                   U_k(f) exp(+2 pi i f.r / n) ],   U_k = DFT(G_p * E_k),

    with G_p = dL/dI_p.  If ``G_override`` (a list of [n, n] arrays, one per
    plane) is given, it replaces the sigmoid-loss residual (vector-Jacobian
    product mode).  ``weights`` (plane weights w_p, default 1) scale each
    plane's loss and residual.  Returns (loss, grad, images).
    """
    n = m.shape[0]
    grad = np.zeros((n, n))
    total = 0.0
    images = []
    for p, (lam, phi) in enumerate(banks):
        B = phi.shape[-1]
        b = (B - 1) // 2
        mhat = mask_spectrum(m, b, method)
        E = fields(mhat, phi, n, method)
        I = np.einsum("k,kyx->yx", lam, np.abs(E) ** 2)
        images.append(I)
        if G_override is None:
            L, G = loss_and_residual(I, T, slope, threshold)
            wp = 1.0 if weights is None else weights[p]
            total += wp * L
            G = wp * G
        else:
            G = G_override[p]
        for kk in range(lam.size):
            U = mask_spectrum(G * E[kk], b, method)            # DFT(G E_k) on the band
            A = np.conj(phi[kk]) * U
            if method == "direct":
                V = dft_matrix(n, np.arange(-b, b + 1), +1.0)
                back = V.T @ A @ V / (n * n)
            else:
                back = np.fft.ifft2(_embed(A, n))
            grad += 2.0 * lam[kk] * np.real(back)
    return total, grad, images


def fd_gradient(m, T, banks, slope, threshold, pixels, h=1e-5, method="direct", weights=None):
    """Central finite differences of ``loss_value`` at the listed pixels (FP64)."""
    out = []
    for (y, x) in pixels:
        mp = m.copy()
        mp[y, x] += h
        mm = m.copy()
        mm[y, x] -= h
        out.append((loss_value(mp, T, banks, slope, threshold, method, weights)
                    - loss_value(mm, T, banks, slope, threshold, method, weights)) / (2 * h))
    return np.array(out)


def upsample_check(I, b):
    """Largest |DFT(I)| outside |f| <= 2b relative to the DC term.

    |E_k|^2 of band-limited fields is band-limited to twice the band, so this is
    zero up to rounding; the HIP path relies on it to image on a coarser grid.
    """
    n = I.shape[0]
    F = np.fft.fft2(I)
    f = np.fft.fftfreq(n, d=1.0 / n)
    outside = (np.abs(f)[:, None] > 2 * b) | (np.abs(f)[None, :] > 2 * b)
    return float(np.abs(F[outside]).max(initial=0.0) / abs(F[0, 0]))
