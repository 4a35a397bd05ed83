"""Oracle optics: source, pupil, TCC and its eigendecomposition (FP64).

Test infrastructure only (see the package docstring).

Conventions (readings where the paper is silent):
  * A clip of N x N pixels of size p is one period; spatial frequencies are
    integers m (cycles per clip), i.e. f = m / (N p).
  * The pupil radius in those index units is R = NA * N * p / lambda.
  * Source points sigma are in units of NA (sigma = sin(theta) / NA), so the
    frequency shift of Eq. 2's P(f + sigma) is sigma * R index units.
  * The band box keeps |m_x|, |m_y| <= b with b = floor((1 + sigma_out) R):
    every P(f + sigma_s) vanishes outside it.
"""
from __future__ import annotations

import math

import numpy as np


def _sigma_max(spec):
    """Largest source radius: sigma_out for lattice sources, max |sigma| for points."""
    if spec.source == "points":
        return max(math.hypot(sx, sy) for sx, sy, _ in spec.points)
    return spec.sigma_out


def band_geometry(spec):
    """Return (b, B, R): band half-width, band side 2b+1, pupil radius (index units)."""
    R = spec.na * spec.n * spec.pixel_nm / spec.wavelength_nm
    b = int(math.floor((1.0 + _sigma_max(spec)) * R))
    return b, 2 * b + 1, R


def source_points(spec):
    """Sampled, normalised source S(sigma) of Eq. 2 (Sec. III-A).

    The source is sampled on a G x G lattice with integer coordinates
    i, j in [-h, h], h = (G - 1) / 2, i.e. sigma = (i, j) / h.  A point is kept
    when sigma_in^2 h^2 <= i^2 + j^2 <= sigma_out^2 h^2 (annular) and, for the
    x-dipole, also |j| <= |i| (45 degree half-opening, diagonals included).
    All kept points weigh the same and the weights sum to one (the paper calls
    S the normalised source intensity).

    The y-dipole keeps |i| <= |j| instead.  A "points" source lists its own
    (sigma_x, sigma_y, weight) samples; the weights are normalised to sum one.

    Returns (sx, sy, w) as float64 arrays.
    """
    if spec.source == "points":
        pts = np.asarray(spec.points, dtype=np.float64).reshape(-1, 3)
        return pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2] / pts[:, 2].sum()
    G = spec.source_grid
    h = (G - 1) // 2
    lo = spec.sigma_in ** 2 * h * h
    hi = spec.sigma_out ** 2 * h * h
    keep = []
    for j in range(-h, h + 1):
        for i in range(-h, h + 1):
            r2 = i * i + j * j
            ok = (lo - 1e-9) <= r2 <= (hi + 1e-9)
            if spec.source == "dipole_x":
                ok = ok and abs(j) <= abs(i)
            elif spec.source == "dipole_y":
                ok = ok and abs(i) <= abs(j)
            elif spec.source != "annular":
                raise ValueError(f"unknown source kind {spec.source!r}")
            if ok:
                keep.append((i / h, j / h))
    sx = np.array([p[0] for p in keep], dtype=np.float64)
    sy = np.array([p[1] for p in keep], dtype=np.float64)
    w = np.full(len(keep), 1.0 / len(keep))
    return sx, sy, w


def pupil_values(u, v, R, wavelength_nm, na, focus_nm):
    """Pupil P of Eq. 2 at index-unit frequencies (u, v) (Sec. III-A).

    P = 1[u^2 + v^2 <= R^2] * exp(i * 2 pi / lambda * W), with the defocus
    aberration written as the Zernike term W = (F NA^2 / 4) (2 rho^2 - 1),
    rho^2 = (u^2 + v^2) / R^2 (paraxial defocus; +F gives +phase).
    """
    d2 = u * u + v * v
    inside = d2 <= R * R
    rho2 = d2 / (R * R)
    coeff = focus_nm * na * na / 4.0
    phase = (2.0 * math.pi / wavelength_nm) * coeff * (2.0 * rho2 - 1.0)
    return np.where(inside, np.exp(1j * phase), 0.0 + 0.0j)


def pupil_near_ties(spec, rel=1e-9):
    """Count band samples whose pupil membership is decided within rel * R^2."""
    b, B, R = band_geometry(spec)
    sx, sy, _ = source_points(spec)
    k = np.arange(-b, b + 1, dtype=np.float64)
    kx, ky = np.meshgrid(k, k)
    n = 0
    for s in range(sx.size):
        u = kx + sx[s] * R
        v = ky + sy[s] * R
        n += int(np.count_nonzero(np.abs(u * u + v * v - R * R) < rel * R * R))
    return n


def _band_coords(b):
    k = np.arange(-b, b + 1, dtype=np.float64)
    kx, ky = np.meshgrid(k, k)          # [ky, kx], centred raster order
    return kx.ravel(), ky.ravel()


def source_pupil_factor(spec, focus_nm):
    """A[f, s] = sqrt(S_s) P(f + sigma_s; F) over the band box (Eq. 2 factored).

    Rows f run over the (2b+1)^2 band samples in centred raster order
    (ky major, kx minor); columns s over the source points.
    """
    b, B, R = band_geometry(spec)
    sx, sy, w = source_points(spec)
    kx, ky = _band_coords(b)
    A = np.empty((kx.size, sx.size), dtype=np.complex128)
    for s in range(sx.size):
        A[:, s] = math.sqrt(w[s]) * pupil_values(kx + sx[s] * R, ky + sy[s] * R, R,
                                                 spec.wavelength_nm, spec.na, focus_nm)
    return A


def tcc_dense(spec, focus_nm):
    """Dense TCC of Eq. 2 over the band box, as the plain source sum.

    TCC(f1, f2) = sum_s S_s P(f1 + sigma_s) conj(P(f2 + sigma_s)).
    Only for small bands (the matrix has (2b+1)^4 entries).
    """
    b, B, R = band_geometry(spec)
    sx, sy, w = source_points(spec)
    kx, ky = _band_coords(b)
    T = np.zeros((kx.size, kx.size), dtype=np.complex128)
    for s in range(sx.size):
        p = pupil_values(kx + sx[s] * R, ky + sy[s] * R, R,
                         spec.wavelength_nm, spec.na, focus_nm)
        T += w[s] * np.outer(p, np.conj(p))
    return T


def _fix_phase(phi):
    """Cosmetic: make the largest-magnitude entry (first in raster order) real positive."""
    a = np.abs(phi)
    idx = int(np.flatnonzero(a >= a.max() * (1.0 - 1e-9))[0])
    return phi * (np.conj(phi[idx]) / a[idx])


def socs_kernels(spec, focus_nm=0.0, K=None, route="auto"):
    """SOCS kernels {lambda_k, Phi_k} of Eq. 3 (Sec. III-A), FP64.

    The TCC is Hermitian positive semi-definite, so its eigendecomposition
    (numpy.linalg.eigh) gives real lambda_k >= 0 and orthonormal Phi_k.

    route="dense": eigh of the dense TCC (small bands only).
    route="gram":  eigh of the source-space Gram matrix A^H A, then
                   Phi_k = A nu_k / sqrt(lambda_k); same nonzero eigenpairs
                   since TCC = A A^H.
    Eigenvalues are sorted descending and the first K kept; each Phi_k has
    unit 2-norm over the band samples.  Returns (lam [K], phi [K, B, B]) with
    phi indexed [ky + b, kx + b].
    """
    b, B, R = band_geometry(spec)
    if K is None:
        K = spec.K
    if route == "auto":
        route = "dense" if B * B <= 2500 else "gram"
    if route == "dense":
        T = tcc_dense(spec, focus_nm)
        lam, vec = np.linalg.eigh(T)
        order = np.argsort(lam)[::-1][:K]
        lam = lam[order]
        phi = vec[:, order].T
    elif route == "gram":
        A = source_pupil_factor(spec, focus_nm)
        gram = A.conj().T @ A
        lam, nu = np.linalg.eigh(gram)
        order = np.argsort(lam)[::-1][:K]
        lam = lam[order]
        if np.any(lam <= 0):
            raise ValueError("K exceeds the TCC rank")
        phi = (A @ nu[:, order] / np.sqrt(lam)).T
    else:
        raise ValueError(route)
    phi = np.array([_fix_phase(p) for p in phi])
    return lam.real.copy(), phi.reshape(len(lam), B, B)
