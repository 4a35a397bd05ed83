"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no imaging arithmetic: it only draws masks and targets from a
seeded ``numpy.random.default_rng`` and lists the optical settings of each
workload as plain numbers.  Both the FP64 oracle and the HIP path read their
inputs from here; neither side's arithmetic lives here.

The workloads stand in for the IMEC EUV layouts the paper evaluates (Sec. III,
25 layouts), which are not available: Manhattan clips are unions of random
axis-aligned rectangles, curvilinear clips are thresholded smoothed noise with a
grey edge, as for the continuous-valued masks of Sec. III-B (Eq. 9).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

__all__ = [
    "OpticsSpec",
    "manhattan_mask",
    "curvilinear_mask",
    "CONFIG1",
    "CONFIG2",
    "CONFIG3",
    "CONFIG5",
    "fd_clip_optics",
    "serve_optics",
]


@dataclass(frozen=True)
class OpticsSpec:
    """Optical settings of one workload (plain numbers, no arithmetic).

    ``source`` is ``"annular"``, ``"dipole_x"``, ``"dipole_y"`` or ``"points"``;
    ``sigma_in``/``sigma_out`` are in units of NA; lattice sources are sampled on
    a ``source_grid`` x ``source_grid`` lattice over [-1, 1]^2.  ``"points"``
    takes ``points``: a tuple of (sigma_x, sigma_y, weight) triples.
    ``focus_nm`` lists the focus planes (one bank each).
    """

    n: int
    pixel_nm: float
    wavelength_nm: float = 13.5
    na: float = 0.33
    source: str = "annular"
    sigma_in: float = 0.5
    sigma_out: float = 0.8
    source_grid: int = 15
    focus_nm: tuple = (0.0,)
    K: int = 8
    points: tuple = ()

    def with_(self, **kw) -> "OpticsSpec":
        return replace(self, **kw)


# Plain forward, 128 x 128 at 4 nm, annular 0.5-0.8, NA 0.33, K = 8.
CONFIG1 = OpticsSpec(n=128, pixel_nm=4.0, na=0.33, source="annular",
                     sigma_in=0.5, sigma_out=0.8, K=8)
# Clip scale, 1024 x 1024 at 2 nm, NA 0.55, dipole 0.3-0.9, K = 24.
CONFIG2 = OpticsSpec(n=1024, pixel_nm=2.0, na=0.55, source="dipole_x",
                     sigma_in=0.3, sigma_out=0.9, K=24)
# Through focus, 2048 x 2048, three planes -30/0/+30 nm, K = 24 per plane.
CONFIG3 = CONFIG2.with_(n=2048, focus_nm=(-30.0, 0.0, 30.0), K=24)
# Full tile, 4096 x 4096, three planes, K = 32 per plane.
CONFIG5 = CONFIG2.with_(n=4096, focus_nm=(-30.0, 0.0, 30.0), K=32)


def fd_clip_optics(n: int = 64) -> OpticsSpec:
    """The through-focus optics on a small periodic clip (finite-difference checks)."""
    return CONFIG3.with_(n=n)


def serve_optics(n: int) -> OpticsSpec:
    """Resident banks of the served stream: clip-scale optics at side ``n``, K_max = 32."""
    return CONFIG2.with_(n=n, K=32)


def manhattan_mask(n: int, seed: int, n_rects: int = 20, side_min: int = 8,
                   side_max: int = 40) -> np.ndarray:
    """Binary float64 mask: union of ``n_rects`` axis-aligned rectangles.

    Width and height are independent uniform integers in [side_min, side_max];
    the top-left corner is uniform so that the rectangle lies inside the clip.
    """
    rng = np.random.default_rng(seed)
    m = np.zeros((n, n), dtype=np.float64)
    for _ in range(n_rects):
        w, h = (int(v) for v in rng.integers(side_min, side_max + 1, size=2))
        x0 = int(rng.integers(0, n - w + 1))
        y0 = int(rng.integers(0, n - h + 1))
        m[y0:y0 + h, x0:x0 + w] = 1.0
    return m


def manhattan_target(n: int, seed: int) -> np.ndarray:
    """Binary target at the 128 x 128 clip density (20 rectangles per 128^2 area)."""
    return manhattan_mask(n, seed, n_rects=max(1, (20 * n * n) // (128 * 128)))


def _periodic_gaussian_blur(w: np.ndarray, sigma_px: float) -> np.ndarray:
    n = w.shape[0]
    f = np.fft.fftfreq(n)
    g = np.exp(-2.0 * (math.pi * sigma_px) ** 2 * (f[:, None] ** 2 + f[None, :] ** 2))
    return np.real(np.fft.ifft2(np.fft.fft2(w) * g))


def curvilinear_mask(n: int, seed: int, sigma_px: float = 3.0, fill: float = 0.4,
                     edge: float = 0.25) -> np.ndarray:
    """Grayscale curvilinear mask in [0, 1] (float64).

    A seeded white-noise field is smoothed by a periodic Gaussian of
    ``sigma_px`` pixels, thresholded at the (1 - fill) quantile and mapped
    through a clipped ramp, which leaves a 1-2 px grey edge and a fraction
    ``fill`` of pixels at or above 0.5.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n))
    ws = _periodic_gaussian_blur(w, sigma_px)
    tau = np.quantile(ws, 1.0 - fill)
    m = np.clip(0.5 + (ws - tau) / (2.0 * edge * ws.std()), 0.0, 1.0)
    return m


def as_f32_exact(a: np.ndarray) -> np.ndarray:
    """Round to float32 and widen back, so FP32 and FP64 consumers see equal values."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@dataclass
class ServeRequestSpec:
    n: int
    kind: str
    mode: int  # 0 forward, 1 forward + gradient
    K_use: int
    arrival_s: float
    seed: int


def served_stream(n_requests: int, seed: int, rate_hz: float,
                  sizes=(256, 512, 1024, 2048), k_range=(16, 32)) -> list:
    """Poisson-arrival request list: side log-uniform over ``sizes``, Manhattan or
    curvilinear 50/50, forward or forward+gradient 50/50, K_use uniform in k_range."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate_hz)) if rate_hz > 0 else 0.0
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        kind = "manhattan" if rng.random() < 0.5 else "curvilinear"
        mode = int(rng.random() < 0.5)
        k_use = int(rng.integers(k_range[0], k_range[1] + 1))
        out.append(ServeRequestSpec(n=n, kind=kind, mode=mode, K_use=k_use,
                                    arrival_s=t, seed=int(seed * 100003 + i)))
    return out


def request_mask(spec: "ServeRequestSpec") -> np.ndarray:
    if spec.kind == "manhattan":
        return manhattan_mask(spec.n, spec.seed, n_rects=max(1, (20 * spec.n * spec.n) // (128 * 128)))
    return curvilinear_mask(spec.n, spec.seed)
