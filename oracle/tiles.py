"""Oracle for layouts larger than one clip: halo (ambit) tiling (FP64).

Test infrastructure only (see the package docstring).  The paper images
full layouts but does not describe how it tiles them; the reading used here
(and by the library) is:

  * the layout is an H x W array; outside it the mask is opaque (m = 0);
  * tiles are n x n windows with a halo of h pixels on every side around a
    core of c = n - 2h pixels; core (i, j) starts at (i c, j c), its window
    at (i c - h, j c - h); ceil(H / c) x ceil(W / c) tiles cover the layout;
  * each window is imaged as one periodic n x n clip (Eq. 4) and the image
    of its core (the part inside the layout) is kept;
  * the loss is the sum over layout pixels (each in exactly one core) of
    w_p (Z - T)^2, and its gradient is the exact derivative of that tiled
    loss: per tile, the adjoint with the residual restricted to the core,
    added into the layout gradient over the whole window.
"""
from __future__ import annotations

import numpy as np

from .socs import gradient, image, resist


def tile_origins(H, W, n, halo):
    """Window origins (y0, x0) of the tiles in raster order, and the core side."""
    c = n - 2 * halo
    if c <= 0:
        raise ValueError("the halo leaves no core")
    ty, tx = -(-H // c), -(-W // c)
    return [(i * c - halo, j * c - halo) for i in range(ty) for j in range(tx)], c


def window(a, y0, x0, n):
    """The n x n window of a at (y0, x0), zero outside a."""
    H, W = a.shape
    out = np.zeros((n, n))
    ya, yb = max(0, y0), min(H, y0 + n)
    xa, xb = max(0, x0), min(W, x0 + n)
    if ya < yb and xa < xb:
        out[ya - y0:yb - y0, xa - x0:xb - x0] = a[ya:yb, xa:xb]
    return out


def _core(H, W, y0, x0, halo, c):
    """(rows, cols) of the core inside the layout, in layout and in window coordinates."""
    cy, cx = y0 + halo, x0 + halo
    hh, ww = min(c, H - cy), min(c, W - cx)
    return (slice(cy, cy + hh), slice(cx, cx + ww)), (slice(halo, halo + hh), slice(halo, halo + ww))


def tiled_image(layout, lam, phi, n, halo, method="fft"):
    """Image of an H x W layout through halo tiling (one focus plane)."""
    H, W = layout.shape
    out = np.zeros((H, W))
    origins, c = tile_origins(H, W, n, halo)
    for y0, x0 in origins:
        It = image(window(layout, y0, x0, n), lam, phi, method)
        dst, src = _core(H, W, y0, x0, halo, c)
        out[dst] = It[src]
    return out


def tiled_gradient(layout, T, banks, slope, threshold, n, halo, method="fft", weights=None):
    """Tiled loss sum_p w_p sum_layout (Z_p - T)^2 (sigmoid resist) and its exact
    gradient with respect to the layout; returns (loss, grad, images per plane)."""
    H, W = layout.shape
    origins, c = tile_origins(H, W, n, halo)
    grad = np.zeros((H, W))
    images = [np.zeros((H, W)) for _ in banks]
    total = 0.0
    for y0, x0 in origins:
        win = window(layout, y0, x0, n)
        Tw = window(T, y0, x0, n)
        dst, src = _core(H, W, y0, x0, halo, c)
        core = np.zeros((n, n))
        core[src] = 1.0
        Gs = []
        for p, (lam, phi) in enumerate(banks):
            I = image(win, lam, phi, method)
            images[p][dst] = I[src]
            Z = resist(I, slope, threshold)
            d = Z - Tw
            wp = 1.0 if weights is None else weights[p]
            total += wp * float(np.sum(core * d * d))
            Gs.append(core * wp * 2.0 * d * slope * Z * (1.0 - Z))
        _, g, _ = gradient(win, None, banks, slope, threshold, method=method, G_override=Gs)
        ya, yb = max(0, y0), min(H, y0 + n)
        xa, xb = max(0, x0), min(W, x0 + n)
        grad[ya:yb, xa:xb] += g[ya - y0:yb - y0, xa - x0:xb - x0]
    return total, grad, images


def tiled_loss(layout, T, banks, slope, threshold, n, halo, method="fft", weights=None):
    """The tiled loss alone (finite-difference checks)."""
    H, W = layout.shape
    origins, c = tile_origins(H, W, n, halo)
    total = 0.0
    for y0, x0 in origins:
        win = window(layout, y0, x0, n)
        Tw = window(T, y0, x0, n)
        _, src = _core(H, W, y0, x0, halo, c)
        for p, (lam, phi) in enumerate(banks):
            d = resist(image(win, lam, phi, method), slope, threshold) - Tw
            wp = 1.0 if weights is None else weights[p]
            total += wp * float(np.sum(d[src] ** 2))
    return total
