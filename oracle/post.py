"""Oracle for the steps after the image (FP64, plain numpy and Python loops).

Test infrastructure only (see the package docstring).  Each function follows
a passage of the paper:
  * resist blur and Gaussian low-pass: Eq. 5 (K_resist) and Eq. 16 (G_sigma);
  * contours: marching squares on the resist image, Sec. II-D / Eq. 5's level set;
  * edge placement error through focus: Eqs. 6-8;
  * AI input channels: Eq. 9;
  * lithography-consistency loss: Eqs. 15-17.
Where the paper is silent the functions take the readings stated in their
docstrings (they are the same readings the library documents).
"""
from __future__ import annotations

import math

import numpy as np

from .socs import fields, gradient, image, mask_spectrum


# ---------------------------------------------------------------- Gaussian kernels

def centred_freqs(n):
    """Integer DFT frequencies in FFT order, mapped to [-n/2, n/2)."""
    f = np.arange(n)
    return np.where(f < n - n // 2, f, f - n).astype(np.float64)


def gaussian_transfer(n, sigma_px, h=None):
    """DFT-domain transfer function of the isotropic Gaussian of standard
    deviation sigma_px pixels: exp(-2 pi^2 s^2 (fx^2 + fy^2) / n^2) at the
    centred integer frequencies (FFT order), zero where |fx| or |fy| > h."""
    f = centred_freqs(n)
    g1 = np.exp(-2.0 * math.pi ** 2 * sigma_px ** 2 * (f / n) ** 2)
    if h is not None:
        g1 = np.where(np.abs(f) <= h, g1, 0.0)
    return g1[:, None] * g1[None, :]


def lowpass_band(n, sigma_px):
    """Band half-width of the library's low-pass: beyond it the Gaussian is
    below 1e-12 (h = ceil(1.1832 n / s), 1.1832 = sqrt(ln(1e12) / (2 pi^2))),
    and never above n/2 - 1."""
    return int(min(n // 2 - 1, math.ceil(1.1832 * n / sigma_px)))


def gaussian_filter(img, sigma_px, threshold=None):
    """Periodic Gaussian low-pass of an n x n image (Eq. 16's G_sigma, and
    Eq. 5's K_resist on arbitrary images): the transfer function truncated to
    |fx|, |fy| <= lowpass_band(n, s).  With a threshold: the 0/1 image of
    filtered >= threshold (Eq. 16's Z_round with tau_round = threshold)."""
    n = img.shape[-1]
    G = gaussian_transfer(n, sigma_px, lowpass_band(n, sigma_px))
    out = np.real(np.fft.ifft2(np.fft.fft2(img) * G))
    if threshold is None:
        return out
    return (out >= np.float32(threshold)).astype(np.float64)


def resist_image(I, sigma_px):
    """R = I (x) K_resist (Eq. 5) for an aerial image I, K_resist the
    continuous Gaussian of standard deviation sigma_px pixels: the full
    transfer function on the centred frequencies (I is band-limited to far
    below n/2, so this is the continuous convolution sampled on the grid)."""
    if sigma_px == 0:
        return np.array(I, dtype=np.float64)
    n = I.shape[-1]
    return np.real(np.fft.ifft2(np.fft.fft2(I) * gaussian_transfer(n, sigma_px)))


def blurred_gradient(m, T, banks, slope, threshold, sigma_px, loss="l2", weights=None):
    """ILT loss and mask gradient when the resist sees R = I (x) K_resist
    (Eq. 5 with a Gaussian K_resist) and the loss is L2 or L1 (Eq. 15):
    dL/dI = K_resist (x) dL/dR (the Gaussian is symmetric), then the adjoint of
    Eq. 4 (oracle.gradient in VJP mode).  Returns (loss, grad, resist images)."""
    Gs, total, Rs = [], 0.0, []
    for p, (lam, phi) in enumerate(banks):
        I = image(m, lam, phi, method="fft")
        R = resist_image(I, sigma_px)
        Rs.append(R)
        Z = 1.0 / (1.0 + np.exp(-slope * (R - threshold)))
        d = Z - T
        wp = 1.0 if weights is None else weights[p]
        if loss == "l2":
            total += wp * float(np.sum(d * d))
            GR = wp * 2.0 * d * slope * Z * (1.0 - Z)
        else:
            total += wp * float(np.sum(np.abs(d)))
            GR = wp * np.sign(d) * slope * Z * (1.0 - Z)
        Gs.append(resist_image(GR, sigma_px))
    _, grad, _ = gradient(m, None, banks, slope, threshold, method="fft", G_override=Gs)
    return total, grad, Rs


def round_target(Zt, sigma_px, tau_round):
    """Z_round of Eq. 16: the Gaussian low-pass of the target, thresholded."""
    return gaussian_filter(Zt, sigma_px, threshold=tau_round)


def litho_loss_binary(I, Z_round, tau_print):
    """Eq. 15 with the binary print of Eq. 17: sum |1[I >= tau_print] - Z_round|."""
    return float(np.sum(np.abs((I >= tau_print).astype(np.float64) - Z_round)))


# ---------------------------------------------------------------- marching squares

def contours(v, level):
    """Marching squares on a periodic image (Sec. II-D).

    Readings: a corner is inside when v >= level (values and level compared in
    float32); on a grid edge whose ends straddle the level the crossing lies
    at the linear-interpolation parameter u = (level - a) / (b - a), measured
    from the edge's first corner (left end of a horizontal edge, top end of a
    vertical one).  In each cell the crossings are joined so that every
    segment separates one corner region from the rest; when two diagonal
    corners are inside, the cell mean decides whether the centre is inside
    (the mean is formed in float32 as 0.25 * ((c0 + c1) + (c2 + c3))).  Each
    segment is oriented with the inside on the side where
    cross(end - start, p - start) > 0 in (x = column, y = row) coordinates,
    the side being taken on the segment between the two edge midpoints (the
    same pairing, so the same side; it stays defined when a crossing falls
    on a corner because a value equals the level).
    Segments are listed by cell (raster order) and start edge; next[j] is the
    segment whose start is segment j's end.

    Edges of cell (y, x): 0 top, 1 right, 2 bottom, 3 left.  Returns a dict of
    numpy arrays: cell, code (start * 4 + end), u [S, 2], next.
    """
    v = np.asarray(v, dtype=np.float32)
    n = v.shape[0]
    L = np.float32(level)
    inside = v >= L
    # cells with mixed corners (the others have no crossing)
    c0, c1 = inside, np.roll(inside, -1, axis=1)
    c3, c2 = np.roll(inside, -1, axis=0), np.roll(np.roll(inside, -1, axis=0), -1, axis=1)
    s = c0.astype(int) + c1 + c2 + c3
    ys, xs = np.nonzero((s > 0) & (s < 4))
    corner_xy = [(0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (0.0, 1.0)]
    edge_corners = [(0, 1), (1, 2), (3, 2), (0, 3)]       # first, second corner of each edge
    edge_mid = [(0.5, 0.0), (1.0, 0.5), (0.5, 1.0), (0.0, 0.5)]
    segs = []
    for y, x in zip(ys.tolist(), xs.tolist()):
        x1, y1 = (x + 1) % n, (y + 1) % n
        c = [v[y, x], v[y, x1], v[y1, x1], v[y1, x]]
        ins = [bool(ci >= L) for ci in c]
        cross = {}
        for e, (a, b) in enumerate(edge_corners):
            if ins[a] != ins[b]:
                u = (float(L) - float(c[a])) / (float(c[b]) - float(c[a]))
                pa, pb = corner_xy[a], corner_xy[b]
                cross[e] = (u, (pa[0] + u * (pb[0] - pa[0]), pa[1] + u * (pb[1] - pa[1])))
        # pair the crossings: two crossings form one segment; four (a saddle)
        # form two, each cutting off a corner on the other side from the centre
        if len(cross) == 2:
            pairs = [tuple(sorted(cross))]
            ref_inside = [corner_xy[i] for i in range(4) if ins[i]][0]
            refs = [ref_inside]
        else:
            mean = np.float32(0.25) * ((np.float32(c[0]) + np.float32(c[1])) + (np.float32(c[2]) + np.float32(c[3])))
            centre_in = bool(mean >= L)
            cut = [i for i in range(4) if ins[i] != centre_in]   # corners separated from the centre
            pairs, refs = [], []
            for i in cut:
                es = tuple(sorted(e for e, (a, b) in enumerate(edge_corners) if i in (a, b)))
                pairs.append(es)
                # a point on the inside side of this segment
                refs.append(corner_xy[i] if ins[i] else (0.5, 0.5))
        for (ea, eb), ref in zip(pairs, refs):
            # which side is inside is a topological property of the pairing:
            # decide it on the segment between the two edge midpoints, which
            # never passes through a corner (a crossing can sit exactly on one
            # when a value equals the level)
            pa, pb = edge_mid[ea], edge_mid[eb]
            d = (pb[0] - pa[0], pb[1] - pa[1])
            w = (ref[0] - pa[0], ref[1] - pa[1])
            if d[0] * w[1] - d[1] * w[0] > 0:
                st, en = ea, eb
            else:
                st, en = eb, ea
            segs.append((y * n + x, st, en, cross[st][0], cross[en][0]))
    segs.sort(key=lambda t: (t[0], t[1]))
    index = {(cell, st): j for j, (cell, st, _, _, _) in enumerate(segs)}
    nxt = []
    for cell, st, en, _, _ in segs:
        y, x = divmod(cell, n)
        yy, xx = [(y - 1, x), (y, x + 1), (y + 1, x), (y, x - 1)][en]
        nxt.append(index[((yy % n) * n + (xx % n), en ^ 2)])
    return {"cell": np.array([t[0] for t in segs], dtype=np.int64),
            "code": np.array([t[1] * 4 + t[2] for t in segs], dtype=np.int64),
            "u": np.array([[t[3], t[4]] for t in segs], dtype=np.float64).reshape(-1, 2),
            "next": np.array(nxt, dtype=np.int64)}


def segment_points(seg, n):
    """Absolute start and end points (x, y) of contour segments, cell-local
    coordinates added to the cell corner (a wrapped edge keeps x or y = n)."""
    cell, code, u = seg["cell"], seg["code"], seg["u"]
    y, x = np.divmod(cell, n)
    out = np.zeros((len(cell), 2, 2))
    for k, e in enumerate((code >> 2, code & 3)):
        t = u[:, k]
        px = np.select([e == 0, e == 1, e == 2, e == 3], [t, 1.0 + 0 * t, t, 0 * t])
        py = np.select([e == 0, e == 1, e == 2, e == 3], [0 * t, t, 1.0 + 0 * t, t])
        out[:, k, 0] = x + px
        out[:, k, 1] = y + py
    return out


# ---------------------------------------------------------------- EPE

def epe_sites(T):
    """Target edge sites: 4-neighbour pixel pairs whose binary targets
    (T >= 0.5) differ; per pixel (y, x) in raster order, first the pair with
    (y, x+1), then with (y+1, x) (mod n).  Returns [(y, x, direction)]."""
    n = T.shape[0]
    b = T >= 0.5
    out = []
    for y in range(n):
        for x in range(n):
            if b[y, x] != b[y, (x + 1) % n]:
                out.append((y, x, 0))
            if b[y, x] != b[(y + 1) % n, x]:
                out.append((y, x, 1))
    return out


def epe(E, sites, t_eff):
    """Eq. 6 at each site: EPE = -(E_eff - E_tgt) / |grad E_eff| with E_tgt = t_eff
    on the target edge.  Reading: E_eff and its gradient at the midpoint of the
    pixel pair, E_eff = (E_p + E_q) / 2, normal derivative E_q - E_p and
    tangential derivative one quarter of the difference between the sums of
    the neighbouring pairs on either side (central differences).  Returns the
    EPE in pixels (-inf / +inf / 0 where the gradient vanishes)."""
    n = E.shape[0]
    out = []
    for y, x, d in sites:
        at = lambda yy, xx: float(E[yy % n, xx % n])
        p = at(y, x)
        if d == 0:
            q = at(y, x + 1)
            gt = 0.25 * ((at(y + 1, x) + at(y + 1, x + 1)) - (at(y - 1, x) + at(y - 1, x + 1)))
        else:
            q = at(y + 1, x)
            gt = 0.25 * ((at(y, x + 1) + at(y + 1, x + 1)) - (at(y, x - 1) + at(y + 1, x - 1)))
        e = 0.5 * (p + q) - t_eff
        g = math.hypot(q - p, gt)
        out.append(-e / g if g > 0 else (0.0 if e == 0 else (-math.inf if e > 0 else math.inf)))
    return np.array(out)


def epe_through_focus(Es, sites, t_eff, f0, tol_neg, tol_pos):
    """Eqs. 7-8: per-plane EPE, their average, and the effective EPE against
    the on-focus plane f0 (EPE_f0 - tol_pos above tol_pos, EPE_f0 - tol_neg
    below tol_neg, the average in between, boundaries included).  Returns
    [S, P + 2]."""
    per = np.stack([epe(E, sites, t_eff) for E in Es], axis=1)
    avg = per.mean(axis=1)
    e0 = per[:, f0]
    eff = np.where(e0 > tol_pos, e0 - tol_pos, np.where(e0 < tol_neg, e0 - tol_neg, avg))
    return np.concatenate([per, avg[:, None], eff[:, None]], axis=1)


# ---------------------------------------------------------------- AI channels (Eq. 9)

def mask_sensitivity(m, lam, phi):
    """dI(r)/dm(r): the derivative of the SOCS image at r with respect to the
    mask pixel at the same r, 2 sum_k lambda_k Re[conj(E_k(r)) phi_k(0)], where
    phi_k = IDFT(Phi_k) is the spatial coherent kernel (E_k = phi_k (x) m)."""
    n = m.shape[0]
    b = (phi.shape[-1] - 1) // 2
    E = fields(mask_spectrum(m, b, "fft"), phi, n, "fft")
    phi0 = phi.reshape(len(lam), -1).sum(axis=1) / (n * n)
    return 2.0 * np.einsum("k,kyx->yx", lam, np.real(np.conj(E) * phi0[:, None, None]))


def ai_channels(Zt, lam, phi, norm=None):
    """Eq. 9's input X = (M0 = Z_t, I0 = image of Z_t, dI/dM) channel last,
    each mapped by clip((v - lo) / (hi - lo), 0, 1) when norm = (lo0, hi0, ...)."""
    chans = [np.asarray(Zt, np.float64), image(Zt, lam, phi, method="fft"), mask_sensitivity(Zt, lam, phi)]
    if norm is not None:
        chans = [np.clip((c - norm[2 * i]) / (norm[2 * i + 1] - norm[2 * i]), 0.0, 1.0) for i, c in enumerate(chans)]
    return np.stack(chans, axis=-1)
