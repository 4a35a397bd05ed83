"""Pins of the oracle's steps after the image (no GPU): Gaussian resist kernel
and low-pass (Eqs. 5, 16), contours (Sec. II-D), EPE (Eqs. 6-8), the Eq. 9
channels and the lithography-consistency loss (Eqs. 15-17).

Each pin checks the oracle against something other than itself: spatial
convolution with the sampled continuous Gaussian, closed forms for cosines,
linear fields and discs, brute-force finite differences, and invariants of
closed contours.
"""
import math

import numpy as np
import pytest

import oracle as O
import oracle.post as OP
import workloads as W


# ---------------------------------------------------------------- Gaussian

def _sampled_gaussian(n, s):
    """The continuous Gaussian of std s sampled at integer offsets and
    periodised over the n x n clip (spatial-domain kernel)."""
    d = np.arange(n)
    d = np.minimum(d, n - d).astype(np.float64)
    g1 = np.zeros(n)
    for j in range(-3, 4):                       # periodic images
        g1 += np.exp(-((np.arange(n) + j * n) ** 2) / (2 * s * s))
    g1 /= math.sqrt(2 * math.pi) * s
    del d
    return g1[:, None] * g1[None, :]


@pytest.mark.parametrize("s", [2.0, 3.5])
def test_resist_blur_equals_spatial_convolution(s):
    # a band-limited image (an aerial image) blurred in the frequency domain
    # equals the direct periodic convolution with the sampled Gaussian
    spec = W.fd_clip_optics(64)
    lam, phi = O.socs_kernels(spec, 0.0, K=8)
    I = O.image(W.curvilinear_mask(64, 3), lam, phi)
    g = _sampled_gaussian(64, s)
    ref = np.zeros_like(I)
    for dy in range(64):
        for dx in range(64):
            ref += g[dy, dx] * np.roll(np.roll(I, dy, axis=0), dx, axis=1)
    got = OP.resist_image(I, s)
    assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()


def test_gaussian_filter_closed_forms():
    n = 128
    x = np.arange(n)
    for m, s in ((5, 2.0), (17, 3.0), (40, 1.5)):
        c = np.cos(2 * np.pi * m * x / n)[None, :] * np.ones((n, 1))
        want = math.exp(-2 * math.pi ** 2 * s * s * (m / n) ** 2)
        got = OP.gaussian_filter(c, s)
        expect = want * c if m <= OP.lowpass_band(n, s) else 0 * c
        assert np.abs(got - expect).max() < 1e-12
    assert np.abs(OP.gaussian_filter(np.full((n, n), 0.7), 2.0) - 0.7).max() < 1e-13      # DC gain 1
    # band: the Gaussian is below 1e-12 just beyond it, and the cut never reaches Nyquist
    for s in (0.5, 2.0, 7.0):
        h = OP.lowpass_band(n, s)
        assert h <= n // 2 - 1
        if h < n // 2 - 1:
            assert math.exp(-2 * math.pi ** 2 * s * s * ((h + 1) / n) ** 2) < 1e-12
            assert math.exp(-2 * math.pi ** 2 * s * s * ((h - 1) / n) ** 2) > 1e-13


def test_round_target_threshold():
    Zt = W.manhattan_target(128, 5)
    zr = OP.round_target(Zt, 3.0, 0.5)
    f = OP.gaussian_filter(Zt, 3.0)
    assert set(np.unique(zr)) <= {0.0, 1.0}
    assert np.array_equal(zr, (f >= np.float32(0.5)).astype(float))
    # a wide uniform region stays, isolated pixels vanish
    Z = np.zeros((128, 128))
    Z[20:80, 20:80] = 1
    Z[100, 100] = 1
    zr = OP.round_target(Z, 3.0, 0.5)
    assert zr[50, 50] == 1 and zr[100, 100] == 0 and zr[5, 5] == 0


@pytest.mark.parametrize("loss", ["l2", "l1"])
def test_blurred_gradient_matches_central_differences(loss):
    spec = W.fd_clip_optics(64).with_(K=8, focus_nm=(0.0, 30.0))
    banks = [O.socs_kernels(spec, F, K=8) for F in spec.focus_nm]
    m = W.curvilinear_mask(64, 21)
    T = W.manhattan_mask(64, 22, n_rects=4, side_min=6, side_max=20)
    s = 2.0
    L0, g, _ = OP.blurred_gradient(m, T, banks, 50.0, 0.3, s, loss=loss)
    rng = np.random.default_rng(1)
    for _ in range(6):
        y, x = (int(v) for v in rng.integers(0, 64, 2))
        h = 1e-6
        mp, mm = m.copy(), m.copy()
        mp[y, x] += h
        mm[y, x] -= h
        fd = (OP.blurred_gradient(mp, T, banks, 50.0, 0.3, s, loss=loss)[0]
              - OP.blurred_gradient(mm, T, banks, 50.0, 0.3, s, loss=loss)[0]) / (2 * h)
        assert abs(fd - g[y, x]) < 1e-6 * np.abs(g).max(), (y, x, fd, g[y, x])


def test_zero_blur_l2_is_the_plain_ilt_loss():
    spec = W.fd_clip_optics(64).with_(K=8)
    banks = [O.socs_kernels(spec, F, K=8) for F in spec.focus_nm]
    m = W.curvilinear_mask(64, 4)
    T = W.manhattan_target(64, 5)
    L0, g0, _ = OP.blurred_gradient(m, T, banks, 50.0, 0.3, 0.0)
    L1, g1, _ = O.gradient(m, T, banks, 50.0, 0.3, method="fft")
    assert abs(L0 - L1) < 1e-10 * L1 and np.abs(g0 - g1).max() < 1e-10 * np.abs(g1).max()


def test_binary_litho_loss_counts_mismatches():
    I = np.array([[0.1, 0.5], [0.3, 0.29]])
    Zr = np.array([[0.0, 0.0], [1.0, 1.0]])
    assert OP.litho_loss_binary(I, Zr, 0.3) == 2.0


# ---------------------------------------------------------------- contours

def _crossed_edges(v, level):
    b = np.asarray(v, np.float32) >= np.float32(level)
    return int((b != np.roll(b, -1, 1)).sum() + (b != np.roll(b, -1, 0)).sum())


def _loops(seg):
    nxt = seg["next"]
    seen = np.zeros(len(nxt), bool)
    loops = []
    for j in range(len(nxt)):
        if seen[j]:
            continue
        loop = []
        k = j
        while not seen[k]:
            seen[k] = True
            loop.append(k)
            k = nxt[k]
        assert k == j            # every chain closes on itself
        loops.append(loop)
    return loops


@pytest.mark.parametrize("seed", [1, 2])
def test_contour_invariants(seed):
    v = W.curvilinear_mask(96, seed).astype(np.float32)
    seg = OP.contours(v, 0.5)
    n = 96
    # one segment per crossed grid edge (each crossing ends exactly one segment)
    assert len(seg["cell"]) == _crossed_edges(v, 0.5)
    # successors form a permutation of closed loops, and each end point is
    # the successor's start point (same edge, same parameter)
    assert sorted(seg["next"].tolist()) == list(range(len(seg["next"])))
    _loops(seg)
    pts = OP.segment_points(seg, n)
    nxt = seg["next"]
    d = (pts[nxt, 0] - pts[:, 1] + n / 2) % n - n / 2
    assert np.abs(d).max() < 1e-12
    # in cells with one segment, every corner is inside (v >= level) exactly
    # when it lies on the positive side of the segment
    single = np.bincount(seg["cell"], minlength=n * n)[seg["cell"]] == 1
    checked = 0
    for j in np.nonzero(single)[0]:
        y, x = divmod(int(seg["cell"][j]), n)
        a, b = pts[j]
        dvec = b - a
        for cx, cy in ((0, 0), (1, 0), (1, 1), (0, 1)):
            w = np.array([x + cx, y + cy]) - a
            cr = dvec[0] * w[1] - dvec[1] * w[0]
            if abs(cr) < 1e-9:
                continue
            assert (cr > 0) == bool(v[(y + cy) % n, (x + cx) % n] >= np.float32(0.5))
            checked += 1
    assert checked > 100
    # shift equivariance: rolling the image shifts the cells
    seg2 = OP.contours(np.roll(np.roll(v, 5, axis=0), 7, axis=1), 0.5)
    y, x = np.divmod(seg["cell"], n)
    moved = ((y + 5) % n) * n + (x + 7) % n
    order = np.lexsort((seg["code"] >> 2, moved))
    assert np.array_equal(moved[order], seg2["cell"]) and np.array_equal(seg["code"][order], seg2["code"])
    assert np.abs(seg["u"][order] - seg2["u"]).max() < 1e-15


def test_contour_orientation_single_corner_cases():
    # one inside corner in an otherwise dark image: a diamond of 4 segments
    # around the pixel, traversed with the inside on the positive side
    v = np.zeros((64, 64), np.float32)
    v[10, 20] = 1.0
    seg = OP.contours(v, 0.5)
    assert len(seg["cell"]) == 4
    pts = OP.segment_points(seg, 64)
    for (a, b) in pts:
        d = b - a
        w = np.array([20.0, 10.0]) - a
        assert d[0] * w[1] - d[1] * w[0] > 0
    # the loop around the bright pixel is traversed once: signed area > 0
    area = sum(a[0] * b[1] - b[0] * a[1] for a, b in pts) / 2
    assert area > 0 and abs(area - 0.5) < 1e-12          # a diamond with half-diagonals 0.5


def test_contour_of_a_linear_field_is_exact():
    # linear interpolation is exact for a plane: every crossing lies on the line
    n = 64
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    v = (0.013 * xx + 0.021 * yy).astype(np.float32)
    lvl = 0.7
    seg = OP.contours(v, lvl)
    pts = OP.segment_points(seg, n).reshape(-1, 2)
    keep = (pts[:, 0] < n - 1) & (pts[:, 1] < n - 1)          # away from the periodic wrap
    val = 0.013 * pts[keep, 0] + 0.021 * pts[keep, 1]
    assert keep.sum() > 50 and np.abs(val - lvl).max() < 1e-6


def test_contour_of_a_disc():
    # a radial field: the contour is a circle of radius r0 (to the linear
    # interpolation error) and its loop encloses pi r0^2
    n, r0, c = 128, 30.0, 64.3
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    v = (r0 - np.hypot(xx - c, yy - c)).astype(np.float32)
    seg = OP.contours(v, 0.0)
    loops = _loops(seg)
    assert len(loops) == 1
    pts = OP.segment_points(seg, n)
    r = np.hypot(pts[:, 0, 0] - c, pts[:, 0, 1] - c)
    assert np.abs(r - r0).max() < 0.01
    area = sum(a[0] * b[1] - b[0] * a[1] for a, b in pts) / 2
    assert abs(area - math.pi * r0 ** 2) < 2e-3 * math.pi * r0 ** 2


def test_contour_saddle_resolution():
    # two diagonal bright corners: the cell mean decides the pairing
    v = np.zeros((64, 64), np.float32)
    v[10, 10] = v[11, 11] = 1.0
    a = OP.contours(v, 0.45)       # mean 0.5 >= 0.45: centre inside, bright corners joined
    b = OP.contours(v, 0.55)       # mean 0.5 < 0.55: two separate diamonds
    cell = 10 * 64 + 10
    ca = sorted(a["code"][a["cell"] == cell].tolist())
    cb = sorted(b["code"][b["cell"] == cell].tolist())
    assert len(ca) == 2 and len(cb) == 2 and ca != cb
    assert len(_loops(a)) == 1 and len(_loops(b)) == 2


# ---------------------------------------------------------------- EPE

def test_epe_of_a_linear_latent_image_is_the_edge_offset():
    # E = s (x - x0) (+ a term along y): the iso-line E = t sits at
    # x = x0 + t / s, so Eq. 6 at a site on the vertical target edge between
    # columns xe and xe + 1 (midpoint xe + 0.5) gives -(s (xe + 0.5 - x0) - t) / |grad E|
    n = 64
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    s, x0, t, ty = 0.05, 30.2, 0.3, 0.01
    E = s * (xx - x0) + ty * yy
    T = np.zeros((n, n))
    T[:, 10:33] = 1.0                                   # edges after columns 9 and 32
    sites = [st for st in OP.epe_sites(T) if st[2] == 0 and 2 <= st[0] <= n - 3]
    got = OP.epe(E, sites, t)
    for (y, x, d), e in zip(sites, got):
        want = -(s * (x + 0.5 - x0) + ty * y - t) / math.hypot(s, ty)
        assert abs(e - want) < 1e-12


def test_epe_sites_and_through_focus_rule():
    T = np.zeros((8, 8))
    T[2:5, 3:6] = 1.0
    sites = OP.epe_sites(T)
    assert len(sites) == 12                               # 3 x 3 square: 4 sides of 3 pairs
    assert sites == sorted(sites)
    E = [np.full((8, 8), 0.2) + 0.05 * np.arange(8)[None, :] * k for k in (1, 2, 3)]
    out = OP.epe_through_focus(E, sites, 0.3, 1, -0.5, 0.5)
    per, avg, eff = out[:, :3], out[:, 3], out[:, 4]
    assert np.allclose(avg, per.mean(axis=1))
    e0 = per[:, 1]
    assert np.allclose(eff, np.where(e0 > 0.5, e0 - 0.5, np.where(e0 < -0.5, e0 + 0.5, avg)))


# ---------------------------------------------------------------- Eq. 9 channels

def test_mask_sensitivity_matches_finite_differences():
    # dI(r)/dm(r) by brute force: perturb each pixel, read the image at the same pixel
    spec = W.fd_clip_optics(64).with_(K=6)
    lam, phi = O.socs_kernels(spec, 0.0, K=6)
    m = W.curvilinear_mask(64, 8)
    S = OP.mask_sensitivity(m, lam, phi)
    rng = np.random.default_rng(2)
    h = 1e-5
    for _ in range(12):
        y, x = (int(v) for v in rng.integers(0, 64, 2))
        mp, mm = m.copy(), m.copy()
        mp[y, x] += h
        mm[y, x] -= h
        fd = (O.image(mp, lam, phi)[y, x] - O.image(mm, lam, phi)[y, x]) / (2 * h)
        assert abs(fd - S[y, x]) < 1e-8 * np.abs(S).max()


def test_ai_channels_layout_and_normalisation():
    spec = W.fd_clip_optics(64).with_(K=6)
    lam, phi = O.socs_kernels(spec, 0.0, K=6)
    Zt = W.manhattan_target(64, 9)
    X = OP.ai_channels(Zt, lam, phi)
    assert X.shape == (64, 64, 3) and np.array_equal(X[..., 0], Zt)
    assert np.allclose(X[..., 1], O.image(Zt, lam, phi))
    Xn = OP.ai_channels(Zt, lam, phi, norm=(0, 1, 0, 0.5, -0.1, 0.1))
    assert Xn.min() >= 0 and Xn.max() <= 1
    assert np.allclose(Xn[..., 1], np.clip(X[..., 1] / 0.5, 0, 1))
