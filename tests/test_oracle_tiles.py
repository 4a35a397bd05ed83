"""Pins of the oracle's halo tiling (oracle.tiles), no GPU.

* One tile covering the whole layout is the SOCS image of the zero-padded
  layout (a plain clip, itself pinned by the imaging tests).
* A layout that repeats a base clip with the tile's period: each interior
  window is a cyclic shift of the base clip, so its core carries the base
  clip's periodic image at the same phase (exact).
* The tiled gradient is the exact derivative of the tiled loss (central
  finite differences at pixels seen by one, two and four windows).
"""
import numpy as np

import oracle as O
import oracle.tiles as OT
import workloads as W


def test_tile_origins_cover_the_layout():
    origins, c = OT.tile_origins(200, 130, 64, 10)
    assert c == 44
    assert len(origins) == 5 * 3
    assert origins[0] == (-10, -10) and origins[-1] == (4 * 44 - 10, 2 * 44 - 10)
    cover = np.zeros((200, 130), int)
    for y0, x0 in origins:
        cover[max(0, y0 + 10):y0 + 10 + c, max(0, x0 + 10):x0 + 10 + c] += 1
    assert (cover == 1).all()          # every layout pixel lies in exactly one core


def test_single_tile_is_the_padded_clip():
    spec = W.fd_clip_optics(64).with_(K=8)
    lam, phi = O.socs_kernels(spec, 0.0, K=8)
    lay = W.curvilinear_mask(40, 3)
    got = OT.tiled_image(lay, lam, phi, 64, 12)
    pad = np.zeros((64, 64))
    pad[12:52, 12:52] = lay
    want = O.image(pad, lam, phi, method="fft")[12:52, 12:52]
    assert np.abs(got - want).max() < 1e-13


def test_interior_tiles_of_a_periodic_layout_are_exact():
    # a layout repeating a base clip with the tile's period: every window
    # inside the layout is a cyclic shift of the base clip, so its core must
    # carry the base clip's periodic image at the same phase
    n, halo = 64, 8
    spec = W.fd_clip_optics(n).with_(K=8)
    lam, phi = O.socs_kernels(spec, 0.0, K=8)
    m0 = W.curvilinear_mask(n, 11)
    lay = np.tile(m0, (3, 3))
    I0 = O.image(m0, lam, phi, method="fft")
    got = OT.tiled_image(lay, lam, phi, n, halo)
    origins, c = OT.tile_origins(192, 192, n, halo)
    checked = 0
    for y0, x0 in origins:
        if y0 < 0 or x0 < 0 or y0 + n > 192 or x0 + n > 192:
            continue
        ys = np.arange(y0 + halo, y0 + halo + c)
        xs = np.arange(x0 + halo, x0 + halo + c)
        want = I0[np.ix_(ys % n, xs % n)]
        assert np.abs(got[np.ix_(ys, xs)] - want).max() < 1e-12
        checked += 1
    assert checked == 4
    # windows that reach past the layout see the opaque surround instead
    assert np.abs(got[:halo, :halo] - I0[:halo, :halo]).max() > 1e-3


def test_tiled_gradient_matches_central_differences():
    spec = W.fd_clip_optics(64).with_(K=8, focus_nm=(0.0, 30.0))
    banks = [O.socs_kernels(spec, F, K=8) for F in spec.focus_nm]
    H, Wd, n, halo = 96, 80, 64, 8                     # core 48: 2 x 2 tiles
    lay = W.curvilinear_mask(96, 7)[:H, :Wd]
    T = W.manhattan_mask(96, 8, n_rects=5, side_min=8, side_max=30)[:H, :Wd]
    L0, g, imgs = OT.tiled_gradient(lay, T, banks, 50.0, 0.3, n, halo)
    assert abs(L0 - OT.tiled_loss(lay, T, banks, 50.0, 0.3, n, halo)) < 1e-10 * L0
    for p, (lam, phi) in enumerate(banks):
        assert np.abs(imgs[p] - OT.tiled_image(lay, lam, phi, n, halo)).max() < 1e-13
    # one window (10, 10), two windows (10, 45) and (45, 10), four windows (45, 45), edge of layout
    for (y, x) in ((10, 10), (10, 45), (45, 10), (45, 45), (52, 50), (95, 79)):
        h = 1e-6
        lp, lm = lay.copy(), lay.copy()
        lp[y, x] += h
        lm[y, x] -= h
        fd = (OT.tiled_loss(lp, T, banks, 50.0, 0.3, n, halo) - OT.tiled_loss(lm, T, banks, 50.0, 0.3, n, halo)) / (2 * h)
        assert abs(fd - g[y, x]) < 1e-6 * np.abs(g).max(), (y, x, fd, g[y, x])
