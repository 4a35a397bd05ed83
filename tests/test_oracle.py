"""Pins of the FP64 oracle against mathematics it must satisfy (no GPU).

The paper prints no image values, so every pin here is a brute-force
equality, a closed form, an invariant or an adjoint identity.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

ANN64 = W.CONFIG1.with_(n=64)                      # annular 0.5-0.8, NA 0.33, 4 nm
DIP64 = W.CONFIG2.with_(n=64, pixel_nm=4.0)         # dipole-x 0.3-0.9, NA 0.55


def _full_rank(spec, F=0.0):
    _, _, w = O.source_points(spec)
    return O.socs_kernels(spec, F, K=w.size, route="gram")


# ---------------------------------------------------------------- geometry

def test_band_sizes_of_the_workloads():
    # b = floor((1 + sigma_out) * NA * N * p / lambda) for each workload
    assert O.band_geometry(W.CONFIG1)[:2] == (22, 45)
    assert O.band_geometry(W.CONFIG2)[:2] == (158, 317)
    assert O.band_geometry(W.CONFIG3)[:2] == (317, 635)
    assert O.band_geometry(W.CONFIG5)[:2] == (634, 1269)


def test_source_point_counts_by_lattice_counting():
    # annular 0.5-0.8 on 15x15: integer points with 12.25 <= i^2+j^2 <= 31.36
    ann = sum(1 for i in range(-7, 8) for j in range(-7, 8) if 13 <= i * i + j * j <= 31)
    dip = sum(1 for i in range(-7, 8) for j in range(-7, 8)
              if 5 <= i * i + j * j <= 39 and abs(j) <= abs(i))
    assert O.source_points(W.CONFIG1)[0].size == ann == 60
    assert O.source_points(W.CONFIG2)[0].size == dip == 60
    _, _, w = O.source_points(W.CONFIG2)
    assert abs(w.sum() - 1.0) < 1e-15


def test_no_pupil_near_ties_in_workloads():
    for spec in (W.CONFIG1, W.CONFIG2.with_(n=256), W.fd_clip_optics(64)):
        assert O.pupil_near_ties(spec) == 0


def test_defocus_phase_is_textbook_paraxial():
    # phase(rho) - phase(0) = (2 pi / lambda) * F NA^2 rho^2 / 2 (paraxial defocus)
    R, lam_nm, na, F = 50.0, 13.5, 0.55, 30.0
    for rho in (0.0, 0.3, 0.7, 1.0):
        p = O.pupil_values(np.array([rho * R]), np.array([0.0]), R, lam_nm, na, F)[0]
        p0 = O.pupil_values(np.array([0.0]), np.array([0.0]), R, lam_nm, na, F)[0]
        want = 2 * math.pi / lam_nm * F * na * na * rho * rho / 2
        got = np.angle(p * np.conj(p0))
        assert abs(np.angle(np.exp(1j * (got - want)))) < 1e-12
        assert abs(abs(p) - 1.0) < 1e-15
    assert O.pupil_values(np.array([R * 1.0001]), np.array([0.0]), R, lam_nm, na, F)[0] == 0


# ---------------------------------------------------------------- TCC / eig

def test_tcc_hermitian_psd_and_reconstruction():
    spec = W.CONFIG1.with_(n=48)
    T = O.tcc_dense(spec, 0.0)
    assert np.abs(T - T.conj().T).max() < 1e-15
    ev = np.linalg.eigvalsh(T)
    assert ev.min() > -1e-12 * ev.max()
    lam, phi = _full_rank(spec)
    flat = phi.reshape(lam.size, -1)
    rec = (flat.T * lam) @ flat.conj()
    assert np.abs(rec - T).max() < 1e-12
    # orthonormal modes
    assert np.abs(flat.conj() @ flat.T - np.eye(lam.size)).max() < 1e-12


def test_trace_equals_pupil_lattice_count():
    # trace TCC = sum_s S_s #{band points inside the shifted pupil}, counted directly
    for spec in (ANN64, DIP64, W.CONFIG1):
        b, B, R = O.band_geometry(spec)
        sx, sy, w = O.source_points(spec)
        count = 0.0
        for s in range(sx.size):
            n_in = 0
            for ky in range(-b, b + 1):
                for kx in range(-b, b + 1):
                    if (kx + sx[s] * R) ** 2 + (ky + sy[s] * R) ** 2 <= R * R:
                        n_in += 1
            count += w[s] * n_in
        lam, _ = _full_rank(spec)
        assert abs(lam.sum() - count) < 1e-9 * count


def test_dense_and_gram_routes_agree():
    spec = W.CONFIG1.with_(n=48)
    l1, p1 = O.socs_kernels(spec, 0.0, K=8, route="dense")
    l2, p2 = O.socs_kernels(spec, 0.0, K=8, route="gram")
    assert np.abs(l1 - l2).max() < 1e-12 * l1[0]
    m = W.manhattan_mask(48, 3, n_rects=6, side_min=4, side_max=14)
    assert np.abs(O.image(m, l1, p1) - O.image(m, l2, p2)).max() < 1e-12


def test_config1_eigen_gap_at_K():
    lam, _ = O.socs_kernels(W.CONFIG1, 0.0, K=9)
    # K = 8 is cut between distinct eigenvalues, so the truncated image is unique
    assert (lam[7] - lam[8]) / lam[0] > 1e-4


# ---------------------------------------------------------------- forward image

@pytest.mark.parametrize("spec,F", [(ANN64, 0.0), (DIP64, 0.0), (DIP64, 30.0)])
def test_full_rank_socs_equals_abbe(spec, F):
    lam, phi = _full_rank(spec, F)
    for seed in range(2):
        m = W.manhattan_mask(64, seed, n_rects=8, side_min=3, side_max=16)
        I = O.image(m, lam, phi)
        Ia = O.abbe_image(m, spec, F)
        assert np.abs(I - Ia).max() < 1e-12 * Ia.max()


def test_direct_dft_equals_numpy_fft():
    lam, phi = O.socs_kernels(DIP64, 0.0, K=12)
    m = W.curvilinear_mask(64, 5)
    b = (phi.shape[-1] - 1) // 2
    assert np.abs(O.mask_spectrum(m, b, "direct") - O.mask_spectrum(m, b, "fft")).max() < 1e-11
    assert np.abs(O.image(m, lam, phi, "direct") - O.image(m, lam, phi, "fft")).max() < 1e-13


def test_image_at_matches_full_image():
    lam, phi = O.socs_kernels(ANN64, 0.0, K=8)
    m = W.manhattan_mask(64, 7, n_rects=8, side_min=3, side_max=16)
    I = O.image(m, lam, phi)
    b = (phi.shape[-1] - 1) // 2
    mh = O.mask_spectrum(m, b)
    ys = np.array([0, 5, 63, 31])
    xs = np.array([0, 60, 2, 31])
    assert np.abs(O.image_at(mh, lam, phi, 64, ys, xs) - I[ys, xs]).max() < 1e-13


def test_image_window_matches_full_image():
    lam, phi = O.socs_kernels(DIP64, 30.0, K=12)
    m = W.curvilinear_mask(64, 17)
    I = O.image(m, lam, phi)
    b = (phi.shape[-1] - 1) // 2
    mh = O.mask_spectrum(m, b)
    win = O.image_window(mh, lam, phi, 64, 10, 37, 20, 27)
    assert np.abs(win - I[10:30, 37:64]).max() < 1e-13


def test_clear_field_dark_field_and_scaling():
    lam, phi = O.socs_kernels(W.CONFIG1, 0.0, K=8)
    b = (phi.shape[-1] - 1) // 2
    clear = float(np.sum(lam * np.abs(phi[:, b, b]) ** 2))
    I1 = O.image(np.ones((128, 128)), lam, phi)
    assert np.abs(I1 - clear).max() < 1e-12
    assert np.abs(O.image(np.zeros((128, 128)), lam, phi)).max() == 0.0
    Ic = O.image(np.full((128, 128), 0.37), lam, phi)
    assert np.abs(Ic - 0.37 ** 2 * clear).max() < 1e-12
    lamf, phif = _full_rank(W.CONFIG1.with_(n=48))
    bf = (phif.shape[-1] - 1) // 2
    assert abs(float(np.sum(lamf * np.abs(phif[:, bf, bf]) ** 2)) - 1.0) < 1e-12


def test_coherent_limit_is_textbook_coherent_imaging():
    spec = ANN64.with_(sigma_in=0.0, sigma_out=0.0)
    sx, sy, w = O.source_points(spec)
    assert sx.size == 1 and sx[0] == 0 and sy[0] == 0
    lam, phi = O.socs_kernels(spec, 0.0, K=1)
    b, B, R = O.band_geometry(spec)
    n_pupil = sum(1 for i in range(-b, b + 1) for j in range(-b, b + 1) if i * i + j * j <= R * R)
    assert abs(lam[0] - n_pupil) < 1e-9
    m = W.manhattan_mask(64, 11, n_rects=8, side_min=3, side_max=16)
    f = np.fft.fftfreq(64, d=1.0 / 64)
    P = (f[:, None] ** 2 + f[None, :] ** 2 <= R * R).astype(float)
    want = np.abs(np.fft.ifft2(P * np.fft.fft2(m))) ** 2
    assert np.abs(O.image(m, lam, phi) - want).max() < 1e-12


def _grating(n, f0, axis):
    x = np.arange(n)
    line = np.cos(2 * np.pi * f0 * x / n)
    return np.tile(line, (n, 1)) if axis == "x" else np.tile(line[:, None], (1, n))


@pytest.mark.parametrize("axis", ["x", "y"])
def test_two_beam_grating_closed_form(axis):
    # m = cos(2 pi f0 x / n): with source point s, orders +-f0 pass with
    # indicators a_s, c_s and I = 1/4 sum_s S_s [a_s + c_s + 2 a_s c_s cos(4 pi f0 x / n)].
    spec = DIP64
    n = spec.n
    _, _, R = O.band_geometry(spec)
    sx, sy, w = O.source_points(spec)
    f0 = 6
    m = _grating(n, f0, axis)
    lam, phi = _full_rank(spec)
    I = O.image(m, lam, phi)
    if axis == "x":
        a = ((f0 + sx * R) ** 2 + (sy * R) ** 2 <= R * R).astype(float)
        c = ((-f0 + sx * R) ** 2 + (sy * R) ** 2 <= R * R).astype(float)
        coord = np.arange(n)[None, :]
    else:
        a = ((sx * R) ** 2 + (f0 + sy * R) ** 2 <= R * R).astype(float)
        c = ((sx * R) ** 2 + (-f0 + sy * R) ** 2 <= R * R).astype(float)
        coord = np.arange(n)[:, None]
    want = 0.25 * (np.sum(w * (a + c)) + 2 * np.sum(w * a * c) * np.cos(4 * np.pi * f0 * coord / n))
    want = np.broadcast_to(want, (n, n))
    assert np.abs(I - want).max() < 1e-12
    # the x-dipole is not x/y symmetric: the two axes modulate differently
    a_y = ((sx * R) ** 2 + (f0 + sy * R) ** 2 <= R * R).astype(float)
    c_y = ((sx * R) ** 2 + (-f0 + sy * R) ** 2 <= R * R).astype(float)
    a_x = ((f0 + sx * R) ** 2 + (sy * R) ** 2 <= R * R).astype(float)
    c_x = ((-f0 + sx * R) ** 2 + (sy * R) ** 2 <= R * R).astype(float)
    assert abs(np.sum(w * a_x * c_x) - np.sum(w * a_y * c_y)) > 0.05


def test_defocused_coherent_grating_closed_form():
    # on-axis coherent light, m = 1 + cos(t): I = 1 + cos^2 t + 2 cos t cos(Delta),
    # Delta = pi F NA^2 rho0^2 / lambda, rho0 = f0 / R (paraxial defocus).
    spec = DIP64.with_(sigma_in=0.0, sigma_out=0.0)
    F = 40.0
    n = spec.n
    _, _, R = O.band_geometry(spec)
    f0 = 9
    m = 1.0 + _grating(n, f0, "x")
    lam, phi = O.socs_kernels(spec, F, K=1)
    I = O.image(m, lam, phi)
    t = 2 * np.pi * f0 * np.arange(n) / n
    delta = math.pi * F * spec.na ** 2 * (f0 / R) ** 2 / spec.wavelength_nm
    assert abs(math.cos(delta)) < 0.9          # the defocus is visible at this pitch
    want = 1 + np.cos(t) ** 2 + 2 * np.cos(t) * math.cos(delta)
    assert np.abs(I - want[None, :]).max() < 1e-12


def test_shift_equivariance_mirror_nonnegativity():
    lam, phi = O.socs_kernels(DIP64, 30.0, K=16)
    m = W.curvilinear_mask(64, 21)
    I = O.image(m, lam, phi)
    assert I.min() >= 0.0
    Is = O.image(np.roll(m, (5, -9), axis=(0, 1)), lam, phi)
    assert np.abs(Is - np.roll(I, (5, -9), axis=(0, 1))).max() < 1e-12
    # x-mirror (x -> -x mod n); the dipole-x source is x-symmetric
    mir = lambda a: np.roll(a[:, ::-1], 1, axis=1)
    assert np.abs(O.image(mir(m), lam, phi) - mir(I)).max() < 1e-12
    # y-mirror too
    miry = lambda a: np.roll(a[::-1, :], 1, axis=0)
    assert np.abs(O.image(miry(m), lam, phi) - miry(I)).max() < 1e-12


def test_plus_minus_focus_symmetry():
    m = W.curvilinear_mask(64, 8)
    lp, pp = O.socs_kernels(DIP64, 30.0, K=20)
    lm, pm = O.socs_kernels(DIP64, -30.0, K=20)
    assert np.abs(lp - lm).max() < 1e-12 * lp[0]
    assert np.abs(O.image(m, lp, pp) - O.image(m, lm, pm)).max() < 1e-11
    l0, p0 = O.socs_kernels(DIP64, 0.0, K=20)
    assert np.abs(O.image(m, l0, p0) - O.image(m, lp, pp)).max() > 1e-3


def test_parseval():
    lam, phi = O.socs_kernels(ANN64, 0.0, K=8)
    m = W.curvilinear_mask(64, 4)
    n = 64
    b = (phi.shape[-1] - 1) // 2
    mh = O.mask_spectrum(m, b)
    I = O.image(m, lam, phi)
    rhs = np.sum(lam[:, None, None] * np.abs(phi * mh[None]) ** 2) / n ** 2
    assert abs(I.sum() - rhs) < 1e-12 * rhs


def test_image_is_band_limited_to_twice_the_band():
    spec = W.CONFIG2.with_(n=128)            # b = 19, so 2b < n / 2
    lam, phi = O.socs_kernels(spec, 0.0, K=24)
    m = W.curvilinear_mask(128, 9)
    b = (phi.shape[-1] - 1) // 2
    assert O.upsample_check(O.image(m, lam, phi), b) < 1e-14
    assert O.upsample_check(m, b) > 1e-3      # a mask is not band-limited


# ---------------------------------------------------------------- resist / adjoint

def test_resist_and_residual_closed_forms():
    I = np.array([0.3, 0.0, 1.0, 0.31])
    Z = O.resist(I, 50.0, 0.3)
    assert Z[0] == 0.5
    assert abs(Z[3] - 1 / (1 + math.exp(-0.5))) < 1e-15
    T = np.array([1.0, 0.0, 1.0, 0.0])
    L, G = O.loss_and_residual(I, T, 50.0, 0.3)
    assert abs(L - np.sum((Z - T) ** 2)) < 1e-15
    h = 1e-6
    for i in range(4):
        Ip = I.copy(); Ip[i] += h
        Im = I.copy(); Im[i] -= h
        fd = (O.loss_and_residual(Ip, T, 50.0, 0.3)[0] - O.loss_and_residual(Im, T, 50.0, 0.3)[0]) / (2 * h)
        assert abs(fd - G[i]) < 1e-6 * max(1.0, abs(G[i]))


def test_adjoint_dot_product_identity():
    # <w, J v> = <J^T w, v> for J = dI/dm, through the VJP mode of the gradient
    spec = W.fd_clip_optics(32)
    banks = [O.socs_kernels(spec, F, K=10) for F in spec.focus_nm]
    rng = np.random.default_rng(0)
    m = W.curvilinear_mask(32, 3)
    v = rng.standard_normal((32, 32))
    wts = [rng.standard_normal((32, 32)) for _ in banks]
    _, JTw, _ = O.gradient(m, None, banks, 50.0, 0.3, G_override=wts)
    h = 1e-6
    lhs = 0.0
    for (lam, phi), wp in zip(banks, wts):
        Jv = (O.image(m + h * v, lam, phi) - O.image(m - h * v, lam, phi)) / (2 * h)
        lhs += np.sum(wp * Jv)
    assert abs(lhs - np.sum(JTw * v)) < 1e-7 * abs(lhs)


@pytest.mark.parametrize("method", ["direct", "fft"])
def test_gradient_matches_central_finite_differences(method):
    spec = W.fd_clip_optics(32)
    banks = [O.socs_kernels(spec, F, K=12) for F in spec.focus_nm]
    m = W.curvilinear_mask(32, 1)
    T = W.manhattan_mask(32, 2, n_rects=3, side_min=4, side_max=10)
    L, g, _ = O.gradient(m, T, banks, 50.0, 0.3, method=method)
    rng = np.random.default_rng(5)
    pix = [tuple(int(v) for v in rng.integers(0, 32, 2)) for _ in range(12)]
    fd = O.fd_gradient(m, T, banks, 50.0, 0.3, pix, h=1e-5, method=method)
    got = np.array([g[p] for p in pix])
    assert np.abs(got - fd).max() < 1e-7 * np.abs(fd).max()
    assert abs(L - O.loss_value(m, T, banks, 50.0, 0.3, method)) < 1e-12 * L


# ---------------------------------------------------------------- source kinds, plane weights

def test_y_dipole_is_the_transposed_x_dipole():
    # the y-dipole keeps |i| <= |j|: the x-dipole mirrored about the diagonal,
    # so imaging the transposed mask gives the transposed image
    sx, sy, _ = O.source_points(DIP64)
    tx, ty, _ = O.source_points(DIP64.with_(source="dipole_y"))
    assert sorted(zip(sy.tolist(), sx.tolist())) == sorted(zip(tx.tolist(), ty.tolist()))
    lx, px = O.socs_kernels(DIP64, 0.0, K=60)
    ly, py = O.socs_kernels(DIP64.with_(source="dipole_y"), 0.0, K=60)
    assert np.allclose(lx, ly, rtol=0, atol=1e-13 * lx[0])
    m = W.manhattan_mask(64, 4, n_rects=6, side_min=3, side_max=20)
    Ix = O.image(m, lx, px)
    Iy = O.image(np.ascontiguousarray(m.T), ly, py)
    assert np.abs(Iy - Ix.T).max() < 1e-12 * Ix.max()
    # and the x-dipole image is not itself transpose-symmetric (the test has teeth)
    assert np.abs(O.image(np.ascontiguousarray(m.T), lx, px) - Ix.T).max() > 1e-3 * Ix.max()


def test_point_list_source_reproduces_the_lattice_source():
    # the annular lattice written out as explicit points (unnormalised weights)
    sx, sy, w = O.source_points(ANN64)
    pts = tuple((float(a), float(b), 3.0) for a, b in zip(sx, sy))
    spec = ANN64.with_(source="points", points=pts)
    assert O.band_geometry(spec) == O.band_geometry(ANN64)
    px, py, pw = O.source_points(spec)
    assert np.array_equal(px, sx) and np.array_equal(py, sy) and np.allclose(pw, w, rtol=0, atol=1e-16)
    la, pa = O.socs_kernels(ANN64, 0.0, K=8)
    lp, pp = O.socs_kernels(spec, 0.0, K=8)
    m = W.curvilinear_mask(64, 9)
    assert np.abs(O.image(m, lp, pp) - O.image(m, la, pa)).max() < 1e-13


def test_plane_weighted_gradient_matches_central_finite_differences():
    spec = W.fd_clip_optics(32)
    banks = [O.socs_kernels(spec, F, K=10) for F in spec.focus_nm]
    m = W.curvilinear_mask(32, 3)
    T = W.manhattan_mask(32, 4, n_rects=3, side_min=4, side_max=10)
    wts = [0.25, 1.0, 2.5]
    L, g, _ = O.gradient(m, T, banks, 50.0, 0.3, weights=wts)
    parts = [O.gradient(m, T, [bk], 50.0, 0.3) for bk in banks]
    assert abs(L - sum(w * p[0] for w, p in zip(wts, parts))) < 1e-12 * L
    rng = np.random.default_rng(8)
    pix = [tuple(int(v) for v in rng.integers(0, 32, 2)) for _ in range(10)]
    fd = O.fd_gradient(m, T, banks, 50.0, 0.3, pix, h=1e-5, weights=wts)
    got = np.array([g[p] for p in pix])
    assert np.abs(got - fd).max() < 1e-7 * np.abs(fd).max()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_gradient_matches_stored_fd_at_every_pixel_64():
    # the adjoint formula against FP64 central differences of the loss at all
    # 4096 pixels of the 64 x 64 three-plane clip (tests/golden/make_fd64_every_pixel.py)
    sys.path.insert(0, GOLDEN)
    import make_fd64_every_pixel as M
    gold = np.load(os.path.join(GOLDEN, "fd64_every_pixel.npz"))
    spec, m, T = M.inputs()
    banks = [O.socs_kernels(spec, F, K=spec.K) for F in spec.focus_nm]
    Lo, g, _ = O.gradient(m, T, banks, 50.0, 0.3)
    fd = gold["fd"]
    assert abs(Lo - float(gold["loss"])) < 1e-12 * Lo
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-7
    assert np.abs(g - fd).max() < 1e-7 * np.abs(fd).max()


def test_stored_directional_fd_2048_is_consistent():
    # the stored 2048 x 2048 directional differences: second-order agreement of
    # the two step sizes, and the oracle's analytic <grad, v> within 1e-7
    gold = np.load(os.path.join(GOLDEN, "fd2048_directions.npz"))
    fd, rich, an = gold["fd"], gold["fd_richardson"], gold["analytic"]
    assert fd.shape == (2, 8) and gold["v"].shape == (8, 64, 64)
    assert np.allclose(np.linalg.norm(gold["v"].reshape(8, -1), axis=1), 1.0)
    assert np.all(np.abs(fd[0] - fd[1]) < 1e-5 * np.abs(fd[0]))
    assert np.all(np.abs(rich - an) < 1e-7 * np.abs(an))
