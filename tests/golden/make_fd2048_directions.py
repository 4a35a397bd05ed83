"""Writes FP64 directional central finite differences of the oracle's
through-focus ILT loss for the 2048 x 2048 clip (three focus planes
-30/0/+30 nm, x-dipole 0.3-0.9, NA 0.55, 2 nm pixels, K = 24 per plane,
sigmoid resist slope 50 / threshold 0.3, L2 loss against a binary target).

Eight directions v, each supported on a 64 x 64 window and scaled to unit L2
norm: smooth random fields (seeded white noise blurred by a Gaussian of 3 px
inside the window).  Windows: the centre crop [992, 1056)^2 for the first four,
seeded random positions for the other four.  For each direction

    D_h(v) = (L(m + h v) - L(m - h v)) / 2h
           = sum_{p,r} (Z+ - Z-) (Z+ + Z- - 2T) / 2h

(the difference taken pixel by pixel before the sum), at h = 1e-3 and 2e-3;
central differences are second order, so the two agree to O(h^2) and their
Richardson combination (4 D_h - D_2h) / 3 is stored as the reference.  The
oracle's own analytic directional derivative <grad L, v> is stored beside it.
Images come from oracle.image (numpy.fft route, pinned to the direct DFT by
the oracle tests); nothing else here does imaging arithmetic.

    python tests/golden/make_fd2048_directions.py     # ~25 min, ~8 GB of RAM
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fd2048_directions.npz")
N = 2048
WIN = 64
HS = (1e-3, 2e-3)
SLOPE, THR = 50.0, 0.3
MASK_SEED, TARGET_SEED, DIR_SEED = 2000, 2001, 2048


def directions():
    """(windows [8, 2], v [8, 64, 64]): smooth unit-norm fields on 64 x 64 windows."""
    rng = np.random.default_rng(DIR_SEED)
    wins = [(992, 992)] * 4 + [tuple(int(v) for v in rng.integers(0, N - WIN, 2)) for _ in range(4)]
    k = np.fft.fftfreq(WIN)
    g = np.exp(-2.0 * (np.pi * 3.0) ** 2 * (k[:, None] ** 2 + k[None, :] ** 2))
    vs = []
    for _ in range(8):
        w = rng.standard_normal((WIN, WIN))
        v = np.real(np.fft.ifft2(np.fft.fft2(w) * g))
        vs.append(v / np.linalg.norm(v))
    return np.array(wins), np.array(vs)


def inputs():
    spec = W.CONFIG3
    m = W.as_f32_exact(W.curvilinear_mask(N, MASK_SEED))
    T = W.manhattan_target(N, TARGET_SEED)
    return spec, m, T


def main():
    spec, m, T = inputs()
    wins, vs = directions()
    banks = [O.socs_kernels(spec, F, K=spec.K) for F in spec.focus_nm]
    _, grad, _ = O.gradient(m, T, banks, SLOPE, THR, method="fft")
    analytic = np.array([float(np.sum(grad[y:y + WIN, x:x + WIN] * v)) for (y, x), v in zip(wins, vs)])
    gnorm = np.array([float(np.linalg.norm(grad[y:y + WIN, x:x + WIN])) for (y, x) in wins])
    print("analytic", analytic, flush=True)
    fd = np.zeros((len(HS), len(vs)))
    for hi, h in enumerate(HS):
        for d, ((y, x), v) in enumerate(zip(wins, vs)):
            mp = m.copy()
            mm = m.copy()
            mp[y:y + WIN, x:x + WIN] += h * v
            mm[y:y + WIN, x:x + WIN] -= h * v
            acc = 0.0
            for lam, phi in banks:
                zp = O.resist(O.image(mp, lam, phi, method="fft"), SLOPE, THR)
                zm = O.resist(O.image(mm, lam, phi, method="fft"), SLOPE, THR)
                acc += float(np.sum((zp - zm) * (zp + zm - 2.0 * T)))
            fd[hi, d] = acc / (2.0 * h)
            print(f"h={h} direction {d}: fd {fd[hi, d]:.12e} analytic {analytic[d]:.12e}", flush=True)
    rich = (4.0 * fd[0] - fd[1]) / 3.0
    np.savez_compressed(OUT, windows=wins, v=vs, h=np.array(HS), fd=fd, fd_richardson=rich,
                        analytic=analytic, window_grad_norm=gnorm,
                        seeds=np.array([MASK_SEED, TARGET_SEED, DIR_SEED]))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
