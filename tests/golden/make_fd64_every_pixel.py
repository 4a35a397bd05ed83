"""Writes FP64 central finite differences of the oracle's through-focus ILT loss
at EVERY pixel of the 64 x 64 periodic clip (three focus planes -30/0/+30 nm,
x-dipole 0.3-0.9, NA 0.55, 2 nm pixels, K = 24 per plane, sigmoid resist with
slope 50 and threshold 0.3, L2 loss against a binary target).

The loss is L(m) = sum_p sum_r (Z_p(r) - T(r))^2 with Z_p the sigmoid of the
SOCS image of plane p (Eqs. 4-5, the sigmoid relaxation).  For pixel q the
difference quotient is formed pixel by pixel before the sum,

    (L(m + h e_q) - L(m - h e_q)) / 2h = sum_{p,r} (Z+ - Z-) (Z+ + Z- - 2T) / 2h,

which avoids cancelling two large sums.  Images come from oracle.image
(direct DFT); nothing else here does imaging arithmetic.

    python tests/golden/make_fd64_every_pixel.py      # about a minute
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fd64_every_pixel.npz")
N = 64
H = 1e-5
SLOPE, THR = 50.0, 0.3
MASK_SEED, TARGET_SEED = 31, 41


def inputs():
    spec = W.fd_clip_optics(N)
    m = W.as_f32_exact(W.curvilinear_mask(N, MASK_SEED))
    T = W.manhattan_mask(N, TARGET_SEED, n_rects=4, side_min=6, side_max=20)
    return spec, m, T


def main():
    spec, m, T = inputs()
    banks = [O.socs_kernels(spec, F, K=spec.K) for F in spec.focus_nm]
    fd = np.zeros((N, N))
    for y in range(N):
        for x in range(N):
            acc = 0.0
            mp = m.copy()
            mp[y, x] += H
            mm = m.copy()
            mm[y, x] -= H
            for lam, phi in banks:
                zp = O.resist(O.image(mp, lam, phi), SLOPE, THR)
                zm = O.resist(O.image(mm, lam, phi), SLOPE, THR)
                acc += float(np.sum((zp - zm) * (zp + zm - 2.0 * T)))
            fd[y, x] = acc / (2.0 * H)
        print(f"row {y} done", flush=True)
    loss, _, _ = O.gradient(m, T, banks, SLOPE, THR)
    np.savez_compressed(OUT, fd=fd, h=np.float64(H), loss=np.float64(loss),
                        seeds=np.array([MASK_SEED, TARGET_SEED]))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
