"""Writes the FP64 oracle's loss and mask gradient for the 4096 x 4096
three-plane tile (K = 32 per plane) on the central 256 x 256 window.

Inputs are the seeded workloads (curvilinear mask seed 4000, Manhattan target
seed 4001); everything else is oracle arithmetic (numpy.fft route, which the
oracle pins against its direct DFT).  The planes are independent terms of the
loss, so each is differentiated separately and the results are summed.

    python tests/golden/make_tile4096_gradient_window.py   # ~15 min, ~25 GB of RAM
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile4096_gradient_window.npz")
Y0 = X0 = 1920
H = 256
SLOPE, THR = 50.0, 0.3


def main():
    spec = W.CONFIG5
    m = W.as_f32_exact(W.curvilinear_mask(4096, 4000))
    T = W.manhattan_target(4096, 4001)
    loss = 0.0
    grad = np.zeros((H, H))
    for F in spec.focus_nm:
        lam, phi = O.socs_kernels(spec, F, K=spec.K)
        L, g, _ = O.gradient(m, T, [(lam, phi)], SLOPE, THR, method="fft")
        loss += L
        grad += g[Y0:Y0 + H, X0:X0 + H]
        print(f"plane F={F}: loss {L:.12e}", flush=True)
    np.savez_compressed(OUT, loss=np.float64(loss), grad=grad, window=np.array([Y0, X0, H]))
    print("wrote", OUT, "loss", loss)


if __name__ == "__main__":
    main()
