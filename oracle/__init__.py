"""FP64 CPU oracle for the SOCS aerial image, resist, loss and ILT adjoint.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or links
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_2602_15036_amd``) and does not import it.

Written from the imaging equations of the paper (Sec. III-A, Eqs. 1-5 and 17);
each function names the passage it follows.  Everything is float64 /
complex128 and deliberately plain: dense DFT matrices (``numpy`` matmuls),
``numpy.linalg.eigh`` for the eigendecomposition, and ``numpy.fft`` only where a
test has pinned it equal to the direct DFT.

Parity status.  The paper prints no image values, kernels or worked example, so
no function here is pinned to a number printed in the paper.  Each function is
pinned instead to mathematics it must satisfy (brute-force Abbe sum, closed
forms, invariants, adjoint identities, finite differences); see the tests
named in each docstring.
"""
from .optics import (band_geometry, source_points, pupil_values, tcc_dense,
                     source_pupil_factor, socs_kernels, pupil_near_ties)
from .socs import (dft_matrix, mask_spectrum, fields, image, image_at, image_window,
                   abbe_image, resist, loss_and_residual, gradient,
                   loss_value, fd_gradient, upsample_check)

__all__ = [
    "band_geometry", "source_points", "pupil_values", "tcc_dense",
    "source_pupil_factor", "socs_kernels", "pupil_near_ties",
    "dft_matrix", "mask_spectrum", "fields", "image", "image_at", "image_window", "abbe_image",
    "resist", "loss_and_residual", "gradient", "loss_value", "fd_gradient",
    "upsample_check",
]
