"""MI355X (gfx950) SOCS aerial-image and ILT-adjoint library.

The compute path is the HIP library ``liblitho.so`` behind the C ABI declared
in ``include/litho.h``; ``paper_2602_15036_amd.litho`` is its Python binding
(argument marshalling only).  Importing the binding fails loudly when the
library has not been built.
"""
__all__ = ["litho"]
