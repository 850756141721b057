"""MI355X (gfx950) matrix-free Stokes hot path of arXiv:1604.07994.

The HIP library (csrc/, built into libiss.so) implements the decoupled
Laplacian-plus-interface stencil apply, the strain and gradient forms, the
divergence/gradient and stabilisation couplings, residuals, Uzawa
multicolour smoothing, P1 transfers, the direct coarse solve, V-cycles and
Richardson / FGMRES solves, in FP64 and FP32.  ``binding`` is the ctypes
layer over the C ABI in include/iss.h.
"""
from .binding import FORMS, IssError, Problem, lib  # noqa: F401
