"""MI355X (gfx950) library for the sharp front-tracking coupling restricted to
interfacial cells (arXiv 2505.06932, section 3): exact polyhedral volume
fractions, PPIC curvature by the volume fit, CSF on interfacial cells and
divergence-preserving vertex-velocity interpolation.

Submodules: ``ftc`` (ctypes binding of include/ftc.h), ``pipeline`` (one
coupling step), ``inputs`` (seeded synthetic fronts and fields), ``build``
(hipcc build of libftc.so).  Importing this package loads nothing; ``ftc``
loads torch and the library on first use.
"""
