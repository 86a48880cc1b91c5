"""CPU FP64 oracle for convolutional gridding / degridding.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct reference that the GPU library is checked against.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import it.  It
shares no code with the GPU library (no kernels, headers, helpers, tables or
constant generators) and it never imports that library.

Layout
  conventions  per-channel scale constants, support rule, table geometry
  pswf         prolate spheroidal taper psi_0(c, eta) by Nystrom
  cfbuild      convolution-function table: screen -> oversampled DFT -> crop
  native       ctypes binding of gridding.c (map, grid, degrid, psf, sumwt)
  imaging      image-plane helpers used by the pins: gcf, direct DFT,
               chi^2 and its gradient
  hogbom       Hogbom minor cycle
  calibration  diagonal G-Jones solve: ratio averages, update direction,
               damped update, exit test
  mosaic       change of phase centre per field and virtual antennas for
               the field-shifted kernels

Parity status: every function is pinned by a CPU test against something
other than itself (closed forms, brute force, library routines, invariants);
see tests/test_oracle_*.py.
"""

from .conventions import (  # noqa: F401
    C_LIGHT, half_widths, channel_constants, screen_size, plane_offsets,
)
from .pswf import pswf0, pswf_nystrom  # noqa: F401
from .cfbuild import OracleCF, build_cf  # noqa: F401
from . import native  # noqa: F401
