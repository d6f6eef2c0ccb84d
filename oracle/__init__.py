"""FP64 CPU oracle for the HEALPix spherical harmonic transforms.

ORACLE -- TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously
correct reference written from the paper's equations.  Only tests/,
__graft_entry__.smoke() and the cpu_baseline leg of bench.py may import, call,
link or execute anything under oracle/.  It shares no code, headers, tables or
constants with the HIP path, and never imports it.

Parity status of each function (see the tests under tests/test_oracle_*.py for
the pins):
  geometry.ring_geometry      pinned (paper's grid counts; closed-form grid)
  legendre.lambda_table       pinned (closed forms l<=4, scipy, mpmath, sum rule)
  sht.map2alm / alm2map       pinned (brute-force dense sums, Nside<=8)
  sht.*_backward              pinned (adjoint identity, finite differences,
                              torch autograd of a dense model)
  sht.jacobi_map2alm          pinned (composition of pinned transforms; residual
                              decrease)
  sht.spectral_loss(_grad)    pinned (finite differences)
  sht.resize_alm              pinned (zero extension leaves the synthesis
                              unchanged, truncation commutes with the
                              analysis, round trip)
  nested.*                    pinned (Nside-1 identity with the base-pixel
                              geometry, bijection, south/east/west/north
                              sub-pixels against the RING geometry)
"""
from . import geometry, legendre, nested, sht  # noqa: F401
from ._clib import build  # noqa: F401
