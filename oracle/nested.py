"""HEALPix NESTED pixel order and its relation to RING order (oracle).

ORACLE -- test infrastructure.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module.  It shares no code with
the HIP path.

The paper (Sec. III-A) works with RING-ordered maps and benchmarks the
conversion between the two pixel orders of HEALPix (Sec. III-A and its
evaluation of the remapping).  The NESTED order itself is that of the HEALPix
definition paper the method cites (Gorski et al. 2005):

  * the sphere is divided into 12 base pixels (faces) f = 0..11: four around
    the north pole (f = 0..3), four on the equator (4..7), four around the
    south pole (8..11), numbered eastwards;
  * each face is an N x N grid of pixels with coordinates (x, y), 0 <= x, y < N;
    x + y grows towards the face's northern corner, x - y towards its eastern
    corner;
  * the NESTED index is f N^2 + (the bits of x and y interleaved, x in the
    even bit positions, y in the odd ones), so that pixels 4p .. 4p+3 at
    resolution 2N are the four parts (south, east, west, north) of pixel p at
    resolution N.

The face of a pixel fixes which ring it lies on and where in that ring.  With
the face's northern-corner ring r_f (2, 3, 4 for the north, equatorial and
south faces, in units of N) and its longitude position q_f (1, 3, 5, 7 for the
polar faces, 0, 2, 4, 6 for the equatorial ones, in units of pi/4):

  ring          i = r_f N - x - y - 1                      (1 .. 4N-1)
  in-ring slot  j = (q_f n_i + x - y + 1 + shift_i) / 2    (1-based)

where n_i is the ring's half-width in pixels per quadrant (i in the north cap,
4N - i in the south cap, N on the belt) and shift_i = (i - N) mod 2 on the
belt, 0 in the caps; j is taken modulo 4 n_i into 1 .. 4 n_i.  The RING index
is then the ring's start (geometry.ring_geometry) plus j - 1.

Parity status: pinned (tests/test_oracle_nested.py: the identity at Nside 1
with the base-pixel geometry, bijection, the south/east/west/north layout of
the four sub-pixels checked against the RING geometry, round trips).
"""
import numpy as np

from . import geometry

_RING_CORNER = np.array([2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4], dtype=np.int64)  # r_f
_LON_POS = np.array([1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7], dtype=np.int64)      # q_f


def _deinterleave(v):
    """Bits 0, 2, 4, ... of v packed into bits 0, 1, 2, ... (plain loop)."""
    out = np.zeros_like(v)
    for k in range(31):
        out |= ((v >> (2 * k)) & 1) << k
    return out


def nest_to_ring_index(nside, ipnest):
    """RING index of each NESTED pixel index in `ipnest` (int64 array)."""
    geometry.check_nside(nside)
    N = int(nside)
    p = np.asarray(ipnest, dtype=np.int64)
    f = p // (N * N)
    ipf = p % (N * N)
    x = _deinterleave(ipf)
    y = _deinterleave(ipf >> 1)
    return ring_index_of_xyf(N, x, y, f)


def ring_index_of_xyf(nside, x, y, f):
    """RING index of the pixel with face coordinates (x, y) on face f."""
    N = int(nside)
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    f = np.asarray(f, dtype=np.int64)
    i = _RING_CORNER[f] * N - x - y - 1
    npix = 12 * N * N
    north = i < N
    south = i > 3 * N
    nr = np.where(north, i, np.where(south, 4 * N - i, N))
    start = np.where(north, 2 * i * (i - 1),
                     np.where(south, npix - 2 * nr * (nr + 1), 2 * N * (N - 1) + 4 * N * (i - N)))
    shift = np.where(north | south, 0, (i - N) & 1)
    j = (_LON_POS[f] * nr + x - y + 1 + shift) // 2
    ring_len = 4 * nr
    j = np.where(j > ring_len, j - ring_len, j)
    j = np.where(j < 1, j + ring_len, j)
    return start + j - 1


def ring_to_nest_index(nside, ipring):
    """NESTED index of each RING index: the inverse permutation of
    nest_to_ring_index over all pixels."""
    N = int(nside)
    n2r = nest_to_ring_index(N, np.arange(12 * N * N, dtype=np.int64))
    r2n = np.empty_like(n2r)
    r2n[n2r] = np.arange(n2r.size, dtype=np.int64)
    return r2n[np.asarray(ipring, dtype=np.int64)]


def nest_to_ring(maps, nside):
    """Reorder maps [..., Npix] from NESTED to RING order."""
    maps = np.asarray(maps)
    out = np.empty_like(maps)
    out[..., nest_to_ring_index(nside, np.arange(maps.shape[-1]))] = maps
    return out


def ring_to_nest(maps, nside):
    """Reorder maps [..., Npix] from RING to NESTED order."""
    maps = np.asarray(maps)
    return maps[..., nest_to_ring_index(nside, np.arange(maps.shape[-1]))]
