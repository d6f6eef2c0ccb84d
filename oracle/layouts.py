"""HEALPix pixel layouts and their conversion through face coordinates
(oracle).

ORACLE -- test infrastructure.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module.  It shares no code with
the HIP path.

The paper (Sec. III-B, Fig. 3-4) orders a map in one of three layouts and
converts between any two of them through an intermediate triplet (x, y, f):
face f = 0..11 of the 12 base pixels and the coordinates 0 <= x, y < N of
the pixel inside that face, i.e. in two steps source -> (x, y, f) -> target.
The layouts:

  RING    pixels by iso-latitude ring, north to south, eastwards in a ring
          (geometry.py; (x, y, f) -> RING by nested.ring_index_of_xyf);
  NESTED  f N^2 + (bits of x and y interleaved, x in the even positions)
          (nested.py);
  FLAT    f N^2 + r N + c: each face stored as an N x N image, row r, column
          c.  The paper characterises a flat layout by a reference corner of
          the face and an orientation (counter-clockwise from the south,
          clockwise from the east, ...) without a formula.  Reading used here:
          with the face's corners S = (0, 0), E = (N-1, 0), N = (N-1, N-1),
          W = (0, N-1) in (x, y) (x + y grows northwards, x - y eastwards) and
          a chosen origin corner k, counter-clockwise means the column axis c
          runs from corner k towards the next corner counter-clockwise
          (S -> E -> N -> W, as seen from outside the sphere with north up)
          and the row axis r towards the previous one; clockwise exchanges
          the two axes.  Origin S counter-clockwise is c = x, r = y.

Layout codes: "ring", "nested", ("flat", origin, clockwise) with origin one of
"S", "E", "N", "W".

Parity status: pinned (tests/test_oracle_layouts.py: the FLAT origin corner
and column axis of every orientation against the pixel centres of the
separately pinned RING geometry, the definitional case origin S
counter-clockwise, bijection of every layout and round trips through every
pair, agreement of the two-step NESTED <-> RING with nested.py).
"""
import numpy as np

from . import geometry, nested

ORIGINS = ("S", "E", "N", "W")


def _spread(v):
    """Bits 0, 1, 2, ... of v moved to bits 0, 2, 4, ... (plain loop)."""
    v = np.asarray(v, dtype=np.int64)
    out = np.zeros_like(v)
    for k in range(31):
        out |= ((v >> k) & 1) << (2 * k)
    return out


def all_xyf(nside):
    """Every pixel as (x, y, f), enumerated face by face."""
    N = int(nside)
    f, y, x = np.meshgrid(np.arange(12), np.arange(N), np.arange(N), indexing="ij")
    return x.ravel().astype(np.int64), y.ravel().astype(np.int64), f.ravel().astype(np.int64)


def _flat_cr(N, x, y, origin, clockwise):
    """(c, r) of face coordinates (x, y) in the flat layout (origin, clockwise)."""
    k = ORIGINS.index(origin)
    if k == 0:
        c, r = x, y
    elif k == 1:
        c, r = y, N - 1 - x
    elif k == 2:
        c, r = N - 1 - x, N - 1 - y
    else:
        c, r = N - 1 - y, x
    return (r, c) if clockwise else (c, r)


def _flat_xy(N, c, r, origin, clockwise):
    """Inverse of _flat_cr."""
    if clockwise:
        c, r = r, c
    k = ORIGINS.index(origin)
    if k == 0:
        return c, r
    if k == 1:
        return N - 1 - r, c
    if k == 2:
        return N - 1 - c, N - 1 - r
    return r, N - 1 - c


def index_of_xyf(nside, layout, x, y, f):
    """Pixel index in `layout` of the pixels (x, y, f)."""
    N = int(nside)
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    f = np.asarray(f, dtype=np.int64)
    if layout == "ring":
        return nested.ring_index_of_xyf(N, x, y, f)
    if layout == "nested":
        return f * N * N + (_spread(x) | (_spread(y) << 1))
    _, origin, clockwise = layout
    c, r = _flat_cr(N, x, y, origin, clockwise)
    return f * N * N + r * N + c


def xyf_of_index(nside, layout, idx):
    """(x, y, f) of pixel indices `idx` in `layout`."""
    N = int(nside)
    idx = np.asarray(idx, dtype=np.int64)
    if layout == "ring":
        # invert the RING index of every pixel (a permutation)
        x, y, f = all_xyf(N)
        pos = np.empty(12 * N * N, dtype=np.int64)
        pos[index_of_xyf(N, "ring", x, y, f)] = np.arange(12 * N * N)
        k = pos[idx]
        return x[k], y[k], f[k]
    f = idx // (N * N)
    q = idx % (N * N)
    if layout == "nested":
        return nested._deinterleave(q), nested._deinterleave(q >> 1), f
    _, origin, clockwise = layout
    x, y = _flat_xy(N, q % N, q // N, origin, clockwise)
    return x, y, f


def convert(maps, nside, src, dst):
    """maps [..., Npix] in layout src -> the same maps in layout dst, in the
    two steps of the paper: source index -> (x, y, f) -> target index."""
    maps = np.asarray(maps)
    n = maps.shape[-1]
    x, y, f = xyf_of_index(nside, src, np.arange(n))
    out = np.empty_like(maps)
    out[..., index_of_xyf(nside, dst, x, y, f)] = maps
    return out


def all_layouts():
    out = ["ring", "nested"]
    for o in ORIGINS:
        for cw in (False, True):
            out.append(("flat", o, cw))
    return out
