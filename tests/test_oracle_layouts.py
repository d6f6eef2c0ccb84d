"""Pins of the oracle's layout conversions through face coordinates
(oracle/layouts.py): the FLAT orientation conventions against the RING pixel
centres of the separately pinned geometry, and bijection / round trips of
every layout (CPU)."""
import numpy as np
import pytest

from oracle import geometry, layouts, nested


def pixel_zphi(nside, layout, x, y, f):
    """z and phi of the pixels (x, y, f), looked up through their RING index."""
    theta, phi = geometry.pixel_angles(nside)
    r = layouts.index_of_xyf(nside, "ring", x, y, f)
    return np.cos(np.asarray(theta))[r], np.asarray(phi)[r]


def dphi(a, b):
    """a - b wrapped to (-pi, pi]."""
    return np.angle(np.exp(1j * (np.asarray(a) - np.asarray(b))))


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 32])
@pytest.mark.parametrize("layout", layouts.all_layouts())
def test_bijection_and_inverse(nside, layout):
    n = 12 * nside * nside
    x, y, f = layouts.all_xyf(nside)
    idx = layouts.index_of_xyf(nside, layout, x, y, f)
    assert np.array_equal(np.sort(idx), np.arange(n))
    x2, y2, f2 = layouts.xyf_of_index(nside, layout, idx)
    assert np.array_equal(x2, x) and np.array_equal(y2, y) and np.array_equal(f2, f)


def test_two_step_matches_direct_nested_ring():
    for nside in (1, 2, 4, 16):
        m = np.random.default_rng(nside).standard_normal((2, 12 * nside * nside))
        assert np.array_equal(layouts.convert(m, nside, "nested", "ring"), nested.nest_to_ring(m, nside))
        assert np.array_equal(layouts.convert(m, nside, "ring", "nested"), nested.ring_to_nest(m, nside))


@pytest.mark.parametrize("nside", [2, 8])
def test_round_trips_through_every_pair(nside):
    m = np.random.default_rng(7).standard_normal((3, 12 * nside * nside))
    ls = layouts.all_layouts()
    for a in ls:
        for b in ls:
            mb = layouts.convert(m, nside, a, b)
            assert np.array_equal(layouts.convert(mb, nside, b, a), m)
            # the same data reaches the same (x, y, f) through either route
            for c in ("ring", ("flat", "E", True)):
                assert np.array_equal(layouts.convert(mb, nside, b, c), layouts.convert(m, nside, a, c))


def test_flat_south_counterclockwise_is_row_major_xy():
    N = 8
    x, y, f = layouts.all_xyf(N)
    assert np.array_equal(layouts.index_of_xyf(N, ("flat", "S", False), x, y, f), f * N * N + y * N + x)


@pytest.mark.parametrize("nside", [2, 4, 16])
@pytest.mark.parametrize("origin", layouts.ORIGINS)
@pytest.mark.parametrize("clockwise", [False, True])
def test_flat_orientation_against_geometry(nside, origin, clockwise):
    """In the flat layout (origin, clockwise) the pixel at column 0, row 0 of
    every face is the face's corner pixel in the direction of the origin
    (southernmost, easternmost, northernmost or westernmost), and the column
    axis leads to the next corner counter-clockwise (S -> E -> N -> W) or, for
    the clockwise layouts, clockwise."""
    N = nside
    lay = ("flat", origin, clockwise)
    for face in range(12):
        idx = face * N * N + np.arange(N * N)
        x, y, f = layouts.xyf_of_index(N, lay, idx)
        z, phi = pixel_zphi(N, lay, x, y, f)
        c = idx % (N * N) % N
        r = idx % (N * N) // N
        # face centre longitude (the mean of its pixel directions)
        lon0 = np.angle(np.mean(np.exp(1j * phi)))
        east = dphi(phi, lon0)  # eastwards offset from the face centre
        # an extreme value per direction: south = lowest z, north = highest z;
        # east / west = largest / smallest longitude offset on the face's
        # middle row of rings (z closest to the face centre's z)
        def corner(direction):
            if direction == "S":
                return np.argmin(z)
            if direction == "N":
                return np.argmax(z)
            zc = np.median(z)
            mid = np.abs(z - zc) <= np.min(np.abs(z - zc)) + 1e-12
            cand = np.where(mid)[0]
            return cand[np.argmax(east[cand])] if direction == "E" else cand[np.argmin(east[cand])]
        k = layouts.ORIGINS.index(origin)
        nxt = layouts.ORIGINS[(k + 3) % 4] if clockwise else layouts.ORIGINS[(k + 1) % 4]
        first = np.where((c == 0) & (r == 0))[0][0]
        along = np.where((c == N - 1) & (r == 0))[0][0]
        want = corner(origin)
        assert first == want, (face, origin, clockwise)
        assert along == corner(nxt), (face, origin, clockwise)
