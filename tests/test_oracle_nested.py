"""Pins of the NESTED <-> RING oracle against the HEALPix grid geometry (CPU).

The NESTED order is fixed by two facts of the HEALPix definition the paper
builds on (Sec. III-A): the 12 base pixels are numbered like the RING pixels
of Nside 1 (north faces 0-3, equatorial 4-7, south 8-11, eastwards), and the
four pixels 4p .. 4p+3 at Nside 2N are the south, east, west and north parts
of pixel p at Nside N.  These tests check the oracle against those facts
using the RING-order pixel centres of the (separately pinned) geometry.
"""
import json
import os

import numpy as np
import pytest

from oracle import geometry, nested

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def unit_vectors(nside):
    theta, phi = geometry.pixel_angles(nside)
    theta = np.asarray(theta)
    phi = np.asarray(phi)
    return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], axis=-1), theta, phi


def test_nside1_is_the_base_pixel_numbering():
    # nside 1: the NESTED index of base pixel f is f, and so is its RING index
    # (12 base pixels on 3 rings of 4, eastwards from phi0)
    assert np.array_equal(nested.nest_to_ring_index(1, np.arange(12)), np.arange(12))
    with open(os.path.join(GOLDEN, "healpix_base_pixels.json")) as f:
        base = json.load(f)
    theta, phi = geometry.pixel_angles(1)
    assert np.allclose(np.cos(np.asarray(theta)), base["z"], atol=1e-15)
    assert np.allclose(np.asarray(phi) / np.pi, base["phi_over_pi"], atol=1e-15)


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 32, 128])
def test_bijection_and_round_trip(nside):
    n = 12 * nside * nside
    r = nested.nest_to_ring_index(nside, np.arange(n))
    assert np.array_equal(np.sort(r), np.arange(n))
    back = nested.ring_to_nest_index(nside, r)
    assert np.array_equal(back, np.arange(n))
    rng = np.random.default_rng(nside)
    m = rng.standard_normal((2, n))
    assert np.array_equal(nested.ring_to_nest(nested.nest_to_ring(m, nside), nside), m)
    assert np.array_equal(nested.nest_to_ring(nested.ring_to_nest(m, nside), nside), m)


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16])
def test_children_are_south_east_west_north(nside):
    # children 4p + (0, 1, 2, 3) at 2N: south, east, west, north of the parent
    N2 = 2 * nside
    _, theta, phi = unit_vectors(N2)
    z = np.cos(theta)
    parents = np.arange(12 * nside * nside)
    rc = [nested.nest_to_ring_index(N2, 4 * parents + k) for k in range(4)]
    z0, z1, z2, z3 = (z[r] for r in rc)
    assert np.all(z3 > z1) and np.all(z1 > z0)
    assert np.array_equal(z1, z2)  # east and west parts share a ring
    dphi = np.mod(phi[rc[1]] - phi[rc[2]], 2 * np.pi)
    assert np.all((dphi > 0) & (dphi < np.pi))  # the east part is east of the west part
    # and they are neighbours in their ring (RING index differs by one, cyclically)
    ring_of = np.searchsorted(np.cumsum(geometry.ring_geometry(N2)["n"]), rc[2], side="right")
    n_ring = geometry.ring_geometry(N2)["n"][ring_of]
    assert np.all(np.mod(rc[1] - rc[2], n_ring) == 1)


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16])
def test_east_west_children_symmetric_about_parent(nside):
    # the east and west parts of a pixel lie on one ring at longitudes
    # symmetric about the parent's centre, to rounding (this also fixes the
    # longitude offsets of the cap rings relative to each other)
    _, _, phi1 = unit_vectors(nside)
    _, _, phi2 = unit_vectors(2 * nside)
    parents = np.arange(12 * nside * nside)
    pphi = phi1[nested.nest_to_ring_index(nside, parents)]
    pe = phi2[nested.nest_to_ring_index(2 * nside, 4 * parents + 1)]
    pw = phi2[nested.nest_to_ring_index(2 * nside, 4 * parents + 2)]
    off = np.angle(np.exp(1j * (pe - pphi))) + np.angle(np.exp(1j * (pw - pphi)))
    assert np.max(np.abs(off)) <= 1e-14


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16])
def test_children_surround_their_parent(nside):
    # the four parts of a pixel lie within about one parent pixel of its centre
    vp, _, _ = unit_vectors(nside)
    vc, _, _ = unit_vectors(2 * nside)
    parents = np.arange(12 * nside * nside)
    pc = vp[nested.nest_to_ring_index(nside, parents)]
    size = np.sqrt(4 * np.pi / (12 * nside * nside))
    mean = np.zeros_like(pc)
    for k in range(4):
        ck = vc[nested.nest_to_ring_index(2 * nside, 4 * parents + k)]
        ang = np.arccos(np.clip(np.sum(ck * pc, axis=-1), -1, 1))
        assert np.all(ang < 1.2 * size)
        mean += ck
    mean /= np.linalg.norm(mean, axis=-1, keepdims=True)
    ang = np.arccos(np.clip(np.sum(mean * pc, axis=-1), -1, 1))
    assert np.all(ang < 0.35 * size)
