"""Pins for the oracle's HEALPix RING geometry (oracle/geometry.py)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import geometry


def test_grid_counts_from_paper(golden_dir):
    """Npix, Nrings and the ring sizes the paper states (Sec. III-A)."""
    with open(os.path.join(golden_dir, "healpix_grid.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        N = c["nside"]
        g = geometry.ring_geometry(N)
        assert geometry.npix(N) == c["npix"]
        assert int(g["n"].sum()) == c["npix"]
        assert len(g["n"]) == c["nrings"] == geometry.nrings(N)
        assert g["n"][0] == g["n"][-1] == c["polar_ring_pixels"]
        assert g["n"][2 * N - 1] == c["equatorial_ring_pixels"]  # equator
        assert g["n"].max() == c["equatorial_ring_pixels"]


def test_base_resolution_pixel_centres(golden_dir):
    with open(os.path.join(golden_dir, "healpix_base_pixels.json")) as f:
        ref = json.load(f)
    theta, phi = geometry.pixel_angles(ref["nside"])
    np.testing.assert_allclose(np.cos(theta), ref["z"], atol=1e-15)
    np.testing.assert_allclose(phi / np.pi, ref["phi_over_pi"], atol=1e-15)


def _frac(s):
    return float(Fraction(s))


def test_pixel_centres_nside2(golden_dir):
    """Every pixel centre at nside 2 against the hand-written fixture: the
    polar-cap rings carry the cap offset pi/(4i), the belt rings alternate
    pi/(4N) and 0 (Sec. III-A and the grid definition it cites)."""
    with open(os.path.join(golden_dir, "healpix_pixel_centres_nside2_4.json")) as f:
        ref = json.load(f)["nside2_pixels"]
    theta, phi = geometry.pixel_angles(2)
    np.testing.assert_allclose(np.cos(theta), [_frac(v) for v in ref["z"]], atol=2e-16)
    np.testing.assert_allclose(np.asarray(phi) / np.pi, [_frac(v) for v in ref["phi_over_pi"]], atol=1e-15)


def test_ring_first_centres_nside4(golden_dir):
    """nside 4: length, z and first-pixel longitude of every ring (three cap
    rings on each side), and the even spacing within each ring."""
    with open(os.path.join(golden_dir, "healpix_pixel_centres_nside2_4.json")) as f:
        rings = json.load(f)["nside4_rings"]
    g = geometry.ring_geometry(4)
    theta, phi = geometry.pixel_angles(4)
    assert len(rings) == len(g["n"])
    for rr in rings:
        r = rr["i"] - 1
        s, n = int(g["start"][r]), int(g["n"][r])
        assert n == rr["n"]
        assert abs(g["z"][r] - _frac(rr["z"])) <= 2e-16
        want = _frac(rr["phi_first_over_pi"]) + 2.0 * np.arange(n) / n
        np.testing.assert_allclose(np.asarray(phi[s:s + n]) / np.pi, want, atol=1e-15)
        np.testing.assert_allclose(np.cos(theta[s:s + n]), _frac(rr["z"]), atol=2e-16)


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 64, 1024])
def test_equal_area_rings(nside):
    """Equal-area property: the pixels on rings 1..i-1 plus half of ring i
    cover exactly the spherical cap above ring i's latitude, area 2 pi (1-z_i).
    This pins z, the ring sizes and the ring starts together."""
    g = geometry.ring_geometry(nside)
    pix_area = 4.0 * np.pi / geometry.npix(nside)
    cum = (g["start"] + g["n"] / 2.0) * pix_area
    np.testing.assert_allclose(cum, 2.0 * np.pi * g["one_minus_z"], rtol=1e-14,
                               atol=1e-14)


@pytest.mark.parametrize("nside", [1, 2, 8, 256])
def test_symmetry_and_identities(nside):
    g = geometry.ring_geometry(nside)
    R = len(g["n"])
    # north/south mirror: z_{4N-i} = -z_i, same length and phi0
    np.testing.assert_allclose(g["z"], -g["z"][::-1], atol=1e-15)
    assert np.array_equal(g["n"], g["n"][::-1])
    np.testing.assert_allclose(g["phi0"], g["phi0"][::-1], atol=0)
    np.testing.assert_allclose(g["sth"] ** 2 + g["z"] ** 2, 1.0, atol=2e-16 * 8)
    np.testing.assert_allclose(g["one_minus_z"], 1.0 - g["z"], atol=4e-16)
    assert g["start"][0] == 0
    assert np.all(np.diff(g["start"]) == g["n"][:-1])
    # the ring next to the equator ring alternates phi0 in the belt
    for r in range(nside - 1, 3 * nside):
        i = r + 1
        want = np.pi / (4 * nside) if (i - nside) % 2 == 0 else 0.0
        assert g["phi0"][r] == want
    assert R == 4 * nside - 1
    # the south-cap ring start closed form s = Npix - 2 i'(i'+1)
    for r in range(3 * nside, R):
        ip = 4 * nside - (r + 1)
        assert g["start"][r] == geometry.npix(nside) - 2 * ip * (ip + 1)


def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        geometry.ring_geometry(3)
