"""Pins for the oracle transforms (oracle/sht.py) against brute force.

Brute force (oracle/brute.py) evaluates Eq. (1) and Eq. (2) densely with
scipy's Y_lm at every pixel centre; it shares no Legendre or FFT code with
oracle/sht.py.  lmax runs up to 4*Nside-1 so that m > n_r/2 (aliasing of the
ring DFT) occurs on many rings.
"""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

from oracle import brute, geometry, sht
from paper_2510_01785_amd import synth


CASES = [(1, 0), (1, 2), (1, 3), (2, 3), (2, 5), (2, 7), (4, 7), (4, 11),
         (4, 15), (8, 15), (8, 23), (8, 31)]


@pytest.mark.parametrize("nside,lmax", CASES)
def test_map2alm_brute_force(nside, lmax):
    rng = np.random.default_rng(100 + nside * 64 + lmax)
    maps = rng.standard_normal((3, geometry.npix(nside)))
    a = sht.map2alm(maps, lmax, nside)
    ref = brute.map2alm_dense(maps, nside, lmax)
    assert np.abs(a - ref).max() <= 1e-13 * np.abs(ref).max()
    # output convention: Im(a_l0) is exactly 0
    assert np.all(a[:, :lmax + 1].imag == 0.0)


@pytest.mark.parametrize("nside,lmax", CASES)
def test_alm2map_brute_force(nside, lmax):
    rng = np.random.default_rng(200 + nside * 64 + lmax)
    n = geometry.nalm(lmax)
    alm = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    f = sht.alm2map(alm, nside, lmax)
    ref_re, ref_im = brute.alm2map_dense(alm, nside, lmax)
    assert np.abs(ref_im).max() <= 1e-13 * np.abs(ref_re).max()  # real field
    assert np.abs(f - ref_re).max() <= 1e-13 * np.abs(ref_re).max()


@pytest.mark.parametrize("nside,lmax", [(1, 3), (4, 11), (32, 95)])
def test_constant_map(nside, lmax):
    """a_00 = sqrt(4 pi) c exactly (to rounding) for f = c."""
    c = 1.75
    a = sht.map2alm(np.full((1, geometry.npix(nside)), c), lmax, nside)
    assert abs(a[0, 0] - math.sqrt(4 * math.pi) * c) < 1e-14 * c * 10


def test_constant_map_residue_matches_brute_force():
    """The other coefficients of a constant map are quadrature residue, not
    zero; brute force fixes them."""
    f = np.full((1, geometry.npix(4)), 1.0)
    a = sht.map2alm(f, 15, 4)
    ref = brute.map2alm_dense(f, 4, 15)
    assert np.abs(a[0, 1:]).max() > 1e-3
    np.testing.assert_allclose(a, ref, atol=1e-14)


@pytest.mark.parametrize("nside,lmax", [(2, 7), (4, 15)])
def test_real_field_symmetry(nside, lmax):
    """a_{l,-m} = (-1)^m conj(a_lm) for a real map: brute force over negative
    m against the oracle's stored m >= 0 coefficients."""
    rng = np.random.default_rng(7)
    f = rng.standard_normal((1, geometry.npix(nside)))
    a = sht.map2alm(f, lmax, nside)[0]
    theta, phi = geometry.pixel_angles(nside)
    w = 4 * np.pi / geometry.npix(nside)
    for l in range(lmax + 1):
        for m in range(1, l + 1):
            neg = w * np.sum(f[0] * np.conj(sph_harm_y(l, -m, theta, phi)))
            want = (-1) ** m * np.conj(a[geometry.alm_index(l, m, lmax)])
            assert abs(neg - want) < 1e-13


@pytest.mark.parametrize("l,m", [(0, 0), (1, 0), (1, 1), (2, 1), (3, 2), (4, 4), (4, 3)])
def test_single_coefficient_reproduces_ylm(l, m):
    """alm2map of a single a_lm = 1 is Y_l0 (m = 0) or 2 Re Y_lm (m > 0) at
    the pixel centres, from the textbook closed forms."""
    from test_oracle_legendre import closed_form
    nside, lmax = 4, 6
    alm = np.zeros((1, geometry.nalm(lmax)), dtype=complex)
    alm[0, geometry.alm_index(l, m, lmax)] = 1.0
    f = sht.alm2map(alm, nside, lmax)[0]
    theta, phi = geometry.pixel_angles(nside)
    y = closed_form(l, m, theta) * np.exp(1j * m * phi)
    want = y.real if m == 0 else 2 * y.real
    np.testing.assert_allclose(f, want, atol=1e-14)


def test_batch_independent():
    rng = np.random.default_rng(9)
    maps = rng.standard_normal((4, geometry.npix(4)))
    a = sht.map2alm(maps, 11, 4)
    for b in range(4):
        np.testing.assert_array_equal(a[b], sht.map2alm(maps[b:b + 1], 11, 4)[0])


def test_odd_parity_vanishes_on_equator():
    """lambda_lm(0) = 0 for odd l+m (parity of Eq. (15))."""
    from oracle import legendre
    for m in range(0, 9):
        lam = legendre.lambda_table(40, m, np.array([0.0]), np.array([1.0]))[:, 0]
        ls = np.arange(m, 41)
        assert np.all(lam[(ls + m) % 2 == 1] == 0.0)


def test_sampled_outputs_match_full_transforms():
    """map2alm_m / alm2map_rings (the full-resolution spot-check forms) return
    exactly the corresponding columns / rings of map2alm / alm2map."""
    nside, lmax = 16, 40
    f = synth.white_map(3, 2, geometry.npix(nside))
    a = sht.map2alm(f, lmax, nside)
    for m, v in sht.map2alm_m(f, lmax, nside, [0, 3, 17, 40]).items():
        ref = a[:, geometry.alm_index(m, m, lmax):geometry.alm_index(lmax, m, lmax) + 1]
        assert np.allclose(v, ref, rtol=0, atol=1e-14)
    alm = synth.random_alm(4, 2, lmax)
    mp = sht.alm2map(alm, nside, lmax)
    g = geometry.ring_geometry(nside)
    for r, v in sht.alm2map_rings(alm, nside, lmax, [0, 5, 31, 62]).items():
        s0, n = int(g["start"][r]), int(g["n"][r])
        assert np.allclose(v, mp[:, s0:s0 + n], rtol=0, atol=1e-12)
