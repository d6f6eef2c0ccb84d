"""Pins for the oracle's normalised Legendre functions (oracle/legendre.c).

lambda_lm(cos theta) = Y_lm(theta, 0) (Eq. (8) with the (-1)^m of Eq. (15)).
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.special import sph_harm_y

from oracle import geometry, legendre

PI = math.pi


def closed_form(l, m, t):
    """Textbook closed forms of Y_lm(theta, 0), l <= 4, Condon-Shortley phase."""
    c, s = np.cos(t), np.sin(t)
    table = {
        (0, 0): 0.5 * np.sqrt(1 / PI) + 0 * c,
        (1, 0): 0.5 * np.sqrt(3 / PI) * c,
        (1, 1): -0.5 * np.sqrt(3 / (2 * PI)) * s,
        (2, 0): 0.25 * np.sqrt(5 / PI) * (3 * c**2 - 1),
        (2, 1): -0.5 * np.sqrt(15 / (2 * PI)) * s * c,
        (2, 2): 0.25 * np.sqrt(15 / (2 * PI)) * s**2,
        (3, 0): 0.25 * np.sqrt(7 / PI) * (5 * c**3 - 3 * c),
        (3, 1): -0.125 * np.sqrt(21 / PI) * s * (5 * c**2 - 1),
        (3, 2): 0.25 * np.sqrt(105 / (2 * PI)) * s**2 * c,
        (3, 3): -0.125 * np.sqrt(35 / PI) * s**3,
        (4, 0): 3 / 16 * np.sqrt(1 / PI) * (35 * c**4 - 30 * c**2 + 3),
        (4, 1): -3 / 8 * np.sqrt(5 / PI) * s * (7 * c**3 - 3 * c),
        (4, 2): 3 / 8 * np.sqrt(5 / (2 * PI)) * s**2 * (7 * c**2 - 1),
        (4, 3): -3 / 8 * np.sqrt(35 / PI) * s**3 * c,
        (4, 4): 3 / 16 * np.sqrt(35 / (2 * PI)) * s**4,
    }
    return table[(l, m)]


def test_closed_forms_l_le_4():
    t = np.linspace(0.01, PI - 0.01, 37)
    z, sth = np.cos(t), np.sin(t)
    for m in range(5):
        lam = legendre.lambda_table(4, m, z, sth)
        for l in range(m, 5):
            np.testing.assert_allclose(lam[l - m], closed_form(l, m, t),
                                       rtol=1e-14, atol=1e-15)


def test_matches_scipy_moderate_l():
    rng = np.random.default_rng(5)
    t = rng.uniform(0.05, PI - 0.05, 16)
    z, sth = np.cos(t), np.sin(t)
    lmax = 160
    for m in [0, 1, 2, 7, 40, 100, 160]:
        lam = legendre.lambda_table(lmax, m, z, sth)
        ls = np.arange(m, lmax + 1)
        ref = sph_harm_y(ls[:, None], m, t[None, :], 0.0).real
        scale = np.abs(ref).max()
        np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("l", [7, 95, 767, 2047, 4095])
def test_sum_rule(l):
    """Addition theorem: lambda_l0^2 + 2 sum_{m>=1} lambda_lm^2 = (2l+1)/(4 pi)
    at every colatitude (an exact invariant independent of the recurrence).
    Rounding in the l-recurrence grows with l and is largest on the rings
    next to the poles (about 5e-12 relative at l = 4095 on ring 1 of
    Nside=1024); any mistake in the recurrence coefficients gives O(1)
    violations, so 1e-11 separates the two."""
    N = 1024
    g = geometry.ring_geometry(N)
    pick = np.array([0, 1, 10, 300, 1023, 1500, 2047, 3000, 4094])
    z, sth = g["z"][pick], g["sth"][pick]
    tot = np.zeros(len(pick))
    for m in range(l + 1):
        lam = legendre.lambda_table(l, m, z, sth)[-1]
        tot += (1.0 if m == 0 else 2.0) * lam**2
    np.testing.assert_allclose(tot, (2 * l + 1) / (4 * PI),
                               rtol=1e-11)


def _mp_lambda(l, m, zval):
    mpmath.mp.dps = 50
    th = mpmath.acos(mpmath.mpf(float(zval)))
    return float(mpmath.spherharm(l, m, th, 0).real)


@pytest.mark.parametrize("ring,l,m", [
    (499, 3500, 600),   # sin(theta) ~ 0.198: lambda_{600,600} ~ 4e-422 underflows
    (3000, 4095, 3000),
    (3000, 4095, 100),
    (2047, 4095, 4095),
    (2047, 4094, 1),
    (10, 2047, 50),
])
def test_mpmath_spot_values_nside2048(ring, l, m):
    """High-precision values (mpmath at 50 digits, evaluated at the exact
    double z) at Nside=2048 ring colatitudes up to l = 4095.  The bound is
    a few ulps per recurrence step: 4 * l * 2^-52 relative."""
    g = geometry.ring_geometry(2048)
    z, sth = g["z"][ring], g["sth"][ring]
    lam = legendre.lambda_table(l, m, np.array([z]), np.array([sth]))[-1, 0]
    ref = _mp_lambda(l, m, z)
    assert abs(lam - ref) <= 4 * l * 2.0**-52 * abs(ref) + 1e-300


def test_underflow_then_recovery():
    """At ring 500 of Nside=2048 lambda_{600,600} is below the double range
    (~4.2e-422) but lambda_{3500,600} ~ 0.178: the scaled-exponent carry must
    return exactly 0 for the former and the full value for the latter."""
    g = geometry.ring_geometry(2048)
    z, sth = g["z"][499:500], g["sth"][499:500]
    lam = legendre.lambda_table(3500, 600, z, sth)[:, 0]
    assert lam[0] == 0.0
    assert abs(lam[-1] - 0.17796720000730817) < 1e-12
    assert np.all(np.isfinite(lam))
