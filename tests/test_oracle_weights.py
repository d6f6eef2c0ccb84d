"""Pins of the oracle's analysis with per-ring and per-pixel quadrature
weights (the ring and pixel weights of Sec. IV-A) against the dense
brute-force weighted sum (CPU, small grids), and of the weighted refinement
loop."""
import numpy as np
import pytest

from oracle import brute, geometry, sht
from paper_2510_01785_amd import synth


def pixel_weights(nside, w_ring):
    g = geometry.ring_geometry(nside)
    return np.repeat(w_ring, g["n"])


@pytest.mark.parametrize("nside,lmax", [(2, 5), (4, 11), (8, 17)])
def test_ring_weighted_analysis_is_the_weighted_sum(nside, lmax):
    rng = np.random.default_rng(nside)
    w_ring = rng.uniform(0.5, 1.5, 4 * nside - 1) * 4 * np.pi / geometry.npix(nside)
    f = sht.alm2map(synth.gaussian_alm(61, 2, lmax, "lp10"), nside, lmax) + rng.standard_normal((2, 12 * nside ** 2))
    got = sht.map2alm(f, lmax, nside, ring_weights=w_ring)
    ref = brute.map2alm_dense(f, nside, lmax, weights=pixel_weights(nside, w_ring))
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("nside,lmax", [(2, 5), (4, 11), (8, 23)])
def test_pixel_weighted_analysis_is_the_weighted_sum(nside, lmax):
    rng = np.random.default_rng(100 + nside)
    w_pix = rng.uniform(0.5, 1.5, 12 * nside ** 2) * 4 * np.pi / geometry.npix(nside)
    f = sht.alm2map(synth.gaussian_alm(64, 2, lmax, "lp10"), nside, lmax) + rng.standard_normal((2, 12 * nside ** 2))
    got = sht.map2alm(f, lmax, nside, pixel_weights=w_pix)
    ref = brute.map2alm_dense(f, nside, lmax, weights=w_pix)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_equal_pixel_weights_are_the_plain_analysis():
    nside, lmax = 8, 23
    f = np.random.default_rng(5).standard_normal((2, 12 * nside ** 2))
    w = np.full(12 * nside ** 2, 4 * np.pi / geometry.npix(nside))
    a = sht.map2alm(f, lmax, nside, pixel_weights=w)
    b = sht.map2alm(f, lmax, nside)
    assert np.abs(a - b).max() < 1e-14 * np.abs(b).max()


@pytest.mark.parametrize("kind", ["ring", "pixel"])
def test_weighted_refinement_is_the_loop_of_weighted_analyses(kind):
    """a^{k+1} = a^k + A_w (f - S a^k): checked against the dense weighted sum
    and dense synthesis, written out step by step (brute force, nside 4)."""
    nside, lmax = 4, 7
    rng = np.random.default_rng(9)
    npx = geometry.npix(nside)
    if kind == "ring":
        w_ring = rng.uniform(0.8, 1.2, 4 * nside - 1) * 4 * np.pi / npx
        kw = dict(ring_weights=w_ring)
        w_pix = pixel_weights(nside, w_ring)
    else:
        w_pix = rng.uniform(0.8, 1.2, npx) * 4 * np.pi / npx
        kw = dict(pixel_weights=w_pix)
    f = sht.alm2map(synth.gaussian_alm(65, 1, lmax, "lp10"), nside, lmax)
    got = sht.jacobi_map2alm(f, lmax, nside, niter=2, **kw)
    a = brute.map2alm_dense(f, nside, lmax, weights=w_pix)
    for k in range(3):
        assert np.abs(got[k] - a).max() < 1e-12 * np.abs(a).max()
        re, _ = brute.alm2map_dense(a, nside, lmax)
        a = a + brute.map2alm_dense(f - re, nside, lmax, weights=w_pix)
