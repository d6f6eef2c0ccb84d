"""Pin of the oracle's analysis with per-ring quadrature weights (the ring
weights of Sec. IV-A) against the dense brute-force sum with the same weight
on every pixel of a ring (CPU, small grids)."""
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
