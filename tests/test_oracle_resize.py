"""Pins of the oracle's spectral resize (truncation / zero extension of a_lm)
against the transforms it serves (CPU)."""
import numpy as np
import pytest

from oracle import geometry, sht
from paper_2510_01785_amd import synth


@pytest.mark.parametrize("lmax,lbig,nside", [(7, 19, 4), (15, 23, 8)])
def test_extension_leaves_the_map_unchanged(lmax, lbig, nside):
    # zero extension adds only zero terms to the synthesis sum
    a = synth.gaussian_alm(91, 2, lmax, "lp10")
    f = sht.alm2map(a, nside, lmax)
    g = sht.alm2map(sht.resize_alm(a, lmax, lbig), nside, lbig)
    assert np.abs(f - g).max() < 1e-13 * np.abs(f).max()


@pytest.mark.parametrize("lmax,lbig", [(0, 5), (7, 19), (30, 31)])
def test_truncation_undoes_extension(lmax, lbig):
    a = synth.gaussian_alm(92, 3, lmax, "lp10")
    assert np.array_equal(sht.resize_alm(sht.resize_alm(a, lmax, lbig), lbig, lmax), a)
    assert np.array_equal(sht.resize_alm(a, lmax, lmax), a)


def test_truncation_commutes_with_the_analysis():
    # each a_lm of the analysis is its own sum over the map, whatever the band
    # limit: analysing at lbig and truncating equals analysing at lmax
    lmax, lbig, nside = 11, 23, 8
    f = sht.alm2map(synth.gaussian_alm(93, 2, lbig, "lp10"), nside, lbig)
    big = sht.map2alm(f, lbig, nside)
    small = sht.map2alm(f, lmax, nside)
    got = sht.resize_alm(big, lbig, lmax)
    assert np.abs(got - small).max() < 1e-13 * np.abs(small).max()
    ext = sht.resize_alm(small, lmax, lbig)
    tail = [geometry.alm_index(l, m, lbig) for m in range(lbig + 1) for l in range(m, lbig + 1) if l > lmax]
    assert np.all(ext[..., tail] == 0)
