"""Ring quadrature weights of the host helper (paper_2510_01785_amd.quadrature)
against the oracle: they integrate the m = 0 Legendre functions (the
least-squares conditions they are fitted to) better than the equal weights,
stay close to the equal weights, and make the oracle's weighted analysis and
refinement more accurate on band-limited fields (CPU).  The weight values
themselves are not the paper's (it gives none): parity unpinned."""
import numpy as np
import pytest

from oracle import sht
from paper_2510_01785_amd import quadrature, synth


def ring_of_pair(w_pair, nside):
    rings = np.arange(1, 4 * nside)
    return w_pair[np.where(rings <= 2 * nside, rings - 1, 4 * nside - 1 - rings)]


@pytest.mark.parametrize("nside", [8, 32])
def test_ring_weights_improve_the_analysis(nside):
    lmax = 2 * nside - 1
    w = quadrature.ring_weights_lsq(nside, lmax)
    eq = 4 * np.pi / (12 * nside * nside)
    assert w.shape == (2 * nside,)
    assert np.all(w > 0.3 * eq) and np.all(w < 2.0 * eq)
    # the conditions they are fitted to: ring sums of the Legendre
    # polynomials P_l (even l <= 2 lmax) against their integrals 4 pi delta_l0
    z, n = quadrature.ring_z(nside)
    mult = np.where(np.arange(2 * nside) == 2 * nside - 1, 1.0, 2.0) * n
    P = np.polynomial.legendre.legvander(z, 2 * lmax)[:, 0::2].T * mult[None, :]
    b = np.zeros(P.shape[0])
    b[0] = 4 * np.pi
    assert abs(P[0] @ w - 4 * np.pi) < 1e-12
    assert np.linalg.norm(P @ w - b) < np.linalg.norm(P @ np.full(2 * nside, eq) - b)
    a0 = synth.gaussian_alm(21, 1, lmax, "lp10")
    f = sht.alm2map(a0, nside, lmax)
    aw = sht.map2alm(f, lmax, nside, ring_weights=ring_of_pair(w, nside))
    ae = sht.map2alm(f, lmax, nside)
    err_w = [np.linalg.norm(x - a0) / np.linalg.norm(a0) for x in
             sht.jacobi_map2alm(f, lmax, nside, niter=2, ring_weights=ring_of_pair(w, nside))]
    err_e = [np.linalg.norm(x - a0) / np.linalg.norm(a0) for x in sht.jacobi_map2alm(f, lmax, nside, niter=2)]
    assert np.linalg.norm(aw - a0) < np.linalg.norm(ae - a0)
    assert err_w[2] < 0.2 * err_e[2]
