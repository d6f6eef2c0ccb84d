"""Dense brute-force transforms for tiny grids (oracle, FP64).

ORACLE -- test infrastructure only; see oracle/__init__.py.

Builds the full matrix of Y_lm at every pixel centre with
scipy.special.sph_harm_y (a library routine independent of legendre.c) and
evaluates Eq. (1) and Eq. (2) as plain matrix-vector products.  Only meant for
Nside <= 16.
"""
import numpy as np
from scipy.special import sph_harm_y

from . import geometry


def ylm_matrix(nside, lmax, negative_m=False):
    """Y[p, k] = Y_{l m}(theta_p, phi_p) for the (l, m) pairs of `lm_list`."""
    theta, phi = geometry.pixel_angles(nside)
    lms = lm_list(lmax, negative_m)
    Y = np.empty((len(theta), len(lms)), dtype=np.complex128)
    for k, (l, m) in enumerate(lms):
        Y[:, k] = sph_harm_y(l, m, theta, phi)
    return Y, lms


def lm_list(lmax, negative_m=False):
    """(l, m) pairs in m-major packed order; optionally all -l <= m <= l."""
    if negative_m:
        return [(l, m) for l in range(lmax + 1) for m in range(-l, l + 1)]
    return [(l, m) for m in range(lmax + 1) for l in range(m, lmax + 1)]


def map2alm_dense(maps, nside, lmax, weights=None):
    """a_lm = sum_p w f_p conj(Y_lm(p)), w = 4 pi / Npix (Eq. (1))."""
    Y, _ = ylm_matrix(nside, lmax)
    w = 4.0 * np.pi / geometry.npix(nside) if weights is None else weights
    return (np.atleast_2d(maps) * w) @ np.conj(Y)


def alm2map_dense(alm, nside, lmax):
    """f_p = sum over all (l, m) of a_lm Y_lm(p), a_{l,-m} = (-1)^m conj(a_lm)."""
    Yall, lms = ylm_matrix(nside, lmax, negative_m=True)
    alm = np.atleast_2d(alm)
    full = np.empty((alm.shape[0], len(lms)), dtype=np.complex128)
    for k, (l, m) in enumerate(lms):
        a = alm[:, geometry.alm_index(l, abs(m), lmax)]
        if m == 0:
            full[:, k] = a.real
        elif m > 0:
            full[:, k] = a
        else:
            full[:, k] = (-1) ** (-m) * np.conj(a)
    f = full @ Yall.T
    return f.real, f.imag
