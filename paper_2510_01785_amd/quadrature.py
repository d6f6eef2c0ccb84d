"""Ring quadrature weights for the weighted analysis (host, numpy).

The paper (Sec. IV-A) compares three quadrature weight schemes for the
analysis sum of Eq. (1) -- equal, per ring and per pixel -- and finds ring
weights the most accurate, without stating how they are computed.  This
module computes one per-ring set: the weights w_r, one per iso-latitude ring
and symmetric about the equator, for which the ring quadrature integrates the
Legendre polynomials exactly, sum_r n_r w_r P_l(z_r) = int P_l(z) dz dphi =
4 pi delta_l0 for even l up to 2 lmax (odd l vanish by symmetry), solved in
the least-squares sense for the deviation from the equal weights 4 pi/Npix,
with singular values below 1e-3 of the largest dropped (the square system is
ill-conditioned; the truncated solution stays within about a factor 1.5 of
the equal weights), then scaled so that the weights add up to the sphere's
area exactly.  A weighted analysis with these weights is exact for
the m = 0 part of fields band-limited to lmax; they are inputs to
shtx_map2alm_weighted / shtx_map2alm_iter_weighted, not part of the
transform.
"""
import numpy as np


def ring_z(nside):
    """cos(theta) and pixel count of the 2 nside rings of the northern
    hemisphere and the equator (ring pair p = north ring p + 1)."""
    N = int(nside)
    i = np.arange(1, 2 * N + 1)
    z = np.where(i < N, 1.0 - (i * i) / (3.0 * N * N), (4.0 * N - 2.0 * i) / (3.0 * N))
    n = np.where(i < N, 4 * i, 4 * N)
    return z, n


def ring_weights_lsq(nside, lmax):
    """Per ring pair quadrature weights [2 nside] (entry p for the north ring
    p + 1 and its southern mirror, the last one for the equator)."""
    z, n = ring_z(nside)
    Rp = len(z)
    mult = np.where(np.arange(Rp) == Rp - 1, 1.0, 2.0) * n  # pixels of the pair
    ls = np.arange(0, 2 * lmax + 1, 2)
    # P_l(z) by the three-term recurrence (l+1) P_{l+1} = (2l+1) z P_l - l P_{l-1}
    P = np.empty((2 * lmax + 1, Rp))
    P[0] = 1.0
    if 2 * lmax >= 1:
        P[1] = z
    for l in range(1, 2 * lmax):
        P[l + 1] = ((2 * l + 1) * z * P[l] - l * P[l - 1]) / (l + 1)
    A = P[ls] * mult[None, :]
    b = np.zeros(len(ls))
    b[0] = 4.0 * np.pi
    w_eq = np.full(Rp, 4.0 * np.pi / (12.0 * nside * nside))
    d, *_ = np.linalg.lstsq(A, b - A @ w_eq, rcond=1e-3)
    w = w_eq + d
    return w * (4.0 * np.pi / np.dot(mult, w))  # the l = 0 condition (total area) exactly
