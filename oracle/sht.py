"""Spherical harmonic transforms on HEALPix RING maps (oracle, FP64).

ORACLE -- test infrastructure only; see oracle/__init__.py.

Analysis (map2alm) is the discrete sum of Eq. (1) / Eq. (26),
    a_lm = sum_p w_p f_p conj(Y_lm)(p),   w_p = 4 pi / Npix (equal weights),
and synthesis (alm2map) is Eq. (2) / Eq. (24),
    f_p = sum_{l, -l<=m<=l} a_lm Y_lm(p),   a_{l,-m} = (-1)^m conj(a_lm),
both evaluated separably (Eq. (12)-(14)): a Fourier sum in longitude on every
ring, then the Legendre sum over rings (analysis) or over l (synthesis).
Only m >= 0 is stored (m-major index, see geometry.alm_index); Im(a_l0) is
ignored on input and 0 on output.  Rings are summed one by one, with no
north/south parity fold.
"""
import numpy as np

from . import geometry
from .legendre import lambda_table, legendre_analysis, legendre_synthesis


def _ring_phase(g, r, mvals, sign):
    """exp(sign * i * m * phi0_r) with m*phi0 reduced mod 2 pi in integers."""
    num, den = int(g["phi0_num"][r]), int(g["phi0_den"][r])
    red = (mvals * num) % (2 * den)
    return np.exp(sign * 1j * np.pi * red / den)


def ring_weights_equal(nside):
    R = geometry.nrings(nside)
    return np.full(R, 4.0 * np.pi / geometry.npix(nside))


def ring_fourier_forward(maps, nside, lmax, ring_weights=None, mvals=None):
    """F[r, m, b] = w_r * sum_j f[b, s_r + j] * exp(-i m phi_{r,j}).

    The sum over a ring is evaluated with numpy's FP64 FFT: for phi_{r,j} =
    phi0_r + 2 pi j / n_r it equals exp(-i m phi0_r) * DFT_n(f)[m mod n].
    mvals selects the m (default 0..lmax); F is indexed by position in mvals.
    """
    g = geometry.ring_geometry(nside)
    maps = np.asarray(maps, dtype=np.float64)
    B = maps.shape[0]
    R = len(g["n"])
    w = ring_weights_equal(nside) if ring_weights is None else ring_weights
    mvals = np.arange(lmax + 1) if mvals is None else np.asarray(mvals, dtype=np.int64)
    F = np.empty((R, len(mvals), B), dtype=np.complex128)
    for r in range(R):
        s, n = int(g["start"][r]), int(g["n"][r])
        X = np.fft.fft(maps[:, s:s + n], axis=1)  # [B, n]
        ph = _ring_phase(g, r, mvals, -1.0)
        F[r] = (w[r] * X[:, mvals % n] * ph[None, :]).T
    return F


def ring_fourier_inverse(G, nside, lmax):
    """maps[b, s_r + j] = sum_{m=-lmax}^{lmax} G[r, |m|, b]' exp(i m phi_{r,j})

    where G' for negative m is conj(G) (real field) and the m = 0 term uses
    Re(G).  The frequencies are folded onto k = m mod n_r and summed with a
    length-n_r inverse DFT.
    """
    g = geometry.ring_geometry(nside)
    R, M, B = G.shape
    out = np.empty((B, geometry.npix(nside)))
    for r in range(R):
        s, n = int(g["start"][r]), int(g["n"][r])
        out[:, s:s + n] = _ring_inverse(g, r, G[r])
    return out


def _ring_inverse(g, r, Gr):
    """Pixels [B, n_r] of ring r from its spectrum Gr [M, B] (m = 0..M-1)."""
    M, B = Gr.shape
    n = int(g["n"][r])
    c = Gr * _ring_phase(g, r, np.arange(M), +1.0)[:, None]  # [M, B]
    rows = -(-M // n)
    pos = np.zeros((rows * n, B), dtype=np.complex128)
    pos[:M] = c
    pos[0] = c[0].real
    neg = np.zeros((rows * n, B), dtype=np.complex128)
    neg[1:M] = np.conj(c[1:])
    Cpos = pos.reshape(rows, n, B).sum(axis=0)       # k = m mod n
    Cneg = neg.reshape(rows, n, B).sum(axis=0)       # indexed by m mod n
    C = Cpos + Cneg[(-np.arange(n)) % n]              # k = -m mod n
    f = np.fft.ifft(C, axis=0) * n
    return f.real.T


def map2alm(maps, lmax, nside=None, ring_weights=None, nthreads=None, pixel_weights=None):
    """Forward SHT of real RING maps [B, Npix] -> complex alm [B, nalm].

    Quadrature weights (the schemes of Sec. IV-A): equal 4 pi / Npix by
    default; ring_weights [R] gives one weight per ring; pixel_weights [Npix]
    (RING order) one weight per pixel, a_lm = sum_p w_p f_p conj(Y_lm(p)) (the
    ring weights, if also given, multiply it; otherwise they are 1)."""
    maps = np.atleast_2d(np.asarray(maps, dtype=np.float64))
    if nside is None:
        nside = int(round(np.sqrt(maps.shape[1] / 12)))
    g = geometry.ring_geometry(nside)
    if pixel_weights is not None:
        maps = maps * np.asarray(pixel_weights, dtype=np.float64)[None, :]
        if ring_weights is None:
            ring_weights = np.ones(geometry.nrings(nside))
    F = ring_fourier_forward(maps, nside, lmax, ring_weights)
    return legendre_analysis(lmax, g["z"], g["sth"], F, nthreads)


def alm2map(alm, nside, lmax, nthreads=None):
    """Inverse SHT of complex alm [B, nalm] -> real RING maps [B, Npix]."""
    alm = np.atleast_2d(np.asarray(alm, dtype=np.complex128)).copy()
    alm[:, :lmax + 1] = alm[:, :lmax + 1].real  # m = 0 block: Im ignored
    g = geometry.ring_geometry(nside)
    G = legendre_synthesis(lmax, g["z"], g["sth"], alm, nthreads)
    return ring_fourier_inverse(G, nside, lmax)


def map2alm_m(maps, lmax, nside, ms):
    """Selected columns of map2alm: {m: alm[b, l - m] for l = m..lmax} for
    each m in ms, from the same ring sums and lambda recurrence as map2alm
    (for full-resolution spot checks where every m would be too slow)."""
    maps = np.atleast_2d(np.asarray(maps, dtype=np.float64))
    g = geometry.ring_geometry(nside)
    F = ring_fourier_forward(maps, nside, lmax, mvals=ms)  # [R, len(ms), B]
    out = {}
    for i, m in enumerate(ms):
        lam = lambda_table(lmax, int(m), g["z"], g["sth"])  # [lmax-m+1, R]
        out[int(m)] = (lam @ F[:, i, :]).T                   # [B, lmax-m+1]
    return out


def alm2map_rings(alm, nside, lmax, rings):
    """Selected rings of alm2map: {r: maps[b, s_r : s_r + n_r]} for each ring
    index r (0-based, north to south), from the same Legendre sums and ring
    Fourier synthesis as alm2map."""
    alm = np.atleast_2d(np.asarray(alm, dtype=np.complex128)).copy()
    alm[:, :lmax + 1] = alm[:, :lmax + 1].real
    g = geometry.ring_geometry(nside)
    rings = [int(r) for r in rings]
    B = alm.shape[0]
    G = np.zeros((len(rings), lmax + 1, B), dtype=np.complex128)
    z = np.asarray(g["z"])[rings]
    sth = np.asarray(g["sth"])[rings]
    for m in range(lmax + 1):
        lam = lambda_table(lmax, m, z, sth)                  # [lmax-m+1, nr]
        a = alm[:, geometry.alm_index(m, m, lmax):geometry.alm_index(lmax, m, lmax) + 1]
        G[:, m, :] = lam.T @ a.T
    return {r: _ring_inverse(g, r, G[i]) for i, r in enumerate(rings)}


def _m_of_index(lmax):
    m = np.empty(geometry.nalm(lmax), dtype=np.int64)
    for mm in range(lmax + 1):
        a = geometry.alm_index(mm, mm, lmax)
        m[a:a + lmax + 1 - mm] = mm
    return m


def _l_of_index(lmax):
    l = np.empty(geometry.nalm(lmax), dtype=np.int64)
    for mm in range(lmax + 1):
        a = geometry.alm_index(mm, mm, lmax)
        l[a:a + lmax + 1 - mm] = np.arange(mm, lmax + 1)
    return l


def map2alm_backward(grad_alm, nside, lmax, nthreads=None):
    """Gradient w.r.t. the map of a real loss, given dL/d(alm).

    Complex gradients follow PyTorch (dL/dRe + i dL/dIm).  With equal
    weights w = 4 pi/Npix the adjoint of map2alm (Sec. III-F: the synthesis
    scaled by the quadrature weights) on the m >= 0 storage is w * alm2map(G') with
    G'_l0 = Re G_l0 and G'_lm = G_lm / 2 for m > 0.
    """
    G = np.atleast_2d(np.asarray(grad_alm, dtype=np.complex128)).copy()
    m = _m_of_index(lmax)
    G[:, m > 0] *= 0.5
    G[:, m == 0] = G[:, m == 0].real
    return alm2map(G, nside, lmax, nthreads) * (4.0 * np.pi / geometry.npix(nside))


def alm2map_backward(grad_map, lmax, nside=None, nthreads=None):
    """Gradient w.r.t. alm of a real loss, given dL/d(map).

    The adjoint of the synthesis (Sec. III-F: the conjugate transpose of its
    matrix) on the m >= 0 storage is the
    unit-weight analysis sum, doubled for m > 0 (each stored a_lm also stands
    for a_{l,-m}); the m = 0 gradient is real.
    """
    g = np.atleast_2d(np.asarray(grad_map, dtype=np.float64))
    if nside is None:
        nside = int(round(np.sqrt(g.shape[1] / 12)))
    ones = np.ones(geometry.nrings(nside))
    out = map2alm(g, lmax, nside, ring_weights=ones, nthreads=nthreads)
    m = _m_of_index(lmax)
    out[:, m > 0] *= 2.0
    out[:, m == 0] = out[:, m == 0].real
    return out


def jacobi_map2alm(maps, lmax, nside, niter=3, nthreads=None, ring_weights=None, pixel_weights=None):
    """Iterative refinement of Eq. (4): a <- a + A(f - S a), niter times,
    with A the analysis of the given quadrature weights (equal by default).

    Returns the list [a^0, a^1, ..., a^niter] (niter+1 forward and niter
    inverse transforms).
    """
    maps = np.atleast_2d(np.asarray(maps, dtype=np.float64))

    def A(f):
        return map2alm(f, lmax, nside, ring_weights=ring_weights, nthreads=nthreads, pixel_weights=pixel_weights)
    a = A(maps)
    out = [a]
    for _ in range(niter):
        r = maps - alm2map(a, nside, lmax, nthreads)
        a = a + A(r)
        out.append(a)
    return out


def spectral_loss(alm, lmax):
    """L = sum_l w_l sum_{stored m>=0} |a_lm|^2 with w_l = 1/(l+1)."""
    l = _l_of_index(lmax)
    w = 1.0 / (l + 1.0)
    return float(np.sum(w[None, :] * np.abs(alm) ** 2))


def spectral_loss_grad(alm, lmax):
    """dL/d(alm) in the PyTorch complex convention: 2 w_l a_lm."""
    l = _l_of_index(lmax)
    return 2.0 * (1.0 / (l + 1.0))[None, :] * alm


def resize_alm(alm, lmax_in, lmax_out):
    """Coefficients of band limit lmax_in re-expressed at band limit lmax_out:
    a_lm kept for l <= min(lmax_in, lmax_out), zero for lmax_in < l <= lmax_out
    (truncation or zero extension of the spectrum; the map is unchanged by an
    extension and band-limited by a truncation).  Plain loops."""
    alm = np.asarray(alm)
    out = np.zeros(alm.shape[:-1] + (geometry.nalm(lmax_out),), dtype=alm.dtype)
    for m in range(min(lmax_in, lmax_out) + 1):
        for l in range(m, min(lmax_in, lmax_out) + 1):
            out[..., geometry.alm_index(l, m, lmax_out)] = alm[..., geometry.alm_index(l, m, lmax_in)]
    return out
