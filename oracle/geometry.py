"""HEALPix RING geometry for the oracle (test infrastructure only).

ORACLE -- test infrastructure.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package.  It shares no code with
the HIP path.

The paper (Sec. III-A, "Structure of HEALPix Grids on a Sphere") fixes
Npix = 12*Nside^2 with Nside a power of two, Nrings = 4*Nside - 1, 4*Nside
pixels on every equatorial-belt ring and 4 pixels on the ring next to each
pole, pixels evenly spaced in longitude within a ring.  The remaining details
(ring colatitudes, the longitude offset phi0 of the first pixel of a ring and
the ring start index in RING order) come from the HEALPix definition paper the
method cites (Gorski et al. 2005); they are written out here:

  rings are i = 1 .. 4N-1 from north to south;
  north cap  (1 <= i < N):   n = 4i,  z = 1 - i^2/(3N^2),       phi0 = pi/(4i)
  belt       (N <= i <= 3N): n = 4N,  z = 4/3 - 2i/(3N),
                             phi0 = pi/(4N) if (i - N) is even else 0
  south cap  (i > 3N, i' = 4N - i): mirror of the north cap ring i'
  pixel j of ring i sits at phi = phi0 + 2*pi*j/n and has RING index s_i + j,
  with s_i the number of pixels on rings 1 .. i-1.

z is rounded to double as 1 - (i^2 / (3N^2)) (caps, division first) or
(4N - 2i) / (3N) (belt), and sin(theta) = sqrt((1 - z)(1 + z)) from that
double z, so that every ring is represented by one consistent colatitude.
"""
import numpy as np


def npix(nside):
    return 12 * nside * nside


def nrings(nside):
    return 4 * nside - 1


def check_nside(nside):
    if nside < 1 or (nside & (nside - 1)) != 0:
        raise ValueError("nside must be a power of two, got %r" % (nside,))


def ring_geometry(nside):
    """Per-ring geometry as a dict of arrays indexed by r = i - 1.

    Keys: n (pixels per ring), start (RING index of the first pixel), z (cos
    theta), one_minus_z, one_plus_z (both without cancellation), sth
    (sin theta), phi0 (longitude of the first pixel) and the integers
    phi0_num, phi0_den with phi0 = pi * phi0_num / phi0_den.
    """
    check_nside(nside)
    N = nside
    R = nrings(N)
    n = np.empty(R, dtype=np.int64)
    z = np.empty(R)
    omz = np.empty(R)
    opz = np.empty(R)
    # phi0 = pi * p0num / p0den, kept as a fraction so that m*phi0 can be
    # reduced modulo 2*pi exactly in integers
    p0num = np.zeros(R, dtype=np.int64)
    p0den = np.ones(R, dtype=np.int64)
    for r in range(R):
        i = r + 1
        if i < N:  # north polar cap
            n[r] = 4 * i
            z[r] = 1.0 - (i * i) / (3.0 * N * N)
            p0num[r], p0den[r] = 1, 4 * i
        elif i <= 3 * N:  # equatorial belt
            n[r] = 4 * N
            z[r] = (4 * N - 2 * i) / (3.0 * N)
            if (i - N) % 2 == 0:
                p0num[r], p0den[r] = 1, 4 * N
        else:  # south polar cap, mirror of ring i' = 4N - i
            ip = 4 * N - i
            n[r] = 4 * ip
            z[r] = -(1.0 - (ip * ip) / (3.0 * N * N))
            p0num[r], p0den[r] = 1, 4 * ip
    phi0 = np.pi * p0num / p0den
    start = np.zeros(R, dtype=np.int64)
    start[1:] = np.cumsum(n)[:-1]
    # sin(theta) is taken consistent with the double z: 1 - z and 1 + z are
    # formed from z itself (exact for |z| >= 1/2), so (z, sth) describe one
    # and the same colatitude acos(z) to rounding.
    omz[:] = 1.0 - z
    opz[:] = 1.0 + z
    sth = np.sqrt(omz * opz)
    return dict(n=n, start=start, z=z, one_minus_z=omz, one_plus_z=opz,
                sth=sth, phi0=phi0, phi0_num=p0num, phi0_den=p0den)


def pixel_angles(nside):
    """(theta, phi) of every pixel centre in RING order (plain loop)."""
    g = ring_geometry(nside)
    theta = np.empty(npix(nside))
    phi = np.empty(npix(nside))
    for r in range(len(g["n"])):
        s, n = g["start"][r], g["n"][r]
        th = np.arctan2(g["sth"][r], g["z"][r])
        for j in range(n):
            theta[s + j] = th
            phi[s + j] = g["phi0"][r] + 2.0 * np.pi * j / n
    return theta, phi


def nalm(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def alm_index(l, m, lmax):
    """m-major packed index of a_lm (0 <= m <= l <= lmax)."""
    return m * (2 * lmax + 1 - m) // 2 + l
