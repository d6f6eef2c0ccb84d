"""Seeded synthetic inputs shared by the tests, the bench and the smoke run.

Only random draws and the prescribed angular power spectra live here; no
transform arithmetic.  Every workload is a Gaussian random field whose
coefficients a_lm are drawn with the stated C_l (a_l0 real), from
numpy.random.Generator(PCG64(seed)) in one standard_normal((B, nalm, 2)) call.
"""
import numpy as np

CONFIGS = {
    # plain FP64 round trip on one map
    "fp64_nside32": dict(nside=32, lmax=95, batch=1, dtype="f64", seed=17851,
                         spectrum="inv_lp1_sq", noise=1e-3),
    # batched FP32 transforms
    "fp32_nside256_b64": dict(nside=256, lmax=767, batch=64, dtype="f32", seed=17852,
                              spectrum="lp10"),
    # ML-shaped transform (the throughput workload)
    "fp32_nside1024_b16": dict(nside=1024, lmax=2047, batch=16, dtype="f32", seed=17853,
                               spectrum="lp10"),
    # finite-difference gradient case
    "fp64_nside16_fd": dict(nside=16, lmax=47, batch=2, dtype="f64", seed=17854,
                            spectrum="lp10"),
    # high-resolution single map with Jacobi refinement
    "nside2048_jacobi": dict(nside=2048, lmax=4095, batch=1, dtype="f64", seed=17855,
                             spectrum="l_m2"),
}


def nalm(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def lm_arrays(lmax):
    """(l, m) of every packed index idx(l,m) = m(2 lmax+1-m)/2 + l."""
    ls = np.empty(nalm(lmax), dtype=np.int64)
    ms = np.empty(nalm(lmax), dtype=np.int64)
    o = 0
    for m in range(lmax + 1):
        k = lmax + 1 - m
        ls[o:o + k] = np.arange(m, lmax + 1)
        ms[o:o + k] = m
        o += k
    return ls, ms


def spectrum(kind, lmax):
    l = np.arange(lmax + 1, dtype=np.float64)
    if kind == "inv_lp1_sq":
        return 1.0 / (l + 1.0) ** 2
    if kind == "lp10":
        return 1.0 / (l + 10.0) ** 2
    if kind == "l_m2":
        c = np.zeros(lmax + 1)
        c[2:] = 1.0 / l[2:] ** 2
        return c
    raise ValueError(kind)


def gaussian_alm(seed, batch, lmax, kind):
    """complex128 [batch, nalm]: Re, Im ~ N(0, C_l/2) for m > 0; a_l0 ~ N(0, C_l)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((batch, nalm(lmax), 2))
    ls, ms = lm_arrays(lmax)
    cl = spectrum(kind, lmax)[ls]
    scale = np.where(ms == 0, np.sqrt(cl), np.sqrt(cl / 2.0))
    re = g[..., 0] * scale
    im = np.where(ms == 0, 0.0, g[..., 1] * scale)
    return re + 1j * im


def pixel_noise(seed, batch, npix, sigma):
    """Independent N(0, sigma^2) per pixel, from a stream derived from seed."""
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    return sigma * rng.standard_normal((batch, npix))


def white_map(seed, batch, npix):
    rng = np.random.Generator(np.random.PCG64([seed, 2]))
    return rng.standard_normal((batch, npix))


def random_alm(seed, batch, lmax):
    """Unit complex Gaussian coefficients (flat spectrum), Im(a_l0) = 0."""
    rng = np.random.Generator(np.random.PCG64([seed, 3]))
    g = rng.standard_normal((batch, nalm(lmax), 2))
    a = g[..., 0] + 1j * g[..., 1]
    a[:, :lmax + 1] = a[:, :lmax + 1].real
    return a
