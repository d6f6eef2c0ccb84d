"""Pins for the oracle adjoints, loss and Jacobi loop (oracle/sht.py)."""
import numpy as np
import pytest
import torch

from oracle import brute, geometry, sht


def _rand_alm(rng, b, lmax):
    n = geometry.nalm(lmax)
    return rng.standard_normal((b, n)) + 1j * rng.standard_normal((b, n))


def _re_inner(a, b):
    return float(np.sum(a.real * b.real + a.imag * b.imag))


@pytest.mark.parametrize("nside,lmax", [(2, 7), (4, 11), (8, 23), (16, 47)])
def test_adjoint_identity_map2alm(nside, lmax):
    """<A f, G> = <f, A* G> (real inner products on the stored entries)."""
    rng = np.random.default_rng(11)
    f = rng.standard_normal((2, geometry.npix(nside)))
    G = _rand_alm(rng, 2, lmax)
    lhs = _re_inner(sht.map2alm(f, lmax, nside), G)
    rhs = float(np.sum(f * sht.map2alm_backward(G, nside, lmax)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("nside,lmax", [(2, 7), (4, 11), (8, 23), (16, 47)])
def test_adjoint_identity_alm2map(nside, lmax):
    """<S a, g> = <a, S* g> with Im(a_l0) ignored by S."""
    rng = np.random.default_rng(12)
    a = _rand_alm(rng, 2, lmax)
    a[:, :lmax + 1] = a[:, :lmax + 1].real
    g = rng.standard_normal((2, geometry.npix(nside)))
    lhs = float(np.sum(sht.alm2map(a, nside, lmax) * g))
    rhs = _re_inner(a, sht.alm2map_backward(g, lmax, nside))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_backward_matches_torch_autograd_dense():
    """PyTorch autograd through a dense complex model (scipy Y matrix) gives
    the same gradients as the oracle's backward formulas."""
    nside, lmax = 2, 7
    Y, lms = brute.ylm_matrix(nside, lmax)
    Yt = torch.from_numpy(Y)
    w = 4 * np.pi / geometry.npix(nside)
    rng = np.random.default_rng(13)
    # map2alm: a = w * f @ conj(Y); loss = Re<a, C> with a fixed complex C
    f = torch.tensor(rng.standard_normal((1, geometry.npix(nside))), requires_grad=True)
    C = _rand_alm(rng, 1, lmax)
    a = w * (f.to(torch.complex128) @ torch.conj(Yt))
    loss = (a * torch.from_numpy(np.conj(C))).real.sum()
    loss.backward()
    ga = sht.map2alm_backward(C, nside, lmax)  # dL/da = C
    np.testing.assert_allclose(f.grad.numpy(), ga, atol=1e-13)
    # alm2map: f = Re(sum over +-m); loss = <f, g>
    Yall, lms_all = brute.ylm_matrix(nside, lmax, negative_m=True)
    at = torch.tensor(_rand_alm(rng, 1, lmax), requires_grad=True)
    cols = []
    for (l, m) in lms_all:
        k = geometry.alm_index(l, abs(m), lmax)
        if m == 0:
            cols.append(at[:, k].real.to(torch.complex128))
        elif m > 0:
            cols.append(at[:, k])
        else:
            cols.append((-1) ** (-m) * torch.conj(at[:, k]))
    full = torch.stack(cols, dim=1)
    fmap = (full @ torch.from_numpy(Yall).T).real
    g = rng.standard_normal(fmap.shape)
    (fmap * torch.from_numpy(g)).sum().backward()
    gs = sht.alm2map_backward(g, lmax, nside)
    np.testing.assert_allclose(at.grad.numpy(), gs, atol=1e-13)


def test_loss_gradient_finite_differences_nside16():
    """Spectral loss L = sum_l w_l sum_m |a_lm|^2 of map2alm(f) at Nside=16,
    lmax=47: the chain rule through map2alm_backward matches central
    differences (L is quadratic in f, so differences are exact up to
    rounding)."""
    nside, lmax = 16, 47
    rng = np.random.default_rng(17854)
    f = rng.standard_normal((2, geometry.npix(nside)))
    a = sht.map2alm(f, lmax, nside)
    grad = sht.map2alm_backward(sht.spectral_loss_grad(a, lmax), nside, lmax)
    h = 1e-3
    for _ in range(4):
        d = rng.standard_normal(f.shape)
        lp = sht.spectral_loss(sht.map2alm(f + h * d, lmax, nside), lmax)
        lm = sht.spectral_loss(sht.map2alm(f - h * d, lmax, nside), lmax)
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(grad * d))
        assert abs(fd - an) <= 1e-9 * max(1.0, abs(an))


def test_jacobi_reduces_residual():
    """Eq. (4): for a band-limited map at lmax = 2 Nside - 1 each iteration
    lowers ||f - S a^k|| (the first step is the plain transform)."""
    nside, lmax = 8, 15
    rng = np.random.default_rng(3)
    a0 = _rand_alm(rng, 1, lmax)
    f = sht.alm2map(a0, nside, lmax)
    its = sht.jacobi_map2alm(f, lmax, nside, niter=3)
    assert len(its) == 4
    res = [np.linalg.norm(f - sht.alm2map(a, nside, lmax)) for a in its]
    assert res[1] < res[0] and res[2] < res[1] and res[3] < res[2]
    err = [np.linalg.norm(a - np.where(np.arange(a.shape[1]) <= lmax, a0.real, a0))
           for a in its]
    assert err[3] < err[0]
