"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Relative l2 tolerance: 1e-12 (FP64), 1e-5 (FP32)."""
import numpy as np
import pytest
import torch

from oracle import geometry, sht
from paper_2510_01785_amd import synth

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def rel_l2(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.linalg.norm((got - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def announce(msg):
    print("\n[case] " + msg, flush=True)


@pytest.fixture(scope="module")
def shtx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_01785_amd as m
    return m


def band_limited_map(seed, batch, nside, lmax, kind="lp10"):
    alm = synth.gaussian_alm(seed, batch, lmax, kind)
    return sht.alm2map(alm, nside, lmax)


CASES = [
    # nside, lmax, batch, dtype
    (1, 0, 1, torch.float64),
    (1, 3, 1, torch.float64),
    (2, 7, 2, torch.float64),
    (4, 15, 3, torch.float64),
    (8, 31, 1, torch.float64),
    (16, 47, 2, torch.float64),
    (32, 95, 1, torch.float64),
    (4, 11, 5, torch.float32),
    (8, 23, 17, torch.float32),
    (32, 95, 4, torch.float32),
    (64, 191, 16, torch.float32),
    (64, 127, 3, torch.float64),
    # every cap length up to 4*127 (Bluestein for lengths with a prime factor > 13)
    (128, 255, 2, torch.float64),
    (256, 300, 2, torch.float32),
    # matrix-core Legendre kernels (FP32, >= 8 channels; partial 16-channel groups)
    (16, 63, 8, torch.float32),
    (128, 383, 16, torch.float32),
    (256, 511, 24, torch.float32),
    # channel slices of the ring FFT that do not divide the batch (8 + 3 at
    # nside 256 FP32, 2 + 1 at nside 512 FP64)
    (256, 300, 11, torch.float32),
    (512, 600, 3, torch.float64),
    # FP64 on the matrix-core kernels (from 3 channels): two 8-channel groups
    # of the analysis and one 16-channel group of the synthesis, and a partial
    # group of 5 (the vector-ALU kernels' channel groups of 2, 2 + 2 + 1, are
    # covered by test_fp64_legendre_paths)
    (64, 191, 16, torch.float64),
    (32, 95, 5, torch.float64),
    # batched FP32 transforms at nside 256, lmax 767, 64 channels: four
    # 16-channel groups of the matrix-core kernels in one launch at lmax = 3N-1
    (256, 767, 64, torch.float32),
]


@pytest.mark.parametrize("nside,lmax,batch,dtype", CASES)
def test_map2alm_parity(shtx, nside, lmax, batch, dtype):
    announce("map2alm nside=%d lmax=%d B=%d %s" % (nside, lmax, batch, dtype))
    maps = synth.white_map(1000 + nside + lmax, batch, geometry.npix(nside))
    maps = maps + band_limited_map(2000 + lmax, batch, nside, min(lmax, 3 * nside - 1))
    x = torch.tensor(maps, dtype=dtype, device="cuda")
    ref = sht.map2alm(x.double().cpu().numpy(), lmax, nside)
    got = shtx.map2alm(x, lmax).cpu().numpy()
    torch.cuda.synchronize()
    assert got.shape == ref.shape
    assert np.all(got[:, :lmax + 1].imag == 0)
    assert rel_l2(got, ref) <= TOL[dtype]


@pytest.mark.parametrize("nside,lmax,batch,dtype", CASES)
def test_alm2map_parity(shtx, nside, lmax, batch, dtype):
    announce("alm2map nside=%d lmax=%d B=%d %s" % (nside, lmax, batch, dtype))
    alm = synth.gaussian_alm(3000 + nside + lmax, batch, lmax, "lp10")
    alm[:, :lmax + 1] += 1j * 0.5  # Im(a_l0) must be ignored
    ct = torch.complex128 if dtype == torch.float64 else torch.complex64
    a = torch.tensor(alm, dtype=ct, device="cuda")
    ref = sht.alm2map(a.cpu().numpy().astype(np.complex128), nside, lmax)
    got = shtx.alm2map(a, nside, lmax).cpu().numpy()
    assert got.shape == ref.shape
    assert rel_l2(got, ref) <= TOL[dtype]


@pytest.mark.parametrize("nside,lmax,batch,dtype", [(4, 15, 2, torch.float64), (16, 47, 2, torch.float64),
                                                    (16, 47, 6, torch.float64),
                                                    (8, 23, 3, torch.float32), (16, 47, 9, torch.float32),
                                                    (32, 95, 18, torch.float32)])
def test_backward_parity(shtx, nside, lmax, batch, dtype):
    announce("backward nside=%d lmax=%d B=%d %s" % (nside, lmax, batch, dtype))
    ct = torch.complex128 if dtype == torch.float64 else torch.complex64
    G = synth.random_alm(4000 + nside, batch, lmax)
    G[:, :lmax + 1] += 0.25j
    g = synth.white_map(5000 + nside, batch, geometry.npix(nside))
    Gt = torch.tensor(G, dtype=ct, device="cuda")
    gt = torch.tensor(g, dtype=dtype, device="cuda")
    got1 = shtx.map2alm_backward_raw(Gt, nside, lmax, dtype).cpu().numpy()
    ref1 = sht.map2alm_backward(Gt.cpu().numpy().astype(np.complex128), nside, lmax)
    assert rel_l2(got1, ref1) <= TOL[dtype]
    got2 = shtx.alm2map_backward_raw(gt, lmax, ct).cpu().numpy()
    ref2 = sht.alm2map_backward(gt.double().cpu().numpy(), lmax, nside)
    assert rel_l2(got2, ref2) <= TOL[dtype]


def test_config_fp64_nside32_round_trip(shtx):
    """Plain FP64 forward + inverse on one map at Nside=32, lmax=95: a band-
    limited field with C_l = 1/(l+1)^2 plus N(0, 1e-3^2) pixel noise."""
    c = synth.CONFIGS["fp64_nside32"]
    announce("config fp64_nside32")
    alm0 = synth.gaussian_alm(c["seed"], 1, c["lmax"], c["spectrum"])
    f = sht.alm2map(alm0, c["nside"], c["lmax"])
    f = f + synth.pixel_noise(c["seed"], 1, f.shape[1], c["noise"])
    x = torch.tensor(f, device="cuda")
    a_ref = sht.map2alm(f, c["lmax"], c["nside"])
    a = shtx.map2alm(x, c["lmax"])
    assert rel_l2(a.cpu().numpy(), a_ref) <= 1e-12
    f2_ref = sht.alm2map(a_ref, c["nside"], c["lmax"])
    f2 = shtx.alm2map(a, c["nside"], c["lmax"])
    assert rel_l2(f2.cpu().numpy(), f2_ref) <= 1e-12


def test_bf16_input_map2alm(shtx):
    announce("bf16 map2alm nside=32 lmax=95 B=4")
    nside, lmax = 32, 95
    f = band_limited_map(6000, 4, nside, lmax)
    x = torch.tensor(f, dtype=torch.float32, device="cuda").to(torch.bfloat16)
    ref = sht.map2alm(x.float().double().cpu().numpy(), lmax, nside)
    got = shtx.map2alm(x, lmax)
    assert got.dtype == torch.complex64
    assert rel_l2(got.cpu().numpy(), ref) <= 1e-5


# path: "mfma" forces the matrix-core Legendre kernels for every batch size,
# "valu" the vector-ALU kernels, "default" leaves the library's choice (the
# vector-ALU kernels below 5 channels for the analysis, below 8 for the
# synthesis).  Both switches are read per call.
_PATH_ENV = {"mfma": ("0", "1"), "valu": ("1", "1"), "default": ("0", None)}


@pytest.mark.parametrize("nside,lmax,batch,path", [(32, 95, 16, "mfma"), (64, 255, 20, "mfma"), (16, 47, 3, "mfma"),
                                                   (32, 95, 7, "valu"), (64, 191, 1, "valu"), (32, 95, 6, "valu"),
                                                   (32, 95, 13, "valu"),
                                                   (64, 191, 3, "default"), (64, 191, 6, "default"),
                                                   (64, 191, 9, "default")])
def test_fp32_legendre_paths(shtx, nside, lmax, batch, path, monkeypatch):
    """FP32 through the matrix-core and the vector-ALU Legendre kernels,
    each against the oracle."""
    force, min_batch = _PATH_ENV[path]
    monkeypatch.setenv("SHTX_FORCE_VALU", force)
    if min_batch is None:
        monkeypatch.delenv("SHTX_MFMA_MIN_BATCH", raising=False)
    else:
        monkeypatch.setenv("SHTX_MFMA_MIN_BATCH", min_batch)
    announce("fp32 legendre path %s nside=%d lmax=%d B=%d" % (path, nside, lmax, batch))
    f = synth.white_map(99, batch, geometry.npix(nside))
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    ref = sht.map2alm(x.double().cpu().numpy(), lmax, nside)
    a = shtx.map2alm(x, lmax)
    assert rel_l2(a.cpu().numpy(), ref) <= 1e-5
    g = shtx.alm2map(a, nside, lmax).cpu().numpy()
    gref = sht.alm2map(a.cpu().numpy().astype(np.complex128), nside, lmax)
    assert rel_l2(g, gref) <= 1e-5


@pytest.mark.parametrize("nside,lmax,batch,path", [(32, 95, 16, "mfma"), (16, 47, 19, "mfma"), (8, 31, 1, "mfma"),
                                                   (64, 255, 9, "mfma"), (1, 0, 4, "mfma"), (2, 7, 3, "mfma"),
                                                   (4, 15, 5, "default"),
                                                   (32, 95, 5, "valu"), (64, 191, 16, "valu"),
                                                   (64, 191, 2, "default"), (64, 191, 3, "default")])
def test_fp64_legendre_paths(shtx, nside, lmax, batch, path, monkeypatch):
    """FP64 through the matrix-core Legendre kernels (8-channel analysis
    groups, 16-channel synthesis groups, partial groups, one channel) and the
    vector-ALU ones (channel groups of 2 and 1), each against the oracle at
    the FP64 bar, analysis and synthesis."""
    force, min_batch = _PATH_ENV[path]
    monkeypatch.setenv("SHTX_FORCE_VALU", force)
    if min_batch is None:
        monkeypatch.delenv("SHTX_MFMA_MIN_BATCH", raising=False)
    else:
        monkeypatch.setenv("SHTX_MFMA_MIN_BATCH", min_batch)
    announce("fp64 legendre path %s nside=%d lmax=%d B=%d" % (path, nside, lmax, batch))
    f = synth.white_map(77, batch, geometry.npix(nside))
    x = torch.tensor(f, dtype=torch.float64, device="cuda")
    ref = sht.map2alm(f, lmax, nside)
    a = shtx.map2alm(x, lmax)
    assert rel_l2(a.cpu().numpy(), ref) <= 1e-12
    g = shtx.alm2map(a, nside, lmax).cpu().numpy()
    gref = sht.alm2map(a.cpu().numpy(), nside, lmax)
    assert rel_l2(g, gref) <= 1e-12


# BF16 gradient maps are the FP32 result rounded to nearest even: each value
# carries a relative rounding error of at most 2^-9, so the relative l2 error
# against the FP64 oracle is at most 2^-9 plus the FP32 arithmetic (~1e-7).
BF16_ROUND_TOL = 2.0 ** -9 + 1e-5
# BF16 matrix-core analysis (BF16 maps, from 5 channels): every product
# lambda * X has both factors rounded to BF16 (relative 2^-9 each), so each
# term carries at most 2^-8 relative error; for sums of white-noise terms
# without strong cancellation the relative l2 error of a_lm is of that order.
# The bar is 2^-8 times a cancellation allowance of 2.5 (a wrong operand
# layout or a lost term gives O(1) errors); the measured value is printed.
BF16_CONTRACT_TOL = 2.5 * 2.0 ** -8


@pytest.mark.parametrize("batch", [2, 9])
def test_bf16_map_autograd(shtx, batch):
    """Map2Alm on bfloat16 maps at nside 16, lmax 47: the backward writes a
    bfloat16 gradient map (the adjoint of Sec. III-F), compared with the
    oracle's map2alm_backward of the same upstream gradient; B=2 takes the
    vector-ALU synthesis kernel, B=9 the matrix-core one."""
    nside, lmax = 16, 47
    announce("bf16 autograd nside=%d lmax=%d B=%d" % (nside, lmax, batch))
    f = band_limited_map(6100 + batch, batch, nside, lmax) + synth.white_map(6100 + batch, batch, 12 * nside * nside)
    x = torch.tensor(f, dtype=torch.float32, device="cuda").to(torch.bfloat16).requires_grad_(True)
    a = shtx.map2alm(x, lmax)
    assert a.dtype == torch.complex64
    ls, _ = synth.lm_arrays(lmax)
    w = torch.tensor(1.0 / (ls + 1.0), device="cuda", dtype=torch.float32)
    loss = (w * a.abs() ** 2).sum()
    loss.backward()
    g = x.grad
    assert g.dtype == torch.bfloat16 and g.shape == x.shape
    a_gpu = a.detach().cpu().numpy().astype(np.complex128)
    a_ref = sht.map2alm(x.detach().float().double().cpu().numpy(), lmax, nside)
    # the backward (the adjoint of Sec. III-F) applied to the upstream
    # gradient of the forward's own output, by the oracle
    ref = sht.map2alm_backward(sht.spectral_loss_grad(a_gpu, lmax), nside, lmax)
    err = rel_l2(g.float().double().cpu().numpy(), ref)
    ea = rel_l2(a_gpu, a_ref)
    print("[bf16 autograd] B=%d rel l2: bf16 gradient map %.3e, forward a_lm %.3e" % (batch, err, ea), flush=True)
    assert err <= BF16_ROUND_TOL
    # the forward: FP32 contraction below 5 channels, BF16 from 5
    assert ea <= (1e-5 if batch < 5 else BF16_CONTRACT_TOL)


@pytest.mark.parametrize("nside,lmax,batch", [(16, 47, 5), (32, 95, 16), (64, 191, 20), (64, 255, 13),
                                              (128, 383, 16), (256, 767, 64), (32, 127, 6), (8, 31, 7)])
def test_bf16_contraction_parity(shtx, nside, lmax, batch, monkeypatch):
    """BF16 maps through the BF16 matrix-core analysis (BF16 spectra and
    Legendre operands, FP32 accumulation) against the FP64 oracle on the same
    BF16-rounded maps; and the same maps with SHTX_BF16_CONTRACT=f32 (FP32
    contraction) at the FP32 tolerance.  Batches not a multiple of 4 take the
    per-channel spectrum loads, B = 20 a partial 16-channel group."""
    announce("bf16 contraction nside=%d lmax=%d B=%d" % (nside, lmax, batch))
    f = synth.white_map(6200 + batch, batch, geometry.npix(nside))
    x = torch.tensor(f, dtype=torch.float32, device="cuda").to(torch.bfloat16)
    ref = sht.map2alm(x.float().double().cpu().numpy(), lmax, nside)
    monkeypatch.delenv("SHTX_BF16_CONTRACT", raising=False)
    monkeypatch.delenv("SHTX_FORCE_VALU", raising=False)
    monkeypatch.delenv("SHTX_MFMA_MIN_BATCH", raising=False)
    got = shtx.map2alm(x, lmax).cpu().numpy()
    err = rel_l2(got, ref)
    print("[bf16 contraction] nside=%d lmax=%d B=%d rel l2 vs oracle %.3e" % (nside, lmax, batch, err), flush=True)
    assert np.all(got[:, :lmax + 1].imag == 0)
    assert err <= BF16_CONTRACT_TOL
    monkeypatch.setenv("SHTX_BF16_CONTRACT", "f32")
    got32 = shtx.map2alm(x, lmax).cpu().numpy()
    assert rel_l2(got32, ref) <= 1e-5


def test_deterministic(shtx):
    announce("determinism nside=64 lmax=191 B=4 f32")
    x = torch.tensor(synth.white_map(7, 4, geometry.npix(64)), dtype=torch.float32, device="cuda")
    a1 = shtx.map2alm(x, 191)
    a2 = shtx.map2alm(x, 191)
    assert torch.equal(a1, a2)
    f1 = shtx.alm2map(a1, 64, 191)
    f2 = shtx.alm2map(a1, 64, 191)
    assert torch.equal(f1, f2)


def test_gradcheck_fp64(shtx):
    announce("gradcheck nside=2 lmax=5")
    x = torch.tensor(synth.white_map(11, 1, 48), dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: shtx.map2alm(t, 5), (x,), eps=1e-6, atol=1e-8)
    a = torch.tensor(synth.random_alm(12, 1, 5), dtype=torch.complex128, device="cuda", requires_grad=True)

    def f(t):
        # Im(a_l0) is ignored by the transform, so perturbations of it give a
        # zero numerical derivative and a zero analytic gradient.
        return shtx.alm2map(t, 2, 5)
    assert torch.autograd.gradcheck(f, (a,), eps=1e-6, atol=1e-8)


def test_loss_gradient_fd_nside16(shtx):
    """Spectral loss sum_l w_l sum_m |a_lm|^2, w_l = 1/(l+1), at Nside=16,
    lmax=47: autograd through the adjoint kernels vs central differences and
    vs the oracle's analytic gradient."""
    c = synth.CONFIGS["fp64_nside16_fd"]
    nside, lmax, B = c["nside"], c["lmax"], c["batch"]
    announce("loss FD nside=16")
    f = band_limited_map(c["seed"], B, nside, lmax) + synth.white_map(c["seed"], B, geometry.npix(nside))
    x = torch.tensor(f, device="cuda", requires_grad=True)
    ls, _ = synth.lm_arrays(lmax)
    w = torch.tensor(1.0 / (ls + 1.0), device="cuda")
    a = shtx.map2alm(x, lmax)
    loss = (w * a.abs() ** 2).sum()
    loss.backward()
    g = x.grad.cpu().numpy()
    ref = sht.map2alm_backward(sht.spectral_loss_grad(sht.map2alm(f, lmax, nside), lmax), nside, lmax)
    assert rel_l2(g, ref) <= 1e-12
    rng = np.random.default_rng(5)
    h = 1e-3
    for _ in range(3):
        d = rng.standard_normal(f.shape)
        lp = sht.spectral_loss(sht.map2alm(f + h * d, lmax, nside), lmax)
        lm = sht.spectral_loss(sht.map2alm(f - h * d, lmax, nside), lmax)
        assert abs((lp - lm) / (2 * h) - float(np.sum(g * d))) <= 1e-8 * max(1.0, abs(lp))


@pytest.mark.parametrize("nside,lmax,batch,dtype,niter", [(32, 95, 2, torch.float64, 3), (16, 47, 1, torch.float64, 0),
                                                          (32, 63, 17, torch.float32, 3), (32, 95, 3, torch.float32, 2),
                                                          (64, 191, 3, torch.float64, 1)])
def test_jacobi_iteration_parity(shtx, nside, lmax, batch, dtype, niter):
    """Iterative refinement a <- a + A(f - S a) (Eq. (4)) through the library's
    one entry point, against the oracle's loop of plain transforms."""
    announce("jacobi nside=%d lmax=%d B=%d %s niter=%d" % (nside, lmax, batch, dtype, niter))
    f = band_limited_map(7000 + nside, batch, nside, min(lmax, 2 * nside - 1))
    f = f + synth.pixel_noise(7000 + nside, batch, f.shape[1], 1e-3)
    x = torch.tensor(f, dtype=dtype, device="cuda")
    ref = sht.jacobi_map2alm(x.double().cpu().numpy(), lmax, nside, niter=niter)[-1]
    got = shtx.map2alm_iter(x, lmax, niter).cpu().numpy()
    assert rel_l2(got, ref) <= TOL[dtype]


@pytest.mark.parametrize("nside,lmax,batch", [(16, 47, 8), (64, 191, 16), (128, 383, 16), (256, 511, 20),
                                              (32, 95, 3)])
def test_stored_lambda_analysis(shtx, nside, lmax, batch, monkeypatch):
    """The stored-lambda analysis (BF16 Legendre tiles built once into a
    resident table, Sec. III-G, then read instead of recomputed): bit-identical
    to the BF16 matrix-core analysis that computes them (from 5 channels; below
    that map2alm takes the FP32 vector-ALU path, so the comparison is with the
    oracle at the BF16 bar), and within the BF16 bar of the oracle."""
    announce("stored lambda nside=%d lmax=%d B=%d" % (nside, lmax, batch))
    for k in ("SHTX_BF16_CONTRACT", "SHTX_FORCE_VALU", "SHTX_MFMA_MIN_BATCH"):
        monkeypatch.delenv(k, raising=False)
    f = synth.white_map(6300 + batch, batch, geometry.npix(nside))
    x = torch.tensor(f, dtype=torch.float32, device="cuda").to(torch.bfloat16)
    got = shtx.map2alm_stored_raw(x, lmax)
    if batch >= 5:
        assert torch.equal(got, shtx.map2alm_raw(x, lmax))
    ref = sht.map2alm(x.float().double().cpu().numpy(), lmax, nside)
    err = rel_l2(got.cpu().numpy(), ref)
    print("[stored lambda] nside=%d lmax=%d B=%d rel l2 vs oracle %.3e" % (nside, lmax, batch, err), flush=True)
    assert err <= BF16_CONTRACT_TOL
