"""GPU parity of the spectral resize (through the C ABI) against the oracle:
bit-exact (a copy with zero fill), and its use between two resolutions."""
import numpy as np
import pytest
import torch

from oracle import sht
from paper_2510_01785_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shtx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_01785_amd as m
    return m


def announce(msg):
    print("\n[case] " + msg, flush=True)


@pytest.mark.parametrize("lin,lout", [(0, 0), (0, 5), (5, 0), (7, 7), (7, 300), (300, 7), (255, 256), (1000, 767)])
@pytest.mark.parametrize("batch", [1, 3])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_resize_parity(shtx, lin, lout, batch, dtype):
    announce("resize %d -> %d batch=%d %s" % (lin, lout, batch, dtype))
    a = synth.gaussian_alm(500 + lin, batch, lin, "lp10")
    x = torch.tensor(a, dtype=dtype)
    ref = sht.resize_alm(x.numpy(), lin, lout)
    got = shtx.alm_resize(x.cuda(), lin, lout).cpu().numpy()
    assert got.dtype == ref.dtype
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))


def test_resize_1d_and_full_size(shtx):
    announce("resize 2047 -> 4095 batch=16 complex64 (sampled) and a 1-D input")
    lin, lout, B = 2047, 4095, 16
    x = torch.tensor(synth.gaussian_alm(77, B, lin, "lp10"), dtype=torch.complex64).cuda()
    got = shtx.alm_resize(x, lin, lout)
    back = shtx.alm_resize(got, lout, lin)
    assert torch.equal(back, x)
    assert torch.equal(shtx.alm_resize(x[3], lin, lout), got[3])
    # the extension is zero above lin: its power equals the input's
    assert torch.allclose(torch.linalg.vector_norm(got, dim=1), torch.linalg.vector_norm(x, dim=1), rtol=1e-5)


def test_resolution_change_through_the_transforms(shtx):
    # analysis at nside 16 (lmax 31), resize to 63, synthesis at nside 32:
    # the band-limited field on the finer grid, against the oracle's
    announce("resolution change 16 -> 32")
    a = synth.gaussian_alm(78, 2, 31, "lp10")
    f16 = sht.alm2map(a, 16, 31)
    alm = shtx.map2alm_raw(torch.tensor(f16, device="cuda:0"), 31)
    f32 = shtx.alm2map_raw(shtx.alm_resize(alm, 31, 63), 32, 63).cpu().numpy()
    ref = sht.alm2map(sht.resize_alm(sht.map2alm(f16, 31, 16), 31, 63), 32, 63)
    assert np.linalg.norm(f32 - ref) / np.linalg.norm(ref) < 1e-12
