"""GPU parity of the RING <-> NESTED pixel order conversion (through the C
ABI) against the oracle's NESTED order: bit-exact (a permutation)."""
import numpy as np
import pytest
import torch

from oracle import nested

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shtx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_01785_amd as m
    return m


def announce(msg):
    print("\n[case] " + msg, flush=True)


def bits(t):
    """Raw bit patterns of a tensor (exact comparison, NaN-safe)."""
    view = {torch.float64: torch.int64, torch.float32: torch.int32, torch.bfloat16: torch.int16}[t.dtype]
    return t.view(view).cpu().numpy()


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 32, 128])
@pytest.mark.parametrize("batch", [1, 3])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_reorder_parity(shtx, nside, batch, dtype):
    announce("reorder nside=%d batch=%d %s" % (nside, batch, dtype))
    g = torch.Generator().manual_seed(1000 + nside + batch)
    x = torch.randn((batch, 12 * nside * nside), generator=g, dtype=torch.float64).to(dtype)
    ref_ring = nested.nest_to_ring(bits(x), nside)
    ref_nest = nested.ring_to_nest(bits(x), nside)
    xd = x.cuda()
    assert np.array_equal(bits(shtx.nest2ring(xd)), ref_ring)
    assert np.array_equal(bits(shtx.ring2nest(xd)), ref_nest)
    assert np.array_equal(bits(shtx.nest2ring(shtx.ring2nest(xd))), bits(x))


def test_reorder_single_map_1d(shtx):
    announce("reorder 1-D map nside=16")
    x = torch.arange(12 * 256, dtype=torch.float32)
    got = shtx.ring2nest(x.cuda()).cpu().numpy()
    assert np.array_equal(got, nested.ring_to_nest(x.numpy(), 16))


@pytest.mark.parametrize("nside,batch", [(1024, 16), (8192, 1)])
def test_reorder_fullsize_sampled(shtx, nside, batch):
    # the index of every pixel in its map: the output names each pixel's
    # source, checked against the oracle at sampled pixels (nside 8192 spans
    # the full 32-bit pixel index range of the kernel)
    announce("reorder full size nside=%d batch=%d" % (nside, batch))
    n = 12 * nside * nside
    dev = torch.device("cuda:0")
    # int32 pixel numbers carried as FP32 bit patterns (the copy is bitwise)
    x = torch.arange(n, dtype=torch.int32, device=dev).unsqueeze(0).expand(batch, n).contiguous()
    x = x.view(torch.float32)
    rng = np.random.default_rng(nside)
    sample = np.concatenate([np.arange(64), n - 64 + np.arange(64), rng.integers(0, n, 200000)])
    r = nested.nest_to_ring_index(nside, sample)
    to_ring = shtx.nest2ring(x)
    got = to_ring[batch - 1].view(torch.int32)[torch.from_numpy(r).to(dev)].cpu().numpy()
    assert np.array_equal(got, sample)  # RING slot r holds NESTED pixel p
    del to_ring
    to_nest = shtx.ring2nest(x)
    got = to_nest[0].view(torch.int32)[torch.from_numpy(sample).to(dev)].cpu().numpy()
    assert np.array_equal(got, r)  # NESTED slot p holds RING pixel r
    del to_nest
    torch.cuda.synchronize()


def test_nested_map_through_the_transform(shtx):
    # a NESTED map converted on the device analyses like its RING original
    announce("nest2ring then map2alm nside=32")
    from oracle import sht
    from paper_2510_01785_amd import synth
    nside, lmax = 32, 95
    alm0 = synth.gaussian_alm(4242, 2, lmax, "lp10")
    f = sht.alm2map(alm0, nside, lmax)
    f_nest = nested.ring_to_nest(f, nside)
    a = shtx.map2alm_raw(shtx.nest2ring(torch.tensor(f_nest, device="cuda:0")), lmax).cpu().numpy()
    ref = sht.map2alm(f, lmax, nside)
    assert np.linalg.norm(a - ref) / np.linalg.norm(ref) < 1e-12
