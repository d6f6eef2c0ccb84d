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


def all_layouts():
    from oracle import layouts
    return layouts.all_layouts()


@pytest.mark.parametrize("nside", [1, 2, 4, 16, 64, 128])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_reorder_any_layout_parity(shtx, nside, dtype):
    """Every pair of RING, NESTED and the eight FLAT orientations (Sec. III-B,
    two-step conversion through (x, y, f)) against the oracle's conversion:
    bit-exact; nside 128 has two 64 x 64 squares per face side."""
    from oracle import layouts
    announce("reorder any layout nside=%d %s" % (nside, dtype))
    g = torch.Generator().manual_seed(2000 + nside)
    x = torch.randn((2, 12 * nside * nside), generator=g, dtype=torch.float64).to(dtype)
    xb = bits(x)
    xd = x.cuda()
    for src in all_layouts():
        for dst in all_layouts():
            got = bits(shtx.reorder(xd, src, dst))
            assert np.array_equal(got, layouts.convert(xb, nside, src, dst)), (src, dst)


def test_reorder_flat_fullsize_sampled(shtx):
    """Nside 1024, 4 FP32 channels: RING -> FLAT (origin E, clockwise) -> NESTED
    -> RING round trip is the identity, and 100k sampled FLAT pixels hold the
    RING pixel the oracle's (x, y, f) mapping names."""
    from oracle import layouts
    nside, B = 1024, 4
    announce("reorder flat full size nside=%d B=%d" % (nside, B))
    x = torch.randn((B, 12 * nside * nside), device="cuda", dtype=torch.float32)
    lay = ("flat", "E", True)
    fl = shtx.reorder(x, "ring", lay)
    back = shtx.reorder(shtx.reorder(fl, lay, "nested"), "nested", "ring")
    assert torch.equal(back, x)
    rng = np.random.default_rng(3)
    idx = rng.integers(0, 12 * nside * nside, 100000)
    xx, yy, ff = layouts.xyf_of_index(nside, lay, idx)
    ring = layouts.index_of_xyf(nside, "ring", xx, yy, ff)
    xs, fls = x.cpu().numpy(), fl.cpu().numpy()
    assert np.array_equal(fls[:, idx], xs[:, ring])


@pytest.mark.parametrize("nside,lmax,batch,dtype", [(4, 11, 2, torch.float64), (16, 47, 3, torch.float64),
                                                    (64, 191, 16, torch.float32), (128, 383, 5, torch.float32),
                                                    (32, 95, 16, torch.bfloat16), (256, 511, 2, torch.float32)])
def test_map2alm_nested_input(shtx, nside, lmax, batch, dtype):
    """Analysis of NESTED-ordered maps with the layout conversion fused into
    the ring FFT's loads: bit-identical to nest2ring followed by map2alm, and
    within the dtype tolerance of the oracle's analysis of the oracle's RING
    reordering."""
    from oracle import geometry, sht
    from paper_2510_01785_amd import synth
    announce("map2alm nested input nside=%d lmax=%d B=%d %s" % (nside, lmax, batch, dtype))
    f_ring = synth.white_map(4400 + nside, batch, geometry.npix(nside))
    f_nest = nested.ring_to_nest(f_ring, nside)
    xn = torch.tensor(f_nest, dtype=torch.float32 if dtype == torch.bfloat16 else dtype).to(dtype).cuda()
    got = shtx.map2alm_nested_raw(xn, lmax)
    two_pass = shtx.map2alm_raw(shtx.nest2ring(xn), lmax)
    torch.cuda.synchronize()
    assert torch.equal(got, two_pass)
    ref = sht.map2alm(nested.nest_to_ring(xn.double().cpu().numpy(), nside), lmax, nside)
    g = got.cpu().numpy()
    err = np.linalg.norm((g - ref).ravel()) / np.linalg.norm(ref.ravel())
    tol = {torch.float64: 1e-12, torch.float32: 1e-5, torch.bfloat16: 2.5 * 2.0 ** -8}[dtype]
    assert err <= tol
