"""The allocation-free analysis entry point (shtx_map2alm_noalloc) against
shtx_map2alm through the C ABI: the same kernels, so the same coefficients
bit for bit, on two calls in a row (the second smaller, reusing the fixed
scratch), plus FP32/FP64 parity with the oracle; and its size limit."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import geometry, sht
from paper_2510_01785_amd import _lib, synth

pytestmark = pytest.mark.gpu


def rel_l2(got, ref):
    return float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_01785_amd import ops as m
    return m


def noalloc(ops, x, lmax):
    L = _lib.lib()
    B, n = x.shape
    nside = ops.nside_of(n)
    code = ops._DTYPES[x.dtype]
    out = torch.empty((B, ops.nalm(lmax)), dtype=ops._ALM_DTYPE[code], device=x.device)
    tab = ops.get_tables(nside, lmax, x.device)
    st = L.shtx_map2alm_noalloc(nside, lmax, B, code, x.data_ptr(), out.data_ptr(), tab.data_ptr(),
                                torch.cuda.current_stream(x.device).cuda_stream)
    return st, out


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-5), (torch.float64, 1e-12), (torch.bfloat16, 2.5 * 2.0 ** -8)])
def test_noalloc_matches_map2alm_twice(ops, dtype, tol):
    cases = [(128, 383, 16), (32, 95, 3)]  # second call smaller than the first
    for i, (nside, lmax, B) in enumerate(cases):
        print("\n[case] noalloc %s nside=%d lmax=%d B=%d call %d" % (dtype, nside, lmax, B, i), flush=True)
        x = torch.tensor(synth.white_map(900 + i, B, geometry.npix(nside)), dtype=torch.float32,
                         device="cuda").to(dtype)
        st, got = noalloc(ops, x, lmax)
        assert st == _lib.OK, _lib.lib().shtx_status_string(st)
        want = ops.map2alm_raw(x, lmax)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        ref = sht.map2alm(x.double().cpu().numpy(), lmax, nside)  # BF16: the BF16-rounded maps
        assert rel_l2(got.cpu().numpy(), ref) <= tol


def test_noalloc_rejects_oversize(ops):
    L = _lib.lib()
    x = torch.zeros((16, geometry.npix(1024)), dtype=torch.float32, device="cuda")
    st, _ = noalloc(ops, x, 2047)
    assert st == _lib.ERR_SCRATCH
    assert b"scratch" in L.shtx_status_string(st)
