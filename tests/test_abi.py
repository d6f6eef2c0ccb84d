"""Host-side checks of the C ABI (no GPU work: validation happens before any
launch, size queries are closed-form)."""
import ctypes
import os
import re

import pytest

from paper_2510_01785_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "shtx.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(shtx_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    decl = declared_functions()
    assert set(decl) == set(_lib.EXPORTS)
    for name in decl:
        assert hasattr(L, name), name


def test_status_strings():
    L = _lib.lib()
    for s in range(7):
        assert L.shtx_status_string(s)
    assert L.shtx_version() >= 100


def test_stage_names_match_the_binding():
    """The profiler's stage indices (an ABI of their own: shtx_profile_read
    takes them) name the stages the binding reads, in its order; indices
    past the last are rejected."""
    L = _lib.lib()
    assert tuple(L.shtx_stage_name(i).decode() for i in range(len(_lib.STAGES))) == _lib.STAGES
    assert L.shtx_stage_name(len(_lib.STAGES)) == b"unknown"
    ms, n = ctypes.c_double(), ctypes.c_longlong()
    assert L.shtx_profile_read(len(_lib.STAGES), ctypes.byref(ms), ctypes.byref(n)) == _lib.ERR_ARG


def nalm(l):
    return (l + 1) * (l + 2) // 2


# (nside, lmax, batch, dtype, spectrum channels: the batch)
@pytest.mark.parametrize("nside,lmax,batch,dtype,bspec", [(32, 95, 1, 0, 1), (1024, 2047, 16, 1, 16),
                                                           (1024, 2047, 16, 2, 16), (2048, 4095, 1, 0, 1),
                                                           (1, 0, 3, 1, 3), (1024, 2047, 5, 1, 5)])
def test_workspace_closed_form(nside, lmax, batch, dtype, bspec):
    cs = 16 if dtype == 0 else 8
    up = lambda x: (x + 255) // 256 * 256
    spec = (lmax + 1) * 2 * nside * bspec * cs
    third = (nalm(lmax) + 8) * batch * cs  # coefficients, 8 padding rows
    if dtype == 2:
        # BF16 maps: or the analysis' spectra in matrix-operand order (groups
        # of 16 channels x 2 parities x (lmax+1) x blocks of 8 ring pairs x 512 B)
        third = max(third, 2 * -(-batch // 16) * (lmax + 1) * -(-2 * nside // 8) * 512)
    want = 2 * up(spec) + up(third)
    assert _lib.lib().shtx_workspace_bytes(nside, lmax, batch, dtype) == want


def test_size_queries_reject_invalid():
    L = _lib.lib()
    assert L.shtx_tables_bytes(3, 10) == 0
    assert L.shtx_tables_bytes(0, 10) == 0
    assert L.shtx_tables_bytes(8, -1) == 0
    assert L.shtx_tables_bytes(4096, 10) == 0  # beyond supported nside
    assert L.shtx_workspace_bytes(8, 10, 0, 0) == 0
    assert L.shtx_workspace_bytes(8, 10, 1, 7) == 0
    assert L.shtx_tables_bytes(1024, 2047) > 0


FAKE = 0x7F0000000000  # never dereferenced: every call below fails validation


@pytest.mark.parametrize("fn", ["shtx_map2alm", "shtx_alm2map", "shtx_map2alm_backward", "shtx_alm2map_backward"])
def test_validation_before_launch(fn):
    L = _lib.lib()
    f = getattr(L, fn)
    wb = L.shtx_workspace_bytes(8, 15, 2, 1)
    # bad nside / lmax / batch / dtype
    assert f(6, 15, 2, 1, FAKE, FAKE, FAKE, FAKE, wb, None) == _lib.ERR_ARG
    assert f(8, -2, 2, 1, FAKE, FAKE, FAKE, FAKE, wb, None) == _lib.ERR_ARG
    assert f(8, 15, 0, 1, FAKE, FAKE, FAKE, FAKE, wb, None) == _lib.ERR_ARG
    assert f(8, 15, 2, 9, FAKE, FAKE, FAKE, FAKE, wb, None) == _lib.ERR_ARG
    # null pointers
    assert f(8, 15, 2, 1, None, FAKE, FAKE, FAKE, wb, None) == _lib.ERR_ARG
    assert f(8, 15, 2, 1, FAKE, None, FAKE, FAKE, wb, None) == _lib.ERR_ARG
    assert f(8, 15, 2, 1, FAKE, FAKE, None, FAKE, wb, None) == _lib.ERR_ARG
    assert f(8, 15, 2, 1, FAKE, FAKE, FAKE, None, wb, None) == _lib.ERR_ARG
    # unaligned workspace
    assert f(8, 15, 2, 1, FAKE, FAKE, FAKE, FAKE + 8, wb, None) == _lib.ERR_ARG
    # unaligned map (16 bytes; 8 for BF16) or alm (its complex element)
    map_first = fn in ("shtx_map2alm", "shtx_alm2map_backward")

    def args(map_off, alm_off):
        return (FAKE + map_off, FAKE + alm_off) if map_first else (FAKE + alm_off, FAKE + map_off)
    wb64 = L.shtx_workspace_bytes(8, 15, 2, 0)
    assert f(8, 15, 2, 1, *args(8, 0), FAKE, FAKE, wb, None) == _lib.ERR_ARG
    assert f(8, 15, 2, 1, *args(0, 4), FAKE, FAKE, wb, None) == _lib.ERR_ARG
    assert f(8, 15, 2, 0, *args(0, 8), FAKE, FAKE, wb64, None) == _lib.ERR_ARG
    # aligned variants pass validation up to the table lookup
    assert f(8, 15, 2, 1, *args(0, 8), FAKE, FAKE, wb, None) == _lib.ERR_TABLES
    # unsupported nside
    assert f(4096, 15, 2, 1, FAKE, FAKE, FAKE, FAKE, wb, None) == _lib.ERR_UNSUPPORTED
    # tables never built for this pointer
    assert f(8, 15, 2, 1, FAKE, FAKE, FAKE, FAKE, wb, None) == _lib.ERR_TABLES


def test_tables_build_validation():
    L = _lib.lib()
    assert L.shtx_tables_build(5, 10, FAKE, 1 << 30, None) == _lib.ERR_ARG
    assert L.shtx_tables_build(8, 10, None, 1 << 30, None) == _lib.ERR_ARG
    assert L.shtx_tables_build(8, 10, FAKE + 16, 1 << 30, None) == _lib.ERR_ARG
    assert L.shtx_tables_build(8, 10, FAKE, 16, None) == _lib.ERR_WORKSPACE
    assert L.shtx_tables_build(4096, 10, FAKE, 1 << 40, None) == _lib.ERR_UNSUPPORTED
    assert L.shtx_tables_release(FAKE) == _lib.ERR_TABLES


@pytest.mark.parametrize("fn", ["shtx_nest2ring", "shtx_ring2nest"])
def test_reorder_validation_before_launch(fn):
    L = _lib.lib()
    f = getattr(L, fn)
    big = 12 * 8 * 8 * 4 * 2  # bytes of one nside-8 FP32 map, twice
    a, b = FAKE, FAKE + 4 * big
    assert f(6, 1, 1, a, b, None) == _lib.ERR_ARG       # nside not a power of two
    assert f(16384, 1, 1, a, b, None) == _lib.ERR_ARG   # nside above 8192
    assert f(8, 0, 1, a, b, None) == _lib.ERR_ARG       # empty batch
    assert f(8, 1, 7, a, b, None) == _lib.ERR_ARG       # unknown dtype
    assert f(8, 1, 1, None, b, None) == _lib.ERR_ARG
    assert f(8, 1, 1, a, None, None) == _lib.ERR_ARG
    assert f(8, 1, 1, a + 2, b, None) == _lib.ERR_ARG   # FP32 element alignment
    assert f(8, 1, 0, a, b + 4, None) == _lib.ERR_ARG   # FP64 element alignment
    assert f(8, 1, 1, a, a + 64, None) == _lib.ERR_ARG  # overlapping input and output
    assert f(8, 2, 1, a, a + 12 * 64 * 4, None) == _lib.ERR_ARG


def test_alm_resize_validation_before_launch():
    L = _lib.lib()
    f = L.shtx_alm_resize
    a, b = FAKE, FAKE + (1 << 30)
    assert f(-1, 7, 1, 1, a, b, None) == _lib.ERR_ARG
    assert f(7, 8192, 1, 1, a, b, None) == _lib.ERR_ARG
    assert f(7, 9, 0, 1, a, b, None) == _lib.ERR_ARG
    assert f(7, 9, 1, 2, a, b, None) == _lib.ERR_ARG      # BF16 coefficients do not exist
    assert f(7, 9, 1, 1, None, b, None) == _lib.ERR_ARG
    assert f(7, 9, 1, 1, a, None, None) == _lib.ERR_ARG
    assert f(7, 9, 1, 1, a + 4, b, None) == _lib.ERR_ARG  # complex64 alignment
    assert f(7, 9, 1, 0, a, b + 8, None) == _lib.ERR_ARG  # complex128 alignment
    assert f(7, 9, 1, 1, a, a + 8, None) == _lib.ERR_ARG  # overlap


def test_weighted_analysis_validation_before_launch():
    L = _lib.lib()
    f = L.shtx_map2alm_weighted
    wb = L.shtx_workspace_bytes(8, 15, 2, 1)
    assert f(8, 15, 2, 1, FAKE, FAKE, None, FAKE, FAKE, wb, None) == _lib.ERR_ARG      # no weights
    assert f(8, 15, 2, 1, FAKE, FAKE, FAKE + 4, FAKE, FAKE, wb, None) == _lib.ERR_ARG  # misaligned weights
    assert f(6, 15, 2, 1, FAKE, FAKE, FAKE, FAKE, FAKE, wb, None) == _lib.ERR_ARG
    assert f(8, 15, 2, 1, FAKE, FAKE, FAKE, FAKE, FAKE, wb, None) == _lib.ERR_TABLES   # tables never built


def test_noalloc_limit_checked_before_any_gpu_work():
    """The allocation-free analysis rejects requests beyond its fixed scratch
    (SHTX_ERR_SCRATCH) and invalid arguments before touching the device."""
    L = _lib.lib()
    cap = L.shtx_noalloc_scratch_bytes()
    assert cap == 64 << 20
    assert L.shtx_map2alm_noalloc(1024, 2047, 16, 1, FAKE, FAKE, FAKE, None) == _lib.ERR_SCRATCH
    assert L.shtx_map2alm_noalloc(6, 15, 2, 1, FAKE, FAKE, FAKE, None) == _lib.ERR_ARG
    assert L.shtx_map2alm_noalloc(8, 15, 0, 1, FAKE, FAKE, FAKE, None) == _lib.ERR_ARG
    assert L.shtx_map2alm_noalloc(8, 15, 2, 5, FAKE, FAKE, FAKE, None) == _lib.ERR_ARG
