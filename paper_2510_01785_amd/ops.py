"""PyTorch-facing transforms over the libshtx C ABI.

PyTorch only provides device memory and the current HIP stream; every step of
the transforms runs in the library's kernels.  Tables are built once per
(nside, lmax, device) and kept resident; workspaces come from torch's caching
allocator per call.
"""
import threading

import torch

from . import _lib

_DTYPES = {torch.float64: _lib.F64, torch.float32: _lib.F32, torch.bfloat16: _lib.BF16}
_ALM_DTYPE = {_lib.F64: torch.complex128, _lib.F32: torch.complex64, _lib.BF16: torch.complex64}
_ALM_CODE = {torch.complex128: _lib.F64, torch.complex64: _lib.F32}

_tables = {}
_tables_lock = threading.Lock()


def nalm(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def npix(nside):
    return 12 * nside * nside


def nside_of(npix_):
    n = int(round((npix_ / 12) ** 0.5))
    if 12 * n * n != npix_:
        raise ValueError("%d is not a HEALPix pixel count" % npix_)
    return n


def _stream_ptr(device):
    return torch.cuda.current_stream(device).cuda_stream


def get_tables(nside, lmax, device):
    """Resident uint8 table tensor for (nside, lmax) on `device`."""
    device = torch.device(device)
    key = (nside, lmax, device.index if device.index is not None else torch.cuda.current_device())
    with _tables_lock:
        t = _tables.get(key)
        if t is not None:
            return t
        L = _lib.lib()
        nb = L.shtx_tables_bytes(nside, lmax)
        if nb == 0:
            raise ValueError("invalid (nside, lmax) = (%d, %d)" % (nside, lmax))
        t = torch.empty(nb, dtype=torch.uint8, device=device)
        _lib.check("shtx_tables_build",
                   L.shtx_tables_build(nside, lmax, t.data_ptr(), nb, _stream_ptr(device)))
        _tables[key] = t
        return t


def tables_work(nside, lmax, device):
    """(executed, full) Legendre triples of the pruned and the full (l, m,
    ring pair) triangle for the tables of (nside, lmax) on `device`."""
    import ctypes
    t = get_tables(nside, lmax, device)
    ex, fu = ctypes.c_longlong(0), ctypes.c_longlong(0)
    _lib.check("shtx_tables_work", _lib.lib().shtx_tables_work(t.data_ptr(), ctypes.byref(ex), ctypes.byref(fu),
                                                               _stream_ptr(torch.device(device))))
    return ex.value, fu.value


def clear_tables():
    with _tables_lock:
        L = _lib.lib()
        for t in _tables.values():
            L.shtx_tables_release(t.data_ptr())
        _tables.clear()


def workspace_bytes(nside, lmax, batch, code):
    return _lib.lib().shtx_workspace_bytes(nside, lmax, batch, code)


def _call(fn, nside, lmax, batch, code, src, dst, device):
    L = _lib.lib()
    tab = get_tables(nside, lmax, device)
    wb = L.shtx_workspace_bytes(nside, lmax, batch, code)
    work = torch.empty(wb, dtype=torch.uint8, device=device)
    st = getattr(L, fn)(nside, lmax, batch, code, src.data_ptr(), dst.data_ptr(), tab.data_ptr(),
                        work.data_ptr(), wb, _stream_ptr(device))
    _lib.check(fn, st)
    return dst


def _as_batched(x):
    return (x.unsqueeze(0), True) if x.dim() == 1 else (x, False)


def _check_device(x):
    if not x.is_cuda:
        raise ValueError("shtx transforms need a tensor on a ROCm device")


# ------------------------------------------------------------------ raw ops
def map2alm_raw(maps, lmax):
    """maps [B, Npix] (float64/float32/bfloat16, RING) -> alm [B, nalm] complex."""
    _check_device(maps)
    code = _DTYPES[maps.dtype]
    maps = maps.contiguous()
    B, n = maps.shape
    nside = nside_of(n)
    out = torch.empty((B, nalm(lmax)), dtype=_ALM_DTYPE[code], device=maps.device)
    return _call("shtx_map2alm", nside, lmax, B, code, maps, out, maps.device)


def map2alm_nested_raw(maps_nest, lmax):
    """maps [B, Npix] in NESTED order -> alm [B, nalm] (the layout conversion
    fused into the analysis' loads); no autograd."""
    _check_device(maps_nest)
    code = _DTYPES[maps_nest.dtype]
    maps_nest = maps_nest.contiguous()
    B, n = maps_nest.shape
    nside = nside_of(n)
    out = torch.empty((B, nalm(lmax)), dtype=_ALM_DTYPE[code], device=maps_nest.device)
    return _call("shtx_map2alm_nested", nside, lmax, B, code, maps_nest, out, maps_nest.device)


def alm2map_raw(alm, nside, lmax):
    """alm [B, nalm] complex128/complex64 -> maps [B, Npix] float64/float32."""
    _check_device(alm)
    code = _ALM_CODE[alm.dtype]
    alm = alm.contiguous()
    B = alm.shape[0]
    if alm.shape[1] != nalm(lmax):
        raise ValueError("alm has %d coefficients, lmax=%d needs %d" % (alm.shape[1], lmax, nalm(lmax)))
    out = torch.empty((B, npix(nside)), dtype=torch.float64 if code == _lib.F64 else torch.float32,
                      device=alm.device)
    return _call("shtx_alm2map", nside, lmax, B, code, alm, out, alm.device)


def map2alm_iter(maps, lmax, niter=3):
    """Iteratively refined analysis (a <- a + A(f - S a), niter times) of
    maps [B, Npix] float64/float32 -> alm [B, nalm] complex; no autograd."""
    _check_device(maps)
    squeeze = maps.dim() == 1
    maps = (maps.unsqueeze(0) if squeeze else maps).contiguous()
    code = _DTYPES[maps.dtype]
    B, n = maps.shape
    nside = nside_of(n)
    out = torch.empty((B, nalm(lmax)), dtype=_ALM_DTYPE[code], device=maps.device)
    L = _lib.lib()
    tab = get_tables(nside, lmax, maps.device)
    wb = L.shtx_iter_workspace_bytes(nside, lmax, B, code)
    if wb == 0:
        raise ValueError("map2alm_iter needs float64 or float32 maps")
    work = torch.empty(wb, dtype=torch.uint8, device=maps.device)
    st = L.shtx_map2alm_iter(nside, lmax, B, code, maps.data_ptr(), out.data_ptr(), int(niter), tab.data_ptr(),
                             work.data_ptr(), wb, _stream_ptr(maps.device))
    _lib.check("shtx_map2alm_iter", st)
    return out[0] if squeeze else out


def map2alm_backward_raw(grad_alm, nside, lmax, map_dtype):
    code = _DTYPES[map_dtype]
    grad_alm = grad_alm.contiguous().to(_ALM_DTYPE[code])
    B = grad_alm.shape[0]
    out = torch.empty((B, npix(nside)), dtype=map_dtype, device=grad_alm.device)
    return _call("shtx_map2alm_backward", nside, lmax, B, code, grad_alm, out, grad_alm.device)


def alm2map_backward_raw(grad_map, lmax, alm_dtype):
    code = _ALM_CODE[alm_dtype]
    grad_map = grad_map.contiguous().to(torch.float64 if code == _lib.F64 else torch.float32)
    B, n = grad_map.shape
    nside = nside_of(n)
    out = torch.empty((B, nalm(lmax)), dtype=alm_dtype, device=grad_map.device)
    return _call("shtx_alm2map_backward", nside, lmax, B, code, grad_map, out, grad_map.device)


# ------------------------------------------------------------- autograd ops
class Map2Alm(torch.autograd.Function):
    """Differentiable analysis; backward is the adjoint kernel chain."""

    @staticmethod
    def forward(ctx, maps, lmax):
        ctx.lmax = lmax
        ctx.nside = nside_of(maps.shape[-1])
        ctx.map_dtype = maps.dtype
        return map2alm_raw(maps, lmax)

    @staticmethod
    def backward(ctx, grad_alm):
        g = map2alm_backward_raw(grad_alm, ctx.nside, ctx.lmax, ctx.map_dtype)
        return g, None


class Alm2Map(torch.autograd.Function):
    """Differentiable synthesis; backward is the adjoint kernel chain."""

    @staticmethod
    def forward(ctx, alm, nside, lmax):
        ctx.lmax = lmax
        ctx.alm_dtype = alm.dtype
        return alm2map_raw(alm, nside, lmax)

    @staticmethod
    def backward(ctx, grad_map):
        g = alm2map_backward_raw(grad_map, ctx.lmax, ctx.alm_dtype)
        return g, None, None


def map2alm(maps, lmax):
    """Analysis of RING maps [..., Npix] (batch of 1-D) -> alm [..., nalm]."""
    x, squeeze = _as_batched(maps)
    out = Map2Alm.apply(x, lmax)
    return out[0] if squeeze else out


def alm2map(alm, nside, lmax):
    """Synthesis of alm [..., nalm] -> RING maps [..., Npix]."""
    x, squeeze = _as_batched(alm)
    out = Alm2Map.apply(x, nside, lmax)
    return out[0] if squeeze else out


# ------------------------------------------------------- pixel order conversion
def _reorder(fn, maps):
    _check_device(maps)
    x, squeeze = _as_batched(maps)
    code = _DTYPES[x.dtype]
    x = x.contiguous()
    B, n = x.shape
    nside = nside_of(n)
    out = torch.empty_like(x)
    _lib.check(fn, getattr(_lib.lib(), fn)(nside, B, code, x.data_ptr(), out.data_ptr(), _stream_ptr(x.device)))
    return out[0] if squeeze else out


def reorder(maps, src, dst):
    """Maps [..., Npix] from pixel layout `src` to layout `dst`, each "ring",
    "nested" or ("flat", origin in "SENW", clockwise)."""
    _check_device(maps)
    x, squeeze = _as_batched(maps)
    code = _DTYPES[x.dtype]
    x = x.contiguous()
    B, n = x.shape
    nside = nside_of(n)
    out = torch.empty_like(x)
    _lib.check("shtx_reorder", _lib.lib().shtx_reorder(nside, B, code, _lib.layout_code(src), _lib.layout_code(dst),
                                                       x.data_ptr(), out.data_ptr(), _stream_ptr(x.device)))
    return out[0] if squeeze else out


def nest2ring(maps):
    """NESTED-ordered maps [..., Npix] -> the same maps in RING order."""
    return _reorder("shtx_nest2ring", maps)


def ring2nest(maps):
    """RING-ordered maps [..., Npix] -> the same maps in NESTED order."""
    return _reorder("shtx_ring2nest", maps)


# ------------------------------------------------------------ spectral resize
def alm_resize(alm, lmax_in, lmax_out):
    """alm [..., nalm(lmax_in)] complex -> [..., nalm(lmax_out)]: kept for
    l <= min(lmax_in, lmax_out), zero above lmax_in."""
    _check_device(alm)
    x, squeeze = _as_batched(alm)
    code = _ALM_CODE[x.dtype]
    x = x.contiguous()
    if x.shape[1] != nalm(lmax_in):
        raise ValueError("alm has %d coefficients, not nalm(%d)" % (x.shape[1], lmax_in))
    out = torch.empty((x.shape[0], nalm(lmax_out)), dtype=x.dtype, device=x.device)
    _lib.check("shtx_alm_resize", _lib.lib().shtx_alm_resize(lmax_in, lmax_out, x.shape[0], code, x.data_ptr(),
                                                             out.data_ptr(), _stream_ptr(x.device)))
    return out[0] if squeeze else out


# ------------------------------------------------------- ring-weighted analysis
def map2alm_weighted_raw(maps, lmax, ring_weights):
    """Analysis with per-ring quadrature weights: maps [B, Npix] (RING),
    ring_weights [2 nside] float64 on the maps' device (entry p: north ring
    p + 1 and its southern mirror) -> alm [B, nalm].  No autograd."""
    _check_device(maps)
    code = _DTYPES[maps.dtype]
    maps = maps.contiguous()
    B, n = maps.shape
    nside = nside_of(n)
    w = ring_weights.to(device=maps.device, dtype=torch.float64).contiguous()
    if w.numel() != 2 * nside:
        raise ValueError("ring_weights needs 2*nside = %d entries" % (2 * nside))
    out = torch.empty((B, nalm(lmax)), dtype=_ALM_DTYPE[code], device=maps.device)
    L = _lib.lib()
    tab = get_tables(nside, lmax, maps.device)
    wb = L.shtx_workspace_bytes(nside, lmax, B, code)
    work = torch.empty(wb, dtype=torch.uint8, device=maps.device)
    _lib.check("shtx_map2alm_weighted",
               L.shtx_map2alm_weighted(nside, lmax, B, code, maps.data_ptr(), out.data_ptr(), w.data_ptr(),
                                       tab.data_ptr(), work.data_ptr(), wb, _stream_ptr(maps.device)))
    return out


# ------------------------------------------------------ pixel-weighted analysis
def map2alm_pixel_weighted_raw(maps, lmax, pixel_weights):
    """Analysis with one quadrature weight per pixel: maps [B, Npix] (RING),
    pixel_weights [Npix] float64 (RING order) -> alm [B, nalm].  No autograd."""
    _check_device(maps)
    code = _DTYPES[maps.dtype]
    maps = maps.contiguous()
    B, n = maps.shape
    nside = nside_of(n)
    w = pixel_weights.to(device=maps.device, dtype=torch.float64).contiguous()
    if w.numel() != n:
        raise ValueError("pixel_weights needs Npix = %d entries" % n)
    out = torch.empty((B, nalm(lmax)), dtype=_ALM_DTYPE[code], device=maps.device)
    L = _lib.lib()
    tab = get_tables(nside, lmax, maps.device)
    wb = L.shtx_workspace_bytes(nside, lmax, B, code)
    work = torch.empty(wb, dtype=torch.uint8, device=maps.device)
    _lib.check("shtx_map2alm_pixel_weighted",
               L.shtx_map2alm_pixel_weighted(nside, lmax, B, code, maps.data_ptr(), out.data_ptr(), w.data_ptr(),
                                             tab.data_ptr(), work.data_ptr(), wb, _stream_ptr(maps.device)))
    return out


def map2alm_iter_weighted(maps, lmax, niter=3, ring_weights=None, pixel_weights=None):
    """Refined analysis a <- a + A_w(f - S a) with the weighted analysis A_w:
    ring_weights [2 nside] (per ring pair) and / or pixel_weights [Npix] (RING
    order), float64; neither: equal weights.  maps [B, Npix] float64/float32."""
    _check_device(maps)
    squeeze = maps.dim() == 1
    maps = (maps.unsqueeze(0) if squeeze else maps).contiguous()
    code = _DTYPES[maps.dtype]
    B, n = maps.shape
    nside = nside_of(n)
    rw = None if ring_weights is None else ring_weights.to(device=maps.device, dtype=torch.float64).contiguous()
    pw = None if pixel_weights is None else pixel_weights.to(device=maps.device, dtype=torch.float64).contiguous()
    if rw is not None and rw.numel() != 2 * nside:
        raise ValueError("ring_weights needs 2*nside = %d entries" % (2 * nside))
    if pw is not None and pw.numel() != n:
        raise ValueError("pixel_weights needs Npix = %d entries" % n)
    out = torch.empty((B, nalm(lmax)), dtype=_ALM_DTYPE[code], device=maps.device)
    L = _lib.lib()
    tab = get_tables(nside, lmax, maps.device)
    wb = L.shtx_iter_workspace_bytes(nside, lmax, B, code)
    if wb == 0:
        raise ValueError("map2alm_iter_weighted needs float64 or float32 maps")
    work = torch.empty(wb, dtype=torch.uint8, device=maps.device)
    st = L.shtx_map2alm_iter_weighted(nside, lmax, B, code, maps.data_ptr(), out.data_ptr(), int(niter),
                                      None if rw is None else rw.data_ptr(), None if pw is None else pw.data_ptr(),
                                      tab.data_ptr(), work.data_ptr(), wb, _stream_ptr(maps.device))
    _lib.check("shtx_map2alm_iter_weighted", st)
    return out[0] if squeeze else out


# ---------------------------------------------------------- stored lambda
_lams = {}


def get_lambda_table(nside, lmax, device):
    """Resident stored-lambda table (uint8 tensor) for (nside, lmax) on
    `device`, built once: the BF16 Legendre operands of the BF16 matrix-core
    analysis (tiles of the pruned triangle)."""
    import ctypes
    device = torch.device(device)
    key = (nside, lmax, device.index if device.index is not None else torch.cuda.current_device())
    with _tables_lock:
        t = _lams.get(key)
        if t is not None:
            return t
    tab = get_tables(nside, lmax, device)
    L = _lib.lib()
    nb = ctypes.c_size_t(0)
    _lib.check("shtx_lambda_table_bytes", L.shtx_lambda_table_bytes(tab.data_ptr(), ctypes.byref(nb),
                                                                     _stream_ptr(device)))
    t = torch.empty(nb.value, dtype=torch.uint8, device=device)
    _lib.check("shtx_lambda_table_build", L.shtx_lambda_table_build(tab.data_ptr(), t.data_ptr(), nb.value,
                                                                     _stream_ptr(device)))
    with _tables_lock:
        _lams[key] = t
    return t


def release_lambda_tables():
    with _tables_lock:
        L = _lib.lib()
        for t in _lams.values():
            L.shtx_lambda_table_release(t.data_ptr())
        _lams.clear()


def map2alm_stored_raw(maps, lmax):
    """BF16 maps [B, Npix] -> alm [B, nalm] complex64 through the BF16
    matrix-core analysis with lambda read from the resident stored table
    (built on first use).  No autograd."""
    _check_device(maps)
    if maps.dtype != torch.bfloat16:
        raise ValueError("the stored-lambda analysis takes bfloat16 maps")
    maps = maps.contiguous()
    B, n = maps.shape
    nside = nside_of(n)
    lam = get_lambda_table(nside, lmax, maps.device)
    L = _lib.lib()
    tab = get_tables(nside, lmax, maps.device)
    wb = L.shtx_workspace_bytes(nside, lmax, B, _lib.BF16)
    work = torch.empty(wb, dtype=torch.uint8, device=maps.device)
    out = torch.empty((B, nalm(lmax)), dtype=torch.complex64, device=maps.device)
    _lib.check("shtx_map2alm_stored",
               L.shtx_map2alm_stored(nside, lmax, B, _lib.BF16, maps.data_ptr(), out.data_ptr(), tab.data_ptr(),
                                     lam.data_ptr(), work.data_ptr(), wb, _stream_ptr(maps.device)))
    return out
