"""ctypes binding of libshtx.so (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshtx.so")

F64, F32, BF16 = 0, 1, 2
OK, ERR_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP, ERR_TABLES, ERR_SCRATCH = range(7)

EXPORTS = ("shtx_version", "shtx_status_string", "shtx_tables_bytes", "shtx_tables_build",
           "shtx_tables_release", "shtx_tables_work", "shtx_workspace_bytes", "shtx_map2alm", "shtx_alm2map",
           "shtx_map2alm_backward", "shtx_alm2map_backward", "shtx_iter_workspace_bytes",
           "shtx_map2alm_iter", "shtx_profile_enable",
           "shtx_profile_reset", "shtx_profile_read", "shtx_stage_name", "shtx_nest2ring", "shtx_ring2nest",
           "shtx_alm_resize", "shtx_map2alm_weighted", "shtx_reorder", "shtx_map2alm_nested",
           "shtx_map2alm_pixel_weighted", "shtx_map2alm_iter_weighted", "shtx_lambda_table_bytes",
           "shtx_lambda_table_build", "shtx_lambda_table_release", "shtx_map2alm_stored",
           "shtx_noalloc_scratch_bytes", "shtx_map2alm_noalloc")
LAYOUT_RING, LAYOUT_NESTED, LAYOUT_FLAT = 0, 1, 2
FLAT_ORIGINS = ("S", "E", "N", "W")
STAGES = ("ring_fft_fwd", "legendre_fwd", "alm_in", "legendre_inv", "ring_fft_inv", "pack_bf16")

_lib = None


class ShtxError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        msg = lib().shtx_status_string(status).decode()
        super().__init__("%s failed: %s (status %d)" % (fn, msg, status))


def lib():
    """Load libshtx.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libshtx.so not built: run python -m paper_2510_01785_amd.build "
                          "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    L.shtx_version.argtypes = []
    L.shtx_version.restype = i
    L.shtx_status_string.argtypes = [i]
    L.shtx_status_string.restype = ctypes.c_char_p
    L.shtx_tables_bytes.argtypes = [i, i]
    L.shtx_tables_bytes.restype = sz
    L.shtx_tables_build.argtypes = [i, i, vp, sz, vp]
    L.shtx_tables_build.restype = i
    L.shtx_tables_release.argtypes = [vp]
    L.shtx_tables_release.restype = i
    L.shtx_tables_work.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong), vp]
    L.shtx_tables_work.restype = i
    L.shtx_workspace_bytes.argtypes = [i, i, i, i]
    L.shtx_workspace_bytes.restype = sz
    for name in ("shtx_map2alm", "shtx_alm2map", "shtx_map2alm_backward", "shtx_alm2map_backward",
                 "shtx_map2alm_nested"):
        f = getattr(L, name)
        f.argtypes = [i, i, i, i, vp, vp, vp, vp, sz, vp]
        f.restype = i
    L.shtx_iter_workspace_bytes.argtypes = [i, i, i, i]
    L.shtx_iter_workspace_bytes.restype = sz
    L.shtx_map2alm_iter.argtypes = [i, i, i, i, vp, vp, i, vp, vp, sz, vp]
    L.shtx_map2alm_iter.restype = i
    L.shtx_profile_enable.argtypes = [i]
    L.shtx_profile_enable.restype = i
    L.shtx_profile_reset.argtypes = []
    L.shtx_profile_reset.restype = i
    L.shtx_profile_read.argtypes = [i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]
    L.shtx_profile_read.restype = i
    L.shtx_stage_name.argtypes = [i]
    L.shtx_stage_name.restype = ctypes.c_char_p
    L.shtx_map2alm_weighted.argtypes = [i, i, i, i, vp, vp, vp, vp, vp, sz, vp]
    L.shtx_map2alm_weighted.restype = i
    L.shtx_map2alm_pixel_weighted.argtypes = [i, i, i, i, vp, vp, vp, vp, vp, sz, vp]
    L.shtx_map2alm_pixel_weighted.restype = i
    L.shtx_map2alm_iter_weighted.argtypes = [i, i, i, i, vp, vp, i, vp, vp, vp, vp, sz, vp]
    L.shtx_map2alm_iter_weighted.restype = i
    L.shtx_lambda_table_bytes.argtypes = [vp, ctypes.POINTER(sz), vp]
    L.shtx_lambda_table_bytes.restype = i
    L.shtx_lambda_table_build.argtypes = [vp, vp, sz, vp]
    L.shtx_lambda_table_build.restype = i
    L.shtx_lambda_table_release.argtypes = [vp]
    L.shtx_lambda_table_release.restype = i
    L.shtx_map2alm_stored.argtypes = [i, i, i, i, vp, vp, vp, vp, vp, sz, vp]
    L.shtx_map2alm_stored.restype = i
    L.shtx_noalloc_scratch_bytes.argtypes = []
    L.shtx_noalloc_scratch_bytes.restype = sz
    L.shtx_map2alm_noalloc.argtypes = [i, i, i, i, vp, vp, vp, vp]
    L.shtx_map2alm_noalloc.restype = i
    L.shtx_alm_resize.argtypes = [i, i, i, i, vp, vp, vp]
    L.shtx_alm_resize.restype = i
    L.shtx_reorder.argtypes = [i, i, i, i, i, vp, vp, vp]
    L.shtx_reorder.restype = i
    for name in ("shtx_nest2ring", "shtx_ring2nest"):
        f = getattr(L, name)
        f.argtypes = [i, i, i, vp, vp, vp]
        f.restype = i
    _lib = L
    return L


def profile_read():
    """{stage name: (total GPU ms, launches)} since the last reset."""
    L = lib()
    out = {}
    for s, name in enumerate(STAGES):
        ms = ctypes.c_double()
        n = ctypes.c_longlong()
        check("shtx_profile_read", L.shtx_profile_read(s, ctypes.byref(ms), ctypes.byref(n)))
        out[name] = (ms.value, n.value)
    return out


def layout_code(layout):
    """"ring", "nested" or ("flat", origin in "SENW", clockwise) -> ABI code."""
    if layout == "ring":
        return LAYOUT_RING
    if layout == "nested":
        return LAYOUT_NESTED
    kind, origin, clockwise = layout
    if kind != "flat" or origin not in FLAT_ORIGINS:
        raise ValueError("unknown layout %r" % (layout,))
    return LAYOUT_FLAT + 2 * FLAT_ORIGINS.index(origin) + int(bool(clockwise))


def check(fn, status):
    if status != OK:
        raise ShtxError(fn, status)
