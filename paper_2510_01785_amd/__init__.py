"""shtx: HEALPix spherical harmonic transforms for AMD MI355X (gfx950).

The transforms run in libshtx.so (hand-written HIP kernels behind a C ABI,
include/shtx.h); this package holds the thin Python binding and the seeded
input generators.  Importing it does not load the library: the first call of
a transform does, and raises if it has not been built.
"""

_LAZY = ("map2alm", "alm2map", "map2alm_raw", "map2alm_nested_raw", "alm2map_raw", "map2alm_backward_raw",
         "alm2map_backward_raw", "map2alm_iter", "Map2Alm", "Alm2Map", "get_tables", "tables_work",
         "clear_tables",
         "workspace_bytes", "nalm", "npix", "nside_of", "nest2ring", "ring2nest", "reorder", "alm_resize",
         "map2alm_weighted_raw", "map2alm_pixel_weighted_raw", "map2alm_iter_weighted",
         "map2alm_stored_raw", "get_lambda_table", "release_lambda_tables")


def __getattr__(name):
    if name in _LAZY:
        from . import ops
        return getattr(ops, name)
    raise AttributeError(name)
