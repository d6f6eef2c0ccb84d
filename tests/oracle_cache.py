"""Disk cache of oracle results for the full-size GPU parity tests.

A full-size oracle transform takes tens of seconds on the host, and several
tests compare against the same one; results are cached under
tests/_oracle_cache/ (not committed), keyed by a name and a digest of the
inputs, so a changed input recomputes.  Only oracle/ is called.
"""
import hashlib
import os

import numpy as np

CACHE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_oracle_cache")


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str((a.dtype.str, a.shape)).encode())
        h.update(memoryview(a).cast("B"))
    return h.hexdigest()[:16]


def cached(name, inputs, compute):
    """compute() once per (name, inputs); later calls load the stored array."""
    path = os.path.join(CACHE_DIR, "%s_%s.npy" % (name, digest(*inputs)))
    if os.path.exists(path):
        return np.load(path)
    out = compute()
    os.makedirs(CACHE_DIR, exist_ok=True)
    tmp = path + ".tmp%d.npy" % os.getpid()
    np.save(tmp, out)
    os.replace(tmp, path)
    return out
