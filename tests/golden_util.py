"""Loading the oracle's stored results for the full-size workloads
(written by ``tests/golden/make_golden.py``, which calls only the oracle and
the input generators) and comparing GPU outputs with them."""
import hashlib
import json
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def sha(a) -> str:
    """SHA-256 of an array's little-endian bytes in C order (as the writer)."""
    a = np.ascontiguousarray(a)
    return hashlib.sha256(a.astype(a.dtype.newbyteorder("<"), copy=False).tobytes()).hexdigest()


def load(name):
    with open(os.path.join(GOLDEN, name + ".json")) as fh:
        doc = json.load(fh)
    path = os.path.join(GOLDEN, name + "_stats.npz")
    arrays = dict(np.load(path, allow_pickle=False)) if os.path.exists(path) else None
    return doc, arrays


def check_labels(cell, doc, what=""):
    """Cell labels against the stored digest; on a mismatch name the first
    z-slab that differs."""
    if sha(cell) == doc["cell_sha256"]:
        return
    for lo, hi, h in doc["cell_slabs"]:
        if sha(cell[lo:hi]) != h:
            raise AssertionError(f"{what} cells differ from the oracle's, first in z-slab [{lo}, {hi})")
    raise AssertionError(f"{what} cells differ from the oracle's")


def level_stats(arrays, prefix, rows=None):
    """An oracle.Stats of the stored arrays (optionally a subset of rows)."""
    get = lambda k: arrays.get(f"{prefix}_{k}")
    st = oracle.Stats(*(get(k) for k in ("n", "mean", "m2", "vmin", "vmax", "hist", "cov")))
    return st


def exact_digests_match(got, digests, name):
    """n, min, max and histogram arrays of a device LevelStats against the
    stored digests of the oracle's."""
    from tests.gpu_util import host
    conv = {"n": lambda a: a.astype(np.uint64), "hist": lambda a: a.view(np.uint32)}
    for k, h in digests.items():
        a = host(getattr(got, k))
        a = conv.get(k, lambda z: z)(a)
        assert sha(a) == h, f"{name} {k} differs from the oracle's"
