"""Helpers for GPU tests: numpy <-> torch device tensors with unsigned views."""
import sys

import numpy as np


def torch():
    import torch as _t
    return _t


def banner(msg):
    """Name the case on stdout before a GPU step (flushed, so it survives a crash)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray):
    """Copy a numpy array to the GPU; uint32 -> int32 view, uint16 -> int16 view."""
    t = torch()
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    elif a.dtype == np.uint16:
        a = a.view(np.int16)
    return t.from_numpy(a.copy()).cuda()


def host(x, dtype=None):
    """Copy a device tensor back; dtype reinterprets the bits (e.g. np.uint32)."""
    a = x.detach().cpu().numpy()
    if dtype is not None:
        a = a.view(dtype)
    return a
