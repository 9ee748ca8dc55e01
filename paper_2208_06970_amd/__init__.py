"""Python binding of the gfx950 LSRVT library (``liblsrvt.so``).

Argument marshalling only: every function below has the name of the C entry
point it wraps (``include/lsrvt.h``), takes torch tensors that live on the GPU
(torch provides device memory and streams, nothing else), and calls the HIP
library through ctypes.  There is no CPU fallback: importing the functions
without a built library raises ``LsrvtError``.

The pipeline (Neuroth et al., "Level Set Restricted Voronoi Tessellation"):

* :func:`lsrvt_isobands`   Sec. 3.1, isoband per voxel
* :func:`lsrvt_components` Sec. 3.1, 6-connected components per isoband
* :func:`lsrvt_vt`         Eq. 1, one restricted geodesic Voronoi pass
* :func:`lsrvt_update`     Sec. 3.1 centroid, one snapped site update
* :func:`lsrvt_cvt`        Algorithm 1 with a fixed number of updates
* :func:`lsrvt_aggregate`  Sec. 3.3 aggregation, cell -> component -> band
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsrvt.so")

OK, EINVAL, ENAN, ECAPACITY, EWORKSPACE, ELIMIT, EDEVICE = range(7)
NONE_ID = 0xFFFFFFFF
STATS_HIST = 1
STATS_COV = 2

EXPORTS = (
    "lsrvt_status_string", "lsrvt_version", "lsrvt_isobands", "lsrvt_components_workspace",
    "lsrvt_components", "lsrvt_vt", "lsrvt_update", "lsrvt_update_noalloc", "lsrvt_cvt_workspace", "lsrvt_cvt",
    "lsrvt_aggregate_workspace", "lsrvt_aggregate", "lsrvt_batch_workspace", "lsrvt_batch_run",
    "lsrvt_layout_workspace", "lsrvt_layout", "lsrvt_extract", "lsrvt_seed_workspace", "lsrvt_seed",
    "lsrvt_comoments_workspace", "lsrvt_comoments", "lsrvt_los_workspace", "lsrvt_los_vt", "lsrvt_los_update",
    "lsrvt_los_cvt", "lsrvt_set_vt_engine", "lsrvt_set_tuning", "lsrvt_timing_enable", "lsrvt_timing_read",
)


class LsrvtError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        msg = f"{what}: status {code}"
        if code >= 0:
            try:
                msg += f" ({_lib().lsrvt_status_string(code).decode()})"
            except Exception:  # pragma: no cover
                pass
        if detail:
            msg += f": {detail}"
        super().__init__(msg)
        self.code = code


class Dims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class MomentsC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_void_p), ("mean", ctypes.c_void_p), ("m2", ctypes.c_void_p), ("m3", ctypes.c_void_p),
                ("m4", ctypes.c_void_p)]


class CellStatsC(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("n", "mean", "m2", "vmin", "vmax", "hist", "cov")]


class GroupStatsC(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("n", "mean", "m2", "vmin", "vmax", "hist", "cov")]


class JobC(ctypes.Structure):
    """Mirror of lsrvt_job."""
    _fields_ = ([("dims", Dims), ("d_field", ctypes.c_void_p), ("h_iso", ctypes.c_void_p), ("n_iso", ctypes.c_int32),
                 ("d_seeds", ctypes.c_void_p), ("n_sites", ctypes.c_uint32), ("d_weights", ctypes.c_void_p),
                 ("iters", ctypes.c_int32), ("d_vars", ctypes.c_void_p), ("n_vars", ctypes.c_int32),
                 ("d_edges", ctypes.c_void_p), ("n_bins", ctypes.c_int32), ("flags", ctypes.c_uint32),
                 ("cap_comp", ctypes.c_uint32)]
                + [(k, ctypes.c_void_p) for k in ("d_band", "d_status", "d_comp", "d_comp_band", "d_comp_size",
                                                  "d_comp_first", "d_band_offset", "d_cell", "d_sites",
                                                  "d_site_comp")]
                + [("cell", CellStatsC), ("comp", GroupStatsC), ("band", GroupStatsC), ("n_comp", ctypes.c_uint32),
                   ("status", ctypes.c_int32)])


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise LsrvtError(-1, "load", f"{LIB_PATH} is not built (run __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        P, S = ctypes.c_void_p, ctypes.c_size_t
        i32, u32 = ctypes.c_int32, ctypes.c_uint32
        lib.lsrvt_status_string.argtypes = [i32]
        lib.lsrvt_status_string.restype = ctypes.c_char_p
        lib.lsrvt_version.restype = i32
        lib.lsrvt_isobands.argtypes = [P, Dims, P, i32, P, P, P]
        lib.lsrvt_components_workspace.argtypes = [Dims, i32]
        lib.lsrvt_components_workspace.restype = S
        lib.lsrvt_components.argtypes = [P, Dims, i32, P, u32, P, P, P, P, P, P, S, P]
        lib.lsrvt_vt.argtypes = [P, Dims, P, u32, P, P, S, P]
        lib.lsrvt_update.argtypes = [P, Dims, P, P, u32, P, P, S, P]
        lib.lsrvt_update_noalloc.argtypes = [P, Dims, P, P, u32, P, P]
        lib.lsrvt_cvt_workspace.argtypes = [Dims, u32, i32]
        lib.lsrvt_cvt_workspace.restype = S
        lib.lsrvt_cvt.argtypes = [P, P, Dims, P, u32, P, i32, P, P, P, P, P, S, P]
        lib.lsrvt_aggregate_workspace.argtypes = [Dims, u32, u32, i32, i32, i32, u32]
        lib.lsrvt_aggregate_workspace.restype = S
        lib.lsrvt_aggregate.argtypes = [P, Dims, P, P, u32, P, u32, i32, P, i32, P, i32, u32,
                                        ctypes.POINTER(CellStatsC), ctypes.POINTER(GroupStatsC),
                                        ctypes.POINTER(GroupStatsC), P, S, P]
        lib.lsrvt_batch_workspace.argtypes = [ctypes.POINTER(JobC), i32, i32]
        lib.lsrvt_batch_workspace.restype = S
        lib.lsrvt_batch_run.argtypes = [ctypes.POINTER(JobC), i32, i32, P, S, P]
        lib.lsrvt_layout_workspace.argtypes = [Dims, u32, u32]
        lib.lsrvt_layout_workspace.restype = S
        lib.lsrvt_layout.argtypes = [P, Dims, P, u32, P, u32, i32, P, P, P, P, P, ctypes.POINTER(u32), P, S, P]
        lib.lsrvt_extract.argtypes = [P, i32, Dims, P, u32, P, P]
        lib.lsrvt_comoments_workspace.argtypes = [Dims, u32, u32, i32, i32]
        lib.lsrvt_comoments_workspace.restype = S
        lib.lsrvt_comoments.argtypes = [P, Dims, P, P, u32, P, u32, i32, P, i32, ctypes.POINTER(MomentsC),
                                        ctypes.POINTER(MomentsC), ctypes.POINTER(MomentsC), P, S, P]
        lib.lsrvt_seed_workspace.argtypes = [Dims, u32, i32, u32]
        lib.lsrvt_seed_workspace.restype = S
        lib.lsrvt_seed.argtypes = [P, P, Dims, u32, P, P, u32, i32, ctypes.c_uint64, u32, P, u32,
                                   ctypes.POINTER(u32), ctypes.POINTER(u32), P, S, P]
        lib.lsrvt_los_workspace.argtypes = [Dims, u32]
        lib.lsrvt_los_workspace.restype = S
        lib.lsrvt_los_vt.argtypes = [P, Dims, P, P, u32, P, P, P, P, P, P, S, P]
        lib.lsrvt_los_update.argtypes = [P, Dims, P, P, P, u32, P, P, P, P, S, P]
        lib.lsrvt_los_cvt.argtypes = [P, Dims, P, u32, P, i32, P, P, P, P, P, P, P, P, S, P]
        lib.lsrvt_set_vt_engine.argtypes = [i32]
        lib.lsrvt_set_vt_engine.restype = i32
        lib.lsrvt_set_tuning.argtypes = [i32, i32]
        lib.lsrvt_set_tuning.restype = i32
        lib.lsrvt_timing_enable.argtypes = [i32]
        lib.lsrvt_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64),
                                          ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int32)]
        for name in ("lsrvt_isobands", "lsrvt_components", "lsrvt_vt", "lsrvt_update", "lsrvt_update_noalloc",
                     "lsrvt_cvt",
                     "lsrvt_aggregate", "lsrvt_batch_run", "lsrvt_layout", "lsrvt_extract", "lsrvt_seed",
                     "lsrvt_comoments", "lsrvt_los_vt", "lsrvt_los_update", "lsrvt_los_cvt",
                     "lsrvt_timing_enable", "lsrvt_timing_read"):
            getattr(lib, name).restype = i32
        _LIB = lib
    return _LIB


def library():
    """The loaded ctypes library (raises if it is not built)."""
    return _lib()


# --------------------------------------------------------------------------
# marshalling helpers
def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dims(shape) -> Dims:
    nz, ny, nx = (int(v) for v in shape)
    return Dims(nx, ny, nz)


def _need(t, dtype, what):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise LsrvtError(EINVAL, what, "expected a CUDA tensor")
    if t.dtype != dtype:
        raise LsrvtError(EINVAL, what, f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise LsrvtError(EINVAL, what, "expected a contiguous tensor")
    return t


def _check(code, what):
    if code != OK:
        raise LsrvtError(int(code), what)


class Workspace:
    """A growable, 256-byte-aligned device scratch buffer owned by the caller."""

    def __init__(self, device=None):
        self.device = device
        self.buf = None
        self.bytes = 0

    def get(self, nbytes: int):
        torch = _torch()
        nbytes = int(nbytes)
        if self.buf is None or self.bytes < nbytes:
            self.buf = torch.empty(nbytes + 512, dtype=torch.uint8, device=self.device or "cuda")
            self.bytes = nbytes
        base = self.buf.data_ptr()
        off = (-base) % 256
        return ctypes.c_void_p(base + off), nbytes


_default_ws = {}


def _ws(ws):
    if ws is not None:
        return ws
    torch = _torch()
    dev = torch.cuda.current_device()
    if dev not in _default_ws:
        _default_ws[dev] = Workspace(f"cuda:{dev}")
    return _default_ws[dev]


# --------------------------------------------------------------------------
# entry points
def lsrvt_isobands(field, iso, band=None, status=None, stream=None):
    """Isoband per voxel: #{k : iso[k] < f} (Sec. 3.1).  Returns (band, status)."""
    torch = _torch()
    _need(field, torch.float32, "lsrvt_isobands")
    iso = np.ascontiguousarray(np.asarray(iso, dtype=np.float32))
    if band is None:
        band = torch.empty(field.shape, dtype=torch.uint8, device=field.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=field.device)
    code = _lib().lsrvt_isobands(_ptr(field), _dims(field.shape), iso.ctypes.data_as(ctypes.c_void_p), len(iso),
                                 _ptr(band), _ptr(status), _stream(stream))
    _check(code, "lsrvt_isobands")
    return band, status


@dataclass
class Components:
    comp: "object"
    n_comp: int
    comp_band: "object"
    comp_size: "object"
    comp_first: "object"
    band_offset: "object"


def lsrvt_components(band, n_bands: int, comp=None, cap_comp: int | None = None, ws: Workspace | None = None,
                     stream=None) -> Components:
    """6-connected components per band, numbered by (band, min index) (Sec. 3.1)."""
    torch = _torch()
    _need(band, torch.uint8, "lsrvt_components")
    dev = band.device
    lib = _lib()
    dims = _dims(band.shape)
    if comp is None:
        comp = torch.empty(band.shape, dtype=torch.int32, device=dev)
    cap = int(cap_comp) if cap_comp is not None else max(1024, band.numel() // 64)
    ws = _ws(ws)
    wptr, wbytes = ws.get(lib.lsrvt_components_workspace(dims, n_bands))
    bo = torch.empty(n_bands + 1, dtype=torch.int32, device=dev)
    ncomp = ctypes.c_uint32(0)
    while True:
        cb = torch.empty(cap, dtype=torch.uint8, device=dev)
        cs = torch.empty(cap, dtype=torch.int64, device=dev)
        cf = torch.empty(cap, dtype=torch.int32, device=dev)
        code = lib.lsrvt_components(_ptr(band), dims, n_bands, _ptr(comp), cap, _ptr(cb), _ptr(cs), _ptr(cf),
                                    _ptr(bo), ctypes.byref(ncomp), wptr, wbytes, _stream(stream))
        if code == ECAPACITY:
            cap = int(ncomp.value)
            continue
        _check(code, "lsrvt_components")
        break
    k = int(ncomp.value)
    return Components(comp, k, cb[:k], cs[:k], cf[:k], bo)


def lsrvt_vt(band, sites, cell=None, ws: Workspace | None = None, stream=None):
    """One restricted geodesic Voronoi pass (Eq. 1, hop metric, id tie-break)."""
    torch = _torch()
    _need(band, torch.uint8, "lsrvt_vt")
    _need(sites, torch.int32, "lsrvt_vt")
    lib = _lib()
    dims = _dims(band.shape)
    if cell is None:
        cell = torch.empty(band.shape, dtype=torch.int32, device=band.device)
    ws = _ws(ws)
    wptr, wbytes = ws.get(lib.lsrvt_cvt_workspace(dims, sites.numel(), 0))
    code = lib.lsrvt_vt(_ptr(band), dims, _ptr(sites), sites.numel(), _ptr(cell), wptr, wbytes, _stream(stream))
    _check(code, "lsrvt_vt")
    return cell


def lsrvt_update(cell, sites, weights=None, ds=None, ws: Workspace | None = None, stream=None):
    """One snapped centroid update of ``sites`` in place; returns (sites, ds)."""
    torch = _torch()
    _need(cell, torch.int32, "lsrvt_update")
    _need(sites, torch.int32, "lsrvt_update")
    if weights is not None:
        _need(weights, torch.int16, "lsrvt_update")
    lib = _lib()
    dims = _dims(cell.shape)
    if ds is None:
        ds = torch.empty(sites.numel(), dtype=torch.float64, device=cell.device)
    ws = _ws(ws)
    wptr, wbytes = ws.get(lib.lsrvt_cvt_workspace(dims, sites.numel(), 0))
    code = lib.lsrvt_update(_ptr(cell), dims, _ptr(weights), _ptr(sites), sites.numel(), _ptr(ds), wptr, wbytes,
                            _stream(stream))
    _check(code, "lsrvt_update")
    return sites, ds


UPDATE_NOALLOC_MAX_SITES = 1 << 18


def lsrvt_update_noalloc(cell, sites, weights=None, ds=None, stream=None):
    """lsrvt_update without a workspace (the library's fixed per-GPU scratch;
    at most UPDATE_NOALLOC_MAX_SITES sites).  ``ds`` must be given by callers
    that cannot allocate; returns (sites, ds)."""
    torch = _torch()
    _need(cell, torch.int32, "lsrvt_update_noalloc")
    _need(sites, torch.int32, "lsrvt_update_noalloc")
    if weights is not None:
        _need(weights, torch.int16, "lsrvt_update_noalloc")
    lib = _lib()
    dims = _dims(cell.shape)
    if ds is None:
        ds = torch.empty(sites.numel(), dtype=torch.float64, device=cell.device)
    code = lib.lsrvt_update_noalloc(_ptr(cell), dims, _ptr(weights), _ptr(sites), sites.numel(), _ptr(ds),
                                    _stream(stream))
    _check(code, "lsrvt_update_noalloc")
    return sites, ds


@dataclass
class CVT:
    cell: "object"
    sites: "object"
    site_comp: "object"
    mean_ds: np.ndarray


def lsrvt_cvt(band, comp, seeds, weights=None, iters: int = 0, cell=None, sites=None, site_comp=None,
              ws: Workspace | None = None, stream=None, want_mean_ds: bool = True) -> CVT:
    """Algorithm 1 with ``iters`` snapped centroid updates and a final pass."""
    torch = _torch()
    _need(band, torch.uint8, "lsrvt_cvt")
    _need(comp, torch.int32, "lsrvt_cvt")
    _need(seeds, torch.int32, "lsrvt_cvt")
    if weights is not None:
        _need(weights, torch.int16, "lsrvt_cvt")
    lib = _lib()
    dims = _dims(band.shape)
    dev = band.device
    S = seeds.numel()
    if cell is None:
        cell = torch.empty(band.shape, dtype=torch.int32, device=dev)
    if sites is None:
        sites = torch.empty(S, dtype=torch.int32, device=dev)
    if site_comp is None:
        site_comp = torch.empty(S, dtype=torch.int32, device=dev)
    mds = np.zeros(max(int(iters), 1), dtype=np.float64)
    ws = _ws(ws)
    wptr, wbytes = ws.get(lib.lsrvt_cvt_workspace(dims, S, max(int(iters), 0)))
    code = lib.lsrvt_cvt(_ptr(band), _ptr(comp), dims, _ptr(seeds), S, _ptr(weights), int(iters), _ptr(cell),
                         _ptr(sites), _ptr(site_comp),
                         mds.ctypes.data_as(ctypes.c_void_p) if want_mean_ds else None, wptr, wbytes,
                         _stream(stream))
    _check(code, "lsrvt_cvt")
    return CVT(cell, sites, site_comp, mds[:max(int(iters), 0)])


@dataclass
class LevelStats:
    n: "object"
    mean: "object"
    m2: "object"
    vmin: "object"
    vmax: "object"
    hist: "object"
    cov: "object"


def _alloc_level(U, m, B, hist, cov, fdt, dev):
    torch = _torch()
    P = m * (m + 1) // 2
    return LevelStats(
        torch.empty(U, dtype=torch.int64, device=dev),
        torch.empty((U, m), dtype=fdt, device=dev),
        torch.empty((U, m), dtype=fdt, device=dev),
        torch.empty((U, m), dtype=torch.float32, device=dev),
        torch.empty((U, m), dtype=torch.float32, device=dev),
        torch.empty((U, m, B), dtype=torch.int32, device=dev) if hist else None,
        torch.empty((U, P), dtype=fdt, device=dev) if cov else None,
    )


def _cstruct(cls, L):
    return cls(*(None if getattr(L, k) is None else getattr(L, k).data_ptr()
                 for k in ("n", "mean", "m2", "vmin", "vmax", "hist", "cov")))


def lsrvt_aggregate(cell, sites, site_comp, comp_band, n_comp: int, n_bands: int, variables, edges=None,
                    cov: bool = False, ws: Workspace | None = None, stream=None, out=None):
    """Per-cell FP32 compensated statistics merged (FP64, Chan) to components and bands.

    Returns (cell_stats, comp_stats, band_stats) as :class:`LevelStats`."""
    torch = _torch()
    _need(cell, torch.int32, "lsrvt_aggregate")
    _need(sites, torch.int32, "lsrvt_aggregate")
    _need(site_comp, torch.int32, "lsrvt_aggregate")
    _need(comp_band, torch.uint8, "lsrvt_aggregate")
    _need(variables, torch.float32, "lsrvt_aggregate")
    if edges is not None:
        _need(edges, torch.float32, "lsrvt_aggregate")
    lib = _lib()
    dims = _dims(cell.shape)
    dev = cell.device
    m = int(variables.shape[0])
    B = 0 if edges is None else int(edges.shape[1]) - 1
    flags = (STATS_HIST if edges is not None else 0) | (STATS_COV if cov else 0)
    S = sites.numel()
    if out is None:
        out = (_alloc_level(S, m, B, edges is not None, cov, torch.float32, dev),
               _alloc_level(n_comp, m, B, edges is not None, cov, torch.float64, dev),
               _alloc_level(n_bands, m, B, edges is not None, cov, torch.float64, dev))
    cs, gs, bs = out
    c_cell, c_comp, c_band = _cstruct(CellStatsC, cs), _cstruct(GroupStatsC, gs), _cstruct(GroupStatsC, bs)
    ws = _ws(ws)
    wptr, wbytes = ws.get(lib.lsrvt_aggregate_workspace(dims, S, n_comp, n_bands, m, B, flags))
    code = lib.lsrvt_aggregate(_ptr(cell), dims, _ptr(sites), _ptr(site_comp), S, _ptr(comp_band), n_comp, n_bands,
                               _ptr(variables), m, _ptr(edges), B, flags, ctypes.byref(c_cell), ctypes.byref(c_comp),
                               ctypes.byref(c_band), wptr, wbytes, _stream(stream))
    _check(code, "lsrvt_aggregate")
    return out


def lsrvt_components_workspace_bytes(shape, n_bands: int) -> int:
    """Workspace bytes of lsrvt_components for a volume of `shape` (nz, ny, nx)."""
    return int(_lib().lsrvt_components_workspace(_dims(shape), int(n_bands)))


def lsrvt_cvt_workspace_bytes(shape, n_sites: int, iters: int) -> int:
    """Workspace bytes of lsrvt_cvt for a volume of `shape` (nz, ny, nx)."""
    return int(_lib().lsrvt_cvt_workspace(_dims(shape), int(n_sites), max(int(iters), 0)))


def lsrvt_aggregate_workspace_bytes(shape, n_sites: int, n_comp: int, n_bands: int, n_vars: int, n_bins: int,
                                    cov: bool) -> int:
    """Workspace bytes of lsrvt_aggregate."""
    flags = (STATS_HIST if n_bins else 0) | (STATS_COV if cov else 0)
    return int(_lib().lsrvt_aggregate_workspace(_dims(shape), int(n_sites), int(n_comp), int(n_bands), int(n_vars),
                                                int(n_bins), flags))


@dataclass
class BatchJob:
    """One job of lsrvt_batch_run: its inputs (device tensors, host isovalues) and, after the call, its
    outputs (labels, tables, statistics) as tensors."""
    field: "object"
    iso: "object"
    seeds: "object"
    weights: "object"
    iters: int
    variables: "object"
    edges: "object" = None
    cov: bool = False
    cap_comp: int = 0
    band: "object" = None
    comp: "object" = None
    comp_band: "object" = None
    comp_size: "object" = None
    comp_first: "object" = None
    band_offset: "object" = None
    cell: "object" = None
    sites: "object" = None
    site_comp: "object" = None
    stats: "object" = None  # (cell, comp, band) LevelStats
    n_comp: int = 0
    status: int = -1


def _job_struct(j: BatchJob, keep: list) -> JobC:
    torch = _torch()
    _need(j.field, torch.float32, "lsrvt_batch_run")
    _need(j.seeds, torch.int32, "lsrvt_batch_run")
    _need(j.variables, torch.float32, "lsrvt_batch_run")
    dev = j.field.device
    shape = tuple(j.field.shape)
    n = j.field.numel()
    iso = np.ascontiguousarray(np.asarray(j.iso, dtype=np.float32))
    keep.append(iso)
    K = len(iso)
    nb = K + 1
    S = j.seeds.numel()
    m = int(j.variables.shape[0])
    B = 0 if j.edges is None else int(j.edges.shape[1]) - 1
    cap = int(j.cap_comp) if j.cap_comp else max(1024, n // 16)
    j.cap_comp = cap
    j.band = torch.empty(shape, dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    j.comp = torch.empty(shape, dtype=torch.int32, device=dev)
    j.comp_band = torch.empty(cap, dtype=torch.uint8, device=dev)
    j.comp_size = torch.empty(cap, dtype=torch.int64, device=dev)
    j.comp_first = torch.empty(cap, dtype=torch.int32, device=dev)
    j.band_offset = torch.empty(nb + 1, dtype=torch.int32, device=dev)
    j.cell = torch.empty(shape, dtype=torch.int32, device=dev)
    j.sites = torch.empty(max(S, 1), dtype=torch.int32, device=dev)
    j.site_comp = torch.empty(max(S, 1), dtype=torch.int32, device=dev)
    hist = j.edges is not None
    j.stats = (_alloc_level(S, m, B, hist, j.cov, torch.float32, dev),
               _alloc_level(cap, m, B, hist, j.cov, torch.float64, dev),
               _alloc_level(nb, m, B, hist, j.cov, torch.float64, dev))
    keep.append(status)
    c = JobC()
    c.dims = _dims(shape)
    c.d_field = j.field.data_ptr()
    c.h_iso = iso.ctypes.data
    c.n_iso = K
    c.d_seeds = j.seeds.data_ptr() if S else None
    c.n_sites = S
    c.d_weights = None if j.weights is None else j.weights.data_ptr()
    c.iters = int(j.iters)
    c.d_vars = j.variables.data_ptr()
    c.n_vars = m
    c.d_edges = None if j.edges is None else j.edges.data_ptr()
    c.n_bins = B
    c.flags = (STATS_HIST if hist else 0) | (STATS_COV if j.cov else 0)
    c.cap_comp = cap
    for k, t in (("d_band", j.band), ("d_status", status), ("d_comp", j.comp), ("d_comp_band", j.comp_band),
                 ("d_comp_size", j.comp_size), ("d_comp_first", j.comp_first), ("d_band_offset", j.band_offset),
                 ("d_cell", j.cell), ("d_sites", j.sites), ("d_site_comp", j.site_comp)):
        setattr(c, k, t.data_ptr())
    c.cell = _cstruct(CellStatsC, j.stats[0])
    c.comp = _cstruct(GroupStatsC, j.stats[1])
    c.band = _cstruct(GroupStatsC, j.stats[2])
    return c


def lsrvt_batch_run(jobs, n_streams: int = 4, ws: Workspace | None = None, stream=None):
    """Run every job's whole path (isobands, components, Lloyd loop, statistics) on up to n_streams streams.

    Fills each job's outputs; raises if a job fails.  Synchronises."""
    lib = _lib()
    keep = []
    arr = (JobC * max(len(jobs), 1))()
    for i, j in enumerate(jobs):
        arr[i] = _job_struct(j, keep)
    nbytes = lib.lsrvt_batch_workspace(arr, len(jobs), int(n_streams))
    if len(jobs) and nbytes == 0:
        raise LsrvtError(EINVAL, "lsrvt_batch_workspace", "a job has invalid sizes")
    ws = _ws(ws)
    wptr, wbytes = ws.get(nbytes)
    code = lib.lsrvt_batch_run(arr, len(jobs), int(n_streams), wptr, wbytes, _stream(stream))
    for i, j in enumerate(jobs):
        j.status = int(arr[i].status)
        j.n_comp = int(arr[i].n_comp)
    _check(code, "lsrvt_batch_run")
    return jobs


@dataclass
class Layout:
    perm: "object"        # int32[n_placed] voxel linear indices in layout order
    site_order: "object"  # int32[S] site of the k-th cell
    cell_off: "object"    # int32[S + 1]
    comp_off: "object"    # int32[n_comp + 1]
    band_off: "object"    # int32[n_bands + 1]
    n_placed: int


def lsrvt_layout(cell, site_comp, comp_band, n_comp: int, n_bands: int, ws: Workspace | None = None,
                 stream=None) -> Layout:
    """Structured hierarchical layout: placed voxels sorted by (band, component, cell, index)."""
    torch = _torch()
    _need(cell, torch.int32, "lsrvt_layout")
    _need(site_comp, torch.int32, "lsrvt_layout")
    _need(comp_band, torch.uint8, "lsrvt_layout")
    lib = _lib()
    dims = _dims(cell.shape)
    dev = cell.device
    S = site_comp.numel()
    perm = torch.empty(cell.numel(), dtype=torch.int32, device=dev)
    order = torch.empty(max(S, 1), dtype=torch.int32, device=dev)
    cell_off = torch.empty(S + 1, dtype=torch.int32, device=dev)
    comp_off = torch.empty(n_comp + 1, dtype=torch.int32, device=dev)
    band_off = torch.empty(n_bands + 1, dtype=torch.int32, device=dev)
    placed = ctypes.c_uint32()
    ws = _ws(ws)
    wptr, wbytes = ws.get(lib.lsrvt_layout_workspace(dims, S, n_comp))
    code = lib.lsrvt_layout(_ptr(cell), dims, _ptr(site_comp), S, _ptr(comp_band), n_comp, n_bands, _ptr(perm),
                            _ptr(order), _ptr(cell_off), _ptr(comp_off), _ptr(band_off), ctypes.byref(placed), wptr,
                            wbytes, _stream(stream))
    _check(code, "lsrvt_layout")
    return Layout(perm[:placed.value], order[:S], cell_off, comp_off, band_off, int(placed.value))


def lsrvt_extract(variables, perm, out=None, stream=None):
    """Raw variables in layout order: out[j][k] = variables[j].flat[perm[k]]."""
    torch = _torch()
    _need(variables, torch.float32, "lsrvt_extract")
    _need(perm, torch.int32, "lsrvt_extract")
    m = int(variables.shape[0])
    dims = _dims(variables.shape[1:])
    k = perm.numel()
    if out is None:
        out = torch.empty((m, k), dtype=torch.float32, device=variables.device)
    _check(_lib().lsrvt_extract(_ptr(variables), m, dims, _ptr(perm), k, _ptr(out), _stream(stream)), "lsrvt_extract")
    return out


VT_AUTO, VT_LEVELS, VT_BRICKS = 0, 1, 2


def lsrvt_set_vt_engine(engine: int) -> int:
    """Schedule of the Voronoi passes for calls from this host thread
    (VT_AUTO, VT_LEVELS or VT_BRICKS; same regions either way); returns the
    previous setting."""
    prev = int(_lib().lsrvt_set_vt_engine(int(engine)))
    if prev < 0:
        raise LsrvtError(EINVAL, "lsrvt_set_vt_engine", f"unknown engine {engine}")
    return prev


TUNE_BR_GRID, TUNE_STATS_TILE, TUNE_KEY_BITS, TUNE_RESET = 1, 2, 3, 4


def lsrvt_set_tuning(knob: int, value: int) -> int:
    """Launch shape of this host thread's later calls (TUNE_BR_GRID:
    workgroups per relaxation round, 256..16384; TUNE_STATS_TILE: voxels per
    thread and staging round of the statistics, 1, 2 or 4; TUNE_KEY_BITS: key
    width of the brick relaxation, 64 = wide keys, 1..30 = narrow keys with at
    least that many id bits; TUNE_RESET: 1 = the reset of an incremental
    relaxation pass by its own kernel, 2 = fused into the first round; 0 = the
    library's choice); returns the previous value."""
    prev = int(_lib().lsrvt_set_tuning(int(knob), int(value)))
    if prev < 0:
        raise LsrvtError(EINVAL, "lsrvt_set_tuning", f"knob {knob} value {value}")
    return prev


def lsrvt_timing_enable(enable: bool = True) -> None:
    """Bracket every batch of the Voronoi passes' dominant launches (levels or
    relaxation rounds) with a hipEvent pair (benchmarks)."""
    _check(_lib().lsrvt_timing_enable(1 if enable else 0), "lsrvt_timing_enable")


def lsrvt_timing_read():
    """(kernel ms, launches, passes, voxels per pass, engines) since the
    previous read; engines has bit 0 set when level passes ran, bit 1 when
    relaxation passes ran."""
    ms, la, pa, vx, en = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int64(), ctypes.c_int32()
    _check(_lib().lsrvt_timing_read(ctypes.byref(ms), ctypes.byref(la), ctypes.byref(pa), ctypes.byref(vx),
                                    ctypes.byref(en)), "lsrvt_timing_read")
    return ms.value, la.value, pa.value, vx.value, en.value


def lsrvt_seed(comp, comp_first, n_comp: int, weights=None, mass_lut=None, rho: int = 4096, block: int = 16,
               seed: int = 0, cap_pairs: int | None = None, cap_sites: int | None = None, ws: Workspace | None = None,
               stream=None):
    """Stratified initial sites (Sec. 3.2.1, Eq. 3 and Eq. 4): int32 tensor of linear indices (uint32 bits)."""
    torch = _torch()
    _need(comp, torch.int32, "lsrvt_seed")
    _need(comp_first, torch.int32, "lsrvt_seed")
    if weights is not None:
        _need(weights, torch.int16, "lsrvt_seed")
    if mass_lut is not None:
        _need(mass_lut, torch.int32, "lsrvt_seed")
        if mass_lut.numel() != 65536:
            raise LsrvtError(EINVAL, "lsrvt_seed", "the mass table has one entry per weight value (65536)")
    lib = _lib()
    dims = _dims(comp.shape)
    dev = comp.device
    n = comp.numel()
    nb = -(-comp.shape[2] // block) * -(-comp.shape[1] // block) * -(-comp.shape[0] // block)
    cap_p = int(cap_pairs) if cap_pairs is not None else min(n, 4 * nb + 2 * int(n_comp))
    cap_s = int(cap_sites) if cap_sites is not None else max(1024, n // max(int(rho), 1) + 2 * int(n_comp))
    ws = _ws(ws)
    n_sites = ctypes.c_uint32(0)
    n_pairs = ctypes.c_uint32(0)
    while True:
        wptr, wbytes = ws.get(lib.lsrvt_seed_workspace(dims, int(n_comp), int(block), cap_p))
        sites = torch.empty(cap_s, dtype=torch.int32, device=dev)
        code = lib.lsrvt_seed(_ptr(comp), _ptr(comp_first), dims, int(n_comp), _ptr(weights), _ptr(mass_lut),
                              int(rho), int(block), int(seed) & 0xFFFFFFFFFFFFFFFF, cap_p, _ptr(sites), cap_s,
                              ctypes.byref(n_sites), ctypes.byref(n_pairs), wptr, wbytes, _stream(stream))
        if code == ECAPACITY:
            cap_p = max(cap_p, int(n_pairs.value))
            cap_s = max(cap_s, int(n_sites.value))
            continue
        _check(code, "lsrvt_seed")
        break
    return sites[:int(n_sites.value)]


@dataclass
class Moments:
    """Joint moments of a set of units (device tensors, float64)."""
    n: "object"      # int64 [U] (uint64 counts)
    mean: "object"   # [U, m]
    m2: "object"     # [U, m(m+1)/2]
    m3: "object"     # [U, m(m+1)(m+2)/6]
    m4: "object"     # [U, m(m+1)(m+2)(m+3)/24]


def _moments(U, m, dev):
    torch = _torch()
    P2, P3, P4 = m * (m + 1) // 2, m * (m + 1) * (m + 2) // 6, m * (m + 1) * (m + 2) * (m + 3) // 24
    f = lambda k: torch.empty((max(U, 1), k), dtype=torch.float64, device=dev)
    mo = Moments(torch.empty(max(U, 1), dtype=torch.int64, device=dev), f(m), f(P2), f(P3), f(P4))
    c = MomentsC(*(ctypes.c_void_p(t.data_ptr()) for t in (mo.n, mo.mean, mo.m2, mo.m3, mo.m4)))
    return mo, c


def lsrvt_comoments(cell, sites, site_comp, comp_band, n_comp: int, n_bands: int, variables,
                    ws: Workspace | None = None, stream=None):
    """Joint moments up to fourth order per cell, component and band (Sec. 4.4)."""
    torch = _torch()
    _need(cell, torch.int32, "lsrvt_comoments")
    _need(variables, torch.float32, "lsrvt_comoments")
    lib = _lib()
    dims = _dims(cell.shape)
    m = int(variables.shape[0])
    S = int(sites.numel())
    dev = cell.device
    cm, cc = _moments(S, m, dev)
    gm, gc = _moments(int(n_comp), m, dev)
    bm, bc = _moments(int(n_bands), m, dev)
    ws = _ws(ws)
    wptr, wbytes = ws.get(lib.lsrvt_comoments_workspace(dims, S, int(n_comp), int(n_bands), m))
    code = lib.lsrvt_comoments(_ptr(cell), dims, _ptr(sites), _ptr(site_comp), S, _ptr(comp_band), int(n_comp),
                               int(n_bands), _ptr(variables), m, ctypes.byref(cc), ctypes.byref(gc),
                               ctypes.byref(bc), wptr, wbytes, _stream(stream))
    _check(code, "lsrvt_comoments")
    trim = lambda mo, U: Moments(mo.n[:U], mo.mean[:U], mo.m2[:U], mo.m3[:U], mo.m4[:U])
    return trim(cm, S), trim(gm, int(n_comp)), trim(bm, int(n_bands))



# --------------------------------------------------------------------------
# Euclidean line-of-sight tessellation (Sec. 3.2.2) and site update (Eq. 2,
# Sec. 3.2.3)
LOS_SITE = 0x80000000


@dataclass
class LosVT:
    dist: "object"   # float64 [nz, ny, nx]
    src: "object"    # int32 (uint32 bits) [nz, ny, nx]: voxel, LOS_SITE | s, or NONE
    phi: "object"    # int32 (uint32 bits) [nz, ny, nx]
    cell: "object"   # int32 (uint32 bits) [nz, ny, nx]
    sweeps: tuple    # sweeps of stage 1 and stage 2 (lsrvt_los_vt) or total (lsrvt_los_cvt)


def _los_out(comp):
    torch = _torch()
    e = lambda dt: torch.empty(comp.shape, dtype=dt, device=comp.device)
    return e(torch.float64), e(torch.int32), e(torch.int32), e(torch.int32)


def lsrvt_los_vt(comp, site_q, anchor, ws: Workspace | None = None, stream=None) -> LosVT:
    """Restricted Voronoi regions with Euclidean line-of-sight paths.  site_q
    int32 [S, 3] in 1/256 voxel (x, y, z), anchor int32 [S] voxel indices."""
    torch = _torch()
    _need(comp, torch.int32, "lsrvt_los_vt")
    _need(site_q, torch.int32, "lsrvt_los_vt")
    _need(anchor, torch.int32, "lsrvt_los_vt")
    S = int(anchor.numel())
    if site_q.numel() != 3 * S:
        raise LsrvtError(EINVAL, "lsrvt_los_vt", "site_q must be [S, 3]")
    lib = _lib()
    dims = _dims(comp.shape)
    dist, src, phi, cell = _los_out(comp)
    ws = _ws(ws)
    wptr, wbytes = ws.get(lib.lsrvt_los_workspace(dims, S))
    sw = (ctypes.c_int32 * 2)()
    code = lib.lsrvt_los_vt(_ptr(comp), dims, _ptr(site_q), _ptr(anchor), S, _ptr(dist), _ptr(src), _ptr(phi),
                            _ptr(cell), sw, wptr, wbytes, _stream(stream))
    _check(code, "lsrvt_los_vt")
    return LosVT(dist, src, phi, cell, (int(sw[0]), int(sw[1])))


def lsrvt_los_update(comp, cell, phi, site_q, anchor, weights=None, ws: Workspace | None = None, stream=None):
    """Eq. 2 target with masses carried to line-of-sight voxels, then the
    ray-clamped move; site_q and anchor are updated in place.  Returns the
    targets, int32 [S, 3] (INT32_MIN rows for empty cells)."""
    torch = _torch()
    for t, dt in ((comp, torch.int32), (cell, torch.int32), (phi, torch.int32), (site_q, torch.int32),
                  (anchor, torch.int32)):
        _need(t, dt, "lsrvt_los_update")
    if weights is not None:
        _need(weights, torch.int16, "lsrvt_los_update")
    S = int(anchor.numel())
    lib = _lib()
    dims = _dims(comp.shape)
    target = torch.empty((max(S, 1), 3), dtype=torch.int32, device=comp.device)
    ws = _ws(ws)
    wptr, wbytes = ws.get(lib.lsrvt_los_workspace(dims, S))
    code = lib.lsrvt_los_update(_ptr(comp), dims, _ptr(weights), _ptr(cell), _ptr(phi), S, _ptr(site_q),
                                _ptr(anchor), _ptr(target), wptr, wbytes, _stream(stream))
    _check(code, "lsrvt_los_update")
    return target[:S]


@dataclass
class LosCVT:
    site_q: "object"  # int32 [S, 3]
    anchor: "object"  # int32 [S]
    vt: LosVT


def lsrvt_los_cvt(comp, seeds, weights=None, iters: int = 0, ws: Workspace | None = None, stream=None) -> LosCVT:
    """Lloyd loop with the line-of-sight tessellation: sites start at the
    centres of the seed voxels; iters x (VT + update), then a final VT."""
    torch = _torch()
    _need(comp, torch.int32, "lsrvt_los_cvt")
    _need(seeds, torch.int32, "lsrvt_los_cvt")
    if weights is not None:
        _need(weights, torch.int16, "lsrvt_los_cvt")
    S = int(seeds.numel())
    lib = _lib()
    dims = _dims(comp.shape)
    dev = comp.device
    site_q = torch.empty((max(S, 1), 3), dtype=torch.int32, device=dev)
    anchor = torch.empty(max(S, 1), dtype=torch.int32, device=dev)
    dist, src, phi, cell = _los_out(comp)
    ws = _ws(ws)
    wptr, wbytes = ws.get(lib.lsrvt_los_workspace(dims, S))
    sw = ctypes.c_int32(0)
    code = lib.lsrvt_los_cvt(_ptr(comp), dims, _ptr(seeds), S, _ptr(weights), int(iters), _ptr(site_q),
                             _ptr(anchor), _ptr(dist), _ptr(src), _ptr(phi), _ptr(cell), ctypes.byref(sw), wptr,
                             wbytes, _stream(stream))
    _check(code, "lsrvt_los_cvt")
    return LosCVT(site_q[:S], anchor[:S], LosVT(dist, src, phi, cell, (int(sw.value),)))
