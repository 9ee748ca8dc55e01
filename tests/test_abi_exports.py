"""The C-ABI library loads and exports every entry point declared in
include/lsrvt.h; host-side validation runs without a GPU."""
import ctypes
import os
import re

import pytest

import paper_2208_06970_amd as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsrvt.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lsrvt_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2208_06970_amd import build
        build.build()
    return L.library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def test_status_strings_and_version(lib):
    assert lib.lsrvt_status_string(0) == b"ok"
    assert b"NaN" in lib.lsrvt_status_string(2)
    assert lib.lsrvt_status_string(99) == b"unknown status"
    assert lib.lsrvt_version() >= 100


def test_host_validation_without_gpu(lib):
    bad = L.Dims(0, 4, 4)
    huge = L.Dims(32768, 1, 1)
    big = L.Dims(32767, 32767, 4)
    nul = ctypes.c_void_p(0)
    iso = (ctypes.c_float * 2)(1.0, 1.0)
    fake = ctypes.c_void_p(4096)
    assert lib.lsrvt_isobands(fake, bad, iso, 1, fake, nul, nul) == L.EINVAL
    assert lib.lsrvt_isobands(fake, huge, iso, 1, fake, nul, nul) == L.ELIMIT
    assert lib.lsrvt_isobands(fake, big, iso, 1, fake, nul, nul) == L.ELIMIT
    assert lib.lsrvt_isobands(fake, L.Dims(4, 4, 4), iso, 2, fake, nul, nul) == L.EINVAL  # not increasing
    assert lib.lsrvt_isobands(fake, L.Dims(4, 4, 4), iso, 255, fake, nul, nul) == L.EINVAL
    d = L.Dims(64, 64, 64)
    assert lib.lsrvt_components_workspace(d, 5) > 64 ** 3 * 4
    assert lib.lsrvt_cvt_workspace(d, 1000, 10) > 0
    assert lib.lsrvt_aggregate_workspace(d, 1000, 100, 5, 3, 16, 3) > 0
    # a workspace that is too small is refused before any launch
    assert lib.lsrvt_components(fake, d, 5, fake, 10, fake, fake, fake, fake, ctypes.byref(ctypes.c_uint32()),
                                fake, 16, nul) == L.EWORKSPACE
    assert lib.lsrvt_cvt(fake, fake, d, fake, 10, nul, -1, fake, fake, fake, nul, fake, 1 << 30, nul) == L.EINVAL
    assert lib.lsrvt_vt(fake, d, fake, 10, fake, fake, 16, nul) == L.EWORKSPACE


def test_seed_host_validation_without_gpu(lib):
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(4096)
    d = L.Dims(64, 64, 64)
    ns, npairs = ctypes.c_uint32(7), ctypes.c_uint32(7)
    assert lib.lsrvt_seed_workspace(d, 100, 16, 1000) > 0
    assert lib.lsrvt_seed_workspace(d, 100, 17, 1000) == 0   # block edge above 16
    assert lib.lsrvt_seed_workspace(d, 100, 16, 0) == 0
    args = lambda **k: [k.get("comp", fake), k.get("first", fake), d, k.get("n_comp", 100), k.get("w", nul),
                        k.get("lut", nul), k.get("rho", 64), k.get("block", 8), 1, k.get("cap", 1000), fake, 10,
                        ctypes.byref(ns), ctypes.byref(npairs), fake, k.get("wb", 16), nul]
    assert lib.lsrvt_seed(*args(rho=0)) == L.EINVAL
    assert lib.lsrvt_seed(*args(first=nul)) == L.EINVAL
    assert lib.lsrvt_seed(*args(lut=fake)) == L.EINVAL          # a mass table needs weights
    assert lib.lsrvt_seed(*args(block=0)) == L.EINVAL
    assert lib.lsrvt_seed(*args(n_comp=0)) == L.EINVAL
    assert lib.lsrvt_seed(*args()) == L.EWORKSPACE              # 16 bytes of workspace
    assert ns.value == 0 and npairs.value == 0


def test_comoments_host_validation_without_gpu(lib):
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(4096)
    d = L.Dims(32, 32, 32)
    assert lib.lsrvt_comoments_workspace(d, 100, 10, 3, 18) > 0
    assert lib.lsrvt_comoments_workspace(d, 100, 10, 3, 19) == 0   # at most 18 variables
    mo = L.MomentsC(fake, fake, fake, fake, fake)
    bad = L.MomentsC(fake, nul, fake, fake, fake)
    call = lambda m, a, b, c, wb=16: lib.lsrvt_comoments(fake, d, fake, fake, 100, fake, 10, 3, fake, m,
                                                        ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), fake, wb,
                                                        nul)
    assert call(0, mo, mo, mo) == L.EINVAL
    assert call(19, mo, mo, mo) == L.EINVAL
    assert call(4, mo, bad, mo) == L.EINVAL
    assert call(4, mo, mo, mo) == L.EWORKSPACE


def test_los_host_validation_without_gpu(lib):
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(4096)
    d = L.Dims(32, 32, 32)
    assert lib.lsrvt_los_workspace(d, 100) > 32 ** 3 * 14
    assert lib.lsrvt_los_workspace(d, 1 << 31) == 0            # site ids must leave the LOS flag bit free
    assert lib.lsrvt_los_workspace(L.Dims(0, 1, 1), 10) == 0
    sw = (ctypes.c_int32 * 2)()
    vt = lambda q, out, S=10, wb=16: lib.lsrvt_los_vt(fake, d, q, fake, S, out, fake, fake, fake, sw, fake, wb, nul)
    assert vt(fake, nul) == L.EINVAL                             # no distance output
    assert vt(nul, fake) == L.EINVAL                             # sites without positions
    assert vt(fake, fake, S=1 << 31) == L.ELIMIT
    assert vt(fake, fake) == L.EWORKSPACE
    assert lib.lsrvt_los_update(fake, d, nul, fake, nul, 10, fake, fake, nul, fake, 16, nul) == L.EINVAL
    assert lib.lsrvt_los_update(fake, d, nul, fake, fake, 10, fake, fake, nul, fake, 16, nul) == L.EWORKSPACE
    cvt = lambda iters, wb=16: lib.lsrvt_los_cvt(fake, d, fake, 10, nul, iters, fake, fake, fake, fake, fake, fake,
                                                 nul, fake, wb, nul)
    assert cvt(-1) == L.EINVAL
    assert cvt(2) == L.EWORKSPACE


def test_set_tuning_validation_without_gpu(lib):
    """Launch-shape knobs: unknown knobs and out-of-range values are refused
    and change nothing; a valid value returns the previous one."""
    assert lib.lsrvt_set_tuning(0, 1) == -1
    assert lib.lsrvt_set_tuning(99, 1) == -1
    assert lib.lsrvt_set_tuning(L.TUNE_BR_GRID, 100) == -1
    assert lib.lsrvt_set_tuning(L.TUNE_BR_GRID, 1 << 20) == -1
    assert lib.lsrvt_set_tuning(L.TUNE_STATS_TILE, 3) == -1
    assert lib.lsrvt_set_tuning(L.TUNE_BR_GRID, 4096) == 0
    assert lib.lsrvt_set_tuning(L.TUNE_BR_GRID, 0) == 4096
    assert lib.lsrvt_set_tuning(L.TUNE_STATS_TILE, 2) == 0
    assert lib.lsrvt_set_tuning(L.TUNE_STATS_TILE, 0) == 2
    assert lib.lsrvt_set_tuning(L.TUNE_KEY_BITS, 31) == -1
    assert lib.lsrvt_set_tuning(L.TUNE_KEY_BITS, 32) == -1
    assert lib.lsrvt_set_tuning(L.TUNE_KEY_BITS, -1) == -1
    assert lib.lsrvt_set_tuning(L.TUNE_KEY_BITS, 64) == 0
    assert lib.lsrvt_set_tuning(L.TUNE_KEY_BITS, 30) == 64
    assert lib.lsrvt_set_tuning(L.TUNE_KEY_BITS, 0) == 30
    assert lib.lsrvt_set_tuning(L.TUNE_RESET, 3) == -1
    assert lib.lsrvt_set_tuning(L.TUNE_RESET, 2) == 0
    assert lib.lsrvt_set_tuning(L.TUNE_RESET, 0) == 2
    assert lib.lsrvt_set_tuning(5, 0) == -1
