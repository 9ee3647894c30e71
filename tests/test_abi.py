"""The C-ABI library loads, exports every symbol include/gsf.h declares, and
its host-side validation returns the documented codes (no GPU needed: every
call here fails validation before anything is enqueued)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsf.h")

torch = pytest.importorskip("torch")
from paper_1507_04941_amd import binding as B  # noqa: E402


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIB_PATH):
        from paper_1507_04941_amd import build
        build.build()
    return B.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(L, n), n
    bound = {s[0] for s in B.SIGNATURES}
    assert set(names) == bound


def test_status_strings(L):
    for s in range(6):
        assert L.gsf_status_string(s)
    assert L.gsf_status_string(99) == b"unknown status"
    assert L.gsf_version().startswith(b"gsf")


def test_mask_words(L):
    assert L.gsf_mask_words(B.Dims(2, 3, 64)) == 6
    assert L.gsf_mask_words(B.Dims(2, 3, 65)) == 12
    assert L.gsf_mask_words(B.Dims(1, 1, 1)) == 1
    assert L.gsf_mask_words(B.Dims(0, 3, 65)) == -1


def _ws_filter(dims, f):
    n = ctypes.c_size_t(0)
    st = B.lib().gsf_filter3d_workspace_size(dims, ctypes.byref(f), ctypes.byref(n))
    return st, n.value


def test_workspace_sizes(L):
    st, n = _ws_filter(B.Dims(512, 512, 1024), B.Filter(4.0, 8.0, 3.0))
    assert st == 0 and n >= 512 * 512 * 1024 * 4
    n2 = ctypes.c_size_t(0)
    assert L.gsf_local_stats_workspace_size(B.Dims(64, 64, 128), B.Box(32, 32, 32),
                                            ctypes.byref(n2)) == 0
    # the fast statistics path: two FP32 cubes of window-sum pairs + shift partials
    assert 2 * 64 * 64 * 128 * 4 <= n2.value < 3 * 64 * 64 * 128 * 4
    n4 = ctypes.c_size_t(0)
    assert L.gsf_local_stats_workspace_size(B.Dims(64, 64, 128), B.Box(12, 32, 32),
                                            ctypes.byref(n4)) == 0
    assert n4.value - n2.value == 2 * 64 * 64 * 128 * 4     # generic path: four cubes
    cubes = (B.Cube * 2)()
    cubes[0].data = 256
    cubes[0].dims = B.Dims(64, 64, 128)
    cubes[1].data = 256
    cubes[1].dims = B.Dims(100, 10, 300)
    filt = (B.Filter * 2)(B.Filter(1, 1, 3), B.Filter(2, 4, 3))
    n3 = ctypes.c_size_t(0)
    assert L.gsf_find_workspace_size(cubes, 2, filt, 2, B.Box(8, 8, 8), ctypes.byref(n3)) == 0
    assert n3.value >= 5 * 100 * 10 * 300 * 4


def _find_ws(L, dims, ncubes):
    cubes = (B.Cube * ncubes)()
    for c in cubes:
        c.data = 256
        c.dims = dims
    filt = (B.Filter * 1)(B.Filter(1, 1, 3))
    n = ctypes.c_size_t(0)
    assert L.gsf_find_workspace_size(cubes, ncubes, filt, 1, B.Box(8, 8, 8), ctypes.byref(n)) == 0
    return n.value


def test_find_workspace_slots(L):
    # one workspace slot per concurrently processed cube, at most 32 of them
    small = B.Dims(64, 64, 128)
    one = _find_ws(L, small, 1)
    assert _find_ws(L, small, 5) == 5 * one
    assert _find_ws(L, small, 32) == 32 * one
    assert _find_ws(L, small, 40) == 32 * one
    # and no more slots than fit 64 GiB (at least one)
    big = B.Dims(1024, 1024, 1024)
    slot = _find_ws(L, big, 1)
    assert _find_ws(L, big, 10) == max(1, (64 << 30) // slot) * slot
    huge = B.Dims(2048, 2048, 2048)
    assert _find_ws(L, huge, 3) == _find_ws(L, huge, 1)


@pytest.mark.parametrize("dims,f,code", [
    (B.Dims(0, 4, 4), B.Filter(1, 1, 3), B.GSF_ERR_INVALID_ARG),
    (B.Dims(4, 4, -1), B.Filter(1, 1, 3), B.GSF_ERR_INVALID_ARG),
    (B.Dims(4, 4, 4), B.Filter(0, 1, 3), B.GSF_ERR_INVALID_ARG),
    (B.Dims(4, 4, 4), B.Filter(1, float("nan"), 3), B.GSF_ERR_INVALID_ARG),
    (B.Dims(4, 4, 4), B.Filter(1, 1, float("inf")), B.GSF_ERR_INVALID_ARG),
    (B.Dims(4, 4, 4), B.Filter(30, 1, 3), B.GSF_ERR_INVALID_ARG),       # radius 90 > 64
    (B.Dims(1 << 20, 1 << 20, 4), B.Filter(1, 1, 3), B.GSF_ERR_INVALID_ARG),
])
def test_filter_validation(L, dims, f, code):
    st, _ = _ws_filter(dims, f)
    assert st == code
    assert L.gsf_last_error()


def test_calls_reject_bad_pointers_before_launch(L):
    d = B.Dims(8, 8, 8)
    f = B.Filter(1, 1, 3)
    # NULL input
    assert L.gsf_filter3d(None, 0, d, ctypes.byref(f), 4096, 0, 8192, 1 << 20, None) == 1
    # misaligned output
    assert L.gsf_filter3d(4096, 0, d, ctypes.byref(f), 4100, 0, 8192, 1 << 20, None) == 1
    # workspace too small
    assert L.gsf_filter3d(4096, 0, d, ctypes.byref(f), 65536, 0, 1 << 20, 16, None) == 3
    # in/out overlap
    assert L.gsf_filter3d(4096, 0, d, ctypes.byref(f), 4096 + 256, 0, 1 << 24, 1 << 20, None) == 1
    # mixed storage types (F16 in, F32 out)
    assert L.gsf_filter3d(4096, 1, d, ctypes.byref(f), 65536, 0, 1 << 20, 1 << 20, None) == 2
    # unknown dtype
    assert L.gsf_filter3d(4096, 7, d, ctypes.byref(f), 65536, 0, 1 << 20, 1 << 20, None) == 1
    # threshold: non-finite k, null mask
    assert L.gsf_threshold(4096, 0, 65536, 131072, d, float("nan"), 1 << 20, None) == 1
    assert L.gsf_threshold(4096, 0, 65536, 131072, d, 4.0, None, None) == 1
    # local stats: both outputs NULL, bad box
    assert L.gsf_local_stats(4096, 0, d, B.Box(4, 4, 4), None, None, 1 << 24, 1 << 24, None) == 1
    assert L.gsf_local_stats(4096, 0, d, B.Box(0, 4, 4), 65536, None, 1 << 24, 1 << 24, None) == 1
    assert L.gsf_local_stats(4096, 0, d, B.Box(4, 4, 5000), 65536, None, 1 << 24, 1 << 24, None) == 1


def test_find_validation(L):
    cubes = (B.Cube * 1)()
    cubes[0].data = 4096
    cubes[0].dims = B.Dims(8, 8, 8)
    filt = (B.Filter * 1)(B.Filter(1, 1, 3))
    masks = (ctypes.c_void_p * 1)(1 << 20)
    box = B.Box(4, 4, 4)
    n = ctypes.c_size_t(0)
    assert L.gsf_find_workspace_size(cubes, 1, filt, 1, box, ctypes.byref(n)) == 0
    need = n.value
    ws = 1 << 30
    assert L.gsf_find(cubes, 0, filt, 1, box, 4.0, masks, None, None, None, ws, need, None) == 1
    assert L.gsf_find(cubes, 1, filt, 0, box, 4.0, masks, None, None, None, ws, need, None) == 1
    assert L.gsf_find(cubes, 1, filt, 1, box, 4.0, None, None, None, None, ws, need, None) == 1
    assert L.gsf_find(cubes, 1, filt, 1, box, 4.0, masks, None, None, None, ws, need - 1, None) == 3
    cubes[0].halo[2] = 4   # 8 - 2*4: no core left
    assert L.gsf_find(cubes, 1, filt, 1, box, 4.0, masks, None, None, None, ws, need, None) == 1
    cubes[0].halo[2] = -1
    assert L.gsf_find(cubes, 1, filt, 1, box, 4.0, masks, None, None, None, ws, need, None) == 1
    cubes[0].halo[2] = 0
    cubes[0].dtype = 9   # unknown storage type
    assert L.gsf_find(cubes, 1, filt, 1, box, 4.0, masks, None, None, None, ws, need, None) == 1
    cubes[0].dtype = 0
    masks2 = (ctypes.c_void_p * 1)(4096 + 64)  # mask overlaps the cube
    assert L.gsf_find(cubes, 1, filt, 1, box, 4.0, masks2, None, None, None, ws, need, None) == 1


def test_tuning_table_validation(L):
    t = B.Tuning(1, 0, 512, 0, 1, 1)
    assert L.gsf_tuning_set(-1, 0, ctypes.byref(t)) == 0
    for bad in (B.Tuning(2, 0, 512, 0, 1, 0), B.Tuning(1, 4, 512, 0, 1, 0),
                B.Tuning(1, -1, 512, 0, 1, 0), B.Tuning(1, 0, 63, 0, 1, 0),
                B.Tuning(1, 0, 70000, 0, 1, 0), B.Tuning(1, 0, 512, 4, 1, 0),
                B.Tuning(1, 0, 512, 0, 2, 0), B.Tuning(1, 0, 512, 0, 1, 2)):
        assert L.gsf_tuning_set(-1, 0, ctypes.byref(bad)) == B.GSF_ERR_INVALID_ARG
    assert L.gsf_tuning_set(41, 0, ctypes.byref(t)) == B.GSF_ERR_INVALID_ARG
    assert L.gsf_tuning_set(-2, 0, ctypes.byref(t)) == B.GSF_ERR_INVALID_ARG
    assert L.gsf_tuning_set(3, 7, ctypes.byref(t)) == B.GSF_ERR_INVALID_ARG
    assert L.gsf_tuning_set(3, 0, None) == B.GSF_ERR_INVALID_ARG
    t2 = B.Tuning(0, 2, 4096, 5, 0, 1)
    assert L.gsf_tuning_set(20, 1, ctypes.byref(t2)) == 0
    got = B.Tuning()
    assert L.gsf_tuning_get(20, 1, ctypes.byref(got)) == 0
    assert (got.merge_sweeps, got.merged_shape, got.sweep_blocks, got.yz_waves,
            got.pair_spectral, got.x_exits) == (0, 2, 4096, 5, 0, 1)
    assert L.gsf_tuning_get(20, 0, ctypes.byref(got)) == 0
    assert (got.merge_sweeps, got.merged_shape, got.sweep_blocks, got.yz_waves,
            got.pair_spectral, got.x_exits) == (1, 0, 512, 0, 1, 1)
    assert L.gsf_tuning_get(-1, 0, ctypes.byref(got)) == B.GSF_ERR_INVALID_ARG
    assert L.gsf_tuning_reset() == 0
    assert L.gsf_tuning_get(20, 1, ctypes.byref(got)) == 0
    assert (got.merge_sweeps, got.sweep_blocks) == (1, 512)


def test_default_tuning_entries(L):
    """Cores of 2^26 voxels and more default to the merged sweep's block
    measured best on the 512x512x1024 cube (FP32 1 row x 16 waves, 16-bit 2
    rows x 4 waves); every other entry to 1 x 8; the x walk's early exit is
    on everywhere."""
    assert L.gsf_tuning_reset() == 0
    got = B.Tuning()
    for cls, dt, shape in ((28, 0, 2), (26, 0, 2), (25, 0, 0), (28, 1, 3), (28, 2, 3), (25, 1, 0),
                           (10, 0, 0)):
        assert L.gsf_tuning_get(cls, dt, ctypes.byref(got)) == 0
        assert got.merged_shape == shape, (cls, dt)
        assert (got.merge_sweeps, got.sweep_blocks, got.pair_spectral, got.x_exits) == (1, 512, 1, 1)


def test_size_class(L):
    assert L.gsf_size_class(B.Dims(1, 1, 1)) == 0
    assert L.gsf_size_class(B.Dims(512, 512, 1024)) == 28
    assert L.gsf_size_class(B.Dims(3, 3, 3)) == 4          # 27 voxels
    assert L.gsf_size_class(B.Dims(0, 3, 3)) == -1


def test_find_workspace_counts_merged_filters(L):
    # one spectral pass shared by three filters needs three F buffers; one
    # filter per pass needs one
    cubes = (B.Cube * 1)()
    cubes[0].data = 256
    cubes[0].dims = B.Dims(64, 64, 128)
    cb = 64 * 64 * 128 * 4

    def ws(filters, box=B.Box(16, 16, 16)):
        filt = (B.Filter * len(filters))(*[B.Filter(a, b, 3) for a, b in filters])
        n = ctypes.c_size_t(0)
        assert L.gsf_find_workspace_size(cubes, 1, filt, len(filters), box, ctypes.byref(n)) == 0
        return n.value

    parts = ((1 << 16) * 8 + 255) // 256 * 256
    single = ws([(1, 1)])
    three = ws([(1, 2), (2, 2), (4, 2)])
    assert three - single == 2 * cb + 2 * parts
    # T1 + F + two window-sum cubes (+ shift partials) for the fast statistics
    assert single >= 4 * cb and single < 4 * cb + (1 << 20)
    # spectral radii 3 and 6 form a compiled pair: the first two groups share
    # one read of the cube into two T1 buffers (the third group reuses the first)
    paired = ws([(1, 1), (2, 2), (2, 4)])
    assert paired - single == cb
    # radii 3 and 15 (sigma_z 5) have no compiled pair: one T1
    assert ws([(1, 1), (1, 5)]) == single
    # four cubes of window sums on the generic statistics path (box 128 > 64)
    assert ws([(1, 1)], B.Box(128, 16, 16)) - ws([(1, 1)]) == 2 * cb


def test_find_noalloc_validation(L):
    """gsf_find_noalloc validates like gsf_find and refuses, before any device
    call, a batch whose one-slot workspace exceeds its scratch."""
    cubes = (B.Cube * 1)()
    cubes[0].data = 4096
    cubes[0].dims = B.Dims(8, 8, 8)
    filt = (B.Filter * 1)(B.Filter(1, 1, 3))
    masks = (ctypes.c_void_p * 1)(1 << 20)
    box = B.Box(4, 4, 4)
    assert L.gsf_find_noalloc(cubes, 0, filt, 1, box, 4.0, masks, None, None, None, None) == 1
    assert L.gsf_find_noalloc(cubes, 1, filt, 0, box, 4.0, masks, None, None, None, None) == 1
    assert L.gsf_find_noalloc(cubes, 1, filt, 1, box, 4.0, None, None, None, None, None) == 1
    assert L.gsf_find_noalloc(cubes, 1, filt, 1, box, float("inf"), masks, None, None, None,
                              None) == 1
    # one FP32 slot with a group of three filters holds T1, three F and two
    # window-sum cubes: 6 x 48 MiB for 256 x 256 x 192 voxels passes 256 MiB
    cubes[0].dims = B.Dims(256, 256, 192)
    filt3 = (B.Filter * 3)(B.Filter(1, 2, 3), B.Filter(2, 2, 3), B.Filter(4, 2, 3))
    box8 = B.Box(8, 8, 8)
    assert L.gsf_find_noalloc(cubes, 1, filt3, 3, box8, 4.0, masks, None, None, None,
                              None) == B.GSF_ERR_BUDGET
    assert b"GSF_NOALLOC_SCRATCH_BYTES" in L.gsf_last_error()
