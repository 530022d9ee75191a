"""The C-ABI boundary without a GPU: libfg.so loads, exports every function
include/fg.h declares (and the binding lists exactly those), and its host-only
paths behave as documented: status strings, workspace sizes, argument
rejection before any device work, and the tune struct's layout.
No kernel is launched here.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2603_23891_amd import fg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fg.h")

FG_OK, FG_ERR_INVALID_ARG, FG_ERR_UNSUPPORTED, FG_ERR_WORKSPACE = 0, -1, -3, -4


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return fg.lib()


def test_header_declares_the_path_entry_points():
    names = declared_functions()
    for n in ("fg_filter", "fg_preprocess", "fg_sort", "fg_render", "fg_activate", "fg_render_backward"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_exactly_the_declared_symbols():
    assert sorted(fg.EXPORTS) == declared_functions()


def test_status_strings(lib):
    for code, text in [(0, b"ok"), (-1, b"invalid argument"), (-4, b"workspace too small"), (99, b"unknown status")]:
        assert lib.fg_status_string(code) == text


def cam_1080p(tile_base=0):
    class Cam:
        R = np.eye(3, dtype=np.float32).reshape(9)
        t = np.zeros(3, np.float32)
        campos = np.zeros(3, np.float32)
        fx = fy = 1662.8
        cx, cy = 960.0, 540.0
        width, height = 1920, 1080
        znear, kx, ky = 0.2, 1.3, 1.3
    Cam.tile_base = tile_base
    return Cam


def test_workspace_sizes_are_monotone_and_reject_bad_sizes():
    a = fg.fg_filter_workspace_size(1000, 100, 1)
    b = fg.fg_filter_workspace_size(100000, 10000, 1)
    c = fg.fg_filter_workspace_size(100000, 10000, 8)
    assert 0 < a < b < c
    cam = cam_1080p()
    s1 = fg.fg_sort_workspace_size(1000, 1, 1000, 5000)
    s2 = fg.fg_sort_workspace_size(100000, 1, 100000, 500000)
    s3 = fg.fg_sort_workspace_size(100000, 8, 100000, 500000)
    assert 0 < s1 < s2 < s3
    assert fg.fg_sort_workspace_size(-1, 1, 5, 5) == 0 and fg.fg_sort_workspace_size(5, 0, 5, 5) == 0
    r = [fg.fg_render_workspace_size(cam, 1 << 20, fg.tune_struct(k)) for k in (128, 256, 512)]
    assert fg.fg_render_workspace_size([cam_1080p(0), cam_1080p(8160)], 1 << 20) > r[1]
    assert fg.fg_render_workspace_size([cam_1080p(0), cam_1080p(5)], 1 << 20) == 0  # tile ids not consecutive
    assert all(x > 0 for x in r)
    assert fg.fg_render_workspace_size(cam, -1) == 0
    assert fg.lib().fg_render_backward_workspace_size(1000) >= 1000 * 9 * 4


def test_entry_points_reject_missing_arguments_on_the_host(lib):
    cam = fg.camera_struct(cam_1080p())
    # null inputs are refused before any device work
    assert lib.fg_filter(None, None, 1, None, C.c_float(3.0), None, None, 0, None, None, None, 0,
                         None) == FG_ERR_INVALID_ARG
    assert lib.fg_preprocess(None, None, None, 0, C.byref(cam), 1, None, C.c_float(0.0), None, None,
                             None) == FG_ERR_INVALID_ARG
    assert lib.fg_sort(None, None, 0, C.byref(cam), 1, 0, None, None, 0, None, None, None, None, 0, None,
                       None) == FG_ERR_INVALID_ARG
    bg = (C.c_float * 3)(0.0, 0.0, 0.0)
    assert lib.fg_render(None, None, None, C.byref(cam), 1, C.cast(bg, C.c_void_p), None, None, None, 0, None,
                         None, None, 0, None, None) == FG_ERR_INVALID_ARG


def test_tune_struct_layout():
    """fg_tune as the header lays it out: four int32, two event handles, then
    the backward's counter pointer."""
    t = fg.tune_struct(512, 7, True)
    assert C.sizeof(t) == 16 + 3 * C.sizeof(C.c_void_p)
    assert fg.FgTune.bwd_stats.offset == 16 + 2 * C.sizeof(C.c_void_p)
    assert (t.render_batch, t.radix_bits, t.save_state) == (512, 7, 1)
    assert t.blend_events[0] is None and t.blend_events[1] is None and t.bwd_stats is None


def test_filter_rejects_inconsistent_trees_on_the_host(lib):
    """FG_ERR_INVALID_TREE is decided from the struct's sizes before any device
    work: the plane pointers (never dereferenced here) only need to be set."""
    cam = (fg.FgCamera * 1)(fg.camera_struct(cam_1080p()))
    fake = 1 << 20  # a non-null address no device work ever reads: the call returns first

    def call(n_nodes, span, max_depth):
        t = fg.FgTree(n_nodes=n_nodes, n_internal_span=span, sh_degree=0, max_depth=max_depth, mean=fake,
                      scale=fake, quat=fake, opacity=fake, sh=fake, parent=fake, flags=fake)
        return lib.fg_filter(C.byref(t), C.cast(cam, C.c_void_p), 1, None, C.c_float(3.0), C.c_void_p(fake),
                             C.c_void_p(fake), 16, C.c_void_p(fake), C.c_void_p(fake), C.c_void_p(fake), 1 << 30,
                             None)

    FG_ERR_INVALID_TREE = -2
    assert call(100, 101, 3) == FG_ERR_INVALID_TREE      # internal span beyond the node count
    assert call(100, -1, 3) == FG_ERR_INVALID_TREE       # negative span
    assert call(100, 10, 16) == FG_ERR_INVALID_TREE      # ancestor chains longer than 15
    assert call(100, 10, -1) == FG_ERR_INVALID_TREE
    assert call(-5, 0, 0) == FG_ERR_INVALID_TREE
    assert call(1 << 31, 0, 0) == FG_ERR_INVALID_TREE    # node ids must fit 31 bits
    assert lib.fg_status_string(FG_ERR_INVALID_TREE) == b"invalid tree"


def test_filter_noalloc_rejects_problems_beyond_its_scratch_on_the_host(lib):
    """fg_filter_noalloc refuses, before any device work, a tree whose filter
    workspace exceeds its fixed scratch array, and checks arguments like
    fg_filter."""
    cam = (fg.FgCamera * 1)(fg.camera_struct(cam_1080p()))
    fake = 1 << 20

    def call(n_nodes, span):
        t = fg.FgTree(n_nodes=n_nodes, n_internal_span=span, sh_degree=0, max_depth=8, mean=fake, scale=fake,
                      quat=fake, opacity=fake, sh=fake, parent=fake, flags=fake)
        return lib.fg_filter_noalloc(C.byref(t), C.cast(cam, C.c_void_p), 1, None, C.c_float(3.0),
                                     C.c_void_p(fake), C.c_void_p(fake), 16, C.c_void_p(fake), C.c_void_p(fake),
                                     None)

    FG_ERR_SCRATCH, FG_ERR_INVALID_TREE = -6, -2
    limit = 16 << 20
    big = (1 << 31) - 1  # every node internal: about 0.53 GB of small/blocked bits
    assert fg.fg_filter_workspace_size(big, big, 1) > limit
    assert call(big, big) == FG_ERR_SCRATCH
    assert call(100, 101) == FG_ERR_INVALID_TREE
    assert lib.fg_filter_noalloc(None, None, 1, None, C.c_float(3.0), None, None, 0, None, None,
                                 None) == FG_ERR_INVALID_ARG
    assert b"fixed scratch" in lib.fg_status_string(FG_ERR_SCRATCH)
