"""The C ABI library loads on the host and exports what include/nm.h declares;
host-side argument checks reject bad input before anything reaches a device.
(No compute calls here: these tests run without a GPU.)"""
import ctypes
import os
import re

import pytest

from paper_2103_10239_amd import nm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(nm_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = nm.lib()
    declared = _declared()
    assert {"nm_build_cells", "nm_knn", "nm_metric_list", "nm_align_step", "nm_step"} <= declared
    for name in sorted(declared):
        assert hasattr(lib, name), f"{name} declared but not exported"


def test_status_strings():
    for code in (0, -1, -2, -3, -4, -5):
        assert nm.status_str(code) not in ("", "unknown status")
    assert nm.status_str(7) == "unknown status"


@pytest.mark.parametrize("n,box,w", [(1, 1 << 20, 1024), (1 << 20, 1000, 8), (1 << 20, 1 << 21, 1024),
                                     (1 << 20, 1 << 20, 3), (1 << 20, 1 << 20, 1 << 21),
                                     (1 << 25, 1 << 20, 1024), (1 << 20, 1 << 20, 1)])
def test_invalid_grids_rejected(n, box, w):
    g = nm.Grid(n, box, w, 0)
    assert nm.lib().nm_workspace_bytes(ctypes.byref(g)) == nm.NM_E_INVAL


@pytest.mark.parametrize("block,ok", [(0, True), (-1, True), (4, True), (15, True), (16, False), (2, False),
                                      (-2, False), (nm.NM_BLOCK_SUBSTRIPS, True),
                                      (nm.NM_BLOCK_SUBSTRIPS | 6, True), (nm.NM_BLOCK_SUBSTRIPS | 2, False),
                                      (nm.NM_BLOCK_SUBSTRIPS | 16, False), (0x200, False)])
def test_block_field_and_substrip_flag(block, ok):
    g = nm.Grid(1 << 20, 1 << 20, 1024, block)
    assert (nm.lib().nm_workspace_bytes(ctypes.byref(g)) > 0) == ok


def test_workspace_size_grows_with_cells_and_particles():
    b = lambda n, w: nm.lib().nm_workspace_bytes(ctypes.byref(nm.Grid(n, 1 << 20, w, 0)))
    assert b(1 << 20, 1024) > b(1 << 20, 2048) > 0
    assert b(1 << 21, 2048) > b(1 << 20, 2048)


def test_suggest_cell_w():
    assert nm.suggest_cell_w(1 << 20, 1 << 20, 1.0) == 1024
    assert nm.suggest_cell_w(1 << 20, 1 << 20, 4.0) == 2048
    assert nm.suggest_cell_w(2, 1 << 20, 2.0) == 1 << 20
    w = nm.suggest_cell_w(1 << 24, 1 << 20, 0.01)
    assert ((1 << 20) // w) ** 2 <= 1 << 28


def test_host_checks_return_before_any_launch():
    lib = nm.lib()
    g = nm.Grid(1024, 1 << 20, 1 << 15, 0)
    fake = ctypes.c_void_p(256)  # never dereferenced: every call below fails validation first
    # k out of range
    assert lib.nm_knn(ctypes.byref(g), fake, 0, fake, None, None) == nm.NM_E_INVAL
    assert lib.nm_knn(ctypes.byref(g), fake, 33, fake, None, None) == nm.NM_E_INVAL
    # workspace too small / misaligned
    assert lib.nm_build_cells(ctypes.byref(g), fake, fake, fake, 16, None) == nm.NM_E_INVAL
    assert lib.nm_build_cells(ctypes.byref(g), fake, fake, ctypes.c_void_p(300), 1 << 30, None) == nm.NM_E_INVAL
    # metric radius out of range
    assert lib.nm_metric_list(ctypes.byref(g), fake, -1, fake, None, 0, None, None) == nm.NM_E_INVAL
    # polar order: null pointers, no headings
    assert lib.nm_polar_order(None, 10, fake, None) == nm.NM_E_INVAL
    assert lib.nm_polar_order(fake, 0, fake, None) == nm.NM_E_INVAL
    assert lib.nm_polar_order(fake, 10, None, None) == nm.NM_E_INVAL
    # bad parameters: box not a power of two, |v0| >= L/2, negative eta, unknown variant bit
    for p in (nm.Params(1000, 64, 0.2, 1, 0, 0, 0), nm.Params(1 << 20, 1 << 19, 0.2, 1, 0, 0, 0),
              nm.Params(1 << 20, 64, -0.1, 1, 0, 0, 0), nm.Params(1 << 20, 64, 0.2, 1, 0, 0, 4),
              nm.Params(1 << 20, 64, float("nan"), 1, 0, 0, 0), nm.Params(1 << 20, 64, 0.2, 2, 0, 0, 0)):
        assert lib.nm_align_step(fake, fake, fake, 16, fake, None, 7, 0, ctypes.byref(p), 0,
                                 ctypes.c_void_p(512), ctypes.c_void_p(768), ctypes.c_void_p(1024),
                                 None, None) == nm.NM_E_INVAL
    p = nm.Params(1 << 20, 64, 0.2, 1, 0, 0, 0)
    # outputs aliasing inputs
    assert lib.nm_align_step(fake, ctypes.c_void_p(512), ctypes.c_void_p(768), 16, fake, None, 7, 0,
                             ctypes.byref(p), 0, fake, ctypes.c_void_p(900), ctypes.c_void_p(1000),
                             None, None) == nm.NM_E_INVAL
    # fused step: p.box must equal grid box
    p2 = nm.Params(1 << 19, 64, 0.2, 1, 0, 0, 0)
    assert lib.nm_step(ctypes.byref(g), fake, fake, fake, 7, ctypes.byref(p2), 0, fake, 1 << 30, fake,
                       fake, fake, fake, None) == nm.NM_E_INVAL


def test_binding_rejects_host_tensors():
    import torch
    with pytest.raises((TypeError, ImportError)):
        nm._dev(torch.zeros(4, dtype=torch.int32), torch.int32, 4, "x")


L = 1 << 20


def test_server_job_bytes_ledger():
    # workspace + double-buffered x, y, theta + the k-NN list, 256-byte aligned pieces
    b1 = nm.server_job_bytes(1024, 7, L)
    assert b1 > (24 + 4 * 7) * 1024
    assert nm.server_job_bytes(4096, 7, L) > b1
    assert nm.server_job_bytes(1024, 12, L) - b1 >= 4 * 5 * 1024
    assert nm.server_job_bytes(1 << 20, 12, L) < 160 * (1 << 20)  # about 127 MiB
    assert nm.server_job_bytes(5, 7, L) < 0 and nm.server_job_bytes(100, 33, L) < 0


def test_batch_plan_is_host_only():
    # planning allocates host memory only and validates its arguments
    L_ = nm.lib()
    h, nbytes = ctypes.c_void_p(), ctypes.c_int64()
    p = nm.make_params(L)
    sizes = (ctypes.c_int32 * 3)(300, 5000, 65536)
    assert L_.nm_batch_plan(3, sizes, L, 7, ctypes.byref(p), None, ctypes.byref(h), ctypes.byref(nbytes)) == 0
    assert nbytes.value > sum((24 + 4 * 7) * n for n in (300, 5000, 65536))
    # not bound to device memory yet: no block choice or tuning can be set
    assert L_.nm_batch_set_block(h, 4, None) == nm.NM_E_INVAL
    assert L_.nm_batch_tune(h, 1, None) == nm.NM_E_INVAL
    L_.nm_batch_destroy(h)
    bad = (ctypes.c_int32 * 2)(300, 7)  # a system with n < k + 1
    assert L_.nm_batch_plan(2, bad, L, 7, ctypes.byref(p), None, ctypes.byref(h), ctypes.byref(nbytes)) == nm.NM_E_INVAL


def test_voronoi_and_noalloc_entry_points_check_arguments_on_the_host():
    # every call below fails validation before touching a device (and exercises
    # the binding's argument lists)
    lib = nm.lib()
    fake = ctypes.c_void_p(256)
    g = nm.Grid(1024, 1 << 20, 1 << 15, 0)
    assert lib.nm_voronoi(ctypes.byref(g), fake, 2, fake, fake, None) == nm.NM_E_INVAL  # dmax < 3
    assert lib.nm_voronoi(ctypes.byref(g), fake, 65, fake, fake, None) == nm.NM_E_INVAL
    assert lib.nm_voronoi(ctypes.byref(g), None, 16, fake, fake, None) == nm.NM_E_INVAL
    assert lib.nm_voronoi_check(ctypes.byref(g), fake, fake, fake, 16, fake, fake, None, None,
                                None) == nm.NM_E_INVAL  # stale missing
    assert lib.nm_voronoi_update(ctypes.byref(g), fake, None, fake, 16, fake, fake, fake, None,
                                 None) == nm.NM_E_INVAL
    vp = nm.VmParams(1.0, 1.0, 1.0, float("nan"))
    assert lib.nm_voronoi_forces(fake, fake, 1024, 1 << 20, 16, fake, fake, ctypes.byref(vp), fake, fake,
                                 fake, fake, None, None, None, None) == nm.NM_E_INVAL  # non-finite P0
    vp = nm.VmParams(1.0, 1.0, 1.0, 1.0)
    assert lib.nm_voronoi_forces(fake, fake, 1024, 1000, 16, fake, fake, ctypes.byref(vp), fake, fake,
                                 fake, fake, None, None, None, None) == nm.NM_E_INVAL  # box not 2^m
    p = nm.make_params(1 << 20)
    big = nm.Grid(1 << 20, 1 << 20, 1024, 0)
    assert lib.nm_step_noalloc(ctypes.byref(big), fake, fake, fake, 7, ctypes.byref(p), 0, fake, fake, fake,
                               fake, None, None) == nm.NM_E_NOMEM  # beyond the device array
    assert lib.nm_step_noalloc(ctypes.byref(nm.Grid(1, 1 << 20, 1024, 0)), fake, fake, fake, 7,
                               ctypes.byref(p), 0, fake, fake, fake, fake, None, None) == nm.NM_E_INVAL
    out = (ctypes.c_int32 * 10)()
    assert lib.nm_knn_layout(ctypes.byref(g), 0, out) == nm.NM_E_INVAL
    assert lib.nm_knn_layout(ctypes.byref(g), 7, out) == nm.NM_OK
