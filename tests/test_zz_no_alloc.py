"""nm_step_noalloc (the step with the library's own device array as its
workspace, for callers that cannot allocate) against nm_step with a caller
workspace, through the C ABI: two calls in a row, the second on a smaller
system, lists, positions and headings identical; the size limit and the
device-side error report."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2103_10239_amd as nm
from paper_2103_10239_amd import workloads

pytestmark = pytest.mark.gpu


def _call_noalloc(grid, X, Y, T, k, p, step, err):
    n = grid.n
    nbr = torch.full((n, k), -9, dtype=torch.int32, device="cuda")
    xo, yo, to = torch.empty_like(X), torch.empty_like(Y), torch.empty_like(T)
    rc = nm.nm.lib().nm_step_noalloc(ctypes.byref(grid), X.data_ptr(), Y.data_ptr(), T.data_ptr(), k,
                                     ctypes.byref(p), step, nbr.data_ptr(), xo.data_ptr(), yo.data_ptr(),
                                     to.data_ptr(), err.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return rc, nbr, xo, yo, to


def _call_plain(grid, X, Y, T, k, p, step):
    ws = nm.Workspace(grid.n, grid.box, grid.cell_w, block=grid.block)
    nbr = torch.empty((grid.n, k), dtype=torch.int32, device="cuda")
    xo, yo, to = torch.empty_like(X), torch.empty_like(Y), torch.empty_like(T)
    nm.step(ws, X, Y, T, k, p, step, nbr, xo, yo, to)
    assert nm.check(ws) == 0
    return nbr, xo, yo, to


def test_noalloc_step_equals_nm_step_twice():
    box = workloads.BOX
    err = torch.full((1,), 123, dtype=torch.int32, device="cuda")
    # a larger system first, then a smaller one on another grid: the shared
    # array still holds the first call's cells and counters
    for n, k, w, kind, step in ((200003, 7, 1024, "clustered", 5), (4097, 12, 4096, "uniform", 9)):
        if kind == "clustered":
            x, y, th = workloads.clustered(n)
        else:
            x, y, th = workloads.uniform(n)
        X, Y, T = (torch.as_tensor(a).cuda() for a in (x, y, th))
        p = nm.make_params(box, v0=64, eta=0.2, seed=11, sys_id=2)
        grid = nm.Grid(n, box, w, 0)
        assert nm.nm.lib().nm_workspace_bytes(ctypes.byref(grid)) <= 32 << 20
        rc, *got = _call_noalloc(grid, X, Y, T, k, p, step, err)
        assert rc == 0
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        ref = _call_plain(grid, X, Y, T, k, p, step)
        for a, b in zip(got, ref):
            assert torch.equal(a, b)


def test_noalloc_limits_and_errors():
    box = workloads.BOX
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    n = 1 << 20  # workspace of about 90 MB: refused before anything runs
    X = torch.zeros(n, dtype=torch.int32, device="cuda")
    T = torch.zeros(n, dtype=torch.float32, device="cuda")
    p = nm.make_params(box)
    rc, *_ = _call_noalloc(nm.Grid(n, box, 1024, 0), X, X, T, 7, p, 0, err)
    assert rc == nm.NM_E_NOMEM
    # a coordinate outside the box: reported through err, and the next call is clean again
    x, y, th = workloads.uniform(5000)
    x[17] = box
    X, Y, T = (torch.as_tensor(a).cuda() for a in (x, y, th))
    rc, *_ = _call_noalloc(nm.Grid(5000, box, 4096, 0), X, Y, T, 7, p, 0, err)
    assert rc == 0
    torch.cuda.synchronize()
    assert int(err.item()) == nm.NM_E_RANGE
    x[17] = 5
    X = torch.as_tensor(x).cuda()
    rc, *_ = _call_noalloc(nm.Grid(5000, box, 4096, 0), X, Y, T, 7, p, 0, err)
    torch.cuda.synchronize()
    assert rc == 0 and int(err.item()) == 0
