"""ctypes binding of libnm.so (include/nm.h): argument marshalling only.

Every step of the neighbour-list / Vicsek path runs in the HIP kernels of
libnm.so; this module checks tensor shapes and dtypes, passes raw device
pointers and torch's current HIP stream, and turns status codes into
exceptions.  PyTorch supplies device memory and streams, nothing else.  There
is no fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnm.so")

NM_OK, NM_E_INVAL, NM_E_RANGE, NM_E_CAPACITY, NM_E_NOMEM, NM_E_DEVICE = 0, -1, -2, -3, -4, -5
NM_MAX_K = 32
NM_NOISE_SCALAR, NM_MOVE_NEW_HEADING = 1, 2  # nm_params.variant flags
NM_BLOCK_SUBSTRIPS = 0x100  # nm_grid.block flag: overflowing strips run as staged sub-strips

_c_i32, _c_i64, _c_u32, _c_u64, _vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                       ctypes.c_uint64, ctypes.c_void_p)


class NMError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


class Grid(ctypes.Structure):
    """nm_grid: n particles, box side L, cell width w (powers of two), and the
    k-NN fast-path block side (0 automatic, -1 exact ring search only), with
    NM_BLOCK_SUBSTRIPS or-ed in to pick the sub-strip kernel."""
    _fields_ = [("n", _c_i32), ("box", _c_i32), ("cell_w", _c_i32), ("block", _c_i32)]


class Params(ctypes.Structure):
    """nm_params: Eq. (1) and Eq. (2) parameters and the Philox identity."""
    _fields_ = [("box", _c_i32), ("v0", _c_i32), ("eta", ctypes.c_float), ("include_self", _c_i32),
                ("seed", _c_u64), ("sys_id", _c_u32), ("variant", _c_u32)]


class VmParams(ctypes.Structure):
    """nm_vm_params: the moduli and preferred area / perimeter of Eq. (3)."""
    _fields_ = [("ka", ctypes.c_double), ("kp", ctypes.c_double), ("a0", ctypes.c_double),
                ("p0", ctypes.c_double)]


class BatchIO(ctypes.Structure):
    """nm_batch_io: concatenated double-buffered state and the list output."""
    _fields_ = [("x", _vp * 2), ("y", _vp * 2), ("theta", _vp * 2), ("nbr", _vp)]


class Job(ctypes.Structure):
    """nm_job: one served job (host inputs, copied at submission)."""
    _fields_ = [("n", _c_i32), ("k", _c_i32), ("nsteps", _c_i32), ("want_nbr", _c_i32), ("p", Params),
                ("x", _vp), ("y", _vp), ("theta", _vp)]


class JobResult(ctypes.Structure):
    _fields_ = [("status", _c_i32), ("steps", _c_i32), ("submit_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("submitted", _c_i64), ("completed", _c_i64), ("iterations", _c_i64),
                ("budget_bytes", _c_i64), ("used_bytes", _c_i64), ("peak_used_bytes", _c_i64),
                ("reserved_bytes", _c_i64), ("active", _c_i32), ("peak_active", _c_i32),
                ("queued", _c_i32), ("status", _c_i32), ("now_s", ctypes.c_double)]


_lib = None


def lib():
    """Load libnm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; "
                          "g.build()'` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    gp, pp = ctypes.POINTER(Grid), ctypes.POINTER(Params)
    L.nm_status_str.argtypes, L.nm_status_str.restype = [ctypes.c_int], ctypes.c_char_p
    L.nm_workspace_bytes.argtypes, L.nm_workspace_bytes.restype = [gp], _c_i64
    L.nm_suggest_cell_w.argtypes = [_c_i32, _c_i32, ctypes.c_double]
    L.nm_suggest_cell_w.restype = _c_i32
    L.nm_workspace_init.argtypes = [gp, _vp, ctypes.c_size_t, _vp]
    L.nm_build_cells.argtypes = [gp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.nm_knn.argtypes = [gp, _vp, _c_i32, _vp, _vp, _vp]
    L.nm_metric_list.argtypes = [gp, _vp, _c_i64, _vp, _vp, _c_i64, ctypes.POINTER(_c_i64), _vp]
    L.nm_align_step.argtypes = [_vp, _vp, _vp, _c_i32, _vp, _vp, _c_i32, _c_i64, pp, _c_u64,
                                _vp, _vp, _vp, _vp, _vp]
    L.nm_step.argtypes = [gp, _vp, _vp, _vp, _c_i32, pp, _c_u64, _vp, ctypes.c_size_t, _vp, _vp,
                          _vp, _vp, _vp]
    L.nm_bin_step.argtypes = [gp, _vp, _vp, _vp, pp, _c_u64, _vp, ctypes.c_size_t, _vp]
    L.nm_knn_align.argtypes = [gp, _vp, _c_i32, pp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.nm_check.argtypes = [_vp, _vp]
    L.nm_polar_order.argtypes = [_vp, _c_i32, _vp, _vp]
    L.nm_knn_fov.argtypes = [gp, _vp, _c_i32, _vp, _c_i32, _vp, _vp]
    L.nm_knn_layout.argtypes = [gp, _c_i32, ctypes.POINTER(_c_i32)]
    L.nm_voronoi.argtypes = [gp, _vp, _c_i32, _vp, _vp, _vp]
    L.nm_voronoi_forces.argtypes = [_vp, _vp, _c_i32, _c_i32, _c_i32, _vp, _vp, ctypes.POINTER(VmParams)] + \
        [_vp] * 8
    L.nm_step_noalloc.argtypes = [gp, _vp, _vp, _vp, _c_i32, pp, _c_u64, _vp, _vp, _vp, _vp, _vp, _vp]
    L.nm_voronoi_check.argtypes = [gp, _vp, _vp, _vp, _c_i32, _vp, _vp, _vp, _vp, _vp]
    L.nm_voronoi_update.argtypes = [gp, _vp, _vp, _vp, _c_i32, _vp, _vp, _vp, _vp, _vp]
    L.nm_tune_grid.argtypes = [gp, _c_i32, _vp, _vp, _vp, _c_i32, pp, _c_u64, _vp, ctypes.c_size_t,
                               _vp, _vp, _vp, _vp, _c_i32, ctypes.POINTER(_c_i32),
                               ctypes.POINTER(ctypes.c_float), _vp]
    L.nm_batch_plan.argtypes = [_c_i32, ctypes.POINTER(_c_i32), _c_i32, _c_i32, pp,
                                ctypes.POINTER(_c_u32), ctypes.POINTER(_vp), ctypes.POINTER(_c_i64)]
    L.nm_batch_bind.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.POINTER(BatchIO), _c_u64, _vp]
    L.nm_batch_step.argtypes = [_vp, _c_i32, _c_i32, _vp]
    L.nm_batch_tune.argtypes = [_vp, _c_i32, _vp]
    L.nm_batch_set_block.argtypes = [_vp, _c_i32, _vp]
    L.nm_batch_system.argtypes = [_vp, _c_i32, gp, ctypes.POINTER(_c_i32)]
    L.nm_batch_steps_done.argtypes, L.nm_batch_steps_done.restype = [_vp], _c_i64
    L.nm_batch_check.argtypes = [_vp, _vp]
    L.nm_batch_destroy.argtypes, L.nm_batch_destroy.restype = [_vp], None
    L.nm_server_job_bytes.argtypes, L.nm_server_job_bytes.restype = [_c_i32, _c_i32, _c_i32], _c_i64
    L.nm_server_create.argtypes = [_c_i64, _c_i32, ctypes.POINTER(_vp)]
    L.nm_server_submit.argtypes = [_vp, ctypes.POINTER(Job), ctypes.POINTER(_c_i64)]
    L.nm_server_poll.argtypes = [_vp, _c_i64]
    L.nm_server_wait.argtypes = [_vp, _c_i64, _vp, _vp, _vp, _vp, ctypes.POINTER(JobResult)]
    L.nm_server_stats.argtypes = [_vp, ctypes.POINTER(ServerInfo)]
    L.nm_server_destroy.argtypes, L.nm_server_destroy.restype = [_vp], None
    for f in ("nm_server_create", "nm_server_submit", "nm_server_poll", "nm_server_wait",
              "nm_server_stats"):
        getattr(L, f).restype = ctypes.c_int
    for f in ("nm_workspace_init", "nm_build_cells", "nm_knn", "nm_knn_layout", "nm_voronoi", "nm_step_noalloc",
              "nm_voronoi_forces",
              "nm_voronoi_check", "nm_voronoi_update", "nm_metric_list", "nm_align_step",
              "nm_step", "nm_bin_step", "nm_knn_align", "nm_check", "nm_tune_grid", "nm_batch_plan", "nm_batch_bind",
              "nm_batch_step", "nm_batch_tune", "nm_batch_set_block", "nm_batch_system", "nm_batch_check"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def status_str(status: int) -> str:
    try:
        return lib().nm_status_str(status).decode()
    except ImportError:
        return str(status)


def _ok(rc: int, what: str) -> None:
    if rc != NM_OK:
        raise NMError(rc, what)


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev(t: torch.Tensor, dtype, numel: int | None, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs {numel} elements, has {t.numel()}")
    return t.data_ptr()


def suggest_cell_w(n: int, box: int, per_cell: float = 2.0) -> int:
    return int(lib().nm_suggest_cell_w(n, box, per_cell))


def make_params(box: int, v0: int = 64, eta: float = 0.2, include_self: int = 1, seed: int = 0,
                sys_id: int = 0, variant: int = 0) -> Params:
    """variant: 0 (Eq. (2) and Eq. (1)), or NM_NOISE_SCALAR and/or NM_MOVE_NEW_HEADING."""
    return Params(box, v0, eta, include_self, seed, sys_id, variant)


def knn_fov(ws: Workspace, k: int, theta: torch.Tensor, cos_q: int, nbr: torch.Tensor | None = None):
    """Field-of-view k-NN lists [n, k] (cone cos(alpha) = cos_q / 4096 around each
    heading) from the cells built in ws.  A particle that sees fewer than k
    others is reported by check() as NM_E_RANGE."""
    n = ws.n
    if nbr is None:
        nbr = torch.empty((n, k), dtype=torch.int32, device=ws.device)
    _ok(lib().nm_knn_fov(ctypes.byref(ws.grid), ws.ptr, k, _dev(theta, torch.float32, n, "theta"), cos_q,
                         _dev(nbr, torch.int32, n * k, "nbr"), _stream(ws.device)), "knn_fov")
    return nbr


NM_VORONOI_MAX_DEG = 64


def voronoi(ws: Workspace, dmax: int = 16, ring: torch.Tensor | None = None,
            deg: torch.Tensor | None = None):
    """Voronoi (Delaunay) neighbour rows from the cells built in ws: (ring [n, dmax]
    counter-clockwise from +x, padded with -1; deg [n])."""
    n = ws.n
    if ring is None:
        ring = torch.empty((n, dmax), dtype=torch.int32, device=ws.device)
    if deg is None:
        deg = torch.empty(n, dtype=torch.int32, device=ws.device)
    _ok(lib().nm_voronoi(ctypes.byref(ws.grid), ws.ptr, dmax, _dev(ring, torch.int32, n * dmax, "ring"),
                         _dev(deg, torch.int32, n, "deg"), _stream(ws.device)), "voronoi")
    return ring, deg


def voronoi_check(ws: Workspace, x, y, ring, deg, stale: torch.Tensor | None = None,
                  nfail: torch.Tensor | None = None):
    """The reuse test of rows (ring, deg) against positions x, y: (stale uint8 [n],
    nfail int32 [1] on the device; 0 means the rows are still exact)."""
    n = ws.n
    dmax = int(ring.shape[1])
    if stale is None:
        stale = torch.empty(n, dtype=torch.uint8, device=ws.device)
    if nfail is None:
        nfail = torch.empty(1, dtype=torch.int32, device=ws.device)
    _ok(lib().nm_voronoi_check(ctypes.byref(ws.grid), ws.ptr, _dev(x, torch.int32, n, "x"),
                               _dev(y, torch.int32, n, "y"), dmax, _dev(ring, torch.int32, n * dmax, "ring"),
                               _dev(deg, torch.int32, n, "deg"), _dev(stale, torch.uint8, n, "stale"),
                               _dev(nfail, torch.int32, 1, "nfail"), _stream(ws.device)), "voronoi_check")
    return stale, nfail


def voronoi_update(ws: Workspace, x, y, ring, deg, stale: torch.Tensor | None = None,
                   nfail: torch.Tensor | None = None):
    """Bring rows (ring, deg) up to date, in place, for positions x, y whose cells
    ws holds; returns nfail (device int32 [1]: particles that failed the first
    reuse test)."""
    n = ws.n
    dmax = int(ring.shape[1])
    if stale is None:
        stale = torch.empty(n, dtype=torch.uint8, device=ws.device)
    if nfail is None:
        nfail = torch.empty(1, dtype=torch.int32, device=ws.device)
    _ok(lib().nm_voronoi_update(ctypes.byref(ws.grid), ws.ptr, _dev(x, torch.int32, n, "x"),
                                _dev(y, torch.int32, n, "y"), dmax, _dev(ring, torch.int32, n * dmax, "ring"),
                                _dev(deg, torch.int32, n, "deg"), _dev(stale, torch.uint8, n, "stale"),
                                _dev(nfail, torch.int32, 1, "nfail"), _stream(ws.device)), "voronoi_update")
    return nfail


def voronoi_forces(x, y, box: int, ring, deg, ka: float, kp: float, a0: float, p0: float,
                   energy: bool = True, vertices: bool = False, ws: Workspace | None = None) -> dict:
    """Voronoi model (Sec. V) on the rows of voronoi(): device tensors area, perim,
    fx, fy [n] (fp64), energy [1] and, with vertices, [n, dmax, 4] (hx, hy, fx, fy)."""
    n = int(x.numel())
    dmax = int(ring.shape[1])
    dev = x.device
    out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("area", "perim", "fx", "fy")}
    out["energy"] = torch.empty(1, dtype=torch.float64, device=dev) if energy else None
    out["vertex"] = torch.empty((n, dmax, 4), dtype=torch.float64, device=dev) if vertices else None
    vp = VmParams(ka, kp, a0, p0)
    ptr = lambda t: t.data_ptr() if t is not None else None
    _ok(lib().nm_voronoi_forces(_dev(x, torch.int32, n, "x"), _dev(y, torch.int32, n, "y"), n, box, dmax,
                                _dev(ring, torch.int32, n * dmax, "ring"), _dev(deg, torch.int32, n, "deg"),
                                ctypes.byref(vp), ptr(out["area"]), ptr(out["perim"]), ptr(out["fx"]),
                                ptr(out["fy"]), ptr(out["energy"]), ptr(out["vertex"]),
                                ws.ptr if ws is not None else None, _stream(dev)), "voronoi_forces")
    return out


KNN_LAYOUT_FIELDS = ("kernel", "tw", "th", "hx", "hy", "bfix", "wide", "bmax", "ntx", "nty")


def knn_layout(n: int, box: int, cell_w: int, block: int, k: int) -> dict:
    """The strip layout nm_knn / nm_step run for this grid and k (host only)."""
    out = (_c_i32 * 10)()
    _ok(lib().nm_knn_layout(ctypes.byref(Grid(n, box, cell_w, block)), k, out), "knn_layout")
    return dict(zip(KNN_LAYOUT_FIELDS, [int(v) for v in out]))


def polar_order(theta: torch.Tensor, sums: torch.Tensor | None = None) -> float:
    """Polar order parameter |sum_i (cos, sin) theta_i| / n of device headings
    (synchronises to read it)."""
    n = int(theta.numel())
    if sums is None:
        sums = torch.empty(3, dtype=torch.float64, device=theta.device)
    _ok(lib().nm_polar_order(_dev(theta, torch.float32, n, "theta"), n,
                             _dev(sums, torch.float64, 3, "sums"), _stream(theta.device)), "polar_order")
    return float(sums[2].item())


class Workspace:
    """Device workspace of one system's cell grid (owned by torch)."""

    def __init__(self, n: int, box: int, cell_w: int | None = None, device="cuda", block: int = 0,
                 nbytes: int | None = None):
        if cell_w is None:
            cell_w = suggest_cell_w(n, box)
        self.grid = Grid(n, box, cell_w, block)
        need = int(lib().nm_workspace_bytes(ctypes.byref(self.grid)))
        if need < 0:
            raise NMError(need, f"workspace_bytes(n={n}, box={box}, cell_w={cell_w})")
        nbytes = max(need, int(nbytes or 0))
        self.device = torch.device(device)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.nbytes = nbytes
        _ok(lib().nm_workspace_init(ctypes.byref(self.grid), self.ptr, nbytes, _stream(self.device)),
            "workspace_init")

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()

    @property
    def n(self) -> int:
        return self.grid.n


def build_cells(ws: Workspace, x: torch.Tensor, y: torch.Tensor) -> None:
    n = ws.n
    _ok(lib().nm_build_cells(ctypes.byref(ws.grid), _dev(x, torch.int32, n, "x"),
                             _dev(y, torch.int32, n, "y"), ws.ptr, ws.nbytes, _stream(ws.device)),
        "build_cells")


def knn(ws: Workspace, k: int, nbr: torch.Tensor | None = None, d2: torch.Tensor | None = None,
        with_d2: bool = False):
    n = ws.n
    if nbr is None:
        nbr = torch.empty((n, k), dtype=torch.int32, device=ws.device)
    if with_d2 and d2 is None:
        d2 = torch.empty((n, k), dtype=torch.int64, device=ws.device)
    _ok(lib().nm_knn(ctypes.byref(ws.grid), ws.ptr, k, _dev(nbr, torch.int32, n * k, "nbr"),
                     _dev(d2, torch.int64, n * k, "d2") if d2 is not None else None,
                     _stream(ws.device)), "knn")
    return nbr, d2


def metric_list(ws: Workspace, rc2: int, offsets: torch.Tensor | None = None,
                idx: torch.Tensor | None = None, cap: int | None = None):
    """CSR metric lists.  Without idx: two-call protocol (count, allocate, fill),
    synchronising once.  With idx (capacity `cap`): one call, no synchronisation;
    an overflow is reported by check()."""
    n = ws.n
    if offsets is None:
        offsets = torch.empty(n + 1, dtype=torch.int32, device=ws.device)
    op = _dev(offsets, torch.int32, n + 1, "offsets")
    s = _stream(ws.device)
    if idx is None:
        nnz = _c_i64(0)
        _ok(lib().nm_metric_list(ctypes.byref(ws.grid), ws.ptr, rc2, op, None, 0, ctypes.byref(nnz), s),
            "metric_list(count)")
        idx = torch.empty(max(int(nnz.value), 1), dtype=torch.int32, device=ws.device)
        _ok(lib().nm_metric_list(ctypes.byref(ws.grid), ws.ptr, rc2, op, idx.data_ptr(), idx.numel(),
                                 ctypes.byref(nnz), s), "metric_list(fill)")
        return offsets, idx[:int(nnz.value)]
    cap = idx.numel() if cap is None else cap
    _ok(lib().nm_metric_list(ctypes.byref(ws.grid), ws.ptr, rc2, op, _dev(idx, torch.int32, cap, "idx"),
                             cap, None, s), "metric_list")
    return offsets, idx


def align_step(x, y, theta, params: Params, step: int, nbr=None, offsets=None, idx=None,
               out=None, ws: Workspace | None = None):
    """Eq. (2) + Eq. (1) for every particle from a fixed-k list (nbr [n, k]) or CSR
    (offsets [n+1], idx).  Returns (x', y', theta')."""
    n = int(x.numel())
    dev = x.device
    if out is None:
        out = (torch.empty_like(x), torch.empty_like(y), torch.empty_like(theta))
    xo, yo, to = out
    if offsets is not None:
        k, cap = 0, int(idx.numel())
        lst = _dev(idx, torch.int32, None, "idx") if cap else None
        offp = _dev(offsets, torch.int32, n + 1, "offsets")
    else:
        k = int(nbr.shape[1]) if nbr.dim() == 2 else int(nbr.numel() // max(n, 1))
        lst = _dev(nbr, torch.int32, n * k, "nbr") if k else None
        offp, cap = None, 0
    _ok(lib().nm_align_step(_dev(x, torch.int32, n, "x"), _dev(y, torch.int32, n, "y"),
                            _dev(theta, torch.float32, n, "theta"), n, lst, offp, k, cap,
                            ctypes.byref(params), step, _dev(xo, torch.int32, n, "x_out"),
                            _dev(yo, torch.int32, n, "y_out"), _dev(to, torch.float32, n, "theta_out"),
                            ws.ptr if ws is not None else None, _stream(dev)), "align_step")
    return xo, yo, to


def step(ws: Workspace, x, y, theta, k: int, params: Params, step_index: int, nbr, x_out, y_out,
         theta_out) -> None:
    """One fused step (Alg. 1): cells, k-NN lists, Eq. (2) and Eq. (1)."""
    n = ws.n
    _ok(lib().nm_step(ctypes.byref(ws.grid), _dev(x, torch.int32, n, "x"), _dev(y, torch.int32, n, "y"),
                      _dev(theta, torch.float32, n, "theta"), k, ctypes.byref(params), step_index,
                      ws.ptr, ws.nbytes, _dev(nbr, torch.int32, n * k, "nbr"),
                      _dev(x_out, torch.int32, n, "x_out"), _dev(y_out, torch.int32, n, "y_out"),
                      _dev(theta_out, torch.float32, n, "theta_out"), _stream(ws.device)), "step")


def bin_step(ws: Workspace, x, y, theta, params: Params, step_index: int) -> None:
    """First stage of step(): cell binning plus the per-particle noise word and
    fp64 heading unit vector for this step."""
    n = ws.n
    _ok(lib().nm_bin_step(ctypes.byref(ws.grid), _dev(x, torch.int32, n, "x"),
                          _dev(y, torch.int32, n, "y"), _dev(theta, torch.float32, n, "theta"),
                          ctypes.byref(params), step_index, ws.ptr, ws.nbytes, _stream(ws.device)),
        "bin_step")


def knn_align(ws: Workspace, k: int, params: Params, theta, nbr, x_out, y_out, theta_out) -> None:
    """Second stage of step(): k-NN lists fused with Eq. (2) and Eq. (1)."""
    n = ws.n
    _ok(lib().nm_knn_align(ctypes.byref(ws.grid), ws.ptr, k, ctypes.byref(params),
                           _dev(theta, torch.float32, n, "theta"), _dev(nbr, torch.int32, n * k, "nbr"),
                           _dev(x_out, torch.int32, n, "x_out"), _dev(y_out, torch.int32, n, "y_out"),
                           _dev(theta_out, torch.float32, n, "theta_out"), _stream(ws.device)),
        "knn_align")


def tune_grid(n: int, box: int, x, y, theta, k: int, params: Params, step_index: int = 0,
              cell_ws=None, blocks=(0,), reps: int = 5, device="cuda", ws: Workspace | None = None,
              pairs=None):
    """Time the one-system step over candidate grids (cell widths x block sides,
    or the given (w, block) pairs) on the given state; returns (Workspace set to
    the fastest grid, {(w, block): ms per step}).  An existing workspace is
    reused if it is large enough for every candidate."""
    if pairs is None:
        if cell_ws is None:
            cell_ws = sorted({suggest_cell_w(n, box, pc) for pc in (1.0, 2.0, 4.0)})
        pairs = [(w, b) for w in cell_ws for b in blocks]
    cands = [(int(w), int(b)) for w, b in pairs]
    arr = (Grid * len(cands))(*[Grid(n, box, w, b) for w, b in cands])
    need = max(int(lib().nm_workspace_bytes(ctypes.byref(g))) for g in arr)
    if ws is None or ws.nbytes < need:
        ws = Workspace(n, box, cands[0][0], device, block=cands[0][1], nbytes=need)
    dev = ws.device
    nbr = torch.empty(n * k, dtype=torch.int32, device=dev)
    xo, yo = torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev)
    to = torch.empty(n, dtype=torch.float32, device=dev)
    best, ms = _c_i32(), (ctypes.c_float * len(cands))()
    _ok(lib().nm_tune_grid(arr, len(cands), _dev(x, torch.int32, n, "x"), _dev(y, torch.int32, n, "y"),
                           _dev(theta, torch.float32, n, "theta"), k, ctypes.byref(params), step_index,
                           ws.ptr, ws.nbytes, nbr.data_ptr(), xo.data_ptr(), yo.data_ptr(), to.data_ptr(),
                           reps, ctypes.byref(best), ms, _stream(dev)), "tune_grid")
    w, b = cands[best.value]
    ws.grid = Grid(n, box, w, b)
    return ws, {c: float(m) for c, m in zip(cands, ms)}


def check(ws: Workspace) -> int:
    """Synchronise and return (and clear) the first device-side error, NM_OK if none."""
    return int(lib().nm_check(ws.ptr, _stream(ws.device)))


@dataclass
class System:
    """One simulated system resident on the device: double-buffered state,
    its workspace and its k-NN list."""
    ws: Workspace
    k: int
    params: Params
    x: torch.Tensor
    y: torch.Tensor
    theta: torch.Tensor
    nbr: torch.Tensor
    step_index: int = 0

    @classmethod
    def create(cls, x, y, theta, k: int, params: Params, cell_w: int | None = None, device="cuda",
               block: int = 0):
        n = int(len(x))
        dev = torch.device(device)
        ws = Workspace(n, params.box, cell_w, dev, block=block)
        t = lambda a, dt: torch.as_tensor(a, dtype=dt).to(dev).contiguous()
        sysm = cls(ws, k, params, t(x, torch.int32), t(y, torch.int32), t(theta, torch.float32),
                   torch.empty((n, k), dtype=torch.int32, device=dev))
        sysm._back = (torch.empty_like(sysm.x), torch.empty_like(sysm.y), torch.empty_like(sysm.theta))
        return sysm

    def step(self) -> None:
        xo, yo, to = self._back
        step(self.ws, self.x, self.y, self.theta, self.k, self.params, self.step_index, self.nbr,
             xo, yo, to)
        self._back = (self.x, self.y, self.theta)
        self.x, self.y, self.theta = xo, yo, to
        self.step_index += 1


class Batch:
    """Batched form (nm_batch_*): independent systems of uneven size in
    concatenated double-buffered arrays, advanced together on the device.

    x, y, theta: host or device arrays of the concatenated initial state
    (system s owns [offsets[s], offsets[s] + n[s])).  After t steps the state
    is in buffer t % 2 (see `current`)."""

    def __init__(self, n, x, y, theta, k: int, params: Params, sys_ids=None, device="cuda",
                 step0: int = 0):
        L = lib()
        self.device = torch.device(device)
        self.n = [int(v) for v in n]
        self.k = int(k)
        nsys = len(self.n)
        narr = (_c_i32 * nsys)(*self.n)
        ids = None if sys_ids is None else (_c_u32 * nsys)(*[int(v) for v in sys_ids])
        h, nbytes = _vp(), _c_i64()
        _ok(L.nm_batch_plan(nsys, narr, params.box, self.k, ctypes.byref(params), ids,
                            ctypes.byref(h), ctypes.byref(nbytes)), "batch_plan")
        self._h = h
        total = sum(self.n)
        self.offsets = [0]
        for v in self.n:
            self.offsets.append(self.offsets[-1] + v)
        t = lambda a, dt: torch.as_tensor(a, dtype=dt).to(self.device).contiguous()
        x0, y0, t0 = t(x, torch.int32), t(y, torch.int32), t(theta, torch.float32)
        if x0.numel() != total or y0.numel() != total or t0.numel() != total:
            raise ValueError(f"state arrays need {total} elements")
        self.x = [x0, torch.empty_like(x0)]
        self.y = [y0, torch.empty_like(y0)]
        self.theta = [t0, torch.empty_like(t0)]
        self.nbr = torch.empty(total * self.k, dtype=torch.int32, device=self.device)
        self.buf = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        io = BatchIO()
        for b in range(2):
            io.x[b], io.y[b], io.theta[b] = (self.x[b].data_ptr(), self.y[b].data_ptr(),
                                             self.theta[b].data_ptr())
        io.nbr = self.nbr.data_ptr()
        self._io = io
        _ok(L.nm_batch_bind(self._h, self.buf.data_ptr(), self.buf.numel(), ctypes.byref(io),
                            int(step0), _stream(self.device)), "batch_bind")

    def step(self, nsteps: int = 1, use_graph: bool = True) -> None:
        _ok(lib().nm_batch_step(self._h, int(nsteps), 1 if use_graph else 0, _stream(self.device)),
            "batch_step")

    def tune(self, reps: int = 3) -> None:
        _ok(lib().nm_batch_tune(self._h, int(reps), _stream(self.device)), "batch_tune")

    def set_block(self, block: int) -> None:
        """Every system's k-NN block choice (nm_grid.block), widths kept."""
        _ok(lib().nm_batch_set_block(self._h, int(block), _stream(self.device)), "batch_set_block")

    def grid(self, s: int) -> Grid:
        g, off = Grid(), _c_i32()
        _ok(lib().nm_batch_system(self._h, int(s), ctypes.byref(g), ctypes.byref(off)), "batch_system")
        return g

    @property
    def steps_done(self) -> int:
        return int(lib().nm_batch_steps_done(self._h))

    def current(self):
        """(x, y, theta) tensors holding the current state."""
        b = self.steps_done % 2
        return self.x[b], self.y[b], self.theta[b]

    def system(self, s: int):
        """Views (x, y, theta, nbr[n_s, k]) of system s's current state and last lists."""
        a, e = self.offsets[s], self.offsets[s + 1]
        x, y, th = self.current()
        return x[a:e], y[a:e], th[a:e], self.nbr[a * self.k:e * self.k].view(e - a, self.k)

    def check(self) -> int:
        return int(lib().nm_batch_check(self._h, _stream(self.device)))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            lib().nm_batch_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def server_job_bytes(n: int, k: int, box: int) -> int:
    """Admission (ledger) bytes of a served job."""
    return int(lib().nm_server_job_bytes(n, k, box))


class Server:
    """Served form (nm_server_*): jobs with host inputs, state resident on the
    device while they run, continuous batching under a device-memory budget."""

    def __init__(self, budget_bytes: int, max_slots: int = 1024):
        h = _vp()
        _ok(lib().nm_server_create(int(budget_bytes), int(max_slots), ctypes.byref(h)), "server_create")
        self._h = h
        self._shape = {}

    def submit(self, x, y, theta, k: int, nsteps: int, params: Params, want_nbr: bool = False) -> int:
        import numpy as np
        x = np.ascontiguousarray(x, dtype=np.int32)
        y = np.ascontiguousarray(y, dtype=np.int32)
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        n = int(x.size)
        if y.size != n or theta.size != n:
            raise ValueError("x, y, theta must have the same length")
        job = Job(n, int(k), int(nsteps), 1 if want_nbr else 0, params, x.ctypes.data, y.ctypes.data,
                  theta.ctypes.data)
        jid = _c_i64()
        _ok(lib().nm_server_submit(self._h, ctypes.byref(job), ctypes.byref(jid)), "server_submit")
        self._shape[int(jid.value)] = (n, int(k), bool(want_nbr))
        return int(jid.value)

    def poll(self, jid: int) -> bool:
        rc = int(lib().nm_server_poll(self._h, int(jid)))
        if rc < 0:
            raise NMError(rc, "server_poll")
        return rc == 1

    def wait(self, jid: int):
        """Final (x, y, theta[, nbr]) host arrays and the job's timing record."""
        import numpy as np
        n, k, want_nbr = self._shape.pop(int(jid))
        x = np.empty(n, np.int32)
        y = np.empty(n, np.int32)
        th = np.empty(n, np.float32)
        nbr = np.empty((n, k), np.int32) if want_nbr else None
        r = JobResult()
        rc = int(lib().nm_server_wait(self._h, int(jid), x.ctypes.data, y.ctypes.data, th.ctypes.data,
                                      nbr.ctypes.data if nbr is not None else None, ctypes.byref(r)))
        res = {"status": rc, "steps": r.steps, "submit_s": r.submit_s, "admit_s": r.admit_s,
               "done_s": r.done_s, "x": x, "y": y, "theta": th, "nbr": nbr}
        return res

    def stats(self) -> dict:
        info = ServerInfo()
        _ok(lib().nm_server_stats(self._h, ctypes.byref(info)), "server_stats")
        return {f: getattr(info, f) for f, _ in ServerInfo._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().nm_server_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
