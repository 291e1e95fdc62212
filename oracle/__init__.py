"""Brute-force CPU oracle for the non-metric neighbour lists and Vicsek step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The GPU library
never imports, links or calls it, and it shares no code with the GPU path.

The arithmetic lives in ``nm_oracle.c`` (plain C, fp64, OpenMP over rows);
this module only marshals numpy arrays through ctypes.  What each function
computes, with the passage of arXiv:2103.10239 it follows:

- ``knn``: the topological rule of Sec. III -- the k nearest neighbours of
  every particle, by evaluating all N^2 pairs (the naive cost named in
  Sec. I), ordered by (squared minimum-image distance, index).
- ``metric_list``: the metric rule of Sec. III -- every j with distance at
  most r_0, as CSR rows ordered the same way.
- ``align_step``: Eq. (2) (alignment with vectorial noise, normalised) and
  Eq. (1) (Euler move with the heading at time t), in fp64.
- ``voronoi``: the Delaunay rule of Sec. III / Sec. IV -- i and j are
  neighbours when their Voronoi cells share an edge, decided pair by pair by
  an exact test on their bisector against every other particle; rows in
  counter-clockwise order.
- ``voronoi_forces``: the Voronoi model of Sec. V -- cell areas and
  perimeters, the energy of Eq. (3), vertex forces (Eqs. 5-8) and particle
  forces (Eqs. 9-19), fp64.
- ``philox4x32_10`` / ``noise_word`` / ``noise_angle``: the counter-based
  generator (Salmon et al., SC'11) that supplies the random unit vector of
  Eq. (2).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, E_INVAL, E_RANGE, E_CAPACITY, E_NOMEM = 0, -1, -2, -3, -4

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_vp = ctypes.c_void_p


class OracleError(RuntimeError):
    def __init__(self, msg: str, status: int = 0):
        super().__init__(msg)
        self.status = status


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build  # noqa: F401  (build on first use)
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    lib.orc_philox4x32_10.restype = None
    lib.orc_noise_word.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64]
    lib.orc_noise_word.restype = ctypes.c_uint32
    lib.orc_noise_angle.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64]
    lib.orc_noise_angle.restype = ctypes.c_double
    lib.orc_d2.argtypes = [ctypes.c_int32] * 5
    lib.orc_d2.restype = ctypes.c_int64
    lib.orc_knn.argtypes = [_i32p, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                            _vp, ctypes.c_int32, _i32p, _vp]
    lib.orc_knn.restype = ctypes.c_int
    lib.orc_metric_count.argtypes = [_i32p, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                     _vp, ctypes.c_int32, _i64p]
    lib.orc_metric_count.restype = ctypes.c_int
    lib.orc_metric_fill.argtypes = [_i32p, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                    _vp, ctypes.c_int32, _i64p, _i32p, _vp]
    lib.orc_metric_fill.restype = ctypes.c_int
    lib.orc_align_step.argtypes = [_i32p, _i32p, _f32p, ctypes.c_int32, ctypes.c_int32,
                                   _i32p, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                   ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint64,
                                   _vp, ctypes.c_int32, _i32p, _i32p, _f32p, ctypes.c_uint32]
    lib.orc_align_step.restype = ctypes.c_int
    lib.orc_knn_fov.argtypes = [_i32p, _i32p, _f32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, _vp, ctypes.c_int32, _i32p]
    lib.orc_knn_fov.restype = ctypes.c_int
    lib.orc_fov_visible.argtypes = [ctypes.c_int64] * 4 + [ctypes.c_int32]
    lib.orc_fov_visible.restype = ctypes.c_int
    lib.orc_polar_order.argtypes = [_f32p, ctypes.c_int32]
    lib.orc_polar_order.restype = ctypes.c_double
    lib.orc_voronoi.argtypes = [_i32p, _i32p, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int32,
                                ctypes.c_int32, _i32p, _i32p]
    lib.orc_voronoi.restype = ctypes.c_int
    lib.orc_voronoi_local.argtypes = [_i32p, _i32p, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, _i32p, _i32p]
    lib.orc_voronoi_local.restype = ctypes.c_int
    _f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
    lib.orc_voronoi_forces.argtypes = [_f64p, _f64p, ctypes.c_int32, ctypes.c_double, _i64p, _i32p] + \
        [ctypes.c_double] * 4 + [_vp, ctypes.c_int32] + [_vp] * 9
    lib.orc_voronoi_forces.restype = ctypes.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != OK:
        raise OracleError(f"{what}: oracle status {rc}", rc)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _rows_arg(rows, n):
    if rows is None:
        return None, n, None
    r = _i32(rows)
    return r.ctypes.data_as(_vp), int(r.size), r


def num_threads() -> int:
    """OpenMP threads the oracle runs on."""
    return int(_load().orc_num_threads())


def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block: 4 counter words, 2 key words -> 4 words."""
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(np.asarray(ctr, dtype=np.uint32), np.asarray(key, dtype=np.uint32), out)
    return out


def noise_word(seed: int, sys_id: int, step: int, i: int) -> int:
    return int(_load().orc_noise_word(seed, sys_id, step, i))


def noise_angle(seed: int, sys_id: int, step: int, i: int) -> float:
    return float(_load().orc_noise_angle(seed, sys_id, step, i))


def d2(xa: int, ya: int, xb: int, yb: int, box: int) -> int:
    return int(_load().orc_d2(xa, ya, xb, yb, box))


def knn(x, y, box: int, k: int, rows=None, with_d2: bool = True):
    """k nearest neighbours (Sec. III), brute force.  Returns (nbr, d2)."""
    x, y = _i32(x), _i32(y)
    n = int(x.size)
    rp, nr, _keep = _rows_arg(rows, n)
    nbr = np.zeros(nr * k, dtype=np.int32)
    dd = np.zeros(nr * k, dtype=np.int64) if with_d2 else None
    rc = _load().orc_knn(x, y, n, box, k, rp, nr, nbr, dd.ctypes.data_as(_vp) if with_d2 else None)
    _check(rc, "knn")
    return nbr.reshape(nr, k), (dd.reshape(nr, k) if with_d2 else None)


def metric_list(x, y, box: int, rc2: int, rows=None, with_d2: bool = True):
    """Metric neighbour lists (Sec. III) as CSR.  Returns (offsets int64[n+1], idx, d2)."""
    x, y = _i32(x), _i32(y)
    n = int(x.size)
    rp, nr, _keep = _rows_arg(rows, n)
    counts = np.zeros(nr, dtype=np.int64)
    _check(_load().orc_metric_count(x, y, n, box, rc2, rp, nr, counts), "metric_count")
    offsets = np.zeros(nr + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    nnz = int(offsets[-1])
    idx = np.zeros(max(nnz, 1), dtype=np.int32)
    dd = np.zeros(max(nnz, 1), dtype=np.int64) if with_d2 else None
    rc = _load().orc_metric_fill(x, y, n, box, rc2, rp, nr, offsets, idx,
                                 dd.ctypes.data_as(_vp) if with_d2 else None)
    _check(rc, "metric_fill")
    return offsets, idx[:nnz], (dd[:nnz] if with_d2 else None)


def align_step(x, y, theta, box: int, nbr=None, offsets=None, idx=None, *, v0: int, eta: float,
               seed: int, sys_id: int = 0, include_self: int = 1, step: int = 0, rows=None,
               variant: int = 0):
    """Eq. (2) then Eq. (1) for each listed particle, fp64 (variant bit 0:
    angular noise; bit 1: move with the new heading).

    Neighbour lists are either ``nbr`` (int32[rows, k]) or CSR ``offsets`` +
    ``idx``.  Returns (x', y', theta') for the listed rows.
    """
    x, y = _i32(x), _i32(y)
    theta = np.ascontiguousarray(theta, dtype=np.float32)
    n = int(x.size)
    rp, nr, _keep = _rows_arg(rows, n)
    if offsets is not None:
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        lst = _i32(idx) if idx is not None and len(idx) else np.zeros(1, dtype=np.int32)
        offp, k = offs.ctypes.data_as(_vp), 0
    else:
        nb = _i32(nbr)
        k = int(nb.shape[1]) if nb.ndim == 2 else int(nb.size // max(nr, 1))
        lst = nb.reshape(-1) if nb.size else np.zeros(1, dtype=np.int32)
        offp, offs = None, None
    xo = np.zeros(nr, dtype=np.int32)
    yo = np.zeros(nr, dtype=np.int32)
    to = np.zeros(nr, dtype=np.float32)
    rc = _load().orc_align_step(x, y, theta, n, box, lst, offp, k, v0, eta, seed, sys_id,
                                include_self, step, rp, nr, xo, yo, to, variant)
    _check(rc, "align_step")
    return xo, yo, to


def knn_fov(x, y, theta, box: int, k: int, cos_q: int, rows=None):
    """Field-of-view k-NN: the k nearest (by (d^2, j)) among the particles inside
    the cone cos(alpha) = cos_q / 4096 around each heading.  Returns (nbr int32
    [rows, k], ok); rows with fewer than k visible particles are padded with -1
    and ok is False."""
    x, y = _i32(x), _i32(y)
    theta = np.ascontiguousarray(theta, dtype=np.float32)
    n = int(x.size)
    rp, nr, _keep = _rows_arg(rows, n)
    nbr = np.zeros((nr, k), dtype=np.int32)
    rc = _load().orc_knn_fov(x, y, theta, n, box, k, cos_q, rp, nr, nbr)
    if rc == -2 and check_coords_ok(x, y, box):
        return nbr, False
    _check(rc, "knn_fov")
    return nbr, True


def check_coords_ok(x, y, box: int) -> bool:
    return bool(((x >= 0) & (x < box) & (y >= 0) & (y < box)).all())


def fov_visible(dx: int, dy: int, hx: int, hy: int, cos_q: int) -> bool:
    """The cone test of knn_fov for one displacement and heading vector."""
    return bool(_load().orc_fov_visible(dx, dy, hx, hy, cos_q))


def polar_order(theta) -> float:
    """Polar order parameter |sum_i (cos, sin) theta_i| / N, fp64 in index order."""
    th = np.ascontiguousarray(theta, dtype=np.float32)
    return float(_load().orc_polar_order(th, int(th.size)))


def step(x, y, theta, box: int, k: int, *, v0: int, eta: float, seed: int, sys_id: int = 0,
         include_self: int = 1, step_index: int = 0, variant: int = 0):
    """One full step of the fundamental loop (Alg. 1) in the topological model:
    rebuild the k-NN lists from r(t), then Eq. (2) and Eq. (1) from time-t state."""
    nbr, _ = knn(x, y, box, k, with_d2=False)
    xo, yo, to = align_step(x, y, theta, box, nbr=nbr, v0=v0, eta=eta, seed=seed, sys_id=sys_id,
                            include_self=include_self, step=step_index, variant=variant)
    return nbr, xo, yo, to


def voronoi(x, y, box: int, rows=None, dmax: int = 64, rho0: int | None = None):
    """Voronoi (Delaunay) neighbour rows, counter-clockwise from the +x axis.

    Returns (offsets int64[rows + 1], idx int32[nnz]).  rows=None: every
    particle, by the bisector test against all others.  With rows and rho0:
    the same rows from the particles within a radius that starts at rho0 and
    doubles until every cell vertex lies within half of it (for sampled rows
    of large systems).  Raises OracleError (status E_RANGE) for coincident
    particles or a cell vertex L/8 or more from its particle."""
    x, y = _i32(x), _i32(y)
    n = int(x.size)
    rp, nr, _keep = _rows_arg(rows, n)
    ring = np.zeros(nr * dmax, dtype=np.int32)
    deg = np.zeros(nr, dtype=np.int32)
    if rho0 is not None:
        if rows is None:
            raise ValueError("rho0 needs rows")
        rc = _load().orc_voronoi_local(x, y, n, box, rp, nr, int(rho0), dmax, ring, deg)
    else:
        rc = _load().orc_voronoi(x, y, n, box, rp, nr, dmax, ring, deg)
    _check(rc, "voronoi")
    offsets = np.zeros(nr + 1, dtype=np.int64)
    np.cumsum(deg, out=offsets[1:])
    ring = ring.reshape(nr, dmax)
    idx = np.concatenate([ring[r, :deg[r]] for r in range(nr)]) if nr else np.zeros(0, np.int32)
    return offsets, idx.astype(np.int32)


def voronoi_forces(x, y, box, offsets, idx, ka: float, kp: float, a0: float, p0: float,
                   vertices: bool = False, rows=None) -> dict:
    """Voronoi model (Sec. V) on the rings (offsets, idx) of every particle, at
    real positions x, y in a periodic box: area, perimeter, force (fx, fy) per
    particle, the energy of Eq. (3), and with vertices=True per ring slot the
    vertex h (relative to its particle) and the vertex force -dE/dh.  With
    rows, only those particles' forces (fx[r] for rows[r]); rows of fewer than
    three entries then mark particles without a cell (NaN areas)."""
    xd = np.ascontiguousarray(x, dtype=np.float64)
    yd = np.ascontiguousarray(y, dtype=np.float64)
    n = int(xd.size)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    ix = _i32(idx) if len(idx) else np.zeros(1, np.int32)
    nnz = int(off[-1])
    rp, nr, _keep = _rows_arg(rows, n)
    out = {k: np.zeros(n) for k in ("area", "perim")}
    out.update({k: np.zeros(nr) for k in ("fx", "fy")})
    e = np.zeros(1)
    vk = ("hx", "hy", "vfx", "vfy")
    if vertices:
        out.update({k: np.zeros(nnz) for k in vk})
    ptr = lambda a: a.ctypes.data_as(_vp)
    rc = _load().orc_voronoi_forces(xd, yd, n, float(box), off, ix, ka, kp, a0, p0, rp, nr, ptr(out["area"]),
                                    ptr(out["perim"]), ptr(out["fx"]), ptr(out["fy"]), ptr(e),
                                    *[ptr(out[k]) if vertices else None for k in vk])
    _check(rc, "voronoi_forces")
    out["energy"] = float(e[0]) if rows is None else None
    return out
