"""Parity of every grid the throughput benchmark can time.

The N = 2^20 benchmark step runs on a grid (cell width, block side) that the
grid tuner picks on the initial state among {1024, 2048} x {0, 4, 6}, and
re-picks every 200 steps among the current grid and cell widths 512-4096 with
block 0; the step-variant benchmark runs (2048, 4).  Each grid selects one
strip layout of the k-NN kernel (strip width, halo, fixed block, 16- or
32-bit staged offsets).  For each of these grids this file checks:

- a reduced system with the same strip layout (same density and cell width,
  box 2^18, N = 2^16; the layout is read back through nm_knn_layout and must
  equal the benchmark's) compared with the brute-force oracle over every
  particle: lists, squared distances and the fused step;
- the full N = 2^20 trajectory of the benchmark (uniform start, Philox
  seed 0, 20 steps), where the 21st step is compared with the oracle on
  sampled particles from the device state, and every row's squared distances
  are compared with scipy's periodic k-d tree (an independent library).

The clustered N = 2^22 benchmark grids (cell width 1024, block 0, both strip
kernels) are checked on sampled rows at the end of this file.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2103_10239_amd as nm
from paper_2103_10239_amd import workloads

pytestmark = pytest.mark.gpu
L = workloads.BOX
N = 1 << 20
K = 7
TOL = 1e-5
S = nm.NM_BLOCK_SUBSTRIPS

# (cell width, block) of every grid the N = 2^20 benchmarks can time
HEADLINE_GRIDS = [(1024, 0), (1024, 4), (1024, 6), (2048, 0), (2048, 4), (2048, 6), (512, 0), (4096, 0)]
SIGNATURE = ("kernel", "tw", "hx", "hy", "bfix", "wide", "bmax")


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).to("cuda")


def _angle_err(a, b):
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return np.abs(np.remainder(d + np.pi, 2 * np.pi) - np.pi)


def _sig(n, box, w, block, k=K):
    lay = nm.knn_layout(n, box, w, block, k)
    return tuple(lay[f] for f in SIGNATURE)


def test_headline_grid_layout_is_the_narrow_fixed_block_strip():
    # the grid the benchmark picked on the driver's run: narrow 16-bit strips,
    # two columns, halo 3 x 4, fixed block 6, default kernel
    lay = nm.knn_layout(N, L, 1024, 6, K)
    assert (lay["kernel"], lay["tw"], lay["hx"], lay["hy"], lay["bfix"], lay["wide"]) == (1, 2, 3, 4, 6, 0)


@pytest.mark.parametrize("w,block", HEADLINE_GRIDS)
def test_reduced_system_with_the_benchmark_layout_matches_oracle(w, block):
    box_s, n_s = 1 << 18, N >> 4  # same particles per cell and cell width
    assert _sig(n_s, box_s, w, block) == _sig(N, L, w, block)
    x, y, th = workloads.uniform(n_s, box=box_s, seed_pos=100 + w + block)
    ws = nm.Workspace(n_s, box_s, w, block=block)
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    nbr, d2 = nm.knn(ws, K, with_d2=True)
    assert nm.check(ws) == 0
    rn, rd = oracle.knn(x, y, box_s, K)
    assert np.array_equal(nbr.cpu().numpy(), rn) and np.array_equal(d2.cpu().numpy(), rd)
    for variant in (0, nm.NM_NOISE_SCALAR | nm.NM_MOVE_NEW_HEADING):
        p = nm.make_params(box_s, v0=64, eta=0.2, seed=workloads.NOISE_SEED, variant=variant)
        sysm = nm.System.create(x, y, th, K, p, cell_w=w, block=block)
        sysm.step()
        assert nm.check(sysm.ws) == 0
        sx, sy, st = oracle.align_step(x, y, th, box_s, nbr=rn, v0=64, eta=0.2, seed=workloads.NOISE_SEED,
                                       variant=variant)
        assert np.array_equal(sysm.nbr.cpu().numpy(), rn)
        assert np.array_equal(sysm.x.cpu().numpy(), sx) and np.array_equal(sysm.y.cpu().numpy(), sy)
        assert _angle_err(sysm.theta.cpu().numpy(), st).max() <= TOL


def _min_image_d2(x, y, nbr, box):
    xi = x.astype(np.int64)[:, None]
    yi = y.astype(np.int64)[:, None]
    dx = x.astype(np.int64)[nbr] - xi
    dy = y.astype(np.int64)[nbr] - yi
    dx = (dx + box // 2) % box - box // 2
    dy = (dy + box // 2) % box - box // 2
    return dx * dx + dy * dy


def _kdtree_d2(x, y, k, box):
    """Squared distances of the k nearest others of every particle (scipy's
    periodic k-d tree; exact after rounding, since d^2 < 2^41)."""
    from scipy.spatial import cKDTree

    pts = np.stack([x, y], axis=1).astype(np.float64)
    tree = cKDTree(pts, boxsize=float(box))
    dist, _ = tree.query(pts, k=k + 1, workers=16)
    d2 = np.rint(dist * dist).astype(np.int64)
    # drop one zero (the particle itself; a coincident partner keeps its zero)
    return d2[:, 1:]


@pytest.mark.parametrize("w,block", HEADLINE_GRIDS)
def test_benchmark_trajectory_on_each_grid(w, block):
    x, y, th = workloads.uniform(N)
    p = nm.make_params(L, v0=64, eta=0.2, include_self=1, seed=workloads.NOISE_SEED)
    sysm = nm.System.create(x, y, th, K, p, cell_w=w, block=block)
    for _ in range(20):
        sysm.step()
    assert nm.check(sysm.ws) == 0
    sx, sy, st = sysm.x.cpu().numpy(), sysm.y.cpu().numpy(), sysm.theta.cpu().numpy()
    t = sysm.step_index
    sysm.step()
    assert nm.check(sysm.ws) == 0
    nbr = sysm.nbr.cpu().numpy()
    # every row: sorted keys, no self, and the k nearest distances
    d2 = _min_image_d2(sx, sy, nbr, L)
    assert (nbr != np.arange(N)[:, None]).all()
    key = d2 * (1 << 24) + nbr
    assert (key[:, 1:] > key[:, :-1]).all()
    assert np.array_equal(d2, _kdtree_d2(sx, sy, K, L))
    # sampled rows: indices, positions and headings against the oracle
    rows = np.unique(np.concatenate([np.random.default_rng(w + block).integers(0, N, 600), [0, N - 1]]))
    rows = rows.astype(np.int32)
    rn, _ = oracle.knn(sx, sy, L, K, rows=rows, with_d2=False)
    assert np.array_equal(nbr[rows], rn)
    rx, ry, rt = oracle.align_step(sx, sy, st, L, nbr=rn, v0=64, eta=0.2, seed=workloads.NOISE_SEED,
                                   rows=rows, step=t)
    sel = torch.as_tensor(rows).long().cuda()
    assert np.array_equal(sysm.x[sel].cpu().numpy(), rx) and np.array_equal(sysm.y[sel].cpu().numpy(), ry)
    assert _angle_err(sysm.theta[sel].cpu().numpy(), rt).max() <= TOL


@pytest.mark.parametrize("block", [0, S])
@pytest.mark.parametrize("k", [6, 12, 20])
def test_clustered_benchmark_grid_every_row_distance(k, block):
    # the clustered N = 2^22 benchmark's grid: w = 1024 (per-query blocks),
    # either strip kernel; every row's distances against the k-d tree, and
    # sampled rows against the oracle
    n = 1 << 22
    x, y, th = workloads.clustered(n)
    p = nm.make_params(L, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    sysm = nm.System.create(x, y, th, k, p, cell_w=1024, block=block)
    sysm.step()
    assert nm.check(sysm.ws) == 0
    nbr = sysm.nbr.cpu().numpy()
    d2 = _min_image_d2(x, y, nbr, L)
    key = d2 * (1 << 24) + nbr
    assert (key[:, 1:] > key[:, :-1]).all()
    assert np.array_equal(d2, _kdtree_d2(x, y, k, L))
    rows = np.unique(np.random.default_rng(k + block).integers(0, n, 300)).astype(np.int32)
    rn, _ = oracle.knn(x, y, L, k, rows=rows, with_d2=False)
    assert np.array_equal(nbr[rows], rn)
