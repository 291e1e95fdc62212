"""Parity of the HIP path (through the C ABI) with the brute-force oracle.

Bar: neighbour lists, squared distances, CSR metric lists and positions
bit-exact; headings within 1e-5 rad (one step from the same state).  Small
and mid sizes are compared element by element over every particle (spanning
many 256-lane tiles, with ragged tails); the full benchmark sizes are
compared on sampled rows that the oracle brute-forces one by one, plus
invariants checked over every row on the device.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2103_10239_amd as nm
from paper_2103_10239_amd import workloads

pytestmark = pytest.mark.gpu
L = workloads.BOX
TOL = 1e-5


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).to("cuda")


def _angle_err(a, b):
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return np.abs(np.remainder(d + np.pi, 2 * np.pi) - np.pi)


def _gen(kind, n):
    if kind == "uniform":
        return workloads.uniform(n)
    if kind == "clustered":
        return workloads.clustered(n)
    if kind == "squeezed":  # many exact duplicates and distance ties
        x, y, th = workloads.uniform(n)
        return (x % 7) * 1000, (y % 5) * 1000, th
    raise ValueError(kind)


def _gpu_knn(x, y, k, w):
    ws = nm.Workspace(len(x), L, w)
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    nbr, d2 = nm.knn(ws, k, with_d2=True)
    assert nm.check(ws) == 0
    return nbr.cpu().numpy(), d2.cpu().numpy(), ws


KNN_CASES = [
    ("uniform", 1024, 7, 2048), ("uniform", 1024, 7, 1024), ("uniform", 1024, 7, L),
    ("uniform", 1024, 7, L // 2), ("uniform", 1024, 7, 256), ("uniform", 2, 1, L // 4),
    ("uniform", 3, 2, 1024), ("uniform", 33, 32, 4096), ("uniform", 257, 1, 8192),
    ("uniform", 4097, 12, 2048), ("uniform", 20013, 20, 2048), ("uniform", 20013, 32, 4096),
    ("clustered", 8191, 6, 2048), ("clustered", 8191, 12, 1024), ("clustered", 20013, 20, 4096),
    ("squeezed", 3000, 7, 1024), ("squeezed", 3000, 16, 4096),
]


@pytest.mark.parametrize("kind,n,k,w", KNN_CASES)
def test_knn_matches_oracle(kind, n, k, w):
    x, y, _ = _gen(kind, n)
    nbr, d2, _ = _gpu_knn(x, y, k, w)
    rn, rd = oracle.knn(x, y, L, k)
    assert np.array_equal(nbr, rn)
    assert np.array_equal(d2, rd)


@pytest.mark.parametrize("k", [1, 4, 7, 8])
@pytest.mark.parametrize("wdiv", [1, 2, 4])
def test_knn_lattice_ties(k, wdiv):
    x, y, a = workloads.lattice(32)
    nbr, d2, _ = _gpu_knn(x, y, k, a // wdiv if wdiv > 1 else a)
    rn, rd = oracle.knn(x, y, L, k)
    assert np.array_equal(nbr, rn) and np.array_equal(d2, rd)


def test_knn_all_coincident():
    n = 33
    nbr, d2, _ = _gpu_knn([777] * n, [4242] * n, 32, 1024)
    assert not d2.any()
    for i in range(n):
        assert nbr[i].tolist() == [j for j in range(n) if j != i]


def test_knn_wrap_pair():
    nbr, d2, _ = _gpu_knn([0, L - 1], [5, 5], 1, 1024)
    assert nbr.tolist() == [[1], [0]] and d2.tolist() == [[1], [1]]


def _gpu_metric(x, y, rc2, w):
    ws = nm.Workspace(len(x), L, w)
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    offs, idx = nm.metric_list(ws, rc2)
    assert nm.check(ws) == 0
    return offs.cpu().numpy().astype(np.int64), idx.cpu().numpy()


@pytest.mark.parametrize("kind,n,mean,w", [("uniform", 4097, 7.0, 1024), ("uniform", 4097, 7.0, 4096),
                                           ("clustered", 8191, 3.0, 2048), ("squeezed", 3000, 1.0, 1024),
                                           ("uniform", 2, 1.0, L // 4)])
def test_metric_matches_oracle(kind, n, mean, w):
    x, y, _ = _gen(kind, n)
    rc2 = workloads.rc2_for_mean(n, mean)
    offs, idx = _gpu_metric(x, y, rc2, w)
    ro, ri, _ = oracle.metric_list(x, y, L, rc2)
    assert np.array_equal(offs, ro)
    assert np.array_equal(idx, ri)


@pytest.mark.parametrize("shell", [(1, 0), (1, -1), (2, 0), (0, 0)])
def test_metric_lattice_shells(shell):
    x, y, a = workloads.lattice(32)
    rc2 = shell[0] * a * a + shell[1]
    offs, idx = _gpu_metric(x, y, rc2, a)
    ro, ri, _ = oracle.metric_list(x, y, L, rc2)
    assert np.array_equal(offs, ro) and np.array_equal(idx, ri)


def test_metric_long_rows_use_several_chunks():
    # 60 coincident points plus a far group: rows of 59 entries need four selection passes.
    x = np.array([1000] * 60 + list(range(500000, 500040)), np.int32)
    y = np.array([2000] * 60 + [7] * 40, np.int32)
    offs, idx = _gpu_metric(x, y, 50 ** 2, 1024)
    ro, ri, _ = oracle.metric_list(x, y, L, 50 ** 2)
    assert np.array_equal(offs, ro) and np.array_equal(idx, ri)


@pytest.mark.parametrize("include_self", [0, 1])
@pytest.mark.parametrize("eta,seed,step,sys_id", [(0.2, 0, 0, 0), (0.7, (1 << 40) + 5, (1 << 33) + 9, 3),
                                                  (0.0, 1, 2, 0)])
def test_align_step_matches_oracle(include_self, eta, seed, step, sys_id):
    n, k = 4097, 7
    x, y, th = workloads.uniform(n)
    rn, _ = oracle.knn(x, y, L, k)
    p = nm.make_params(L, v0=64, eta=eta, include_self=include_self, seed=seed, sys_id=sys_id)
    xo, yo, to = nm.align_step(_dev(x, torch.int32), _dev(y, torch.int32), _dev(th, torch.float32), p,
                               step, nbr=_dev(rn, torch.int32))
    torch.cuda.synchronize()
    rx, ry, rt = oracle.align_step(x, y, th, L, nbr=rn, v0=64, eta=eta, seed=seed, sys_id=sys_id,
                                   include_self=include_self, step=step)
    assert np.array_equal(xo.cpu().numpy(), rx) and np.array_equal(yo.cpu().numpy(), ry)
    assert _angle_err(to.cpu().numpy(), rt).max() <= TOL


@pytest.mark.parametrize("include_self", [0, 1])
def test_align_step_metric_mode(include_self):
    n = 4097
    x, y, th = workloads.clustered(n)
    rc2 = workloads.rc2_for_mean(n, 2.0)
    ro, ri, _ = oracle.metric_list(x, y, L, rc2)
    assert (np.diff(ro) == 0).any()  # some isolated particles
    p = nm.make_params(L, v0=-37, eta=0.3, include_self=include_self, seed=12)
    ws = nm.Workspace(n, L, 2048)
    xo, yo, to = nm.align_step(_dev(x, torch.int32), _dev(y, torch.int32), _dev(th, torch.float32), p, 5,
                               offsets=_dev(ro, torch.int32), idx=_dev(ri, torch.int32), ws=ws)
    assert nm.check(ws) == 0
    rx, ry, rt = oracle.align_step(x, y, th, L, offsets=ro, idx=ri, v0=-37, eta=0.3, seed=12,
                                   include_self=include_self, step=5)
    assert np.array_equal(xo.cpu().numpy(), rx) and np.array_equal(yo.cpu().numpy(), ry)
    assert _angle_err(to.cpu().numpy(), rt).max() <= TOL


@pytest.mark.parametrize("variant", [nm.NM_NOISE_SCALAR, nm.NM_MOVE_NEW_HEADING,
                                     nm.NM_NOISE_SCALAR | nm.NM_MOVE_NEW_HEADING])
@pytest.mark.parametrize("include_self,eta", [(1, 0.2), (0, 1.0), (1, 0.0)])
def test_align_step_variants_match_oracle(variant, include_self, eta):
    n, k = 4097, 7
    x, y, th = workloads.clustered(n)
    rn, _ = oracle.knn(x, y, L, k)
    p = nm.make_params(L, v0=64, eta=eta, include_self=include_self, seed=77, sys_id=2, variant=variant)
    xo, yo, to = nm.align_step(_dev(x, torch.int32), _dev(y, torch.int32), _dev(th, torch.float32), p,
                               4, nbr=_dev(rn, torch.int32))
    torch.cuda.synchronize()
    rx, ry, rt = oracle.align_step(x, y, th, L, nbr=rn, v0=64, eta=eta, seed=77, sys_id=2,
                                   include_self=include_self, step=4, variant=variant)
    assert np.array_equal(xo.cpu().numpy(), rx) and np.array_equal(yo.cpu().numpy(), ry)
    assert _angle_err(to.cpu().numpy(), rt).max() <= TOL
    # metric mode, with isolated particles (empty rows)
    rc2 = workloads.rc2_for_mean(n, 2.0)
    ro, ri, _ = oracle.metric_list(x, y, L, rc2)
    xo, yo, to = nm.align_step(_dev(x, torch.int32), _dev(y, torch.int32), _dev(th, torch.float32), p, 4,
                               offsets=_dev(ro, torch.int32), idx=_dev(ri, torch.int32))
    torch.cuda.synchronize()
    rx, ry, rt = oracle.align_step(x, y, th, L, offsets=ro, idx=ri, v0=64, eta=eta, seed=77, sys_id=2,
                                   include_self=include_self, step=4, variant=variant)
    assert np.array_equal(xo.cpu().numpy(), rx) and np.array_equal(yo.cpu().numpy(), ry)
    assert _angle_err(to.cpu().numpy(), rt).max() <= TOL


@pytest.mark.parametrize("variant", [nm.NM_NOISE_SCALAR, nm.NM_MOVE_NEW_HEADING,
                                     nm.NM_NOISE_SCALAR | nm.NM_MOVE_NEW_HEADING])
@pytest.mark.parametrize("kind,n,w", [("uniform", 4097, 2048), ("clustered", (1 << 17) + 3, 1024)])
@pytest.mark.parametrize("block", [0, nm.NM_BLOCK_SUBSTRIPS])
def test_fused_step_variants_match_oracle(variant, kind, n, w, block):
    k = 7
    x, y, th = _gen(kind, n) if kind == "uniform" else workloads.clustered(n)
    p = nm.make_params(L, v0=64, eta=0.4, seed=workloads.NOISE_SEED, variant=variant)
    sysm = nm.System.create(x, y, th, k, p, cell_w=w, block=block)
    sysm.step()
    assert nm.check(sysm.ws) == 0
    rows = None if n < 10000 else np.concatenate([_sample_rows(n, 400, 3), [0, n - 1]]).astype(np.int32)
    rn, _ = oracle.knn(x, y, L, k, rows=rows, with_d2=False)
    rx, ry, rt = oracle.align_step(x, y, th, L, nbr=rn, v0=64, eta=0.4, seed=workloads.NOISE_SEED,
                                   rows=rows, variant=variant)
    sel = torch.arange(n, device="cuda") if rows is None else torch.as_tensor(rows).long().cuda()
    assert np.array_equal(sysm.nbr[sel].cpu().numpy(), rn)
    assert np.array_equal(sysm.x[sel].cpu().numpy(), rx) and np.array_equal(sysm.y[sel].cpu().numpy(), ry)
    assert _angle_err(sysm.theta[sel].cpu().numpy(), rt).max() <= TOL


@pytest.mark.parametrize("n", [1, 1000, 100003, 1 << 20])
def test_polar_order_matches_oracle(n):
    rng = np.random.default_rng(n)
    for th in (rng.uniform(-np.pi, np.pi, n).astype(np.float32),
               (0.3 + 0.05 * rng.standard_normal(n)).astype(np.float32)):
        got = nm.polar_order(_dev(th, torch.float32))
        ref = oracle.polar_order(th)
        assert abs(got - ref) <= 1e-12 * max(1.0, ref) + 1e-13
    assert abs(nm.polar_order(_dev(np.full(n, -1.1, np.float32), torch.float32)) - 1.0) < 1e-12


@pytest.mark.parametrize("kind,n,k,w", [("uniform", 1024, 7, 2048), ("clustered", 8191, 12, 2048),
                                        ("uniform", 20013, 20, 1024), ("uniform", 2, 1, L // 2),
                                        ("squeezed", 3000, 7, 2048)])
def test_fused_step_matches_oracle(kind, n, k, w):
    x, y, th = _gen(kind, n)
    p = nm.make_params(L, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    sysm = nm.System.create(x, y, th, k, p, cell_w=w)
    sysm.step()
    assert nm.check(sysm.ws) == 0
    rn, rx, ry, rt = oracle.step(x, y, th, L, k, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    assert np.array_equal(sysm.nbr.cpu().numpy(), rn)
    assert np.array_equal(sysm.x.cpu().numpy(), rx) and np.array_equal(sysm.y.cpu().numpy(), ry)
    assert _angle_err(sysm.theta.cpu().numpy(), rt).max() <= TOL


@pytest.mark.parametrize("w", [1024, 4096])
def test_rebuild_after_arbitrary_new_positions(w):
    # A build walks the particles in the previous build's cell order; that
    # order must stay a complete walk whatever the new positions are.
    n, k = 20013, 7
    x1, y1, _ = workloads.uniform(n, seed_pos=31)
    x2, y2, _ = workloads.clustered(n, seed=32)
    ws = nm.Workspace(n, L, w)
    for x, y in ((x1, y1), (x2, y2), (x1, y1), (x1, y1)):
        nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
        nbr, d2 = nm.knn(ws, k, with_d2=True)
        assert nm.check(ws) == 0
        rn, rd = oracle.knn(x, y, L, k)
        assert np.array_equal(nbr.cpu().numpy(), rn) and np.array_equal(d2.cpu().numpy(), rd)


def test_rebuild_after_out_of_range_build():
    # an incomplete build (a coordinate outside the box) must not be walked
    n, k = 5000, 7
    x, y, _ = workloads.uniform(n, seed_pos=41)
    ws = nm.Workspace(n, L, 2048)
    bad = x.copy()
    bad[123] = L + 7
    nm.build_cells(ws, _dev(bad, torch.int32), _dev(y, torch.int32))
    assert nm.check(ws) == nm.NM_E_RANGE
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    nbr, d2 = nm.knn(ws, k, with_d2=True)
    assert nm.check(ws) == 0
    rn, rd = oracle.knn(x, y, L, k)
    assert np.array_equal(nbr.cpu().numpy(), rn) and np.array_equal(d2.cpu().numpy(), rd)


def test_fused_step_equals_separate_calls():
    n, k = 20013, 7
    x, y, th = workloads.clustered(n)
    p = nm.make_params(L, v0=64, eta=0.2, seed=3, sys_id=1)
    X, Y, T = _dev(x, torch.int32), _dev(y, torch.int32), _dev(th, torch.float32)
    ws = nm.Workspace(n, L, 2048)
    nbr = torch.empty((n, k), dtype=torch.int32, device="cuda")
    out = (torch.empty_like(X), torch.empty_like(Y), torch.empty_like(T))
    nm.step(ws, X, Y, T, k, p, 11, nbr, *out)
    ws2 = nm.Workspace(n, L, 1024)
    nm.build_cells(ws2, X, Y)
    nbr2, _ = nm.knn(ws2, k)
    xo, yo, to = nm.align_step(X, Y, T, p, 11, nbr=nbr2)
    assert nm.check(ws) == 0 and nm.check(ws2) == 0
    assert torch.equal(nbr, nbr2) and torch.equal(out[0], xo) and torch.equal(out[1], yo)
    assert torch.equal(out[2], to)


def test_trajectory_each_step_matches_oracle_from_gpu_state():
    n, k = 4096, 7
    x, y, th = workloads.uniform(n)
    p = nm.make_params(L, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    sysm = nm.System.create(x, y, th, k, p, cell_w=2048)
    for _ in range(6):
        sx, sy, st = sysm.x.cpu().numpy(), sysm.y.cpu().numpy(), sysm.theta.cpu().numpy()
        t = sysm.step_index
        sysm.step()
        rn, rx, ry, rt = oracle.step(sx, sy, st, L, k, v0=64, eta=0.2, seed=workloads.NOISE_SEED,
                                     step_index=t)
        assert np.array_equal(sysm.nbr.cpu().numpy(), rn)
        assert np.array_equal(sysm.x.cpu().numpy(), rx) and np.array_equal(sysm.y.cpu().numpy(), ry)
        assert _angle_err(sysm.theta.cpu().numpy(), rt).max() <= TOL
    assert nm.check(sysm.ws) == 0


def test_steps_are_deterministic():
    n, k = 65536, 7
    x, y, th = workloads.clustered(n)
    p = nm.make_params(L, seed=5)
    outs = []
    for _ in range(2):
        s = nm.System.create(x, y, th, k, p, cell_w=2048)
        for _ in range(3):
            s.step()
        outs.append((s.nbr.clone(), s.x.clone(), s.y.clone(), s.theta.clone()))
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def _device_invariants(x, y, nbr, k):
    """Every row: k distinct indices, no self, ascending by (d^2, j)."""
    n = x.numel()
    i = torch.arange(n, device="cuda").unsqueeze(1)
    nb = nbr.long()
    assert bool((nb >= 0).all()) and bool((nb < n).all()) and not bool((nb == i).any())
    dx = (x[nb] - x.unsqueeze(1)).long()
    dy = (y[nb] - y.unsqueeze(1)).long()
    dx = (dx + L // 2) % L - L // 2
    dy = (dy + L // 2) % L - L // 2
    key = (dx * dx + dy * dy) * (1 << 24) + nb
    assert bool((key[:, 1:] > key[:, :-1]).all())


def _sample_rows(n, count, seed):
    rng = np.random.default_rng(seed)
    return np.unique(rng.integers(0, n, size=count)).astype(np.int32)


def test_full_size_uniform_1m_sampled():
    n, k = 1 << 20, 7
    rc2 = workloads.rc2_for_mean(n, 7.0)
    x, y, th = workloads.uniform(n)
    p = nm.make_params(L, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    sysm = nm.System.create(x, y, th, k, p, cell_w=2048)
    sysm.step()
    offs, idx = nm.metric_list(sysm.ws, rc2)
    assert nm.check(sysm.ws) == 0
    assert rc2 == 2336407
    _device_invariants(_dev(x, torch.int32), _dev(y, torch.int32), sysm.nbr, k)
    rows = _sample_rows(n, 1000, 7)
    rn, _ = oracle.knn(x, y, L, k, rows=rows, with_d2=False)
    assert np.array_equal(sysm.nbr[torch.as_tensor(rows).long().cuda()].cpu().numpy(), rn)
    rx, ry, rt = oracle.align_step(x, y, th, L, nbr=rn, v0=64, eta=0.2, seed=workloads.NOISE_SEED,
                                   rows=rows)
    sel = torch.as_tensor(rows).long().cuda()
    assert np.array_equal(sysm.x[sel].cpu().numpy(), rx) and np.array_equal(sysm.y[sel].cpu().numpy(), ry)
    assert _angle_err(sysm.theta[sel].cpu().numpy(), rt).max() <= TOL
    ro, ri, _ = oracle.metric_list(x, y, L, rc2, rows=rows, with_d2=False)
    offs_np, idx_np = offs.cpu().numpy(), idx.cpu().numpy()
    got = np.concatenate([idx_np[offs_np[r]:offs_np[r + 1]] for r in rows])
    assert np.array_equal(np.diff(ro), offs_np[rows + 1] - offs_np[rows])
    assert np.array_equal(got, ri)
    assert abs(offs_np[-1] / n - 7.0) < 0.05  # mean metric degree of the chosen r_c


@pytest.mark.parametrize("block", [0, nm.NM_BLOCK_SUBSTRIPS])
@pytest.mark.parametrize("k", [6, 12, 20])
def test_full_size_clustered_4m_sampled(k, block):
    # (at w = 1024 about one strip in 17 (k = 6) and one in four (k = 12) has
    # a halo larger than LDS)
    n = 1 << 22
    x, y, th = workloads.clustered(n)
    p = nm.make_params(L, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    sysm = nm.System.create(x, y, th, k, p, cell_w=nm.suggest_cell_w(n, L, 1.0), block=block)
    sysm.step()
    assert nm.check(sysm.ws) == 0
    _device_invariants(_dev(x, torch.int32), _dev(y, torch.int32), sysm.nbr, k)
    rows = _sample_rows(n, 300, k)
    rn, _ = oracle.knn(x, y, L, k, rows=rows, with_d2=False)
    sel = torch.as_tensor(rows).long().cuda()
    assert np.array_equal(sysm.nbr[sel].cpu().numpy(), rn)
    rx, ry, rt = oracle.align_step(x, y, th, L, nbr=rn, v0=64, eta=0.2, seed=workloads.NOISE_SEED,
                                   rows=rows)
    assert np.array_equal(sysm.x[sel].cpu().numpy(), rx) and np.array_equal(sysm.y[sel].cpu().numpy(), ry)
    assert _angle_err(sysm.theta[sel].cpu().numpy(), rt).max() <= TOL


@pytest.mark.parametrize("kind,w", [("uniform", 512), ("uniform", 2048), ("clustered", 1024),
                                    ("uniform", 16384), ("uniform", 4096)])
def test_two_level_binning_sampled(kind, w):
    # N >= 2^17 takes the two-level binning (coarse bins of up to 4096 cells at
    # w = 512, of 4 cells at w = 16384); ragged N, one fused step, sampled rows.
    n, k = (1 << 17) + 1234, 7
    if kind == "clustered":
        x, y, th = workloads.clustered(n)
    else:
        x, y, th = _gen(kind, n)
    p = nm.make_params(L, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    sysm = nm.System.create(x, y, th, k, p, cell_w=w)
    sysm.step()
    assert nm.check(sysm.ws) == 0
    _device_invariants(_dev(x, torch.int32), _dev(y, torch.int32), sysm.nbr, k)
    rows = np.concatenate([_sample_rows(n, 300, w), [0, n - 1]]).astype(np.int32)
    rn, _ = oracle.knn(x, y, L, k, rows=rows, with_d2=False)
    sel = torch.as_tensor(rows).long().cuda()
    assert np.array_equal(sysm.nbr[sel].cpu().numpy(), rn)
    rx, ry, rt = oracle.align_step(x, y, th, L, nbr=rn, v0=64, eta=0.2, seed=workloads.NOISE_SEED,
                                   rows=rows)
    assert np.array_equal(sysm.x[sel].cpu().numpy(), rx) and np.array_equal(sysm.y[sel].cpu().numpy(), ry)
    assert _angle_err(sysm.theta[sel].cpu().numpy(), rt).max() <= TOL
    rc2 = workloads.rc2_for_mean(n, 5.0)
    offs, idx = nm.metric_list(sysm.ws, rc2)
    assert nm.check(sysm.ws) == 0
    ro, ri, _ = oracle.metric_list(x, y, L, rc2, rows=rows, with_d2=False)
    offs_np, idx_np = offs.cpu().numpy().astype(np.int64), idx.cpu().numpy()
    assert np.array_equal(np.diff(ro), offs_np[rows + 1] - offs_np[rows])
    assert np.array_equal(np.concatenate([idx_np[offs_np[r]:offs_np[r + 1]] for r in rows]), ri)


def _coarse_bin_sizes(x, y, n, w):
    """Particles per coarse bin under the workspace's sizing rule: at most 1024
    bins of 2^sb cells, grown towards 1024 particles at the mean density, at
    most 4096 cells."""
    g = L // w
    c = g * g
    sb = 0
    while (c >> sb) > 1024:
        sb += 1
    while (1 << sb) < 4096 and (n << sb) < 1024 * c:
        sb += 1
    lw = w.bit_length() - 1
    cell = (y.astype(np.int64) >> lw) * g + (x.astype(np.int64) >> lw)
    return np.bincount(cell >> sb)


def test_fine_sort_stage_rounds_clustered():
    # The fine sort writes a bin through its LDS stage of 1280 ranks, in two
    # rounds for bins of 1281-2048 particles, and bins of more than 2048
    # directly.  Three grids of one clustered system cover all three; the
    # lists are exact, so every grid must give the same lists and the same
    # fused step, which must match the oracle on sampled rows.
    n, k = (1 << 18) + 77, 7
    x, y, th = workloads.clustered(n)
    sizes = {w: _coarse_bin_sizes(x, y, n, w) for w in (1024, 4096, 8192)}
    assert ((sizes[1024] > 1280) & (sizes[1024] <= 2048)).any()
    assert (sizes[8192] > 2048).any()
    p = nm.make_params(L, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    xd, yd = _dev(x, torch.int32), _dev(y, torch.int32)
    outs = []
    for w in sizes:
        sysm = nm.System.create(x, y, th, k, p, cell_w=w)
        sysm.step()
        assert nm.check(sysm.ws) == 0
        _device_invariants(xd, yd, sysm.nbr, k)
        outs.append([t.cpu().numpy() for t in (sysm.nbr, sysm.x, sysm.y, sysm.theta)])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
    rows = np.concatenate([_sample_rows(n, 200, 5), [0, n - 1]]).astype(np.int32)
    rn, _ = oracle.knn(x, y, L, k, rows=rows, with_d2=False)
    assert np.array_equal(outs[0][0][rows], rn)
    rx, ry, rt = oracle.align_step(x, y, th, L, nbr=rn, v0=64, eta=0.2, seed=workloads.NOISE_SEED,
                                   rows=rows)
    assert np.array_equal(outs[0][1][rows], rx) and np.array_equal(outs[0][2][rows], ry)
    assert _angle_err(outs[0][3][rows], rt).max() <= TOL


def test_two_level_binning_reports_range_error():
    n = (1 << 17) + 5
    x, y, th = workloads.uniform(n)
    x[70000] = L
    ws = nm.Workspace(n, L, 2048)
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    assert nm.check(ws) == nm.NM_E_RANGE


def test_range_error_is_reported():
    n = 1000
    x, y, th = workloads.uniform(n)
    x[17] = L  # outside [0, L)
    ws = nm.Workspace(n, L, 2048)
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    nm.knn(ws, 7)
    assert nm.check(ws) == nm.NM_E_RANGE
    assert nm.check(ws) == 0  # cleared


def test_metric_capacity_overflow_is_reported():
    n = 4097
    x, y, _ = workloads.uniform(n)
    ws = nm.Workspace(n, L, 2048)
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    small = torch.empty(100, dtype=torch.int32, device="cuda")
    nm.metric_list(ws, workloads.rc2_for_mean(n, 7.0), idx=small)
    assert nm.check(ws) == nm.NM_E_CAPACITY


def test_grid_mismatch_is_reported():
    n = 1000
    x, y, _ = workloads.uniform(n)
    ws = nm.Workspace(n, L, 2048)
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    other = nm.Workspace(n, L, 4096)
    other.buf = ws.buf  # same memory, different grid description
    nm.knn(other, 7)
    assert nm.check(ws) == nm.NM_E_INVAL


def _gpu_knn_block(x, y, k, w, block):
    ws = nm.Workspace(len(x), L, w, block=block)
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    nbr, d2 = nm.knn(ws, k, with_d2=True)
    assert nm.check(ws) == 0
    return nbr.cpu().numpy(), d2.cpu().numpy()


@pytest.mark.parametrize("k", [4, 7, 8, 12])
@pytest.mark.parametrize("block", [0, 4, nm.NM_BLOCK_SUBSTRIPS])
def test_knn_wide_strips_near_ties(k, block):
    # A 128 x 128 lattice (spacing 8192) jittered by at most 2 units.  Its
    # strips are wide (blocks span more than 2^15 units), where the 32-bit
    # keys take fp32 squared distances; many neighbours lie within a few
    # distance-field units of each other, which the certificate must defer
    # or re-sort by the exact (d^2, index).
    x, y, a = workloads.lattice(128)
    rng = np.random.default_rng(5)
    x = ((x.astype(np.int64) + rng.integers(-2, 3, x.size)) % L).astype(np.int32)
    y = ((y.astype(np.int64) + rng.integers(-2, 3, y.size)) % L).astype(np.int32)
    lay = nm.knn_layout(len(x), L, a, block, k)
    assert lay["wide"] == 1 and lay["kernel"] in (1, 2)
    nbr, d2 = _gpu_knn_block(x, y, k, a, block)
    rn, rd = oracle.knn(x, y, L, k)
    assert np.array_equal(nbr, rn) and np.array_equal(d2, rd)


@pytest.mark.parametrize("block", [-1, 0, 3, 4, 5, 6, 8, nm.NM_BLOCK_SUBSTRIPS, nm.NM_BLOCK_SUBSTRIPS | 5])
@pytest.mark.parametrize("kind,n,k,w", [("uniform", 20013, 7, 4096), ("uniform", 20013, 1, 8192),
                                        ("uniform", 20013, 20, 4096), ("clustered", 20013, 12, 2048),
                                        ("squeezed", 3000, 7, 1024), ("clustered", 8191, 32, 4096)])
def test_knn_every_search_path_matches_oracle(kind, n, k, w, block):
    # block = -1: exact ring search only; 0: automatic fast block; >0: that block side.
    x, y, _ = _gen(kind, n)
    nbr, d2 = _gpu_knn_block(x, y, k, w, block)
    rn, rd = oracle.knn(x, y, L, k)
    assert np.array_equal(nbr, rn) and np.array_equal(d2, rd)


# Sparse systems (mean spacing several thousand units): the k-NN halo spans
# more than 2^15 units, so the staged tiles hold int32 offset pairs and the
# block search uses 64-bit squared distances.
WIDE_CASES = [("uniform", 16384, 7, 16384, 0), ("uniform", 16384, 12, 8192, 0),
              ("uniform", 4096, 7, 32768, 0), ("clustered", 16384, 7, 8192, 0),
              ("uniform", 16384, 20, 16384, 5), ("uniform", 3001, 1, 65536, 0),
              ("uniform", 16384, 7, 8192, 9), ("squeezed", 3000, 7, 16384, 0)]


@pytest.mark.parametrize("kind,n,k,w,block", WIDE_CASES)
def test_knn_wide_tiles_match_oracle(kind, n, k, w, block):
    x, y, _ = _gen(kind, n)
    if kind == "squeezed":  # duplicates and ties spread over a sparse box
        x, y = (x * 37) % L, (y * 53) % L
    nbr, d2 = _gpu_knn_block(x, y, k, w, block)
    rn, rd = oracle.knn(x, y, L, k)
    assert np.array_equal(nbr, rn) and np.array_equal(d2, rd)


@pytest.mark.parametrize("kind,n,k,w,block", WIDE_CASES[:4])
def test_fused_step_wide_tiles_match_oracle(kind, n, k, w, block):
    x, y, th = _gen(kind, n)
    p = nm.make_params(L, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    ws = nm.Workspace(n, L, w, block=block)
    X, Y, T = _dev(x, torch.int32), _dev(y, torch.int32), _dev(th, torch.float32)
    nbr = torch.empty((n, k), dtype=torch.int32, device="cuda")
    out = (torch.empty_like(X), torch.empty_like(Y), torch.empty_like(T))
    nm.step(ws, X, Y, T, k, p, 0, nbr, *out)
    assert nm.check(ws) == 0
    rn, rx, ry, rt = oracle.step(x, y, th, L, k, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    assert np.array_equal(nbr.cpu().numpy(), rn)
    assert np.array_equal(out[0].cpu().numpy(), rx) and np.array_equal(out[1].cpu().numpy(), ry)
    assert _angle_err(out[2].cpu().numpy(), rt).max() <= TOL


@pytest.mark.parametrize("block", [-1, 0, 4, 6])
def test_knn_lattice_ties_every_path(block):
    # every distance is tied: the fast path must always hand over to the exact search
    x, y, a = workloads.lattice(64)
    for k in (4, 7, 8):
        nbr, d2 = _gpu_knn_block(x, y, k, a, block)
        rn, rd = oracle.knn(x, y, L, k)
        assert np.array_equal(nbr, rn) and np.array_equal(d2, rd)


@pytest.mark.parametrize("block", [-1, 0])
def test_fused_step_every_path(block):
    n, k = 20013, 7
    x, y, th = workloads.uniform(n)
    p = nm.make_params(L, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    ws = nm.Workspace(n, L, 4096, block=block)
    X, Y, T = _dev(x, torch.int32), _dev(y, torch.int32), _dev(th, torch.float32)
    nbr = torch.empty((n, k), dtype=torch.int32, device="cuda")
    out = (torch.empty_like(X), torch.empty_like(Y), torch.empty_like(T))
    nm.step(ws, X, Y, T, k, p, 0, nbr, *out)
    assert nm.check(ws) == 0
    rn, rx, ry, rt = oracle.step(x, y, th, L, k, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    assert np.array_equal(nbr.cpu().numpy(), rn)
    assert np.array_equal(out[0].cpu().numpy(), rx) and np.array_equal(out[1].cpu().numpy(), ry)
    assert _angle_err(out[2].cpu().numpy(), rt).max() <= TOL


@pytest.mark.parametrize("kind,n,mean,w", [("uniform", 20013, 7.0, 4096), ("uniform", 20013, 7.0, 8192),
                                           ("clustered", 20013, 3.0, 2048), ("squeezed", 3000, 2.0, 1024)])
def test_metric_fast_block_matches_oracle(kind, n, mean, w):
    x, y, _ = _gen(kind, n)
    rc2 = workloads.rc2_for_mean(n, mean)
    offs, idx = _gpu_metric(x, y, rc2, w)
    ro, ri, _ = oracle.metric_list(x, y, L, rc2)
    assert np.array_equal(offs, ro) and np.array_equal(idx, ri)


def _dense_patch(n_patch, n_rest, side, seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([500000 + rng.integers(0, side, n_patch), rng.integers(0, L, n_rest)])
    y = np.concatenate([700000 + rng.integers(0, side, n_patch), rng.integers(0, L, n_rest)])
    return x.astype(np.int32), y.astype(np.int32)


@pytest.mark.parametrize("case", ["narrow", "wide_cells", "wide_halo", "box_sized_halo", "dense_patch"])
def test_metric_strip_layouts(case):
    # narrow: 16-bit staged offsets; wide_cells / wide_halo: int32 offsets because
    # the halo spans 2^15 or more (large cells, or a halo of ~22 cells); box_sized_halo:
    # 2h + 1 > G, rows walked in global memory; dense_patch: 3000 particles in a
    # 2000 x 2000 patch overflow the staged strip and fall back beside staged ones.
    if case == "dense_patch":
        x, y = _dense_patch(3000, 1000, 2000, 5)
        rc2, w = 100 ** 2, 1024
    else:
        n = 20013
        x, y, _ = workloads.uniform(n)
        mean, w = {"narrow": (7.0, 2048), "wide_cells": (7.0, 16384), "wide_halo": (30.0, 1024),
                   "box_sized_halo": (7.0, L // 4)}[case]
        rc2 = workloads.rc2_for_mean(n, mean)
        if case == "box_sized_halo":  # G = 4 cells a side, h = 2
            rc2 = (L // 4 + 100) ** 2
            x, y = x[:500], y[:500]
    offs, idx = _gpu_metric(x, y, rc2, w)
    ro, ri, _ = oracle.metric_list(x, y, L, rc2)
    assert np.array_equal(offs, ro) and np.array_equal(idx, ri)


def test_metric_rows_across_slot_widths():
    # Isolated groups of 5 .. 48 points in disks of radius 40 (r_c = 100): rows of
    # 4 .. 47 entries take the 8-, 16- and 32-wide sorts of the one-pass fill and,
    # past its slot column, the chunked selection; sparse points elsewhere keep
    # short rows in the same launch.  Cells of 8192 make the strips wide.
    rng = np.random.default_rng(33)
    sizes = [5, 9, 10, 16, 17, 18, 25, 30, 31, 32, 33, 40, 48]
    xs, ys = [], []
    for g, size in enumerate(sizes):
        r = 40 * np.sqrt(rng.uniform(0, 1, size))
        a = rng.uniform(0, 2 * np.pi, size)
        xs.append(40000 + 60000 * g + np.round(r * np.cos(a)))
        ys.append(300000 + 5000 * g + np.round(r * np.sin(a)))
    xs.append(rng.integers(0, L, 3000))
    ys.append(rng.integers(0, L, 3000))
    x = np.concatenate(xs).astype(np.int32)
    y = np.concatenate(ys).astype(np.int32)
    rc2 = 100 ** 2
    ro, ri, _ = oracle.metric_list(x, y, L, rc2)
    lengths = set(np.diff(ro).tolist())
    assert {4, 8, 9, 15, 16, 17, 29, 30, 31, 47} <= lengths
    for w in (1024, 8192):
        offs, idx = _gpu_metric(x, y, rc2, w)
        assert np.array_equal(offs, ro) and np.array_equal(idx, ri)


def test_metric_rows_longer_than_a_wave_sort():
    # 700 coincident points: rows of 699 entries, beyond what one wave sorts in LDS,
    # take the chunked selection; 300 more points in a ring keep other rows mid-sized.
    rng = np.random.default_rng(9)
    ang = rng.uniform(0, 2 * np.pi, 300)
    x = np.concatenate([np.full(700, 300000), 300000 + np.round(80 * np.cos(ang))]).astype(np.int32)
    y = np.concatenate([np.full(700, 90000), 90000 + np.round(80 * np.sin(ang))]).astype(np.int32)
    offs, idx = _gpu_metric(x, y, 100 ** 2, 2048)
    ro, ri, _ = oracle.metric_list(x, y, L, 100 ** 2)
    assert np.array_equal(offs, ro) and np.array_equal(idx, ri)


def test_metric_heavy_rows_sorted_by_a_wave():
    # 300 coincident points and 150 in a 150 x 150 square beside them: rows of
    # 200-450 entries over ~450 staged candidates are gathered and sorted by a
    # whole wave (with many equal distances, ordered by index); sparse uniform
    # points elsewhere keep light rows in the same launch.
    rng = np.random.default_rng(21)
    x = np.concatenate([np.full(300, 700000), 700000 + rng.integers(-75, 75, 150),
                        rng.integers(0, L, 2000)]).astype(np.int32)
    y = np.concatenate([np.full(300, 400000), 400000 + rng.integers(-75, 75, 150),
                        rng.integers(0, L, 2000)]).astype(np.int32)
    rc2 = 120 ** 2
    for w in (1024, 8192):
        offs, idx = _gpu_metric(x, y, rc2, w)
        ro, ri, _ = oracle.metric_list(x, y, L, rc2)
        assert np.array_equal(offs, ro) and np.array_equal(idx, ri)
        assert (np.diff(ro)[:450] > 150).all()


def test_knn_fast_path_query_last_in_home_row():
    # Particle 0 is the only particle in its block row, so both parts of its home
    # row around its own slot are empty; its nearest neighbour (1) lies in the next
    # block row, and particle 2 (same cell row, far outside the block) sits between
    # them in cell order.  The ordinal -> slot map must skip the empty ranges.
    w = 4096
    x = [100 * w + 2048, 100 * w + 2048, 200 * w + 5, 30 * w]
    y = [100 * w + 4000, 101 * w + 104, 100 * w + 7, 30 * w]
    for block in (3, 4, 0):
        nbr, d2 = _gpu_knn_block(x, y, 1, w, block)
        rn, rd = oracle.knn(x, y, L, 1)
        assert np.array_equal(nbr, rn) and np.array_equal(d2, rd)
        assert nbr[0, 0] == 1


# Tight clusters in an otherwise sparse box: strips sized for the mean density
# hold halos larger than the staging buffer.  Such a strip runs as sub-strips
# of whole rows staged one after another; a row whose own halo is too large is
# searched in global memory.  Each case reaches both kinds (counted with a host
# model of the strip tables): (box, n, clusters, width, k, cell width).  Both
# kernels run each case: block 0 (such strips search global memory) and
# NM_BLOCK_SUBSTRIPS (sub-strips).
SPLIT_CASES = [
    (1 << 16, 40000, 16, 0.005, 7, 256),    # narrow strips: 17 overflow, 42 sub-strips, 6 rows global
    (1 << 16, 40000, 8, 0.003, 12, 128),    # narrow: 21 overflow, 396 sub-strips, 353 global
    (1 << 20, 20013, 16, 0.005, 12, 2048),  # wide strips: 11 overflow, 89 sub-strips, 64 global
    (1 << 20, 40000, 64, 0.01, 7, 2048),    # wide: 11 overflow, every row stageable
]


@pytest.mark.parametrize("block", [0, nm.NM_BLOCK_SUBSTRIPS, nm.NM_BLOCK_SUBSTRIPS | 4])
@pytest.mark.parametrize("box,n,ncl,sf,k,w", SPLIT_CASES)
def test_knn_strips_larger_than_lds_match_oracle(box, n, ncl, sf, k, w, block):
    x, y, th = workloads.clustered(n, box=box, n_clusters=ncl, sigma_frac=sf)
    ws = nm.Workspace(n, box, w, block=block)
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    nbr, d2 = nm.knn(ws, k, with_d2=True)
    assert nm.check(ws) == 0
    rn, rd = oracle.knn(x, y, box, k)
    assert np.array_equal(nbr.cpu().numpy(), rn) and np.array_equal(d2.cpu().numpy(), rd)
    # the fused step over the same strips
    p = nm.make_params(box, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    sysm = nm.System.create(x, y, th, k, p, cell_w=w, block=block)
    sysm.step()
    assert nm.check(sysm.ws) == 0
    sn, sx, sy, st = oracle.step(x, y, th, box, k, v0=64, eta=0.2, seed=workloads.NOISE_SEED)
    assert np.array_equal(sysm.nbr.cpu().numpy(), sn)
    assert np.array_equal(sysm.x.cpu().numpy(), sx) and np.array_equal(sysm.y.cpu().numpy(), sy)
    assert _angle_err(sysm.theta.cpu().numpy(), st).max() <= TOL


# block 0 and 4: the strip kernel with the cone as a candidate filter; -1:
# one lane per query running the exact ring search.
@pytest.mark.parametrize("block", [0, 4, -1])
@pytest.mark.parametrize("kind,n,w", [("uniform", 4097, 2048), ("clustered", 8191, 1024), ("squeezed", 3000, 2048)])
@pytest.mark.parametrize("cos_q", [-4096, -2048, 0, 2048, 3500])
def test_knn_fov_matches_oracle(kind, n, w, cos_q, block):
    x, y, th = _gen(kind, n)
    ws = nm.Workspace(n, L, w, block=block)
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    T = _dev(th, torch.float32)
    for k in (1, 7):
        ref, ok = oracle.knn_fov(x, y, th, L, k, cos_q)
        got = nm.knn_fov(ws, k, T, cos_q)
        st = nm.check(ws)
        if ok:
            assert st == 0
            assert np.array_equal(got.cpu().numpy(), ref)
        else:  # a particle sees fewer than k others
            assert st == nm.NM_E_RANGE
            rows = (ref >= 0).all(axis=1)
            assert np.array_equal(got.cpu().numpy()[rows], ref[rows])


# Strips of int32 offset pairs (sparse box) and strips whose halo overflows
# LDS (their queries take the exact search), against the full oracle lists.
@pytest.mark.parametrize("case", ["wide", "overflow"])
@pytest.mark.parametrize("cos_q", [-2048, 0, 2048])
def test_knn_fov_strip_layouts_match_oracle(case, cos_q):
    if case == "wide":
        box, w = L, 16384
        x, y, th = workloads.uniform(16384)
    else:
        box, w = 1 << 16, 256
        x, y, th = workloads.clustered(40000, box=box, n_clusters=16, sigma_frac=0.005)
    n = len(x)
    ws = nm.Workspace(n, box, w)
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    got = nm.knn_fov(ws, 7, _dev(th, torch.float32), cos_q)
    st = nm.check(ws)
    ref, ok = oracle.knn_fov(x, y, th, box, 7, cos_q)
    if ok:
        assert st == 0
        assert np.array_equal(got.cpu().numpy(), ref)
    else:
        assert st == nm.NM_E_RANGE
        rows = (ref >= 0).all(axis=1)
        assert np.array_equal(got.cpu().numpy()[rows], ref[rows])


@pytest.mark.parametrize("cos_q", [0, 3500])
def test_knn_fov_full_size_sampled(cos_q):
    n, k = 1 << 20, 7
    x, y, th = workloads.uniform(n)
    ws = nm.Workspace(n, L, 2048)
    nm.build_cells(ws, _dev(x, torch.int32), _dev(y, torch.int32))
    got = nm.knn_fov(ws, k, _dev(th, torch.float32), cos_q)
    assert nm.check(ws) == 0
    rows = _sample_rows(n, 500, 17)
    ref, ok = oracle.knn_fov(x, y, th, L, k, cos_q, rows=rows)
    assert ok
    assert np.array_equal(got[torch.as_tensor(rows).long().cuda()].cpu().numpy(), ref)


def test_knn_fov_after_fused_binning():
    # nm_bin_step builds the same cells (with the noise beside them)
    n, k = 20013, 7
    x, y, th = workloads.clustered(n)
    p = nm.make_params(L, v0=64, eta=0.2, seed=3)
    ws = nm.Workspace(n, L, 2048)
    X, Y, T = _dev(x, torch.int32), _dev(y, torch.int32), _dev(th, torch.float32)
    nm.bin_step(ws, X, Y, T, p, 0)
    got = nm.knn_fov(ws, k, T, 1000)
    ref, ok = oracle.knn_fov(x, y, th, L, k, 1000)
    assert ok and nm.check(ws) == 0
    assert np.array_equal(got.cpu().numpy(), ref)
