"""Served form (nm_server_*): jobs submitted with host inputs, kept on the
device while they run, advanced together with continuous batching under a
device-memory budget.

Bar: every job's final state and last lists equal those of the plain
one-system steps from the same inputs (bit-exact, positions, lists and
headings), whether the job runs alone or in a mix that changes while it runs;
the first step matches the brute-force oracle; the ledger never exceeds the
budget.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import paper_2103_10239_amd as nm
from paper_2103_10239_amd import workloads

pytestmark = pytest.mark.gpu
L = workloads.BOX
TOL = 1e-5


def _angle_err(a, b):
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return np.abs(np.remainder(d + np.pi, 2 * np.pi) - np.pi)


def _inputs(n, clustered, seed):
    if clustered:
        x, y, _ = workloads.clustered(n, n_clusters=16, seed=seed)
    else:
        x, y, _ = workloads.uniform(n, seed_pos=seed)
    return x, y, workloads.headings(n, seed=5000 + seed)


def _plain(x, y, th, k, p, nsteps):
    sysm = nm.System.create(x, y, th, k, p)
    for _ in range(nsteps):
        sysm.step()
    torch.cuda.synchronize()
    assert nm.check(sysm.ws) == 0
    return (sysm.x.cpu().numpy(), sysm.y.cpu().numpy(), sysm.theta.cpu().numpy(),
            sysm.nbr.cpu().numpy())


def _same(res, ref):
    rx, ry, rt, rn = ref
    assert res["status"] == 0
    assert np.array_equal(res["x"], rx) and np.array_equal(res["y"], ry)
    assert np.array_equal(res["theta"].view(np.uint32), rt.view(np.uint32))
    if res["nbr"] is not None:
        assert np.array_equal(res["nbr"], rn)


JOBS = [(1500, 7, 3, False, 11), (40000, 12, 2, True, 12), (300, 7, 5, True, 13),
        (9000, 12, 1, False, 14), (70000, 7, 4, False, 15), (13, 12, 2, False, 16)]


def test_served_jobs_match_plain_steps():
    srv = nm.Server(budget_bytes=4 << 30, max_slots=64)
    ids = []
    for n, k, steps, cl, seed in JOBS:
        x, y, th = _inputs(n, cl, seed)
        p = nm.make_params(L, v0=64, eta=0.2, seed=seed, sys_id=seed * 7)
        ids.append((srv.submit(x, y, th, k, steps, p, want_nbr=True), (x, y, th, k, p, steps, n)))
    for jid, (x, y, th, k, p, steps, n) in ids:
        res = srv.wait(jid)
        assert res["steps"] == steps
        assert res["submit_s"] <= res["admit_s"] <= res["done_s"]
        _same(res, _plain(x, y, th, k, p, steps))
    st = srv.stats()
    assert st["completed"] == len(JOBS) and st["used_bytes"] == 0 and st["status"] == 0
    srv.close()


def test_served_first_step_matches_oracle():
    srv = nm.Server(budget_bytes=1 << 30)
    cases = [(1024, 7, False, 1), (777, 12, True, 2)]
    ids = []
    for n, k, cl, seed in cases:
        x, y, th = _inputs(n, cl, seed)
        p = nm.make_params(L, v0=64, eta=0.2, seed=workloads.NOISE_SEED, sys_id=seed)
        ids.append((srv.submit(x, y, th, k, 1, p, want_nbr=True), x, y, th, k, n, seed))
    for jid, x, y, th, k, n, seed in ids:
        res = srv.wait(jid)
        rn, rx, ry, rt = oracle.step(x, y, th, L, k, v0=64, eta=0.2, seed=workloads.NOISE_SEED,
                                     sys_id=seed, step_index=0)
        assert res["status"] == 0
        assert np.array_equal(res["nbr"], rn)
        assert np.array_equal(res["x"], rx) and np.array_equal(res["y"], ry)
        assert _angle_err(res["theta"], rt).max() <= TOL
    srv.close()


def test_served_variant_first_step_matches_oracle():
    srv = nm.Server(budget_bytes=1 << 30)
    v = nm.NM_NOISE_SCALAR | nm.NM_MOVE_NEW_HEADING
    x, y, th = _inputs(2500, True, 8)
    p = nm.make_params(L, v0=64, eta=0.6, seed=workloads.NOISE_SEED, sys_id=8, variant=v)
    res = srv.wait(srv.submit(x, y, th, 7, 1, p, want_nbr=True))
    srv.close()
    rn, rx, ry, rt = oracle.step(x, y, th, L, 7, v0=64, eta=0.6, seed=workloads.NOISE_SEED, sys_id=8,
                                 step_index=0, variant=v)
    assert res["status"] == 0
    assert np.array_equal(res["nbr"], rn)
    assert np.array_equal(res["x"], rx) and np.array_equal(res["y"], ry)
    assert _angle_err(res["theta"], rt).max() <= TOL


def test_served_alone_equals_in_mix():
    n, k, steps, seed = 30000, 7, 150, 99
    x, y, th = _inputs(n, True, seed)
    p = nm.make_params(L, v0=64, eta=0.2, seed=seed, sys_id=3)
    alone = nm.Server(budget_bytes=2 << 30)
    ref = alone.wait(alone.submit(x, y, th, k, steps, p, want_nbr=True))
    alone.close()
    assert ref["status"] == 0

    mix = nm.Server(budget_bytes=2 << 30, max_slots=32)
    others = []
    for i in range(4):  # long jobs running before the job arrives (hundreds of steps)
        xo, yo, to = _inputs(20000 + 5000 * i, i % 2 == 0, 200 + i)
        others.append(mix.submit(xo, yo, to, 7 if i % 2 else 12, 300 + 100 * i,
                                 nm.make_params(L, 64, 0.2, 1, 200 + i, i), want_nbr=False))
    time.sleep(0.02)
    jid = mix.submit(x, y, th, k, steps, p, want_nbr=True)
    for i in range(4):  # short jobs arriving while it runs
        time.sleep(0.005)
        xo, yo, to = _inputs(2000 + 1000 * i, i % 2 == 1, 300 + i)
        others.append(mix.submit(xo, yo, to, 7, 5 + i, nm.make_params(L, 64, 0.2, 1, 300 + i, 10 + i)))
    res = mix.wait(jid)
    done = [mix.wait(o) for o in others]
    mix.close()
    for o in done:
        assert o["status"] == 0
    assert res["status"] == 0
    assert np.array_equal(res["x"], ref["x"]) and np.array_equal(res["y"], ref["y"])
    assert np.array_equal(res["theta"].view(np.uint32), ref["theta"].view(np.uint32))
    assert np.array_equal(res["nbr"], ref["nbr"])
    # the job really shared the device: other jobs were on it at the same time,
    # and at least one was admitted while it ran (the batch changed under it)
    a, b = res["admit_s"], res["done_s"]
    assert any(o["admit_s"] < b and o["done_s"] > a for o in done)
    assert any(a < o["admit_s"] < b for o in done)


def test_served_admission_respects_budget():
    sizes = [20000, 15000, 25000, 10000, 20000, 5000]
    need = [nm.server_job_bytes(n, 7, L) for n in sizes]
    budget = max(need) + min(need)  # at most about two jobs at once
    srv = nm.Server(budget_bytes=budget, max_slots=16)
    ids = []
    for i, n in enumerate(sizes):
        x, y, th = _inputs(n, False, 40 + i)
        p = nm.make_params(L, v0=64, eta=0.2, seed=40 + i, sys_id=i)
        ids.append((srv.submit(x, y, th, 7, 3, p), x, y, th, p, n))
    for jid, x, y, th, p, n in ids:
        res = srv.wait(jid)
        _same(res, _plain(x, y, th, 7, p, 3))
    st = srv.stats()
    srv.close()
    assert st["peak_used_bytes"] <= budget
    assert st["completed"] == len(sizes)


def test_served_slot_limit():
    srv = nm.Server(budget_bytes=4 << 30, max_slots=2)
    ids = []
    for i in range(6):
        x, y, th = _inputs(3000, False, 60 + i)
        ids.append(srv.submit(x, y, th, 7, 4, nm.make_params(L, 64, 0.2, 1, 60 + i, i)))
    for jid in ids:
        assert srv.wait(jid)["status"] == 0
    st = srv.stats()
    srv.close()
    assert st["peak_active"] <= 2


def test_served_rejects_job_over_budget():
    srv = nm.Server(budget_bytes=1 << 20)
    x, y, th = _inputs(50000, False, 1)
    with pytest.raises(nm.NMError) as e:
        srv.submit(x, y, th, 7, 1, nm.make_params(L))
    assert e.value.status == nm.NM_E_NOMEM
    srv.close()


def test_served_reports_out_of_range_coordinate():
    srv = nm.Server(budget_bytes=1 << 30)
    x, y, th = _inputs(2000, False, 3)
    x = x.copy()
    x[17] = L + 1
    jid = srv.submit(x, y, th, 7, 2, nm.make_params(L))
    res = srv.wait(jid)
    assert res["status"] == nm.NM_E_RANGE
    srv.close()
