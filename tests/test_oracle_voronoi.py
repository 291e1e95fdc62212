"""Pins of the Voronoi (Delaunay) neighbour oracle and the Voronoi-model
oracle (Sec. III-V) to facts independent of their code:

- scipy's Qhull Delaunay triangulation (an independent implementation) of
  the periodic tiling, for points in general position;
- Euler's formula on the torus: a triangulation in general position has
  exactly 3N edges, mean degree 6 (Sec. IV mentions the global consistency
  Euler's formula imposes);
- reciprocity of Delaunay neighbours (Sec. III);
- the empty-circumcircle property of every triangle of consecutive ring
  neighbours, checked against every particle in exact integers (Sec. IV);
- closed forms on lattices and a hand-derived perturbed lattice
  (tests/golden/voronoi_perturbed_lattice.txt);
- exact translation, rotation and reflection symmetry;
- for the forces (Sec. V): central finite differences of the energy of
  Eq. (3), the tiling identity sum of areas = L^2, zero net force, and the
  lattice's closed-form cell.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2103_10239_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(off, idx):
    return [idx[off[r]:off[r + 1]].tolist() for r in range(len(off) - 1)]


def _min_image(d, box):
    return (d + box // 2) % box - box // 2


def _scipy_delaunay_sets(x, y, box):
    from scipy.spatial import Delaunay

    n = len(x)
    pts, ids = [], []
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            pts.append(np.stack([x + a * box, y + b * box], axis=1))
            ids.append(np.arange(n))
    pts = np.concatenate(pts).astype(np.float64)
    ids = np.concatenate(ids)
    central = np.zeros(len(pts), bool)
    central[4 * n:5 * n] = True  # (a, b) = (0, 0)
    tri = Delaunay(pts)
    sets = [set() for _ in range(n)]
    for s in tri.simplices:
        for u in range(3):
            for v in range(3):
                if u != v and central[s[u]]:
                    sets[ids[s[u]]].add(int(ids[s[v]]))
    return sets


@pytest.mark.parametrize("kind,n,box", [("uniform", 600, 1 << 20), ("uniform", 2000, 1 << 16),
                                        ("clustered", 3000, 1 << 20)])
def test_voronoi_matches_qhull_delaunay(kind, n, box):
    if kind == "uniform":
        x, y, _ = workloads.uniform(n, box=box, seed_pos=n)
    else:
        x, y, _ = workloads.clustered(n, box=box, n_clusters=128, sigma_frac=0.02)
    off, idx = oracle.voronoi(x, y, box)
    mine = [set(r) for r in _rows(off, idx)]
    assert mine == _scipy_delaunay_sets(x, y, box)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_voronoi_euler_reciprocity_and_ring_order(seed):
    n, box = 1500, 1 << 20
    x, y, _ = workloads.uniform(n, box=box, seed_pos=seed)
    off, idx = oracle.voronoi(x, y, box)
    assert off[-1] == 6 * n  # Euler on the torus: E = 3N
    rows = _rows(off, idx)
    for i, r in enumerate(rows):
        assert i not in r and len(set(r)) == len(r) >= 3
        for j in r:
            assert i in rows[j]  # reciprocal
        # counter-clockwise from the +x axis: angles strictly increasing in [0, 2 pi)
        dx = _min_image(x[r].astype(np.int64) - x[i], box)
        dy = _min_image(y[r].astype(np.int64) - y[i], box)
        ang = np.mod(np.arctan2(dy, dx), 2 * np.pi)
        assert (np.diff(ang) > 0).all()


def _incircle(ax, ay, bx, by, qx, qy):
    """Sign-exact in-circle determinant of the points q against the ccw
    triangle (0, a, b): > 0 inside, < 0 outside (int64; |coordinates| < 2^13
    keeps every term below 2^56)."""
    adx, ady, bdx, bdy, cdx, cdy = -qx, -qy, ax - qx, ay - qy, bx - qx, by - qy
    return ((adx * adx + ady * ady) * (bdx * cdy - cdx * bdy)
            - (bdx * bdx + bdy * bdy) * (adx * cdy - cdx * ady)
            + (cdx * cdx + cdy * cdy) * (adx * bdy - bdx * ady))


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_voronoi_triangles_have_empty_circumcircles(kind):
    n, box = 1000, 1 << 14
    if kind == "uniform":
        x, y, _ = workloads.uniform(n, box=box, seed_pos=9)
    else:
        x, y, _ = workloads.clustered(n, box=box, n_clusters=128, sigma_frac=0.01, seed=9)
    off, idx = oracle.voronoi(x, y, box)
    rows = _rows(off, idx)
    X, Y = x.astype(np.int64), y.astype(np.int64)
    for i, r in enumerate(rows):
        qx = _min_image(X - X[i], box)
        qy = _min_image(Y - Y[i], box)
        for t in range(len(r)):
            a, b = r[t], r[(t + 1) % len(r)]
            assert qx[a] * qy[b] - qy[a] * qx[b] > 0  # consecutive neighbours turn counter-clockwise
            # the triangle is a triangle of the triangulation: i follows b in a's ring
            ra = rows[a]
            assert ra[(ra.index(b) + 1) % len(ra)] == i
            inside = _incircle(qx[a], qy[a], qx[b], qy[b], qx, qy)
            inside[[i, a, b]] = -1
            assert (inside < 0).all()


def test_square_lattice_has_four_neighbours():
    x, y, a = workloads.lattice(32)
    m = 32
    off, idx = oracle.voronoi(x, y, workloads.BOX)
    for p, r in enumerate(_rows(off, idx)):
        row, col = divmod(p, m)
        right, up = row * m + (col + 1) % m, ((row + 1) % m) * m + col
        left, down = row * m + (col - 1) % m, ((row - 1) % m) * m + col
        assert r == [right, up, left, down]


def _centred_lattice(m, box):
    """m x m points: row r at y = r a, x = c a + (r mod 2) a / 2 (a = box / m):
    the lattice with basis (a, 0), (a/2, a)."""
    a = box // m
    idx = np.arange(m * m)
    r, c = idx // m, idx % m
    return (c * a + (r % 2) * (a // 2)).astype(np.int32), (r * a).astype(np.int32), a


def test_centred_lattice_closed_form():
    m, box = 16, 1 << 20
    x, y, a = _centred_lattice(m, box)
    off, idx = oracle.voronoi(x, y, box)
    for p, r in enumerate(_rows(off, idx)):
        dx = _min_image(x[r].astype(np.int64) - x[p], box)
        dy = _min_image(y[r].astype(np.int64) - y[p], box)
        got = list(zip(dx.tolist(), dy.tolist()))
        assert got == [(a, 0), (a // 2, a), (-a // 2, a), (-a, 0), (-a // 2, -a), (a // 2, -a)]
    # Voronoi model: every cell the same hexagon, area a^2, perimeter a (sqrt(5) + 3/2),
    # vertices (a/2, 3a/8), (0, 5a/8), ...; no net force by the lattice's inversion symmetry
    f = oracle.voronoi_forces(x, y, box, off, idx, ka=1.0, kp=1.0, a0=0.9 * a * a, p0=3.0 * a,
                              vertices=True)
    assert np.allclose(f["area"], a * a, rtol=1e-13)
    assert np.allclose(f["perim"], a * (np.sqrt(5.0) + 1.5), rtol=1e-13)
    assert np.allclose(f["hx"][:6], [a / 2, 0, -a / 2, -a / 2, 0, a / 2], rtol=0, atol=1e-9 * a)
    assert np.allclose(f["hy"][:6], [3 * a / 8, 5 * a / 8, 3 * a / 8, -3 * a / 8, -5 * a / 8, -3 * a / 8],
                       rtol=0, atol=1e-9 * a)
    scale = 2 * (0.1 * a * a) * a + 2 * abs(a * (np.sqrt(5.0) + 1.5) - 3.0 * a)
    assert np.abs(f["fx"]).max() <= 1e-9 * scale and np.abs(f["fy"]).max() <= 1e-9 * scale


def test_perturbed_lattice_worked_example():
    x, y, a = workloads.lattice(8)
    x, y = x.copy(), y.copy()
    x[0], y[0] = 1, 1
    expect = {}
    with open(os.path.join(GOLDEN, "voronoi_perturbed_lattice.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            p, rest = line.split(":")
            expect[int(p)] = [int(v) for v in rest.split()]
    off, idx = oracle.voronoi(x, y, workloads.BOX)
    for p, r in enumerate(_rows(off, idx)):
        if p in expect:
            assert r == expect[p], p
        else:
            row, col = divmod(p, 8)
            assert r == [row * 8 + (col + 1) % 8, ((row + 1) % 8) * 8 + col, row * 8 + (col - 1) % 8,
                         ((row - 1) % 8) * 8 + col]


def test_voronoi_exact_symmetries():
    n, box = 800, 1 << 20
    x, y, _ = workloads.uniform(n, box=box, seed_pos=44)
    base = [set(r) for r in _rows(*oracle.voronoi(x, y, box))]
    base_rows = _rows(*oracle.voronoi(x, y, box))
    # translation: identical rows (the order depends on relative vectors only)
    assert _rows(*oracle.voronoi((x + 12345) % box, (y + 777777) % box, box)) == base_rows
    # rotation by 90 degrees and reflection: the same neighbour sets
    assert [set(r) for r in _rows(*oracle.voronoi((box - y) % box, x, box))] == base
    assert [set(r) for r in _rows(*oracle.voronoi((box - x) % box, y, box))] == base


def test_voronoi_local_rows_equal_full_rows():
    n, box = 5000, 1 << 20
    x, y, _ = workloads.clustered(n, box=box, n_clusters=128, sigma_frac=0.02)
    off, idx = oracle.voronoi(x, y, box)
    rows = np.arange(0, n, 7).astype(np.int32)
    o2, i2 = oracle.voronoi(x, y, box, rows=rows, rho0=2000)
    full = _rows(off, idx)
    assert _rows(o2, i2) == [full[r] for r in rows]


def test_coincident_particles_share_a_site():
    # the diagram of distinct positions: a set with particle 9 moved onto
    # particle 5 has the rows of the set without particle 9, with 9 listed
    # beside 5 wherever 5 appears, and 5 and 9 listing each other first
    n, box = 700, 1 << 20
    x, y, _ = workloads.uniform(n, box=box, seed_pos=12)
    x[9], y[9] = x[5], y[5]
    x[40], y[40] = x[5], y[5]  # a third particle at the same site
    rows = _rows(*oracle.voronoi(x, y, box))
    keep = np.array([i for i in range(n) if i not in (9, 40)])
    sub = _rows(*oracle.voronoi(x[keep], y[keep], box))
    back = {k: int(i) for k, i in enumerate(keep)}
    for k, r in enumerate(sub):
        i = back[k]
        want = []
        for j in (back[v] for v in r):
            want += [5, 9, 40] if j == 5 else [j]
        if i == 5:
            want = [9, 40] + want
        assert rows[i] == want, i
    assert rows[9] == [5, 40] + rows[5][2:] and rows[40] == [5, 9] + rows[5][2:]
    # the Voronoi model gives every particle its own cell: coincident ones have none
    off, idx = oracle.voronoi(x, y, box)
    with pytest.raises(oracle.OracleError) as e:
        oracle.voronoi_forces(x, y, box, off, idx, 1.0, 1.0, 1.0, 1.0)
    assert e.value.status == oracle.E_RANGE


def test_voronoi_errors():
    x, y, _ = workloads.uniform(6)  # cells far larger than L/8
    with pytest.raises(oracle.OracleError) as e:
        oracle.voronoi(x, y, workloads.BOX)
    assert e.value.status == oracle.E_RANGE


def _energy(x, y, box, off, idx, ka, kp, a0, p0):
    return oracle.voronoi_forces(x, y, box, off, idx, ka, kp, a0, p0)["energy"]


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_forces_are_minus_the_energy_gradient(kind):
    n, box = 1000, 1 << 20
    if kind == "uniform":
        x, y, _ = workloads.uniform(n, box=box, seed_pos=77)
    else:
        x, y, _ = workloads.clustered(n, box=box, n_clusters=128, sigma_frac=0.02, seed=78)
    off, idx = oracle.voronoi(x, y, box)
    a_mean = box * box / n
    ka, kp, a0, p0 = 1.0 / a_mean, 1.0, 1.0 * a_mean, 3.7 * np.sqrt(a_mean)
    xd, yd = x.astype(np.float64), y.astype(np.float64)
    f = oracle.voronoi_forces(xd, yd, box, off, idx, ka, kp, a0, p0)
    assert abs(f["area"].sum() - float(box) ** 2) <= 1e-9 * float(box) ** 2  # the cells tile the torus
    assert abs(f["fx"].sum()) <= 1e-6 * np.abs(f["fx"]).max() * n
    assert abs(f["fy"].sum()) <= 1e-6 * np.abs(f["fy"]).max() * n
    h = 0.25  # grid units; the spacing is ~5e4, so the topology is unchanged
    rng = np.random.default_rng(3)
    fmax = max(np.abs(f["fx"]).max(), np.abs(f["fy"]).max())
    for i in rng.choice(n, 25, replace=False):
        for comp, key in ((xd, "fx"), (yd, "fy")):
            c0 = comp[i]
            comp[i] = c0 + h
            ep = _energy(xd, yd, box, off, idx, ka, kp, a0, p0)
            comp[i] = c0 - h
            em = _energy(xd, yd, box, off, idx, ka, kp, a0, p0)
            comp[i] = c0
            fd = -(ep - em) / (2 * h)
            assert abs(fd - f[key][i]) <= 1e-6 * fmax, (i, key, fd, f[key][i])


def test_vertex_forces_are_minus_the_energy_gradient():
    # vertex model (Sec. V.A, Eqs. 5-8): the energy of Eq. (3) as a function of
    # the vertices with the tiling's topology fixed, each cell's area and
    # perimeter from its polygon
    n, box = 300, 1 << 20
    x, y, _ = workloads.uniform(n, box=box, seed_pos=91)
    off, idx = oracle.voronoi(x, y, box)
    a_mean = box * box / n
    ka, kp, a0, p0 = 2.0 / a_mean, 0.5, 0.8 * a_mean, 3.9 * np.sqrt(a_mean)
    f = oracle.voronoi_forces(x, y, box, off, idx, ka, kp, a0, p0, vertices=True)
    rows = _rows(off, idx)
    # absolute vertex positions, one per triangle (i, a_t, a_{t+1}) keyed by its sorted indices
    key_of, vpos = {}, {}
    for i, r in enumerate(rows):
        for t in range(len(r)):
            key = tuple(sorted((i, r[t], r[(t + 1) % len(r)])))
            s = off[i] + t
            if key not in vpos:
                vpos[key] = np.array([x[i] + f["hx"][s], y[i] + f["hy"][s]])
            key_of[(i, t)] = key

    def energy(vp):
        e = 0.0
        for i, r in enumerate(rows):
            poly = [vp[key_of[(i, t)]] for t in range(len(r))]
            # unwrap around the particle (vertices are within L/8 of it)
            ref = np.array([x[i], y[i]], float)
            poly = [ref + (q - ref + box / 2) % box - box / 2 for q in poly]
            area = 0.5 * sum(poly[t][0] * poly[(t + 1) % len(poly)][1] - poly[(t + 1) % len(poly)][0] * poly[t][1]
                             for t in range(len(poly)))
            per = sum(np.hypot(*(poly[(t + 1) % len(poly)] - poly[t])) for t in range(len(poly)))
            e += ka * (area - a0) ** 2 + kp * (per - p0) ** 2
        return e

    h = 0.5
    fmax = np.abs(np.concatenate([f["vfx"], f["vfy"]])).max()
    for (i, t) in list(key_of)[::97][:12]:
        key = key_of[(i, t)]
        s = off[i] + t
        for c, name in ((0, "vfx"), (1, "vfy")):
            vp = dict(vpos)
            q = vp[key].copy()
            q[c] += h
            vp[key] = q
            ep = energy(vp)
            q = vpos[key].copy()
            q[c] -= h
            vp[key] = q
            em = energy(vp)
            assert abs(-(ep - em) / (2 * h) - f[name][s]) <= 1e-6 * fmax


def test_forces_of_sampled_rows_equal_the_full_forces():
    n, box = 1500, 1 << 20
    x, y, _ = workloads.uniform(n, box=box, seed_pos=99)
    off, idx = oracle.voronoi(x, y, box)
    a_mean = box * box / n
    args = (1.0 / a_mean, 1.0, a_mean, 3.8 * np.sqrt(a_mean))
    full = oracle.voronoi_forces(x, y, box, off, idx, *args)
    rows = np.array([3, 77, 1499, 640], np.int32)
    # only the rows the sampled forces need: the particles and their neighbours
    need = set(rows.tolist())
    for r in rows:
        need |= set(idx[off[r]:off[r + 1]].tolist())
    keep = [idx[off[i]:off[i + 1]] if i in need else np.zeros(0, np.int32) for i in range(n)]
    off2 = np.zeros(n + 1, np.int64)
    np.cumsum([len(k) for k in keep], out=off2[1:])
    part = oracle.voronoi_forces(x, y, box, off2, np.concatenate(keep), *args, rows=rows)
    assert np.array_equal(part["fx"], full["fx"][rows]) and np.array_equal(part["fy"], full["fy"][rows])
