"""Every seeded mesh generator yields a valid mesh, for several seeds and sizes.

Valid means:
  * every cell is a convex, counter-clockwise polygon of positive area;
  * every edge belongs to two cells, or to one cell and exactly one listed
    boundary face;
  * periodic pairs join two listed periodic edges of equal length;
  * the areas add up to the domain's area.
These are checks of the input generators, which hold none of the method's
arithmetic.
"""
import math

import numpy as np
import pytest

from paper_1812_00390_amd import meshgen as mg
from paper_1812_00390_amd import workloads as W


def _check(m, area=None):
    P = m.nodes
    ptr = m.cell_ptr
    edges = {}
    total = 0.0
    for c in range(m.n_cells):
        ids = m.cell_nodes[ptr[c]:ptr[c + 1]]
        k = len(ids)
        assert k in (3, 4), (m.name, c, k)
        q = P[ids]
        a2 = 0.0
        for j in range(k):
            p0, p1, p2 = q[j], q[(j + 1) % k], q[(j + 2) % k]
            cross = (p1[0] - p0[0]) * (p2[1] - p1[1]) - (p1[1] - p0[1]) * (p2[0] - p1[0])
            assert cross > 0.0, (m.name, c, "not convex and counter-clockwise")
            a2 += q[j][0] * q[(j + 1) % k][1] - q[(j + 1) % k][0] * q[j][1]
        total += 0.5 * a2
        for j in range(k):
            e = tuple(sorted((int(ids[j]), int(ids[(j + 1) % k]))))
            edges[e] = edges.get(e, 0) + 1
    assert max(edges.values()) <= 2
    open_edges = {e for e, n in edges.items() if n == 1}
    listed = [tuple(sorted(map(int, b))) for b in m.bface_nodes]
    assert len(listed) == len(set(listed)), "a boundary face listed twice"
    assert set(listed) == open_edges, (m.name, len(set(listed) ^ open_edges))
    assert np.all((m.bface_group >= -1) & (m.bface_group < len(m.groups)))
    for a, b in np.asarray(m.periodic).reshape(-1, 2):
        assert m.bface_group[a] == -1 and m.bface_group[b] == -1
        la = np.linalg.norm(np.subtract(*P[m.bface_nodes[a]]))
        lb = np.linalg.norm(np.subtract(*P[m.bface_nodes[b]]))
        assert la == pytest.approx(lb, rel=1e-12)
    n_per_edges = int(np.sum(m.bface_group == -1))
    assert n_per_edges == 2 * np.asarray(m.periodic).reshape(-1, 2).shape[0]
    if area is not None:
        assert total == pytest.approx(area, rel=1e-12)
    return total


@pytest.mark.parametrize("seed", range(5))
def test_cavity_and_channel_generators(seed):
    assert _check(mg.cavity(n=24, jitter=0.2, seed=seed), 1.0)
    assert _check(mg.cavity(n=12, jitter=0.2, seed=seed, tri=False), 1.0)
    assert _check(mg.streaming_cavity(16, seed=seed), 1.0)
    for tri in (True, False):
        for top in ("inlet", "symmetry", "wall"):
            _check(mg.channel(14, 7, jitter=0.2, seed=seed, tri=tri, top=top))
    _check(mg.channel(12, 6, jitter=0.2, seed=seed, tri=True, internal=1))


@pytest.mark.parametrize("seed", range(5))
def test_periodic_and_hybrid_generators(seed):
    _check(mg.periodic_box(9, 7, jitter=0.25, seed=seed))
    _check(mg.periodic_box(6, 6, jitter=0.25, seed=seed, tri=False))
    _check(mg.hybrid(10, seed=seed), 1.0)


@pytest.mark.parametrize("tri", [False, True])
def test_couette_generator(tri):
    m = mg.couette(8, 6, tri=tri)
    _check(m, 1.0)
    assert m.n_cells == (96 if tri else 48)


def test_cylinder_generators():
    for nr, nt in ((8, 12), (24, 36), (40, 60)):
        m = mg.cylinder(nr=nr, nt=nt, R=10.0, h0=0.02)
        assert m.n_cells == nr * nt
        # an annulus of polygonal rings: between the inscribed polygons of the two radii
        a = _check(m)
        inner = 0.5 * nt * 0.5 ** 2 * math.sin(2 * math.pi / nt)
        outer = 0.5 * nt * 10.0 ** 2 * math.sin(2 * math.pi / nt)
        assert a == pytest.approx(outer - inner, rel=1e-9)
    _check(mg.two_cylinders(nr=6, nt=16, half_width=8.0, height=8.0, h0=0.05))
    _check(mg.two_cylinders(nr=10, nt=24, half_width=8.0, height=8.0, h0=0.03))


def test_workload_instances():
    rng = np.random.default_rng(3)
    for _ in range(6):
        inst = W.served_instance(rng, float(np.exp(rng.uniform(math.log(2e3), math.log(2e4)))),
                                 kinds=("couette", "cavity", "cylinder"))
        _check(inst.mesh)
    _check(W.two_cylinder_instance(6, 12, 120.0).mesh)
