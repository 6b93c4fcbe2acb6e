"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and rejects invalid meshes and arguments before touching the device."""
import os
import re

import numpy as np
import pytest

from paper_1812_00390_amd import fvlbm as F
from paper_1812_00390_amd import meshgen as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "fvlbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fvlbm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 20
    L = F.lib()
    for n in names:
        assert hasattr(L, n), n
        assert n in F.SIGNATURES, n


def test_struct_layouts_match_header():
    import ctypes as C
    assert C.sizeof(F.BC) == 32
    assert C.sizeof(F.Params) == 4 * 8 + 2 * 4 + 2 * 8 + 2 * 4 + 2 * 8


def _raises_status(fn, status):
    with pytest.raises(F.FvlbmError) as ei:
        fn()
    assert ei.value.status == status, str(ei.value)


def test_rejects_clockwise_cells():
    bad = mg.couette(4, 4)
    bad.cell_nodes = bad.cell_nodes.reshape(-1, 4)[:, ::-1].ravel().copy()
    _raises_status(lambda: F.Mesh(bad, stream=0), -2)


def test_rejects_open_boundary():
    m = mg.couette(4, 4)
    m.bface_nodes = m.bface_nodes[1:]; m.bface_group = m.bface_group[1:]
    m.periodic = m.periodic - 1
    _raises_status(lambda: F.Mesh(m, stream=0), -2)


def test_rejects_mismatched_periodic_pair():
    m = mg.couette(4, 4)
    m.periodic_shift = m.periodic_shift * 0.5
    _raises_status(lambda: F.Mesh(m, stream=0), -2)


def test_rejects_bad_group_and_polygon():
    m = mg.couette(4, 4)
    m.bface_group = m.bface_group.copy(); m.bface_group[m.bface_group >= 0] = 7
    _raises_status(lambda: F.Mesh(m, stream=0), -2)
    m = mg.cavity(n=4, jitter=0.0)
    m.groups = [mg.BCGroup(9)] + m.groups[1:]
    _raises_status(lambda: F.Mesh(m, stream=0), -1)


def test_rejects_nonconvex_cell():
    m = mg.cavity(n=3, jitter=0.0, tri=False)
    nodes = m.nodes.copy()
    nodes[5] = nodes[5] + np.array([0.3, 0.3])     # pull an interior node far inside a neighbour
    m.nodes = nodes
    _raises_status(lambda: F.Mesh(m, stream=0), -2)


def test_null_arguments():
    L = F.lib()
    assert L.fvlbm_step(None, 1) == -1
    assert L.fvlbm_macros(None, None, None, None) == -1
    assert L.fvlbm_state_bytes(None, None) == 0
    assert L.fvlbm_mesh_cfl_length(None) == -1.0
    assert L.fvlbm_solver_dt(None) == -1.0
    assert L.fvlbm_batch_create(None, 0, None) == -1
    assert L.fvlbm_batch_remove(None, None) == -1
    L.fvlbm_solver_destroy(None); L.fvlbm_mesh_destroy(None); L.fvlbm_batch_destroy(None)
    assert b"bad arguments" in L.fvlbm_last_error()


def test_rejects_empty_and_degenerate_meshes():
    """No cells, no nodes, a cell of two corners or of more corners than a cell may
    have, a corner index out of range, a zero-area (collinear) triangle: each is an
    argument or mesh error, raised before any device call."""
    m = mg.cavity(n=2, jitter=0.0)
    empty = mg.RawMesh(m.nodes, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros((0, 2), np.int32),
                       np.zeros(0, np.int32), m.groups, np.zeros((0, 2), np.int32), np.zeros((0, 2)), name="empty")
    _raises_status(lambda: F.Mesh(empty, stream=0), -1)
    no_nodes = mg.RawMesh(np.zeros((0, 2)), m.cell_ptr, m.cell_nodes, m.bface_nodes, m.bface_group, m.groups,
                          m.periodic, m.periodic_shift, name="no_nodes")
    _raises_status(lambda: F.Mesh(no_nodes, stream=0), -1)
    for ptr, nodes_of in ((np.array([0, 2], np.int32), np.array([0, 1], np.int32)),
                          (np.array([0, 5], np.int32), np.array([0, 1, 4, 3, 2], np.int32))):
        bad = mg.RawMesh(m.nodes, ptr, nodes_of, m.bface_nodes, m.bface_group, m.groups, m.periodic,
                         m.periodic_shift, name="bad_polygon")
        with pytest.raises(F.FvlbmError):
            F.Mesh(bad, stream=0)
    out_of_range = mg.cavity(n=2, jitter=0.0)
    out_of_range.cell_nodes = out_of_range.cell_nodes.copy()
    out_of_range.cell_nodes[0] = out_of_range.n_nodes + 3
    with pytest.raises(F.FvlbmError):
        F.Mesh(out_of_range, stream=0)
    flat = mg.cavity(n=2, jitter=0.0)
    nodes = flat.nodes.copy()
    a, b, c = flat.cell_nodes[:3]
    nodes[c] = 0.5 * (nodes[a] + nodes[b])          # the first triangle's third corner on its first edge
    flat.nodes = nodes
    _raises_status(lambda: F.Mesh(flat, stream=0), -2)
