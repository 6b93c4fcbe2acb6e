"""GPU: handle lifetimes across the C ABI.

A mesh destroyed while solvers still use it, a solver destroyed while a
batch holds it, and meshes and solvers released by the cycle collector in any
order must neither fault nor corrupt the host heap.  The library defers the
release of a mesh to its last solver and of a solver to its last batch.
"""
import gc

import numpy as np
import pytest

from paper_1812_00390_amd import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_00390_amd import fvlbm
    fvlbm.lib()
    return fvlbm


def _fresh_solve(F, n=10, steps=12):
    mesh = F.Mesh(mg.cavity(n=n, jitter=0.2, seed=30))
    s = F.Solver(mesh, F.make_params(tau=1e-3, scheme="rk4", storage="fp32dev"))
    s.step(steps)
    rho, u, st = s.macros()
    assert np.all(np.isfinite(u)) and st["steps"] == steps
    return mesh, s, u


def test_mesh_destroyed_before_its_solver(F):
    _, _, u_ref = _fresh_solve(F)
    mesh = F.Mesh(mg.cavity(n=10, jitter=0.2, seed=30))
    s = F.Solver(mesh, F.make_params(tau=1e-3, scheme="rk4", storage="fp32dev"))
    # release the mesh through the C ABI while the solver still reads it
    F.lib().fvlbm_mesh_destroy(mesh.h)
    F.lib().fvlbm_mesh_destroy(mesh.h)          # a second call while deferred is a no-op
    mesh.h = None
    s.step(12)
    _, u, st = s.macros()
    assert np.array_equal(u, u_ref) and st["steps"] == 12
    s.close()                                    # frees the mesh too
    _fresh_solve(F)                              # the heap and the device are intact


def test_cycle_collector_releases_meshes_and_solvers_in_any_order(F):
    _, _, u_ref = _fresh_solve(F)
    for k in range(6):
        mesh = F.Mesh(mg.cavity(n=10, jitter=0.2, seed=30))
        s = F.Solver(mesh, F.make_params(tau=1e-3, scheme="rk4", storage="fp32dev"))
        s.step(12)
        b = F.Batch([s])
        # a reference cycle through all three objects, so their finalizers run in
        # the collector's order rather than by reference counts
        mesh.cycle, s.cycle, b.cycle = s, b, mesh
        del mesh, s, b
        gc.collect()
    _, _, u = _fresh_solve(F)
    assert np.array_equal(u, u_ref)


def test_solver_destroyed_while_in_a_batch(F):
    mesh_a, a, _ = _fresh_solve(F)
    mesh_b, b_s, _ = _fresh_solve(F, n=8)
    b = F.Batch([a, b_s])
    b.step(3)
    a.close()                                    # deferred: the batch still holds it
    with pytest.raises(F.FvlbmError) as e:
        b.step(1)
    assert e.value.status == -7
    b.close()                                    # frees the destroyed member
    b_s.step(2)                                  # the other member is usable alone
    assert b_s.stats()["steps"] == 12 + 3 + 2
    _fresh_solve(F)


def test_batch_reports_the_schedule_it_runs(F):
    meshes = [mg.cavity(n=14, jitter=0.2, seed=16), mg.cylinder(nr=10, nt=16, R=6.0, h0=0.05)]
    solvers = []
    for m in meshes:
        mesh = F.Mesh(m)
        solvers.append((mesh, F.Solver(mesh, F.make_params(tau=2e-3, scheme="rk4", storage="fp32dev", u_ref=0.2))))
    b = F.Batch([s for _, s in solvers])
    for block, x, p in [(128, False, True), (512, True, False), (64, True, False)]:
        b.set_schedule(block, x, p)
        assert b.get_schedule() == dict(block=block, xcd_remap=x, persistent=p)
    b.autotune(8)
    sch = b.get_schedule()
    assert sch["block"] in (64, 128, 256, 512)
    # the reported schedule is the one the batch holds: setting it again changes nothing
    b.set_schedule(sch["block"], sch["xcd_remap"], sch["persistent"])
    assert b.get_schedule() == sch
