"""GPU: a request's result is the same served in a changing mix as run alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_00390_amd import fvlbm
    fvlbm.lib()
    return fvlbm


def test_served_equals_alone_bitwise(F):
    from paper_1812_00390_amd import workloads as W
    from paper_1812_00390_amd.serve import GpuBackend, Request, Server
    rng = np.random.default_rng(7)
    insts = [W.cavity_instance(20, 400.0, seed=3), W.cylinder_instance(12, 18, 150.0),
             W.two_cylinder_instance(6, 12, 120.0), W.cavity_instance(14, 900.0, seed=4),
             W.cylinder_instance(10, 16, 300.0)]
    chunk = 64
    budgets = [128, 320, 192, 256, 128]
    reqs = [Request(k, inst, tol=0.0, budget=b, arrival=0.0) for k, (inst, b) in enumerate(zip(insts, budgets))]
    backend = GpuBackend(chunk=chunk, autotune=False)
    srv = Server(backend, hbm_budget=2 ** 31, max_slots=3, chunk=chunk, keep_fields=True, prep_workers=2)
    res = {r.rid: r for r in srv.run(reqs)}
    assert sorted(res) == list(range(5))
    # membership changed while requests ran: more requests than slots
    assert srv.used == 0
    for k, inst in enumerate(insts):
        mesh = F.Mesh(inst.mesh, reorder=inst.order)
        p = F.make_params(tau=inst.tau, cfl=0.5, u_ref=inst.u_ref, scheme="rk4", storage=backend.storage,
                          u_dev=inst.u0, residual_lag=chunk)
        s = F.Solver(mesh, p, u=np.tile(np.asarray(inst.u0, float), (inst.n_cells, 1)))
        for _ in range(budgets[k] // chunk):
            s.step(chunk)
        rho, u, st = s.macros()
        assert st["steps"] == res[k].steps
        assert np.array_equal(rho, res[k].rho) and np.array_equal(u, res[k].u), k
