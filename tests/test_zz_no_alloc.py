"""GPU: fvlbm_macros_noalloc (no allocation, partial sums in the library's
static scratch) against fvlbm_macros, through the C ABI: two calls in a row,
the second on a smaller mesh, then a diverged state (flag set) and a healthy
one again (the flag is cleared by the call)."""
import ctypes as C

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


def _noalloc(F, s):
    import torch
    n = s.n
    rho = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
    u = torch.full((n, 2), -7.0, dtype=torch.float64, device="cuda")
    stats = torch.full((2,), -7.0, dtype=torch.float64, device="cuda")
    st = F.lib().fvlbm_macros_noalloc(s.h, C.c_void_p(rho.data_ptr()), C.c_void_p(u.data_ptr()),
                                      C.c_void_p(stats.data_ptr()))
    assert st == 0, F.lib().fvlbm_last_error().decode()
    torch.cuda.synchronize()
    return rho.cpu().numpy(), u.cpu().numpy(), stats.cpu().numpy()


def test_noalloc_macros_match_macros(F):
    cases = [(mg.cylinder(nr=40, nt=60, R=8.0, h0=0.02), "fp16dev", 3e-3, (0.1, 0.0), 0.2),
             (mg.cavity(n=12, jitter=0.2, seed=4, lid_u=0.1), "fp32dev", 3e-3, (0.0, 0.0), 0.1)]
    sizes = []
    for m, storage, tau, u0, u_ref in cases:      # the second mesh is the smaller one
        mesh = F.Mesh(m)
        s = F.Solver(mesh, F.make_params(tau=tau, scheme="rk4", storage=storage, u_ref=u_ref, u_dev=u0),
                     u=np.tile(np.asarray(u0, float), (m.n_cells, 1)))
        s.step(60)
        rho_n, u_n, stats_n = _noalloc(F, s)
        rho, u, st = s.macros()
        assert np.array_equal(rho_n, rho) and np.array_equal(u_n, u)
        assert stats_n[0] == st["mass"] and stats_n[1] == 0.0
        sizes.append(m.n_cells)
    assert sizes[1] < sizes[0]


def test_noalloc_flags_a_diverged_state_and_clears_the_flag(F):
    m = mg.cavity(n=6)
    mesh = F.Mesh(m)
    bad = F.Solver(mesh, F.make_params(tau=1e-3, dt=1e-2, flags=F.FLAG_FORCE_DT))   # dt > 2 tau: diverges
    bad.step(400)
    _, _, stats = _noalloc(F, bad)
    assert stats[1] == 1.0
    good = F.Solver(mesh, F.make_params(tau=1e-3, scheme="rk4"))
    good.step(5)
    rho, u, stats = _noalloc(F, good)
    assert stats[1] == 0.0 and np.all(np.isfinite(u))
    assert stats[0] == good.stats()["mass"]
