"""GPU against the FP64 oracle for the parts of the path that are not one
solver's fields: the time step rule (Eqs. 14, 15), the FP64 mass and
velocity residual (Eq. 32), batched solves and a served request.

Tolerances:
  * dt: both sides evaluate Eqs. 14-15 in FP64 from FP64 geometry computed
    independently (device and host), so they agree to a few FP64 ulps; 1e-12
    relative is asserted;
  * mass = sum A_i rho_i: the device sum is FP64 over the stored state; it
    equals the same sum formed on the host from the device's own rho and the
    oracle's areas to 1e-13 relative (summation order and area rounding), and
    the oracle's mass to total area x (density tolerance 1e-6 of FP32 storage);
  * residual: the device value equals Eq. 32 evaluated on the host from the
    device's own snapshots' fields to 1e-12 relative, and the oracle's value to
    the bound the field differences give (see _residual_bound);
  * batched and served fields: the tolerances of a single solve of the same
    storage (1e-5 U for FP32 deviations, 1e-3 U for the 16-bit formats).
"""
import numpy as np
import pytest

from paper_1812_00390_amd import meshgen as mg

pytestmark = pytest.mark.gpu

U = 0.1


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_00390_amd import fvlbm
    fvlbm.lib()
    return fvlbm


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


@pytest.mark.parametrize("name", ["cavity_cfg2", "cylinder_cfg3", "couette_cfg1"])
def test_device_time_step_matches_oracle(F, O, name):
    make, tau, cfl, u_ref = {
        "cavity_cfg2": (lambda: mg.cavity(n=100, ratio=1.08, jitter=0.2, seed=0, lid_u=0.1), 3e-4, 0.5, 0.1),
        "cylinder_cfg3": (lambda: mg.cylinder(nr=256, nt=384), 3e-3, 0.5, 0.2),
        "couette_cfg1": (lambda: mg.couette(16, 16, U=0.1), 0.8, 0.5, 0.1),
    }[name]
    m = make()
    o = O.Oracle(m, tau=tau, cfl=cfl, u_ref=u_ref, scheme="rk4")
    mesh = F.Mesh(m)
    s = F.Solver(mesh, F.make_params(tau=tau, dt=0.0, cfl=cfl, u_ref=u_ref, scheme="rk4"))
    assert s.dt == pytest.approx(o.dt, rel=1e-12, abs=0)
    # the CFL limit binds on these meshes (Eq. 15's 2 tau does not)
    assert s.dt < 2 * tau


def _residual_bound(u_g, uo_g, u_o, uo_o):
    """|r_g - r_o| for r = ||u - u_old|| / ||u_old|| from the two sides' fields:
    ||a_g|| / ||b_g|| - ||a_o|| / ||b_o|| with a = u - u_old, b = u_old is bounded
    by (||a_g - a_o|| + r_o ||b_g - b_o||) / ||b_g||."""
    a_g, a_o = u_g - uo_g, u_o - uo_o
    r_o = np.linalg.norm(a_o) / np.linalg.norm(uo_o)
    return (np.linalg.norm(a_g - a_o) + r_o * np.linalg.norm(uo_g - uo_o)) / np.linalg.norm(uo_g)


@pytest.mark.parametrize("storage", ["fp32dev", "i16dev", "fp16dev"])
def test_mass_and_residual_match_oracle(F, O, storage):
    """A closed cavity (mass conserved) and an open channel (mass changes through
    the inlet and outlet), with a residual lag of 60 steps."""
    cases = [(mg.cavity(n=24, jitter=0.2, seed=5, lid_u=U), 3e-3, (0.0, 0.0)),
             (mg.channel(20, 8, jitter=0.2, seed=2, tri=True, internal=1, top="symmetry", bottom="wall"),
              1e-2, (0.1, 0.0))]
    lag = 60
    for m, tau, u0 in cases:
        o = O.Oracle(m, tau=tau, cfl=0.5, u_ref=0.2, scheme="rk4")
        o.init(u0=u0)
        mesh = F.Mesh(m)
        s = F.Solver(mesh, F.make_params(tau=tau, dt=o.dt, scheme="rk4", storage=storage, u_ref=0.2, u_dev=u0,
                                         residual_lag=lag), u=np.tile(np.asarray(u0, float), (m.n_cells, 1)))
        area = o.geometry()["area"]
        mass0_o = o.mass()
        # Step 0's equilibrium differs from the storage reference (rounded to FP32) by
        # about 1e-9 w; FP16 deviations hold that in the moment carry, itself an FP16
        # value (11 significant bits): 1e-11 relative
        assert s.stats()["mass"] == pytest.approx(mass0_o, rel=1e-11 if storage == "fp16dev" else 1e-13)
        o.step(2 * lag)
        s.step(2 * lag)
        rho_g1, u_g1, _ = s.macros()
        rho_o1, u_o1 = o.macros()
        o.step(lag)
        s.step(lag)
        rho_g, u_g, st = s.macros()
        rho_o, u_o = o.macros()
        utol = 1e-5 if storage == "fp32dev" else 1e-3
        assert np.abs(u_g - u_o).max() <= utol * U
        # mass: the device's FP64 reduction, then against the oracle's
        assert st["mass"] == pytest.approx(float(np.sum(area * rho_g)), rel=1e-13)
        assert abs(st["mass"] - o.mass()) <= (1e-6 if storage == "fp32dev" else 1e-4) * area.sum()
        # residual of Eq. 32 over the last lag
        r_g, r_o = st["residual"], O.residual(u_o, u_o1)
        assert r_g > 0 and r_o > 0
        assert r_g == pytest.approx(O.residual(u_g, u_g1), rel=1e-12)
        assert abs(r_g - r_o) <= 1.01 * _residual_bound(u_g, u_g1, u_o, u_o1) + 1e-14
        s.close()
        mesh.close()


@pytest.mark.parametrize("storage,utol", [("fp32dev", 1e-5), ("i16dev", 1e-3), ("fp16dev", 1e-3)])
def test_batched_members_match_their_oracle_runs(F, O, storage, utol):
    """Triangles, quads and a hybrid mesh with different tau and dt, advanced by
    shared launches; every member against its own FP64 run."""
    cases = [(mg.cavity(n=20, jitter=0.2, seed=10, lid_u=U), 3e-3, 0.1, (0.0, 0.0)),
             (mg.cylinder(nr=12, nt=18, R=6.0, h0=0.05), 3e-3, 0.2, (0.1, 0.0)),
             (mg.hybrid(10), 2e-3, 0.1, (0.0, 0.0)),
             (mg.cavity(n=9, jitter=0.2, seed=11, tri=False, lid_u=U), 1e-3, 0.1, (0.0, 0.0))]
    steps = 150
    members, oracles = [], []
    for m, tau, u_ref, u0 in cases:
        o = O.Oracle(m, tau=tau, cfl=0.5, u_ref=u_ref, scheme="rk4")
        o.init(u0=u0)
        o.step(steps)
        oracles.append(o)
        mesh = F.Mesh(m)
        members.append((mesh, F.Solver(mesh, F.make_params(tau=tau, dt=o.dt, scheme="rk4", storage=storage,
                                                           u_ref=u_ref, u_dev=u0),
                                       u=np.tile(np.asarray(u0, float), (m.n_cells, 1)))))
    b = F.Batch([s for _, s in members])
    b.step(steps)
    for (mesh, s), o in zip(members, oracles):
        rho_g, u_g, st = s.macros()
        rho_o, u_o = o.macros()
        assert st["steps"] == steps
        err = np.abs(u_g - u_o).max()
        print(f"batched {storage} {mesh.n_cells} cells: max|u-u_oracle|/U = {err / U:.3e}")
        assert err <= utol * U
        assert np.abs(rho_g - rho_o).max() <= utol * U


@pytest.mark.parametrize("storage,utol", [("fp32dev", 1e-5), ("i16dev", 1e-3), ("fp16dev", 1e-3)])
def test_served_request_matches_its_oracle_run(F, O, storage, utol):
    from paper_1812_00390_amd import workloads as W
    from paper_1812_00390_amd.serve import GpuBackend, Request, Server
    insts = [W.cavity_instance(16, 400.0, seed=3), W.cylinder_instance(10, 16, 150.0),
             W.cavity_instance(12, 900.0, seed=4)]
    chunk, budget = 50, 150
    reqs = [Request(k, inst, tol=0.0, budget=budget, arrival=0.0) for k, inst in enumerate(insts)]
    backend = GpuBackend(chunk=chunk, storage=storage, autotune=False)
    srv = Server(backend, hbm_budget=2 ** 31, max_slots=2, chunk=chunk, keep_fields=True, prep_workers=2)
    res = {r.rid: r for r in srv.run(reqs)}
    assert sorted(res) == [0, 1, 2]
    for k, inst in enumerate(insts):
        o = O.Oracle(inst.mesh, tau=inst.tau, cfl=0.5, u_ref=inst.u_ref, scheme="rk4")
        o.init(u0=inst.u0)
        o.step(budget)
        rho_o, u_o = o.macros()
        assert res[k].steps == budget
        err = np.abs(res[k].u - u_o).max()
        print(f"served {storage} request {k} ({inst.n_cells} cells): max|u-u_oracle|/U = {err / U:.3e}")
        assert err <= utol * U
        assert np.abs(res[k].rho - rho_o).max() <= utol * U


def test_batched_workload_full_size_vs_stored_oracle(F):
    """The benchmark's batched workload: 64 seeded instances (2.9M cells), FP16
    deviations, shared launches at the autotuned schedule, 1000 RK4 steps; every
    instance against its stored FP64 oracle run (tests/golden)."""
    import os
    from paper_1812_00390_amd import workloads as W
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "oracle_batched64_rk4_1000.npz"))
    insts = W.batched()
    assert len(insts) == int(ref["n"])
    pairs = []
    for inst in insts:
        mesh = F.Mesh(inst.mesh)
        s = F.Solver(mesh, F.make_params(tau=inst.tau, cfl=0.5, u_ref=inst.u_ref, scheme="rk4", storage="fp16dev",
                                         u_dev=inst.u0), u=np.tile(np.asarray(inst.u0, float), (inst.n_cells, 1)))
        pairs.append((mesh, s))
    for k, (_, s) in enumerate(pairs):
        assert s.dt == pytest.approx(float(ref[f"dt_{k}"]), rel=1e-12)
    b = F.Batch([s for _, s in pairs])
    b.autotune(8)
    b.step(int(ref["steps"]))
    worst = 0.0
    for k, (_, s) in enumerate(pairs):
        rho, u, st = s.macros()
        assert st["steps"] == int(ref["steps"])
        err = np.abs(u[ref[f"idx_{k}"]] - ref[f"u_{k}"]).max() / U
        worst = max(worst, err)
        assert err <= 1e-3, (k, err)
        # density: the velocity target through the acoustic relation d rho = d u / c_s
        # (c_s^2 = 1/3 in the equilibrium, Eq. 3), sqrt(3) 1e-3 U, rounded up
        assert np.abs(rho[ref[f"idx_{k}"]] - ref[f"rho_{k}"]).max() <= 2e-4
    print(f"batched 64 instances fp16dev 1000 steps: worst max|u-u_oracle|/U = {worst:.3e}, schedule {b.get_schedule()}")
