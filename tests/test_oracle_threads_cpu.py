"""The oracle's OpenMP timing build (the same source compiled with -fopenmp,
used only to time the oracle on all host cores) gives bitwise the results of
the one-thread build: its parallel loops are over cells, each iteration
writing only its own cell and keeping its own summation order."""
import numpy as np
import pytest

from paper_1812_00390_amd import meshgen as mg


@pytest.mark.parametrize("scheme", ["rk4", "euler", "ab2"])
def test_openmp_build_is_bitwise_the_one_thread_build(oracle_mod, scheme):
    cases = [(mg.cylinder(nr=24, nt=36, R=8.0, h0=0.02), 3e-3, 0.2, (0.1, 0.0)),
             (mg.cavity(n=14, jitter=0.2, seed=3, lid_u=0.1), 3e-3, 0.1, (0.0, 0.0)),
             (mg.channel(12, 6, jitter=0.2, seed=4, tri=True, internal=1, top="symmetry"), 1e-2, 0.2, (0.1, 0.0))]
    for m, tau, u_ref, u0 in cases:
        a = oracle_mod.Oracle(m, tau=tau, cfl=0.5, u_ref=u_ref, scheme=scheme)
        b = oracle_mod.Oracle(m, tau=tau, cfl=0.5, u_ref=u_ref, scheme=scheme, threads=4)
        assert b.threads == 4
        for o in (a, b):
            o.init(u0=u0)
            o.step(15)
        assert np.array_equal(a.f, b.f)
        assert a.mass() == b.mass()
