"""GPU: a batch whose members change in place (fvlbm_batch_set_members) advances
every member bitwise as it advances alone, with its instantiated graphs
re-pointed at the new members rather than built again."""
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


# triangles and quadrilaterals of several sizes (the launch grid and the LDS size
# change with the membership)
MESHES = [(lambda: mg.cavity(n=20, jitter=0.2, seed=30), 3e-4),
          (lambda: mg.cylinder(nr=12, nt=18, R=6.0, h0=0.05), 3e-3),
          (lambda: mg.cavity(n=9, jitter=0.2, seed=31), 1e-3),
          (lambda: mg.hybrid(8), 2e-3),
          (lambda: mg.cylinder(nr=20, nt=30, R=6.0, h0=0.05), 2e-3),
          (lambda: mg.cavity(n=30, jitter=0.2, seed=32), 1e-3)]


def _pairs(F, storage, lag=None):
    alone, mixed = [], []
    for make, tau in MESHES:
        m = make()
        for dst in (alone, mixed):
            mesh = F.Mesh(m)
            p = F.make_params(tau=tau, scheme="rk4", storage=storage, u_ref=0.2,
                              **({} if lag is None else dict(residual_lag=lag)))
            dst.append((mesh, F.Solver(mesh, p)))
    return alone, mixed


@pytest.mark.parametrize("storage,persistent", [("fp32dev", False), ("fp16dev", False), ("fp32dev", True)])
def test_members_change_in_place_bitwise(F, storage, persistent):
    alone, mixed = _pairs(F, storage)
    S = [s for _, s in mixed]
    steps = [0] * len(S)
    plan = [([0, 1, 2], 16),
            ([2, 1, 4], 24),              # one leaves, one joins, order changes: same cell kinds
            ([3, 5, 0], 16),              # the first member rejoins: both cell kinds again
            ([2, 5], 8),                  # triangles only: graphs rebuilt
            ([3, 0, 5, 1, 2, 4], 16)]     # grows back to both kinds
    b = None
    repointed = []
    for members, n in plan:
        if b is None:
            b = F.Batch([S[i] for i in members])
            b.set_schedule(128, True, persistent)      # (work-queue form: one queue per cell kind)
        else:
            b.set_members([S[i] for i in members])
        repointed.append(b.graph_counts()["repointed"])
        b.step(n)
        for i in members:
            steps[i] += n
    c = b.graph_counts()
    assert repointed[1] >= 1 and repointed[2] > repointed[1], repointed   # kinds unchanged: re-pointed
    assert repointed[3] == repointed[2] and repointed[4] == repointed[3], repointed  # kinds changed: rebuilt
    assert c["built"] >= 2
    for k, ((_, a), x) in enumerate(zip(alone, S)):
        a.step(steps[k])
        assert x.stats()["steps"] == steps[k]
        assert np.array_equal(a.f, x.f), k
    if storage == "fp16dev":
        for (_, a), x in zip(alone, S):
            ra, ua, _ = a.macros()
            rx, ux, _ = x.macros()
            assert np.array_equal(ra, rx) and np.array_equal(ua, ux)
    b.close()


def test_residuals_follow_the_members(F):
    alone, mixed = _pairs(F, "fp32dev", lag=16)
    S = [s for _, s in mixed]
    b = F.Batch([S[0], S[1]])
    b.step(32)
    b.set_members([S[4], S[0], S[3]])
    b.step(32)
    res, steps = b.residuals()
    for (_, a), n in zip((alone[4], alone[0], alone[3]), (32, 64, 32)):
        a.step(n)
    assert list(steps) == [32, 64, 32]
    for r, (_, a) in zip(res, (alone[4], alone[0], alone[3])):
        assert r == a.stats()["residual"] > 0
    b.close()


def test_rejected_members_leave_the_batch_unchanged(F):
    alone, mixed = _pairs(F, "fp32dev")
    S = [s for _, s in mixed]
    b = F.Batch([S[0], S[1]])
    b.step(8)
    with pytest.raises(F.FvlbmError):
        b.set_members([S[2], S[2]])                     # a solver twice
    other = F.Solver(mixed[3][0], F.make_params(tau=2e-3, scheme="euler", storage="fp32dev", u_ref=0.2))
    with pytest.raises(F.FvlbmError):
        b.set_members([S[2], other])                    # another scheme
    b.step(8)
    for (_, a), x in zip(alone[:2], S[:2]):
        a.step(16)
        assert np.array_equal(a.f, x.f)
    other.close()
    b.close()


def test_member_destroyed_in_the_batch_is_freed_when_it_leaves(F):
    _, mixed = _pairs(F, "fp32dev")
    S = [s for _, s in mixed]
    b = F.Batch([S[0], S[1], S[2]])
    b.step(8)
    S[1].close()                                        # deferred: the batch still holds it
    with pytest.raises(F.FvlbmError):
        b.step(8)                                       # a destroyed member: the batch refuses
    mixed[1][0].close()
    b.set_members([S[0], S[2]])                         # it leaves and is freed with its mesh
    b.step(8)
    assert S[0].stats()["steps"] == 16 and S[2].stats()["steps"] == 16
    b.close()


def test_remove_one_member(F):
    """fvlbm_batch_remove: the others go on bitwise as alone, with the graphs re-pointed
    while the batch keeps its cell kinds; the removed solver steps on alone; a
    non-member or the last member is refused and leaves the batch as it was."""
    alone, mixed = _pairs(F, "fp32dev")
    S = [s for _, s in mixed]                           # 0, 2, 5 triangles; 1 quadrilaterals
    b = F.Batch([S[0], S[1], S[2], S[5]])
    b.step(16)
    before = b.graph_counts()["repointed"]
    b.remove(S[2])                                      # both cell kinds stay: graphs re-pointed
    assert b.graph_counts()["repointed"] > before
    assert [s.h.value for s in b.solvers] == [S[0].h.value, S[1].h.value, S[5].h.value]
    b.step(8)
    S[2].step(8)                                        # on its own again
    with pytest.raises(F.FvlbmError) as e:
        b.remove(S[3])                                  # never a member
    assert e.value.status == -1
    b.remove(S[0]); b.remove(S[5])
    with pytest.raises(F.FvlbmError) as e:
        b.remove(S[1])                                  # the last member
    assert e.value.status == -7
    b.step(8)                                           # S[1] alone in the batch
    for k, n in ((0, 24), (1, 32), (2, 24), (5, 24)):
        alone[k][1].step(n)
        assert S[k].stats()["steps"] == n
        assert np.array_equal(alone[k][1].f, S[k].f), k
    b.close()
