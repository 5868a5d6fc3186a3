"""GPU parity of launch schedules and ensembles, through the C ABI.

Every tile shape and workgroup count must give bit-identical results (the
arithmetic of a cell never depends on the tile that computes it), an
ensemble member must reproduce its own oracle run exactly as if it ran
alone (each member keeps its own time step), an error in one member must not
stop the others, and the tuner must not change results.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2403_04267_amd import inputs

from .test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def ctx(problems):
    from paper_2403_04267_amd.salec import Salec
    return Salec(problems)


class Member:
    """View of one ensemble member with the Salec interface compare() uses."""

    def __init__(self, c, k):
        self.c, self.k = c, k

    def fields(self):
        return self.c.fields(k=self.k)

    def pml_aux(self):
        return self.c.pml_aux(k=self.k)

    def diag(self):
        return self.c.diag(k=self.k)


def small_members():
    # uneven sizes, radii, speeds and strengths; ragged against every tile shape
    spec = [(30, 5, 4, 6e3, 5e6), (47, 7, 5, 11e3, 20e6), (23, 3, 3, 17e3, 1e6), (64, 9, 6, 9e3, 45e6),
            (38, 6, 4, 14e3, 12e6)]
    return [inputs.impact(n, p, R, v, nmat=2, strength=True, cycles=0, Y0=y, name=f"m{n}")
            for (n, p, R, v, y) in spec]


def test_every_tile_shape_matches_the_oracle():
    from paper_2403_04267_amd.salec import SalecError, num_variants
    pb = inputs.impact(61, 13, 6, 15e3, nmat=2, strength=True, cycles=0, name="shapes")
    o = Oracle(pb)
    o.step(60)
    for v in range(num_variants()):
        for grid in (0, 24):
            c = ctx(pb)
            try:
                c.set_schedule(v, grid)
            except SalecError:
                assert v in (11, 14)  # built for three slots and the per-material closure only
                continue
            sch = c.schedule()
            assert sch["variant"] == v
            c.step(60)
            compare(c, o, f"variant {v} grid {grid} ({sch['tile_r']}x{sch['tile_z']})", tol=0.0)


def test_ensemble_members_match_their_own_oracles():
    members = small_members()
    c = ctx(members)
    assert c.num_instances == len(members)
    oracles = [Oracle(pb) for pb in members]
    done = 0
    for n in (1, 40, 150):
        c.step(n - done)
        for o in oracles:
            o.step(n - done)
        done = n
        for k, o in enumerate(oracles):
            compare(Member(c, k), o, f"member {k} cycle {n}")
    dts = {c.diag(k=k)["dt"] for k in range(len(members))}
    assert len(dts) == len(members)  # every member kept its own step


def test_ensemble_error_in_one_member_leaves_the_others_running():
    from paper_2403_04267_amd.salec import SalecError
    members = small_members()[:3]
    c = ctx(members)
    oracles = [Oracle(pb) for pb in members]
    g = members[1].grid
    F = oracles[1].fields(eos=False)
    I = F["I"].copy()
    I[g.NZ // 2, 3] = np.nan
    c.set_fields(F["rho"], I, F["f"], F["v"], F["s"], k=1)
    with pytest.raises(SalecError) as e:
        c.step(10)
    assert e.value.code == -4
    assert c.diag(k=1)["err"] == -4 and c.diag(k=1)["err_cycle"] == 1
    for k in (0, 2):
        oracles[k].step(10)
        compare(Member(c, k), oracles[k], f"healthy member {k}")
    # the healthy members keep advancing while the failed one stays put
    assert c.step(5, check=False) == -4
    assert c.diag(k=0)["cycle"] == 15 and c.diag(k=1)["cycle"] == 1
    # a new state for the failed member clears its error
    c.set_fields(F["rho"], F["I"], F["f"], F["v"], F["s"], k=1)
    assert c.step(3) == 0


def test_tuner_picks_a_schedule_without_changing_results():
    from paper_2403_04267_amd.salec import num_variants
    members = small_members()
    a, b = ctx(members), ctx(members)
    sch = a.tune(2)
    assert 0 <= sch["variant"] < num_variants() and sch["ms_per_cycle"] > 0
    # (cycles + 1) per candidate: every shape, some also with a persistent grid
    advanced = int(a.diag(k=0)["cycle"])
    # (two shapes are not built for two-material shared-closure contexts)
    assert advanced % 3 == 0 and 3 * (num_variants() - 2) <= advanced <= 6 * num_variants()
    b.step(advanced)
    a.step(20)
    b.step(20)
    for k in range(len(members)):
        Fa, Fb = a.fields(k=k), b.fields(k=k)
        for name in Fa:
            assert np.array_equal(Fa[name], Fb[name]), (k, name)


def test_ensemble_checkpoint_restart_is_bitwise():
    members = small_members()[:3]
    a, b = ctx(members), ctx(members)
    a.step(50)
    b.step(20)
    blob = b.get_state()
    b.step(7)
    b.set_state(blob)
    b.step(30)
    for k in range(len(members)):
        Fa, Fb = a.fields(k=k), b.fields(k=k)
        for name in Fa:
            assert np.array_equal(Fa[name], Fb[name]), (k, name)


def test_kernel_timing_advances_like_step():
    """salec_time_kernels runs the same kernels eagerly: same bits as graphs."""
    members = small_members()[:2]
    a, b = ctx(members), ctx(members)
    a.step(25)
    ms_cycle, ms_fin = b.time_kernels(25)
    assert ms_cycle > 0 and ms_fin > 0
    for k in range(len(members)):
        assert b.diag(k=k)["cycle"] == 25
        Fa, Fb = a.fields(k=k), b.fields(k=k)
        for name in Fa:
            assert np.array_equal(Fa[name], Fb[name]), (k, name)
