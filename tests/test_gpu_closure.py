"""GPU parity of the per-material closure (each material's own density and
specific energy in mixed cells), through the C ABI.

FP64 bit for bit against the oracle: the two-gas contact at rest and
advected, layered and three-layer impacts on uniform and stretched grids,
every tile shape built for the closure and the tuner, ensembles of one-,
two- and three-material members, and the per-material state set and read
through salec_set_materials / salec_get_materials (also from an odd cycle).
The mixed mode meets the conserved-density bar of the other impacts.
"""
import dataclasses

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2403_04267_amd import inputs

from .crater import conserved_errors
from .test_gpu_parity import compare
from .test_oracle_closure import contact
from .test_oracle_three_layer import impact3

pytestmark = pytest.mark.gpu


def ctx(problems):
    from paper_2403_04267_amd.salec import Salec
    return Salec(problems)


class Member:
    def __init__(self, c, k):
        self.c, self.k = c, k

    def fields(self):
        return self.c.fields(k=self.k)

    def pml_aux(self):
        return self.c.pml_aux(k=self.k)

    def diag(self):
        return self.c.diag(k=self.k)

    def materials(self):
        return self.c.materials(k=self.k)


def pm(pb):
    return pb.replace(grid=dataclasses.replace(pb.grid, closure=1))


def same_materials(g, o, label):
    A, B = g.materials(), o.materials()
    for k in ("mu", "Im"):
        assert np.array_equal(A[k], B[k]), (label, k, np.abs(A[k] - B[k]).max())


def gpu_contact(n_r, n_z, j_mix, U=0.0, top_closed=1):
    """The oracle's two-gas contact (closure 1) and the same state on the GPU."""
    o = contact(n_r, n_z, j_mix, U=U, closure=1, top_closed=top_closed)
    c = ctx(o.problem)
    F, M = o.fields(eos=False), o.materials()
    c.set_fields(F["rho"], F["I"], F["f"], F["v"])
    c.set_materials(M["mu"], M["Im"])
    return c, o


def step_both(g, o, n):
    g.step(n)
    o.step(n)


def test_contact_at_rest_is_exact_on_the_gpu():
    c, o = gpu_contact(4, 30, 15)
    step_both(c, o, 200)
    F = c.fields()
    assert not np.any(F["v"]) and np.all(F["p"] == 1.0)
    compare(c, o, "contact at rest", tol=0.0, pml=False)
    same_materials(c, o, "contact at rest")


def test_advected_contact_fp64_bitwise():
    c, o = gpu_contact(6, 160, 80, U=1.0, top_closed=0)
    step_both(c, o, 8)
    compare(c, o, "advected contact", tol=0.0, pml=False)
    same_materials(c, o, "advected contact")


def test_layered_impact_per_material_fp64_bitwise():
    pb = pm(inputs.layered_impact(60, 12, 6, 15e3, 10, name="layered-pm"))
    g, o = ctx(pb), Oracle(pb)
    done = 0
    for n in (1, 60, 200):
        step_both(g, o, n - done)
        done = n
        compare(g, o, f"layered pm cycle {n}", tol=0.0)
        same_materials(g, o, f"layered pm cycle {n}")


def test_three_layer_per_material_fp64_bitwise():
    pb = pm(impact3())
    g, o = ctx(pb), Oracle(pb)
    done = 0
    for n in (1, 60, 150):
        step_both(g, o, n - done)
        done = n
        compare(g, o, f"three-layer pm cycle {n}", tol=0.0)
        same_materials(g, o, f"three-layer pm cycle {n}")


def test_stretched_three_layer_per_material_fp64_bitwise():
    from .test_gpu_three_layer import stretched3
    pb = pm(stretched3())
    g, o = ctx(pb), Oracle(pb)
    step_both(g, o, 80)
    compare(g, o, "stretched three-layer pm", tol=0.0)
    same_materials(g, o, "stretched three-layer pm")


@pytest.mark.parametrize("nmat", [2, 3])
def test_every_per_material_tile_shape_matches_the_oracle(nmat):
    from paper_2403_04267_amd.salec import SalecError, num_variants
    pb = pm(impact3() if nmat == 3 else inputs.layered_impact(50, 10, 5, 14e3, 8, name="layered-pm"))
    o = Oracle(pb)
    o.step(40)
    ran = []
    for v in range(num_variants()):
        c = ctx(pb)
        try:
            c.set_schedule(v, 0)
        except SalecError:
            continue  # not built for the per-material closure
        c.step(40)
        compare(c, o, f"pm nmat {nmat} shape {v}", tol=0.0)
        same_materials(c, o, f"pm nmat {nmat} shape {v}")
        ran.append(v)
    assert len(ran) >= 3, ran
    c = ctx(pb)
    s = c.tune(2)
    assert s["variant"] in ran
    advanced = int(c.diag()["cycle"])
    o2 = Oracle(pb)
    o2.step(advanced + 20)
    c.step(20)
    compare(c, o2, f"pm nmat {nmat} tuned", tol=0.0)


def test_ensemble_of_per_material_members():
    pbs = [pm(impact3()), pm(inputs.impact(41, 7, 5, 11e3, nmat=2, strength=True, cycles=0, name="two")),
           pm(inputs.impact(33, 5, 4, 9e3, nmat=1, strength=False, cycles=0, name="one")),
           pm(inputs.layered_impact(44, 8, 4, 13e3, 6, name="layered"))]
    c = ctx(pbs)
    os_ = [Oracle(p) for p in pbs]
    c.step(80)
    for k, o in enumerate(os_):
        o.step(80)
        compare(Member(c, k), o, f"pm member {pbs[k].name}", tol=0.0)
        same_materials(Member(c, k), o, f"pm member {pbs[k].name}")


def test_material_state_round_trip_and_restart_from_an_odd_cycle():
    pb = pm(inputs.layered_impact(40, 8, 4, 12e3, 6, name="layered-pm"))
    g, o = ctx(pb), Oracle(pb)
    step_both(g, o, 31)  # odd: the current state is the second level
    same_materials(g, o, "after 31 cycles")
    M = o.materials()
    rng = np.random.default_rng(5)
    Im = M["Im"] * rng.uniform(0.9, 1.1, size=M["Im"].shape)
    g.set_materials(M["mu"], Im)
    o.set_materials(M["mu"], Im)
    assert int(g.diag()["cycle"]) == 0
    compare(g, o, "after set_materials", tol=0.0)
    step_both(g, o, 40)
    compare(g, o, "40 cycles after set_materials", tol=0.0)
    same_materials(g, o, "40 cycles after set_materials")


def test_shared_closure_has_no_material_state():
    from paper_2403_04267_amd.salec import SalecError
    c = ctx(inputs.impact(30, 5, 4, 9e3, nmat=2, strength=False, cycles=0))
    with pytest.raises(SalecError):
        c.materials()


def test_three_layer_per_material_mixed_against_oracle():
    pb = pm(impact3())
    g, o = ctx(pb.replace(precision="mixed")), Oracle(pb)
    step_both(g, o, 100)
    e = conserved_errors(g.fields(), o.fields(), pb.grid)
    print("[three-layer pm mixed cycle 100] " + " ".join(f"{k} {v:.2e}" for k, v in e.items()), flush=True)
    bad = {k: v for k, v in e.items() if not v <= 1e-4}
    assert not bad, bad


def test_a_refused_shape_leaves_the_context_usable():
    from paper_2403_04267_amd.salec import SalecError
    pb = pm(impact3())
    c = ctx(pb)
    before = c.schedule()
    with pytest.raises(SalecError):
        c.set_schedule(0, 0)  # 64 x 14 does not fit the LDS with three per-material slots
    assert c.schedule() == before
    o = Oracle(pb)
    step_both(c, o, 30)
    compare(c, o, "after a refused shape", tol=0.0)
