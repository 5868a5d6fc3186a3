"""GPU parity of the PML placement that follows Sec. 3's sentence as printed
(salec_pml.placement = 1: phi2 in the node force, phi1 on the mass and phi3
on the energy at the end of the Lagrangian step, psi2 in the cell remap, psi1
in the momentum remap), through the C ABI.

FP64 bit for bit against the oracle run with the same placement: impacts with
and without strength, a seeded random state with void and prestress, the
layered lithostatic target under the per-material closure, a stretched grid
and an ensemble mixing both placements. The mixed mode meets the
conserved-density bar of the other impacts.
"""
import dataclasses

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2403_04267_amd import inputs

from .crater import conserved_errors
from .test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def printed(pb, **kw):
    return pb.replace(pml=dataclasses.replace(pb.pml, placement=1, **kw))


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


def run_pair(pb, checkpoints, label):
    g, o = ctx(pb), Oracle(pb)
    done = 0
    for n in checkpoints:
        g.step(n - done)
        o.step(n - done)
        done = n
        compare(g, o, f"{label} cycle {n}", tol=0.0)
    return g, o


def test_printed_placement_small_hydro_impact_bitwise():
    pb = printed(inputs.config_small())
    g, o = run_pair(pb, [1, 10, 100, 300], "printed hydro")
    # the layers' sink took the phi1 mass in the Lagrangian step too
    assert g.diag()["mass_pml"] != 0.0


def test_printed_placement_strength_impact_bitwise():
    pb = printed(inputs.impact(61, 13, 6, 15e3, nmat=2, strength=True, cycles=0, name="strength-61"))
    run_pair(pb, [1, 40, 200], "printed strength")


def test_printed_placement_random_state_bitwise():
    pb = printed(inputs.impact(70, 10, 5, 1e4, nmat=2, strength=True, cycles=0, name="random"),
                 damp_stress=1)
    pb.scene = None
    g = pb.grid
    rng = np.random.default_rng(23)
    NR, NZ = g.NR, g.NZ
    f = np.zeros((2, NZ, NR))
    f[0] = np.clip(rng.uniform(-0.3, 1.3, size=(NZ, NR)), 0, 1)
    f[1] = np.clip(rng.uniform(-0.5, 1.0, size=(NZ, NR)), 0, 1) * (1 - f[0])
    rho = 2860.0 * f.sum(0) * rng.uniform(0.9, 1.3, size=(NZ, NR))
    I = rng.uniform(0, 3e7, size=(NZ, NR))
    v = rng.uniform(-2e3, 2e3, size=(2, NZ + 1, NR + 1))
    s = rng.uniform(-5e6, 5e6, size=(3, NZ, NR))
    gc, oc = ctx(pb), Oracle(pb)
    gc.set_fields(rho, I, f, v, s)
    oc.set_fields(rho, I, f, v, s)
    done = 0
    for n in (1, 5, 30):
        gc.step(n - done)
        oc.step(n - done)
        done = n
        compare(gc, oc, f"printed random cycle {n}", tol=0.0)


def test_printed_placement_per_material_layered_bitwise():
    pb = printed(inputs.layered_impact(60, 12, 6, 15e3, 10, name="layered-pm"))
    pb = pb.replace(grid=dataclasses.replace(pb.grid, closure=1))
    g, o = run_pair(pb, [1, 60, 200], "printed layered pm")
    A, B = g.materials(), o.materials()
    for k in ("mu", "Im"):
        assert np.array_equal(A[k], B[k]), k


def test_printed_placement_stretched_grid_bitwise():
    pb = printed(inputs.stretched_impact(48, 8, 8, 5, 12e3, name="stretched"))
    run_pair(pb, [1, 50, 150], "printed stretched")


def test_ensemble_mixing_both_placements_bitwise():
    pbs = [inputs.impact(40 + 7 * k, 6 + k, 4 + k, 9e3 + 2e3 * k, nmat=2, strength=True, cycles=0,
                         name=f"mix{k}") for k in range(4)]
    pbs = [printed(pb) if k % 2 else pb for k, pb in enumerate(pbs)]
    c = ctx(pbs)
    os_ = [Oracle(pb) for pb in pbs]
    c.step(80)
    for o in os_:
        o.step(80)
    for k, o in enumerate(os_):
        compare(Member(c, k), o, f"mixed-placement member {k}", tol=0.0)


def test_printed_placement_mixed_precision_meets_the_bar():
    pb = printed(inputs.impact(61, 13, 6, 15e3, nmat=2, strength=True, cycles=0, name="strength-61"))
    g = ctx(pb.replace(precision="mixed"))
    o = Oracle(pb)
    g.step(100)
    o.step(100)
    e = conserved_errors(g.fields(), o.fields(), pb.grid)
    print("printed placement, mixed vs oracle at cycle 100:", e, flush=True)
    assert max(e.values()) < 1e-4, e
