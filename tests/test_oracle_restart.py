"""The state of the scheme between two cycles is complete in what the oracle
hands over: the staggered fields (Sec. 2), each material's partial density
and energy under the per-material closure, the auxiliary fields of Sec. 3's
PML with its reference density and sink, and the clock (the time, and the
step of the next cycle that Sec. 7's Courant condition chose at the end of
the cycle before). A run continued from them in a fresh oracle must repeat the
uninterrupted run bit for bit. A hand-over that drops the PML memory or the
reference density changes the continued fields, and one that drops the clock
restarts the time at zero (its fields agree while the Courant limit, not the
growth cap, sets the step, since the step is recomputed from the same state),
which the second test checks, so the pin has teeth.
"""
import dataclasses

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2403_04267_amd import inputs


def _pm(pb):
    return pb.replace(grid=dataclasses.replace(pb.grid, closure=1))


def _damped(pb):
    return pb.replace(pml=dataclasses.replace(pb.pml, damp_stress=1))


CASES = {
    "impact-strength": lambda: inputs.impact(24, 6, 3, 12e3, 2, True, 0, name="impact"),
    "layered-damped": lambda: _damped(inputs.layered_impact(24, 6, 3, 14e3, 5, name="layered")),
    "three-layer-pm": lambda: _pm(inputs.three_layer_impact(26, 6, 3, 14e3, 3, 5, name="three-pm")),
    "stretched": lambda: inputs.stretched_impact(18, 4, 5, 3, 12e3, name="stretched"),
}

N_HAND, N_MORE = 61, 25


def state(o):
    out = dict(o.fields())
    if o.problem.grid.closure:
        out.update({"M." + k: v for k, v in o.materials().items()})
    out.update({"pml." + k: v for k, v in o.pml_aux().items()})
    d = o.diag()
    out.update({"diag." + k: np.array(d[k]) for k in ("t", "dt", "mass", "ie", "ke", "mass_pml")})
    return out


@pytest.mark.parametrize("case", list(CASES))
def test_continued_oracle_run_repeats_the_uninterrupted_one(case):
    pb = CASES[case]()
    a = Oracle(pb)
    a.step(N_HAND)
    assert max(float(np.abs(v).max()) for k, v in a.pml_aux().items() if k.startswith(("phi", "psi"))) > 0
    b = Oracle(pb)
    b.step(5)
    b.continue_from(a)
    a.step(N_MORE)
    b.step(N_MORE)
    Sa, Sb = state(a), state(b)
    bad = [k for k in Sa if not np.array_equal(Sa[k], Sb[k])]
    assert not bad, bad
    assert int(b.diag()["cycle"]) == N_MORE


def test_a_partial_hand_over_does_not_repeat_the_run():
    pb = CASES["impact-strength"]()
    a = Oracle(pb)
    a.step(N_HAND)
    F, A, d = a.fields(eos=False), a.pml_aux(), a.diag()
    a.step(N_MORE)
    ref = dict(a.fields(eos=False))
    t_ref = a.diag()["t"]

    def continued(with_pml=True, with_rref=True, with_clock=True):
        b = Oracle(pb)
        b.set_fields(F["rho"], F["I"], F["f"], F["v"], F["s"])
        if with_pml:
            aux = dict(A)
            if not with_rref:
                aux.pop("rho_ref")
                aux["rho_ref"] = b.pml_aux()["rho_ref"]  # the run start's own reference
            b.set_pml(aux)
        if with_clock:
            b.set_clock(d["t"], d["dt"])
        b.step(N_MORE)
        out = dict(b.fields(eos=False))
        out["t"] = np.array(b.diag()["t"])
        return out

    ref["t"] = np.array(t_ref)
    full = continued()
    assert all(np.array_equal(full[k], ref[k]) for k in ref)
    for kw in ({"with_pml": False}, {"with_rref": False}):
        part = continued(**kw)
        assert not all(np.array_equal(part[k], ref[k]) for k in ref if k != "t"), kw
    part = continued(with_clock=False)
    assert part["t"] != ref["t"]


def test_clock_arguments_are_checked():
    pb = CASES["impact-strength"]()
    o = Oracle(pb)
    o.step(3)
    d = o.diag()
    for t, dt in ((d["t"], 0.0), (d["t"], -1.0), (-1.0, d["dt"]), (d["t"], float("nan")),
                  (float("inf"), d["dt"]), (d["t"], 2 * pb.grid.dt_max)):
        with pytest.raises(ValueError):
            o.set_clock(t, dt)
    assert o.diag()["t"] == d["t"] and o.diag()["dt"] == d["dt"]
