"""GPU run of the PML payoff study (what the layer buys, Sec. 4) at a small
size: the same impact on a domain with a PML, on the same domain with plain
walls and on a 6x larger domain, to the same stop time after the first
reflections from the small domain's walls have crossed the crater region.
The layer must bring the interior within a fraction of the plain-wall
error against the large domain, at a fraction of the large domain's cells."""
import pytest

pytestmark = pytest.mark.gpu


def test_pml_brings_the_interior_close_to_the_large_domain():
    from paper_2403_04267_amd.pml_study import Setup, run
    r = run(Setup(n=60, p=12, radius=6, v_imp=10e3, t_end=0.04, big=6))
    for k in ("pml", "bare", "big"):
        print(k, {q: r[k][q] for q in ("cells", "cycles", "t", "device_ms", "crater_depth", "crater_radius")},
              r[k].get("err_vs_big"), flush=True)
    for k in ("pml", "bare", "big"):
        assert r[k]["t"] == pytest.approx(0.04, rel=1e-9)
    e_pml, e_bare = r["pml"]["err_vs_big"], r["bare"]["err_vs_big"]
    assert e_bare["reflected_energy"] > 1e-3  # the plain walls' reflections have reached the window
    assert e_pml["reflected_energy"] < 0.1 * e_bare["reflected_energy"], (e_pml, e_bare)
    for q in ("rho", "momentum"):
        assert e_pml[q] < 0.5 * e_bare[q], (q, e_pml, e_bare)
    assert abs(r["pml"]["crater_depth"] - r["big"]["crater_depth"]) <= 1.0
    assert r["pml"]["cells"] < 0.1 * r["big"]["cells"]


def test_pml_in_the_paper_setting():
    """Sec. 4's setting on Table 2's grid (two layers, gravity) at 20 s, when
    the shock has reached the bottom boundary: against a reference whose
    extension zones reach ~200 km further, the PML run's target is within a
    fraction of a percent while plain walls send back measurable energy."""
    from paper_2403_04267_amd.pml_study import PaperSetup, paper_run
    r = paper_run(PaperSetup(t_end=20.0))
    for k in ("pml", "bare", "ref"):
        print(k, r[k], flush=True)
        assert r[k]["t"] == pytest.approx(20.0, rel=1e-9)
    e_pml, e_bare = r["pml"]["err_vs_ref"], r["bare"]["err_vs_ref"]
    assert e_bare["reflected_energy"] > 1e-3
    assert e_pml["reflected_energy"] < 1e-2 * e_bare["reflected_energy"], (e_pml, e_bare)
    assert e_pml["dp"] < 0.2 * e_bare["dp"], (e_pml, e_bare)
    assert r["pml"]["cells"] < 0.65 * r["ref"]["cells"]
