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
