"""The 1050 x 1050 strength impact (1000 x 1000 cells + 50-cell PML, two
materials, Y0 = 10 MPa, friction 0.8, Ylim = 2.5 GPa, R = 50 cells, 15 km/s)
for its whole 5000 cycles against the FP64 oracle at full resolution, in the
launch configuration the benchmark times (the schedule the tuner picks for
this problem, applied to a fresh context).

Every field, every PML auxiliary, t, dt, the cycle count and the
diagnostics equal the oracle's bit for bit at cycles 10, 1000 and 5000
(5.5e9 cell-updates; the oracle takes about 90 s on 16 host cores).
"""
import pytest

from oracle.oracle import Oracle
from paper_2403_04267_amd import inputs

from .test_gpu_parity import compare

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(1800)
def test_scale_workload_whole_run_equals_the_oracle():
    from paper_2403_04267_amd.salec import Salec
    pb = inputs.config_scale()
    t = Salec(pb)
    s = t.tune(2)
    del t
    g = Salec(pb)
    g.set_schedule(s["variant"], s["grid"])
    o = Oracle(pb)
    print(f"[1050^2] schedule {s['tile_r']}x{s['tile_z']}/{s['threads']} grid {s['grid']}", flush=True)
    done = 0
    for c in (10, 1000, 5000):
        g.step(c - done)
        while done < c:
            n = min(500, c - done)
            o.step(n)
            done += n
            print(f"[1050^2] oracle at cycle {done}", flush=True)
        compare(g, o, f"1050^2 cycle {c}", tol=0.0)
