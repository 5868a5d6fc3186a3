"""Host-side checks of the benchmark's contract (no GPU needed): more than
one GPU is refused with a message, the algorithmic bytes per cell-update of
the headline workload follow from the state it reads and writes, and the
recorded counters are used only for the kernel sources and schedule they
were taken with."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2403_04267_amd import inputs  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_algorithmic_bytes_of_the_headline_workload():
    pb = inputs.config_scale()
    g = pb.grid
    # state read and written once: rho, I, f0, f1 (8 B) and s_rr, s_zz, s_rz, v_r, v_z (8 B)
    state = 2 * (8 * 4 + 8 * 5)
    # PML: 7 values per strip cell per damped direction read + written, the
    # reference density read and the sink read + written per layer cell
    bottom, right = g.pml_b * g.NR, g.pml_r * g.NZ
    union = bottom + g.n_z * g.pml_r
    aux = (2 * 8 * 7 * (bottom + right) + 8 * 3 * union) / (g.NR * g.NZ)
    assert bench.algorithmic_bytes_per_cell(pb) == pytest.approx(state + aux, rel=1e-15)
    assert 150.0 < state + aux < 160.0
    mixed = bench.algorithmic_bytes_per_cell(pb.replace(precision="mixed"))
    assert mixed == pytest.approx(state + aux - 2 * 4 * 5, rel=1e-15)  # FP32 stress and velocity


def test_counters_apply_only_to_their_sources_and_schedule(monkeypatch):
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    sched = dict(rec["records"][0]["schedule"])
    if rec["records"][0]["kernel_sources_sha256"] == bench.kernel_sources_sha():
        assert bench.traffic_per_launch(sched) == rec["records"][0]["hbm_bytes_per_launch"]
    other = dict(sched, grid=sched["grid"] + 8)
    assert bench.traffic_per_launch(other) is None or any(
        r["schedule"] == other for r in rec["records"])
    valu = rec.get("valu")
    for v in ([valu] if isinstance(valu, dict) else valu or []):
        if v["kernel_sources_sha256"] == bench.kernel_sources_sha():
            assert bench.valu_per_launch(dict(v["schedule"])) == v["sq_insts_valu_per_dispatch"]
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda: "0" * 64)
    assert bench.traffic_per_launch(sched) is None
    assert bench.valu_per_launch(sched) is None
