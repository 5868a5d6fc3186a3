"""salec_diag_totals, the entry point that allocates nothing (its partial
sums live in the library's per-GPU scratch array), through the C ABI: two
calls in a row, the second on a smaller member, each equal to salec_diag's
totals bit for bit; the values beyond the six totals are left alone."""
import numpy as np
import pytest

from paper_2403_04267_amd import inputs

pytestmark = pytest.mark.gpu

NAMES = ("mass", "ie", "ke", "mass_out", "mass_pml", "ie_out")


def test_diag_totals_equal_salec_diag_on_two_calls_in_a_row():
    import torch
    from paper_2403_04267_amd.salec import Salec
    pbs = [inputs.impact(100, 20, 10, 10e3, nmat=1, strength=False, cycles=0, name="larger"),
           inputs.impact(40, 8, 4, 8e3, nmat=2, strength=True, cycles=0, name="smaller")]
    c = Salec(pbs)
    c.step(37)
    out = torch.full((2, 8), -1.0, dtype=torch.float64, device="cuda")
    print("salec_diag_totals on member 0 (140 x 140), then member 1 (48 x 48)", flush=True)
    c.diag_totals(out[0], k=0)
    c.diag_totals(out[1], k=1)  # the second call, on the smaller member
    c.stream.synchronize()
    tot = out.cpu().numpy()
    for k in (0, 1):
        d = c.diag(k=k)
        want = np.array([d[n] for n in NAMES])
        assert np.array_equal(tot[k, :6], want), (k, tot[k, :6], want)
        assert np.all(tot[k, 6:] == -1.0)
    assert tot[0, 0] > tot[1, 0] > 0.0
    # again after more cycles: the shared scratch holds the last call's
    # partials, which every call overwrites
    c.step(5)
    c.diag_totals(out[1], k=1)
    c.stream.synchronize()
    d = c.diag(k=1)
    assert np.array_equal(out[1, :6].cpu().numpy(), np.array([d[n] for n in NAMES]))
