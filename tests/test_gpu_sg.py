"""Shapiro-Giroux verification on the GPU: the four rows of the verification
section's table at 32^3, from z0 to z = 0 with adaptive theta = 0.51 steps,
against the analytic I-front solution (tests/sg_convergence.py)."""
import pytest

import sg_convergence as SG

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("row", [0, 1, 2, 3])
def test_shapiro_giroux_front(hip_device, row):
    out = SG.run_row(row, 32, dev=hip_device, log=print)
    assert len(out) >= 5 and out[-1][0] >= 5.0
    for A, r, ra, err, steps in out:
        assert abs(err) < 0.02, (A, r, ra, err)
