"""GPU runs of the closed-loop collision sweep: determinism, the shield with no
iterations equals the DCBF-cost controller, rates in range."""
import pytest

from paper_2302_11719_amd import sweep
from paper_2302_11719_amd import workloads as W

from gpu_helpers import ctx, say

pytestmark = pytest.mark.gpu


def test_sweep_cells_deterministic_and_consistent():
    say("sweep: K=256 T=20, 8 runs x 15 steps, three controllers")
    a = sweep.run_cell(ctx(), 256, 20, "mppi", runs=8, steps=15, seed=3)
    b = sweep.run_cell(ctx(), 256, 20, "mppi", runs=8, steps=15, seed=3)
    assert a.collision_rate == b.collision_rate and a.collisions_per_run == b.collisions_per_run
    d = sweep.run_cell(ctx(), 256, 20, "mppi_dcbf", runs=8, steps=15, seed=3)
    s0 = sweep.run_cell(ctx(), 256, 20, "shield", runs=8, steps=15, seed=3,
                        repair=dict(n_steps=0, step=0.05, objective=W.OBJ_SHIELD))
    assert s0.collision_rate == d.collision_rate and s0.collisions_per_run == d.collisions_per_run
    s = sweep.run_cell(ctx(), 256, 20, "shield", runs=8, steps=15, seed=3)
    for c in (a, d, s):
        assert 0.0 <= c.collision_rate <= 1.0 and c.ms_per_step > 0.0
    assert ctx().device_errors() == 0
