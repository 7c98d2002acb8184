"""GPU parity at projection-window half widths other than the default 4: the shield's
lane-row window (half width <= 7) and its sequential rule (wider), the rollouts' general
window search, in the plain kernels and in both plan modes, against the oracle (the rule
of reading R25 at any half width)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2302_11719_amd import core
from paper_2302_11719_amd import workloads as W

from gpu_helpers import band_mask, ctx, oracle_iteration, params, prep, rel_err, say

pytestmark = pytest.mark.gpu
F32 = torch.float32


def _problems(window):
    """Three spline problems starting 0.5 m off the centre line, heading 0.5 rad towards
    the edge at 5 m/s (so the shield has violations to repair)."""
    probs = []
    for b in range(3):
        tr = W.spline_track(10 + b)
        tr.window = window
        T = 20 + 7 * b
        x0 = W.start_state(tr, vx=5.0)
        dx, dy = tr.poly[0, 2], tr.poly[0, 3]
        n = float(np.hypot(dx, dy))
        x0[0] += 0.5 * (-dy / n)
        x0[1] += 0.5 * (dx / n)
        x0[2] += 0.5
        probs.append(W.Problem(200 + 37 * b, T, tr, x0, W.test_sequences(1, T, seed=40 + b, scale=0.3)[0], b,
                               b + 1))
    return prep(probs, F32)


@pytest.mark.parametrize("window", [2, 7, 9])
def test_window_widths_rollout_plans_and_shield(window):
    probs = _problems(window)
    M, C = params(F32)
    db = core.DeviceBatch(probs, dtype=F32)
    say(f"window {window}: rollout")
    S = core.rollout(ctx(), db, M, C, 6)
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    Ss = db.per_problem(S)
    for b, p in enumerate(probs):
        r = oracle_iteration(p, M, C, 6, W.LAMBDA)
        ok = band_mask(r["margin"], 1e-3, f"window {window}, problem {b}", Ss[b], r["S"])
        assert rel_err(Ss[b], r["S"])[ok].max() <= 1e-4, b
    # plans in both modes (latency mode: the general window on every lane) give the
    # plain rollout's costs
    for pipeline in (1, -1):
        say(f"window {window}: plan pipeline={pipeline}")
        pl = core.Plan(ctx(), db, M, C, 6, W.LAMBDA, use_graph=False, pipeline=pipeline,
                       block=0 if pipeline == 1 else 256)
        pl.launch()
        torch.cuda.synchronize()
        assert ctx().device_errors() == 0
        err = float(rel_err(pl.S.cpu().numpy(), S.cpu().numpy().astype(np.float64)).max())
        assert err <= 1e-5, (pipeline, err)
        pl.close()
    # Algorithm 1 from sequences whose nominal trajectories violate the DCBF condition
    say(f"window {window}: shield")
    viol = [oracle.objective(M, C, p.track, p.x0, p.V, W.OBJ_SHIELD)[0] for p in probs]
    assert max(viol) > 0.0, viol
    Vs = core.shield_repair(ctx(), db, M, C, db.V, 10, 0.05, W.OBJ_SHIELD)
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    got = db.controls(Vs)
    for b, p in enumerate(probs):
        ref = oracle.repair(M, C, p.track, p.x0, p.V, 10, 0.05, W.OBJ_SHIELD)
        assert np.abs(got[b] - ref).max() <= 1e-3 * max(np.linalg.norm(p.V), 1.0), b
    # the shield inside the latency-mode launch equals the shield kernel, bit for bit
    rep = dict(n_steps=10, step=0.05, objective=W.OBJ_SHIELD)
    pl = core.Plan(ctx(), db, M, C, 6, W.LAMBDA, repair=rep, use_graph=False, pipeline=1, fuse_shield=1)
    pl.launch()
    torch.cuda.synchronize()
    sep = core.shield_repair(ctx(), db, M, C, pl.V_plus, 10, 0.05, W.OBJ_SHIELD)
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    assert torch.equal(pl.V_safe, sep)
    pl.close()
