"""The per-call C ABI under HIP graph capture.

One closed-loop iteration through the plain calls (rollout, weights, update, shield,
plant step) is captured with torch's graph API and replayed, for the six-state and the
eight-state model.  The calls allocate nothing and synchronise nothing (their scratch is
reserved beforehand), so the graph holds only their kernels.  The replays, with eager
work and synchronisations between them, must equal the eager iterations bit for bit:
the same outputs, the same plant state, the same warm start and iteration counters.
"""
import numpy as np
import pytest
import torch

from paper_2302_11719_amd import core
from paper_2302_11719_amd import workloads as W

from gpu_helpers import ctx, params, say

pytestmark = pytest.mark.gpu
F32 = torch.float32
N_IT = 4


def _replays_match_eager(db, iteration, label):
    start = [db.x0.clone(), db.V.clone(), db.iter.clone()]

    def reset():
        for dst, src in zip((db.x0, db.V, db.iter), start):
            dst.copy_(src)

    def snapshot(outs):
        return [t.clone() for t in outs] + [db.x0.clone(), db.V.clone(), db.iter.clone()]

    ref = []
    for i in range(N_IT):
        ref.append(snapshot(iteration()))
        torch.cuda.synchronize()
    reset()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs = iteration()
    torch.cuda.synchronize()
    assert torch.equal(db.x0, start[0]) and torch.equal(db.iter, start[2])  # capture ran nothing
    rng = torch.Generator(device="cuda").manual_seed(7)
    for i in range(N_IT):
        say(f"{label} replay {i}")
        g.replay()
        torch.cuda.synchronize()
        # eager work of the program's own between the replays
        _ = (torch.rand(4096, device="cuda", generator=rng) * 2.0).cumsum(0)
        torch.cuda.synchronize()
        got = snapshot(outs)
        for k, (a, b) in enumerate(zip(got, ref[i])):
            assert torch.equal(a, b), (label, i, k)
    assert ctx().device_errors() == 0
    del g


def test_cartesian_closed_loop_graph_replays():
    M, C = params(F32)
    p = W.round_to_f32(W.config1(K=1024, T=30))
    db = core.DeviceBatch([p], dtype=F32)
    dist = torch.as_tensor(W.disturbances(3, 8).astype(np.float32).reshape(8, 1, 2), device="cuda")

    def iteration():
        S = core.rollout(ctx(), db, M, C, 9)
        w, stats = core.weights(ctx(), db, S, W.LAMBDA)
        Vp = core.update(ctx(), db, M, C, 9, w)
        Vs = core.shield_repair(ctx(), db, M, C, Vp, 10, 0.05, W.OBJ_SHIELD)
        core.execute(ctx(), db, M, Vs, Vp, dist=dist, n_dist=8)
        return S, w, stats, Vp, Vs

    _replays_match_eager(db, iteration, "cartesian")


def test_curvilinear_closed_loop_graph_replays():
    M, C = params(F32)
    WH = W.wheels_f32()
    base = W.config1(K=1024, T=30)
    kap, ds = W.curvature_table(base.track, 1024)
    ct = core.CurvTrackArrays([(kap, ds)], [base.track.half_width])
    p = W.Problem(1024, 30, base.track, W.start_state_c8(3.0), np.zeros((30, 2)), 0, 0)
    db = core.DeviceBatch([W.round_to_f32(p)], dtype=F32)

    def iteration():
        S = core.rollout_curvilinear(ctx(), db, ct, M, WH, C, 9)
        w, stats = core.weights(ctx(), db, S, W.LAMBDA)
        Vp = core.update(ctx(), db, M, C, 9, w)
        Vs = core.shield_repair_curvilinear(ctx(), db, ct, M, WH, C, Vp, 10, 0.05, W.OBJ_SHIELD)
        core.execute_curvilinear(ctx(), db, ct, M, WH, Vs, Vp)
        return S, w, stats, Vp, Vs

    _replays_match_eager(db, iteration, "curvilinear")
