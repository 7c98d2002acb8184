"""GPU parity of the curvilinear-model rollout (through smppi_rollout_curvilinear)
against the FP64 oracle, and a full MPPI iteration (weights and update unchanged)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2302_11719_amd import core
from paper_2302_11719_amd import workloads as W

from gpu_helpers import ctx, params, rel_err, say

pytestmark = pytest.mark.gpu
F32, F64 = torch.float32, torch.float64
BAND = 1e-3


def _problems(dtype):
    """Three problems: spline tables of 1024 and 512 points, a circle (constant
    curvature); uneven K and T; start states off the centre line."""
    specs = [(W.spline_track(0), 1024, 4096 if dtype == F32 else 256, 50, (0.0, 0.1, 0.05, 3.0, 0.0, 0.0)),
             (W.spline_track(1), 512, 300, 23, (12.0, -0.2, -0.1, 4.0, 0.1, 0.0)),
             (W.circle_track(10.0, 1.0), 256, 65, 7, (1.0, 0.0, 0.0, 2.5, 0.0, 0.1))]
    probs, tables, widths = [], [], []
    for b, (tr, n, K, T, x0) in enumerate(specs):
        kap, ds = W.curvature_table(tr, n)
        if dtype == F32:
            kap, ds = kap.astype(np.float32).astype(np.float64), float(np.float32(ds))
        V = W.test_sequences(1, T, seed=40 + b, scale=0.4)[0]
        x = np.asarray(x0, dtype=np.float64)
        if dtype == F32:
            V, x = V.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64)
        probs.append(W.Problem(K, T, W.circle_track(10.0, 1.0), x, V, b, 2))
        tables.append((kap, ds))
        widths.append(tr.half_width)
    return probs, tables, widths


@pytest.mark.parametrize("dtype", [F32, F64])
def test_curvilinear_rollout_vs_oracle(dtype):
    probs, tables, widths = _problems(dtype)
    M, C = params(dtype)
    db = core.DeviceBatch(probs, dtype=dtype)
    ct = core.CurvTrackArrays(tables, widths, dtype=dtype)
    say(f"curvilinear rollout {dtype}")
    S, eps = core.rollout_curvilinear(ctx(), db, ct, M, C, 6, want_eps=True)
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    Ss = db.per_problem(S)
    k0 = 0
    for b, p in enumerate(probs):
        kap, ds = tables[b]
        Sr, er, mg = oracle.rollout_curv(M, C, kap, ds, widths[b], p.x0, p.V, p.K, 6, p.pid, p.it)
        ok = mg > (BAND if dtype == F32 else 0.0)
        assert ok.mean() > 0.9
        e = rel_err(Ss[b], Sr)
        assert e[ok].max() <= (1e-4 if dtype == F32 else 1e-10), (b, e[ok].max())
        ed = eps[k0:k0 + p.K, :p.T].cpu().numpy().astype(np.float64)
        assert np.abs(ed - er).max() <= (2e-6 if dtype == F32 else 1e-12)
        k0 += p.K


def test_curvilinear_mppi_iteration_fp64():
    """Weights and update of the curvilinear costs (calls shared with the Cartesian model)."""
    probs, tables, widths = _problems(F64)
    M, C = params(F64)
    db = core.DeviceBatch(probs, dtype=F64)
    ct = core.CurvTrackArrays(tables, widths, dtype=F64)
    say("curvilinear MPPI iteration fp64")
    S = core.rollout_curvilinear(ctx(), db, ct, M, C, 8)
    w, stats = core.weights(ctx(), db, S, W.LAMBDA)
    Vp = core.update(ctx(), db, M, C, 8, w)
    torch.cuda.synchronize()
    Vps = db.controls(Vp)
    for b, p in enumerate(probs):
        kap, ds = tables[b]
        Sr, er, _ = oracle.rollout_curv(M, C, kap, ds, widths[b], p.x0, p.V, p.K, 8, p.pid, p.it)
        wr, _ = oracle.weights(Sr, W.LAMBDA)
        assert np.abs(Vps[b] - oracle.update(p.V, wr, er)).max() <= 1e-9
