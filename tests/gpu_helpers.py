"""Shared helpers of the GPU parity tests (device runs through the C ABI, oracle on the CPU)."""
import os

import numpy as np
import torch

import oracle
from paper_2302_11719_amd import core
from paper_2302_11719_amd import workloads as W

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = core.Context(0)
    return _CTX


def say(msg):
    print(msg, flush=True)


# (test, what, samples near a switch, of them off by indicator flips, samples) of every
# FP32 cost comparison; the conftest prints them in the terminal summary, also under -q.
EXCLUSIONS = []


def band_mask(margin, band, what="", S_dev=None, S_ref=None, tol=1e-4, c_obs=None):
    """Samples whose costs must match the oracle to `tol`: those whose trajectory stays
    farther than `band` from every collision-indicator switch.  The indicator is
    discontinuous, so FP32 rounding may flip it inside the band; given the costs, the
    other samples are checked too: they must differ from the oracle by a whole number
    of indicator terms (C_obs each), to `tol`.  Records the counts."""
    margin = np.asarray(margin)
    ok = margin > band
    n_ex = int((~ok).sum())
    flips = 0
    if S_dev is not None and n_ex:
        c = float(W.COST["C_obs"] if c_obs is None else c_obs)
        sd = np.asarray(S_dev, np.float64)[~ok]
        sr = np.asarray(S_ref, np.float64)[~ok]
        k = np.rint((sd - sr) / c)
        resid = np.abs(sd - sr - k * c) / np.maximum(np.abs(sr), 1.0)
        assert resid.max() <= tol, (what, "near-switch residual", resid.max())
        flips = int((k != 0).sum())
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    EXCLUSIONS.append((test, what, n_ex, flips, int(margin.size)))
    say(f"  near an indicator switch: {n_ex} of {margin.size} {what} ({flips} off by whole indicator terms)")
    return ok


def params(dtype):
    if dtype == torch.float32:
        return W.params_f32(W.MODEL, W.COST)
    return W.MODEL, W.COST


def prep(problems, dtype):
    """Round inputs to FP32 for FP32 runs so both sides see identical data."""
    if dtype == torch.float32:
        return [W.round_to_f32(p) for p in problems]
    return list(problems)


def rel_err(a, ref, floor=1.0):
    return np.abs(np.asarray(a, np.float64) - ref) / np.maximum(np.abs(ref), floor)


def oracle_iteration(p, M, C, seed, lam, pid=None, nominal=False):
    return oracle.mppi_iteration(M, C, p.track, p.x0, p.V, p.K, seed, p.pid if pid is None else pid, p.it, lam,
                                 nominal=nominal)


def device_iteration(problems, dtype, seed, lam, nominal=False, want_eps=False):
    M, C = params(dtype)
    db = core.DeviceBatch(problems, dtype=dtype)
    c = ctx()
    out = {}
    if want_eps:
        S, eps = core.rollout(c, db, M, C, seed, nominal, want_eps=True)
        out["eps"] = eps
    else:
        S = core.rollout(c, db, M, C, seed, nominal)
    w, stats = core.weights(c, db, S, lam)
    Vp = core.update(c, db, M, C, seed, w, nominal)
    torch.cuda.synchronize()
    assert c.device_errors() == 0
    out.update(db=db, S=S, w=w, stats=stats, V_plus=Vp)
    return out


def ragged_problems(n_obs=8):
    """Mixed batch: circle and spline tracks, obstacles, K with several tiles and a
    ragged tail (and K = 1), horizons from 1 to 37."""
    specs = [(300, 21, "spline", 0), (1, 5, "circle", 0), (65, 37, "spline", n_obs), (257, 1, "circle", 0),
             (513, 8, "spline", 0)]
    out = []
    for b, (K, T, kind, no) in enumerate(specs):
        if kind == "circle":
            tr = W.circle_track(10.0, 1.0)
        else:
            tr = W.spline_track(b, 0.9)
            if no:
                tr.obs = W.obstacles(tr, b, no)
        x0 = W.start_state(tr, vx=2.0 + 0.5 * b)
        V = W.test_sequences(1, T, seed=b, scale=0.4)[0]
        out.append(W.Problem(K=K, T=T, track=tr, x0=x0, V=V, pid=b, it=b + 1))
    return out
