"""GPU parity where the FP32 obstacle barriers are evaluated per wave.

The FP32 kernels skip, for each transition, the obstacles whose DCBF term is
provably zero for every lane of a wave (a bound from the wave's bounding box and
largest step), and evaluate the others for the whole wave.  These tests put many
obstacles at distances on both sides of that bound, around and on the sampled
trajectories (inside and outside the track, some over the start), so that both
kinds occur in most steps, and compare every sample with the oracle: costs
(rollout kernel and fused plan, which must also agree bit for bit, since they run
the same arithmetic), and the adjoint.  Ragged K leaves partly filled waves,
whose spare lanes run a copy of the last sample.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2302_11719_amd import core
from paper_2302_11719_amd import workloads as W

from gpu_helpers import band_mask, ctx, params, prep, rel_err, say

pytestmark = pytest.mark.gpu
F32 = torch.float32
BAND = 1e-3


def _near_obstacles(track, seed, n=64, s_range=(0.3, 12.0), lat=2.5, margin=0.15):
    """n obstacles at arclength positions in s_range and lateral offsets in [-lat, lat]
    (beyond the half width too), radius U[0.1, 0.4]; rows (cx, cy, (r + margin)^2, r^2)."""
    rng = np.random.default_rng(900 + seed)
    poly = track.poly
    seg = np.hypot(poly[:, 2], poly[:, 3])
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    out = np.zeros((n, 4))
    for i in range(n):
        s = rng.uniform(*s_range)
        off = rng.uniform(-lat, lat)
        r = rng.uniform(0.1, 0.4)
        j = min(int(np.searchsorted(cum, s, side="right")) - 1, len(poly) - 1)
        f = (s - cum[j]) / seg[j]
        ax, ay, dx, dy = poly[j, :4]
        nx, ny = -dy / seg[j], dx / seg[j]
        out[i] = (ax + f * dx + off * nx, ay + f * dy + off * ny, (r + margin) ** 2, r * r)
    return out


def _problems():
    out = []
    for b, (K, T, seed) in enumerate([(1000, 40, 3), (130, 25, 4), (64, 60, 5)]):
        tr = W.spline_track(seed, 0.9)
        tr.obs = _near_obstacles(tr, seed)
        V = W.test_sequences(1, T, seed=70 + b, scale=0.6)[0]
        out.append(W.Problem(K=K, T=T, track=tr, x0=W.start_state(tr, vx=3.0 + b), V=V, pid=b, it=2 * b))
    return prep(out, F32)


def test_dense_obstacles_rollout_and_plan():
    probs = _problems()
    M, C = params(F32)
    db = core.DeviceBatch(probs, dtype=F32)
    say(f"dense obstacles K={[p.K for p in probs]}")
    S = core.rollout(ctx(), db, M, C, 21)
    plan = core.Plan(ctx(), db, M, C, 21, W.LAMBDA, use_graph=False, pipeline=-1)
    plan.launch()
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    Ss, Sp = db.per_problem(S), db.per_problem(plan.S)
    for b, p in enumerate(probs):
        assert np.array_equal(Ss[b], Sp[b]), b
        S_ref, _, margin = oracle.rollout(M, C, p.track, p.x0, p.V, p.K, 21, b, p.it, want_eps=False)
        ok = band_mask(margin, BAND, f"problem {b}", Ss[b], S_ref)
        assert rel_err(Ss[b], S_ref)[ok].max() <= 1e-4, b
        # the obstacles matter: without them most costs change
        tr0 = W.Track(**{**p.track.__dict__, "obs": np.zeros((0, 4))})
        S_free, _, _ = oracle.rollout(M, C, tr0, p.x0, p.V, p.K, 21, b, p.it, want_eps=False)
        frac = float(np.mean(np.abs(S_ref - S_free) > 1e-6 * np.maximum(np.abs(S_ref), 1.0)))
        say(f"  problem {b}: {frac:.2f} of the samples pay an obstacle term")
        assert frac > 0.2, (b, frac)


def test_dense_obstacles_adjoint():
    probs = _problems()
    M, C = params(F32)
    db = core.DeviceBatch(probs, dtype=F32)
    rng = np.random.default_rng(3)
    gs = []
    for p in probs:
        g = np.zeros(p.K)
        idx = np.unique(np.concatenate([np.linspace(0, p.K - 1, 10).astype(int), [p.K - 1]]))
        g[idx] = rng.uniform(0.5, 1.5, size=len(idx)).astype(np.float32)
        gs.append(g)
    say("dense obstacles adjoint")
    gS = torch.as_tensor(np.concatenate(gs), dtype=F32, device="cuda")
    gV = core.rollout_backward(ctx(), db, M, C, 21, gS, W.OBJ_TOTAL)
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    got = db.controls(gV)
    sig = np.array(C["sigma"])
    for b, p in enumerate(probs):
        ref = np.zeros((p.T, 2))
        for m in np.nonzero(gs[b])[0]:
            eps = oracle.normals(21, b, p.it, int(m), p.T) * sig
            ref += gs[b][m] * oracle.gradient_dual(M, C, p.track, p.x0, p.V, W.OBJ_TOTAL, eps)
        err = np.linalg.norm(got[b] - ref) / max(np.linalg.norm(ref), 1e-30)
        emax = np.abs(got[b] - ref).max() / max(np.abs(ref).max(), 1e-30)
        say(f"  problem {b}: rel err {err:.2e} (max {emax:.2e})")
        assert err <= 1e-3 and emax <= 1e-3, (b, err, emax)


def test_latency_mode_counts_hits_on_both_lanes_of_a_pair():
    """The latency-mode plan splits each sample's obstacles between a pair of lanes
    (even slots on one, odd slots on the other) and exchanges the collision flags
    between them.  With 64 obstacles that the sampled trajectories run into, some hits
    fall on odd slots only: the costs must match the tile-mode plan's on every sample (to
    the per-sample cost bar, 1e-4: the latency mode's RK4 rounds differently, and a missed
    indicator term would be of order 1e-1), and the oracle's on the samples that hit an
    odd-slot obstacle."""
    M, C = params(F32)
    c_obs = W.COST["C_obs"]

    def costs(p, pipeline):
        db = core.DeviceBatch([p], dtype=F32)
        pl = core.Plan(ctx(), db, M, C, 0, W.LAMBDA, use_graph=False, pipeline=pipeline)
        pl.launch()
        torch.cuda.synchronize()
        S = pl.S.cpu().numpy().astype(np.float64)
        pl.close()
        return S

    full = W.config4(K=4096, T=100, n_obs=64)
    even = W.config4(K=4096, T=100, n_obs=64)
    far = even.track.obs.copy()
    far[1::2, 0:2] = 1e4  # odd slots moved far away
    even.track.obs = far
    say("latency mode, obstacles on both lanes of a pair")
    pf = W.round_to_f32(full)
    S_tile, S_lat = costs(pf, -1), costs(pf, 1)
    S_even = costs(W.round_to_f32(even), -1)
    assert ctx().device_errors() == 0
    odd_hits = np.nonzero(S_tile - S_even >= 0.5 * c_obs)[0]
    say(f"  {len(odd_hits)} of 4096 samples cost at least half an indicator term more with the odd slots")
    assert len(odd_hits) > 0
    rel = np.abs(S_lat - S_tile) / np.maximum(np.abs(S_tile), 1.0)
    assert rel.max() <= 1e-4, (int((rel > 1e-4).sum()), rel.max())
    idx = odd_hits[:64]
    S_ref, _, margin = oracle.rollout(M, C, pf.track, pf.x0, pf.V, pf.K, 0, 0, pf.it, want_eps=False,
                                      n_threads=8, samples=idx)
    ok = band_mask(margin, BAND, "odd-slot hits", S_lat[idx], S_ref)
    assert rel_err(S_lat[idx], S_ref)[ok].max() <= 1e-4


@pytest.mark.parametrize("T", [1, 2, 3, 8])
def test_short_horizons_obstacles_per_step_pair(T):
    """The rollouts take the obstacle live set once per pair of steps (the box of
    both steps' end points, the larger step) and a last odd step on its own:
    horizons of one tail step, one pair, a pair and a tail, and four pairs, with
    obstacles packed from 0.9 to 3 m ahead (6 m/s: 0.3 m per step) so that their
    terms fall on either transition of a pair; rollout and fused plan bit for
    bit, and the oracle."""
    tr = W.spline_track(6, 0.9)
    tr.obs = _near_obstacles(tr, 6 + T, s_range=(0.9, 3.0), lat=1.2)
    V = W.test_sequences(1, T, seed=80 + T, scale=0.8)[0]
    p = prep([W.Problem(K=300, T=T, track=tr, x0=W.start_state(tr, vx=6.0), V=V, pid=0, it=T)], F32)[0]
    M, C = params(F32)
    db = core.DeviceBatch([p], dtype=F32)
    say(f"short horizon T={T}, K={p.K}, {len(tr.obs)} obstacles")
    S = core.rollout(ctx(), db, M, C, 23)
    plan = core.Plan(ctx(), db, M, C, 23, W.LAMBDA, use_graph=False, pipeline=-1)
    plan.launch()
    torch.cuda.synchronize()
    assert ctx().device_errors() == 0
    Sd, Sp = db.per_problem(S)[0], db.per_problem(plan.S)[0]
    assert np.array_equal(Sd, Sp)
    S_ref, _, margin = oracle.rollout(M, C, p.track, p.x0, p.V, p.K, 23, 0, p.it, want_eps=False)
    ok = band_mask(margin, BAND, f"T={T}", Sd, S_ref)
    assert rel_err(Sd, S_ref)[ok].max() <= 1e-4
    tr0 = W.Track(**{**p.track.__dict__, "obs": np.zeros((0, 4))})
    S_free, _, _ = oracle.rollout(M, C, tr0, p.x0, p.V, p.K, 23, 0, p.it, want_eps=False)
    frac = float(np.mean(np.abs(S_ref - S_free) > 1e-6 * np.maximum(np.abs(S_ref), 1.0)))
    say(f"  {frac:.2f} of the samples pay an obstacle term")
    assert frac > 0.05, frac
