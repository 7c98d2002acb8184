"""Host side of the collision sweep: the boundary and obstacle checks against the
oracle's lateral offset (global search) and closed forms."""
import numpy as np

import oracle
from paper_2302_11719_amd import sweep
from paper_2302_11719_amd import workloads as W


def test_segment_distance_matches_oracle_global_search():
    tr = W.spline_track(3)
    rng = np.random.default_rng(1)
    P = tr.poly[rng.integers(0, len(tr.poly), 200), :2] + rng.normal(scale=1.5, size=(200, 2))
    got = sweep.segment_distance_sq(tr.poly, P)
    ref = np.array([oracle.lateral_sq(tr, x, y, -1)[0] for x, y in P])
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_collision_checks_closed_forms():
    c = W.circle_track(10.0, 1.0)
    pts = np.array([[10.5, 0.0], [11.2, 0.0], [0.0, -8.9], [0.0, -9.1]])
    assert sweep.collided(c, pts).tolist() == [False, True, True, False]
    tr = W.spline_track(0)
    tr.obs = np.array([[tr.poly[10, 0], tr.poly[10, 1], 0.5 ** 2, 0.3 ** 2]])
    p = np.array([[tr.poly[10, 0] + 0.29, tr.poly[10, 1]], [tr.poly[10, 0] + 0.31, tr.poly[10, 1]]])
    assert sweep.collided(tr, p).tolist() == [True, False]


def test_batch_check_equals_per_track_check():
    tracks = [W.spline_track(s) for s in range(6)]
    rng = np.random.default_rng(2)
    P = np.stack([t.poly[5, :2] for t in tracks]) + rng.normal(scale=1.0, size=(6, 2))
    per = np.array([sweep.collided(t, P[i:i + 1])[0] for i, t in enumerate(tracks)])
    assert np.array_equal(sweep.batch_collided(tracks, P), per)
