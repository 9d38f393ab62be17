"""Pins of the exploration-support oracle (oracle/rrg_oracle.c) to facts outside it:
the published Philox4x32-10 known-answer vectors, an independent grid-based
neighbour search (the seeded input generator), hand-made geometric cases on the
closed obstacle sets, and closed forms of the heuristic."""
import numpy as np
import pytest

import workloads as W
from oracle import rrg as R


# Known-answer vectors published with the Random123 library (Salmon et al., SC'11):
# (counter, key) -> output of philox4x32 with 10 rounds.
PHILOX_KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", PHILOX_KAT)
def test_philox_known_answers(ctr, key, want):
    assert tuple(int(x) for x in R.philox(ctr, key)) == want


def test_candidate_is_philox_words():
    # coordinate i of candidate k is (w_i >> 8) * 2^-24 with the documented counter
    seed, stream, k = 0x0123456789ABCDEF, 7, (5 << 32) + 11
    x = R.candidate(6, seed, stream, k)
    w0 = R.philox((k & 0xFFFFFFFF, k >> 32, stream, 0), (seed & 0xFFFFFFFF, seed >> 32))
    w1 = R.philox((k & 0xFFFFFFFF, k >> 32, stream, 1), (seed & 0xFFFFFFFF, seed >> 32))
    w = np.concatenate([w0, w1])
    assert np.array_equal(x, (w[:6] >> 8).astype(np.float64) * 2.0 ** -24)


def test_sampling_continues_and_rejects():
    obs = W.make_obstacles(3, 10, "mixed", 3)
    a, c1 = R.sample(3, 99, 2, 0, 500, obs)
    b, c2 = R.sample(3, 99, 2, c1, 700, obs)
    ab, c3 = R.sample(3, 99, 2, 0, 1200, obs)
    assert c2 == c3 and np.array_equal(np.concatenate([a, b]), ab)
    assert not obs.blocked(ab).any()
    # the rejected candidates between 0 and c3 are exactly the blocked ones
    cands = np.array([R.candidate(3, 99, 2, k) for k in range(c3)])
    assert np.array_equal(cands[~obs.blocked(cands)], ab)
    assert abs(ab.mean() - 0.5) < 0.05


def scene(d, count, kinds, seed):
    return W.make_obstacles(d, count, kinds, seed)


@pytest.mark.parametrize("d,count,kinds,n", [(2, 8, "box", 1500), (3, 12, "mixed", 1200), (4, 20, "sphere", 1000),
                                             (6, 40, "sphere", 1500), (8, 15, "mixed", 800)])
def test_rows_match_grid_search(d, count, kinds, n):
    """Brute force against the generator's grid search (independent code)."""
    obs = scene(d, count, kinds, 11 * d)
    pts, _ = R.sample(d, 5 + d, 0, 0, n, obs)
    pts = np.concatenate([np.full((1, d), 0.05), np.full((1, d), 0.95), pts])
    r = W.radius(len(pts), d)
    rp, col, cost = R.build_rows(pts, 0, r, obs)
    ref = W.build_rows(pts, 0, len(pts), r, obs, nthreads=2)
    assert np.array_equal(rp, ref.row_ptr)
    assert np.array_equal(col, ref.col)
    assert np.array_equal(cost.view(np.uint32), ref.cost.view(np.uint32))
    assert len(col) > 2 * len(pts)
    # a second batch (n_old > 0) gives the tail of the same rows
    k = len(pts) // 3
    rp2, col2, cost2 = R.build_rows(pts, len(pts) - k, r, obs)
    assert np.array_equal(rp2, rp[-k - 1:] - rp[-k - 1])
    assert np.array_equal(col2, col[rp[-k - 1]:])


class Obs:
    def __init__(self, d, kind, centre, size):
        self.d = d
        self.kind = np.array(kind, np.int32)
        self.centre = np.array(centre, np.float64).reshape(len(kind), d)
        self.size = np.array(size, np.float64).reshape(len(kind), d)


def test_closed_sphere_and_box_cases():
    sph = Obs(2, [0], [[0.5, 0.5]], [[0.25, 0.0]])
    # tangent segment: closest approach exactly R (binary fractions, exact) -> blocked
    assert R.segment_blocked([0.0, 0.75], [1.0, 0.75], sph)
    assert not R.segment_blocked([0.0, 0.75 + 2.0 ** -20], [1.0, 0.75 + 2.0 ** -20], sph)
    # the closest point is an endpoint (t clamped): a segment ending short of the sphere
    assert not R.segment_blocked([0.0, 0.5], [0.25 - 2.0 ** -20, 0.5], sph)
    assert R.segment_blocked([0.0, 0.5], [0.25, 0.5], sph)
    assert R.point_blocked([0.75, 0.5], sph) and not R.point_blocked([0.75 + 2.0 ** -30, 0.5], sph)
    box = Obs(3, [1], [[0.5, 0.5, 0.5]], [[0.125, 0.25, 0.0625]])
    # along a face (closed): blocked; just outside: free
    assert R.segment_blocked([0.0, 0.75, 0.5], [1.0, 0.75, 0.5], box)
    assert not R.segment_blocked([0.0, 0.75 + 2.0 ** -20, 0.5], [1.0, 0.75 + 2.0 ** -20, 0.5], box)
    # diagonal through the corner (0.625, 0.75, 0.5625) only
    corner = np.array([0.625, 0.75, 0.5625])
    assert R.segment_blocked(corner + 0.25, corner, box)
    assert not R.segment_blocked(corner + 0.25, corner + 2.0 ** -20, box)
    assert not R.segment_blocked(np.array([0.7, 0.9, 0.6]), np.array([0.9, 0.7, 0.6]), box)
    assert R.point_blocked([0.375, 0.25, 0.4375], box) and not R.point_blocked([0.375, 0.25, 0.4375 - 2.0 ** -30], box)


def test_rows_free_space_complete_graph():
    """No obstacles and r >= sqrt(d): every pair is an edge, cost = length."""
    d = 3
    pts, _ = R.sample(d, 1, 0, 0, 60, None)
    rp, col, cost = R.build_rows(pts, 0, 2.0, None)
    assert np.array_equal(np.diff(rp), np.arange(60))
    v = np.repeat(np.arange(60), np.arange(60))
    exact = np.sqrt(((pts[col] - pts[v]) ** 2).sum(axis=1))
    assert np.max(np.abs(cost.astype(np.float64) - exact) / exact) < 2.0 ** -23


def test_heuristic_closed_forms():
    pts = np.array([[0.95, 0.95], [0.95, 0.45], [0.65, 0.55], [0.05, 0.05]])
    h = R.heuristic(pts, pts[0])
    assert h[0] == 0.0
    assert h[1] == np.float32(0.5)
    assert h[2] == np.float32(0.5)  # 3-4-5 triangle: (0.3, 0.4)
    assert abs(float(h[3]) - 0.9 * np.sqrt(2)) < 1e-6
