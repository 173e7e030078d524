"""Pins of the oracle's TR curvature (Sec. II.B: a triangle fan of the PLIC
points of the 3x3x3 block, curvature by a variant of Taubin's estimate).

- Points on a sphere: every edge curvature 2 (d.n)/|d|^2 equals 1/R exactly,
  so K = 2/R whatever the fan and its weights.
- The 8-point ring on the quadric w = A u^2 + B v^2: the estimate tends to
  K = 2(A + B), twice the mean curvature at the apex, with an O(delta^2)
  error, which needs the fan order and the area weights to be right.
- Planes give 0; fewer than three points give 0; an open fan (all points in
  a half-plane) keeps only the triangles inside it.
- Invariance under rotations of the whole configuration (moves the points
  across the angle branch cut) and under permutations of the input order.
"""
import numpy as np
import pytest

import oracle as O


def _rot(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return q * np.sign(np.diag(r))


def _sphere_points(R, m, seed, spread=1.5):
    rng = np.random.default_rng(seed)
    n = np.array([0.0, 0.0, 1.0])  # inward normal at p = (0, 0, -R) + c
    pts = []
    for _ in range(m):
        ang = rng.uniform(0, 2 * np.pi)
        t = rng.uniform(0.3, spread) / R
        dirv = np.array([np.sin(t) * np.cos(ang), np.sin(t) * np.sin(ang), -np.cos(t)])
        pts.append(R * dirv - np.array([0, 0, -R]))
    return np.array(pts), n


@pytest.mark.parametrize("R", [4.0, 9.5, 30.0])
def test_points_on_a_sphere_give_two_over_R(R):
    d, n = _sphere_points(R, 12, seed=int(R))
    assert O.tr_curvature_points(d, n) == pytest.approx(2.0 / R, rel=1e-12)
    # a bubble: the normal points the other way
    assert O.tr_curvature_points(d, -n) == pytest.approx(-2.0 / R, rel=1e-12)


def _ring(A, B, delta):
    pts = []
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            if a == 0 and b == 0:
                continue
            u, v = a * delta, b * delta
            pts.append((u, v, A * u * u + B * v * v))
    return np.array(pts)


@pytest.mark.parametrize("A,B", [(0.3, 0.3), (0.5, -0.2), (0.1, 0.4)])
def test_quadric_ring_converges_to_twice_mean_curvature(A, B):
    n = np.array([0.0, 0.0, 1.0])
    errs = []
    for delta in (0.2, 0.1, 0.05):
        K = O.tr_curvature_points(_ring(A, B, delta), n)
        errs.append(abs(K - 2 * (A + B)))
    assert errs[2] < 1e-2 * abs(2 * (A + B)) + 1e-12
    # second order: halving delta divides the error by about 4
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.1)


def test_plane_and_degenerate_cases():
    n = np.array([0.0, 0.0, 1.0])
    assert O.tr_curvature_points(_ring(0.0, 0.0, 1.0), n) == 0.0
    assert O.tr_curvature_points(_ring(0.3, 0.1, 1.0)[:2], n) == 0.0
    # points on the normal line are left out
    pts = np.array([[0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0.1]])
    assert O.tr_curvature_points(pts, n) == 0.0


def test_open_fan_keeps_the_inner_triangles():
    R = 6.0
    d, n = _sphere_points(R, 40, seed=3)
    ang = np.arctan2(d[:, 1], d[:, 0])
    half = d[(ang > 0.2) & (ang < 2.6)]  # all within less than pi
    assert len(half) >= 3
    assert O.tr_curvature_points(half, n) == pytest.approx(2.0 / R, rel=1e-12)
    # with a cubic term the closed ring nearly cancels it, the open half not
    ring = _ring(0.5, -0.2, 0.3)
    ring[:, 2] += 0.3 * ring[:, 0] ** 3
    right = ring[ring[:, 0] >= 0]
    assert O.tr_curvature_points(right, n) != pytest.approx(O.tr_curvature_points(ring, n), rel=1e-3)


@pytest.mark.parametrize("seed", range(4))
def test_rotation_and_permutation_invariance(seed):
    rng = np.random.default_rng(100 + seed)
    n = np.array([0.0, 0.0, 1.0])
    uv = rng.uniform(-1.5, 1.5, size=(14, 2))
    w = 0.3 * uv[:, 0] ** 2 - 0.1 * uv[:, 1] ** 2 + 0.05 * uv[:, 0] * uv[:, 1] + 0.02 * uv[:, 0] ** 3
    d = np.column_stack([uv, w])
    K0 = O.tr_curvature_points(d, n)
    for r in range(3):
        Q = _rot(seed * 10 + r)
        assert O.tr_curvature_points(d @ Q.T, Q @ n) == pytest.approx(K0, rel=1e-10)
    perm = rng.permutation(len(d))
    assert O.tr_curvature_points(d[perm], n) == pytest.approx(K0, rel=1e-12)
