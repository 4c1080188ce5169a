"""Pins of the oracle's primitives against mathematics it does not share.

* point-box distance: closed forms and numpy's clip (the closest point of a
  box is the clipped point);
* segment-box minimum: closed forms, a golden-section search on the convex
  distance function, and dense sampling;
* motion and forward kinematics: scipy's rotations and Slerp, plain rotation
  matrices, and the planar chain written with cumulative sums;
* the chord-deviation bound delta (Sec. 3.2's swept volume, outer
  approximation as a superset): dense sampling of the true centre path, and
  its tightness for small rotations.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation, Slerp

from paper_2603_28674_amd import synth
from refgeom import fk_arm_ref, fk_se2_ref, fk_se3_ref, centre_path


# --------------------------------------------------------------------------
# point-box
# --------------------------------------------------------------------------

def box(lo, hi):
    b = np.zeros(6)
    b[:len(lo)] = lo
    b[3:3 + len(hi)] = hi
    return b


def test_point_box_closed_forms(oracle_lib):
    O = oracle_lib
    # centre (0,0), box [1,2]x[-1,1]: distance 1 exactly (touching at r = 1)
    assert O.point_box_d2([0.0, 0.0], box([1, -1], [2, 1])) == 1.0
    # corner region: (0,0,0) to [1,2]^3 is sqrt(3)
    assert O.point_box_d2([0.0, 0.0, 0.0], box([1, 1, 1], [2, 2, 2])) == 3.0
    # inside and on the boundary: 0
    assert O.point_box_d2([1.5, 0.5], box([1, 0], [2, 1])) == 0.0
    assert O.point_box_d2([2.0, 1.0], box([1, 0], [2, 1])) == 0.0
    # face region: only one axis counts
    assert O.point_box_d2([0.5, 5.0, 0.5], box([0, 0, 0], [1, 1, 1])) == 16.0


def test_point_box_matches_clip(oracle_lib):
    rng = np.random.default_rng(11)
    for D in (2, 3):
        for _ in range(2000):
            lo = rng.uniform(-5, 5, D)
            hi = lo + rng.uniform(0, 4, D)
            c = rng.uniform(-10, 10, D)
            ref = float(np.sum((c - np.clip(c, lo, hi)) ** 2))
            got = oracle_lib.point_box_d2(c, box(lo, hi))
            assert abs(got - ref) <= 1e-13 * max(1.0, ref)


# --------------------------------------------------------------------------
# segment-box
# --------------------------------------------------------------------------

def seg_dist2(a, b, lo, hi, t):
    p = a + np.multiply.outer(np.atleast_1d(t), b - a)
    return np.sum((p - np.clip(p, lo, hi)) ** 2, axis=-1)


def golden_min(a, b, lo, hi):
    f = lambda t: float(seg_dist2(a, b, lo, hi, t)[0])
    x0, x1 = 0.0, 1.0
    g = (math.sqrt(5) - 1) / 2
    c, d = x1 - g * (x1 - x0), x0 + g * (x1 - x0)
    fc, fd = f(c), f(d)
    for _ in range(120):
        if fc < fd:
            x1, d, fd = d, c, fc
            c = x1 - g * (x1 - x0)
            fc = f(c)
        else:
            x0, c, fc = c, d, fd
            d = x0 + g * (x1 - x0)
            fd = f(d)
    return min(f(0.0), f(1.0), f(0.5 * (x0 + x1)))


def test_segbox_closed_forms(oracle_lib):
    O = oracle_lib
    B2 = box([0, 0], [1, 1])
    # horizontal segment above the box: distance 1
    assert O.segbox_fmin([-1.0, 2.0], [3.0, 2.0], B2) == 1.0
    # diagonal line x + y = -1 passes closest to corner (0,0) at (-1/2,-1/2), t = 1/2
    assert O.segbox_fmin([-2.0, 1.0], [1.0, -2.0], B2) == 0.5
    # segment through the box: 0
    assert O.segbox_fmin([-1.0, 0.5], [2.0, 0.5], B2) == 0.0
    # endpoint closest: A = (-3, 0.5) faces the left side at distance 3
    assert O.segbox_fmin([-3.0, 0.5], [-10.0, 5.0], B2) == 9.0
    # reversed orientation gives the same value
    assert O.segbox_fmin([-10.0, 5.0], [-3.0, 0.5], B2) == 9.0
    # axis-parallel 3-D segment at offset (2, 2) from an edge of the unit cube
    B3 = box([0, 0, 0], [1, 1, 1])
    assert O.segbox_fmin([3.0, 3.0, -5.0], [3.0, 3.0, 5.0], B3) == 8.0
    # degenerate segment is the point test
    assert O.segbox_fmin([2.0, 3.0, -1.0], [2.0, 3.0, -1.0], B3) == O.point_box_d2([2.0, 3.0, -1.0], B3)


@pytest.mark.parametrize("D", [2, 3])
def test_segbox_against_search(oracle_lib, D):
    rng = np.random.default_rng(100 + D)
    worst = 0.0
    for it in range(3000):
        lo = rng.uniform(-2, 2, D)
        hi = lo + rng.uniform(0.0, 2, D)
        a = rng.uniform(-5, 5, D)
        b = a + rng.normal(0, 3, D)
        if it % 7 == 0:           # axis-aligned direction components
            b[rng.integers(D)] = a[rng.integers(D)] if D > 1 else b[0]
        got = oracle_lib.segbox_fmin(a, b, box(lo, hi))
        ref = golden_min(a, b, lo, hi)
        dense = float(np.min(seg_dist2(a, b, lo, hi, np.linspace(0, 1, 4097))))
        scale = 1.0 + float(np.max(np.abs(np.concatenate([a, b, lo, hi])))) ** 2
        # the oracle finds the minimum: never above the search or dense minimum,
        # never below the true minimum (golden search is within ~1e-14 of it)
        assert got <= ref + 1e-12 * scale
        assert got <= dense + 1e-12 * scale
        assert got >= ref - 1e-9 * scale
        worst = max(worst, abs(got - ref) / scale)
    assert worst < 1e-9


# --------------------------------------------------------------------------
# motion and forward kinematics
# --------------------------------------------------------------------------

def test_se2_motion_and_fk(oracle_lib):
    rng = np.random.default_rng(5)
    rob = synth.robot_se2(rng)
    R = oracle_lib.Robot(rob)
    for _ in range(300):
        qa = np.array([*rng.uniform(0, 10, 2), rng.uniform(-math.pi, math.pi)])
        qb = np.array([*rng.uniform(0, 10, 2), rng.uniform(-math.pi, math.pi)])
        t = rng.uniform()
        q = R.interp(qa, qb, t)
        # heading goes the short way round
        dth = (qb[2] - qa[2] + math.pi) % (2 * math.pi) - math.pi
        assert abs(q[2] - (qa[2] + t * dth)) < 1e-12
        assert np.allclose(q[:2], qa[:2] + t * (qb[:2] - qa[:2]), atol=1e-12)
        assert np.allclose(R.fk(q), fk_se2_ref(rob, q), atol=1e-12)
    # wrap: from heading 3 to -3 rotates by 2 pi - 6 (positive), not by -6
    q = R.interp([0, 0, 3.0], [0, 0, -3.0], 0.5)
    assert abs(q[2] - (3.0 + (2 * math.pi - 6.0) / 2)) < 1e-14


def test_se3_motion_and_fk(oracle_lib):
    rng = np.random.default_rng(6)
    rob = synth.robot_se3(rng)
    R = oracle_lib.Robot(rob)
    for _ in range(300):
        na = synth.nodes_se3(rng, 1, 10.0)[0]
        nb = synth.nodes_se3(rng, 1, 10.0)[0]
        t = rng.uniform()
        q = R.interp(na, nb, t)
        # scipy: quaternions are scalar-last; Slerp takes the shorter arc
        rots = Rotation.from_quat([np.r_[na[4:], na[3]], np.r_[nb[4:], nb[3]]])
        rt = Slerp([0.0, 1.0], rots)([t])[0]
        p = na[:3] + t * (nb[:3] - na[:3])
        assert np.allclose(q[:3], p, atol=1e-12)
        assert abs(np.linalg.norm(q[3:]) - 1.0) < 1e-12
        assert np.allclose(R.fk(q), fk_se3_ref(rob, p, rt), atol=1e-10)


def test_arm_motion_and_fk(oracle_lib):
    rng = np.random.default_rng(7)
    rob = synth.robot_arm(rng)
    R = oracle_lib.Robot(rob)
    for _ in range(300):
        qa = rng.uniform(-math.pi, math.pi, rob.n_links)
        qb = rng.uniform(-math.pi, math.pi, rob.n_links)
        t = rng.uniform()
        q = R.interp(qa, qb, t)
        assert np.allclose(q, qa + t * (qb - qa), atol=1e-12)
        assert np.allclose(R.fk(q), fk_arm_ref(rob, q), atol=1e-12)
    # straight arm along +x: spheres at cumulative distances
    c = R.fk(np.zeros(rob.n_links))
    start = np.concatenate([[0], np.cumsum(rob.link_length)])[rob.sphere_link]
    assert np.allclose(c[:, 0], start + rob.sphere_pos, atol=1e-14)
    assert np.all(c[:, 1] == 0.0)
    # first joint at +90 degrees, others straight: arm along +y
    q = np.zeros(rob.n_links)
    q[0] = math.pi / 2
    c = R.fk(q)
    assert np.allclose(c[:, 1], start + rob.sphere_pos, atol=1e-12)


def test_sample_count(oracle_lib):
    rob = synth.Robot(synth.SE2, np.array([[0.5, 0.0]]), np.array([0.1]))
    R = oracle_lib.Robot(rob)
    # |e| = sqrt(3^2 + 4^2) = 5, eps = 0.5 -> 10 segments (11 configurations)
    assert R.n_segments([0, 0, 0], [3, 4, 0], 0.5) == 10
    assert R.n_segments([0, 0, 0], [3, 4, 0], 0.49) == 11
    # zero-length edge still has one segment (both ends)
    assert R.n_segments([1, 1, 1], [1, 1, 1], 0.5) == 1
    # a fixed count wins over the resolution
    assert R.n_segments([0, 0, 0], [3, 4, 0], 0.5, samples_per_edge=20) == 19


def _quat_z(angle):
    """Unit quaternion (w, x, y, z) of a turn by `angle` about +z."""
    return [math.cos(angle / 2), 0.0, 0.0, math.sin(angle / 2)]


def test_sample_count_se3(oracle_lib):
    """Sec. 3.2's |e|/eps for a spatial body: |e| is the Euclidean length of
    (translation, rotation angle), the angle being that of the relative turn
    (twice the half-angle of the quaternion arc), taken the short way round.
    The expected counts come from angles known by construction."""
    rob = synth.Robot(synth.SE3, np.array([[0.5, 0.0, 0.0]]), np.array([0.1]))
    R = oracle_lib.Robot(rob)
    qa = [0.0, 0.0, 0.0, *_quat_z(0.0)]
    # a quarter turn about z and no translation: |e| = pi/2 -> ceil(15.7) = 16
    assert R.n_segments(qa, [0.0, 0.0, 0.0, *_quat_z(math.pi / 2)], 0.1) == 16
    # the same turn written with the opposite quaternion sign: same motion
    assert R.n_segments(qa, [0.0, 0.0, 0.0, *(-np.array(_quat_z(math.pi / 2)))], 0.1) == 16
    # a three-quarter turn is a quarter turn the other way round
    assert R.n_segments(qa, [0.0, 0.0, 0.0, *_quat_z(1.5 * math.pi)], 0.1) == 16
    # translation (3, 4, 0) plus the quarter turn: sqrt(25 + pi^2/4) = 5.2406
    # -> ceil(52.41) = 53 (a half-angle slip would give 51, no rotation 50)
    assert R.n_segments(qa, [3.0, 4.0, 0.0, *_quat_z(math.pi / 2)], 0.1) == 53
    # a turn about a tilted axis: the angle does not depend on the axis
    ax = np.array([1.0, 2.0, 2.0]) / 3.0
    qb = [1.0, 0.0, 0.0, math.cos(0.6), *(math.sin(0.6) * ax)]   # angle 1.2
    # sqrt(1 + 1.44) = 1.5620 -> ceil(15.62) = 16 with eps 0.1, 32 with 0.05
    assert R.n_segments(qa, qb, 0.1) == 16
    assert R.n_segments(qa, qb, 0.05) == 32
    # a fixed count wins
    assert R.n_segments(qa, qb, 0.1, samples_per_edge=20) == 19


def test_sample_count_arm(oracle_lib):
    """Sec. 3.2's |e|/eps for a serial arm: |e| is the Euclidean length of the
    joint-angle change (not of the absolute link angles)."""
    rng = np.random.default_rng(3)
    rob = synth.robot_arm(rng, 3)
    R = oracle_lib.Robot(rob)
    # dq = (0.3, -0.4, 1.2): |dq| = 1.3 -> 1.3/0.07 = 18.57 -> 19; the
    # cumulative angles (0.3, -0.1, 1.1) would give 1.1446 -> 17
    assert R.n_segments([0.0, 0.0, 0.0], [0.3, -0.4, 1.2], 0.07) == 19
    assert R.n_segments([1.0, 2.0, -1.0], [1.3, 1.6, 0.2], 0.07) == 19
    # no wrap for joints: -3 to 3 is a change of 6, not 2 pi - 6
    assert R.n_segments([-3.0, 0.0, 0.0], [3.0, 0.0, 0.0], 0.7) == 9
    assert R.n_segments([0.5, 0.5, 0.5], [0.5, 0.5, 0.5], 0.1) == 1


# --------------------------------------------------------------------------
# delta: the chord-deviation bound
# --------------------------------------------------------------------------

def chord_dev(path):
    """max distance of a sampled path (T, B, D) from the chord of its ends."""
    a, b = path[0], path[-1]
    t = np.linspace(0, 1, path.shape[0])[:, None, None]
    return np.max(np.linalg.norm(path - (a + t * (b - a)), axis=-1), axis=0)


@pytest.mark.parametrize("kind", [synth.SE2, synth.SE3, synth.ARM])
def test_delta_bounds_chord_deviation(oracle_lib, kind):
    rng = np.random.default_rng(20 + kind)
    rob = {synth.SE2: synth.robot_se2, synth.SE3: synth.robot_se3, synth.ARM: synth.robot_arm}[kind](rng)
    R = oracle_lib.Robot(rob)
    ts = np.linspace(0, 1, 2001)
    for _ in range(60):
        if kind == synth.SE2:
            qa, qb = synth.nodes_se2(rng, 2, 10.0)
        elif kind == synth.SE3:
            qa, qb = synth.nodes_se3(rng, 2, 10.0)
        else:
            qa, qb = synth.nodes_arm(rng, 2, rob.n_links)
        dl = R.deltas(qa, qb)
        dev = chord_dev(centre_path(rob, qa, qb, ts))
        assert np.all(dev <= dl * (1 + 1e-9) + 1e-12), (dev, dl)


def test_delta_bounds_levers_behind_their_joint(oracle_lib):
    """Spheres behind their joint (negative distance along the link) and a
    link of negative length: the bound takes each lever by its length
    (|p''| <= sum |l_k| dPhi_k^2 + |s| dPhi_L^2).  Dense sampling of the true
    centre path checks it; the same edges show that a signed lever would
    understate the deviation, so the case has teeth."""
    rng = np.random.default_rng(31)
    rob = synth.Robot(synth.ARM, np.array([-0.6, 0.4, -0.9, 0.2]), np.array([0.1, 0.1, 0.1, 0.1]),
                      np.array([0, 1, 1, 2], dtype=np.int32), np.array([1.0, -0.7, 0.8]), (0.0, 0.0))
    R = oracle_lib.Robot(rob)
    ts = np.linspace(0, 1, 2001)
    understated = 0
    for _ in range(80):
        qa, qb = rng.uniform(-math.pi, math.pi, 3), rng.uniform(-math.pi, math.pi, 3)
        dl = R.deltas(qa, qb)
        dev = chord_dev(centre_path(rob, qa, qb, ts))
        assert np.all(dev <= dl * (1 + 1e-9) + 1e-12), (dev, dl)
        dphi = np.cumsum(qb - qa)
        for i in range(rob.n_spheres):
            L = rob.sphere_link[i]
            signed = (np.sum(rob.link_length[:L] * dphi[:L] ** 2) + rob.sphere_pos[i] * dphi[L] ** 2) / 8
            understated += int(dev[i] > signed * (1 + 1e-9) + 1e-12)
    assert understated > 0


def test_delta_pure_translation_is_zero(oracle_lib):
    rng = np.random.default_rng(9)
    for mk in (synth.robot_se2, synth.robot_se3):
        rob = mk(rng)
        R = oracle_lib.Robot(rob)
        if rob.kind == synth.SE2:
            qa, qb = [1.0, 2.0, 0.7], [5.0, -3.0, 0.7]
        else:
            qa, qb = [1, 2, 3, 0.5, 0.5, 0.5, 0.5], [4, 0, 1, 0.5, 0.5, 0.5, 0.5]
        assert np.all(R.deltas(qa, qb) == 0.0)
    rob = synth.robot_arm(rng)
    q = rng.uniform(-1, 1, rob.n_links)
    assert np.all(oracle_lib.Robot(rob).deltas(q, q) == 0.0)


def test_delta_is_tight_for_small_rotation(oracle_lib):
    # a point at radius rho turning by a small angle a: the arc's sagitta is
    # rho (1 - cos(a/2)) ~ rho a^2 / 8, the bound itself
    rob = synth.Robot(synth.SE2, np.array([[2.0, 0.0]]), np.array([0.1]))
    R = oracle_lib.Robot(rob)
    for a in (0.01, 0.1, 0.3):
        dl = R.deltas([0, 0, 0], [0, 0, a])[0]
        sag = 2.0 * (1 - math.cos(a / 2))
        assert sag <= dl <= sag * 1.01
    # Delta theta = pi: the turn is a half circle, deviation = rho exactly
    dl = R.deltas([0, 0, -math.pi / 2], [0, 0, math.pi / 2])[0]
    assert dl == pytest.approx(2.0 * math.pi ** 2 / 8)
    assert dl >= 2.0
