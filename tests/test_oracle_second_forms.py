"""Pins of the oracle's second approximation forms (paper Sec. 4.2).

Outer: an oriented box (OBB) per robot body, fitted to the principal axes of
the point cloud of the body's sphere centres along the edge, tested against a
box obstacle by the separating-axis theorem; the edge's outer approximation
is then each sphere's capsule intersected with its body's box.
Inner: each sphere's spline (the polyline through its centres), shortened by
Agarwal et al.'s greedy simplification and thickened to the radius that keeps
it inside the swept sphere.

Each part is checked against something outside the oracle:
* the Jacobi eigenvectors against numpy's symmetric eigensolver;
* the separating-axis test against a linear-programming feasibility check of
  the two boxes' intersection (scipy), including cases only an edge-edge
  axis separates;
* the boxes and the spline capsules against a dense sampling of the
  continuous motion (reference kinematics in refgeom.py);
* the simplification against a hand-derived vertex list and its defining
  properties (every kept shortcut within tolerance, none extendable);
* labels: soundness by brute force, monotonicity, incremental == scratch,
  and the relations to the capsule/copy forms (red unchanged by the boxes,
  green only grows).
"""
import math

import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.spatial.transform import Rotation

from paper_2603_28674_amd import synth
from refgeom import box_d2, centre_path
from test_oracle_labels import tiny


# --------------------------------------------------------------------------
# principal axes
# --------------------------------------------------------------------------

@pytest.mark.parametrize("D", [2, 3])
def test_jacobi_eigen_matches_numpy(oracle_lib, D):
    rng = np.random.default_rng(11 + D)
    mats = [rng.normal(size=(D, D)) for _ in range(200)]
    mats = [m @ m.T for m in mats]
    mats += [np.diag(rng.uniform(0, 5, D)), np.eye(D), np.zeros((D, D)), np.ones((D, D))]
    if D == 3:
        Q = Rotation.random(random_state=3).as_matrix()
        mats.append(Q @ np.diag([2.0, 2.0, 5.0]) @ Q.T)    # a repeated eigenvalue
    for a in mats:
        v = oracle_lib.jacobi_eigen(a)
        assert np.allclose(v.T @ v, np.eye(D), atol=1e-14)
        assert abs(np.linalg.det(v) - 1.0) < 1e-13           # a product of rotations
        d = v.T @ a @ v
        scale = max(np.abs(a).max(), 1e-300)
        assert np.abs(d - np.diag(np.diag(d))).max() <= 1e-12 * scale
        assert np.allclose(np.sort(np.diag(d)), np.linalg.eigvalsh(a), atol=1e-12 * scale)


# --------------------------------------------------------------------------
# separating-axis test
# --------------------------------------------------------------------------

def _lp_meet(c, u, h, box, D, grow=0.0):
    """Feasibility of {x : lo <= x <= hi, |u_k . (x - c)| <= h_k}, with both
    boxes grown by `grow` (negative shrinks)."""
    lo, hi = box[:D] - grow, box[3:3 + D] + grow
    A = np.vstack([u, -u])
    b = np.concatenate([h + grow + u @ c, h + grow - u @ c])
    r = linprog(np.zeros(D), A_ub=A, b_ub=b, bounds=list(zip(lo, hi)), method="highs")
    return r.status == 0


def _rand_frame(rng, D):
    if D == 2:
        a = rng.uniform(-math.pi, math.pi)
        return np.array([[math.cos(a), math.sin(a)], [-math.sin(a), math.cos(a)]])
    return Rotation.random(random_state=int(rng.integers(1 << 30))).as_matrix().T


@pytest.mark.parametrize("D", [2, 3])
def test_sat_matches_linear_program(oracle_lib, D):
    rng = np.random.default_rng(21 + D)
    decided = edge_only = 0
    for _ in range(1500):
        u = _rand_frame(rng, D)
        h = rng.uniform(0.05, 1.0, D)
        c = rng.uniform(-1.5, 1.5, D)
        lo = rng.uniform(-1.0, 0.5, D)
        hi = lo + rng.uniform(0.05, 1.0, D)
        box = np.zeros(6)
        box[:D], box[3:3 + D] = lo, hi
        got = oracle_lib.obb_box_meet(c, u, h, box)
        if _lp_meet(c, u, h, box, D, grow=-1e-7):
            assert got, "boxes that overlap were separated"
            decided += 1
        elif not _lp_meet(c, u, h, box, D, grow=1e-7):
            assert not got, "disjoint boxes were not separated"
            decided += 1
            # separated although no face normal of either box separates
            bc, bh = 0.5 * (lo + hi), 0.5 * (hi - lo)
            t = c - bc
            faces = any(abs(t[d]) > bh[d] + np.sum(h * np.abs(u[:, d])) for d in range(D)) or \
                any(abs(u[k] @ t) > h[k] + np.sum(bh * np.abs(u[k])) for k in range(D))
            edge_only += int(not faces)
    assert decided > 1400
    if D == 3:
        assert edge_only >= 5, "no case needed an edge-edge axis"


def test_sat_hand_cases(oracle_lib):
    I3 = np.eye(3)
    box = np.array([-1.0, -1.0, -1.0, 1.0, 1.0, 1.0])
    ones = np.ones(3)
    # face separation along x: a gap of 1, then touching faces (closed sets)
    assert not oracle_lib.obb_box_meet(np.array([3.0, 0, 0]), I3, ones, box)
    assert oracle_lib.obb_box_meet(np.array([2.0, 0, 0]), I3, ones, box)
    # a cube turned 45 degrees about z, its edge pointing at the face x = 1:
    # the edge reaches x = c - sqrt(2) (box's face normal separates iff c > 1 + sqrt(2))
    Rz = Rotation.from_euler("z", 45, degrees=True).as_matrix().T
    assert oracle_lib.obb_box_meet(np.array([2.4, 0, 0]), Rz, ones, box)
    assert not oracle_lib.obb_box_meet(np.array([2.45, 0, 0]), Rz, ones, box)
    # edge against edge: the box's edge along z at (1, 1), the oriented box's
    # edge along (1, -1, 0)/sqrt(2) after turning 45 degrees about z and
    # 45 degrees about its new x; only the axis (1, 1, 0) x ... separates.
    # The oriented cube's extent along w = (1,1,0)/sqrt(2) from its centre is
    # |u_k . w| summed: 1 (u_0 = (1,1,0)/sqrt(2) turned about itself keeps w),
    # so it reaches down to c.w - 1; the box reaches sqrt(2) along w.
    R = (Rotation.from_euler("z", 45, degrees=True) * Rotation.from_euler("x", 45, degrees=True)).as_matrix().T
    w = np.array([1.0, 1.0, 0.0]) / math.sqrt(2)
    for s, want in ((math.sqrt(2) + 1.0 + 1e-6, False), (math.sqrt(2) + 1.0 - 1e-6, True)):
        c = s * w
        got = oracle_lib.obb_box_meet(c, R, ones, box)
        assert got == want
        assert got == _lp_meet(c, R, ones, box, 3)
    # planar
    I2 = np.eye(2)
    b2 = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 0.0])
    assert oracle_lib.obb_box_meet(np.array([2.0, 0.5]), I2, np.array([1.0, 1.0]), b2)
    assert not oracle_lib.obb_box_meet(np.array([2.0 + 1e-9, 0.5]), I2, np.array([1.0, 1.0]), b2)


# --------------------------------------------------------------------------
# the boxes hold the continuous swept volume
# --------------------------------------------------------------------------

def _bodies(rob):
    if rob.kind == synth.ARM:
        return [np.nonzero(rob.sphere_link == b)[0] for b in range(rob.n_links)]
    return [np.arange(rob.n_spheres)]


@pytest.mark.parametrize("kind", [synth.SE2, synth.SE3, synth.ARM])
def test_obb_contains_swept_volume(oracle_lib, kind):
    worst = -np.inf
    for seed in (1, 2, 3):
        rob, q, edges, res, spe, boxes = tiny(kind, 300 + seed, n_nodes=14)
        rm = oracle_lib.Roadmap(rob, q, edges, res, spe, n_slots=1, threads=2, outer_obb=True)
        for e, (a, b) in enumerate(edges):
            n = rm.n_configs(e) - 1
            dense = centre_path(rob, q[a], q[b], np.linspace(0.0, 1.0, 64 * n + 1))   # (T, B, D)
            for bi, members in enumerate(_bodies(rob)):
                got = rm.obb(e, bi)
                if members.size == 0:
                    assert got is None
                    continue
                c, u, h = got
                # coordinates of every centre in the box's frame, widened by its radius
                s = np.abs((dense[:, members] - c) @ u.T) + rob.sphere_radius[members][None, :, None]
                excess = s - h[None, None, :]
                worst = max(worst, float(np.max(excess / (1.0 + np.abs(h)))))
    assert worst <= 1e-9, f"a sphere leaves its body's box by {worst}"


# --------------------------------------------------------------------------
# spline simplification
# --------------------------------------------------------------------------

def test_spline_hand_cases(oracle_lib):
    # collinear centres: one segment, full radius less eta
    pts = np.stack([np.arange(7.0), np.zeros(7)], axis=1)
    seg = oracle_lib.sphere_spline(pts, 0.3, 0.01, 0.05)
    assert seg.shape == (1, 5)
    assert np.allclose(seg[0], [0, 0, 6, 0, 0.29])
    # one bump of height d between two collinear neighbours
    for d, tol, k in ((0.01, 0.05, 1), (0.02, 0.05, 2)):
        pts = np.array([[0.0, 0.0], [1.0, d], [2.0, 0.0]])
        seg = oracle_lib.sphere_spline(pts, 0.3, 0.0, tol)          # lim = 0.015
        assert len(seg) == k
        if k == 1:
            assert math.isclose(seg[0, 4], 0.3 - d, rel_tol=1e-15)
        else:
            assert np.allclose(seg[:, 4], 0.3)
    # six collinear centres along x, then four up along x = 5: the
    # exponential search accepts b = 2, 4, rejects 8, bisects to 5 (b = 6
    # leaves (5,0) at 5/sqrt(26) = 0.98 from the segment); from 5 the rest
    # is collinear: segments (0,5) and (5,9)
    pts = np.array([[j, 0.0] for j in range(6)] + [[5.0, j - 5.0] for j in range(6, 10)])
    seg = oracle_lib.sphere_spline(pts, 1.0, 0.0, 0.5)
    assert np.allclose(seg[:, :4], [[0, 0, 5, 0], [5, 0, 5, 4]])
    # a negative radius drops the segment
    assert len(oracle_lib.sphere_spline(pts, 0.1, 0.2, 0.5)) == 0


def test_spline_quarter_arc_vertices(oracle_lib):
    """A disk at offset 1 turning a quarter circle, 33 centres on the unit
    circle at angles j pi/64, tolerance 0.05 r = 0.0125.  A shortcut over k
    steps leaves its middle vertex 1 - cos(k pi/128) from the chord: k = 6
    gives 0.01082 (accepted), k = 7 leaves vertices 3 and 4 at
    cos(pi/128) - cos(7 pi/128) = 0.01442 (rejected), k = 8 gives 0.01921.
    The search accepts 2 and 4, rejects 8, bisects to 6 (7 rejected): the
    vertices are 0, 6, 12, 18, 24, 30 and then 32 (two steps, 0.00120)."""
    rob = synth.Robot(synth.SE2, np.array([[1.0, 0.0]]), np.array([0.25]))
    q = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, math.pi / 2]])
    rm = oracle_lib.Roadmap(rob, q, np.array([[0, 1]]), 0.05, 0, n_slots=1, threads=1,
                            inner_splines=True, spline_tol=0.05)
    assert rm.n_configs(0) == 33
    seg = rm.spline(0, 0)
    cen = rm.centres(0)[:, 0]
    verts = [0, 6, 12, 18, 24, 30, 32]
    assert len(seg) == len(verts) - 1
    eta = (math.pi / 2) ** 2 / 8 / 32 ** 2
    for k in range(len(seg)):
        a, b = verts[k], verts[k + 1]
        assert np.array_equal(seg[k, :2], cen[a]) and np.array_equal(seg[k, 2:4], cen[b])
        err = 1 - math.cos((b - a) * math.pi / 128)
        assert math.isclose(seg[k, 4], 0.25 - err - eta, rel_tol=1e-12)


def _seg_dist(p, a, b):
    d = b - a
    dd = d @ d
    t = 0.0 if dd == 0 else min(max((p - a) @ d / dd, 0.0), 1.0)
    return float(np.linalg.norm(a + t * d - p))


@pytest.mark.parametrize("kind", [synth.SE2, synth.SE3, synth.ARM])
@pytest.mark.parametrize("tol", [0.0, 0.05, 0.3])
def test_spline_properties_and_containment(oracle_lib, kind, tol):
    """Every kept segment joins two centres of the sphere, in order, within
    tolerance of the centres it skips and not extendable by one more; and
    the capsule of radius rho around it lies in the sphere's swept volume:
    each of its points is within r - rho of the continuous centre path."""
    rob, q, edges, res, spe, boxes = tiny(kind, 400 + kind, n_nodes=12)
    rm = oracle_lib.Roadmap(rob, q, edges, res, spe, n_slots=1, threads=2, inner_splines=True, spline_tol=tol)
    worst = -np.inf
    for e, (a, b) in enumerate(edges):
        n = rm.n_configs(e) - 1
        cen = rm.centres(e)
        ts = np.linspace(0.0, 1.0, 256 * n + 1)
        dense = centre_path(rob, q[a], q[b], ts)
        for i in range(rob.n_spheres):
            r = rob.sphere_radius[i]
            seg = rm.spline(e, i)
            path = dense[:, i]
            step = float(np.max(np.linalg.norm(np.diff(path, axis=0), axis=1)))
            for g in seg:
                A, B, rho = g[:rob.dim], g[rob.dim:2 * rob.dim], g[-1]
                ia = np.nonzero(np.all(cen[:, i] == A, axis=1))[0]
                ib = np.nonzero(np.all(cen[:, i] == B, axis=1))[0]
                assert ia.size and ib.size
                ja, jb = ia.min(), ib.max()
                err = max([_seg_dist(cen[m, i], A, B) for m in range(ja + 1, jb)] + [0.0])
                assert err <= tol * r * (1 + 1e-12)
                assert rho >= 0.0
                if jb < n:
                    nxt = max(_seg_dist(cen[m, i], A, cen[jb + 1, i]) for m in range(ja + 1, jb + 1))
                    assert nxt > tol * r
                for s in np.linspace(0.0, 1.0, 33):
                    x = A + s * (B - A)
                    gap = float(np.min(np.linalg.norm(path - x, axis=1)))
                    worst = max(worst, gap - (r - rho) - step / 2)
    assert worst <= 1e-9, f"a spline capsule leaves the swept sphere by {worst}"


def test_spline_covers_the_whole_edge_without_tolerance(oracle_lib):
    """tol = 0 keeps every vertex of a curved path: n segments from
    configuration 0 to n."""
    rob, q, edges, res, spe, boxes = tiny(synth.SE2, 8)
    rm = oracle_lib.Roadmap(rob, q, edges, res, spe, n_slots=1, threads=1, inner_splines=True, spline_tol=0.0)
    for e in range(len(edges)):
        n = rm.n_configs(e) - 1
        cen = rm.centres(e)
        for i in range(rob.n_spheres):
            seg = rm.spline(e, i)
            if len(seg) == n:
                assert np.array_equal(seg[0, :2], cen[0, i]) and np.array_equal(seg[-1, 2:4], cen[n, i])


# --------------------------------------------------------------------------
# labels
# --------------------------------------------------------------------------

MODES = [(True, False), (False, True), (True, True)]


@pytest.mark.parametrize("kind", [synth.SE2, synth.SE3, synth.ARM])
@pytest.mark.parametrize("mode", MODES, ids=["obb", "splines", "obb+splines"])
def test_second_forms_soundness_brute_force(oracle_lib, kind, mode):
    """RED implies a real collision on the continuous motion (the inner form
    lies in the swept volume); GREEN implies none (the outer form holds it)."""
    obb, spl = mode
    for seed in (1, 2):
        rob, q, edges, res, spe, boxes = tiny(kind, 500 + seed)
        rm = oracle_lib.Roadmap(rob, q, edges, res, spe, n_slots=len(boxes), threads=2, outer_obb=obb,
                                inner_splines=spl, spline_tol=0.05)
        labels, _ = rm.classify(boxes)
        D = rob.dim
        rad2 = rob.sphere_radius ** 2
        for e, (u, v) in enumerate(edges):
            n = rm.n_configs(e) - 1
            dense = centre_path(rob, q[u], q[v], np.linspace(0.0, 1.0, 128 * n + 1))
            step = float(np.max(np.linalg.norm(np.diff(dense, axis=0), axis=-1)))
            hit = near = False
            for b in boxes:
                dd = box_d2(dense, b, D) - rad2
                hit |= bool(np.any(dd <= -1e-9))
                # within half a dense step of touching
                near |= bool(np.any(np.sqrt(box_d2(dense, b, D)) <= rob.sphere_radius + step / 2 + 1e-9))
            if labels[e] == 0:
                assert not hit, "green edge collides"
            if labels[e] == 2:
                assert near, "red edge has no collision"


@pytest.mark.parametrize("kind", [synth.SE2, synth.SE3, synth.ARM])
def test_obb_only_shrinks_gray(oracle_lib, kind):
    """The boxes narrow the outer approximation and leave the inner one: red
    is unchanged, every green edge stays green, gray can only turn green."""
    for seed in (1, 2, 3):
        rob, q, edges, res, spe, boxes = tiny(kind, 600 + seed, n_nodes=20, n_boxes=10)
        plain = oracle_lib.Roadmap(rob, q, edges, res, spe, n_slots=len(boxes), threads=2)
        with_obb = oracle_lib.Roadmap(rob, q, edges, res, spe, n_slots=len(boxes), threads=2, outer_obb=True)
        lp, _ = plain.classify(boxes)
        lo, _ = with_obb.classify(boxes)
        assert np.array_equal(lp == 2, lo == 2)
        assert np.all(lo[lp == 0] == 0)
        assert np.all((lo == lp) | ((lp == 1) & (lo == 0)))


@pytest.mark.parametrize("kind", [synth.SE2, synth.SE3, synth.ARM])
@pytest.mark.parametrize("mode", MODES, ids=["obb", "splines", "obb+splines"])
def test_second_forms_incremental_equals_scratch(oracle_lib, kind, mode):
    obb, spl = mode
    rob, q, edges, res, spe, boxes = tiny(kind, 700 + kind, n_nodes=25, n_boxes=10)
    M = len(boxes)
    kw = dict(outer_obb=obb, inner_splines=spl, spline_tol=0.05)
    inc = oracle_lib.Roadmap(rob, q, edges, res, spe, n_slots=M, threads=3, **kw)
    scr = oracle_lib.Roadmap(rob, q, edges, res, spe, n_slots=M, threads=1, **kw)
    rng = np.random.default_rng(9)
    cur = np.tile(synth.ABSENT_BOX, (M, 1))
    D = rob.dim
    for step in range(10):
        nxt = cur.copy()
        for k in rng.choice(M, size=rng.integers(1, M + 1), replace=False):
            r = rng.uniform()
            if r < 0.2:
                nxt[k] = synth.ABSENT_BOX
            elif np.any(cur[k, :D] > cur[k, 3:3 + D]) or r < 0.4:
                nxt[k] = boxes[rng.integers(M)]
            else:
                off = rng.normal(0, 0.4, D)
                nxt[k, :D] += off
                nxt[k, 3:3 + D] += off
        li, gi = inc.update(cur, nxt)
        ls, gs = scr.classify(nxt)
        assert np.array_equal(li, ls) and np.array_equal(gi, gs)
        oi, ii = inc.counters()
        assert np.all(oi[ii > 0] > 0)          # S implies C
        cur = nxt


@pytest.mark.parametrize("mode", MODES, ids=["obb", "splines", "obb+splines"])
def test_second_forms_monotone(oracle_lib, mode):
    obb, spl = mode
    for kind in (synth.SE2, synth.SE3, synth.ARM):
        rob, q, edges, res, spe, boxes = tiny(kind, 800 + kind, n_nodes=20, n_boxes=6)
        rm = oracle_lib.Roadmap(rob, q, edges, res, spe, n_slots=len(boxes), threads=2, outer_obb=obb,
                                inner_splines=spl, spline_tol=0.05)
        base, _ = rm.classify(boxes)
        D = rob.dim
        rng = np.random.default_rng(17)
        for _ in range(5):
            grown = boxes.copy()
            k = rng.integers(len(boxes))
            grown[k, :D] -= rng.uniform(0, 0.5, D)
            grown[k, 3:3 + D] += rng.uniform(0, 0.5, D)
            lab, _ = rm.classify(grown)
            assert np.all(lab[base == 2] == 2)
            assert np.all(lab[base == 1] >= 1)


def test_spline_pure_translation_has_no_gray(oracle_lib):
    """Without rotation delta = 0 and the centres of a sphere are collinear:
    its spline is one segment of the full radius, equal to its capsule (up
    to the rounding of the centres), so the inner and outer forms coincide
    and no edge is gray."""
    rng = np.random.default_rng(5)
    rob = synth.robot_se2(rng)
    q = synth.nodes_se2(rng, 30, 6.0)
    q[:, 2] = 0.3                                   # one heading for every node
    edges = synth.knn_se2(q, 4)
    boxes = synth.random_boxes(rng, 12, 2, 0.2, 1.5, 0.0, 6.0)
    rm = oracle_lib.Roadmap(rob, q, edges, 0.25, 0, n_slots=len(boxes), threads=2, inner_splines=True,
                            spline_tol=0.05)
    lab, gray = rm.classify(boxes)
    assert len(gray) == 0 and np.any(lab == 2)
    for e in range(len(edges)):
        for i in range(rob.n_spheres):
            seg = rm.spline(e, i)
            # the centres are collinear up to rounding: full radius up to rounding
            assert len(seg) == 1 and math.isclose(seg[0, -1], rob.sphere_radius[i], rel_tol=1e-12)


def test_bad_spline_tolerance_refused(oracle_lib):
    rob, q, edges, res, spe, boxes = tiny(synth.SE2, 1)
    for tol in (-0.1, 1.0, float("nan")):
        with pytest.raises(ValueError):
            oracle_lib.Roadmap(rob, q, edges, res, spe, n_slots=1, inner_splines=True, spline_tol=tol)
