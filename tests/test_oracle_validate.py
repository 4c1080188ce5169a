"""Pins of the oracle's full validation of an edge (Alg. 1 when not lazy:
every edge left unknown gets a full collision check; here a continuous one,
by dyadic refinement of the outer and inner approximations of Sec. 3.2).

* the validation's sin/cos against the C library's (numpy), with exact odd
  and even symmetry, which catches a wrong quadrant map;
* the validation's sphere centres against the independent reference
  geometry (rotation matrices, scipy's Slerp, cumulative sums);
* hand-built cases whose verdict, stopping level and witness follow from
  elementary geometry;
* soundness on tiny random roadmaps against a dense brute-force check of the
  continuous motion: COLLIDES has a colliding witness configuration, FREE
  has no collision anywhere, and the verdict agrees with the edge's label
  where the label decides it;
* monotonicity: shrinking obstacles keeps FREE, growing them never turns
  COLLIDES into FREE; nodes (edges (v, v)) validate to their own label.
"""
import math

import numpy as np
import pytest

from paper_2603_28674_amd import synth
from refgeom import box_d2, centre_path
from test_oracle_labels import tiny

FREE, COLLIDES, UNRESOLVED = 0, 2, 3


def test_vsincos_matches_libm(oracle_lib):
    xs = np.concatenate([np.linspace(-200.0, 200.0, 40001),
                         np.array([0.0, 1e-300, math.pi / 4, math.pi / 2, math.pi, 1.5 * math.pi,
                                   100 * math.pi, 0.785398, 2.356194])])
    for x in xs:
        s, c = oracle_lib.vsincos(x)
        tol = 4e-16 * max(1.0, abs(x))
        assert abs(s - math.sin(x)) <= tol, x
        assert abs(c - math.cos(x)) <= tol, x
        ns, nc = oracle_lib.vsincos(-x)
        assert ns == -s and nc == c, f"symmetry at {x}"
    assert oracle_lib.vsincos(0.0) == (0.0, 1.0)


@pytest.mark.parametrize("kind", [synth.SE2, synth.SE3, synth.ARM])
def test_validation_centres_match_reference(oracle_lib, kind):
    rob, q, edges, *_ = tiny(kind, 90 + kind)
    orob = oracle_lib.Robot(rob)
    for (u, v) in edges[:10]:
        ts = np.array([0.0, 0.125, 1 / 3, 0.5, 0.7, 1.0])
        ref = centre_path(rob, q[u], q[v], ts)
        for k, t in enumerate(ts):
            got = orob.centres_v(q[u], q[v], t)
            assert np.allclose(got, ref[k], atol=1e-12), (u, v, t)


def one_sphere_se2(offset, radius):
    return synth.Robot(synth.SE2, np.array([offset], dtype=float), np.array([radius], dtype=float))


def test_translation_between_samples_collides(oracle_lib):
    """A disc (r = 0.5) translating along y = 0 from x = 0 to x = 10 with
    samples only at the ends; a box reaching down to y = 0.3 over x in
    [4, 5] is missed by both samples but met by the capsule (GRAY).  The
    midpoint t = 1/2 puts the disc at (5, 0), 0.3 from the box: COLLIDES at
    level 1 with witness 1/2."""
    rob = one_sphere_se2((0.0, 0.0), 0.5)
    q = np.array([[0.0, 0.0, 0.0], [10.0, 0.0, 0.0]])
    rm = oracle_lib.Roadmap(rob, q, np.array([[0, 1]]), 0.0, 2, n_slots=1, threads=1)
    box = np.array([[4.0, 0.3, 0.0, 5.0, 1.0, 0.0]])
    lab, gray = rm.classify(box)
    assert lab[0] == 1 and list(gray) == [0]
    v, lv, w = rm.validate([0])
    assert (v[0], lv[0], w[0]) == (COLLIDES, 1, 0.5)
    # no depth allowed: UNRESOLVED at level 0
    v, lv, w = rm.validate([0], max_level=0)
    assert (v[0], lv[0]) == (UNRESOLVED, 0) and math.isnan(w[0])
    # a box over the end node only: the end configuration is the witness
    rm.classify(np.array([[9.8, -0.2, 0.0, 10.6, 0.2, 0.0]]))
    v, lv, w = rm.validate([0])
    assert (v[0], lv[0], w[0]) == (COLLIDES, 0, 1.0)


def test_smallest_witness_at_the_first_colliding_level(oracle_lib):
    """Path x in [0, 16]; boxes over x in [3.5, 4.5] and [11.5, 12.5] reaching
    y = 0.2.  Level 1's midpoint x = 8 misses; level 2's midpoints x = 4
    and x = 12 both hit, and the witness is the smaller, t = 1/4."""
    rob = one_sphere_se2((0.0, 0.0), 0.5)
    q = np.array([[0.0, 0.0, 0.0], [16.0, 0.0, 0.0]])
    rm = oracle_lib.Roadmap(rob, q, np.array([[0, 1]]), 0.0, 2, n_slots=2, threads=1)
    boxes = np.array([[11.5, 0.2, 0.0, 12.5, 1.0, 0.0], [3.5, 0.2, 0.0, 4.5, 1.0, 0.0]])
    rm.classify(boxes)
    v, lv, w = rm.validate([0])
    assert (v[0], lv[0], w[0]) == (COLLIDES, 2, 0.25)


def rotating_case(oracle_lib, corner):
    """A disc (r = 0.1) at offset (2, 0) turning a quarter turn about the
    origin: its centre runs on the arc of radius 2 from (2, 0) to (0, 2).
    The chord passes sqrt(2) from the origin and delta = 2 (pi/2)^2 / 8, so
    the capsule (radius 0.1 + pi^2/16) reaches a small box whose far corner
    is (corner, corner); the disc never comes closer to the origin than
    1.9, so the motion is free while sqrt(2) corner < 1.9."""
    rob = one_sphere_se2((2.0, 0.0), 0.1)
    q = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, math.pi / 2]])
    rm = oracle_lib.Roadmap(rob, q, np.array([[0, 1]]), 0.0, 2, n_slots=1, threads=1)
    box = np.array([[corner - 0.1, corner - 0.1, 0.0, corner, corner, 0.0]])
    lab, _ = rm.classify(box)
    return rm, lab


def test_rotation_gray_but_free(oracle_lib):
    rm, lab = rotating_case(oracle_lib, 0.85)
    assert lab[0] == 1                             # the capsule meets, no sample does
    v, lv, w = rm.validate([0])
    # level 1: chords (2,0)-(sqrt2,sqrt2) and (sqrt2,sqrt2)-(0,2), radius
    # 0.1 + delta/4 ~ 0.254, pass 2 cos(pi/8) ~ 1.85 from the origin
    assert (v[0], lv[0]) == (FREE, 1) and math.isnan(w[0])
    # the closer the box to the arc, the deeper the search; never COLLIDES.
    # The stopping level is the first l at which every one of the 2^l
    # chords of the arc, inflated to 0.1 + delta 4^-l, misses the box
    # (chord-box distances by dense sampling of each chord).
    levels = []
    for corner in (0.95, 1.1, 1.25, 1.3):
        rm, _ = rotating_case(oracle_lib, corner)
        v, lv, _ = rm.validate([0])
        assert v[0] == FREE, corner
        levels.append(int(lv[0]))
        box = np.array([corner - 0.1, corner - 0.1, 0.0, corner, corner, 0.0])
        delta = math.pi ** 2 / 16
        for level in range(0, 12):
            k = 2 ** level
            ang = np.arange(k + 1) * (math.pi / 2) / k
            ends = 2 * np.stack([np.cos(ang), np.sin(ang)], axis=1)
            s = np.linspace(0.0, 1.0, 2001)[:, None, None]
            pts = ends[:-1][None] + s * (ends[1:] - ends[:-1])[None]
            dist = np.sqrt(np.min(box_d2(pts, box, 2)))
            if dist > 0.1 + delta / 4 ** level + 1e-6:
                break
        assert lv[0] == level, (corner, int(lv[0]), level)
    assert levels == sorted(levels) and levels[-1] > levels[0]
    # a box straddling the arc collides
    rm, _ = rotating_case(oracle_lib, 1.45)
    v, _, w = rm.validate([0])
    assert v[0] == COLLIDES
    t = float(w[0])
    c = np.array([2 * math.cos(t * math.pi / 2), 2 * math.sin(t * math.pi / 2)])
    assert box_d2(c[None], np.array([1.35, 1.35, 0, 1.45, 1.45, 0]), 2)[0] <= 0.01 + 1e-12


def test_active_limit(oracle_lib):
    """The two-box path above: level 1's midpoint misses and both halves stay
    unknown, so with one active interval allowed the search stops
    UNRESOLVED at level 1."""
    rob = one_sphere_se2((0.0, 0.0), 0.5)
    q = np.array([[0.0, 0.0, 0.0], [16.0, 0.0, 0.0]])
    rm = oracle_lib.Roadmap(rob, q, np.array([[0, 1]]), 0.0, 2, n_slots=2, threads=1)
    rm.classify(np.array([[11.5, 0.2, 0.0, 12.5, 1.0, 0.0], [3.5, 0.2, 0.0, 4.5, 1.0, 0.0]]))
    v, lv, w = rm.validate([0], max_active=1)
    assert (v[0], lv[0]) == (UNRESOLVED, 1) and math.isnan(w[0])
    v, lv, w = rm.validate([0], max_active=2)
    assert (v[0], lv[0], w[0]) == (COLLIDES, 2, 0.25)
    with pytest.raises(ValueError):
        rm.validate([0], max_level=31)
    with pytest.raises(ValueError):
        rm.validate([1])


@pytest.mark.parametrize("kind", [synth.SE2, synth.SE3, synth.ARM])
@pytest.mark.parametrize("seed", [1, 2])
def test_validation_sound_brute_force(oracle_lib, kind, seed):
    rob, q, edges, res, spe, boxes = tiny(kind, seed, n_nodes=20, n_boxes=4)
    rm = oracle_lib.Roadmap(rob, q, edges, res, spe, n_slots=len(boxes), threads=2)
    labels, _ = rm.classify(boxes)
    verdict, level, witness = rm.validate(np.arange(len(edges)), max_level=20, max_active=512)
    D = rob.dim
    rad2 = rob.sphere_radius ** 2
    seen = np.zeros(4, dtype=int)
    for e, (u, v) in enumerate(edges):
        ts = np.linspace(0.0, 1.0, 4097)
        dense = centre_path(rob, q[u], q[v], ts)
        gap = np.min([np.min(box_d2(dense, b, D) - rad2) for b in boxes])
        if verdict[e] == COLLIDES:
            c = centre_path(rob, q[u], q[v], [witness[e]])[0]
            assert min(np.min(box_d2(c, b, D) - rad2) for b in boxes) <= 1e-9, e
        elif verdict[e] == FREE:
            assert gap > -1e-9, f"edge {e}: FREE but the dense check collides"
            assert np.isnan(witness[e])
        if labels[e] == 2:
            assert verdict[e] != FREE
        if labels[e] == 0:
            assert verdict[e] == FREE and level[e] == 0
        if gap < -1e-6:
            assert verdict[e] != FREE
        seen[verdict[e]] += 1
    assert seen[FREE] > 0 and seen[COLLIDES] > 0


@pytest.mark.parametrize("kind", [synth.SE2, synth.SE3, synth.ARM])
def test_validation_monotone(oracle_lib, kind):
    rob, q, edges, res, spe, boxes = tiny(kind, 50 + kind, n_nodes=16, n_boxes=8)
    D = rob.dim
    rm = oracle_lib.Roadmap(rob, q, edges, res, spe, n_slots=len(boxes), threads=2)
    ids = np.arange(len(edges))
    rm.classify(boxes)
    base, _, _ = rm.validate(ids, max_level=16)
    rng = np.random.default_rng(kind)
    for _ in range(3):
        grown = boxes.copy()
        grown[:, :D] -= rng.uniform(0, 0.3, (len(boxes), D))
        grown[:, 3:3 + D] += rng.uniform(0, 0.3, (len(boxes), D))
        rm.classify(grown)
        g, _, _ = rm.validate(ids, max_level=16)
        assert not np.any((base == COLLIDES) & (g == FREE))
        shrunk = boxes.copy()
        mid = 0.5 * (boxes[:, :D] + boxes[:, 3:3 + D])
        shrunk[:, :D] = mid - 0.4 * (mid - boxes[:, :D])
        shrunk[:, 3:3 + D] = mid + 0.4 * (boxes[:, 3:3 + D] - mid)
        rm.classify(shrunk)
        s, _, _ = rm.validate(ids, max_level=16)
        assert np.all(s[base == FREE] == FREE)


def test_nodes_validate_to_their_label(oracle_lib):
    rob, q, edges, res, spe, boxes = tiny(synth.SE2, 5, n_nodes=30, n_boxes=10)
    nodes = np.stack([np.arange(len(q))] * 2, axis=1)
    rm = oracle_lib.Roadmap(rob, q, nodes, res, spe, n_slots=len(boxes), threads=2)
    lab, gray = rm.classify(boxes)
    assert len(gray) == 0
    v, lv, w = rm.validate(np.arange(len(q)))
    assert np.all(v[lab == 2] == COLLIDES) and np.all(w[lab == 2] == 0.0)
    assert np.all(v[lab == 0] == FREE) and np.all(lv == 0)


def grazing_case(oracle_lib, radius_of_corner):
    """The quarter turn of rotating_case with a box whose corner lies on the
    ray at 30 degrees (t = 1/3, not dyadic), at `radius_of_corner` from the
    origin: 1.9 touches the disc's sweep, less clears it, more enters it."""
    rob = one_sphere_se2((2.0, 0.0), 0.1)
    q = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, math.pi / 2]])
    rm = oracle_lib.Roadmap(rob, q, np.array([[0, 1]]), 0.0, 2, n_slots=1, threads=1)
    cx, cy = radius_of_corner * math.cos(math.pi / 6), radius_of_corner * math.sin(math.pi / 6)
    rm.classify(np.array([[cx - 0.3, cy - 0.3, 0.0, cx, cy, 0.0]]))
    return rm


def test_deep_search_tracks_the_clearance(oracle_lib):
    """The chord deviation of a level-l interval is delta 4^-l, so a clearance
    g is certified once delta 4^-l falls below about g: dividing g by 10^6
    deepens the FREE level by log4(10^6) ~ 10 levels.  A penetration is
    found once a midpoint lands inside it, within 2^-l of t = 1/3."""
    levels = {}
    for g in (1e-6, 1e-12):
        v, lv, _ = grazing_case(oracle_lib, 1.9 - g).validate([0], max_level=30, max_active=1024)
        assert v[0] == FREE
        levels[g] = int(lv[0])
    assert abs((levels[1e-12] - levels[1e-6]) - math.log(1e6, 4)) <= 1.5, levels
    assert 4.0 ** -levels[1e-6] * math.pi ** 2 / 16 < 1e-5
    v, lv, w = grazing_case(oracle_lib, 1.9 + 1e-12).validate([0], max_level=30, max_active=1024)
    assert v[0] == COLLIDES and abs(w[0] - 1.0 / 3.0) < 2.0 ** -(int(lv[0]) - 1)
    # not enough levels: UNRESOLVED at the limit
    v, lv, _ = grazing_case(oracle_lib, 1.9 + 1e-12).validate([0], max_level=16, max_active=1024)
    assert (v[0], lv[0]) == (UNRESOLVED, 16)
