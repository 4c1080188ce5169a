"""GPU parity of the full validation (rgg_validate, rgg_validate_async)
with the oracle's: verdicts, stopping levels and witness parameters must be
identical, element by element (the search's decisions are binary64
predicates evaluated in a fixed order on both sides).

Cases: the gray lists of update sequences of all three robot kinds in both
precision modes, samples of the other edges, tight refinement limits (so
UNRESOLVED occurs), more candidate boxes than one LDS page, the device-side
pipeline chained after an update (count read from the update's result, a
failed update validating nothing), ids that are not edges, and argument
errors.
"""
import numpy as np
import pytest

from paper_2603_28674_amd import synth

pytestmark = pytest.mark.gpu

FREE, COLLIDES, UNRESOLVED, BAD_ID = 0, 2, 3, 255


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2603_28674_amd import rgg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = rgg.rgg_context_create(0)
    yield c
    rgg.rgg_context_destroy(c)


def workload(kind, n_updates):
    if kind == "planar":
        return synth.planar_rigid(seed=21, n_nodes=1500, n_boxes=40, n_updates=n_updates)
    if kind == "spatial":
        return synth.spatial_rigid(seed=22, n_nodes=2000, n_boxes=100, n_updates=n_updates, world=4.0)
    return synth.planar_arm(seed=23, n_nodes=1500, n_boxes=40, n_updates=n_updates)


def same(got, want, what):
    gv, gl, gw = got
    ov, ol, ow = want
    bad = np.nonzero((gv != ov) | (gl != ol) | ~((gw == ow) | (np.isnan(gw) & np.isnan(ow))))[0]
    assert bad.size == 0, (f"{what}: {bad.size} of {len(gv)} differ; first {bad[:5]}: "
                           f"gpu {list(zip(gv[bad[:3]], gl[bad[:3]], gw[bad[:3]]))} "
                           f"oracle {list(zip(ov[bad[:3]], ol[bad[:3]], ow[bad[:3]]))}")


@pytest.mark.parametrize("kind", ["planar", "spatial", "arm"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_validate_gray_lists_match_oracle(ctx, kind, prec):
    from paper_2603_28674_amd import rgg
    import oracle
    n_updates = 3
    w = workload(kind, n_updates)
    precision = rgg.RGG_PREC_FP32_RECHECK if prec == "fp32" else rgg.RGG_PREC_FP64
    print(f"[validate] {w.name} E={w.n_edges} M={w.n_slots} {prec}", flush=True)
    g = rgg.Roadmap.from_workload(ctx, w, precision=precision)
    o = oracle.from_workload(w)
    rng = np.random.default_rng(len(kind))
    prev = w.absent()
    mix = np.zeros(4, dtype=int)
    for u in range(n_updates):
        lab, gray, n, _ = g.update(prev, w.boxes[u])
        ol, og = o.update(prev, w.boxes[u])
        assert np.array_equal(gray, og)
        got = g.validate(gray)
        same(got, o.validate(gray), f"update {u} gray list")
        mix += np.bincount(got[0], minlength=4)[:4]
        # every kind of edge, not only gray ones
        others = np.sort(rng.choice(w.n_edges, size=min(300, w.n_edges), replace=False))
        same(g.validate(others), o.validate(others), f"update {u} sampled edges")
        # tight limits: UNRESOLVED appears
        tight = g.validate(gray, max_level=3, max_active=2)
        same(tight, o.validate(gray, max_level=3, max_active=2), f"update {u} tight limits")
        print(f"[validate] update {u}: {len(gray)} gray -> verdicts {np.bincount(got[0], minlength=4)}, "
              f"tight {np.bincount(tight[0], minlength=4)}, max level {int(got[1].max(initial=0))}",
              flush=True)
        prev = w.boxes[u]
    assert mix[FREE] + mix[COLLIDES] > 0
    g.close()


def test_validate_many_candidate_boxes(ctx):
    """A disc (r = 0.1) at offset (2, 0) turning about the origin in quarter
    turns: its arc (radius 2) is free of 600 tiny boxes scattered inside
    radius 1.75, but each quarter turn's capsule (chord 1.41 from the origin,
    radius 0.1 + pi^2/16) meets many of them, and the candidate region
    (chords widened by 0.1 + pi^2/8) holds more boxes than one LDS page.
    One more box straddles the arc at 45 degrees."""
    import math
    from paper_2603_28674_amd import rgg
    import oracle
    rob = synth.Robot(synth.SE2, np.array([[2.0, 0.0]]), np.array([0.1]))
    q = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, math.pi / 2], [0.0, 0.0, math.pi],
                  [0.0, 0.0, -math.pi / 2], [0.3, 0.0, 0.0]])
    edges = np.array([[0, 1], [1, 2], [2, 3], [3, 0], [0, 4], [4, 1]])
    rng = np.random.default_rng(32)
    ang = rng.uniform(0, 2 * math.pi, 600)
    rad = 1.75 * np.sqrt(rng.uniform(0, 1, 600))
    ctr = np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)
    side = rng.uniform(0.01, 0.03, (600, 1))
    boxes = np.zeros((601, 6))
    boxes[:600, :2] = ctr - side / 2
    boxes[:600, 3:5] = ctr + side / 2
    boxes[600] = [1.36, 1.36, 0.0, 1.46, 1.46, 0.0]
    reach = 0.1 + math.pi ** 2 / 8
    near = np.sum(np.all((boxes[:600, :2] <= 2.0 + reach) & (boxes[:600, 3:5] >= -reach), axis=1))
    assert near > 256
    print(f"[validate] paging: {near} boxes in the first quarter turn's candidate region", flush=True)
    g = rgg.Roadmap(ctx, rob, q, edges, len(boxes), samples_per_edge=2,
                    precision=rgg.RGG_PREC_FP32_RECHECK)
    o = oracle.Roadmap(rob, q, edges, 0.0, 2, len(boxes))
    absent = np.tile(synth.ABSENT_BOX, (len(boxes), 1))
    lab, gray, n, _ = g.update(absent, boxes)
    o.update(absent, boxes)
    ids = np.arange(len(edges))
    got = g.validate(ids)
    same(got, o.validate(ids), "paging")
    assert got[0][0] == COLLIDES and got[1][0] == 1 and got[2][0] == 0.5
    assert np.all(got[0][1:4] == FREE)
    print(f"[validate] paging: labels {lab.tolist()}, verdicts {got[0].tolist()}, levels {got[1].tolist()}",
          flush=True)
    g.close()


def test_validate_async_after_update(ctx):
    import torch
    from paper_2603_28674_amd import rgg
    import oracle
    w = workload("spatial", 2)
    print(f"[validate] async after update: E={w.n_edges}", flush=True)
    dev = torch.device("cuda:0")
    g = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK)
    o = oracle.from_workload(w)
    E = w.n_edges
    states = torch.from_numpy(np.stack([w.absent()] + w.boxes)).to(dev)
    labels = torch.zeros(E, dtype=torch.uint8, device=dev)
    gray = torch.zeros(E, dtype=torch.int64, device=dev)
    res = torch.zeros(rgg.RESULT_BYTES, dtype=torch.uint8, device=dev)
    ver = torch.full((E,), 77, dtype=torch.uint8, device=dev)
    lev = torch.full((E,), -7, dtype=torch.int32, device=dev)
    wit = torch.full((E,), -1.0, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    g.update_async(stream, states[0], states[1], labels, gray, res)
    rgg.rgg_validate_async(g.h, stream, gray, E, res, ver, lev, wit)
    torch.cuda.synchronize()
    r = rgg.result_from_tensor(res)
    assert r.status == 0
    n = r.n_gray
    _, og = o.update(w.absent(), w.boxes[0])
    assert n == len(og)
    same((ver[:n].cpu().numpy(), lev[:n].cpu().numpy(), wit[:n].cpu().numpy()), o.validate(og), "async")
    assert torch.all(ver[n:] == 77) and torch.all(lev[n:] == -7)
    # non-lazy labels: the validated gray edges become GREEN (FREE) or RED
    final = labels.clone()
    rgg.rgg_validate_async(g.h, stream, gray, E, res, ver, lev, wit, d_labels=final)
    torch.cuda.synchronize()
    before, after = labels.cpu().numpy(), final.cpu().numpy()
    ov = o.validate(og)[0]
    assert not np.any(after == 1), "a validated label stayed GRAY"
    assert np.array_equal(after[og], np.where(ov == FREE, 0, 2))
    rest = np.ones(E, dtype=bool)
    rest[og] = False
    assert np.array_equal(after[rest], before[rest])
    assert np.array_equal(g.labels(), before), "the roadmap keeps its RGG labels"
    # a failed update (stale `old`) validates nothing
    ver.fill_(77)
    g.update_async(stream, states[0], states[2], labels, gray, res)
    rgg.rgg_validate_async(g.h, stream, gray, E, res, ver, lev, wit)
    torch.cuda.synchronize()
    assert rgg.result_from_tensor(res).status == rgg.RGG_E_STATE_MISMATCH
    assert torch.all(ver == 77)
    # ids that are not edges
    ids = torch.tensor([-1, 0, E, E - 1], dtype=torch.int64, device=dev)
    rgg.rgg_validate_async(g.h, stream, ids, 4, None, ver, lev, wit)
    torch.cuda.synchronize()
    v = ver[:4].cpu().numpy()
    assert v[0] == BAD_ID and v[2] == BAD_ID and v[1] != BAD_ID and v[3] != BAD_ID
    ov, ol, ow = o.validate([0, E - 1])
    assert v[1] == ov[0] and v[3] == ov[1]
    g.close()


def test_validate_argument_errors(ctx):
    from paper_2603_28674_amd import rgg
    w = workload("planar", 1)
    g = rgg.Roadmap.from_workload(ctx, w)
    g.update(w.absent(), w.boxes[0])
    print("[validate] argument errors", flush=True)
    for bad in ([w.n_edges], [-1]):
        with pytest.raises(rgg.RggError) as ei:
            g.validate(bad)
        assert ei.value.status == rgg.RGG_E_INVALID_ARG
    with pytest.raises(rgg.RggError):
        g.validate([0], max_level=31)
    with pytest.raises(rgg.RggError):
        g.validate([0], max_active=513)
    v, lv, wt = g.validate(np.zeros(0, dtype=np.int64))
    assert v.size == 0
    g.close()


def test_validate_deep_searches(ctx):
    """Grazing contacts that take the search to level 21-28 (dyadic indices
    near 2^28), at several limits: verdicts, levels and witnesses equal the
    oracle's."""
    import math
    from paper_2603_28674_amd import rgg
    import oracle
    rob = synth.Robot(synth.SE2, np.array([[2.0, 0.0]]), np.array([0.1]))
    q = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, math.pi / 2]])
    edges = np.array([[0, 1]])
    print("[validate] deep searches", flush=True)
    for rc in (1.9, 1.9 - 1e-12, 1.9 + 1e-12, 1.9 - 1e-6):
        cx, cy = rc * math.cos(math.pi / 6), rc * math.sin(math.pi / 6)
        box = np.array([[cx - 0.3, cy - 0.3, 0.0, cx, cy, 0.0]])
        g = rgg.Roadmap(ctx, rob, q, edges, 1, samples_per_edge=2, precision=rgg.RGG_PREC_FP32_RECHECK)
        o = oracle.Roadmap(rob, q, edges, 0.0, 2, 1)
        absent = np.tile(synth.ABSENT_BOX, (1, 1))
        g.update(absent, box)
        o.update(absent, box)
        for ml, ma in ((30, 512), (30, 4), (24, 256), (16, 1)):
            got, want = g.validate([0], ml, ma), o.validate([0], ml, ma)
            same(got, want, f"corner radius {rc!r} limits {ml}/{ma}")
        print(f"[validate] corner {rc!r}: {got[0].tolist()} level {got[1].tolist()}", flush=True)
        g.close()
