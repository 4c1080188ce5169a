"""GPU parity: librgg's labels and gray lists equal the FP64 oracle's.

Every comparison is exact (labels are integers, gray lists are edge ids).
Sizes span several label tiles (4096 edges) with a ragged tail; sequences
start from the all-ABSENT state (Sec. 5: roadmaps are built without
obstacles), add the first obstacle set, then move obstacles (Sec. 5: random
translations), and include removals and re-additions through ABSENT.
"""
import numpy as np
import pytest

from paper_2603_28674_amd import synth
from neartangent import near_tangent_boxes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2603_28674_amd import rgg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = rgg.rgg_context_create(0)
    yield c
    rgg.rgg_context_destroy(c)


def workload(kind, n_updates=6, seed=None):
    if kind == "planar":
        return synth.planar_rigid(seed=seed or 11, n_nodes=2000, n_boxes=50, n_updates=n_updates)
    if kind == "spatial":
        return synth.spatial_rigid(seed=seed or 12, n_nodes=3000, n_boxes=120, n_updates=n_updates,
                                   world=4.0)
    if kind == "arm":
        return synth.planar_arm(seed=seed or 13, n_nodes=3000, n_boxes=60, n_updates=n_updates)
    raise ValueError(kind)


def with_removals(w, rng):
    """Appends states that remove some slots (ABSENT) and add them back."""
    last = w.boxes[-1].copy()
    rem = last.copy()
    idx = rng.choice(w.n_slots, size=max(1, w.n_slots // 5), replace=False)
    rem[idx] = synth.ABSENT_BOX
    back = rem.copy()
    back[idx[: len(idx) // 2]] = last[idx[: len(idx) // 2]]
    w.boxes = w.boxes + [rem, back]
    return w


def check_sequence(ctx, w, precision, cell_size=0.0, band_rel=0.0, device_buffers=False,
                   retest_capacity=0, item_edges=0, outer_obb=False, inner_splines=False, spline_tol=0.05,
                   pair_list_capacity=0, inline_rounds=0):
    import torch
    from paper_2603_28674_amd import rgg
    import oracle
    print(f"[parity] {w.name} E={w.n_edges} M={w.n_slots} precision={precision} "
          f"cell={cell_size} band={band_rel} device_buffers={device_buffers} "
          f"retest_capacity={retest_capacity} item_edges={item_edges} obb={outer_obb} "
          f"splines={inner_splines} tol={spline_tol} pair_list_capacity={pair_list_capacity} "
          f"inline_rounds={inline_rounds}", flush=True)
    g = rgg.Roadmap.from_workload(ctx, w, precision=precision, cell_size=cell_size,
                                  band_rel=band_rel, retest_capacity=retest_capacity,
                                  item_edges=item_edges, outer_obb=outer_obb,
                                  inner_splines=inner_splines, spline_tol=spline_tol,
                                  pair_list_capacity=pair_list_capacity, inline_rounds=inline_rounds)
    o = oracle.from_workload(w, outer_obb=outer_obb, inner_splines=inner_splines, spline_tol=spline_tol)
    prev = w.absent()
    stats = []
    if device_buffers:
        dev = torch.device("cuda:0")
        states = [torch.from_numpy(b.copy()).to(dev) for b in [prev] + w.boxes]
        labels = torch.zeros(w.n_edges, dtype=torch.uint8, device=dev)
        gray = torch.zeros(max(w.n_edges, 1), dtype=torch.int64, device=dev)
        res = torch.zeros(rgg.RESULT_BYTES, dtype=torch.uint8, device=dev)
        stream = torch.cuda.current_stream().cuda_stream
    for u, cur in enumerate(w.boxes):
        ol, og = o.update(prev, cur)
        if device_buffers:
            g.update_async(stream, states[u], states[u + 1], labels, gray, res)
            torch.cuda.synchronize()
            r = rgg.result_from_tensor(res)
            assert r.status == 0
            gl = labels.cpu().numpy()
            gg = gray[: r.n_gray].cpu().numpy()
            n = r.n_gray
        else:
            gl, gg, n, r = g.update(prev, cur)
        assert n == len(og), f"update {u}: n_gray {n} vs oracle {len(og)}"
        bad = np.nonzero(gl != ol)[0]
        assert bad.size == 0, f"update {u}: {bad.size} labels differ, first {bad[:10]}"
        assert np.array_equal(gg, og), f"update {u}: gray list differs"
        stats.append(r.as_dict())
        prev = cur
    # the library's own label query agrees with the last update
    assert np.array_equal(g.labels(), ol)
    gl2, n2 = g.gray_list()
    assert n2 == len(og) and np.array_equal(gl2, og)
    g.close()
    return stats


@pytest.mark.parametrize("kind", ["planar", "spatial", "arm"])
def test_parity_fp64(ctx, kind):
    from paper_2603_28674_amd import rgg
    w = with_removals(workload(kind), np.random.default_rng(1))
    stats = check_sequence(ctx, w, rgg.RGG_PREC_FP64)
    assert all(s["n_rechecked"] == 0 for s in stats)
    assert sum(s["n_pairs"] for s in stats) > 0


@pytest.mark.parametrize("kind", ["planar", "spatial", "arm"])
def test_parity_fp32_recheck(ctx, kind):
    from paper_2603_28674_amd import rgg
    w = with_removals(workload(kind), np.random.default_rng(2))
    stats = check_sequence(ctx, w, rgg.RGG_PREC_FP32_RECHECK)
    assert sum(s["n_pairs"] for s in stats) > 0


@pytest.mark.parametrize("cell_size", [-1.0, 0.0, 0.5, 3.0])
def test_grid_cell_size_does_not_change_labels(ctx, cell_size):
    from paper_2603_28674_amd import rgg
    w = workload("spatial", n_updates=3, seed=21)
    check_sequence(ctx, w, rgg.RGG_PREC_FP32_RECHECK, cell_size=cell_size)


@pytest.mark.parametrize("item_edges", [64, 200, 300, 482, 512])
@pytest.mark.parametrize("cell_size", [-1.0, 0.0])
@pytest.mark.parametrize("kind", ["spatial", "planar", "arm"])
def test_item_size_does_not_change_labels(ctx, kind, item_edges, cell_size):
    """Every work decomposition gives the oracle's labels, for each robot
    dimension: items of more than 256 edges use the second edge slot of each
    thread (482 is the arm's tuned one-cell size, 512 the batch's)."""
    from paper_2603_28674_amd import rgg
    w = with_removals(workload(kind, seed=31), np.random.default_rng(8))
    check_sequence(ctx, w, rgg.RGG_PREC_FP32_RECHECK, cell_size=cell_size, item_edges=item_edges)


@pytest.mark.parametrize("item_edges", [482, 512])
def test_item_size_fp64_planar_and_arm(ctx, item_edges):
    from paper_2603_28674_amd import rgg
    for kind in ("planar", "arm"):
        w = workload(kind, n_updates=3, seed=32)
        check_sequence(ctx, w, rgg.RGG_PREC_FP64, cell_size=-1.0, item_edges=item_edges)


def test_device_buffer_entry_point(ctx):
    from paper_2603_28674_amd import rgg
    w = workload("spatial", n_updates=4, seed=22)
    check_sequence(ctx, w, rgg.RGG_PREC_FP32_RECHECK, device_buffers=True)
    w = workload("planar", n_updates=3, seed=23)
    check_sequence(ctx, w, rgg.RGG_PREC_FP64, device_buffers=True)


def test_graph_entry_point(ctx):
    """rgg_graph_create: a chain of updates on one roadmap and an independent
    second roadmap in one graph; every output equals the oracle's."""
    import torch
    from paper_2603_28674_amd import rgg
    import oracle
    dev = torch.device("cuda:0")
    ws = [workload("spatial", n_updates=3, seed=31), workload("arm", n_updates=3, seed=32)]
    print(f"[graph] E={[w.n_edges for w in ws]}", flush=True)
    reqs, keep, outs = [], [], []
    gs = [rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK) for w in ws]
    for g, w in zip(gs, ws):
        states = torch.from_numpy(np.stack([w.absent()] + w.boxes)).to(dev)
        keep.append(states)
        per = []
        for u in range(len(w.boxes)):
            lab = torch.zeros(w.n_edges, dtype=torch.uint8, device=dev)
            gray = torch.zeros(w.n_edges, dtype=torch.int64, device=dev)
            res = torch.zeros(rgg.RESULT_BYTES, dtype=torch.uint8, device=dev)
            per.append((lab, gray, res))
            reqs.append(rgg.rgg_update_req(g.h.value, w.n_slots, states[u].data_ptr(),
                                           states[u + 1].data_ptr(), lab.data_ptr(), gray.data_ptr(),
                                           w.n_edges, res.data_ptr()))
        outs.append(per)
    graph = rgg.rgg_graph_create(ctx, reqs)
    rgg.rgg_graph_launch(graph, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    for w, per in zip(ws, outs):
        o = oracle.from_workload(w)
        prev = w.absent()
        for u, cur in enumerate(w.boxes):
            ol, og = o.update(prev, cur)
            lab, gray, res = per[u]
            r = rgg.result_from_tensor(res)
            assert r.status == 0 and r.n_gray == len(og)
            assert np.array_equal(lab.cpu().numpy(), ol)
            assert np.array_equal(gray[: r.n_gray].cpu().numpy(), og)
            prev = cur
    rgg.rgg_graph_destroy(graph)
    for g in gs:
        g.close()


def test_band_infinite_rechecks_every_decision(ctx):
    from paper_2603_28674_amd import rgg
    w = workload("spatial", n_updates=2, seed=24)
    stats = check_sequence(ctx, w, rgg.RGG_PREC_FP32_RECHECK, band_rel=float("inf"))
    assert all(s["n_rechecked"] == s["n_pairs"] for s in stats)


@pytest.mark.parametrize("kind", ["spatial", "planar"])
@pytest.mark.parametrize("pair_list_capacity,inline_rounds", [(0, 0), (0, -1), (1, -1), (64, -1), (0, 2)])
def test_full_retest_regions_defer_whole_items(ctx, kind, pair_list_capacity, inline_rounds):
    """With room for one re-test pair per block and every decision inside the
    band, blocks leave whole work items to the binary64 pass.  With room for
    one pair (or 64) in each listing block's pair list, the listing blocks
    test most rounds themselves (the fused path, deferring items and
    withdrawing their listed pairs); with no inline rounds (-1) the shares
    get every round that fits, with every round inline (0, the fused kernel)
    there are no shares.  The pairs of a deferred item count once whichever
    block listed or tested them."""
    from paper_2603_28674_amd import rgg
    w = workload(kind, n_updates=2, seed=26)
    stats = check_sequence(ctx, w, rgg.RGG_PREC_FP32_RECHECK, band_rel=float("inf"),
                           retest_capacity=1, pair_list_capacity=pair_list_capacity, inline_rounds=inline_rounds)
    assert all(s["n_rechecked"] == s["n_pairs"] > 0 for s in stats)


@pytest.mark.parametrize("kind", ["spatial", "planar", "arm"])
@pytest.mark.parametrize("inline_rounds", [-1, 1, 3])
def test_inline_rounds_do_not_change_labels(ctx, kind, inline_rounds):
    """However the pair rounds are split between the listing blocks and the
    balanced pair testing, labels and gray lists are the oracle's, and every
    pair is counted once."""
    from paper_2603_28674_amd import rgg
    w = with_removals(workload(kind, n_updates=3, seed=28), np.random.default_rng(6))
    stats = check_sequence(ctx, w, rgg.RGG_PREC_FP32_RECHECK, inline_rounds=inline_rounds)
    ref = check_sequence(ctx, w, rgg.RGG_PREC_FP32_RECHECK)   # every round inline
    assert [s["n_pairs"] for s in stats] == [s["n_pairs"] for s in ref]


@pytest.mark.parametrize("kind", ["spatial", "arm"])
@pytest.mark.parametrize("pair_list_capacity", [1, 100])
def test_pair_list_capacity_does_not_change_labels(ctx, kind, pair_list_capacity):
    """Pair lists too small for the items: rounds that do not fit are tested
    by the listing blocks themselves; labels do not change."""
    from paper_2603_28674_amd import rgg
    w = with_removals(workload(kind, n_updates=3, seed=27), np.random.default_rng(5))
    check_sequence(ctx, w, rgg.RGG_PREC_FP32_RECHECK, pair_list_capacity=pair_list_capacity,
                   inline_rounds=rgg.RGG_INLINE_NONE)


@pytest.mark.parametrize("kind", ["planar", "arm"])
def test_band_infinite_other_robots(ctx, kind):
    """Every pair through the binary64 re-test, for the planar rigid body and
    the arm."""
    from paper_2603_28674_amd import rgg
    w = workload(kind, n_updates=2, seed=26)
    stats = check_sequence(ctx, w, rgg.RGG_PREC_FP32_RECHECK, band_rel=float("inf"))
    assert all(s["n_rechecked"] == s["n_pairs"] > 0 for s in stats)


@pytest.mark.parametrize("kind", ["spatial", "planar", "arm"])
def test_band_near_tangent(ctx, kind):
    """Near-tangent boxes: with the default band every label equals the
    oracle's (the undecided tests went to binary64).  With a band far below
    the rounding error (1e-12) the same inputs give wrong labels, so they do
    reach the cases the band has to cover."""
    from paper_2603_28674_amd import rgg
    import oracle
    w = workload(kind, n_updates=1, seed=41)
    o = oracle.from_workload(w)
    # an arm edge sweeps a large area: few boxes keep labels other than RED
    n_near = 4 if kind == "arm" else w.n_slots
    boxes = w.absent()
    boxes[:n_near] = near_tangent_boxes(o, w, np.random.default_rng(7), n_near)
    w.boxes = [boxes]
    stats = check_sequence(ctx, w, rgg.RGG_PREC_FP32_RECHECK)
    assert stats[0]["n_rechecked"] > 0
    ol, _ = oracle.from_workload(w).update(w.absent(), w.boxes[0])
    g = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK, band_rel=1e-12)
    lab, _, _, _ = g.update(w.absent(), w.boxes[0])
    g.close()
    bad = int(np.count_nonzero(lab != ol))
    print(f"[teeth] {kind}: {bad} labels differ with band 1e-12", flush=True)
    assert bad > 0


def test_errors_leave_state_unchanged(ctx):
    from paper_2603_28674_amd import rgg
    import oracle
    w = workload("planar", n_updates=2, seed=25)
    print(f"[errors] E={w.n_edges}", flush=True)
    g = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP64)
    lab0, gray0, n0, _ = g.update(w.absent(), w.boxes[0])
    # stale `old`
    with pytest.raises(rgg.RggError) as ei:
        g.update(w.absent(), w.boxes[1])
    assert ei.value.status == rgg.RGG_E_STATE_MISMATCH
    assert np.array_equal(g.labels(), lab0)
    # non-finite box
    bad = w.boxes[1].copy()
    bad[3, 1] = np.nan
    with pytest.raises(rgg.RggError) as ei:
        g.update(w.boxes[0], bad)
    assert ei.value.status == rgg.RGG_E_INVALID_ARG
    assert np.array_equal(g.labels(), lab0)
    # wrong slot count
    with pytest.raises(rgg.RggError):
        g.update(w.boxes[0][:-1], w.boxes[1][:-1])
    # gray capacity: committed, partial list, status CAPACITY
    o = oracle.from_workload(w)
    o.update(w.absent(), w.boxes[0])
    ol, og = o.update(w.boxes[0], w.boxes[1])
    lab, gray, n, _ = g.update(w.boxes[0], w.boxes[1], gray_cap=3)
    assert n == len(og) and np.array_equal(gray, og[:3])
    assert np.array_equal(lab, ol)
    g.close()


def test_empty_and_degenerate(ctx):
    from paper_2603_28674_amd import rgg
    import oracle
    rng = np.random.default_rng(5)
    rob = synth.robot_se2(rng)
    q = synth.nodes_se2(rng, 50, 20.0)
    print("[empty] no edges", flush=True)
    g = rgg.Roadmap(ctx, rob, q, np.zeros((0, 2), dtype=np.int64), 3, resolution=0.1)
    boxes = synth.random_boxes(rng, 3, 2, 1.0, 3.0, 0.0, 20.0)
    lab, gray, n, _ = g.update(np.tile(synth.ABSENT_BOX, (3, 1)), boxes)
    assert lab.size == 0 and n == 0
    g.close()
    print("[empty] no slots", flush=True)
    edges = synth.knn_se2(q, 4)
    g = rgg.Roadmap(ctx, rob, q, edges, 0, resolution=0.1)
    lab, gray, n, _ = g.update(np.zeros((0, 6)), np.zeros((0, 6)))
    assert np.all(lab == 0) and n == 0
    g.close()
    print("[degenerate] duplicated nodes, box over everything, box far away", flush=True)
    q2 = np.concatenate([q, q])
    e2 = np.concatenate([edges, np.stack([np.arange(50), np.arange(50) + 50], axis=1)])
    big = np.array([[-100, -100, 0, 200, 200, 0], [500, 500, 0, 501, 501, 0]], dtype=float)
    g = rgg.Roadmap(ctx, rob, q2, e2, 2, resolution=0.1)
    o = oracle.Roadmap(rob, q2, e2, 0.1, 0, 2)
    lab, gray, n, _ = g.update(np.tile(synth.ABSENT_BOX, (2, 1)), big)
    ol, og = o.update(np.tile(synth.ABSENT_BOX, (2, 1)), big)
    assert np.array_equal(lab, ol) and np.all(lab == 2) and n == 0
    g.close()


@pytest.mark.parametrize("case", ["se3_64_spheres_4096_slots", "arm_32_links_64_spheres"])
def test_maximum_sizes(ctx, case):
    """The largest robot (64 spheres, one wavefront of lanes per edge), the
    longest arm (32 links) and the most obstacle slots (4096): labels, gray
    lists and the full validation of the gray list equal the oracle's."""
    from paper_2603_28674_amd import rgg
    import oracle
    rng = np.random.default_rng(91)
    if case.startswith("se3"):
        rob = synth.robot_se3(rng, n_spheres=64)
        q = synth.nodes_se3(rng, 600, 4.0)
        edges = synth.knn_se3(q, 6)
        M = 4096
        seq = [synth.random_boxes(rng, M, 3, 0.02, 0.1, -12.0, 16.0)]
        res, spe = 0.0, 12
    else:
        L = 32
        lengths = rng.uniform(0.1, 0.3, size=L)
        along = np.concatenate([[0.25 * l, 0.75 * l] for l in lengths])
        link = np.repeat(np.arange(L, dtype=np.int32), 2)
        rad = np.repeat(lengths / 4.0, 2)
        rob = synth.Robot(synth.ARM, along, rad, link, lengths, (0.0, 0.0))
        q = rng.uniform(-0.3, 0.3, size=(500, L))
        edges = synth.knn_euclid(q, 6)
        M = 30
        rho = float(lengths.sum())
        seq = [synth.random_boxes(rng, M, 2, 0.1, 0.5, -rho, rho)]
        res, spe = 0.0, 10
    for _ in range(2):
        nxt = seq[-1].copy()
        k = rng.choice(M, size=max(1, M // 10), replace=False)
        nxt[k, :rob.dim] += rng.normal(0, 0.2, (len(k), rob.dim))
        nxt[k, 3:3 + rob.dim] = nxt[k, :rob.dim] + (seq[-1][k, 3:3 + rob.dim] - seq[-1][k, :rob.dim])
        seq.append(nxt)
    print(f"[max] {case}: B={rob.n_spheres} E={len(edges)} M={M}", flush=True)
    g = rgg.Roadmap(ctx, rob, q, edges, M, resolution=res, samples_per_edge=spe,
                    precision=rgg.RGG_PREC_FP32_RECHECK)
    o = oracle.Roadmap(rob, q, edges, res, spe, M)
    prev = np.tile(synth.ABSENT_BOX, (M, 1))
    for u, cur in enumerate(seq):
        lab, gray, n, _ = g.update(prev, cur)
        ol, og = o.update(prev, cur)
        assert np.array_equal(lab, ol), f"update {u}: labels differ"
        assert np.array_equal(gray, og), f"update {u}: gray list differs"
        got, want = g.validate(gray), o.validate(og)
        assert all(np.array_equal(x, y, equal_nan=True) for x, y in zip(got, want)), f"update {u}: validation"
        print(f"[max] update {u}: labels {np.bincount(lab, minlength=3).tolist()}, "
              f"verdicts {np.bincount(got[0], minlength=4).tolist()}", flush=True)
        prev = cur
    g.close()


def test_roadmap_admission_by_device_memory(ctx):
    """mem_budget admits a roadmap only when its arrays fit: the exact size
    it ends up holding is admitted, one byte less is refused before
    anything is allocated."""
    import torch
    from paper_2603_28674_amd import rgg
    w = workload("spatial", n_updates=1, seed=61)
    for mode in (dict(), dict(outer_obb=True, inner_splines=True)):
        g = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK, **mode)
        need = g.info()["device_bytes"]
        g.close()
        torch.cuda.synchronize()
        before = torch.cuda.mem_get_info()[0]
        with pytest.raises(rgg.RggError) as ei:
            rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK, mem_budget=need - 1, **mode)
        assert ei.value.status == rgg.RGG_E_OUT_OF_MEMORY
        assert torch.cuda.mem_get_info()[0] == before
        g = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK, mem_budget=need, **mode)
        assert g.info()["device_bytes"] == need
        g.close()


@pytest.mark.parametrize("precision,inline_rounds", [(1, 0), (1, -1), (0, 0)])
def test_stage_timing(ctx, precision, inline_rounds):
    """Per-update stage timing: every timed update is counted, the item
    kernel's stage takes time in its slot (FP32: ms[2], with the pair
    testing in ms[3] when pairs are listed; FP64: ms[3]), and the timed
    updates still give the oracle's labels."""
    from paper_2603_28674_amd import rgg
    import oracle
    w = workload("spatial", n_updates=3, seed=29)
    print(f"[timing] precision={precision} inline_rounds={inline_rounds}", flush=True)
    g = rgg.Roadmap.from_workload(ctx, w, precision=precision, inline_rounds=inline_rounds)
    o = oracle.from_workload(w)
    rgg.rgg_timing_enable(g.h, True)
    prev = w.absent()
    for cur in w.boxes:
        gl, gg, n, r = g.update(prev, cur)
        ol, og = o.update(prev, cur)
        assert np.array_equal(gl, ol) and np.array_equal(gg, og)
        prev = cur
    ms, n = rgg.rgg_timing_read(g.h)
    assert n == len(w.boxes) and ms[0] > 0 and ms[5] > 0
    if precision == rgg.RGG_PREC_FP64:
        assert ms[3] > 0
    else:
        assert ms[2] > 0 and ms[4] > 0
        assert r.item_bytes > 0 and (r.test_bytes - r.item_bytes - r.fp64_bytes > 0) == (inline_rounds != 0)
    ms, n = rgg.rgg_timing_read(g.h)
    assert n == 0 and not ms.any()
    g.close()
