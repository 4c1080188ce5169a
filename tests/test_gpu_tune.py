"""GPU tests of the work-decomposition autotuner (rgg_tune).

Tuning times every candidate (work-item size x grid cell size) on round
trips a -> b -> a, keeps the fastest, and must leave the roadmap exactly as
it was: the labels right after tuning, and after every later update, equal
the FP64 oracle's.  The tuner is refused while a graph or batch holds the
roadmap, and a stale `a` changes nothing."""
import numpy as np
import pytest

from paper_2603_28674_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2603_28674_amd import rgg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = rgg.rgg_context_create(0)
    yield c
    rgg.rgg_context_destroy(c)


def workload(kind, n_updates):
    if kind == "spatial":
        return synth.spatial_rigid(seed=41, n_nodes=3000, n_boxes=120, n_updates=n_updates, world=4.0)
    if kind == "planar":
        return synth.planar_rigid(seed=42, n_nodes=2000, n_boxes=50, n_updates=n_updates)
    return synth.planar_arm(seed=43, n_nodes=3000, n_boxes=60, n_updates=n_updates)


@pytest.mark.parametrize("kind", ["spatial", "planar", "arm"])
def test_tune_then_updates_match_oracle(ctx, kind):
    import oracle
    from paper_2603_28674_amd import rgg
    w = workload(kind, 5)
    print(f"[tune] {w.name} E={w.n_edges} M={w.n_slots}", flush=True)
    g = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK)
    o = oracle.from_workload(w)
    g.update(w.absent(), w.boxes[0])
    ol, og = o.update(w.absent(), w.boxes[0])
    rep = g.tune(w.boxes[0], w.boxes[1], reps=2)
    print(f"[tune] {w.name}: chose item_edges={rep['item_edges']} cell={rep['cell_size']} "
          f"{rep['us_per_update']:.1f} us (was {rep['us_before']:.1f})", flush=True)
    assert 10 <= rep["n_candidates"] <= rgg.TUNE_MAX_CANDIDATES
    assert all(c["us"] > 0.0 for c in rep["candidates"])
    assert rep["us_per_update"] <= rep["us_before"]
    assert 1 <= rep["item_edges"] <= 512
    info = g.info()
    assert info["item_edges"] == rep["item_edges"]
    # the state is unchanged: current labels and gray list are the oracle's
    assert np.array_equal(g.labels(), ol)
    gl, n = g.gray_list()
    assert n == len(og) and np.array_equal(gl, og)
    prev = w.boxes[0]
    for u in range(1, len(w.boxes)):
        ol, og = o.update(prev, w.boxes[u])
        lab, gray, n, r = g.update(prev, w.boxes[u])
        assert n == len(og) and np.array_equal(lab, ol) and np.array_equal(gray, og), f"update {u}"
        prev = w.boxes[u]
    g.close()


def test_tune_refusals_leave_state_unchanged(ctx):
    import torch
    from paper_2603_28674_amd import rgg
    w = workload("planar", 3)
    g = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK)
    g.update(w.absent(), w.boxes[0])
    before = g.labels()
    info0 = g.info()
    # a stale `a`
    with pytest.raises(rgg.RggError) as ei:
        g.tune(w.boxes[1], w.boxes[2])
    assert ei.value.status == rgg.RGG_E_STATE_MISMATCH
    # held by a batch, then by a graph
    b = rgg.rgg_batch_create(ctx, [g.h])
    with pytest.raises(rgg.RggError) as ei:
        g.tune(w.boxes[0], w.boxes[1])
    assert ei.value.status == rgg.RGG_E_BUSY
    rgg.rgg_batch_destroy(b)
    dev = torch.device("cuda:0")
    st = torch.from_numpy(np.stack([w.boxes[0], w.boxes[1]])).to(dev)
    lab = torch.zeros(w.n_edges, dtype=torch.uint8, device=dev)
    gr = torch.zeros(w.n_edges, dtype=torch.int64, device=dev)
    res = torch.zeros(rgg.RESULT_BYTES, dtype=torch.uint8, device=dev)
    req = rgg.rgg_update_req(g.h.value, w.n_slots, st[0].data_ptr(), st[1].data_ptr(),
                             lab.data_ptr(), gr.data_ptr(), w.n_edges, res.data_ptr())
    gh = rgg.rgg_graph_create(ctx, [req])
    with pytest.raises(rgg.RggError) as ei:
        g.tune(w.boxes[0], w.boxes[1])
    assert ei.value.status == rgg.RGG_E_BUSY
    rgg.rgg_graph_destroy(gh)
    info1 = g.info()
    assert info1["grid_cells"] == info0["grid_cells"] and info1["item_edges"] == info0["item_edges"]
    assert np.array_equal(g.labels(), before)
    # free again: tuning now runs
    rep = g.tune(w.boxes[0], w.boxes[1], reps=1)
    assert rep["n_candidates"] >= 10
    assert np.array_equal(g.labels(), before)
    g.close()


def test_tune_on_several_states(ctx):
    import oracle
    from paper_2603_28674_amd import rgg
    w = workload("arm", 6)
    g = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK)
    o = oracle.from_workload(w)
    g.update(w.absent(), w.boxes[0])
    ol, og = o.update(w.absent(), w.boxes[0])
    rep = g.tune(w.boxes[0], w.boxes[1:5], reps=1)
    assert rep["n_candidates"] >= 10
    assert np.array_equal(g.labels(), ol)
    lab, gray, n, _ = g.update(w.boxes[0], w.boxes[5])
    ol, og = o.update(w.boxes[0], w.boxes[5])
    assert np.array_equal(lab, ol) and np.array_equal(gray, og)
    with pytest.raises(rgg.RggError) as ei:      # a state with a NaN box
        bad = w.boxes[1].copy()
        bad[0, 0] = np.nan
        g.tune(w.boxes[5], [w.boxes[1], bad])
    assert ei.value.status == rgg.RGG_E_INVALID_ARG
    assert np.array_equal(g.labels(), ol)
    g.close()


def test_batch_tune_then_batched_updates_match_oracle(ctx):
    """One decomposition for a mixed batch (three robot kinds, both
    precisions), then batched updates, stream-launched and as the rebuilt
    captured graph, each equal to the oracle."""
    import oracle
    import torch
    from paper_2603_28674_amd import rgg
    n_updates = 5
    specs = [(workload("spatial", n_updates), rgg.RGG_PREC_FP32_RECHECK, -1.0),
             (workload("planar", n_updates), rgg.RGG_PREC_FP64, 0.0),
             (workload("arm", n_updates), rgg.RGG_PREC_FP32_RECHECK, 0.0),
             (synth.planar_rigid(seed=44, n_nodes=800, n_boxes=20, n_updates=n_updates),
              rgg.RGG_PREC_FP32_RECHECK, 0.0)]
    ws = [w for w, _, _ in specs]
    gs = [rgg.Roadmap.from_workload(ctx, w, precision=p, cell_size=c) for w, p, c in specs]
    os_ = [oracle.from_workload(w) for w in ws]
    dev = torch.device("cuda:0")
    bufs = [(torch.from_numpy(np.stack([w.absent()] + w.boxes)).to(dev),
             torch.zeros(w.n_edges, dtype=torch.uint8, device=dev),
             torch.zeros(w.n_edges, dtype=torch.int64, device=dev),
             torch.zeros(rgg.RESULT_BYTES, dtype=torch.uint8, device=dev)) for w in ws]
    stream = torch.cuda.current_stream().cuda_stream

    def reqs(u):
        return [rgg.rgg_update_req(g.h.value, w.n_slots, st[u].data_ptr(), st[u + 1].data_ptr(),
                                   lab.data_ptr(), gr.data_ptr(), w.n_edges, res.data_ptr())
                for w, g, (st, lab, gr, res) in zip(ws, gs, bufs)]

    def check(u):
        torch.cuda.synchronize()
        for k, (w, o, (_, lab, gr, res)) in enumerate(zip(ws, os_, bufs)):
            ol, og = o.update(w.absent() if u == 0 else w.boxes[u - 1], w.boxes[u])
            r = rgg.result_from_tensor(res)
            assert r.status == 0 and r.n_gray == len(og), f"update {u} roadmap {k}"
            assert np.array_equal(lab.cpu().numpy(), ol), f"update {u} roadmap {k}: labels"
            assert np.array_equal(gr[: r.n_gray].cpu().numpy(), og), f"update {u} roadmap {k}: gray"

    batch = rgg.rgg_batch_create(ctx, [g.h for g in gs])
    rgg.rgg_batch_launch(batch, reqs(0), stream)
    check(0)
    # another holder of a roadmap makes batch tuning refuse
    other = rgg.rgg_batch_create(ctx, [gs[0].h])
    with pytest.raises(rgg.RggError) as ei:
        rgg.rgg_batch_tune(batch, [w.boxes[0] for w in ws], [w.boxes[1] for w in ws])
    assert ei.value.status == rgg.RGG_E_BUSY
    rgg.rgg_batch_destroy(other)
    rep = rgg.rgg_batch_tune(batch, [w.boxes[0] for w in ws], [w.boxes[1] for w in ws], reps=2)
    print(f"[batch tune] item_edges={rep['item_edges']} factor={rep['cell_size']} "
          f"{rep['us_per_update']:.1f} us (was {rep['us_before']:.1f})", flush=True)
    assert rep["n_candidates"] >= 10 and rep["us_per_update"] <= rep["us_before"]
    for k, (g, o) in enumerate(zip(gs, os_)):   # state unchanged
        ol, _ = o.classify(ws[k].boxes[0])
        assert np.array_equal(g.labels(), ol), f"roadmap {k} after tuning"
    for u in range(1, n_updates):
        if u % 2:
            rgg.rgg_batch_launch(batch, reqs(u), stream)
        else:
            rgg.rgg_batch_launch_graph(batch, reqs(u), stream)
        check(u)
    rgg.rgg_batch_destroy(batch)
    for g in gs:
        g.close()
