"""GPU parity of batched updates: every roadmap of a batch gets exactly the
labels and gray list of the FP64 oracle, after every batched update.

A batch mixes robot kinds (planar rigid, spatial rigid, planar arm), both
precisions, one-cell and grid roadmaps, and roadmaps of very different sizes,
as the batched configuration of many planar roadmaps does."""
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


def mixed_workloads(n_updates):
    from paper_2603_28674_amd import rgg
    fp32, fp64 = rgg.RGG_PREC_FP32_RECHECK, rgg.RGG_PREC_FP64
    specs = [
        (synth.planar_rigid(seed=51, n_nodes=1500, n_boxes=40, n_updates=n_updates), fp32, -1.0),
        (synth.spatial_rigid(seed=52, n_nodes=2500, n_boxes=100, n_updates=n_updates, world=4.0), fp32, -1.0),
        (synth.planar_arm(seed=53, n_nodes=2000, n_boxes=40, n_updates=n_updates), fp32, 0.0),
        (synth.planar_rigid(seed=54, n_nodes=300, n_boxes=20, n_updates=n_updates), fp64, -1.0),
        (synth.spatial_rigid(seed=55, n_nodes=1200, n_boxes=60, n_updates=n_updates, world=3.0), fp32, 0.0),
        (synth.planar_rigid(seed=56, n_nodes=80, n_boxes=5, n_updates=n_updates), fp32, -1.0),
    ]
    return specs


def run_batched(ctx, specs, n_updates, one_shot=False, item_edges=0, **build):
    import torch
    from paper_2603_28674_amd import rgg
    import oracle
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    gs, ors, bufs = [], [], []
    for w, prec, cell in specs:
        print(f"[batch] {w.name} E={w.n_edges} M={w.n_slots} prec={prec} cell={cell}", flush=True)
        gs.append(rgg.Roadmap.from_workload(ctx, w, precision=prec, cell_size=cell, item_edges=item_edges, **build))
        ors.append(oracle.from_workload(w))
        states = torch.from_numpy(np.stack([w.absent()] + w.boxes)).to(dev)
        lab = torch.zeros(w.n_edges, dtype=torch.uint8, device=dev)
        gray = torch.zeros(max(w.n_edges, 1), dtype=torch.int64, device=dev)
        res = torch.zeros(rgg.RESULT_BYTES, dtype=torch.uint8, device=dev)
        bufs.append((states, lab, gray, res))
    batch = None if one_shot else rgg.rgg_batch_create(ctx, [g.h for g in gs])
    for u in range(n_updates):
        reqs = []
        for (w, _, _), g, (states, lab, gray, res) in zip(specs, gs, bufs):
            reqs.append(rgg.rgg_update_req(g.h.value, w.n_slots, states[u].data_ptr(), states[u + 1].data_ptr(),
                                           lab.data_ptr(), gray.data_ptr(), w.n_edges, res.data_ptr()))
        if one_shot:
            rgg.rgg_update_batch(ctx, reqs, stream)
        elif u % 2:
            rgg.rgg_batch_launch_graph(batch, reqs, stream)   # the captured-graph form
        else:
            rgg.rgg_batch_launch(batch, reqs, stream)
        torch.cuda.synchronize()
        for k, ((w, _, _), o, (states, lab, gray, res)) in enumerate(zip(specs, ors, bufs)):
            prev = w.absent() if u == 0 else w.boxes[u - 1]
            ol, og = o.update(prev, w.boxes[u])
            r = rgg.result_from_tensor(res)
            assert r.status == 0, f"roadmap {k} update {u}: status {r.status}"
            assert r.n_gray == len(og), f"roadmap {k} update {u}: n_gray {r.n_gray} vs {len(og)}"
            gl = lab.cpu().numpy()
            bad = np.nonzero(gl != ol)[0]
            assert bad.size == 0, f"roadmap {k} update {u}: {bad.size} labels differ"
            assert np.array_equal(gray[: r.n_gray].cpu().numpy(), og), f"roadmap {k} update {u}: gray list"
    if batch is not None:
        rgg.rgg_batch_destroy(batch)
    for g in gs:
        g.close()


def test_batch_mixed_parity(ctx):
    run_batched(ctx, mixed_workloads(4), 4)


def test_update_batch_one_shot(ctx):
    run_batched(ctx, mixed_workloads(2)[:3], 2, one_shot=True)


def test_batch_many_planar(ctx):
    """Twenty planar roadmaps of 60..3000 nodes in one batch."""
    from paper_2603_28674_amd import rgg
    rng = np.random.default_rng(57)
    specs = []
    for k in range(20):
        n = int(round(np.exp(rng.uniform(np.log(60), np.log(3000)))))
        specs.append((synth.planar_rigid(seed=600 + k, n_nodes=n, n_boxes=int(rng.integers(5, 40)), n_updates=3),
                      rgg.RGG_PREC_FP32_RECHECK, -1.0))
    run_batched(ctx, specs, 3)


@pytest.mark.parametrize("item_edges", [482, 512])
def test_batch_planar_tuned_decomposition(ctx, item_edges):
    """The decomposition the planar batch is tuned to: items of 512 edges (the
    second edge slot of every thread) over grid cells of twice the mean edge
    extent (the build's default cell), plus one-cell roadmaps with the same
    items."""
    from paper_2603_28674_amd import rgg
    rng = np.random.default_rng(59)
    specs = []
    for k in range(12):
        n = int(round(np.exp(rng.uniform(np.log(300), np.log(6000)))))
        specs.append((synth.planar_rigid(seed=700 + k, n_nodes=n, n_boxes=int(rng.integers(20, 120)), n_updates=3,
                                         k=8), rgg.RGG_PREC_FP32_RECHECK, 0.0 if k % 3 else -1.0))
    run_batched(ctx, specs, 3, item_edges=item_edges)


@pytest.mark.parametrize("band_rel,retest_capacity", [(0.0, 0), (0.0, 4), (float("inf"), 2)])
def test_batch_claimed_items(ctx, band_rel, retest_capacity):
    """More work items than the batched item kernel's blocks take statically
    (two for each of its 1,024 blocks): seven one-cell planar roadmaps of
    about 28,000 edges in 64-edge items, about 3,050 items, every one of them
    work in every update.  Blocks claim the rest one at a time and come back
    to roadmaps they visited, so re-test regions continue across visits.  A
    re-test capacity of 4 pairs fills some regions; an infinite band with 2
    pairs leaves nearly every item whole to the binary64 pass (its list of
    deferred items); an FP64 roadmap rides along in its own group."""
    from paper_2603_28674_amd import rgg
    specs = [(synth.planar_rigid(seed=800 + k, n_nodes=6000, n_boxes=60, n_updates=3, k=8),
              rgg.RGG_PREC_FP32_RECHECK, -1.0) for k in range(7)]
    specs.append((synth.planar_rigid(seed=810, n_nodes=1500, n_boxes=40, n_updates=3, k=8), rgg.RGG_PREC_FP64, -1.0))
    assert sum((w.n_edges + 63) // 64 for w, p, _ in specs if p == rgg.RGG_PREC_FP32_RECHECK) > 2 * 1024
    run_batched(ctx, specs, 3, item_edges=64, band_rel=band_rel, retest_capacity=retest_capacity)


def test_batch_errors(ctx):
    from paper_2603_28674_amd import rgg
    w = synth.planar_rigid(seed=58, n_nodes=200, n_boxes=5, n_updates=1)
    print("[batch errors]", flush=True)
    g = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK)
    with pytest.raises(rgg.RggError):
        rgg.rgg_batch_create(ctx, [g.h, g.h])   # a roadmap twice
    b = rgg.rgg_batch_create(ctx, [g.h])
    with pytest.raises(rgg.RggError):
        # m does not match the roadmap
        rgg.rgg_batch_launch(b, [rgg.rgg_update_req(g.h.value, w.n_slots + 1, 1, 1, 0, 0, 0, 1)], 0)
    rgg.rgg_batch_destroy(b)
    g.close()


def test_batch_stage_timing(ctx):
    """Stage timing of batched launches: every timed launch is counted, the
    item stage takes time, and the results are still the oracle's."""
    import torch
    from paper_2603_28674_amd import rgg
    import oracle
    dev = torch.device("cuda:0")
    specs = mixed_workloads(3)[:3]
    gs = [rgg.Roadmap.from_workload(ctx, w, precision=p, cell_size=c) for w, p, c in specs]
    ors = [oracle.from_workload(w) for w, _, _ in specs]
    b = rgg.rgg_batch_create(ctx, [g.h for g in gs])
    rgg.rgg_batch_timing_enable(b, True)
    stream = torch.cuda.current_stream().cuda_stream
    bufs = []
    for w, _, _ in specs:
        states = torch.from_numpy(np.stack([w.absent()] + w.boxes)).to(dev)
        bufs.append((states, torch.zeros(w.n_edges, dtype=torch.uint8, device=dev),
                     torch.zeros(w.n_edges, dtype=torch.int64, device=dev),
                     torch.zeros(rgg.RESULT_BYTES, dtype=torch.uint8, device=dev)))
    for u in range(3):
        reqs = [rgg.rgg_update_req(g.h.value, w.n_slots, st[u].data_ptr(), st[u + 1].data_ptr(), lab.data_ptr(),
                                   gr.data_ptr(), w.n_edges, res.data_ptr())
                for (w, _, _), g, (st, lab, gr, res) in zip(specs, gs, bufs)]
        rgg.rgg_batch_launch(b, reqs, stream)
        torch.cuda.synchronize()
        for (w, _, _), o, (st, lab, gr, res) in zip(specs, ors, bufs):
            ol, og = o.update(w.absent() if u == 0 else w.boxes[u - 1], w.boxes[u])
            assert np.array_equal(lab.cpu().numpy(), ol)
    ms, n = rgg.rgg_batch_timing_read(b)
    assert n == 3 and ms[0] > 0 and ms[3] > 0 and ms[5] > 0 and ms[2] == 0
    ms, n = rgg.rgg_batch_timing_read(b)
    assert n == 0 and not ms.any()
    rgg.rgg_batch_destroy(b)
    for g in gs:
        g.close()


def test_batch_graph_ring_wraps(ctx):
    """Ten graph launches in a row, past the eight ring slots (each slot has
    its own graph, whose first node copies that slot's host rows): every
    update is the oracle's, with and without a stream synchronisation
    between launches."""
    import torch
    from paper_2603_28674_amd import rgg
    import oracle
    dev = torch.device("cuda:0")
    specs = mixed_workloads(10)[:3]
    gs = [rgg.Roadmap.from_workload(ctx, w, precision=p, cell_size=c) for w, p, c in specs]
    ors = [oracle.from_workload(w) for w, _, _ in specs]
    b = rgg.rgg_batch_create(ctx, [g.h for g in gs])
    stream = torch.cuda.current_stream().cuda_stream
    bufs = []
    for w, _, _ in specs:
        states = torch.from_numpy(np.stack([w.absent()] + w.boxes)).to(dev)
        # one label / gray / result buffer per update, so pipelined launches
        # do not overwrite what is checked afterwards
        bufs.append((states, torch.zeros((10, w.n_edges), dtype=torch.uint8, device=dev),
                     torch.zeros((10, w.n_edges), dtype=torch.int64, device=dev),
                     torch.zeros((10, rgg.RESULT_BYTES), dtype=torch.uint8, device=dev)))
    print("[batch graph ring] 10 launches", flush=True)
    for u in range(10):
        reqs = [rgg.rgg_update_req(g.h.value, w.n_slots, st[u].data_ptr(), st[u + 1].data_ptr(), lab[u].data_ptr(),
                                   gr[u].data_ptr(), w.n_edges, res[u].data_ptr())
                for (w, _, _), g, (st, lab, gr, res) in zip(specs, gs, bufs)]
        rgg.rgg_batch_launch_graph(b, reqs, stream)
        if u % 3 == 2:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    for u in range(10):
        for (w, _, _), o, (st, lab, gr, res) in zip(specs, ors, bufs):
            ol, og = o.update(w.absent() if u == 0 else w.boxes[u - 1], w.boxes[u])
            r = rgg.result_from_tensor(res[u])
            assert r.status == 0 and r.n_gray == len(og), f"update {u}"
            assert np.array_equal(lab[u].cpu().numpy(), ol), f"update {u}: labels"
            assert np.array_equal(gr[u][: r.n_gray].cpu().numpy(), og), f"update {u}: gray list"
    rgg.rgg_batch_destroy(b)
    for g in gs:
        g.close()
