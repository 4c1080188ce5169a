"""GPU parity at the workloads' full sizes, in the launch configurations the
benchmark times (device buffers, one stream; the planar batch through
rgg_batch_launch).

The oracle cannot classify every edge of a 300k-edge roadmap against every
update in a test's time, so it classifies a seeded sample of edge ids (the
oracle's result for an edge depends on that edge alone, Sec. 4.2), and the
GPU's labels must equal its labels on the sample, bit for bit.  Properties
that hold at any size are checked on every edge: labels are 0, 1 or 2, the
gray list is exactly the ascending list of GRAY edge ids and n_gray its
length.
"""
import numpy as np
import pytest

from paper_2603_28674_amd import synth

pytestmark = pytest.mark.gpu

GREEN, GRAY, RED = 0, 1, 2


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2603_28674_amd import rgg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = rgg.rgg_context_create(0)
    yield c
    rgg.rgg_context_destroy(c)


def sample_oracle(w, n_sample, seed):
    import oracle
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(w.n_edges, size=min(n_sample, w.n_edges), replace=False))
    o = oracle.Roadmap(w.robot, w.q, w.edges[idx], w.resolution, w.samples_per_edge, w.n_slots)
    return idx, o


def check_whole(labels, gray, n_gray):
    assert labels.min() >= GREEN and labels.max() <= RED
    want = np.nonzero(labels == GRAY)[0]
    assert n_gray == len(want), f"n_gray {n_gray} vs {len(want)} GRAY labels"
    assert np.array_equal(gray[:n_gray], want), "gray list is not the GRAY edges in order"


FULL = {
    # name: (generator, precision, cell size, edges per item): the work
    # decompositions the benchmark's autotuner settles on for each workload
    # (one cell; 288-, 64- and 482-edge items), plus the heuristic grid
    "spatial_fp32": (lambda n: synth.spatial_rigid(n_updates=n), "fp32", -1.0, 288),
    "planar_fp64": (lambda n: synth.planar_rigid(n_updates=n), "fp64", -1.0, 64),
    "arm_fp32": (lambda n: synth.planar_arm(n_updates=n), "fp32", -1.0, 482),
    "arm_fp32_grid": (lambda n: synth.planar_arm(n_updates=n), "fp32", 0.0, 256),
}


@pytest.mark.parametrize("name", list(FULL))
def test_full_size_sampled(ctx, name):
    import torch
    from paper_2603_28674_amd import rgg
    gen, prec, cell, item = FULL[name]
    n_updates = 3
    w = gen(n_updates)
    precision = rgg.RGG_PREC_FP32_RECHECK if prec == "fp32" else rgg.RGG_PREC_FP64
    print(f"[full] {name} E={w.n_edges} M={w.n_slots} cell={cell} item_edges={item}", flush=True)
    idx, o = sample_oracle(w, 4000, seed=len(name))
    dev = torch.device("cuda:0")
    g = rgg.Roadmap.from_workload(ctx, w, precision=precision, cell_size=cell, item_edges=item)
    states = torch.from_numpy(np.stack([w.absent()] + w.boxes)).to(dev)
    labels = torch.zeros(w.n_edges, dtype=torch.uint8, device=dev)
    gray = torch.zeros(w.n_edges, dtype=torch.int64, device=dev)
    res = torch.zeros(rgg.RESULT_BYTES, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    prev = w.absent()
    for u in range(n_updates):
        g.update_async(stream, states[u], states[u + 1], labels, gray, res)
        torch.cuda.synchronize()
        r = rgg.result_from_tensor(res)
        assert r.status == 0
        gl = labels.cpu().numpy()
        check_whole(gl, gray.cpu().numpy(), r.n_gray)
        ol, _ = o.update(prev, w.boxes[u])
        bad = np.nonzero(gl[idx] != ol)[0]
        assert bad.size == 0, f"update {u}: {bad.size} sampled labels differ, edges {idx[bad[:10]]}"
        print(f"[full] {name} update {u}: gray {r.n_gray}, pairs {r.n_pairs}, "
              f"rechecked {r.n_rechecked}, sample mix "
              f"{np.bincount(ol, minlength=3).tolist()}", flush=True)
        if u == n_updates - 1:
            # full validation of the whole gray list, chained on the device
            # after the update; the sampled gray edges against the oracle
            n = r.n_gray
            ver = torch.zeros(max(n, 1), dtype=torch.uint8, device=dev)
            lev = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
            wit = torch.zeros(max(n, 1), dtype=torch.float64, device=dev)
            rgg.rgg_validate_async(g.h, stream, gray, n, res, ver, lev, wit)
            torch.cuda.synchronize()
            gids = gray[:n].cpu().numpy()
            pos = np.nonzero(np.isin(idx, gids))[0]            # sampled edges that are gray
            at = np.searchsorted(gids, idx[pos])
            ov, olv, ow = o.validate(pos)
            gv, glv, gw = ver.cpu().numpy()[at], lev.cpu().numpy()[at], wit.cpu().numpy()[at]
            assert np.array_equal(gv, ov) and np.array_equal(glv, olv)
            assert np.array_equal(gw, ow, equal_nan=True)
            print(f"[full] {name} validation: {n} gray -> verdicts "
                  f"{np.bincount(ver[:n].cpu().numpy(), minlength=4).tolist()}, "
                  f"{len(pos)} sampled match the oracle", flush=True)
        prev = w.boxes[u]
    g.close()


def test_full_size_planar_batch_sampled(ctx):
    """The 64-roadmap planar batch, updated twice through one batch launch
    per round."""
    import torch
    from paper_2603_28674_amd import rgg
    n_rounds = 2
    ws = synth.batch_of_planar(seed=3, n_updates=n_rounds)
    print(f"[full] planar batch: {len(ws)} roadmaps, {sum(w.n_edges for w in ws)} edges", flush=True)
    dev = torch.device("cuda:0")
    # the batch's tuned decomposition: 512-edge items, cells of twice the mean
    # edge extent (the build's default cell)
    gs = [rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK, cell_size=0.0, item_edges=512)
          for w in ws]
    bufs = []
    for w in ws:
        bufs.append((torch.from_numpy(np.stack([w.absent()] + w.boxes)).to(dev),
                     torch.zeros(w.n_edges, dtype=torch.uint8, device=dev),
                     torch.zeros(w.n_edges, dtype=torch.int64, device=dev),
                     torch.zeros(rgg.RESULT_BYTES, dtype=torch.uint8, device=dev)))
    samples = [sample_oracle(w, 300, seed=100 + k) for k, w in enumerate(ws)]
    batch = rgg.rgg_batch_create(ctx, [g.h for g in gs])
    stream = torch.cuda.current_stream().cuda_stream
    for u in range(n_rounds):
        reqs = [rgg.rgg_update_req(g.h.value, w.n_slots, st[u].data_ptr(), st[u + 1].data_ptr(),
                                   lab.data_ptr(), gr.data_ptr(), w.n_edges, res.data_ptr())
                for w, g, (st, lab, gr, res) in zip(ws, gs, bufs)]
        rgg.rgg_batch_launch(batch, reqs, stream)
        torch.cuda.synchronize()
        for k, (w, (_, lab, gr, res), (idx, o)) in enumerate(zip(ws, bufs, samples)):
            r = rgg.result_from_tensor(res)
            assert r.status == 0
            gl = lab.cpu().numpy()
            check_whole(gl, gr.cpu().numpy(), r.n_gray)
            ol, _ = o.update(w.absent() if u == 0 else w.boxes[u - 1], w.boxes[u])
            bad = np.nonzero(gl[idx] != ol)[0]
            assert bad.size == 0, f"round {u} roadmap {k}: {bad.size} sampled labels differ"
        print(f"[full] planar batch round {u} ok", flush=True)
    rgg.rgg_batch_destroy(batch)
    for g in gs:
        g.close()
