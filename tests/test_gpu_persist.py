"""GPU tests of persistence (rgg_save / rgg_load) and of node labels.

Sec. 1 and Sec. 4.3 keep the approximations between planning iterations:
a roadmap read back from a file must hold the same labels and gray list as
the one saved, and every later update of either must equal the FP64
oracle's.  Sec. 3.1 treats a node as an edge whose two ends coincide: an
edge (v, v) carries node v's label, is never gray (its inner and outer
approximations are the same spheres) and, because every edge's samples
include its end configurations, a RED node makes every incident edge RED.
"""
import os

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


def workload(kind, n_updates):
    if kind == "planar":
        return synth.planar_rigid(seed=41, n_nodes=1500, n_boxes=40, n_updates=n_updates)
    if kind == "spatial":
        return synth.spatial_rigid(seed=42, n_nodes=2500, n_boxes=100, n_updates=n_updates, world=4.0)
    return synth.planar_arm(seed=43, n_nodes=2000, n_boxes=50, n_updates=n_updates)


CASES = [
    # kind, precision, cell size, edges per item, tune before saving
    ("planar", "fp64", 0.0, 0, False),
    ("spatial", "fp32", -1.0, 288, False),
    ("spatial", "fp32", 0.0, 0, True),
    ("arm", "fp32", 0.0, 128, False),
]


@pytest.mark.parametrize("kind,prec,cell,item_edges,tune", CASES)
def test_save_load_round_trip(ctx, tmp_path, kind, prec, cell, item_edges, tune):
    from paper_2603_28674_amd import rgg
    import oracle
    n_updates = 5
    w = workload(kind, n_updates)
    precision = rgg.RGG_PREC_FP32_RECHECK if prec == "fp32" else rgg.RGG_PREC_FP64
    print(f"[persist] {w.name} E={w.n_edges} {prec} cell={cell} item_edges={item_edges} tune={tune}",
          flush=True)
    g = rgg.Roadmap.from_workload(ctx, w, precision=precision, cell_size=cell, item_edges=item_edges)
    o = oracle.from_workload(w)
    prev = w.absent()
    for u in range(2):
        g.update(prev, w.boxes[u])
        o.update(prev, w.boxes[u])
        prev = w.boxes[u]
    if tune:
        g.tune(prev, w.boxes[2:4], reps=1)
    path = tmp_path / "roadmap.rgg"
    g.save(path)
    h = rgg.Roadmap.load(ctx, path)
    a, b = g.info(), h.info()
    for key in ("n_edges", "n_slots", "dim", "n_spheres", "n_sphere_samples", "grid_cells", "cell_size",
                "grid_entries", "item_edges"):
        assert a[key] == b[key], f"info {key}: {a[key]} vs {b[key]}"
    assert np.array_equal(g.labels(), h.labels())
    (ga, na), (gb, nb) = g.gray_list(), h.gray_list()
    assert na == nb and np.array_equal(ga, gb)
    # the full validation reads the stored robot and motions
    ids = np.arange(0, w.n_edges, 7)
    va, vb = g.validate(ids), h.validate(ids)
    assert all(np.array_equal(x, y, equal_nan=True) for x, y in zip(va, vb))
    for u in range(2, n_updates):
        ol, og = o.update(prev, w.boxes[u])
        for name, r in (("saved", g), ("loaded", h)):
            lab, gray, n, res = r.update(prev, w.boxes[u])
            assert res.status == 0
            assert np.array_equal(lab, ol), f"{name} update {u}: labels differ from the oracle"
            assert n == len(og) and np.array_equal(gray, og), f"{name} update {u}: gray list differs"
        prev = w.boxes[u]
    # a file written by the loaded roadmap reads back to the same state again
    path2 = tmp_path / "again.rgg"
    h.save(path2)
    k = rgg.Roadmap.load(ctx, path2)
    assert np.array_equal(k.labels(), h.labels())
    g.close()
    h.close()
    k.close()


def test_load_rejects_bad_files(ctx, tmp_path):
    from paper_2603_28674_amd import rgg
    w = workload("planar", 1)
    print("[persist] bad files", flush=True)
    g = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK)
    g.update(w.absent(), w.boxes[0])
    path = tmp_path / "good.rgg"
    g.save(path)
    raw = path.read_bytes()

    def rejected(data, name):
        p = tmp_path / name
        p.write_bytes(data)
        with pytest.raises(rgg.RggError) as ei:
            rgg.rgg_load(ctx, p)
        assert ei.value.status == rgg.RGG_E_INVALID_ARG, name

    rejected(b"", "empty")
    rejected(raw[: len(raw) // 2], "truncated")
    rejected(raw[:-1], "short_checksum")
    flipped = bytearray(raw)
    flipped[len(raw) // 3] ^= 0x10
    rejected(bytes(flipped), "flipped")
    rejected(b"NOTAMAP!" + raw[8:], "magic")
    version = bytearray(raw)
    version[8] ^= 0x02
    rejected(bytes(version), "version")
    with pytest.raises(rgg.RggError):
        rgg.rgg_load(ctx, tmp_path / "missing.rgg")
    with pytest.raises(rgg.RggError):
        g.save(tmp_path / "no_such_dir" / "x.rgg")
    # a roadmap held by a batch is not saved
    batch = rgg.rgg_batch_create(ctx, [g.h])
    with pytest.raises(rgg.RggError) as ei:
        g.save(tmp_path / "held.rgg")
    assert ei.value.status == rgg.RGG_E_BUSY
    rgg.rgg_batch_destroy(batch)
    g.save(tmp_path / "released.rgg")
    assert os.path.getsize(tmp_path / "released.rgg") == len(raw)
    g.close()


@pytest.mark.parametrize("kind", ["planar", "spatial", "arm"])
def test_node_labels(ctx, kind):
    """Edges (v, v) appended to a roadmap carry the node labels."""
    from paper_2603_28674_amd import rgg
    import oracle
    n_updates = 3
    w = workload(kind, n_updates)
    n_nodes = w.q.shape[0]
    E = w.n_edges
    w.edges = np.concatenate([w.edges, np.stack([np.arange(n_nodes)] * 2, axis=1)])
    print(f"[nodes] {w.name} E={E} nodes={n_nodes}", flush=True)
    g = rgg.Roadmap.from_workload(ctx, w, precision=rgg.RGG_PREC_FP32_RECHECK, cell_size=0.0)
    o = oracle.from_workload(w)
    prev = w.absent()
    for u in range(n_updates):
        lab, gray, n, res = g.update(prev, w.boxes[u])
        ol, og = o.update(prev, w.boxes[u])
        assert np.array_equal(lab, ol) and np.array_equal(gray, og)
        node = lab[E:]
        assert not np.any(node == GRAY), "a node is never gray"
        red_nodes = np.nonzero(node == RED)[0]
        inc = np.isin(w.edges[:E, 0], red_nodes) | np.isin(w.edges[:E, 1], red_nodes)
        assert np.all(lab[:E][inc] == RED), "an edge at a RED node is RED"
        print(f"[nodes] update {u}: {red_nodes.size} red nodes, {int(inc.sum())} edges at them", flush=True)
        prev = w.boxes[u]
    g.close()


def _fnv1a64(data):
    h = 14695981039346656037
    for b in data:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def test_load_rejects_inconsistent_contents(ctx, tmp_path):
    """Files whose checksum is right but whose contents contradict each other
    (header dimension, sample offsets, robot kind) are refused."""
    import struct
    from paper_2603_28674_amd import rgg
    w = synth.planar_rigid(seed=44, n_nodes=60, n_boxes=5, n_updates=1, resolution=0.5)
    g = rgg.Roadmap.from_workload(ctx, w)
    g.update(w.absent(), w.boxes[0])
    path = tmp_path / "small.rgg"
    g.save(path)
    g.close()
    raw = bytearray(path.read_bytes())
    assert struct.unpack_from("<Q", raw, len(raw) - 8)[0] == _fnv1a64(raw[:-8])
    print(f"[persist] {len(raw)} bytes", flush=True)
    D, B = struct.unpack_from("<ii", raw, 12)
    E, M = struct.unpack_from("<qq", raw, 32)
    n_samp, n_cap = struct.unpack_from("<qq", raw, 64)
    hdr = 80
    robot_at = hdr + 8 * (E + 1) + 8 * n_samp + 8 * n_cap + 8 * B + 32 * E + 48 * M + 8 * E

    def refused(mutate, name):
        data = bytearray(raw)
        mutate(data)
        struct.pack_into("<Q", data, len(data) - 8, _fnv1a64(data[:-8]))
        p = tmp_path / name
        p.write_bytes(bytes(data))
        with pytest.raises(rgg.RggError) as ei:
            rgg.rgg_load(ctx, p)
        assert ei.value.status == rgg.RGG_E_INVALID_ARG, name

    assert (D, B) == (2, 4) and struct.unpack_from("<i", raw, robot_at)[0] == 0   # an SE2 robot record
    refused(lambda d: struct.pack_into("<i", d, 12, 3), "dimension")
    refused(lambda d: struct.pack_into("<q", d, hdr + 8, -4), "offsets")
    refused(lambda d: struct.pack_into("<i", d, robot_at, 1), "robot_kind")
    refused(lambda d: struct.pack_into("<i", d, robot_at + 4, B + 1), "robot_spheres")
    # the unmodified bytes with a recomputed checksum still load
    p = tmp_path / "same.rgg"
    p.write_bytes(bytes(raw))
    h = rgg.Roadmap.load(ctx, p)
    h.close()
