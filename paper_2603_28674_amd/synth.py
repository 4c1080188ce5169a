"""Seeded synthetic workloads for Red-Green-Gray edge classification.

This module draws the inputs that both the FP64 oracle and the device path
consume: a robot made of spheres, roadmap nodes, k-nearest-neighbour edges,
axis-aligned box obstacles and sequences of obstacle moves.  It holds none of
the classification arithmetic (no forward kinematics, no interpolation, no
distance tests); it only produces arrays.

The paper evaluates on PRMs built without obstacles (Sec. 5, mobile-robot
setup) and on random obstacle translations between updates (Sec. 5,
introduction of the experiments).  Its environments and robot models are not
available, so the workloads below are synthetic stand-ins with the shapes and
distributions stated for each configuration.

Box rows are float64 arrays of six numbers ``lo_x lo_y lo_z hi_x hi_y hi_z``.
A box with ``lo_k > hi_k`` on any axis is ABSENT.  Planar workloads set the
z entries to zero.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
from scipy.spatial import cKDTree

SE2, SE3, ARM = 0, 1, 2

#: Canonical ABSENT box: every slot of a freshly built roadmap holds it.
ABSENT_BOX = np.array([1.0, 1.0, 1.0, -1.0, -1.0, -1.0], dtype=np.float64)


@dataclasses.dataclass
class Robot:
    kind: int
    sphere_pos: np.ndarray          # SE2 (B,2) / SE3 (B,3) body offsets; ARM (B,) along-link distance
    sphere_radius: np.ndarray       # (B,)
    sphere_link: Optional[np.ndarray] = None   # ARM (B,) int32
    link_length: Optional[np.ndarray] = None   # ARM (L,)
    base: tuple = (0.0, 0.0)

    @property
    def n_spheres(self) -> int:
        return int(self.sphere_radius.shape[0])

    @property
    def n_links(self) -> int:
        return 0 if self.link_length is None else int(self.link_length.shape[0])

    @property
    def dim(self) -> int:
        """Workspace dimension D."""
        return 3 if self.kind == SE3 else 2

    @property
    def dof(self) -> int:
        return {SE2: 3, SE3: 7}.get(self.kind, self.n_links)


@dataclasses.dataclass
class Workload:
    name: str
    robot: Robot
    q: np.ndarray                  # (N, dof) float64
    edges: np.ndarray              # (E, 2) int64, u < v, sorted
    resolution: float              # C-space step for SE2 sampling
    samples_per_edge: int          # > 0 fixes the sample count (SE3, ARM)
    boxes: List[np.ndarray]        # boxes[0]: first obstacle set; boxes[u]: state after update u
    world_lo: np.ndarray
    world_hi: np.ndarray

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    @property
    def n_slots(self) -> int:
        return int(self.boxes[0].shape[0])

    def absent(self) -> np.ndarray:
        return np.tile(ABSENT_BOX, (self.n_slots, 1))


# --------------------------------------------------------------------------
# robots
# --------------------------------------------------------------------------

def robot_se2(rng: np.random.Generator, n_spheres: int = 4) -> Robot:
    """Planar rigid body of disks: radii U[0.2,0.5], offsets U[-1,1]^2."""
    pos = rng.uniform(-1.0, 1.0, size=(n_spheres, 2))
    rad = rng.uniform(0.2, 0.5, size=n_spheres)
    return Robot(SE2, pos, rad)


def robot_se3(rng: np.random.Generator, n_spheres: int = 8) -> Robot:
    """Spatial rigid body of spheres: radii U[0.05,0.2], offsets U[-0.5,0.5]^3."""
    pos = rng.uniform(-0.5, 0.5, size=(n_spheres, 3))
    rad = rng.uniform(0.05, 0.2, size=n_spheres)
    return Robot(SE3, pos, rad)


def robot_arm(rng: np.random.Generator, n_links: int = 7) -> Robot:
    """Planar serial arm, base at the origin, link lengths U[0.5,1.5].

    Each link carries three spheres at 1/6, 1/2 and 5/6 of its length with
    radius length/6, so the spheres tile the link's centre line.
    """
    lengths = rng.uniform(0.5, 1.5, size=n_links)
    along, link, rad = [], [], []
    for m, ell in enumerate(lengths):
        for f in (1.0 / 6.0, 0.5, 5.0 / 6.0):
            along.append(f * ell)
            link.append(m)
            rad.append(ell / 6.0)
    return Robot(ARM, np.array(along), np.array(rad), np.array(link, dtype=np.int32),
                 lengths, (0.0, 0.0))


# --------------------------------------------------------------------------
# nodes and k-nearest-neighbour edges (PRM built without obstacles)
# --------------------------------------------------------------------------

def _undirected(nbr: np.ndarray) -> np.ndarray:
    n, k = nbr.shape
    u = np.repeat(np.arange(n, dtype=np.int64), k)
    v = nbr.reshape(-1).astype(np.int64)
    keep = u != v
    a = np.minimum(u[keep], v[keep])
    b = np.maximum(u[keep], v[keep])
    key = np.unique(a * n + b)
    return np.stack([key // n, key % n], axis=1).astype(np.int64)


def nodes_se2(rng, n, world):
    xy = rng.uniform(0.0, world, size=(n, 2))
    th = rng.uniform(-math.pi, math.pi, size=(n, 1))
    return np.concatenate([xy, th], axis=1)


def knn_se2(q: np.ndarray, k: int) -> np.ndarray:
    """kNN under sqrt(dx^2 + dy^2 + dtheta^2) with theta wrapped to (-pi, pi]."""
    two_pi = 2.0 * math.pi
    th = np.mod(q[:, 2] + math.pi, two_pi)
    th = np.where(th >= two_pi, 0.0, th)
    span = float(np.max(np.abs(q[:, :2]))) * 4.0 + 1.0
    pts = np.stack([q[:, 0], q[:, 1], th], axis=1)
    pts[:, :2] -= np.min(pts[:, :2], axis=0)
    tree = cKDTree(pts, boxsize=[span, span, two_pi])
    _, idx = tree.query(pts, k=k + 1)
    return _undirected(idx[:, 1:])


def nodes_se3(rng, n, world):
    p = rng.uniform(0.0, world, size=(n, 3))
    quat = rng.normal(size=(n, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    return np.concatenate([p, quat], axis=1)        # x y z qw qx qy qz


def knn_se3(q: np.ndarray, k: int) -> np.ndarray:
    """kNN under sqrt(|dp|^2 + 4 min(|qa-qb|^2, |qa+qb|^2)).

    The quaternion chord distance (both signs, since q and -q are the same
    rotation) makes the metric Euclidean in an embedding, so a k-d tree
    answers it.
    """
    n = q.shape[0]
    emb = np.concatenate([np.concatenate([q[:, :3], 2.0 * q[:, 3:]], axis=1),
                          np.concatenate([q[:, :3], -2.0 * q[:, 3:]], axis=1)], axis=0)
    tree = cKDTree(emb)
    _, idx = tree.query(emb[:n], k=2 * k + 2)
    idx = idx % n
    nbr = np.empty((n, k), dtype=np.int64)
    for i in range(n):
        row = idx[i]
        seen = []
        for j in row:
            if j != i and j not in seen:
                seen.append(int(j))
                if len(seen) == k:
                    break
        while len(seen) < k:
            seen.append(i)
        nbr[i] = seen
    return _undirected(nbr)


def nodes_arm(rng, n, n_links):
    return rng.uniform(-math.pi, math.pi, size=(n, n_links))


def knn_euclid(q: np.ndarray, k: int) -> np.ndarray:
    tree = cKDTree(q)
    _, idx = tree.query(q, k=k + 1)
    return _undirected(idx[:, 1:])


# --------------------------------------------------------------------------
# obstacles
# --------------------------------------------------------------------------

def random_boxes(rng, m, dim, side_lo, side_hi, c_lo, c_hi) -> np.ndarray:
    side = rng.uniform(side_lo, side_hi, size=(m, dim))
    ctr = rng.uniform(c_lo, c_hi, size=(m, dim))
    out = np.zeros((m, 6))
    out[:, :dim] = ctr - 0.5 * side
    out[:, 3:3 + dim] = ctr + 0.5 * side
    return out


def move_sequence(rng, boxes0, dim, n_updates, n_move, sigma) -> List[np.ndarray]:
    """boxes[0] = boxes0; every later state translates ``n_move`` distinct
    slots of the previous one by independent N(0, sigma) offsets per axis."""
    seq = [boxes0.copy()]
    cur = boxes0.copy()
    m = boxes0.shape[0]
    for _ in range(n_updates):
        nxt = cur.copy()
        cnt = n_move if isinstance(n_move, int) else int(rng.integers(n_move[0], n_move[1] + 1))
        cnt = min(cnt, m)
        slots = rng.choice(m, size=cnt, replace=False)
        off = rng.normal(0.0, sigma, size=(cnt, dim))
        nxt[slots, :dim] += off
        nxt[slots, 3:3 + dim] += off
        seq.append(nxt)
        cur = nxt
    return seq


# --------------------------------------------------------------------------
# the workload configurations
# --------------------------------------------------------------------------

def planar_rigid(seed: int = 1, n_nodes: int = 2000, k: int = 10, n_boxes: int = 50,
                 n_updates: int = 8, n_move=5, world: float = 100.0,
                 resolution: float = 0.05) -> Workload:
    """Planar rigid robot of 4 disks in a 100 x 100 workspace; PRM of uniform
    (x, y, theta) nodes with k-NN edges; boxes with sides U[1,5]; each update
    translates ``n_move`` boxes by N(0, 2) per axis."""
    rng = np.random.default_rng(seed)
    rob = robot_se2(rng)
    q = nodes_se2(rng, n_nodes, world)
    edges = knn_se2(q, k)
    b0 = random_boxes(rng, n_boxes, 2, 1.0, 5.0, 0.0, world)
    seq = move_sequence(rng, b0, 2, n_updates, n_move, 2.0)
    return Workload("planar_rigid", rob, q, edges, resolution, 0, seq,
                    np.zeros(3), np.array([world, world, 0.0]))


def spatial_rigid(seed: int = 2, n_nodes: int = 50000, k: int = 10, n_boxes: int = 500,
                  n_updates: int = 8, move_frac: float = 0.1, world: float = 10.0,
                  samples: int = 20) -> Workload:
    """Spatial rigid robot of 8 spheres in a 10^3 workspace; 50k nodes
    (position + unit quaternion), k-NN edges, 20 samples per edge; 500 boxes
    with sides U[0.2,1.5]; each update translates 10% of them by N(0, 0.3)."""
    rng = np.random.default_rng(seed)
    rob = robot_se3(rng)
    q = nodes_se3(rng, n_nodes, world)
    edges = knn_se3(q, k)
    b0 = random_boxes(rng, n_boxes, 3, 0.2, 1.5, 0.0, world)
    seq = move_sequence(rng, b0, 3, n_updates, max(1, int(round(move_frac * n_boxes))), 0.3)
    return Workload("spatial_rigid", rob, q, edges, 0.0, samples, seq,
                    np.zeros(3), np.array([world] * 3))


def planar_arm(seed: int = 4, n_nodes: int = 100000, k: int = 8, n_boxes: int = 300,
               n_updates: int = 8, n_move: int = 30, n_links: int = 7,
               samples: int = 20) -> Workload:
    """Planar 7-link revolute arm (joint limits [-pi, pi]); k-NN edges in joint
    space; 300 boxes with sides U[0.3,2] centred in [-6 rho, 6 rho]^2 where rho
    is the arm's reach; each update translates 30 boxes by N(0, 2)."""
    rng = np.random.default_rng(seed)
    rob = robot_arm(rng, n_links)
    q = nodes_arm(rng, n_nodes, n_links)
    edges = knn_euclid(q, k)
    rho = float(np.sum(rob.link_length))
    b0 = random_boxes(rng, n_boxes, 2, 0.3, 2.0, -6.0 * rho, 6.0 * rho)
    seq = move_sequence(rng, b0, 2, n_updates, n_move, 2.0)
    return Workload("planar_arm", rob, q, edges, 0.0, samples, seq,
                    np.array([-6 * rho, -6 * rho, 0.0]), np.array([6 * rho, 6 * rho, 0.0]))


def batch_of_planar(seed: int = 3, n_roadmaps: int = 64, n_lo: int = 1000, n_hi: int = 100000,
                    k: int = 8, n_updates: int = 4, resolution: float = 0.05) -> List[Workload]:
    """Many independent planar roadmaps: node counts log-uniform in
    [n_lo, n_hi], box counts U{20..400}, each update moves U{1..20} boxes."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_roadmaps):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        m = int(rng.integers(20, 401))
        sub = int(rng.integers(0, 2 ** 31 - 1))
        w = planar_rigid(seed=sub, n_nodes=n, k=k, n_boxes=m, n_updates=n_updates,
                         n_move=(1, 20), resolution=resolution)
        w.name = f"planar_batch_{r}"
        out.append(w)
    return out


def serving_mix(seed: int = 5, n_spatial: int = 8, n_arm: int = 8, e_lo: float = 1e4,
                e_hi: float = 5e5) -> List[Workload]:
    """Resident roadmaps of the serving configuration: spatial rigid-body and
    planar-arm roadmaps whose edge counts are log-uniform in [e_lo, e_hi]
    (node counts from the edges per node that k = 10 and k = 8 give: about
    5.9 and 4.6).  Each carries only its first obstacle set; the requests'
    moves are drawn by ``serving_requests``."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_spatial + n_arm):
        e = math.exp(rng.uniform(math.log(e_lo), math.log(e_hi)))
        if k < n_spatial:
            out.append(spatial_rigid(seed=int(rng.integers(1 << 30)), n_nodes=max(200, int(e / 5.9)),
                                     n_updates=0))
        else:
            out.append(planar_arm(seed=int(rng.integers(1 << 30)), n_nodes=max(200, int(e / 4.6)),
                                  n_updates=0))
    return out


def serving_requests(rng: np.random.Generator, workloads: List[Workload], rate: float, duration: float,
                     max_move: int = 50, start: Optional[List[np.ndarray]] = None):
    """Open-loop Poisson arrivals at ``rate`` per second for ``duration``
    seconds; each request moves U{1..max_move} boxes of a uniformly chosen
    roadmap (N(0, 0.3) per axis for spatial roadmaps, N(0, 2) for arms),
    starting from that roadmap's current state (``start``, else its first
    obstacle set).  Returns a list of (arrival_time, roadmap_index,
    old_boxes, new_boxes) and the final states."""
    cur = [b.copy() for b in start] if start is not None else [w.boxes[0].copy() for w in workloads]
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        r = int(rng.integers(len(workloads)))
        w = workloads[r]
        dim = w.robot.dim
        sigma = 0.3 if w.robot.kind == SE3 else 2.0
        nxt = move_sequence(rng, cur[r], dim, 1, (1, max_move), sigma)[1]
        out.append((t, r, cur[r], nxt))
        cur[r] = nxt
    return out, cur

