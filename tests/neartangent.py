"""Near-tangent obstacle boxes: inputs that put an edge's decisive distance
test within rounding of its threshold (shared by the CPU pins of the oracle
and the GPU band tests)."""
import numpy as np


def near_tangent_boxes(o, w, rng, n_boxes):
    """Small boxes, each just beyond the extreme point of one edge's swept
    robot along one axis: one face at distance r (1 + eps) from the extreme
    sphere copy, or at R (1 + eps) from the extreme capsule axis end (R =
    capsule radius), |eps| log-uniform in [1e-9, 1e-3] with a random sign.
    Each box puts one edge's decisive distance test at or inside binary32
    rounding of its threshold."""
    D = w.robot.dim
    rad = w.robot.sphere_radius
    out = np.zeros((n_boxes, 6))
    for b in range(n_boxes):
        e = int(rng.integers(w.n_edges))
        cen = o.centres(e)                      # [J, B, D]
        ax = int(rng.integers(D))
        side = float(rng.choice([-1.0, 1.0]))
        eps = float(rng.choice([-1.0, 1.0]) * 10.0 ** rng.uniform(-9.0, -3.0))
        if rng.random() < 0.5:
            reach = side * cen[:, :, ax] + rad[None, :]
            j, i = np.unravel_index(int(np.argmax(reach)), reach.shape)
            p = cen[j, i]
            dist = rad[i] * (1.0 + eps)
        else:
            R = o.capsule_radius(e)
            ends = np.stack([cen[0], cen[-1]])  # [2, B, D]
            reach = side * ends[:, :, ax] + R[None, :]
            j, i = np.unravel_index(int(np.argmax(reach)), reach.shape)
            p = ends[j, i]
            dist = R[i] * (1.0 + eps)
        face = p[ax] + side * dist
        depth = rng.uniform(0.01, 0.1)
        lo = np.zeros(3)
        hi = np.zeros(3)
        for k in range(D):
            if k == ax:
                lo[k], hi[k] = (face, face + depth) if side > 0 else (face - depth, face)
            else:
                lo[k] = p[k] - rng.uniform(0.01, 0.1)
                hi[k] = p[k] + rng.uniform(0.01, 0.1)
        out[b, :3], out[b, 3:] = lo, hi
    return out
