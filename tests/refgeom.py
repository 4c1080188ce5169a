"""Reference geometry for the tests, written independently of the oracle:
rotation matrices, scipy's Rotation and Slerp, and cumulative sums for the
planar chain.  Used to check the oracle's forward kinematics and to run dense
brute-force collision checks of the continuous edge motion."""
import math

import numpy as np
from scipy.spatial.transform import Rotation, Slerp

from paper_2603_28674_amd import synth


def fk_se2_ref(rob, q):
    c, s = math.cos(q[2]), math.sin(q[2])
    R = np.array([[c, -s], [s, c]])
    return q[:2] + rob.sphere_pos @ R.T


def fk_se3_ref(rob, p, rot):
    return p + rot.apply(rob.sphere_pos)


def fk_arm_ref(rob, q):
    phi = np.cumsum(q)
    L = rob.link_length
    jx = np.concatenate([[rob.base[0]], rob.base[0] + np.cumsum(L * np.cos(phi))])
    jy = np.concatenate([[rob.base[1]], rob.base[1] + np.cumsum(L * np.sin(phi))])
    m = rob.sphere_link
    return np.stack([jx[m] + rob.sphere_pos * np.cos(phi[m]),
                     jy[m] + rob.sphere_pos * np.sin(phi[m])], axis=1)



def centre_path(rob, qa, qb, ts):
    """Sphere centres (T, B, D) along the continuous edge motion at times ts."""
    kind = rob.kind
    if kind == synth.SE2:
        dth = (qb[2] - qa[2] + math.pi) % (2 * math.pi) - math.pi
        return np.stack([fk_se2_ref(rob, np.r_[qa[:2] + t * (qb[:2] - qa[:2]), qa[2] + t * dth])
                         for t in ts])
    if kind == synth.SE3:
        rots = Rotation.from_quat([np.r_[qa[4:], qa[3]], np.r_[qb[4:], qb[3]]])
        sl = Slerp([0.0, 1.0], rots)(ts)
        return np.stack([fk_se3_ref(rob, qa[:3] + t * (qb[:3] - qa[:3]), sl[k])
                         for k, t in enumerate(ts)])
    return np.stack([fk_arm_ref(rob, qa + t * (qb - qa)) for t in ts])




def box_d2(c, box, D):
    lo, hi = box[:D], box[3:3 + D]
    return np.sum((c - np.clip(c, lo, hi)) ** 2, axis=-1)
