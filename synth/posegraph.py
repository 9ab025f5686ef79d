"""Seeded synthetic pose graphs (the paper's second workload, PGO, Sec. IV-D).

The paper's PGO benchmarks (sphere-a: 2,500 poses / 9,799 edges, and
parking-garage) are not available here; these graphs stand in for them with
the structure of a sphere trajectory: `rings` rings of `per_ring` poses on a
sphere of radius 10, odometry edges between consecutive poses and
loop-closure edges from each pose to the poses of the previous ring at the
nearest angles.  Measurements are the ground-truth relative poses perturbed
by Exp(eps), eps ~ N(0, diag(sigma_t^2 I, sigma_r^2 I)); the information
matrix is the inverse of that covariance.  The initial estimate composes the
noisy odometry from the fixed first pose (dead reckoning), as a front end
would.  Poses are [tx ty tz qx qy qz qw] (scalar-last unit quaternion); the
generator uses scipy for rotations and the matrix exponential, and shares
no arithmetic with the oracle or the GPU library."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg
from scipy.spatial.transform import Rotation

__all__ = ["PoseGraph", "make_pose_graph", "to_matrix", "from_matrix", "se3_exp"]


@dataclass
class PoseGraph:
    n_poses: int
    ei: np.ndarray        # int32 [m]
    ej: np.ndarray        # int32 [m]
    T: np.ndarray         # [m, 7] measured relative poses zeta_i^-1 zeta_j
    omega: np.ndarray     # [m, 6, 6] information matrices
    poses_gt: np.ndarray  # [n, 7]
    poses0: np.ndarray    # [n, 7] initial estimate
    fixed: np.ndarray     # int32 indices of fixed poses

    @property
    def n_edges(self) -> int:
        return int(self.ei.size)


def to_matrix(p) -> np.ndarray:
    M = np.eye(4)
    M[:3, :3] = Rotation.from_quat(p[3:7]).as_matrix()
    M[:3, 3] = p[:3]
    return M


def from_matrix(M) -> np.ndarray:
    q = Rotation.from_matrix(M[:3, :3]).as_quat()
    if q[3] < 0:
        q = -q
    return np.concatenate([M[:3, 3], q])


def se3_exp(xi) -> np.ndarray:
    """Exp of xi = (rho, phi) as the matrix exponential of its 4x4 twist."""
    rho, phi = np.asarray(xi[:3], float), np.asarray(xi[3:], float)
    X = np.zeros((4, 4))
    X[:3, :3] = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    X[:3, 3] = rho
    return scipy.linalg.expm(X)


def make_pose_graph(seed: int = 0, rings: int = 50, per_ring: int = 50, radius: float = 10.0,
                    sigma_t: float = 0.05, sigma_r: float = 0.01, loop_k: int = 3,
                    noise: bool = True) -> PoseGraph:
    rng = np.random.default_rng([7, seed])
    n = rings * per_ring
    gt = np.zeros((n, 4, 4))
    for r in range(rings):
        el = np.pi * (r + 0.5) / rings - np.pi / 2
        for k in range(per_ring):
            az = 2 * np.pi * k / per_ring + 0.1 * r
            c = radius * np.array([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)])
            # heading along the ring, z axis outward
            zax = c / np.linalg.norm(c)
            xax = np.array([-np.sin(az), np.cos(az), 0.0])
            yax = np.cross(zax, xax)
            M = np.eye(4)
            M[:3, :3] = np.stack([xax, yax, zax], axis=1)
            M[:3, 3] = c
            gt[r * per_ring + k] = M
    edges = [(a, a + 1) for a in range(n - 1)]
    for r in range(1, rings):
        for k in range(per_ring):
            a = r * per_ring + k
            # the loop_k poses of the previous ring nearest in azimuth
            for d in range(loop_k):
                kk = (k + d - loop_k // 2) % per_ring
                b = (r - 1) * per_ring + kk
                if b != a - 1:
                    edges.append((b, a))
    ei = np.array([e[0] for e in edges], np.int32)
    ej = np.array([e[1] for e in edges], np.int32)
    m = ei.size
    cov = np.diag([sigma_t ** 2] * 3 + [sigma_r ** 2] * 3)
    omega = np.broadcast_to(np.linalg.inv(cov), (m, 6, 6)).copy()
    T = np.zeros((m, 7))
    Tm = np.zeros((m, 4, 4))
    for e in range(m):
        rel = np.linalg.inv(gt[ei[e]]) @ gt[ej[e]]
        if noise:
            eps = np.concatenate([rng.normal(size=3) * sigma_t, rng.normal(size=3) * sigma_r])
            rel = se3_exp(eps) @ rel
        Tm[e] = rel
        T[e] = from_matrix(rel)
    # dead reckoning along the odometry chain from the first pose
    init = np.zeros((n, 4, 4))
    init[0] = gt[0]
    for a in range(n - 1):
        init[a + 1] = init[a] @ Tm[a]
    poses_gt = np.stack([from_matrix(M) for M in gt])
    poses0 = np.stack([from_matrix(M) for M in init])
    return PoseGraph(n, ei, ej, T, omega, poses_gt, poses0, np.array([0], np.int32))
