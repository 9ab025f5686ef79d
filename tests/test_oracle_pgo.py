"""Pins of the pose-graph oracle (Sec. IV-D: r_ij = Log(zeta_i^-1 zeta_j T_ij^-1),
Eq. 4 cost) against what the mathematics fixes: scipy's matrix exponential
of the se(3) twist, the textbook closed form of SO(3)'s inverse left
Jacobian, central differences of the residual along the retraction, a LAPACK
solve of the damped normal equations, and invariants of the LM iteration."""
import numpy as np
import pytest

from oracle import oracle as O
from synth.posegraph import from_matrix, make_pose_graph, se3_exp, to_matrix


def random_pose(rng, scale=3.0):
    xi = np.concatenate([rng.normal(size=3) * scale, rng.normal(size=3)])
    return from_matrix(se3_exp(xi))


def test_residual_is_the_log_of_the_pose_error():
    """With T = Exp(xi)^-1 zeta_i^-1 zeta_j the error zeta_i^-1 zeta_j T^-1
    is Exp(xi) exactly, so r must give xi back (Exp by scipy's expm)."""
    rng = np.random.default_rng(0)
    for _ in range(20):
        Zi, Zj = random_pose(rng), random_pose(rng)
        xi = np.concatenate([rng.normal(size=3), rng.normal(size=3) * 0.5])
        T = from_matrix(np.linalg.inv(se3_exp(xi)) @ np.linalg.inv(to_matrix(Zi)) @ to_matrix(Zj))
        r, _ = O.pgo_edge(Zi, Zj, T)
        np.testing.assert_allclose(r, xi, rtol=0, atol=1e-10)


def test_retraction_is_the_left_se3_exponential():
    rng = np.random.default_rng(1)
    for _ in range(10):
        Z = random_pose(rng)
        d = np.concatenate([rng.normal(size=3) * 0.3, rng.normal(size=3) * 0.2])
        want = se3_exp(d) @ to_matrix(Z)
        got = to_matrix(O.pgo_retract(Z, d))
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_inverse_left_jacobian_rotation_block_closed_form():
    """For xi = (0, phi) the rotation block of Jl^-1 is SO(3)'s
    I - phi^/2 + (1/th^2 - (1 + cos th) / (2 th sin th)) phi^2 (textbook),
    the identity at 0."""
    np.testing.assert_array_equal(O.se3_jl_inv(np.zeros(6)), np.eye(6))
    rng = np.random.default_rng(2)
    for _ in range(10):
        phi = rng.normal(size=3) * 0.7
        th = np.linalg.norm(phi)
        P = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
        want = np.eye(3) - 0.5 * P + (1 / th ** 2 - (1 + np.cos(th)) / (2 * th * np.sin(th))) * P @ P
        J = O.se3_jl_inv(np.concatenate([np.zeros(3), phi]))
        np.testing.assert_allclose(J[3:, 3:], want, rtol=0, atol=1e-13)
        np.testing.assert_allclose(J[:3, :3], want, rtol=0, atol=1e-13)
        np.testing.assert_allclose(J[3:, :3], 0.0, atol=0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_edge_jacobian_matches_central_differences(seed):
    """d r / d delta_j and d r / d delta_i = -d r / d delta_j against central
    differences along the retraction (h = 1e-6): relative error < 1e-7."""
    rng = np.random.default_rng(10 + seed)
    Zi, Zj = random_pose(rng), random_pose(rng)
    rel = np.linalg.inv(to_matrix(Zi)) @ to_matrix(Zj)
    T = from_matrix(se3_exp(np.concatenate([rng.normal(size=3) * 0.3, rng.normal(size=3) * 0.3])) @ rel)
    r0, Jj = O.pgo_edge(Zi, Zj, T)
    h = 1e-6
    for side, Jwant in ((1, Jj), (0, -Jj)):
        fd = np.zeros((6, 6))
        for k in range(6):
            d = np.zeros(6)
            d[k] = h
            if side == 1:
                rp, _ = O.pgo_edge(Zi, O.pgo_retract(Zj, d), T)
                rm, _ = O.pgo_edge(Zi, O.pgo_retract(Zj, -d), T)
            else:
                rp, _ = O.pgo_edge(O.pgo_retract(Zi, d), Zj, T)
                rm, _ = O.pgo_edge(O.pgo_retract(Zi, -d), Zj, T)
            fd[:, k] = (rp - rm) / (2 * h)
        assert np.linalg.norm(fd - Jwant) <= 1e-7 * np.linalg.norm(Jwant)


def test_noise_free_graph_has_zero_residual_at_ground_truth():
    g = make_pose_graph(0, rings=8, per_ring=10, noise=False)
    o = O.PgoOracle(g)
    assert o.cost(g.poses_gt) <= 1e-20
    o.set_poses(g.poses_gt)
    o.lm_step()
    _, _, _, gr, _ = o.system()
    assert np.abs(gr).max() <= 1e-8


def dense_system(g, Z):
    """J (central differences of the oracle's residuals, one pose at a time,
    fixed poses left out) and r of the whole graph."""
    n, m = g.n_poses, g.n_edges
    r = np.zeros(6 * m)
    J = np.zeros((6 * m, 6 * n))
    for e in range(m):
        r[6 * e:6 * e + 6], _ = O.pgo_edge(Z[g.ei[e]], Z[g.ej[e]], g.T[e])
    h = 1e-6
    for a in range(n):
        if a in set(g.fixed.tolist()):
            continue
        for k in range(6):
            d = np.zeros(6)
            d[k] = h
            Zp, Zm = Z.copy(), Z.copy()
            Zp[a] = O.pgo_retract(Z[a], d)
            Zm[a] = O.pgo_retract(Z[a], -d)
            for e in np.nonzero((g.ei == a) | (g.ej == a))[0]:
                rp, _ = O.pgo_edge(Zp[g.ei[e]], Zp[g.ej[e]], g.T[e])
                rm, _ = O.pgo_edge(Zm[g.ei[e]], Zm[g.ej[e]], g.T[e])
                J[6 * e:6 * e + 6, 6 * a + k] = (rp - rm) / (2 * h)
    return J, r


@pytest.mark.parametrize("solver,lam", [(0, 1e-3), (1, 1e-3), (1, 1e-8)])
def test_lm_step_matches_dense_damped_solve(solver, lam):
    """The step of one LM iteration against a LAPACK solve of
    (J^T W J + lam diag(clamp(diag))) dx = -J^T W r with J from central
    differences (FD accuracy ~1e-9: bound 1e-6); the predicted reduction
    against its dense formula."""
    g = make_pose_graph(1, rings=4, per_ring=6)
    o = O.PgoOracle(g, cg_rtol=1e-14, cg_maxiter=500, solver=solver)
    o.lam = lam
    info = o.lm_step()
    _, _, _, _, dx = o.system()
    J, r = dense_system(g, g.poses0)
    W = np.zeros((6 * g.n_edges, 6 * g.n_edges))
    for e in range(g.n_edges):
        W[6 * e:6 * e + 6, 6 * e:6 * e + 6] = g.omega[e]
    A = J.T @ W @ J
    b = J.T @ W @ r
    keep = np.ones(6 * g.n_poses, bool)
    for a in g.fixed:
        keep[6 * a:6 * a + 6] = False
    Ak = A[np.ix_(keep, keep)]
    Ad = Ak + lam * np.diag(np.clip(np.diag(Ak), 1e-6, 1e32))
    want = np.zeros(6 * g.n_poses)
    want[keep] = np.linalg.solve(Ad, -b[keep])
    got = dx.reshape(-1)
    assert np.linalg.norm(got - want) <= 1e-6 * np.linalg.norm(want)
    pred = -(b @ got) - 0.5 * got @ A @ got
    assert abs(info["pred"] - pred) <= 1e-6 * abs(pred)


def test_lm_converges_and_accepts_only_decreases():
    g = make_pose_graph(2, rings=10, per_ring=12)
    o = O.PgoOracle(g)
    prev = None
    for _ in range(15):
        info = o.lm_step()
        if info["accepted"]:
            assert info["cost_after"] < info["cost_before"]
        if prev is not None:
            assert info["cost_before"] <= prev
        prev = info["cost_after"] if info["accepted"] else info["cost_before"]
    # the optimum lies below the ground truth's cost (noise is fitted)
    assert o.cost() <= o.cost(g.poses_gt)
    # noise-free: back to the ground truth
    g0 = make_pose_graph(2, rings=10, per_ring=12, noise=False)
    o0 = O.PgoOracle(g0, cg_rtol=1e-12, cg_maxiter=2000)
    for _ in range(15):
        o0.lm_step()
    assert o0.cost() <= 1e-16 * g0.n_edges
