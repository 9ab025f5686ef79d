"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: the references are a
hand-derived closed form, the scene generator's independent imaging, complex-
step derivatives, central differences, scipy's matrix exponential, LAPACK
solves of the dense damped normal equations (Eq. 2), and invariants of the LM
iteration (Alg. 1).
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as O
from synth.scenes import image_points, make_scene
from tests import dense_ref as DR

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_scene(n_cams=3, n_pts=20, noise=1.0, seed=0, cfg=0):
    return make_scene(cfg, seed=seed, noise_px=noise, n_cams=n_cams, n_pts=n_pts)


# --------------------------------------------------------------------------
# camera model (Eq. 1)
# --------------------------------------------------------------------------

def test_projection_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "projection_example.json")))
    pix, Jc, Jp, yz = O.project(g["camera"], g["point"], 9)
    assert yz == -5.0
    np.testing.assert_allclose(pix, g["pixel"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(Jp, g["Jp"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(Jc, g["Jc"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("cfg,kw", [(0, {}), (1, dict(n_cams=60, n_pts=400)),
                                    (3, dict(n_cams=20, n_pts=300))])
def test_noise_free_ground_truth_has_zero_residual_and_gradient(cfg, kw):
    s = make_scene(cfg, noise_px=0.0, perturb=False, **kw)
    o = O.Oracle.from_scene(s)
    r, w, Jc, Jp, F = o.linearization()
    px, _ = image_points(s.cams_gt[s.cam_idx], s.pts_gt[s.pt_idx])
    assert np.abs(r).max() <= 1e-9 * max(1.0, np.abs(px).max())
    U, V, gc, gp = o.normal()
    scale = np.abs(Jc).max()
    assert np.abs(gc).max() <= 1e-8 * scale and np.abs(gp).max() <= 1e-8 * scale
    assert F <= 1e-18 * s.n_obs


def test_generator_imaging_agrees_with_oracle_projection():
    s = make_scene(1, n_cams=40, n_pts=200)
    px, _ = image_points(s.cams0[s.cam_idx], s.pts0[s.pt_idx])
    for k in range(0, s.n_obs, 7):
        pix, _, _, _ = O.project(s.cams0[s.cam_idx[k]], s.pts0[s.pt_idx[k]])
        np.testing.assert_allclose(pix, px[k], rtol=1e-13, atol=1e-10)


# --------------------------------------------------------------------------
# Jacobian blocks (Sec. III-C: 2x6 pose and 2x3 point blocks, plus intrinsics)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [9, 6])
def test_jacobian_matches_complex_step(d):
    s = make_scene(0)
    o = O.Oracle.from_scene(s, options=O.OracleOptions(d=d))
    _, _, Jc, Jp, _ = o.linearization()
    Jc_ref, Jp_ref = DR.jacobian_blocks(s.cams0, s.pts0, s.cam_idx, s.pt_idx, d)
    for A, B in ((Jc, Jc_ref), (Jp, Jp_ref)):
        err = np.linalg.norm(A - B, axis=(1, 2)) / np.linalg.norm(B, axis=(1, 2))
        assert err.max() < 1e-12


def test_jacobian_matches_central_differences():
    s = make_scene(1, n_cams=30, n_pts=100)
    rng = np.random.default_rng(5)
    for k in rng.choice(s.n_obs, 25, replace=False):
        cam, X = s.cams0[s.cam_idx[k]], s.pts0[s.pt_idx[k]]
        _, Jc, Jp, _ = O.project(cam, X, 9)
        Jc_fd = np.zeros((2, 9))
        for m in range(9):
            h = 1e-6 * (max(1.0, abs(cam[7])) if m == 6 else 1.0)
            e = np.zeros(9)
            e[m] = h
            pp = O.project(O.retract_camera(cam, e), X)[0]
            pm = O.project(O.retract_camera(cam, -e), X)[0]
            Jc_fd[:, m] = (pp - pm) / (2 * h)
        Jp_fd = np.zeros((2, 3))
        for m in range(3):
            h = 1e-6 * max(1.0, abs(X[m]))
            e = np.zeros(3)
            e[m] = h
            Jp_fd[:, m] = (O.project(cam, X + e)[0] - O.project(cam, X - e)[0]) / (2 * h)
        assert np.linalg.norm(Jc - Jc_fd) / np.linalg.norm(Jc) < 1e-7
        assert np.linalg.norm(Jp - Jp_fd) / np.linalg.norm(Jp) < 1e-7


def _pose_matrix(cam):
    from scipy.spatial.transform import Rotation
    T = np.eye(4)
    T[:3, :3] = Rotation.from_quat(cam[3:7]).as_matrix()
    T[:3, 3] = cam[0:3]
    return T


def test_retraction_is_left_se3_exponential():
    rng = np.random.default_rng(1)
    s = make_scene(0)
    for i in range(8):
        cam = s.cams0[i]
        delta = np.concatenate([rng.normal(size=3) * 0.7, rng.normal(size=3) * 0.4,
                                rng.normal(size=3) * [1.0, 1e-3, 1e-3]])
        if i == 0:
            delta[3:6] *= 1e-7  # small-angle branch
        Xi = np.zeros((4, 4))
        Xi[:3, :3] = DR._hat(delta[3:6])
        Xi[:3, 3] = delta[0:3]
        T_ref = scipy.linalg.expm(Xi) @ _pose_matrix(cam)
        out = O.retract_camera(cam, delta)
        np.testing.assert_allclose(_pose_matrix(out), T_ref, rtol=0, atol=1e-12)
        np.testing.assert_allclose(out[7:10], cam[7:10] + delta[6:9], rtol=1e-15)
        assert abs(np.linalg.norm(out[3:7]) - 1) < 1e-15


def test_gauge_null_space():
    """Moving the whole scene rigidly (or scaling it) does not change any pixel,
    so J v = 0 for the induced tangent vectors: cameras -Ad_T xi, points
    rho + phi x X; scale: cameras (t, 0), points X."""
    s = tiny_scene(4, 30)
    o = O.Oracle.from_scene(s)
    _, _, Jc, Jp, _ = o.linearization()
    R_all = np.stack([_pose_matrix(c)[:3, :3] for c in s.cams0])
    t_all = s.cams0[:, 0:3]
    gens = []
    for m in range(7):
        vc = np.zeros((s.n_cams, 9))
        vp = np.zeros((s.n_pts, 3))
        if m < 6:
            xi = np.zeros(6)
            xi[m] = 1.0
            rho, phi = xi[:3], xi[3:]
            for i in range(s.n_cams):
                R, t = R_all[i], t_all[i]
                vc[i, 0:3] = -(R @ rho + np.cross(t, R @ phi))
                vc[i, 3:6] = -(R @ phi)
            vp[:] = rho + np.cross(phi[None, :], s.pts0)
        else:
            vc[:, 0:3] = t_all
            vp[:] = s.pts0
        gens.append((vc, vp))
    for vc, vp in gens:
        Jv = np.einsum("kij,kj->ki", Jc, vc[s.cam_idx]) + np.einsum("kij,kj->ki", Jp, vp[s.pt_idx])
        nrm = np.sqrt(np.sum(Jc ** 2) + np.sum(Jp ** 2)) * np.sqrt(np.sum(vc ** 2) + np.sum(vp ** 2))
        assert np.linalg.norm(Jv) <= 1e-12 * nrm


# --------------------------------------------------------------------------
# robust loss (Sec. IV-A-2: robust kernels are arithmetic on the residual)
# --------------------------------------------------------------------------

def test_huber_reduces_to_l2_when_all_residuals_are_small():
    s = make_scene(0, noise_px=0.0, perturb=False)
    s.obs = s.obs + np.random.default_rng(3).normal(size=s.obs.shape) * 0.1
    l2 = O.Oracle.from_scene(s, options=O.OracleOptions(huber_delta=0.0))
    hub = O.Oracle.from_scene(s, options=O.OracleOptions(huber_delta=10.0))
    a, b = l2.linearization(), hub.linearization()
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_huber_outlier_weight():
    s = make_scene(0, noise_px=0.0, perturb=False)
    s.obs = s.obs.copy()
    s.obs[17] += [30.0, -40.0]  # |r| = 50
    o = O.Oracle.from_scene(s, options=O.OracleOptions(huber_delta=2.0))
    r, w, _, _, F = o.linearization()
    assert abs(np.linalg.norm(r[17]) - 50.0) < 1e-9
    assert abs(w[17] - 2.0 / np.linalg.norm(r[17])) < 1e-15
    # cost is 1/2 (2 delta |r| - delta^2) for the outlier, ~0 elsewhere
    assert abs(F - 0.5 * (2 * 2.0 * np.linalg.norm(r[17]) - 4.0)) < 1e-9


# --------------------------------------------------------------------------
# normal equations (Alg. 1: A = J^T J, g = J^T R) and the damped solve (Eq. 2)
# --------------------------------------------------------------------------

def _weighted_tiny(seed=0, huber=1.0, noise=3.0):
    s = tiny_scene(3, 20, noise=noise, seed=seed)
    s.obs_w = np.random.default_rng(seed + 100).uniform(0.5, 1.5, size=s.n_obs)
    s.huber_delta = huber
    return s


def test_normal_equations_match_dense_products():
    s = _weighted_tiny()
    o = O.Oracle.from_scene(s)
    J, r, w, F = DR.dense_system(s.cams0, s.pts0, s.cam_idx, s.pt_idx, s.obs, s.obs_w,
                                 s.huber_delta)
    A = J.T @ (w[:, None] * J)
    g = J.T @ (w * r)
    U, V, gc, gp = o.normal()
    d, nc = 9, s.n_cams
    sc = np.abs(A).max()
    for i in range(nc):
        np.testing.assert_allclose(U[i], A[d * i:d * i + d, d * i:d * i + d], rtol=0, atol=1e-12 * sc)
    for j in range(s.n_pts):
        o0 = d * nc + 3 * j
        np.testing.assert_allclose(V[j], A[o0:o0 + 3, o0:o0 + 3], rtol=0, atol=1e-12 * sc)
    gs = np.abs(g).max()
    np.testing.assert_allclose(gc.reshape(-1), g[:d * nc], rtol=0, atol=1e-12 * gs)
    np.testing.assert_allclose(gp.reshape(-1), g[d * nc:], rtol=0, atol=1e-12 * gs)
    assert abs(o.linearization()[4] - F) <= 1e-13 * F


@pytest.mark.parametrize("lam,fixed", [(1e-2, ()), (1e-4, ()), (1.0, (0,))])
def test_schur_pcg_step_matches_dense_solve(lam, fixed):
    s = _weighted_tiny(seed=2)
    s.fixed_cams = np.array(fixed, np.int32)
    o = O.Oracle.from_scene(s)
    o.lam = lam
    info = o.compute_step(rtol=1e-15, maxiter=500)
    dc, dp, _ = o.step()
    J, r, w, F = DR.dense_system(s.cams0, s.pts0, s.cam_idx, s.pt_idx, s.obs, s.obs_w,
                                 s.huber_delta, fixed=fixed)
    delta, A, g = DR.dense_step(J, r, w, lam)
    got = np.concatenate([dc.reshape(-1), dp.reshape(-1)])
    assert np.linalg.norm(got - delta) <= 1e-10 * np.linalg.norm(delta)
    for i in fixed:
        assert np.all(dc[i] == 0)
    # predicted reduction of the Gauss-Newton model
    pred = -(g @ delta) - 0.5 * delta @ (A @ delta)
    assert abs(info["pred"] - pred) <= 1e-9 * abs(pred)


@pytest.mark.parametrize("lam,fixed", [(1e-2, []), (1e-6, [0])])
def test_cholesky_step_matches_dense_solve(lam, fixed):
    """The direct solve (dense Cholesky of the reduced camera system) gives
    the step of a LAPACK solve of the full damped normal equations built
    from complex-step Jacobians, with no CG tolerance involved."""
    s = _weighted_tiny(seed=2)
    s.fixed_cams = np.array(fixed, np.int32)
    o = O.Oracle.from_scene(s, options=O.OracleOptions(huber_delta=s.huber_delta, solver=1))
    o.lam = lam
    info = o.compute_step()
    dc, dp, _ = o.step()
    J, r, w, F = DR.dense_system(s.cams0, s.pts0, s.cam_idx, s.pt_idx, s.obs, s.obs_w,
                                 s.huber_delta, fixed=fixed)
    delta, A, g = DR.dense_step(J, r, w, lam)
    got = np.concatenate([dc.reshape(-1), dp.reshape(-1)])
    assert np.linalg.norm(got - delta) <= 1e-10 * np.linalg.norm(delta)
    assert info["cg_iters"] == 0 and info["cg_rel_resid"] <= 1e-13
    pred = -(g @ delta) - 0.5 * delta @ (A @ delta)
    assert abs(info["pred"] - pred) <= 1e-9 * abs(pred)


def test_cholesky_lm_run_matches_converged_pcg_run():
    """Ten LM iterations with the direct solve follow those of a PCG run
    converged to 1e-14 (the same steps up to round-off)."""
    s = make_scene(0, seed=8)
    a = O.Oracle.from_scene(s, options=O.OracleOptions(solver=1))
    b = O.Oracle.from_scene(s, options=O.OracleOptions(cg_rtol=1e-14, cg_maxiter=2000))
    for it in range(10):
        ia, ib = a.lm_step(), b.lm_step()
        assert abs(ia["cost_after"] - ib["cost_after"]) <= 1e-10 * ib["cost_after"], it
        if abs(ib["cost_before"] - ib["cost_after"]) <= 1e-11 * ib["cost_before"]:
            break
        assert ia["accepted"] == ib["accepted"]


def test_schur_blocks_match_dense_elimination():
    s = _weighted_tiny(seed=4)
    o = O.Oracle.from_scene(s)
    lam = 3e-3
    o.lam = lam
    o.compute_step(rtol=1e-15, maxiter=200)
    J, r, w, F = DR.dense_system(s.cams0, s.pts0, s.cam_idx, s.pt_idx, s.obs, s.obs_w,
                                 s.huber_delta)
    A = J.T @ (w[:, None] * J)
    g = J.T @ (w * r)
    Ad = A + lam * np.diag(np.clip(np.diag(A), 1e-6, 1e32))
    n = 9 * s.n_cams
    Sd = Ad[:n, :n] - Ad[:n, n:] @ np.linalg.solve(Ad[n:, n:], Ad[n:, :n])
    bd = -g[:n] + Ad[:n, n:] @ np.linalg.solve(Ad[n:, n:], g[n:])
    ptr, col, S, bS = o.schur()
    sc = np.abs(Sd).max()
    for a in range(s.n_cams):
        for e in range(ptr[a], ptr[a + 1]):
            b = col[e]
            np.testing.assert_allclose(S[e], Sd[9 * a:9 * a + 9, 9 * b:9 * b + 9], rtol=0,
                                       atol=1e-10 * sc)
    np.testing.assert_allclose(bS.reshape(-1), bd, rtol=0, atol=1e-10 * np.abs(bd).max())


def test_disjoint_tracks_make_block_jacobi_exact():
    """No point shared between cameras: S is block diagonal, the block-Jacobi
    preconditioner is S^-1 and PCG stops after one iteration."""
    s = tiny_scene(3, 30, seed=7)
    keep = []
    seen = {}
    for k in range(s.n_obs):
        j = s.pt_idx[k]
        if j not in seen:
            seen[j] = s.cam_idx[k]
        if s.cam_idx[k] == seen[j]:
            keep.append(k)
    s = s.subset_observations(np.array(keep))
    o = O.Oracle.from_scene(s)
    info = o.compute_step(rtol=1e-9, maxiter=50)
    assert o.nnzb() == s.n_cams
    assert info["cg_iters"] == 1 and info["cg_rel_resid"] < 1e-9


# --------------------------------------------------------------------------
# LM iteration invariants (Alg. 1 and the trust-region strategy of Sec. V)
# --------------------------------------------------------------------------

def test_lm_accepts_only_decreases_and_rejects_leave_params_untouched():
    s = make_scene(0, seed=1)
    o = O.Oracle.from_scene(s)
    o.lam = 1e-9  # start overly optimistic so that some steps get rejected
    n_rej = 0
    for _ in range(25):
        before = o.get_params()
        info = o.lm_step()
        after = o.get_params()
        if info["accepted"]:
            assert info["cost_after"] < info["cost_before"]
            assert o.cost() == info["cost_after"]
        else:
            n_rej += 1
            assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
            assert info["lambda_next"] == min(16 * info["lambda_used"], 1e12)
    assert n_rej >= 1


def test_weight_scaling_by_four_is_exact():
    """omega -> 4 omega scales A, g, F by 4 exactly (a power of four keeps the
    Cholesky factors exact), so every step is bit-identical."""
    s = make_scene(0, seed=2)
    s.huber_delta = 2.0
    a = O.Oracle.from_scene(s)
    s4 = make_scene(0, seed=2)
    s4.huber_delta = 2.0
    s4.obs_w = np.full(s4.n_obs, 4.0)
    b = O.Oracle.from_scene(s4)
    for _ in range(4):
        ia, ib = a.lm_step(), b.lm_step()
        assert ib["cost_before"] == 4 * ia["cost_before"]
        assert ib["cg_iters"] == ia["cg_iters"] and ib["accepted"] == ia["accepted"]
        pa, pb = a.get_params(), b.get_params()
        assert np.array_equal(pa[0], pb[0]) and np.array_equal(pa[1], pb[1])


def test_noise_free_scene_converges_to_zero_cost():
    s = make_scene(0, noise_px=0.0)
    o = O.Oracle.from_scene(s)
    for _ in range(10):
        info = o.lm_step()
    assert o.cost() <= 1e-20 * s.n_obs


def test_observation_order_does_not_matter():
    s = make_scene(0, seed=3)
    perm = np.random.default_rng(0).permutation(s.n_obs)
    a = O.Oracle.from_scene(s)
    b = O.Oracle.from_scene(s.permuted(perm))
    assert abs(a.cost() - b.cost()) <= 1e-14 * a.cost()
    ia, ib = a.lm_step(rtol=0.0, maxiter=20), b.lm_step(rtol=0.0, maxiter=20)
    assert abs(ia["cost_after"] - ib["cost_after"]) <= 1e-12 * ia["cost_after"]
    pa, pb = a.get_params(), b.get_params()
    np.testing.assert_allclose(pa[1], pb[1], rtol=0, atol=1e-9)


def test_gradient_is_derivative_of_cost():
    s = make_scene(0, seed=4)
    s.huber_delta = 1.5
    o = O.Oracle.from_scene(s)
    _, _, gc, gp = o.normal()
    rng = np.random.default_rng(9)
    vc = rng.normal(size=gc.shape) * 1e-3
    vp = rng.normal(size=gp.shape) * 1e-3
    h = 1e-4

    def F_at(t):
        cams = np.stack([O.retract_camera(c, t * v) for c, v in zip(s.cams0, vc)])
        return o.cost(cams, s.pts0 + t * vp)

    fd = (F_at(h) - F_at(-h)) / (2 * h)
    an = np.sum(gc * vc) + np.sum(gp * vp)
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_predicted_reduction_matches_actual_for_short_steps():
    s = make_scene(0, seed=5)
    o = O.Oracle.from_scene(s)
    o.lm_step()  # move off the initial point
    o.lam = 1e3
    info = o.lm_step(rtol=1e-12, maxiter=300)
    ratio = (info["cost_before"] - info["cost_after"]) / info["pred"]
    assert info["accepted"] and abs(ratio - 1) < 1e-2


def test_zero_gradient_gives_zero_step():
    s = make_scene(0, noise_px=0.0, perturb=False)
    s.obs = image_points(s.cams_gt[s.cam_idx], s.pts_gt[s.pt_idx])[0]
    o = O.Oracle.from_scene(s)
    info = o.compute_step()
    dc, dp, _ = o.step()
    assert info["grad_inf"] < 1e-8
    assert np.abs(dc).max() < 1e-10 and np.abs(dp).max() < 1e-10


# --------------------------------------------------------------------------
# trust-region damping and the stopping rules (Sec. V: TrustRegion(up=2,
# down=0.5**4), StopOnPlateau)
# --------------------------------------------------------------------------

# (accepted, ratio, lambda) -> lambda after the step.  The factors are the
# paper's: the trust radius 1/lambda grows by up = 2 (lambda halves) and
# shrinks by down = 1/16 (lambda x 16); the thresholds 1/4 and 3/4 on the
# ratio of actual to predicted reduction, the lower branch taking the tie at
# exactly 1/4 and a rejection counting as a shrink, are the reading the
# oracle takes where the paper gives no values.
LAMBDA_TABLE = [
    (True, 0.10, 1e-3, 1.6e-2),
    (True, 0.25, 1e-3, 1.6e-2),
    (True, 0.50, 1e-3, 1e-3),
    (True, 0.75, 1e-3, 1e-3),
    (True, 0.80, 1e-3, 5e-4),
    (True, 1.70, 4.0, 2.0),
    (False, 0.90, 1e-3, 1.6e-2),
    (False, -3.0, 2.0, 32.0),
    (True, 0.90, 1.5e-12, 1e-12),   # halving clamped at lambda_min
    (False, 0.90, 1e11, 1e12),      # growth clamped at lambda_max
    (True, 0.10, 1e12, 1e12),
]


@pytest.mark.parametrize("accepted,ratio,lam,expect", LAMBDA_TABLE)
def test_trust_region_damping_rule(accepted, ratio, lam, expect):
    got = O.lambda_update(accepted, ratio, lam, 1e-12, 1e12)
    assert got == pytest.approx(expect, rel=1e-15)


def test_lm_damping_follows_the_rule_on_accepted_and_rejected_steps():
    """Every step of an LM run moves lambda by the factor the table above
    fixes for its own ratio of actual to predicted reduction; the run must
    visit all three branches (halve, keep, x16)."""
    s = make_scene(0, seed=1)
    o = O.Oracle.from_scene(s)
    o.lam = 1e-9
    seen = set()
    for _ in range(40):
        info = o.lm_step()
        lam, nxt = info["lambda_used"], info["lambda_next"]
        ratio = (info["cost_before"] - info["cost_after"]) / info["pred"]
        if not info["accepted"] or ratio <= 0.25:
            assert nxt == min(16 * lam, 1e12)
            seen.add("x16")
        elif ratio > 0.75:
            assert nxt == max(lam / 2, 1e-12)
            seen.add("half")
        else:
            assert nxt == lam
            seen.add("keep")
    assert {"x16", "half"} <= seen


def test_solve_stops_at_the_first_plateau_of_five_flat_steps():
    s = make_scene(0, seed=6)
    o = O.Oracle.from_scene(s)
    st, infos, why = o.solve(60, rel_tol=1e-6, plateau_steps=5)
    assert st == 0 and why in ("plateau", "gradient")
    dec = [(i["cost_before"] - i["cost_after"]) / i["cost_before"] if i["accepted"] else 0.0
           for i in infos]
    flat = [d < 1e-6 for d in dec]
    runs = 0
    for n, f in enumerate(flat):
        runs = runs + 1 if f else 0
        g_ok = infos[n]["grad_inf"] <= 1e-12 * (1 + infos[n]["cost_before"])
        if runs >= 5 or g_ok:
            assert n == len(infos) - 1, "solve ran past a stopping rule"
            assert why == ("plateau" if runs >= 5 else "gradient")
            break
    else:
        pytest.fail("no stopping rule held at the last iteration")
    assert all(i["cost_after"] < i["cost_before"] for i in infos if i["accepted"])


def test_solve_noise_free_scene_converges_then_stops():
    """Noise-free observations: the solve reaches the zero-cost optimum (up to
    round-off) and then stops by a rule, not by the iteration cap."""
    s = make_scene(0, noise_px=0.0)
    o = O.Oracle.from_scene(s)
    st, infos, why = o.solve(60, rel_tol=1e-6, plateau_steps=5)
    assert st == 0 and why in ("plateau", "gradient") and len(infos) < 60
    assert o.cost() <= 1e-20 * s.n_obs


def test_solve_iteration_cap():
    s = make_scene(0, seed=7)
    o = O.Oracle.from_scene(s)
    st, infos, why = o.solve(3, rel_tol=1e-6, plateau_steps=5)
    assert st == 0 and why == "max_iters" and len(infos) == 3


def test_solve_reports_rejection_at_lambda_max():
    """Noise-free scene with lambda capped at its start value: once the
    optimum is reached, round-off rejections grow lambda to the cap, and the
    first rejection there ends the solve as not converged, leaving theta as
    it was before that step."""
    s = make_scene(0, noise_px=0.0)
    opt = O.OracleOptions(lambda0=1e-4, lambda_min=1e-12, lambda_max=1e-4)
    o = O.Oracle.from_scene(s, options=opt)
    st, infos, why = o.solve(60, rel_tol=0.0, plateau_steps=5)
    assert why == "lambda_max" and st == -4
    assert not infos[-1]["accepted"] and infos[-1]["lambda_used"] == 1e-4
    assert all(i["lambda_used"] <= 1e-4 for i in infos)
    assert all(i["accepted"] or i["lambda_used"] < 1e-4 for i in infos[:-1])
    assert o.cost() == infos[-1]["cost_before"]


def test_thread_count_does_not_change_results():
    s = make_scene(3, n_cams=24, n_pts=600)
    out = []
    for n in (1, 3, 8):
        O.set_threads(n)
        o = O.Oracle.from_scene(s)
        infos = [o.lm_step() for _ in range(3)]
        out.append((infos, o.get_params()))
    O.set_threads(os.cpu_count() or 1)
    for infos, (c, p) in out[1:]:
        assert infos == out[0][0]
        assert np.array_equal(c, out[0][1][0]) and np.array_equal(p, out[0][1][1])
