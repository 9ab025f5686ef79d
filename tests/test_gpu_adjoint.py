"""GPU implicit-function adjoint (ba_backward, through the C ABI) against
the oracle's adjoint, and the differentiable layer against finite
differences through the GPU solver.

Inputs: the seeded scene generator; expected values: the oracle only (its
adjoint is pinned in test_oracle_adjoint.py).  The loss is the squared pose
error against the generated ground truth plus a small point term; the GPU
receives its gradient with respect to the stored parameters, the oracle the
tangent gradient formed independently by complex-step differentiation of
the loss along the retraction.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth.scenes import make_scene
from tests import dense_ref as R
from tests.test_oracle_adjoint import solve_to_stationary, tiny_scene

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2409_12190_amd import ba as B  # noqa: E402

PT_W = 0.01  # weight of the point term of the loss


def loss_np(cams, pts, s):
    Rm = R._quat_to_rot(cams[:, 3:7])
    Rg = R._quat_to_rot(s.cams_gt[:, 3:7])
    return (np.sum((cams[:, 0:3] - s.cams_gt[:, 0:3]) ** 2) + np.sum((Rm - Rg) ** 2)
            + PT_W * np.sum((pts - s.pts_gt) ** 2))


def storage_gradient(cams, pts, s):
    """dL/d(stored rows): analytic in t and the points, complex-step in q."""
    gc = np.zeros_like(cams)
    gc[:, 0:3] = 2 * (cams[:, 0:3] - s.cams_gt[:, 0:3])
    Rg = R._quat_to_rot(s.cams_gt[:, 3:7])
    for m in range(4):
        q = cams[:, 3:7].astype(np.complex128)
        q[:, m] += 1j * R.H
        gc[:, 3 + m] = np.sum((R._quat_to_rot(q) - Rg) ** 2, axis=(1, 2)).imag / R.H
    gp = 2 * PT_W * (pts - s.pts_gt)
    return gc, gp


def tangent_gradient(cams, pts, s):
    """dL/d(tangent) by complex-step along the left retraction (rotation
    matrix form, independent of the quaternion algebra)."""
    nc = s.n_cams
    gc = np.zeros((nc, 9))
    Rq = R._quat_to_rot(cams[:, 3:7])
    Rg = R._quat_to_rot(s.cams_gt[:, 3:7])
    for a in range(nc):
        if a in s.fixed_cams:
            continue
        for m in range(6):
            d = np.zeros(6, np.complex128)
            d[m] = 1j * R.H
            Rd, td = R._exp_se3(d[None])
            Rn = Rd[0] @ Rq[a]
            tn = Rd[0] @ cams[a, 0:3] + td[0]
            La = np.sum((tn - s.cams_gt[a, 0:3]) ** 2) + np.sum((Rn - Rg[a]) ** 2)
            gc[a, m] = La.imag / R.H
    gp = 2 * PT_W * (pts - s.pts_gt)
    return gc, gp


def gpu_problem(s, cams, pts, precision=B.BA_FP64, **kw):
    print(f"[gpu] adjoint scene nc={s.n_cams} np={s.n_pts} no={s.n_obs} precision={precision}",
          flush=True)
    kw.setdefault("cg_maxiter", 3000)
    kw.setdefault("adjoint_rtol", 1e-12)
    return B.Problem(s.n_cams, s.n_pts, s.cam_idx, s.pt_idx, s.obs, s.obs_w, precision=precision,
                     fixed_cams=s.fixed_cams, cams=cams, pts=pts, enable_backward=True, **kw)


def close(got, ref, tol, what=""):
    """Element by element: |got - ref| <= tol * max|ref| for every entry."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    assert got.shape == ref.shape, what
    np.testing.assert_allclose(got, ref, rtol=0, atol=tol * float(np.abs(ref).max()), err_msg=what)


def maxerr(got, ref):
    """Largest entry error relative to the largest reference entry."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def test_backward_through_a_long_track_matches_oracle():
    """A ring of 300 cameras whose point 0 is seen by 280 of them (more than
    a chunk of 256 observations: the adjoint's point blocks and
    back-substitution run through their long-track kernels), solved to a
    stationary point by the oracle: v and the gradients match its adjoint."""
    s = make_scene(0, n_cams=300, n_pts=1500, long_track=280)
    s.obs_w = np.random.default_rng([7, 300]).uniform(0.5, 1.5, s.n_obs)
    s.fixed_cams = np.array([0, 1], np.int32)
    o = solve_to_stationary(s)
    cams, pts = o.get_params()
    gcs, gps = storage_gradient(cams, pts, s)
    gct, gpt = tangent_gradient(cams, pts, s)
    dx_o, dw_o, vc_o, vp_o = o.backward(gct, gpt)
    g = gpu_problem(s, cams, pts)
    dx, dw, info = g.backward(gcs, gps)
    vp = g.export(B.BA_X_ADJ_VP)
    print(f"  adjoint cg {info['cg_iters']} rel resid {info['cg_rel_resid']:.2e}; max errors v_c "
          f"{maxerr(g.export(B.BA_X_ADJ_VC), vc_o):.1e} v_p {maxerr(vp, vp_o):.1e} "
          f"dL/dx {maxerr(dx.cpu().numpy(), dx_o):.1e} dL/dw {maxerr(dw.cpu().numpy(), dw_o):.1e}", flush=True)
    assert info["cg_rel_resid"] <= 1e-12
    close(g.export(B.BA_X_ADJ_VC), vc_o, 1e-8, "v cameras")
    close(vp, vp_o, 1e-8, "v points")
    close(vp[0], vp_o[0], 1e-8, "v of the long track")
    close(dx.cpu().numpy(), dx_o, 1e-8, "dL/dx")
    close(dw.cpu().numpy(), dw_o, 1e-8, "dL/dw")


@pytest.mark.parametrize("precision", [B.BA_FP64, B.BA_MIXED])
def test_backward_matches_oracle_adjoint(precision):
    s = tiny_scene(seed=2)
    o = solve_to_stationary(s)
    cams, pts = o.get_params()
    gcs, gps = storage_gradient(cams, pts, s)
    gct, gpt = tangent_gradient(cams, pts, s)
    dx_o, dw_o, vc_o, vp_o = o.backward(gct, gpt)
    g = gpu_problem(s, cams, pts, precision=precision)
    dx, dw, info = g.backward(gcs, gps)
    print(f"  adjoint cg {info['cg_iters']} rel resid {info['cg_rel_resid']:.2e}", flush=True)
    assert info["cg_rel_resid"] <= 1e-12
    close(g.export(B.BA_X_ADJ_VC), vc_o, 1e-8, "v cameras")
    close(g.export(B.BA_X_ADJ_VP), vp_o, 1e-8, "v points")
    close(dx.cpu().numpy(), dx_o, 1e-8, "dL/dx")
    close(dw.cpu().numpy(), dw_o, 1e-8, "dL/dw")


def test_backward_on_the_weighted_trajectory_scene_matches_oracle():
    """128 cameras / 20,000 points / ~100k weighted observations, cameras 0
    and 1 fixed, solved to a stationary point by the oracle.

    The exact Hessian of this scene is ill-conditioned along the weakly
    observed intrinsics of the trajectory cameras (the adjoint vector reaches
    1e9 for a unit-size loss gradient), so the oracle's dense Cholesky solve
    and the GPU's PCG, stopped at a relative residual eps below 1e-12, agree
    to the conditioning: entry by entry, |dv|_inf / |v|_inf <= kappa(S) eps
    sqrt(n) with kappa(S) the condition number of the reduced matrix the
    adjoint solved (exported after the backward pass) and n its size; the
    gradients with respect to x and w, whose sensitivity to v is weaker,
    within 1e-4 of their largest entry."""
    s = make_scene(3)
    o = solve_to_stationary(s, iters=40)
    cams, pts = o.get_params()
    gcs, gps = storage_gradient(cams, pts, s)
    gct, gpt = tangent_gradient(cams, pts, s)
    dx_o, dw_o, vc_o, vp_o = o.backward(gct, gpt)
    g = gpu_problem(s, cams, pts)
    dx, dw, info = g.backward(gcs, gps)
    e_v = maxerr(g.export(B.BA_X_ADJ_VC), vc_o)
    e_x = maxerr(dx.cpu().numpy(), dx_o)
    e_w = maxerr(dw.cpu().numpy(), dw_o)
    Sa = g.export(B.BA_X_S)
    ptr, col = g.export(B.BA_X_S_PTR), g.export(B.BA_X_S_COL)
    n = 9 * s.n_cams
    dense = np.zeros((n, n))
    for a in range(s.n_cams):
        for e in range(ptr[a], ptr[a + 1]):
            b = col[e]
            dense[9 * a:9 * a + 9, 9 * b:9 * b + 9] = Sa[e]
            dense[9 * b:9 * b + 9, 9 * a:9 * a + 9] = Sa[e].T
    kappa = np.linalg.cond(dense)
    bound_v = kappa * max(info["cg_rel_resid"], 1e-16) * np.sqrt(n)
    print(f"  adjoint cg {info['cg_iters']} rel resid {info['cg_rel_resid']:.2e}; kappa {kappa:.2e}; "
          f"max-entry error v {e_v:.2e} (bound {bound_v:.2e}) dL/dx {e_x:.2e} dL/dw {e_w:.2e}",
          flush=True)
    assert info["cg_rel_resid"] <= 1e-12
    assert e_v <= bound_v and e_x < 1e-4 and e_w < 1e-4


def test_backward_refuses_a_point_that_is_not_stationary():
    """The adjoint is valid only where the gradient vanishes: after three LM
    steps from the perturbed start (far from converged) ba_backward returns
    BA_ENOTCONV and writes nothing; at the converged point it runs."""
    s = tiny_scene(seed=2)
    g = gpu_problem(s, s.cams0, s.pts0)
    st, infos = g.solve(3, rel_tol=1e-12, plateau_steps=5)
    assert infos[-1]["stop_reason"] == B.BA_STOP_MAX_ITERS
    cams, pts = g.get_params()
    gcs, gps = storage_gradient(cams.cpu().numpy(), pts.cpu().numpy(), s)
    sentinel = torch.full((s.n_obs, 2), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(B.BaError) as e:
        B.ba_backward(g.h, g._dev(gcs), g._dev(gps), sentinel, None)
    assert e.value.status == B.BA_ENOTCONV and "stationary" in str(e.value)
    assert bool((sentinel == 7.0).all())
    o = solve_to_stationary(s)
    cs, ps = o.get_params()
    g.set_params(cs, ps)
    gcs, gps = storage_gradient(cs, ps, s)
    dx, dw, info = g.backward(gcs, gps)
    assert info["status"] == B.BA_OK and info["grad_inf"] >= 0.0


def test_backward_leaves_the_forward_path_working():
    s = tiny_scene(seed=2)
    o = solve_to_stationary(s)
    cams, pts = o.get_params()
    g = gpu_problem(s, s.cams0, s.pts0, cg_variant=B.BA_CG_STANDARD)
    g.set_cg(1e-12, 3000)
    first = [g.lm_step()["cost_before"] for _ in range(3)]
    g.set_params(cams, pts)
    gcs, gps = storage_gradient(cams, pts, s)
    g.backward(gcs, gps)
    g.set_params(s.cams0, s.pts0)
    g.set_lambda(1e-4)
    again = [g.lm_step()["cost_before"] for _ in range(3)]
    assert again == first


def test_layer_gradients_match_finite_differences_through_the_gpu_solver():
    s = tiny_scene(seed=2)
    o = solve_to_stationary(s)
    cams_star, pts_star = o.get_params()
    g = gpu_problem(s, cams_star, pts_star, cg_rtol=1e-12, cg_variant=B.BA_CG_STANDARD,
                    lambda0=1e-8)
    obs = torch.tensor(s.obs, dtype=torch.float64, device="cuda", requires_grad=True)
    w = torch.tensor(s.obs_w, dtype=torch.float64, device="cuda", requires_grad=True)
    cams, pts = B.bundle_adjust(g, obs, w, max_iters=50)
    cams_gt = torch.tensor(s.cams_gt, device="cuda")
    pts_gt = torch.tensor(s.pts_gt, device="cuda")

    def tloss(c, p):
        # rotation part through the quaternion: R(q) - R_gt, Frobenius
        q = c[:, 3:7]
        x, y, z, ww = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
        Rm = torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * ww), 2 * (x * z + y * ww),
                          2 * (x * y + z * ww), 1 - 2 * (x * x + z * z), 2 * (y * z - x * ww),
                          2 * (x * z - y * ww), 2 * (y * z + x * ww), 1 - 2 * (x * x + y * y)], 1)
        qg = cams_gt[:, 3:7]
        xg, yg, zg, wg = qg[:, 0], qg[:, 1], qg[:, 2], qg[:, 3]
        Rg = torch.stack([1 - 2 * (yg * yg + zg * zg), 2 * (xg * yg - zg * wg), 2 * (xg * zg + yg * wg),
                          2 * (xg * yg + zg * wg), 1 - 2 * (xg * xg + zg * zg), 2 * (yg * zg - xg * wg),
                          2 * (xg * zg - yg * wg), 2 * (yg * zg + xg * wg), 1 - 2 * (xg * xg + yg * yg)], 1)
        return (((c[:, 0:3] - cams_gt[:, 0:3]) ** 2).sum() + ((Rm - Rg) ** 2).sum()
                + PT_W * ((p - pts_gt) ** 2).sum())

    L = tloss(cams, pts)
    L.backward()
    gx, gw = obs.grad.cpu().numpy(), w.grad.cpu().numpy()

    def resolved(o_xy, o_w):
        g.set_params(cams_star, pts_star)
        g.set_lambda(1e-8)
        c, p = B.bundle_adjust(g, o_xy, o_w, max_iters=50)
        return float(tloss(c, p))

    base_obs = torch.tensor(s.obs, dtype=torch.float64, device="cuda")
    base_w = torch.tensor(s.obs_w, dtype=torch.float64, device="cuda")
    h = 0.1   # large enough that stopping at round-off of the cost does not matter
    for k in np.random.default_rng(3).choice(s.n_obs, 3, replace=False):
        e = torch.zeros_like(base_obs)
        e[k, 0] = h
        fd = (resolved(base_obs + e, base_w) - resolved(base_obs - e, base_w)) / (2 * h)
        assert abs(fd - gx[k, 0]) <= 2e-5 * np.abs(gx).max(), (k, fd, gx[k, 0])
        ew = torch.zeros_like(base_w)
        ew[k] = 0.05
        fd = (resolved(base_obs, base_w + ew) - resolved(base_obs, base_w - ew)) / 0.1
        assert abs(fd - gw[k]) <= 2e-5 * np.abs(gw).max() + 1e-3 * abs(gw[k]), (k, fd, gw[k])
