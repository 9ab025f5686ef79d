"""Pins of the oracle's implicit-function adjoint (no GPU).

- the per-observation curvature term sum_m r_m Hess(pi_m) against central
  differences of complex-step Jacobians of the retracted camera model;
- the adjoint vector and the gradients with respect to observations and
  weights against a dense solve with the Hessian of delta -> F(theta (+) delta)
  formed by central differences of complex-step gradients (no Schur
  complement, LAPACK solve);
- the gradients against finite differences through the solver itself:
  perturb one observation (or weight), re-solve the problem to a stationary
  point, difference the loss;
- a planted mistake: dropping the curvature term (Gauss-Newton Hessian) is
  caught by the finite-difference comparison.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth.scenes import make_scene
from tests import dense_ref as R

HR = 1e-5  # real step of the central differences


def tiny_scene(seed=0):
    """Six ring cameras, 50 points seen by four cameras each, per-observation
    weights U(0.5, 1.5), cameras 0 and 1 fixed (gauge)."""
    s = make_scene(0, n_cams=6, n_pts=50, seed=seed)
    s.obs_w = np.random.default_rng([7, seed]).uniform(0.5, 1.5, s.n_obs)
    s.fixed_cams = np.array([0, 1], np.int32)
    return s


def solve_to_stationary(s, obs=None, w=None, cams=None, pts=None, iters=60):
    o = O.Oracle(s.n_cams, s.n_pts, s.cam_idx, s.pt_idx, s.obs if obs is None else obs,
                 s.obs_w if w is None else w, s.fixed_cams,
                 options=O.OracleOptions(cg_rtol=1e-14, cg_maxiter=2000, lambda0=1e-6))
    o.set_params(s.cams0 if cams is None else cams, s.pts0 if pts is None else pts)
    rejected = 0
    for _ in range(iters):
        info = o.lm_step()
        rejected = 0 if info["accepted"] else rejected + 1
        if rejected == 3:   # no decrease left above round-off
            break
    # the cost cannot resolve the last digits of the optimum (it is flat to
    # round-off there): finish with undamped Gauss-Newton steps, taken
    # unconditionally, which drive the gradient itself to round-off
    for _ in range(6):
        o.lam = 1e-12
        o.compute_step()
        dc, dp, _ = o.step()
        c, p = o.get_params()
        c = np.array([O.retract_camera(c[a], dc[a]) for a in range(s.n_cams)])
        o.set_params(c, p + dp)
    return o


def tangent_pixels(cams, pts, cidx, pidx, dcam, dpt):
    """Pixels of every observation after the tangent update (dcam per camera,
    dpt per point); complex-capable."""
    return R.pixels(cams[cidx], pts[pidx] + dpt[pidx], dcam[cidx], 9)


def loss(cams, pts, s):
    """Squared pose error against the generated ground truth."""
    Rm = R._quat_to_rot(cams[:, 3:7])
    Rg = R._quat_to_rot(s.cams_gt[:, 3:7])
    return np.sum((cams[:, 0:3] - s.cams_gt[:, 0:3]) ** 2) + np.sum((Rm - Rg) ** 2)


def retracted(cams, pts, dcam, dpt):
    """theta (+) delta, complex-capable (for complex-step derivatives of the loss)."""
    Rq = R._quat_to_rot(cams[:, 3:7])
    Rd, td = R._exp_se3(dcam[:, 0:6])
    Rn = np.einsum("kij,kjl->kil", Rd, Rq)
    tn = np.einsum("kij,kj->ki", Rd, cams[:, 0:3]) + td
    return Rn, tn, pts + dpt


def loss_tangent_gradient(o, s):
    cams, pts = o.get_params()
    nc, npt = s.n_cams, s.n_pts
    gc = np.zeros((nc, 9))
    Rg = R._quat_to_rot(s.cams_gt[:, 3:7])
    for a in range(nc):
        for m in range(6):
            dcam = np.zeros((nc, 9), np.complex128)
            dcam[a, m] = 1j * R.H
            Rn, tn, _ = retracted(cams.astype(np.complex128), pts, dcam, np.zeros((npt, 3)))
            L = np.sum((tn - s.cams_gt[:, 0:3]) ** 2) + np.sum((Rn - Rg) ** 2)
            gc[a, m] = L.imag / R.H
    gc[s.fixed_cams] = 0.0
    return gc, np.zeros((npt, 3))


def test_curvature_term_matches_finite_differences():
    s = tiny_scene()
    o = O.Oracle.from_scene(s)
    cams, pts = s.cams0, s.pts0
    for k in [0, 7, 31, s.n_obs - 1]:
        r, J, Cm = o.obs_second_order(k)
        cam = cams[s.cam_idx[k]][None].astype(np.complex128)
        X = pts[s.pt_idx[k]][None].astype(np.complex128)

        def jac(dreal):
            Jk = np.zeros((2, 12))
            for i in range(12):
                d = dreal.astype(np.complex128).copy()
                d[i] += 1j * R.H
                p = R.pixels(cam, X + d[None, 9:12], d[None, 0:9], 9)[0]
                Jk[:, i] = p.imag / R.H
            return Jk

        J0 = jac(np.zeros(12))
        np.testing.assert_allclose(J, J0, rtol=1e-12, atol=1e-12 * np.abs(J0).max())
        H = np.zeros((2, 12, 12))
        for j in range(12):
            e = np.zeros(12)
            e[j] = HR
            H[:, :, j] = (jac(e) - jac(-e)) / (2 * HR)
        Cref = r[0] * H[0] + r[1] * H[1]
        Cref = 0.5 * (Cref + Cref.T)
        assert np.abs(Cm - Cref).max() <= 1e-6 * np.abs(Cref).max()
        pix = R.pixels(cam, X, None, 9)[0].real
        np.testing.assert_allclose(r, pix - s.obs[k], rtol=1e-12, atol=1e-9)


def dense_exact_hessian(s, cams, pts):
    """Hessian of delta -> F(theta (+) delta) at 0 by central differences of
    the complex-step gradient, over [cameras (9 each), points (3 each)]."""
    nc, npt = s.n_cams, s.n_pts
    n = 9 * nc + 3 * npt
    w = np.ones(s.n_obs) if s.obs_w is None else s.obs_w

    def F_of(delta):
        dcam = delta[:9 * nc].reshape(nc, 9)
        dpt = delta[9 * nc:].reshape(npt, 3)
        p = tangent_pixels(cams.astype(np.complex128), pts.astype(np.complex128), s.cam_idx,
                           s.pt_idx, dcam, dpt)
        rr = p - s.obs
        return 0.5 * np.sum(w * np.sum(rr * rr, axis=1))

    def grad(dreal):
        g = np.zeros(n)
        for i in range(n):
            d = dreal.astype(np.complex128).copy()
            d[i] += 1j * R.H
            g[i] = F_of(d).imag / R.H
        return g

    Hm = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = HR
        Hm[:, j] = (grad(e) - grad(-e)) / (2 * HR)
    return 0.5 * (Hm + Hm.T), grad(np.zeros(n))


@pytest.mark.slow
def test_adjoint_matches_dense_exact_hessian_solve():
    s = tiny_scene(seed=3)
    o = solve_to_stationary(s)
    cams, pts = o.get_params()
    Hm, g = dense_exact_hessian(s, cams, pts)
    nc = s.n_cams
    free = np.ones(Hm.shape[0], bool)
    for a in s.fixed_cams:
        free[9 * a:9 * a + 9] = False
    assert np.abs(g[free]).max() < 1e-4
    rng = np.random.default_rng(1)
    gLc = rng.normal(size=(nc, 9))
    gLc[s.fixed_cams] = 0
    gLp = rng.normal(size=(s.n_pts, 3))
    gL = np.concatenate([gLc.reshape(-1), gLp.reshape(-1)])
    v = np.zeros_like(gL)
    v[free] = np.linalg.solve(Hm[np.ix_(free, free)], gL[free])
    dx, dw, vc, vp = o.backward(gLc, gLp)
    vo = np.concatenate([vc.reshape(-1), vp.reshape(-1)])
    assert np.linalg.norm(vo - v) <= 1e-6 * np.linalg.norm(v)
    Jc, Jp = R.jacobian_blocks(cams, pts, s.cam_idx, s.pt_idx, 9)
    Jc[np.isin(s.cam_idx, s.fixed_cams)] = 0
    e = (np.einsum("kij,kj->ki", Jc, v[:9 * nc].reshape(nc, 9)[s.cam_idx])
         + np.einsum("kij,kj->ki", Jp, v[9 * nc:].reshape(-1, 3)[s.pt_idx]))
    r = R.pixels(cams[s.cam_idx], pts[s.pt_idx], None, 9).real - s.obs
    np.testing.assert_allclose(dx, s.obs_w[:, None] * e, rtol=1e-6, atol=1e-6 * np.abs(dx).max())
    np.testing.assert_allclose(dw, -np.sum(r * e, axis=1), rtol=1e-6, atol=1e-6 * np.abs(dw).max())


def central(f, h):
    return (f(h) - f(-h)) / (2 * h)


def ring16_scene():
    """The 16-camera workload (1,024 points, 4,096 observations) with the same
    weights U(0.5, 1.5) and fixed cameras 0 and 1."""
    s = make_scene(0)
    s.obs_w = np.random.default_rng([7, 16]).uniform(0.5, 1.5, s.n_obs)
    s.fixed_cams = np.array([0, 1], np.int32)
    return s


@pytest.mark.parametrize("scene", ["six_cameras", "ring16"])
def test_adjoint_matches_finite_differences_through_the_solver(scene):
    s = tiny_scene(seed=2) if scene == "six_cameras" else ring16_scene()
    o = solve_to_stationary(s)
    cams, pts = o.get_params()
    gLc, gLp = loss_tangent_gradient(o, s)
    dx, dw, _, _ = o.backward(gLc, gLp)
    # central differences at 1e-3 (pixels and weights): truncation ~1e-9
    # relative once the re-solve reaches the optimum to round-off
    tol_x = 1e-6 * 5e-2 * np.abs(dx).max()
    tol_w = 1e-6 * 5e-2 * np.abs(dw).max()

    def resolved_loss(obs=None, w=None):
        o2 = solve_to_stationary(s, obs=obs, w=w, cams=cams, pts=pts, iters=30)
        c2, p2 = o2.get_params()
        return loss(c2, p2, s)

    rng = np.random.default_rng(5)
    for k in rng.choice(s.n_obs, 4, replace=False):
        for m in range(2):
            def fx(h):
                obs = s.obs.copy()
                obs[k, m] += h
                return resolved_loss(obs=obs)
            fd = central(fx, 1e-3)
            assert abs(fd - dx[k, m]) <= max(1e-6 * abs(fd), tol_x), (k, m, fd, dx[k, m])

        def fw(h):
            w = s.obs_w.copy()
            w[k] += h
            return resolved_loss(w=w)
        fd = central(fw, 1e-3)
        assert abs(fd - dw[k]) <= max(1e-6 * abs(fd), tol_w), (k, fd, dw[k])


def test_gauss_newton_hessian_is_caught_by_finite_differences():
    """Planted mistake: the adjoint with the curvature term dropped misses the
    finite-difference derivative by far more than the tolerance above."""
    s = tiny_scene(seed=2)
    o = solve_to_stationary(s)
    cams, pts = o.get_params()
    gLc, gLp = loss_tangent_gradient(o, s)
    dx, _, _, _ = o.backward(gLc, gLp)
    # Gauss-Newton adjoint from the oracle's own blocks (curvature removed)
    nc, npt = s.n_cams, s.n_pts
    n = 9 * nc + 3 * npt
    Hgn = np.zeros((n, n))
    Js = []
    for k in range(s.n_obs):
        r, J, _ = o.obs_second_order(k)
        a, j = s.cam_idx[k], s.pt_idx[k]
        if a in s.fixed_cams:
            J[:, :9] = 0
        idx = np.r_[9 * a:9 * a + 9, 9 * nc + 3 * j:9 * nc + 3 * j + 3]
        Hgn[np.ix_(idx, idx)] += s.obs_w[k] * J.T @ J
        Js.append((idx, J))
    free = np.ones(n, bool)
    for a in s.fixed_cams:
        free[9 * a:9 * a + 9] = False
    gL = np.concatenate([gLc.reshape(-1), gLp.reshape(-1)])
    v = np.zeros(n)
    v[free] = np.linalg.solve(Hgn[np.ix_(free, free)], gL[free])
    dx_gn = np.array([s.obs_w[k] * (J @ v[idx]) for k, (idx, J) in enumerate(Js)])
    assert np.abs(dx_gn - dx).max() > 1e-3 * np.abs(dx).max()


def test_weight_derivative_is_orthogonal_to_the_weights():
    """Scaling every weight by c scales F by c and leaves its minimiser in
    place, so any loss of the solution has zero derivative along omega:
    sum_k omega_k dL/d omega_k = 0 (up to the solve's round-off)."""
    s = tiny_scene(seed=3)
    o = solve_to_stationary(s)
    gLc, gLp = loss_tangent_gradient(o, s)
    _, dw, _, _ = o.backward(gLc, gLp)
    terms = s.obs_w * dw
    assert np.abs(terms).max() > 1e-6                       # a loss that does depend on the weights
    assert abs(terms.sum()) <= 1e-8 * np.abs(terms).sum(), (terms.sum(), np.abs(terms).sum())


def test_envelope_case_loss_equal_to_the_objective():
    """L = F: at the optimum dF/dx = 0, so the adjoint's implicit part
    vanishes for that loss, and the derivative of the optimal cost F* along
    omega_k is the explicit term (1/2) |r_k|^2 alone (checked by central
    differences of F*, re-solving at each perturbed weight)."""
    s = tiny_scene(seed=3)
    o = solve_to_stationary(s)
    cams, pts = o.get_params()
    o.compute_step()                                        # linearisation at the optimum
    r, _, _, _, F = o.linearization()
    _, _, gc, gp = o.normal()
    explicit = 0.5 * np.sum(r * r, axis=1)
    _, dw_impl, _, _ = o.backward(gc, gp)
    assert np.abs(dw_impl).max() <= 1e-8 * explicit.max(), (np.abs(dw_impl).max(), explicit.max())

    def optimal_cost(h, k):
        w = s.obs_w.copy()
        w[k] += h
        return solve_to_stationary(s, w=w, cams=cams, pts=pts, iters=30).cost()

    rng = np.random.default_rng(11)
    for k in rng.choice(s.n_obs, 4, replace=False):
        fd = central(lambda h: optimal_cost(h, k), 1e-3)
        assert abs(fd - explicit[k]) <= 1e-6 * max(abs(fd), explicit.max()), (k, fd, explicit[k])
