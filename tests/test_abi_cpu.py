"""C ABI checks that need no GPU: the library loads, exports every function
include/ba.h declares, validates its inputs, and its host-side symbolic
analysis agrees with the oracle's block pattern."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_12190_amd import ba as B
from synth.scenes import make_scene

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ba.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ba_[a-z_0-9]+)\s*\(", src)))


def test_header_functions_are_exported():
    names = declared_functions()
    assert "ba_lm_step" in names and "ba_problem_create" in names
    lib = B.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTED_SYMBOLS) == names


def test_default_options():
    o = B.ba_default_options()
    assert o.cam_dof == 9 and o.precision == B.BA_FP64
    assert o.cg_rtol == 1e-4 and o.cg_maxiter == 250
    assert o.lambda0 == 1e-4 and o.diag_min == 1e-6


def _create(n_c, n_p, ci, pi, **kw):
    o = B.ba_default_options()
    for k, v in kw.items():
        setattr(o, k, v)
    return B.ba_problem_create(o, n_c, n_p, ci, pi)


def test_create_rejects_bad_indices_and_sizes():
    with pytest.raises(B.BaError) as e:
        _create(3, 3, [0, 1, 3], [0, 1, 2])
    assert e.value.status == B.BA_EINVAL
    with pytest.raises(B.BaError) as e:
        _create(3, 3, [0, 1, 2], [0, -1, 2])
    assert e.value.status == B.BA_EINVAL
    with pytest.raises(B.BaError) as e:
        _create(3, 3, [], [])
    assert e.value.status == B.BA_EINVAL
    with pytest.raises(B.BaError) as e:
        _create(3, 3, [0], [0], cam_dof=7)
    assert e.value.status == B.BA_EUNSUPPORTED
    # the 6-DoF camera: supported, but not with the learned preconditioner or the adjoint
    B.ba_problem_destroy(_create(3, 3, [0, 1, 2], [0, 1, 2], cam_dof=6))
    for kw in (dict(precond=B.BA_PRECOND_LEARNED), dict(enable_backward=1)):
        with pytest.raises(B.BaError) as e:
            _create(3, 3, [0, 1, 2], [0, 1, 2], cam_dof=6, **kw)
        assert e.value.status == B.BA_EUNSUPPORTED


def test_long_tracks_are_accepted():
    # a point seen more than a chunk of 256 observations holds gets a chunk
    # of its own (its kernels are checked on the GPU); its cameras all share
    # a block of S, so n stays within a PCG workgroup's 768 block columns
    for n in (256, 257, 600):
        B.ba_problem_destroy(_create(n, 2, np.r_[np.arange(n), [0]], np.r_[np.zeros(n), [1]]))


def test_state_calls_before_bind_fail():
    s = make_scene(0)
    h = _create(s.n_cams, s.n_pts, s.cam_idx, s.pt_idx)
    try:
        info = B.ba_step_info()
        assert B.lib().ba_lm_step(h, ctypes.byref(info)) == B.BA_ESTATE
        assert B.lib().ba_set_observations(h, None, None) == B.BA_EINVAL
        assert B.lib().ba_backward(h, None, None, None, None, None) == B.BA_ESTATE
    finally:
        B.ba_problem_destroy(h)


@pytest.mark.parametrize("cfg,kw", [(0, {}), (1, dict(n_cams=200, n_pts=3000)),
                                    (2, dict(n_cams=2000, n_pts=20000))])
def test_block_pattern_matches_oracle(cfg, kw):
    s = make_scene(cfg, **kw)
    h = _create(s.n_cams, s.n_pts, s.cam_idx, s.pt_idx)
    try:
        o = O.Oracle.from_scene(s)
        assert B.ba_problem_nnzb(h) == o.nnzb()
        ptr = np.zeros(s.n_cams + 1, np.int64)
        col = np.zeros(o.nnzb(), np.int32)
        assert B.lib().ba_export(h, B.BA_X_S_PTR, ptr.ctypes.data, ptr.nbytes) == B.BA_ESTATE
    finally:
        B.ba_problem_destroy(h)


def test_backward_needs_squared_loss_and_enabled_buffers():
    s = make_scene(0)
    h = _create(s.n_cams, s.n_pts, s.cam_idx, s.pt_idx, huber_delta=1.0, enable_backward=1)
    try:
        assert B.lib().ba_backward(h, None, None, None, None, None) == B.BA_EUNSUPPORTED
    finally:
        B.ba_problem_destroy(h)


def test_backward_buffers_add_to_the_workspace():
    s = make_scene(3, n_cams=40, n_pts=2500)
    # (the caller's camera order: a renumbered problem adds a [n_cams][10]
    # staging copy of dL/dcams)
    g = B.BA_ORDER_GIVEN
    h0 = _create(s.n_cams, s.n_pts, s.cam_idx, s.pt_idx, camera_order=g)
    h1 = _create(s.n_cams, s.n_pts, s.cam_idx, s.pt_idx, enable_backward=1, camera_order=g)
    h2 = _create(s.n_cams, s.n_pts, s.cam_idx, s.pt_idx, enable_backward=1, precision=B.BA_MIXED, camera_order=g)
    h3 = _create(s.n_cams, s.n_pts, s.cam_idx, s.pt_idx, precision=B.BA_MIXED, camera_order=g)
    try:
        nc, np_, no, nz = s.n_cams, s.n_pts, s.n_obs, B.ba_problem_nnzb(h0)
        extra = 8 * (no * (78 + 24 + 27) + nc * (81 + 9 + 9) + np_ * 3)
        d64 = B.ba_problem_workspace_bytes(h1) - B.ba_problem_workspace_bytes(h0)
        d32 = B.ba_problem_workspace_bytes(h2) - B.ba_problem_workspace_bytes(h3)
        assert abs(d64 - extra) < 16 * 256
        assert abs(d32 - extra - 8 * 81 * nz) < 16 * 256   # FP64 copy of S in mixed mode
    finally:
        for h in (h0, h1, h2, h3):
            B.ba_problem_destroy(h)


def test_workspace_grows_linearly_with_observations():
    s = make_scene(1, n_cams=200, n_pts=3000)
    h1 = _create(s.n_cams, s.n_pts, s.cam_idx, s.pt_idx)
    h2 = _create(s.n_cams, s.n_pts, s.cam_idx, s.pt_idx, precision=B.BA_MIXED)
    try:
        b64, b32 = B.ba_problem_workspace_bytes(h1), B.ba_problem_workspace_bytes(h2)
        # FP32 storage of the observation rows (Jacobian blocks, Schur
        # factor, weight: 32 values) and of S saves 4 bytes per stored value
        saved = s.n_obs * 32 * 4 + B.ba_problem_nnzb(h1) * 81 * 4
        assert abs((b64 - b32) - saved) < 64 * 256
    finally:
        B.ba_problem_destroy(h1)
        B.ba_problem_destroy(h2)


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_option_struct_layout_matches_the_binding():
    """ba_default_options fills the last fields of ba_options where the
    binding's ctypes mirror expects them."""
    from paper_2409_12190_amd import ba as B
    o = B.ba_default_options()
    assert o.cam_dof == 9 and o.cg_maxiter == 250 and o.cg_rtol == 1e-4
    assert o.precond == B.BA_PRECOND_BLOCK_JACOBI and o.adjoint_rtol == 1e-10
    assert o.adjoint_grad_tol == 1e-6


def test_pose_graph_create_validates_and_matches_the_oracle_pattern():
    from synth.posegraph import make_pose_graph
    o = B.ba_default_options()
    for ei, ej in (([0, 1], [1, 4]), ([0, -1], [1, 2]), ([0, 2], [1, 2])):
        with pytest.raises(B.BaError) as e:
            B.ba_pgo_create(o, 4, ei, ej)
        assert e.value.status == B.BA_EINVAL
    for k, v in (("huber_delta", 1.0), ("precond", B.BA_PRECOND_LEARNED), ("enable_backward", 1)):
        oo = B.ba_default_options()
        setattr(oo, k, v)
        with pytest.raises(B.BaError) as e:
            B.ba_pgo_create(oo, 4, [0, 1], [1, 2])
        assert e.value.status == B.BA_EUNSUPPORTED
    g = make_pose_graph(1, rings=5, per_ring=7)
    h = B.ba_pgo_create(o, g.n_poses, g.ei, g.ej)
    try:
        assert B.ba_problem_nnzb(h) == O.PgoOracle(g).system()[1].size
        assert B.ba_problem_workspace_bytes(h) > 0
        with pytest.raises(B.BaError) as e:
            B.ba_lm_step(h)
        assert e.value.status == B.BA_ESTATE
    finally:
        B.ba_problem_destroy(h)
