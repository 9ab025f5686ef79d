"""The allocation-free binding (ba_problem_bind_static) through the C ABI:
a problem bound to the device's static scratch runs exactly like the same
problem bound to a caller-allocated workspace, on two problems in a row
(the second smaller, reusing the scratch the first left behind); the first
handle loses the scratch to the second; a problem whose workspace exceeds
the scratch is refused."""
import numpy as np
import pytest

from synth.scenes import make_scene

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2409_12190_amd import ba as B  # noqa: E402


def run(problem, steps):
    infos = [problem.lm_step() for _ in range(steps)]
    c, p = problem.get_params()
    return infos, c.cpu().numpy(), p.cpu().numpy()


def test_static_binding_matches_workspace_binding():
    big = make_scene(0)                                   # 16 cameras, 4,096 observations
    small = make_scene(0, n_cams=8, n_pts=300, seed=5)    # 8 cameras, 1,200 observations
    first = None
    for s in (big, small):
        print(f"[gpu] static scratch: nc={s.n_cams} no={s.n_obs}", flush=True)
        ref = B.Problem.from_scene(s)
        got = B.Problem.from_scene(s, static_workspace=True)
        assert got.workspace is None
        ia, ca, pa = run(ref, 4)
        ib, cb, pb = run(got, 4)
        assert ia == ib                                   # every kernel reduces in a fixed order
        assert np.array_equal(ca, cb) and np.array_equal(pa, pb)
        np.testing.assert_array_equal(got.export(B.BA_X_S), ref.export(B.BA_X_S))
        ref.close()
        if first is None:
            first = got
        else:
            # the second static problem took the scratch: the first is refused
            with pytest.raises(B.BaError) as e:
                first.lm_step()
            assert e.value.status == B.BA_ESTATE
            got.close()
    first.close()


def test_static_binding_refuses_oversize_problems():
    s = make_scene(1)                                     # ~1M observations: far beyond the scratch
    opt = B.ba_default_options()
    h = B.ba_problem_create(opt, s.n_cams, s.n_pts, s.cam_idx, s.pt_idx)
    try:
        need = B.ba_problem_workspace_bytes(h)
        assert need > B.BA_STATIC_SCRATCH_BYTES
        with pytest.raises(B.BaError) as e:
            B.ba_problem_bind_static(h, torch.cuda.current_stream().cuda_stream)
        assert e.value.status == B.BA_EINVAL and "scratch" in str(e.value)
    finally:
        B.ba_problem_destroy(h)
