"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the C oracle (bundle adjustment with both solvers and the adjoint, and the
pose graph) driven by tests/native/oracle_drive.c, and the plan builder
driven by tests/native/plan_check.cpp, each compiled with
-fsanitize=address,undefined and run on generated inputs.  Any report aborts
the program (-fno-sanitize-recover), so the test only has to see exit 0;
oracle_drive's results are also checked against the ordinarily built oracle."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from synth.posegraph import make_pose_graph
from synth.scenes import make_scene

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_12190_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def _build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("the sanitizer runtime is not installed: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_drive")
    _build(["gcc", "-std=gnu99", "-fopenmp", "-ffp-contract=off", *SAN, os.path.join(NATIVE, "oracle_drive.c"),
            os.path.join(ROOT, "oracle", "ba_oracle.c"), os.path.join(ROOT, "oracle", "pgo_oracle.c"), "-lm",
            "-o", exe])
    s = make_scene(0)
    g = make_pose_graph(2, rings=5, per_ring=8)
    pre = str(tmp_path / "in")
    np.array([s.n_cams, s.n_pts, s.n_obs, g.n_poses, g.n_edges], np.int64).tofile(pre + ".hdr")
    np.asarray(s.cam_idx, np.int32).tofile(pre + ".cam")
    np.asarray(s.pt_idx, np.int32).tofile(pre + ".pt")
    np.asarray(s.obs, np.float64).tofile(pre + ".obs")
    np.asarray(s.cams0, np.float64).tofile(pre + ".cams")
    np.asarray(s.pts0, np.float64).tofile(pre + ".pts")
    np.asarray(g.ei, np.int32).tofile(pre + ".ei")
    np.asarray(g.ej, np.int32).tofile(pre + ".ej")
    np.asarray(g.T, np.float64).tofile(pre + ".T")
    np.asarray(g.omega, np.float64).tofile(pre + ".om")
    np.asarray(g.poses0, np.float64).tofile(pre + ".Z")
    r = subprocess.run([exe, pre], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    lines = r.stdout.strip().splitlines()
    assert len(lines) == 5, lines
    got = {}
    for ln in lines:
        f = ln.split()
        got[" ".join(f[:3]) if f[0] != "adjoint" else "adjoint"] = f
    # the same computations through the ordinarily built oracle
    for solver in (0, 1):
        opt = O.OracleOptions(huber_delta=1.0 if solver == 0 else 0.0, cg_rtol=1e-10, cg_maxiter=500,
                              solver=solver)
        o = O.Oracle(s.n_cams, s.n_pts, s.cam_idx, s.pt_idx, s.obs, None, [0, 1], options=opt)
        o.set_params(s.cams0, s.pts0)
        st, infos, _ = o.solve(40, 1e-12, 3)
        last = infos[-1]
        F = last["cost_after"] if last["accepted"] else last["cost_before"]
        f = got[f"ba solver {solver}"]
        assert int(f[4]) == st and int(f[6]) == len(infos)
        assert float(f[10]) == pytest.approx(F, rel=1e-13)
        if solver == 1:
            gc = np.zeros((s.n_cams, 9))
            gc[:, 0] = 1.0
            dx = o.backward(gc, np.zeros((s.n_pts, 3)))[0]
            assert int(got["adjoint"][2]) == 0
            assert float(got["adjoint"][4]) == pytest.approx(float(np.sum(dx)), rel=1e-9, abs=1e-12)
    for solver in (0, 1):
        o = O.PgoOracle(g, cg_rtol=1e-10, cg_maxiter=1000, solver=solver)
        for _ in range(6):
            info = o.lm_step()
        F = info["cost_after"] if info["accepted"] else info["cost_before"]
        assert float(got[f"pgo solver {solver}"][4]) == pytest.approx(F, rel=1e-13)


@pytest.mark.parametrize("which", ["ring_streamed", "pose_graph"])
def test_plan_builder_under_sanitizers(tmp_path, which):
    _need("g++")
    if not os.path.isdir("/opt/rocm/include"):
        pytest.skip("ROCm headers not available")
    exe = str(tmp_path / "plan_check")
    _build(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I",
            os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(NATIVE, "plan_check.cpp"),
            os.path.join(CSRC, "ba_plan.cpp"), "-o", exe])
    if which == "ring_streamed":
        s = make_scene(0, n_cams=300, n_pts=20000)
        nc, npt, cam, pt = s.n_cams, s.n_pts, s.cam_idx, s.pt_idx
    else:
        # a pose graph's plan: each edge is a point seen by its two poses
        g = make_pose_graph(0, rings=20, per_ring=25)
        nc, npt = g.n_poses, g.n_edges
        cam = np.stack([g.ei, g.ej], 1).reshape(-1)
        pt = np.repeat(np.arange(g.n_edges), 2)
    pre = str(tmp_path / "scene")
    np.array([nc, npt, len(cam)], np.int64).tofile(pre + ".hdr")
    np.asarray(cam, np.int32).tofile(pre + ".cam")
    np.asarray(pt, np.int32).tofile(pre + ".pt")
    r = subprocess.run([exe, pre], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert r.stdout.startswith("ok"), r.stdout
