"""Host-side symbolic analysis of streamed PCG plans, checked without a GPU:
the plan builder is compiled with g++ together with a checker
(tests/native/plan_check.cpp) and run on generated scenes."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from synth.scenes import make_scene

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_12190_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir(ROCM_INC):
        pytest.skip("g++ or the ROCm headers are not available")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_check")
    cmd = ["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INC,
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "native", "plan_check.cpp"), os.path.join(CSRC, "ba_plan.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def run_check(exe, tmp_path, cam, pt, n_cams, n_pts, *mode):
    pre = str(tmp_path / "scene")
    np.array([n_cams, n_pts, len(cam)], dtype=np.int64).tofile(pre + ".hdr")
    np.asarray(cam, dtype=np.int32).tofile(pre + ".cam")
    np.asarray(pt, dtype=np.int32).tofile(pre + ".pt")
    r = subprocess.run([exe, pre, *mode], capture_output=True, text=True, timeout=300)
    return r.returncode, r.stdout.strip()


def test_camera_order_recovers_a_band(checker, tmp_path):
    """Reverse Cuthill-McKee numbering of the cameras: a permutation that
    keeps the blocks; a trajectory whose cameras were shuffled gets back a
    band about as narrow as the trajectory's own, and a multi-lap circuit
    (loop closures between laps at the same phase) gets a band far below
    the lap length."""
    s = make_scene(1, n_cams=1000, n_pts=20000, seed=3)
    rc, out = run_check(checker, tmp_path, s.cam_idx, s.pt_idx, s.n_cams, s.n_pts, "order")
    assert rc == 0, out
    bw_given = int(out.split()[2])
    shuffle = np.random.default_rng(0).permutation(s.n_cams)
    rc, out = run_check(checker, tmp_path, shuffle[s.cam_idx], s.pt_idx, s.n_cams, s.n_pts, "order")
    assert rc == 0, out
    bw_shuffled, bw_rcm = int(out.split()[2]), int(out.split()[3])
    assert bw_shuffled > 5 * bw_given and bw_rcm <= 2 * bw_given, out
    s = make_scene(2, n_cams=2000, n_pts=40000, per_lap=400)
    rc, out = run_check(checker, tmp_path, s.cam_idx, s.pt_idx, s.n_cams, s.n_pts, "order")
    assert rc == 0, out
    assert int(out.split()[2]) > 1000 and int(out.split()[3]) < 200, out


def test_dense_ring_streamed_decomposition(checker, tmp_path):
    """Nearly every camera pair co-visible: block rows too long for
    registers, so the plan streams; senders and received sums are many."""
    s = make_scene(0, n_cams=400, n_pts=40000)
    rc, out = run_check(checker, tmp_path, s.cam_idx, s.pt_idx, s.n_cams, s.n_pts)
    assert rc == 0, out
    assert out.startswith("ok streamed"), out


def test_banded_scene_stays_resident(checker, tmp_path):
    s = make_scene(1, n_cams=300, n_pts=3000, seed=4)
    rc, out = run_check(checker, tmp_path, s.cam_idx, s.pt_idx, s.n_cams, s.n_pts)
    assert rc == 0 and out == "ok resident", out


def clique(n_clique, n_cams, n_pts, seed):
    rng = np.random.default_rng(seed)
    cams, pts = [], []
    for j in range(n_pts):
        c = rng.choice(n_clique, size=rng.integers(2, 12), replace=False)
        cams += c.tolist()
        pts += [j] * len(c)
    return cams, pts


def test_clique_with_unobserved_cameras(checker, tmp_path):
    """300 mutually co-visible cameras next to cameras that see nothing: rows
    with no upper blocks, rows that receive from nearly every sender."""
    cams, pts = clique(300, 380, 20000, 3)
    rc, out = run_check(checker, tmp_path, cams, pts, 380, 20000)
    assert rc == 0, out
    assert out.startswith("ok streamed"), out


def test_clique_beyond_column_capacity_is_not_streamed(checker, tmp_path):
    """500 mutually co-visible cameras: a workgroup's first row alone has
    more block columns than the streamed kernel holds in LDS, so the plan
    carries no streamed decomposition (and is still built)."""
    cams, pts = clique(500, 600, 30000, 3)
    rc, out = run_check(checker, tmp_path, cams, pts, 600, 30000)
    assert rc == 0, out
    assert out.startswith("ok unstreamed"), out


def test_long_tracks_get_chunks_of_their_own(checker, tmp_path):
    """Points seen more than a chunk's 256 observations: the first point, two
    consecutive points and a point after an unobserved one each get one
    chunk, listed as long; no chunk is empty of points (checked by the
    program with the other chunk invariants)."""
    n_cams = 700
    rng = np.random.default_rng(3)
    cams, pts = [], []
    lengths = {0: 600, 1: 300, 2: 257, 4: 400}
    for j in range(40):
        k = lengths.get(j, 0 if j == 3 else int(rng.integers(2, 20)))
        cams.append(np.sort(rng.choice(n_cams, size=k, replace=False)))
        pts.append(np.full(k, j))
    cam, pt = np.concatenate(cams), np.concatenate(pts)
    rc, out = run_check(checker, tmp_path, cam, pt, n_cams, 40)
    assert rc == 0, out


def test_long_track_of_the_ring_workload(checker, tmp_path):
    s = make_scene(0, n_cams=700, n_pts=3000, long_track=600)
    rc, out = run_check(checker, tmp_path, s.cam_idx, s.pt_idx, s.n_cams, s.n_pts)
    assert rc == 0, out
