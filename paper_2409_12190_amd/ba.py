"""Python binding of the C ABI in include/ba.h (argument marshalling only).

Every step of the LM iteration runs in the gfx950 kernels of libba.so; this
module only converts arguments.  PyTorch provides the device memory (one
workspace tensor per problem) and the HIP stream.  Loading fails loudly if
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libba.so")

BA_OK, BA_EINVAL, BA_ENUMERIC, BA_EHIP, BA_ENOTCONV, BA_ESTATE, BA_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
BA_FP64, BA_MIXED = 0, 1
BA_CG_PIPELINED, BA_CG_STANDARD = 0, 1
(BA_X_RESIDUAL, BA_X_WEIGHT, BA_X_JC, BA_X_JP, BA_X_COST, BA_X_GRAD_C, BA_X_GRAD_P, BA_X_V,
 BA_X_S_PTR, BA_X_S_COL, BA_X_S, BA_X_BS, BA_X_DC, BA_X_DP, BA_X_ADJ_VC, BA_X_ADJ_VP,
 BA_X_PRECOND, BA_X_PLAN) = range(1, 19)
PCG_LAYOUTS = {0: "resident", 1: "per_item", 2: "streamed"}
BA_PRECOND_BLOCK_JACOBI, BA_PRECOND_LEARNED = 0, 1
BA_SOLVER_PCG, BA_SOLVER_CHOLESKY = 0, 1
BA_ORDER_BANDWIDTH, BA_ORDER_GIVEN = 0, 1
(BA_STOP_NONE, BA_STOP_MAX_ITERS, BA_STOP_PLATEAU, BA_STOP_GRADIENT, BA_STOP_LAMBDA_MAX,
 BA_STOP_ERROR) = range(6)
BA_GNN_FEATURES, BA_GNN_HIDDEN, BA_GNN_OUTPUTS, BA_GNN_LAYERS = 47, 64, 45, 3

EXPORTED_SYMBOLS = [
    "ba_default_options", "ba_problem_create", "ba_problem_workspace_bytes", "ba_problem_bind",
    "ba_set_observations", "ba_set_fixed_cameras", "ba_set_params", "ba_get_params",
    "ba_set_lambda", "ba_get_lambda", "ba_set_cg", "ba_lm_step", "ba_solve", "ba_backward",
    "ba_get_state", "ba_set_state", "ba_export", "ba_problem_nnzb", "ba_set_profiling",
    "ba_set_profiling_mask", "ba_get_phase_times", "ba_problem_destroy", "ba_last_error", "ba_gnn_num_params",
    "ba_set_gnn_params", "ba_graph_create", "ba_graph_workspace_bytes", "ba_graph_bind",
    "ba_graph_build", "ba_gnn_loss_grad", "ba_gnn_adam", "ba_graph_destroy", "ba_problem_bind_static",
    "ba_pgo_create", "ba_pgo_set_edges", "ba_pgo_set_poses", "ba_pgo_get_poses",
]
BA_STATIC_SCRATCH_BYTES = 64 << 20
BA_NUM_PHASES = 13
PHASE_NAMES = ["linearize", "reduce_cost", "damp_points", "point_q", "camera_vec", "schur_pairs",
               "camera_finish", "pcg", "backsub", "retract_cameras", "candidate_cost", "finalize",
               "precond_net"]


class BaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ba status {status}: {msg}")
        self.status = status


class ba_options(C.Structure):
    _fields_ = [("cam_dof", C.c_int32), ("precision", C.c_int32), ("huber_delta", C.c_double),
                ("cg_rtol", C.c_double), ("cg_maxiter", C.c_int32), ("lambda0", C.c_double),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double), ("diag_min", C.c_double),
                ("diag_max", C.c_double), ("cg_variant", C.c_int32), ("enable_backward", C.c_int32),
                ("adjoint_rtol", C.c_double), ("precond", C.c_int32),
                ("adjoint_grad_tol", C.c_double), ("linear_solver", C.c_int32),
                ("camera_order", C.c_int32)]


class ba_step_info(C.Structure):
    _fields_ = [("cost_before", C.c_double), ("cost_after", C.c_double),
                ("lambda_used", C.c_double), ("lambda_next", C.c_double),
                ("cg_rel_resid", C.c_double), ("pred", C.c_double), ("grad_inf", C.c_double),
                ("accepted", C.c_int32), ("cg_iters", C.c_int32), ("cg_breakdown", C.c_int32),
                ("status", C.c_int32), ("precond_used", C.c_int32), ("stop_reason", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded libba.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        P, S = C.c_void_p, C.c_int
        L.ba_default_options.argtypes = [C.POINTER(ba_options)]
        L.ba_default_options.restype = None
        L.ba_problem_create.argtypes = [C.POINTER(ba_options), C.c_int32, C.c_int32, C.c_int64, P, P,
                                        C.POINTER(P)]
        L.ba_problem_workspace_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
        L.ba_problem_bind.argtypes = [P, P, C.c_size_t, P]
        L.ba_problem_bind_static.argtypes = [P, P]
        L.ba_set_observations.argtypes = [P, P, P]
        L.ba_set_fixed_cameras.argtypes = [P, P]
        L.ba_set_params.argtypes = [P, P, P]
        L.ba_get_params.argtypes = [P, P, P]
        L.ba_set_lambda.argtypes = [P, C.c_double]
        L.ba_get_lambda.argtypes = [P, C.POINTER(C.c_double)]
        L.ba_set_cg.argtypes = [P, C.c_double, C.c_int32]
        L.ba_lm_step.argtypes = [P, C.POINTER(ba_step_info)]
        L.ba_solve.argtypes = [P, C.c_int32, C.c_double, C.c_int32, C.POINTER(ba_step_info),
                               C.POINTER(C.c_int32)]
        L.ba_backward.argtypes = [P, P, P, P, P, C.POINTER(ba_step_info)]
        L.ba_get_state.argtypes = [P, P, C.POINTER(C.c_size_t)]
        L.ba_set_state.argtypes = [P, P, C.c_size_t]
        L.ba_export.argtypes = [P, C.c_int32, P, C.c_size_t]
        L.ba_problem_nnzb.argtypes = [P, C.POINTER(C.c_int64)]
        L.ba_set_profiling.argtypes = [P, C.c_int32]
        L.ba_set_profiling_mask.argtypes = [P, C.c_uint32]
        L.ba_get_phase_times.argtypes = [P, P, P, C.c_int32]
        L.ba_problem_destroy.argtypes = [P]
        L.ba_problem_destroy.restype = None
        L.ba_gnn_num_params.argtypes = []
        L.ba_gnn_num_params.restype = C.c_int64
        L.ba_set_gnn_params.argtypes = [P, P]
        L.ba_graph_create.argtypes = [P, C.POINTER(P)]
        L.ba_graph_workspace_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
        L.ba_graph_bind.argtypes = [P, P, C.c_size_t, P]
        L.ba_graph_build.argtypes = [P, P]
        L.ba_gnn_loss_grad.argtypes = [P, P, P, C.POINTER(C.c_double)]
        L.ba_gnn_adam.argtypes = [C.c_int64, P, P, P, P, C.c_int32, C.c_float, C.c_float, C.c_float,
                                  C.c_float, C.c_float, P]
        L.ba_graph_destroy.argtypes = [P]
        L.ba_graph_destroy.restype = None
        L.ba_pgo_create.argtypes = [C.POINTER(ba_options), C.c_int32, C.c_int64, P, P, C.POINTER(P)]
        L.ba_pgo_set_edges.argtypes = [P, P, P]
        L.ba_pgo_set_poses.argtypes = [P, P]
        L.ba_pgo_get_poses.argtypes = [P, P]
        L.ba_last_error.argtypes = []
        L.ba_last_error.restype = C.c_char_p
        for name in EXPORTED_SYMBOLS:
            if name not in ("ba_default_options", "ba_problem_destroy", "ba_last_error",
                            "ba_gnn_num_params", "ba_graph_destroy"):
                getattr(L, name).restype = S
        _lib = L
    return _lib


def _check(status: int):
    if status != BA_OK:
        raise BaError(status, lib().ba_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


# ---- functions with the C names (marshalling only) ----------------------------

def ba_default_options() -> ba_options:
    o = ba_options()
    lib().ba_default_options(C.byref(o))
    return o


def ba_problem_create(opt: ba_options, n_cams: int, n_pts: int, cam_idx, pt_idx) -> int:
    ci = np.ascontiguousarray(cam_idx, np.int32)
    pi = np.ascontiguousarray(pt_idx, np.int32)
    if ci.shape != pi.shape:
        raise ValueError("cam_idx and pt_idx differ in length")
    h = C.c_void_p()
    _check(lib().ba_problem_create(C.byref(opt), n_cams, n_pts, ci.size, ci.ctypes.data,
                                   pi.ctypes.data, C.byref(h)))
    return h.value


def ba_pgo_create(opt: ba_options, n_poses: int, ei, ej) -> int:
    a = np.ascontiguousarray(ei, np.int32)
    b = np.ascontiguousarray(ej, np.int32)
    if a.shape != b.shape:
        raise ValueError("ei and ej differ in length")
    h = C.c_void_p()
    _check(lib().ba_pgo_create(C.byref(opt), int(n_poses), int(a.size), a.ctypes.data, b.ctypes.data,
                               C.byref(h)))
    return h.value


def ba_pgo_set_edges(h: int, T, omega=None):
    _check(lib().ba_pgo_set_edges(h, _ptr(T), _ptr(omega)))


def ba_pgo_set_poses(h: int, poses):
    _check(lib().ba_pgo_set_poses(h, _ptr(poses)))


def ba_pgo_get_poses(h: int, poses):
    _check(lib().ba_pgo_get_poses(h, _ptr(poses)))


def ba_problem_workspace_bytes(h: int) -> int:
    n = C.c_size_t()
    _check(lib().ba_problem_workspace_bytes(h, C.byref(n)))
    return n.value


def ba_problem_nnzb(h: int) -> int:
    n = C.c_int64()
    _check(lib().ba_problem_nnzb(h, C.byref(n)))
    return n.value


def ba_problem_bind(h: int, workspace_ptr: int, nbytes: int, stream_ptr: Optional[int]):
    _check(lib().ba_problem_bind(h, workspace_ptr, nbytes, stream_ptr))


def ba_problem_bind_static(h: int, stream_ptr: Optional[int]):
    _check(lib().ba_problem_bind_static(h, stream_ptr))


def ba_set_observations(h: int, obs_xy, obs_w=None):
    _check(lib().ba_set_observations(h, _ptr(obs_xy), _ptr(obs_w)))


def ba_set_fixed_cameras(h: int, mask: Optional[np.ndarray]):
    m = None if mask is None else np.ascontiguousarray(mask, np.uint8)
    _check(lib().ba_set_fixed_cameras(h, None if m is None else m.ctypes.data))


def ba_set_params(h: int, cams, pts):
    _check(lib().ba_set_params(h, _ptr(cams), _ptr(pts)))


def ba_get_params(h: int, cams, pts):
    _check(lib().ba_get_params(h, _ptr(cams), _ptr(pts)))


def ba_set_lambda(h: int, lam: float):
    _check(lib().ba_set_lambda(h, lam))


def ba_get_lambda(h: int) -> float:
    v = C.c_double()
    _check(lib().ba_get_lambda(h, C.byref(v)))
    return v.value


def ba_set_cg(h: int, rtol: float, maxiter: int):
    _check(lib().ba_set_cg(h, rtol, maxiter))


def ba_lm_step(h: int) -> dict:
    info = ba_step_info()
    st = lib().ba_lm_step(h, C.byref(info))
    d = info.as_dict()
    d["status"] = st
    if st != BA_OK and st != BA_ENUMERIC:
        _check(st)
    return d


def ba_solve(h: int, max_iters: int, rel_tol: float = 1e-6, plateau_steps: int = 5):
    infos = (ba_step_info * max(1, max_iters))()
    done = C.c_int32()
    st = lib().ba_solve(h, max_iters, rel_tol, plateau_steps, infos, C.byref(done))
    return st, [infos[i].as_dict() for i in range(done.value)]


def ba_backward(h: int, dL_dcams, dL_dpts, dL_dobs, dL_dw=None) -> dict:
    info = ba_step_info()
    st = lib().ba_backward(h, _ptr(dL_dcams), _ptr(dL_dpts), _ptr(dL_dobs), _ptr(dL_dw),
                           C.byref(info))
    _check(st)
    return info.as_dict()


def ba_get_state(h: int) -> bytes:
    n = C.c_size_t()
    _check(lib().ba_get_state(h, None, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(lib().ba_get_state(h, buf, C.byref(n)))
    return buf.raw


def ba_set_state(h: int, blob: bytes):
    buf = C.create_string_buffer(blob, len(blob))
    _check(lib().ba_set_state(h, buf, len(blob)))


def ba_export(h: int, field: int, out: np.ndarray) -> np.ndarray:
    _check(lib().ba_export(h, field, out.ctypes.data, out.nbytes))
    return out


def ba_set_profiling(h: int, enable: bool):
    _check(lib().ba_set_profiling(h, 1 if enable else 0))


def ba_set_profiling_mask(h: int, mask: int):
    _check(lib().ba_set_profiling_mask(h, mask))


def ba_get_phase_times(h: int):
    ms = np.zeros(BA_NUM_PHASES)
    n = np.zeros(BA_NUM_PHASES, np.int64)
    _check(lib().ba_get_phase_times(h, ms.ctypes.data, n.ctypes.data, BA_NUM_PHASES))
    return ms, n


def ba_problem_destroy(h: int):
    lib().ba_problem_destroy(h)


# ---- convenience wrapper holding the torch-owned memory -----------------------

def _release(destroy, handle, stream, workspace):
    """Finalizer of a Problem or Graph: waits for the handle's stream, then
    destroys the handle, while the HIP runtime and this module are still
    alive (weakref.finalize runs leftover finalizers at interpreter exit,
    before module globals are cleared).  The workspace tensor is held until
    the handle is gone, since queued kernels may still use it."""
    if stream is not None:
        try:
            stream.synchronize()
        except Exception:
            pass
    destroy(handle)
    del workspace


class Problem:
    """One bundle-adjustment problem on the current CUDA (HIP) device.

    cam_idx / pt_idx: host integer arrays; obs_xy: float64 [n_obs, 2] and
    obs_w: float64 [n_obs] (or None), host or device; cams [n_cams, 10] and
    pts [n_pts, 3] float64 initial parameters."""

    def __init__(self, n_cams, n_pts, cam_idx, pt_idx, obs_xy, obs_w=None, *, precision=BA_FP64,
                 huber_delta=0.0, cg_rtol=1e-4, cg_maxiter=250, lambda0=1e-4, fixed_cams=None,
                 cams=None, pts=None, stream=None, cg_variant=BA_CG_PIPELINED,
                 enable_backward=False, adjoint_rtol=1e-10, precond=BA_PRECOND_BLOCK_JACOBI,
                 lambda_min=None, lambda_max=None, adjoint_grad_tol=None, cam_dof=9,
                 linear_solver=BA_SOLVER_PCG, static_workspace=False, camera_order=BA_ORDER_BANDWIDTH):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device())
        opt = ba_default_options()
        opt.precision = precision
        opt.huber_delta = huber_delta
        opt.cg_rtol = cg_rtol
        opt.cg_maxiter = cg_maxiter
        opt.lambda0 = lambda0
        opt.cg_variant = cg_variant
        opt.enable_backward = 1 if enable_backward else 0
        opt.adjoint_rtol = adjoint_rtol
        opt.precond = precond
        opt.cam_dof = cam_dof
        opt.linear_solver = linear_solver
        opt.camera_order = camera_order
        if lambda_min is not None:
            opt.lambda_min = lambda_min
        if lambda_max is not None:
            opt.lambda_max = lambda_max
        if adjoint_grad_tol is not None:
            opt.adjoint_grad_tol = adjoint_grad_tol
        self.opt = opt
        self.n_cams, self.n_pts = int(n_cams), int(n_pts)
        self.n_obs = int(np.asarray(cam_idx).size)
        self.h = ba_problem_create(opt, self.n_cams, self.n_pts, cam_idx, pt_idx)
        self._finalizer = weakref.finalize(self, _release, lib().ba_problem_destroy, self.h, None, None)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if static_workspace:
            # the library's fixed device scratch: nothing allocated here
            self.workspace = None
            ba_problem_bind_static(self.h, self.stream.cuda_stream)
        else:
            nbytes = ba_problem_workspace_bytes(self.h)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            if self.workspace.data_ptr() % 256:
                raise RuntimeError("workspace allocation is not 256-byte aligned")
            ba_problem_bind(self.h, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
        self._finalizer.detach()
        self._finalizer = weakref.finalize(self, _release, lib().ba_problem_destroy, self.h,
                                           self.stream, self.workspace)
        self.set_observations(obs_xy, obs_w)
        if fixed_cams is not None and len(fixed_cams):
            mask = np.zeros(self.n_cams, np.uint8)
            mask[np.asarray(fixed_cams)] = 1
            ba_set_fixed_cameras(self.h, mask)
        if cams is not None:
            self.set_params(cams, pts)

    @classmethod
    def from_scene(cls, scene, precision=BA_FP64, **kw):
        kw.setdefault("huber_delta", scene.huber_delta)
        return cls(scene.n_cams, scene.n_pts, scene.cam_idx, scene.pt_idx, scene.obs, scene.obs_w,
                   precision=precision, fixed_cams=scene.fixed_cams, cams=scene.cams0,
                   pts=scene.pts0, **kw)

    def _dev(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(self.device, t.float64).contiguous()
        return t.as_tensor(np.ascontiguousarray(a, np.float64), device=self.device)

    def close(self):
        """Releases the library handle (its pinned staging buffers and timing
        events) after the stream has drained; the workspace tensor is
        dropped with it.  Idempotent; also runs at interpreter exit, before
        module teardown, for problems still alive then."""
        fin = getattr(self, "_finalizer", None)
        if fin is not None:
            fin()
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def set_observations(self, obs_xy, obs_w=None):
        xy = self._dev(obs_xy).reshape(self.n_obs, 2)
        w = None if obs_w is None else self._dev(obs_w).reshape(self.n_obs)
        self.stream.synchronize()
        ba_set_observations(self.h, xy, w)

    @property
    def nnzb(self) -> int:
        return ba_problem_nnzb(self.h)

    def set_params(self, cams, pts):
        c = self._dev(cams).reshape(self.n_cams, 10)
        p = self._dev(pts).reshape(self.n_pts, 3)
        self.stream.synchronize()
        ba_set_params(self.h, c, p)
        self.stream.synchronize()

    def get_params(self):
        t = self.torch
        c = t.empty((self.n_cams, 10), dtype=t.float64, device=self.device)
        p = t.empty((self.n_pts, 3), dtype=t.float64, device=self.device)
        ba_get_params(self.h, c, p)
        self.stream.synchronize()
        return c, p

    def set_lambda(self, lam):
        ba_set_lambda(self.h, lam)

    @property
    def lam(self) -> float:
        return ba_get_lambda(self.h)

    def set_cg(self, rtol, maxiter):
        ba_set_cg(self.h, rtol, maxiter)

    def lm_step(self) -> dict:
        return ba_lm_step(self.h)

    def solve(self, max_iters, rel_tol=1e-6, plateau_steps=5):
        return ba_solve(self.h, max_iters, rel_tol, plateau_steps)

    def backward(self, dL_dcams, dL_dpts, want_dw: bool = True):
        """Implicit-function adjoint at the current (stationary) parameters:
        dL_dcams [n_cams, 10] (gradient w.r.t. the stored camera rows),
        dL_dpts [n_pts, 3]; returns (dL/dobs [n_obs, 2], dL/dw [n_obs] or
        None, info dict)."""
        t = self.torch
        gc = self._dev(dL_dcams).reshape(self.n_cams, 10)
        gp = self._dev(dL_dpts).reshape(self.n_pts, 3)
        dx = t.empty((self.n_obs, 2), dtype=t.float64, device=self.device)
        dw = t.empty(self.n_obs, dtype=t.float64, device=self.device) if want_dw else None
        self.stream.synchronize()
        info = ba_backward(self.h, gc, gp, dx, dw)
        return dx, dw, info

    def set_gnn_params(self, params):
        """Learned preconditioner parameters (device float32 tensor of
        gnn_num_params() values), or None for plain block-Jacobi."""
        if params is None:
            _check(lib().ba_set_gnn_params(self.h, None))
            return
        t = self.torch
        self._gnn = params.detach().to(self.device, t.float32).contiguous()
        self.stream.synchronize()
        _check(lib().ba_set_gnn_params(self.h, self._gnn.data_ptr()))

    def set_profiling(self, enable: bool = True, phases=None):
        """Events around every phase (enable), or only around the named
        phases (PHASE_NAMES entries)."""
        if phases is None:
            ba_set_profiling(self.h, enable)
        else:
            ba_set_profiling_mask(self.h, sum(1 << PHASE_NAMES.index(n) for n in phases) if enable else 0)

    def phase_times(self) -> dict:
        ms, n = ba_get_phase_times(self.h)
        return {name: (float(ms[i]), int(n[i])) for i, name in enumerate(PHASE_NAMES)}

    def get_state(self) -> bytes:
        return ba_get_state(self.h)

    def set_state(self, blob: bytes):
        ba_set_state(self.h, blob)

    @property
    def plan(self) -> dict:
        """How the problem runs: PCG layout and grid, Schur pairs and workgroups."""
        v = self.export(BA_X_PLAN)
        return {"pcg_layout": PCG_LAYOUTS[int(v[0])], "pcg_grid": int(v[1]), "pairs": int(v[2]),
                "schur_workgroups": int(v[3])}

    def export(self, field: int) -> np.ndarray:
        no, nc, np_, nz = self.n_obs, self.n_cams, self.n_pts, self.nnzb
        shapes = {BA_X_RESIDUAL: ((no, 2), np.float64), BA_X_WEIGHT: ((no,), np.float64),
                  BA_X_JC: ((no, 2, 9), np.float64), BA_X_JP: ((no, 2, 3), np.float64),
                  BA_X_COST: ((1,), np.float64), BA_X_GRAD_C: ((nc, 9), np.float64),
                  BA_X_GRAD_P: ((np_, 3), np.float64), BA_X_V: ((np_, 3, 3), np.float64),
                  BA_X_S_PTR: ((nc + 1,), np.int64), BA_X_S_COL: ((nz,), np.int32),
                  BA_X_S: ((nz, 9, 9), np.float64), BA_X_BS: ((nc, 9), np.float64),
                  BA_X_DC: ((nc, 9), np.float64), BA_X_DP: ((np_, 3), np.float64),
                  BA_X_ADJ_VC: ((nc, 9), np.float64), BA_X_ADJ_VP: ((np_, 3), np.float64),
                  BA_X_PRECOND: ((nc, 9, 9), np.float64), BA_X_PLAN: ((4,), np.int64)}
        shape, dt = shapes[field]
        return ba_export(self.h, field, np.zeros(shape, dt))


class PoseGraph:
    """One pose graph (ba_pgo_create) on the current CUDA (HIP) device.

    ei / ej: host integer arrays of the edges' endpoints; T [m, 7] measured
    relative poses and omega [m, 6, 6] information matrices (or None);
    poses [n, 7]; fixed: indices of fixed poses.  The LM iteration is the
    library's (lm_step, solve); the methods mirror Problem's."""

    def __init__(self, n_poses, ei, ej, T, omega=None, poses=None, *, fixed=None, precision=BA_FP64,
                 cg_rtol=1e-4, cg_maxiter=250, lambda0=1e-4, lambda_min=None, lambda_max=None,
                 cg_variant=BA_CG_PIPELINED, linear_solver=BA_SOLVER_PCG, stream=None,
                 static_workspace=False, camera_order=BA_ORDER_BANDWIDTH):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device())
        opt = ba_default_options()
        opt.precision = precision
        opt.cg_rtol = cg_rtol
        opt.cg_maxiter = cg_maxiter
        opt.lambda0 = lambda0
        opt.cg_variant = cg_variant
        opt.linear_solver = linear_solver
        opt.camera_order = camera_order
        if lambda_min is not None:
            opt.lambda_min = lambda_min
        if lambda_max is not None:
            opt.lambda_max = lambda_max
        self.opt = opt
        self.n_poses = int(n_poses)
        self.n_edges = int(np.asarray(ei).size)
        self.h = ba_pgo_create(opt, self.n_poses, ei, ej)
        self._finalizer = weakref.finalize(self, _release, lib().ba_problem_destroy, self.h, None, None)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if static_workspace:
            self.workspace = None
            ba_problem_bind_static(self.h, self.stream.cuda_stream)
        else:
            nbytes = ba_problem_workspace_bytes(self.h)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            if self.workspace.data_ptr() % 256:
                raise RuntimeError("workspace allocation is not 256-byte aligned")
            ba_problem_bind(self.h, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
        self._finalizer.detach()
        self._finalizer = weakref.finalize(self, _release, lib().ba_problem_destroy, self.h,
                                           self.stream, self.workspace)
        self.set_edges(T, omega)
        if fixed is not None and len(fixed):
            mask = np.zeros(self.n_poses, np.uint8)
            mask[np.asarray(fixed)] = 1
            ba_set_fixed_cameras(self.h, mask)
        if poses is not None:
            self.set_poses(poses)

    @classmethod
    def from_graph(cls, g, **kw):
        """From a synth.posegraph.PoseGraph (its initial estimate and fixed poses)."""
        kw.setdefault("fixed", g.fixed)
        return cls(g.n_poses, g.ei, g.ej, g.T, g.omega, g.poses0, **kw)

    _dev = Problem._dev
    close = Problem.close
    __enter__ = Problem.__enter__
    __exit__ = Problem.__exit__
    set_lambda = Problem.set_lambda
    lam = Problem.lam
    set_cg = Problem.set_cg
    lm_step = Problem.lm_step
    solve = Problem.solve
    get_state = Problem.get_state
    set_state = Problem.set_state
    set_profiling = Problem.set_profiling
    phase_times = Problem.phase_times
    plan = Problem.plan
    nnzb = Problem.nnzb

    def set_edges(self, T, omega=None):
        t = self._dev(T).reshape(self.n_edges, 7)
        o = None if omega is None else self._dev(omega).reshape(self.n_edges, 6, 6)
        self.stream.synchronize()
        ba_pgo_set_edges(self.h, t, o)

    def set_poses(self, poses):
        z = self._dev(poses).reshape(self.n_poses, 7)
        self.stream.synchronize()
        ba_pgo_set_poses(self.h, z)
        self.stream.synchronize()

    def get_poses(self):
        t = self.torch
        z = t.empty((self.n_poses, 7), dtype=t.float64, device=self.device)
        ba_pgo_get_poses(self.h, z)
        self.stream.synchronize()
        return z

    def export(self, field: int) -> np.ndarray:
        nc, nz = self.n_poses, self.nnzb
        shapes = {BA_X_COST: (1,), BA_X_GRAD_C: (nc, 9), BA_X_S_PTR: (nc + 1,), BA_X_S_COL: (nz,),
                  BA_X_S: (nz, 9, 9), BA_X_BS: (nc, 9), BA_X_DC: (nc, 9), BA_X_PRECOND: (nc, 9, 9),
                  BA_X_PLAN: (4,)}
        dt = {BA_X_S_PTR: np.int64, BA_X_S_COL: np.int32, BA_X_PLAN: np.int64}.get(field, np.float64)
        return ba_export(self.h, field, np.zeros(shapes[field], dt))


# ---- learned preconditioner: graphs and training --------------------------------

def gnn_num_params() -> int:
    return int(lib().ba_gnn_num_params())


class Graph:
    """Network inputs of one reduced camera system (built from a problem
    created with precond=BA_PRECOND_LEARNED after a step) plus training
    activations, in a torch-owned device workspace."""

    def __init__(self, problem: Problem, stream=None):
        import torch
        self.torch = torch
        h = C.c_void_p()
        _check(lib().ba_graph_create(problem.h, C.byref(h)))
        self.h = h.value
        self._finalizer = weakref.finalize(self, _release, lib().ba_graph_destroy, self.h, None, None)
        n = C.c_size_t()
        _check(lib().ba_graph_workspace_bytes(self.h, C.byref(n)))
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device=problem.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(problem.device)
        _check(lib().ba_graph_bind(self.h, self.workspace.data_ptr(), n.value, self.stream.cuda_stream))
        self._finalizer.detach()
        self._finalizer = weakref.finalize(self, _release, lib().ba_graph_destroy, self.h,
                                           self.stream, self.workspace)
        self.build(problem)

    def build(self, problem: Problem):
        _check(lib().ba_graph_build(self.h, problem.h))

    def loss_grad(self, params, grad) -> float:
        """Adds d loss / d params to grad (device float32); returns the loss."""
        loss = C.c_double()
        self.stream.synchronize()
        _check(lib().ba_gnn_loss_grad(self.h, params.data_ptr(), grad.data_ptr(), C.byref(loss)))
        return loss.value

    def close(self):
        """Releases the graph handle (idempotent; also runs at interpreter
        exit for graphs still alive then)."""
        fin = getattr(self, "_finalizer", None)
        if fin is not None:
            fin()
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False


def gnn_adam(params, grad, m, v, step: int, lr: float = 1e-3, beta1: float = 0.9,
             beta2: float = 0.999, eps: float = 1e-8, grad_scale: float = 1.0, stream=None):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(params.device)
    _check(lib().ba_gnn_adam(params.numel(), params.data_ptr(), grad.data_ptr(), m.data_ptr(),
                             v.data_ptr(), step, lr, beta1, beta2, eps, grad_scale, st.cuda_stream))


# ---- differentiable layer ------------------------------------------------------

def _layer_function():
    import torch

    class _BundleAdjust(torch.autograd.Function):
        """theta* = argmin F(theta; x, w) from the problem's current parameters;
        backward through the implicit-function adjoint (ba_backward)."""

        @staticmethod
        def forward(ctx, obs_xy, obs_w, problem, max_iters, rel_tol, plateau_steps):
            problem.set_observations(obs_xy.detach(), None if obs_w is None else obs_w.detach())
            st, _ = problem.solve(max_iters, rel_tol, plateau_steps)
            if st not in (BA_OK, BA_ENOTCONV):
                _check(st)
            ctx.problem = problem
            ctx.want_dw = obs_w is not None
            cams, pts = problem.get_params()
            return cams, pts

        @staticmethod
        def backward(ctx, g_cams, g_pts):
            p = ctx.problem
            if g_cams is None:
                g_cams = torch.zeros((p.n_cams, 10), dtype=torch.float64, device=p.device)
            if g_pts is None:
                g_pts = torch.zeros((p.n_pts, 3), dtype=torch.float64, device=p.device)
            dx, dw, _ = p.backward(g_cams, g_pts, want_dw=ctx.want_dw)
            return dx, dw, None, None, None, None

    return _BundleAdjust


_LAYER = None


def bundle_adjust(problem: Problem, obs_xy, obs_w=None, max_iters: int = 100, rel_tol: float = 1e-10,
                  plateau_steps: int = 5):
    """Differentiable bundle adjustment: solves from the problem's current
    parameters and returns (cams [n_cams, 10], pts [n_pts, 3]); gradients flow
    to obs_xy and obs_w through the implicit-function adjoint.  The problem
    must be created with enable_backward=True and the squared loss."""
    global _LAYER
    if _LAYER is None:
        _LAYER = _layer_function()
    return _LAYER.apply(obs_xy, obs_w, problem, max_iters, rel_tol, plateau_steps)
