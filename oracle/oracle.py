"""ORACLE -- test infrastructure, not part of the product.

ctypes binding of the plain FP64 CPU oracle in ba_oracle.c.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
this module.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ba_oracle.c")
_SRC_PGO = os.path.join(_HERE, "pgo_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libba_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3 for the generic x86-64 target, OpenMP,
    no fast-math, no FMA contraction: every sum keeps its written order)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=gnu99", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, _SRC_PGO, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Options(C.Structure):
    _fields_ = [("d", C.c_int32), ("huber_delta", C.c_double), ("cg_rtol", C.c_double),
                ("cg_maxiter", C.c_int32), ("lambda0", C.c_double), ("lambda_min", C.c_double),
                ("lambda_max", C.c_double), ("diag_min", C.c_double), ("diag_max", C.c_double),
                ("solver", C.c_int32)]


class StepInfo(C.Structure):
    _fields_ = [("cost_before", C.c_double), ("cost_after", C.c_double),
                ("lambda_used", C.c_double), ("lambda_next", C.c_double),
                ("cg_rel_resid", C.c_double), ("pred", C.c_double), ("grad_inf", C.c_double),
                ("accepted", C.c_int32), ("cg_iters", C.c_int32), ("cg_breakdown", C.c_int32),
                ("status", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _LIB_PATH if os.path.exists(_LIB_PATH) else build(force=False)
        L = C.CDLL(path)
        P = C.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(Options), C.c_int32, C.c_int32, C.c_int64, P, P, P, P, P]
        L.orc_destroy.argtypes = [P]
        L.orc_set_params.argtypes = [P, P, P]
        L.orc_get_params.argtypes = [P, P, P]
        L.orc_set_lambda.argtypes = [P, C.c_double]
        L.orc_get_lambda.argtypes = [P]
        L.orc_get_lambda.restype = C.c_double
        L.orc_nnzb.argtypes = [P]
        L.orc_nnzb.restype = C.c_int64
        L.orc_cost.argtypes = [P, P, P]
        L.orc_cost.restype = C.c_double
        L.orc_compute_step.argtypes = [P, C.c_double, C.c_int32, C.POINTER(StepInfo)]
        L.orc_lm_step.argtypes = [P, C.c_double, C.c_int32, C.POINTER(StepInfo)]
        L.orc_get_linearization.argtypes = [P, P, P, P, P, P]
        L.orc_get_normal.argtypes = [P, P, P, P, P]
        L.orc_get_schur.argtypes = [P, P, P, P, P]
        L.orc_get_step.argtypes = [P, P, P, P]
        L.orc_project.argtypes = [P, P, C.c_int32, P, P, P]
        L.orc_project.restype = C.c_double
        L.orc_retract_camera.argtypes = [P, P, C.c_int32, P]
        L.orc_obs_second_order.argtypes = [P, C.c_int64, P, P, P]
        L.orc_backward.argtypes = [P, P, P, P, P, P, P]
        L.orc_backward.restype = C.c_int
        L.orc_lambda_update.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_lambda_update.restype = C.c_double
        L.orc_solve.argtypes = [P, C.c_int32, C.c_double, C.c_int32, C.c_double, C.c_int32,
                                C.POINTER(StepInfo), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.orc_solve.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_set_threads.restype = None
        L.orc_get_threads.argtypes = []
        L.orc_get_threads.restype = C.c_int32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def project(cam, X, d: int = 9):
    """(pixel[2], Jc[2,d], Jp[2,3], Y_z) of one observation."""
    cam = np.ascontiguousarray(cam, np.float64)
    X = np.ascontiguousarray(X, np.float64)
    pix = np.zeros(2)
    Jc = np.zeros((2, d))
    Jp = np.zeros((2, 3))
    yz = lib().orc_project(_p(cam), _p(X), d, _p(pix), _p(Jc), _p(Jp))
    return pix, Jc, Jp, yz


def retract_camera(cam, delta, d: int = 9):
    cam = np.ascontiguousarray(cam, np.float64)
    delta = np.ascontiguousarray(delta, np.float64)
    out = np.zeros(10)
    lib().orc_retract_camera(_p(cam), _p(delta), d, _p(out))
    return out


def lambda_update(accepted: bool, ratio: float, lam: float, lam_min: float = 1e-12,
                  lam_max: float = 1e12) -> float:
    """The oracle's trust-region damping rule for one step."""
    return lib().orc_lambda_update(1 if accepted else 0, ratio, lam, lam_min, lam_max)


def set_threads(n: int):
    """Threads of the oracle's parallel loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


STOP_NAMES = {0: "none", 1: "max_iters", 2: "plateau", 3: "gradient", 4: "lambda_max", 5: "error"}


@dataclass
class OracleOptions:
    d: int = 9
    huber_delta: float = 0.0
    cg_rtol: float = 1e-4
    cg_maxiter: int = 250
    lambda0: float = 1e-4
    lambda_min: float = 1e-12
    lambda_max: float = 1e12
    diag_min: float = 1e-6
    diag_max: float = 1e32
    solver: int = 0   # 0 PCG, 1 dense Cholesky of the reduced camera system

    def c(self) -> Options:
        return Options(self.d, self.huber_delta, self.cg_rtol, self.cg_maxiter, self.lambda0,
                       self.lambda_min, self.lambda_max, self.diag_min, self.diag_max,
                       self.solver)


class Oracle:
    """One BA problem held by the C oracle."""

    def __init__(self, n_cams, n_pts, cam_idx, pt_idx, obs, obs_w=None, fixed=None,
                 options: OracleOptions | None = None):
        self.opt = options or OracleOptions()
        self.d = self.opt.d
        self.nc, self.np = int(n_cams), int(n_pts)
        self._cidx = np.ascontiguousarray(cam_idx, np.int32)
        self._pidx = np.ascontiguousarray(pt_idx, np.int32)
        self.no = int(self._cidx.size)
        self._obs = np.ascontiguousarray(obs, np.float64).reshape(self.no, 2)
        self._w = None if obs_w is None else np.ascontiguousarray(obs_w, np.float64)
        fx = np.zeros(self.nc, np.uint8)
        if fixed is not None and len(fixed):
            fx[np.asarray(fixed)] = 1
        self._fixed = fx
        self._copt = self.opt.c()
        self._h = lib().orc_create(C.byref(self._copt), self.nc, self.np, self.no,
                                   _p(self._cidx), _p(self._pidx), _p(self._obs),
                                   _p(self._w), _p(self._fixed))

    @classmethod
    def from_scene(cls, scene, **kw):
        opt = kw.pop("options", None) or OracleOptions(huber_delta=scene.huber_delta)
        o = cls(scene.n_cams, scene.n_pts, scene.cam_idx, scene.pt_idx, scene.obs,
                scene.obs_w, scene.fixed_cams, options=opt, **kw)
        o.set_params(scene.cams0, scene.pts0)
        return o

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def set_params(self, cams, pts):
        cams = np.ascontiguousarray(cams, np.float64)
        pts = np.ascontiguousarray(pts, np.float64)
        lib().orc_set_params(self._h, _p(cams), _p(pts))

    def get_params(self):
        cams = np.zeros((self.nc, 10))
        pts = np.zeros((self.np, 3))
        lib().orc_get_params(self._h, _p(cams), _p(pts))
        return cams, pts

    @property
    def lam(self) -> float:
        return lib().orc_get_lambda(self._h)

    @lam.setter
    def lam(self, v: float):
        lib().orc_set_lambda(self._h, float(v))

    def cost(self, cams=None, pts=None) -> float:
        if cams is None:
            cams, pts = self.get_params()
        cams = np.ascontiguousarray(cams, np.float64)
        pts = np.ascontiguousarray(pts, np.float64)
        return lib().orc_cost(self._h, _p(cams), _p(pts))

    def compute_step(self, rtol: float = -1.0, maxiter: int = -1) -> dict:
        info = StepInfo()
        lib().orc_compute_step(self._h, rtol, maxiter, C.byref(info))
        return info.as_dict()

    def lm_step(self, rtol: float = -1.0, maxiter: int = -1) -> dict:
        info = StepInfo()
        lib().orc_lm_step(self._h, rtol, maxiter, C.byref(info))
        return info.as_dict()

    def solve(self, max_iters: int, rel_tol: float = 1e-6, plateau_steps: int = 5,
              rtol: float = -1.0, maxiter: int = -1):
        """LM iterations with the stopping rules of Sec. V; returns
        (status, infos, stop reason name)."""
        infos = (StepInfo * max(1, max_iters))()
        done = C.c_int32()
        why = C.c_int32()
        st = lib().orc_solve(self._h, max_iters, rel_tol, plateau_steps, rtol, maxiter, infos,
                             C.byref(done), C.byref(why))
        n = done.value + (1 if why.value == 5 else 0)
        return st, [infos[i].as_dict() for i in range(n)], STOP_NAMES[why.value]

    def linearization(self):
        r = np.zeros((self.no, 2))
        w = np.zeros(self.no)
        Jc = np.zeros((self.no, 2, self.d))
        Jp = np.zeros((self.no, 2, 3))
        F = C.c_double()
        lib().orc_get_linearization(self._h, _p(r), _p(w), _p(Jc), _p(Jp), C.byref(F))
        return r, w, Jc, Jp, F.value

    def normal(self):
        d = self.d
        U = np.zeros((self.nc, d, d))
        V = np.zeros((self.np, 3, 3))
        gc = np.zeros((self.nc, d))
        gp = np.zeros((self.np, 3))
        lib().orc_get_normal(self._h, _p(U), _p(V), _p(gc), _p(gp))
        return U, V, gc, gp

    def nnzb(self) -> int:
        return int(lib().orc_nnzb(self._h))

    def schur(self):
        d = self.d
        nnzb = self.nnzb()
        ptr = np.zeros(self.nc + 1, np.int64)
        col = np.zeros(nnzb, np.int32)
        S = np.zeros((nnzb, d, d))
        bS = np.zeros((self.nc, d))
        lib().orc_get_schur(self._h, _p(ptr), _p(col), _p(S), _p(bS))
        return ptr, col, S, bS

    def step(self):
        dc = np.zeros((self.nc, self.d))
        dp = np.zeros((self.np, 3))
        Vinv = np.zeros((self.np, 3, 3))
        lib().orc_get_step(self._h, _p(dc), _p(dp), _p(Vinv))
        return dc, dp, Vinv

    def obs_second_order(self, k: int):
        """(r[2], J[2, d+3], C[d+3, d+3]) of observation k at the current
        parameters: residual, Jacobian in the tangent order [camera, point]
        and sum_m r_m Hess(pi_m)."""
        n = self.d + 3
        r = np.zeros(2)
        J = np.zeros((2, n))
        Cm = np.zeros((n, n))
        lib().orc_obs_second_order(self._h, int(k), _p(r), _p(J), _p(Cm))
        return r, J, Cm

    def backward(self, gL_cams, gL_pts):
        """Implicit-function adjoint at the current (stationary) parameters:
        returns (dL/dobs [no, 2], dL/dw [no], v_cams [nc, d], v_pts [np, 3])."""
        gc = np.ascontiguousarray(gL_cams, np.float64).reshape(self.nc, self.d)
        gp = np.ascontiguousarray(gL_pts, np.float64).reshape(self.np, 3)
        dx = np.zeros((self.no, 2))
        dw = np.zeros(self.no)
        vc = np.zeros((self.nc, self.d))
        vp = np.zeros((self.np, 3))
        st = lib().orc_backward(self._h, _p(gc), _p(gp), _p(dx), _p(dw), _p(vc), _p(vp))
        if st != 0:
            raise RuntimeError(f"oracle backward failed ({st})")
        return dx, dw, vc, vp


# ---- pose graph optimisation (pgo_oracle.c) ------------------------------------

class PgoOptions(C.Structure):
    _fields_ = [("cg_rtol", C.c_double), ("cg_maxiter", C.c_int32), ("lambda0", C.c_double),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double), ("diag_min", C.c_double),
                ("diag_max", C.c_double), ("solver", C.c_int32)]


def _pgo_lib():
    L = lib()
    if not getattr(L, "_pgo_bound", False):
        P = C.c_void_p
        L.orc_pgo_create.restype = P
        L.orc_pgo_create.argtypes = [C.POINTER(PgoOptions), C.c_int32, C.c_int32, P, P, P, P, P]
        L.orc_pgo_destroy.argtypes = [P]
        L.orc_pgo_set_poses.argtypes = [P, P]
        L.orc_pgo_get_poses.argtypes = [P, P]
        L.orc_pgo_set_lambda.argtypes = [P, C.c_double]
        L.orc_pgo_nnzb.argtypes = [P]
        L.orc_pgo_nnzb.restype = C.c_int64
        L.orc_pgo_cost.argtypes = [P, P]
        L.orc_pgo_cost.restype = C.c_double
        L.orc_pgo_lm_step.argtypes = [P, C.c_double, C.c_int32, C.POINTER(StepInfo)]
        L.orc_pgo_get_system.argtypes = [P, P, P, P, P, P]
        L.orc_pgo_edge.argtypes = [P, P, P, P, P]
        L.orc_pgo_retract.argtypes = [P, P, P]
        L.orc_se3_jl_inv.argtypes = [P, P]
        L._pgo_bound = True
    return L


def pgo_edge(Zi, Zj, T):
    """(r[6], d r / d delta_j [6, 6]) of one edge (d r / d delta_i = -that)."""
    Zi, Zj, T = (np.ascontiguousarray(a, np.float64) for a in (Zi, Zj, T))
    r = np.zeros(6)
    J = np.zeros((6, 6))
    _pgo_lib().orc_pgo_edge(_p(Zi), _p(Zj), _p(T), _p(r), _p(J))
    return r, J


def pgo_retract(Z, delta):
    Z, delta = np.ascontiguousarray(Z, np.float64), np.ascontiguousarray(delta, np.float64)
    out = np.zeros(7)
    _pgo_lib().orc_pgo_retract(_p(Z), _p(delta), _p(out))
    return out


def se3_jl_inv(xi):
    xi = np.ascontiguousarray(xi, np.float64)
    out = np.zeros((6, 6))
    _pgo_lib().orc_se3_jl_inv(_p(xi), _p(out))
    return out


class PgoOracle:
    """One pose graph held by the C oracle."""

    def __init__(self, graph, cg_rtol=1e-4, cg_maxiter=250, lambda0=1e-4, lambda_min=1e-12,
                 lambda_max=1e12, diag_min=1e-6, diag_max=1e32, solver=0):
        self._opt = PgoOptions(cg_rtol, cg_maxiter, lambda0, lambda_min, lambda_max, diag_min,
                               diag_max, solver)
        self.n, self.m = int(graph.n_poses), int(graph.n_edges)
        self._i = np.ascontiguousarray(graph.ei, np.int32)
        self._j = np.ascontiguousarray(graph.ej, np.int32)
        self._T = np.ascontiguousarray(graph.T, np.float64)
        self._O = np.ascontiguousarray(graph.omega, np.float64)
        fx = np.zeros(self.n, np.uint8)
        if graph.fixed is not None and len(graph.fixed):
            fx[np.asarray(graph.fixed)] = 1
        self._fx = fx
        self._h = _pgo_lib().orc_pgo_create(C.byref(self._opt), self.n, self.m, _p(self._i), _p(self._j),
                                            _p(self._T), _p(self._O), _p(self._fx))
        self.set_poses(graph.poses0)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _pgo_lib().orc_pgo_destroy(h)
            self._h = None

    def set_poses(self, Z):
        Z = np.ascontiguousarray(Z, np.float64)
        _pgo_lib().orc_pgo_set_poses(self._h, _p(Z))

    def get_poses(self):
        Z = np.zeros((self.n, 7))
        _pgo_lib().orc_pgo_get_poses(self._h, _p(Z))
        return Z

    @property
    def lam(self):
        raise AttributeError("write-only")

    @lam.setter
    def lam(self, v):
        _pgo_lib().orc_pgo_set_lambda(self._h, float(v))

    def cost(self, Z=None):
        Z = self.get_poses() if Z is None else np.ascontiguousarray(Z, np.float64)
        return _pgo_lib().orc_pgo_cost(self._h, _p(Z))

    def lm_step(self, rtol: float = -1.0, maxiter: int = -1) -> dict:
        info = StepInfo()
        _pgo_lib().orc_pgo_lm_step(self._h, rtol, maxiter, C.byref(info))
        return info.as_dict()

    def system(self):
        nnzb = int(_pgo_lib().orc_pgo_nnzb(self._h))
        ptr = np.zeros(self.n + 1, np.int64)
        col = np.zeros(nnzb, np.int32)
        H = np.zeros((nnzb, 6, 6))
        g = np.zeros((self.n, 6))
        dx = np.zeros((self.n, 6))
        _pgo_lib().orc_pgo_get_system(self._h, _p(ptr), _p(col), _p(H), _p(g), _p(dx))
        return ptr, col, H, g, dx
