"""ctypes wrapper of the FP64 CPU oracle (``liblbaref.so``, built from ``lbaref.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's CPU
baseline.  The GPU library and its Python binding never import it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbaref.c")
_LIB = os.path.join(_HERE, "liblbaref.so")

DEFAULT_OPTIONS = dict(iters_round1=5, iters_round2=10, max_trials=10, round2_robust=1,
                       huber2_mono=5.991, huber2_stereo=7.815, chi2_mono=5.991,
                       chi2_stereo=7.815, tau=1e-5)


def build(cc: str = "gcc") -> str:
    """Compile the oracle (-O2, no fast-math) into oracle/liblbaref.so."""
    cmd = [cc, "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
           "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


class Problem(C.Structure):
    _fields_ = [("n_kf", C.c_int32), ("n_pt", C.c_int32), ("n_obs", C.c_int32),
                ("n_levels", C.c_int32),
                ("T_cw", C.POINTER(C.c_double)), ("fixed", C.POINTER(C.c_uint8)),
                ("X_w", C.POINTER(C.c_double)), ("obs_kf", C.POINTER(C.c_int32)),
                ("obs_pt", C.POINTER(C.c_int32)), ("obs_z", C.POINTER(C.c_double)),
                ("obs_type", C.POINTER(C.c_uint8)), ("obs_oct", C.POINTER(C.c_uint8)),
                ("sigma2", C.POINTER(C.c_double)),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("bf", C.c_double)]


class Options(C.Structure):
    _fields_ = [("iters_round1", C.c_int32), ("iters_round2", C.c_int32),
                ("max_trials", C.c_int32), ("round2_robust", C.c_int32),
                ("huber2_mono", C.c_double), ("huber2_stereo", C.c_double),
                ("chi2_mono", C.c_double), ("chi2_stereo", C.c_double), ("tau", C.c_double)]


class LogRec(C.Structure):
    _fields_ = [("round", C.c_int32), ("iter", C.c_int32), ("trial", C.c_int32),
                ("accepted", C.c_int32), ("solve_ok", C.c_int32), ("pad", C.c_int32),
                ("lam", C.c_double), ("F", C.c_double), ("F_trial", C.c_double),
                ("gain", C.c_double)]


_lib = None


def _load(path: str):
    L = C.CDLL(path)
    P, O = C.POINTER(Problem), C.POINTER(Options)
    dp, u8p = C.POINTER(C.c_double), C.POINTER(C.c_uint8)
    L.lbaref_solve.argtypes = [P, O, dp, dp, u8p, dp, C.POINTER(LogRec), C.c_int,
                               C.POINTER(C.c_int)]
    L.lbaref_solve.restype = C.c_int
    L.lbaref_se3_exp.argtypes = [dp, dp, dp]
    L.lbaref_se3_left_jacobian.argtypes = [dp, dp]
    L.lbaref_cholesky.argtypes = [C.c_int, dp]
    L.lbaref_cholesky.restype = C.c_int
    L.lbaref_project.argtypes = [P, dp, dp, C.c_int, dp, dp]
    L.lbaref_project.restype = C.c_int
    L.lbaref_jacobians.argtypes = [P, dp, dp, C.c_int, dp, dp]
    L.lbaref_huber.argtypes = [C.c_double, C.c_double, dp, dp]
    L.lbaref_cost.argtypes = [P, O, dp, dp, u8p, C.c_int]
    L.lbaref_cost.restype = C.c_double
    L.lbaref_flags.argtypes = [P, O, dp, dp, u8p]
    L.lbaref_system.argtypes = [P, O, dp, dp, u8p, C.c_int, C.c_double, dp, dp, dp, dp, dp,
                                dp, dp, dp]
    L.lbaref_system.restype = C.c_int
    L.lbaref_dense_system.argtypes = [P, O, dp, dp, u8p, C.c_int, dp, dp]
    L.lbaref_cost_grad.argtypes = [P, O, dp, dp, dp, dp]
    L.lbaref_cost_grad.restype = C.c_double
    L.lbaref_initial_damping.argtypes = [C.c_double, C.c_double]
    L.lbaref_initial_damping.restype = C.c_double
    L.lbaref_damping_update.argtypes = [C.c_double, C.c_int, dp, dp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _load(_LIB)
    return _lib


class use_library:
    """Context manager that points this module at another build of the oracle (the
    mutation tests load deliberately broken copies through it)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def build_variant(src_text: str, out_path: str, cc: str = "gcc") -> str:
    """Compile modified oracle source text (used by the mutation tests only)."""
    src = out_path[:-3] + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run([cc, "-O1", "-std=c11", "-fPIC", "-shared", "-o", out_path, src, "-lm"],
                   check=True)
    return out_path


def _p(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ct))


class _Bound:
    """Keeps the numpy arrays behind a ``Problem`` alive."""

    def __init__(self, w: dict):
        self.arrs = dict(
            T_cw=np.ascontiguousarray(w["T_cw"], dtype=np.float64).reshape(-1, 12),
            fixed=np.ascontiguousarray(w["fixed"], dtype=np.uint8),
            X_w=np.ascontiguousarray(w["X"], dtype=np.float64).reshape(-1, 3),
            obs_kf=np.ascontiguousarray(w["obs_kf"], dtype=np.int32),
            obs_pt=np.ascontiguousarray(w["obs_pt"], dtype=np.int32),
            obs_z=np.ascontiguousarray(w["obs_z"], dtype=np.float64).reshape(3, -1),
            obs_type=np.ascontiguousarray(w["obs_type"], dtype=np.uint8),
            obs_oct=np.ascontiguousarray(w["obs_oct"], dtype=np.uint8),
            sigma2=np.ascontiguousarray(w["sigma2"], dtype=np.float64),
        )
        a = self.arrs
        cam = np.asarray(w["cam"], dtype=np.float64)
        self.P = Problem(len(a["fixed"]), len(a["X_w"]), len(a["obs_kf"]), len(a["sigma2"]),
                         _p(a["T_cw"], C.c_double), _p(a["fixed"], C.c_uint8),
                         _p(a["X_w"], C.c_double), _p(a["obs_kf"], C.c_int32),
                         _p(a["obs_pt"], C.c_int32), _p(a["obs_z"], C.c_double),
                         _p(a["obs_type"], C.c_uint8), _p(a["obs_oct"], C.c_uint8),
                         _p(a["sigma2"], C.c_double), *[float(x) for x in cam])
        self.K = len(a["fixed"])
        self.M = len(a["X_w"])
        self.N = len(a["obs_kf"])
        self.Kopt = int((a["fixed"] == 0).sum())


def options(**kw) -> Options:
    o = dict(DEFAULT_OPTIONS)
    o.update(kw)
    return Options(*[o[f] for f, _ in Options._fields_])


def solve(w: dict, log_cap: int = 4096, **opts) -> dict:
    """Run the full two-round LM on one window.  Returns final poses (K,12), points
    (M,3), outlier flags (N,), stats and the per-trial log."""
    b = _Bound(w)
    O = options(**opts)
    T = np.zeros((b.K, 12))
    X = np.zeros((b.M, 3))
    fl = np.zeros(b.N, dtype=np.uint8)
    st = np.zeros(12)
    log = (LogRec * log_cap)()
    nlog = C.c_int(0)
    rc = lib().lbaref_solve(C.byref(b.P), C.byref(O), _p(T, C.c_double), _p(X, C.c_double),
                            _p(fl, C.c_uint8), _p(st, C.c_double), log, log_cap, C.byref(nlog))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    recs = [dict(round=r.round, iter=r.iter, trial=r.trial, accepted=bool(r.accepted),
                 solve_ok=bool(r.solve_ok), lam=r.lam, F=r.F, F_trial=r.F_trial, gain=r.gain)
            for r in log[: nlog.value]]
    names = ["F_initial", "F_final", "iters_r1", "iters_r2", "trials", "lambda", "term_r1",
             "term_r2", "n_outliers", "F_end_r1", "F_start_r2", "Kopt"]
    return dict(T=T, X=X, outlier=fl.astype(bool), stats=dict(zip(names, st.tolist())), log=recs)


def se3_exp(xi) -> np.ndarray:
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    R = np.zeros(9)
    t = np.zeros(3)
    lib().lbaref_se3_exp(_p(xi, C.c_double), _p(R, C.c_double), _p(t, C.c_double))
    return np.concatenate([R.reshape(3, 3), t[:, None]], axis=1)


def se3_left_jacobian(xi) -> np.ndarray:
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    J = np.zeros(36)
    lib().lbaref_se3_left_jacobian(_p(xi, C.c_double), _p(J, C.c_double))
    return J.reshape(6, 6)


def cholesky(A) -> np.ndarray | None:
    A = np.array(A, dtype=np.float64, order="C")
    n = A.shape[0]
    rc = lib().lbaref_cholesky(n, _p(A, C.c_double))
    return None if rc else A


def huber(s: float, d2: float) -> tuple[float, float]:
    rho, w = C.c_double(), C.c_double()
    lib().lbaref_huber(s, d2, C.byref(rho), C.byref(w))
    return rho.value, w.value


def project(w: dict, T, X, stereo: bool):
    b = _Bound(w)
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(12)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(3)
    pi = np.zeros(3)
    Xc = np.zeros(3)
    r = lib().lbaref_project(C.byref(b.P), _p(T, C.c_double), _p(X, C.c_double), int(stereo),
                             _p(pi, C.c_double), _p(Xc, C.c_double))
    return pi[:r], Xc


def jacobians(w: dict, T, X, stereo: bool):
    b = _Bound(w)
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(12)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(3)
    Jp = np.zeros(18)
    Jx = np.zeros(9)
    lib().lbaref_jacobians(C.byref(b.P), _p(T, C.c_double), _p(X, C.c_double), int(stereo),
                           _p(Jp, C.c_double), _p(Jx, C.c_double))
    r = 3 if stereo else 2
    return Jp.reshape(3, 6)[:r], Jx.reshape(3, 3)[:r]


def cost(w: dict, T=None, X=None, active=None, robust: bool = True, **opts) -> float:
    b = _Bound(w)
    O = options(**opts)
    T = b.arrs["T_cw"] if T is None else np.ascontiguousarray(T, dtype=np.float64)
    X = b.arrs["X_w"] if X is None else np.ascontiguousarray(X, dtype=np.float64)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    return lib().lbaref_cost(C.byref(b.P), C.byref(O), _p(T, C.c_double), _p(X, C.c_double),
                             _p(act, C.c_uint8), int(robust))


def flags(w: dict, T=None, X=None, **opts) -> np.ndarray:
    b = _Bound(w)
    O = options(**opts)
    T = b.arrs["T_cw"] if T is None else np.ascontiguousarray(T, dtype=np.float64)
    X = b.arrs["X_w"] if X is None else np.ascontiguousarray(X, dtype=np.float64)
    fl = np.zeros(b.N, dtype=np.uint8)
    lib().lbaref_flags(C.byref(b.P), C.byref(O), _p(T, C.c_double), _p(X, C.c_double),
                       _p(fl, C.c_uint8))
    return fl.astype(bool)


def system(w: dict, lam: float, T=None, X=None, active=None, robust: bool = True, **opts) -> dict:
    """Linearisation + damped Schur system + step at (T, X)."""
    b = _Bound(w)
    O = options(**opts)
    T = b.arrs["T_cw"] if T is None else np.ascontiguousarray(T, dtype=np.float64)
    X = b.arrs["X_w"] if X is None else np.ascontiguousarray(X, dtype=np.float64)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    n = 6 * b.Kopt
    S = np.zeros((n, n))
    r = np.zeros(n)
    bp = np.zeros(n)
    Hll = np.zeros((b.M, 9))
    bl = np.zeros((b.M, 3))
    Fmd = np.zeros(2)
    dp = np.zeros(n)
    dl = np.zeros((b.M, 3))
    rc = lib().lbaref_system(C.byref(b.P), C.byref(O), _p(T, C.c_double), _p(X, C.c_double),
                             _p(act, C.c_uint8), int(robust), float(lam), _p(S, C.c_double),
                             _p(r, C.c_double), _p(bp, C.c_double), _p(Hll, C.c_double),
                             _p(bl, C.c_double), _p(Fmd, C.c_double), _p(dp, C.c_double),
                             _p(dl, C.c_double))
    return dict(ok=rc == 0, S=S, r=r, bp=bp, Hll=Hll.reshape(-1, 3, 3), bl=bl, F=Fmd[0],
                maxdiag=Fmd[1], dp=dp, dl=dl)


def dense_system(w: dict, T=None, X=None, active=None, robust: bool = True, **opts):
    b = _Bound(w)
    O = options(**opts)
    T = b.arrs["T_cw"] if T is None else np.ascontiguousarray(T, dtype=np.float64)
    X = b.arrs["X_w"] if X is None else np.ascontiguousarray(X, dtype=np.float64)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    D = 6 * b.Kopt + 3 * b.M
    H = np.zeros((D, D))
    g = np.zeros(D)
    lib().lbaref_dense_system(C.byref(b.P), C.byref(O), _p(T, C.c_double), _p(X, C.c_double),
                              _p(act, C.c_uint8), int(robust), _p(H, C.c_double),
                              _p(g, C.c_double))
    return H, g


def cost_grad(w: dict, xi=None, **opts):
    """Robust cost over all observations at Exp(xi) T and its gradients
    (xi: (K,6) or None; returns F, g_xi (K,6), g_X (M,3), g_z (3,N))."""
    b = _Bound(w)
    O = options(**opts)
    x = None if xi is None else np.ascontiguousarray(xi, dtype=np.float64).reshape(b.K, 6)
    gxi = np.zeros((b.K, 6))
    gX = np.zeros((b.M, 3))
    gz = np.zeros((3, b.N))
    F = lib().lbaref_cost_grad(C.byref(b.P), C.byref(O), _p(x, C.c_double),
                               _p(gxi, C.c_double), _p(gX, C.c_double), _p(gz, C.c_double))
    return F, gxi, gX, gz


def initial_damping(tau: float, max_diag: float) -> float:
    return lib().lbaref_initial_damping(tau, max_diag)


def damping_update(gain: float, accepted: bool, lam: float, nu: float) -> tuple[float, float]:
    """One application of the oracle's damping rule: returns (lambda', nu')."""
    l, n = C.c_double(lam), C.c_double(nu)
    lib().lbaref_damping_update(gain, int(accepted), C.byref(l), C.byref(n))
    return l.value, n.value


# ---------------------------------------------------------------------------------------
# stereo-inertial local bundle adjustment
# ---------------------------------------------------------------------------------------
class Inertial(C.Structure):
    _fields_ = [("n_edges", C.c_int32), ("pad", C.c_int32)] + \
        [(k, C.c_void_p) for k in ("edge_i", "edge_j", "dt", "dR", "dv", "dp", "J_Rg", "J_vg", "J_va", "J_pg",
                                   "J_pa", "bg_bar", "ba_bar", "info", "info_bg", "info_ba", "T_cb")] + \
        [("g", C.c_double * 3)]


VI_KEYS = [("edge_i", np.int32, 1), ("edge_j", np.int32, 1), ("dt", np.float64, 1), ("dR", np.float64, 9),
           ("dv", np.float64, 3), ("dp", np.float64, 3), ("J_Rg", np.float64, 9), ("J_vg", np.float64, 9),
           ("J_va", np.float64, 9), ("J_pg", np.float64, 9), ("J_pa", np.float64, 9), ("bg_bar", np.float64, 3),
           ("ba_bar", np.float64, 3), ("info", np.float64, 81), ("info_bg", np.float64, 1),
           ("info_ba", np.float64, 1)]


class _BoundVI:
    """Keeps the numpy arrays behind an ``Inertial`` alive."""

    def __init__(self, vi: dict):
        self.arrs = {k: np.ascontiguousarray(vi[k], dtype=dt).reshape(-1) for k, dt, _ in VI_KEYS}
        self.arrs["T_cb"] = np.ascontiguousarray(vi["T_cb"], dtype=np.float64).reshape(12)
        n = len(self.arrs["edge_i"])
        for k, _, m in VI_KEYS:
            assert self.arrs[k].size == n * m, k
        self.I = Inertial(n, 0, *[self.arrs[k].ctypes.data for k, _, _ in VI_KEYS],
                          self.arrs["T_cb"].ctypes.data, (C.c_double * 3)(*[float(x) for x in vi["g"]]))


def _vi_lib():
    L = lib()
    if not getattr(L, "_vi_ready", False):
        dp, vp = C.POINTER(C.c_double), C.c_void_p
        IP, P, O = C.POINTER(Inertial), C.POINTER(Problem), C.POINTER(Options)
        L.lbaref_so3_log.argtypes = [dp, dp]
        L.lbaref_so3_jr.argtypes = [dp, dp]
        L.lbaref_so3_jr_inv.argtypes = [dp, dp]
        L.lbaref_vi_residual.argtypes = [IP, C.c_int, vp, vp, vp, vp, vp]
        L.lbaref_vi_jacobian.argtypes = [IP, C.c_int, vp, vp, vp, vp, vp]
        L.lbaref_vi_cost.argtypes = [IP, vp, vp, vp, vp]
        L.lbaref_vi_cost.restype = C.c_double
        L.lbaref_solve_vi.argtypes = [P, O, IP, vp, vp, vp, vp, vp, vp, vp, C.POINTER(LogRec), C.c_int,
                                      C.POINTER(C.c_int)]
        L.lbaref_solve_vi.restype = C.c_int
        L.lbaref_vi_system_step.argtypes = [P, O, IP, vp, vp, vp, vp, vp, C.c_double, vp, vp, vp]
        L.lbaref_vi_system_step.restype = C.c_int
        L._vi_ready = True
    return L


def _d(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def so3_log(R) -> np.ndarray:
    R = _d(R, 9)
    w = np.zeros(3)
    _vi_lib().lbaref_so3_log(_p(R, C.c_double), _p(w, C.c_double))
    return w


def so3_jr(w) -> np.ndarray:
    w = _d(w, 3)
    J = np.zeros(9)
    _vi_lib().lbaref_so3_jr(_p(w, C.c_double), _p(J, C.c_double))
    return J.reshape(3, 3)


def so3_jr_inv(w) -> np.ndarray:
    w = _d(w, 3)
    J = np.zeros(9)
    _vi_lib().lbaref_so3_jr_inv(_p(w, C.c_double), _p(J, C.c_double))
    return J.reshape(3, 3)


def _vi_states(vi, T=None, V=None, BG=None, BA=None, w=None):
    T = _d(w["T_cw"] if T is None else T, (-1, 12))
    V = _d(vi["v"] if V is None else V, (-1, 3))
    BG = _d(vi["bg"] if BG is None else BG, (-1, 3))
    BA = _d(vi["ba"] if BA is None else BA, (-1, 3))
    return T, V, BG, BA


def vi_residual(w: dict, vi: dict, e: int, T=None, V=None, BG=None, BA=None) -> np.ndarray:
    bv = _BoundVI(vi)
    T, V, BG, BA = _vi_states(vi, T, V, BG, BA, w)
    r = np.zeros(15)
    _vi_lib().lbaref_vi_residual(C.byref(bv.I), int(e), T.ctypes.data, V.ctypes.data, BG.ctypes.data,
                                 BA.ctypes.data, r.ctypes.data)
    return r


def vi_jacobian(w: dict, vi: dict, e: int, T=None, V=None, BG=None, BA=None) -> np.ndarray:
    bv = _BoundVI(vi)
    T, V, BG, BA = _vi_states(vi, T, V, BG, BA, w)
    J = np.zeros(450)
    _vi_lib().lbaref_vi_jacobian(C.byref(bv.I), int(e), T.ctypes.data, V.ctypes.data, BG.ctypes.data,
                                 BA.ctypes.data, J.ctypes.data)
    return J.reshape(15, 30)


def vi_cost(w: dict, vi: dict, T=None, V=None, BG=None, BA=None) -> float:
    bv = _BoundVI(vi)
    T, V, BG, BA = _vi_states(vi, T, V, BG, BA, w)
    return _vi_lib().lbaref_vi_cost(C.byref(bv.I), T.ctypes.data, V.ctypes.data, BG.ctypes.data, BA.ctypes.data)


def solve_vi(w: dict, vi: dict, log_cap: int = 4096, **opts) -> dict:
    """The two-round stereo-inertial LM on one window (states v, bg, ba from vi)."""
    b = _Bound(w)
    bv = _BoundVI(vi)
    O = options(**opts)
    T = np.zeros((b.K, 12))
    X = np.zeros((b.M, 3))
    V = _d(vi["v"], (-1, 3)).copy()
    BG = _d(vi["bg"], (-1, 3)).copy()
    BA = _d(vi["ba"], (-1, 3)).copy()
    fl = np.zeros(b.N, dtype=np.uint8)
    st = np.zeros(12)
    log = (LogRec * log_cap)()
    nlog = C.c_int(0)
    rc = _vi_lib().lbaref_solve_vi(C.byref(b.P), C.byref(O), C.byref(bv.I), T.ctypes.data, X.ctypes.data,
                                   V.ctypes.data, BG.ctypes.data, BA.ctypes.data, fl.ctypes.data, st.ctypes.data,
                                   log, log_cap, C.byref(nlog))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    recs = [dict(round=r.round, iter=r.iter, trial=r.trial, accepted=bool(r.accepted),
                 solve_ok=bool(r.solve_ok), lam=r.lam, F=r.F, F_trial=r.F_trial, gain=r.gain)
            for r in log[: nlog.value]]
    names = ["F_initial", "F_final", "iters_r1", "iters_r2", "trials", "lambda", "term_r1",
             "term_r2", "n_outliers", "F_end_r1", "F_start_r2", "Kopt"]
    return dict(T=T, X=X, V=V, BG=BG, BA=BA, outlier=fl.astype(bool), stats=dict(zip(names, st.tolist())),
                log=recs)


def vi_system_step(w: dict, vi: dict, lam: float, T=None, X=None, V=None, BG=None, BA=None, **opts) -> dict:
    """The damped visual-inertial step at a state (no outlier mask, robust): d (15 Kopt)
    and the point step dl (M, 3)."""
    b = _Bound(w)
    bv = _BoundVI(vi)
    O = options(**opts)
    T, V, BG, BA = _vi_states(vi, T, V, BG, BA, w)
    X = _d(w["X"] if X is None else X, (-1, 3))
    d = np.zeros(15 * b.Kopt)
    dl = np.zeros((b.M, 3))
    Fmd = np.zeros(2)
    rc = _vi_lib().lbaref_vi_system_step(C.byref(b.P), C.byref(O), C.byref(bv.I), T.ctypes.data, X.ctypes.data,
                                         V.ctypes.data, BG.ctypes.data, BA.ctypes.data, float(lam), d.ctypes.data,
                                         dl.ctypes.data, Fmd.ctypes.data)
    return dict(ok=rc == 0, d=d, dl=dl, F=Fmd[0])
