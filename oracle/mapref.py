"""ctypes wrapper of the CPU oracle of the local-mapping searches (``libmapref.so``, built
from ``mapref.c``): keypoint correspondence search, fusion candidate search and the
keyframe-culling counters.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's CPU baseline.  The GPU
library and its Python binding never import it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mapref.c")
_LIB = os.path.join(_HERE, "libmapref.so")

CORR_DEFAULTS = dict(th_low=50, resolve=1, epi_chi2=3.84, epipole_min=100.0)
FUSE_DEFAULTS = dict(th_low=50, radius_th=3.0, chi2_mono=5.991, chi2_stereo=7.815)


def build(cc: str = "gcc") -> str:
    cmd = [cc, "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
           "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


class Store(C.Structure):
    _fields_ = [("n_kf", C.c_int32), ("n_kp", C.c_int32), ("n_levels", C.c_int32), ("width", C.c_int32),
                ("height", C.c_int32), ("pad", C.c_int32), ("kp_off", C.c_void_p), ("T_cw", C.c_void_p),
                ("kp_u", C.c_void_p), ("kp_v", C.c_void_p), ("kp_ur", C.c_void_p), ("kp_oct", C.c_void_p),
                ("kp_free", C.c_void_p), ("kp_desc", C.c_void_p), ("sigma2", C.c_void_p),
                ("scale", C.c_void_p), ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double),
                ("cy", C.c_double), ("bf", C.c_double)]


class CorrParams(C.Structure):
    _fields_ = [("th_low", C.c_int32), ("resolve", C.c_int32), ("epi_chi2", C.c_double),
                ("epipole_min", C.c_double)]


class FuseParams(C.Structure):
    _fields_ = [("th_low", C.c_int32), ("pad", C.c_int32), ("radius_th", C.c_double),
                ("chi2_mono", C.c_double), ("chi2_stereo", C.c_double)]


_lib = None


def _load(path):
    L = C.CDLL(path)
    vp, i32 = C.c_void_p, C.c_int
    L.mapref_hamming.argtypes = [vp, vp]
    L.mapref_hamming.restype = i32
    L.mapref_fundamental.argtypes = [C.POINTER(Store), i32, i32, vp]
    L.mapref_epipole.argtypes = [C.POINTER(Store), i32, i32, vp]
    L.mapref_epipolar_dist2.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double]
    L.mapref_epipolar_dist2.restype = C.c_double
    L.mapref_correspondence.argtypes = [C.POINTER(Store), C.POINTER(CorrParams), i32, vp, vp, vp, vp, vp]
    L.mapref_fusion.argtypes = [C.POINTER(Store), C.POINTER(FuseParams), vp, vp, vp, vp, vp, i32, vp, vp, vp,
                                vp, vp, vp, vp]
    L.mapref_culling.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _load(_LIB)
    return _lib


class use_library:
    """Point this module at another build of the oracle (the mutation tests)."""

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
    src = out_path[:-3] + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run([cc, "-O1", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-o", out_path, src, "-lm"],
                   check=True)
    return out_path


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class _BoundStore:
    def __init__(self, s: dict):
        self.a = dict(kp_off=_c(s["kp_off"], np.int32), T_cw=_c(s["T_cw"], np.float64).reshape(-1, 12),
                      kp_u=_c(s["kp_u"], np.float32), kp_v=_c(s["kp_v"], np.float32),
                      kp_ur=_c(s["kp_ur"], np.float32), kp_oct=_c(s["kp_oct"], np.uint8),
                      kp_free=_c(s["kp_free"], np.uint8), kp_desc=_c(s["kp_desc"], np.uint32).reshape(-1, 8),
                      sigma2=_c(s["sigma2"], np.float64), scale=_c(s["scale"], np.float64))
        a = self.a
        cam = np.asarray(s["cam"], dtype=np.float64)
        self.S = Store(len(a["kp_off"]) - 1, len(a["kp_u"]), len(a["sigma2"]), int(s["width"]), int(s["height"]), 0,
                       *[a[k].ctypes.data for k in ("kp_off", "T_cw", "kp_u", "kp_v", "kp_ur", "kp_oct",
                                                     "kp_free", "kp_desc", "sigma2", "scale")],
                       *[float(x) for x in cam])


def hamming(a, b) -> int:
    a, b = _c(a, np.uint32), _c(b, np.uint32)
    return lib().mapref_hamming(a.ctypes.data, b.ctypes.data)


def fundamental(store: dict, a: int, b: int) -> np.ndarray:
    bs = _BoundStore(store)
    F = np.zeros(9)
    lib().mapref_fundamental(C.byref(bs.S), a, b, F.ctypes.data)
    return F.reshape(3, 3)


def epipole(store: dict, a: int, b: int) -> np.ndarray:
    bs = _BoundStore(store)
    e = np.zeros(2)
    lib().mapref_epipole(C.byref(bs.S), a, b, e.ctypes.data)
    return e


def epipolar_dist2(F, ua, va, ub, vb) -> float:
    F = _c(F, np.float64).reshape(9)
    return lib().mapref_epipolar_dist2(F.ctypes.data, ua, va, ub, vb)


def out_offsets(counts) -> np.ndarray:
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    return off


def correspondence(store: dict, cur, nbr, **params):
    """(match, dist, out_off): per query q the entries out_off[q] .. out_off[q + 1] are the
    keypoints of cur[q] in order."""
    bs = _BoundStore(store)
    p = dict(CORR_DEFAULTS)
    p.update(params)
    P = CorrParams(int(p["th_low"]), int(p["resolve"]), float(p["epi_chi2"]), float(p["epipole_min"]))
    cur, nbr = _c(cur, np.int32), _c(nbr, np.int32)
    ko = bs.a["kp_off"]
    off = out_offsets(ko[cur + 1] - ko[cur])
    match = np.zeros(off[-1], dtype=np.int32)
    dist = np.zeros(off[-1], dtype=np.int32)
    lib().mapref_correspondence(C.byref(bs.S), C.byref(P), len(cur), cur.ctypes.data, nbr.ctypes.data,
                                off.ctypes.data, match.ctypes.data, dist.ctypes.data)
    return match, dist, off


def fusion(store: dict, pts: dict, queries, skip=None, **params):
    """(match, dist, out_off) of the fusion candidate search; queries = (p0, p1, nbr)."""
    bs = _BoundStore(store)
    p = dict(FUSE_DEFAULTS)
    p.update(params)
    P = FuseParams(int(p["th_low"]), 0, float(p["radius_th"]), float(p["chi2_mono"]), float(p["chi2_stereo"]))
    q0, q1, qn = (_c(x, np.int32) for x in queries)
    off = out_offsets(q1 - q0)
    X, nrm = _c(pts["X"], np.float64), _c(pts["normal"], np.float64)
    dmin, dmax = _c(pts["dmin"], np.float64), _c(pts["dmax"], np.float64)
    desc = _c(pts["desc"], np.uint32)
    sk = None if skip is None else _c(skip, np.uint8)
    match = np.zeros(off[-1], dtype=np.int32)
    dist = np.zeros(off[-1], dtype=np.int32)
    lib().mapref_fusion(C.byref(bs.S), C.byref(P), X.ctypes.data, nrm.ctypes.data, dmin.ctypes.data,
                        dmax.ctypes.data, desc.ctypes.data, len(q0), q0.ctypes.data, q1.ctypes.data,
                        qn.ctypes.data, off.ctypes.data, None if sk is None else sk.ctypes.data,
                        match.ctypes.data, dist.ctypes.data)
    return match, dist, off


def culling(w: dict, n_levels: int = 8, active=None, protect=None, min_obs: int = 3, slack: int = 0,
            num: int = 9, den: int = 10) -> dict:
    """Keyframe-culling counts of one window (dict with obs_kf, obs_pt, obs_oct, fixed, X)."""
    K, M = len(w["fixed"]), len(w["X"])
    kf, pt, oc = _c(w["obs_kf"], np.int32), _c(w["obs_pt"], np.int32), _c(w["obs_oct"], np.uint8)
    act = None if active is None else _c(active, np.uint8)
    pro = None if protect is None else _c(protect, np.uint8)
    cnt = np.zeros((M, n_levels), dtype=np.int32)
    ko = np.zeros(K, dtype=np.int32)
    kr = np.zeros(K, dtype=np.int32)
    cull = np.zeros(K, dtype=np.uint8)
    lib().mapref_culling(K, M, len(kf), n_levels, kf.ctypes.data, pt.ctypes.data, oc.ctypes.data,
                         None if act is None else act.ctypes.data, None if pro is None else pro.ctypes.data,
                         min_obs, slack, num, den, cnt.ctypes.data, ko.ctypes.data, kr.ctypes.data, cull.ctypes.data)
    return dict(counters=cnt, kf_obs=ko, kf_red=kr, cull=cull.astype(bool))
