"""Python binding of the local-mapping searches of liblba.so (the C ABI declared in
include/lmap.h): the GPU-resident keyframe store and its index, the keypoint
correspondence search, the fusion candidate search and the keyframe-culling counters.

Argument marshalling only: torch tensors provide device memory and the stream, ctypes
passes their pointers through the C ABI, and every step runs in the library's HIP
kernels.  There is no fallback: without the library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lba as _lba

STATUS = {0: "ok", -1: "invalid argument", -3: "HIP runtime error", -4: "workspace too small",
          -5: "unsupported problem size"}

# every symbol include/lmap.h declares
EXPORTS = ["lmap_abi_version", "lmap_status_string", "lmap_last_error", "lmap_default_corr_params",
           "lmap_default_fuse_params", "lmap_default_cull_params", "lmap_index_size", "lmap_index_build",
           "lmap_corr_workspace_size", "lmap_correspondence", "lmap_fuse_workspace_size", "lmap_fusion",
           "lmap_cull_workspace_size", "lmap_culling", "lmap_profile_enable", "lmap_profile_read",
           "lmap_correspondence_noalloc"]

NOALLOC_SCRATCH_BYTES = 16 << 20

KERNEL_CLASSES = ["index", "prep", "corr_search", "corr_resolve", "fuse", "cull_count", "cull_redundant",
                  "cull_decide", "check"]


class Store(C.Structure):
    _fields_ = [("n_kf", C.c_int32), ("n_kp", C.c_int32), ("max_kp", C.c_int32), ("n_levels", C.c_int32),
                ("width", C.c_int32), ("height", C.c_int32), ("kp_off", C.c_void_p), ("T_cw", C.c_void_p),
                ("kp_u", C.c_void_p), ("kp_v", C.c_void_p), ("kp_ur", C.c_void_p), ("kp_oct", C.c_void_p),
                ("kp_desc", C.c_void_p), ("index", C.c_void_p), ("sigma2", C.c_void_p), ("scale", C.c_void_p),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("bf", C.c_double)]


class CorrParams(C.Structure):
    _fields_ = [("th_low", C.c_int32), ("resolve", C.c_int32), ("epi_chi2", C.c_double),
                ("epipole_min", C.c_double)]


class FuseParams(C.Structure):
    _fields_ = [("th_low", C.c_int32), ("reserved", C.c_int32), ("radius_th", C.c_double),
                ("chi2_mono", C.c_double), ("chi2_stereo", C.c_double)]


class Points(C.Structure):
    _fields_ = [("n_pt", C.c_int32), ("reserved", C.c_int32), ("X", C.c_void_p), ("normal", C.c_void_p),
                ("dmin", C.c_void_p), ("dmax", C.c_void_p), ("desc", C.c_void_p)]


class CullParams(C.Structure):
    _fields_ = [("min_obs", C.c_int32), ("slack", C.c_int32), ("num", C.c_int32), ("den", C.c_int32)]


_declared = False


def library():
    global _declared
    L = _lba.library()
    if not _declared:
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        L.lmap_abi_version.restype = i32
        L.lmap_status_string.restype = C.c_char_p
        L.lmap_status_string.argtypes = [C.c_int]
        L.lmap_last_error.restype = C.c_char_p
        L.lmap_default_corr_params.argtypes = [C.POINTER(CorrParams)]
        L.lmap_default_fuse_params.argtypes = [C.POINTER(FuseParams)]
        L.lmap_default_cull_params.argtypes = [C.POINTER(CullParams)]
        L.lmap_index_size.argtypes = [C.POINTER(Store), C.POINTER(sz)]
        L.lmap_index_build.argtypes = [C.POINTER(Store), i32, i32, sz, i32, vp]
        L.lmap_corr_workspace_size.argtypes = [C.POINTER(Store), i32, C.POINTER(sz)]
        L.lmap_correspondence.argtypes = [C.POINTER(Store), C.POINTER(CorrParams), vp, i32, vp, vp, vp, i64,
                                          vp, vp, vp, sz, i32, vp]
        L.lmap_fuse_workspace_size.argtypes = [C.POINTER(sz)]
        L.lmap_fusion.argtypes = [C.POINTER(Store), C.POINTER(FuseParams), C.POINTER(Points), i32, vp, vp, vp, vp,
                                  i64, i32, vp, vp, vp, vp, sz, i32, vp]
        L.lmap_cull_workspace_size.argtypes = [C.POINTER(sz)]
        L.lmap_culling.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, C.POINTER(CullParams), vp, vp, vp, vp,
                                   vp, sz, i32, vp]
        L.lmap_correspondence_noalloc.argtypes = [C.POINTER(Store), C.POINTER(CorrParams), vp, i32, vp, vp, vp,
                                                  i64, vp, vp, i32, vp]
        L.lmap_profile_enable.argtypes = [i32]
        L.lmap_profile_read.argtypes = [i32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        for name in EXPORTS[6:]:
            getattr(L, name).restype = C.c_int
        _declared = True
    return L


class LMapError(RuntimeError):
    pass


def _check(st, what):
    if st != 0:
        raise LMapError(f"{what}: {STATUS.get(st, st)}: {library().lmap_last_error().decode()}")


def profile(enable: bool = True):
    """Enable (and reset) or disable the per-kernel event timing of the searches."""
    _check(library().lmap_profile_enable(1 if enable else 0), "lmap_profile_enable")


def profile_read() -> dict:
    """{kernel class: (launches, total ms)} since profiling was enabled."""
    out = {}
    for i, name in enumerate(KERNEL_CLASSES):
        n, ms = C.c_int64(), C.c_double()
        _check(library().lmap_profile_read(i, C.byref(n), C.byref(ms)), "lmap_profile_read")
        out[name] = (n.value, ms.value)
    return out


def corr_params(**kw) -> CorrParams:
    p = CorrParams()
    library().lmap_default_corr_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def fuse_params(**kw) -> FuseParams:
    p = FuseParams()
    library().lmap_default_fuse_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def cull_params(**kw) -> CullParams:
    p = CullParams()
    library().lmap_default_cull_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


def _stream(device):
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class DeviceStore:
    """A keyframe store resident in device memory (Section IV-B): the immutable keyframe
    data uploaded once, and its index (signed-byte descriptors, keypoints by cell) built
    once by lmap_index_build."""

    def __init__(self, store: dict, device="cuda:0", build_index: bool = True, check: bool = True):
        import torch
        self.device = torch.device(device)
        dev = self.device
        kp_off = np.asarray(store["kp_off"], dtype=np.int32)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a, dtype=dt)).to(dev)
        self.kp_off = t(kp_off, np.int32)
        self.T = t(np.asarray(store["T_cw"], dtype=np.float64).reshape(-1, 12), np.float64)
        self.u = t(store["kp_u"], np.float32)
        self.v = t(store["kp_v"], np.float32)
        self.ur = t(store["kp_ur"], np.float32)
        self.oct = t(store["kp_oct"], np.uint8)
        self.desc = t(np.asarray(store["kp_desc"], dtype=np.uint32).view(np.int32).reshape(-1, 8), np.int32)
        self.sigma2 = np.ascontiguousarray(store["sigma2"], dtype=np.float64)
        self.scale = np.ascontiguousarray(store["scale"], dtype=np.float64)
        cam = [float(x) for x in np.asarray(store["cam"], dtype=np.float64)]
        self.n_kf = len(kp_off) - 1
        self.n_kp = int(kp_off[-1])
        self.kp_counts = np.diff(kp_off)
        self.max_kp = max(1, int(self.kp_counts.max())) if self.n_kf else 1
        self.S = Store(self.n_kf, self.n_kp, self.max_kp, len(self.sigma2), int(store["width"]),
                       int(store["height"]), _ptr(self.kp_off), _ptr(self.T), _ptr(self.u), _ptr(self.v),
                       _ptr(self.ur), _ptr(self.oct), _ptr(self.desc), None,
                       self.sigma2.ctypes.data, self.scale.ctypes.data, *cam)
        n = C.c_size_t()
        _check(library().lmap_index_size(C.byref(self.S), C.byref(n)), "lmap_index_size")
        self.index = torch.zeros(n.value, dtype=torch.uint8, device=dev)
        self.S.index = self.index.data_ptr()
        if build_index:
            self.build_index(0, self.n_kf, check=check)

    def build_index(self, k0: int, k1: int, check: bool = True):
        _check(library().lmap_index_build(C.byref(self.S), int(k0), int(k1), self.index.numel(), int(check),
                                          _stream(self.device)), "lmap_index_build")

    def upload_free(self, kp_free):
        import torch
        return torch.as_tensor(np.ascontiguousarray(kp_free, dtype=np.uint8)).to(self.device)


def out_offsets(counts) -> np.ndarray:
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    return off


class Correspondence:
    """Device buffers of one batch of correspondence queries (cur[q], nbr[q])."""

    def __init__(self, ds: DeviceStore, cur, nbr):
        import torch
        dev = ds.device
        self.ds = ds
        cur = np.ascontiguousarray(cur, dtype=np.int32)
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        self.n_q = len(cur)
        cnt = ds.kp_counts[np.clip(cur, 0, ds.n_kf - 1)] if self.n_q else np.zeros(0, np.int64)
        self.off_np = out_offsets(cnt)
        self.cur = torch.as_tensor(cur).to(dev)
        self.nbr = torch.as_tensor(nbr).to(dev)
        self.off = torch.as_tensor(self.off_np).to(dev)
        self.n_out = int(self.off_np[-1])
        self.match = torch.empty(max(self.n_out, 1), dtype=torch.int32, device=dev)
        self.dist = torch.empty(max(self.n_out, 1), dtype=torch.int32, device=dev)
        n = C.c_size_t()
        _check(library().lmap_corr_workspace_size(C.byref(ds.S), self.n_q, C.byref(n)), "lmap_corr_workspace_size")
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=dev)

    def run(self, kp_free_dev, params: CorrParams | None = None, check: bool = True, stream=None):
        p = params or corr_params()
        st = C.c_void_p(stream.cuda_stream) if stream is not None else _stream(self.ds.device)
        _check(library().lmap_correspondence(C.byref(self.ds.S), C.byref(p), _ptr(kp_free_dev), self.n_q,
                                             _ptr(self.cur), _ptr(self.nbr), _ptr(self.off), self.n_out,
                                             _ptr(self.match), _ptr(self.dist), _ptr(self.ws), self.ws.numel(),
                                             int(check), st), "lmap_correspondence")

    def run_noalloc(self, kp_free_dev, params: CorrParams | None = None, check: bool = True, stream=None):
        """The same search through lmap_correspondence_noalloc (library-held scratch)."""
        p = params or corr_params()
        st = C.c_void_p(stream.cuda_stream) if stream is not None else _stream(self.ds.device)
        _check(library().lmap_correspondence_noalloc(C.byref(self.ds.S), C.byref(p), _ptr(kp_free_dev), self.n_q,
                                                     _ptr(self.cur), _ptr(self.nbr), _ptr(self.off), self.n_out,
                                                     _ptr(self.match), _ptr(self.dist), int(check), st),
               "lmap_correspondence_noalloc")

    def result(self):
        return (self.match[:self.n_out].cpu().numpy(), self.dist[:self.n_out].cpu().numpy(), self.off_np)


def correspondence(ds: DeviceStore, kp_free, cur, nbr, check: bool = True, **params):
    """(match, dist, out_off) of the correspondence search, like the oracle's."""
    import torch
    job = Correspondence(ds, cur, nbr)
    job.run(ds.upload_free(kp_free), corr_params(**params), check=check)
    torch.cuda.synchronize(ds.device)
    return job.result()


class Fusion:
    """Device buffers of one batch of fusion queries (point range, neighbour keyframe)."""

    def __init__(self, ds: DeviceStore, pts: dict, queries, skip=None):
        import torch
        dev = ds.device
        self.ds = ds
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a, dtype=dt)).to(dev)
        self.X = t(pts["X"], np.float64)
        self.normal = t(pts["normal"], np.float64)
        self.dmin = t(pts["dmin"], np.float64)
        self.dmax = t(pts["dmax"], np.float64)
        self.desc = t(np.asarray(pts["desc"], dtype=np.uint32).view(np.int32), np.int32)
        self.P = Points(len(pts["X"]), 0, _ptr(self.X), _ptr(self.normal), _ptr(self.dmin), _ptr(self.dmax),
                        _ptr(self.desc))
        q0, q1, qn = (np.ascontiguousarray(x, dtype=np.int32) for x in queries)
        self.n_q = len(q0)
        self.off_np = out_offsets(q1 - q0)
        self.n_out = int(self.off_np[-1])
        self.max_len = max(1, int((q1 - q0).max())) if self.n_q else 1
        self.p0, self.p1, self.nbr = t(q0, np.int32), t(q1, np.int32), t(qn, np.int32)
        self.off = t(self.off_np, np.int64)
        self.skip = None if skip is None else t(skip, np.uint8)
        self.match = torch.empty(max(self.n_out, 1), dtype=torch.int32, device=dev)
        self.dist = torch.empty(max(self.n_out, 1), dtype=torch.int32, device=dev)
        n = C.c_size_t()
        _check(library().lmap_fuse_workspace_size(C.byref(n)), "lmap_fuse_workspace_size")
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=dev)

    def run(self, params: FuseParams | None = None, check: bool = True, stream=None):
        p = params or fuse_params()
        st = C.c_void_p(stream.cuda_stream) if stream is not None else _stream(self.ds.device)
        _check(library().lmap_fusion(C.byref(self.ds.S), C.byref(p), C.byref(self.P), self.n_q, _ptr(self.p0),
                                     _ptr(self.p1), _ptr(self.nbr), _ptr(self.off), self.n_out, self.max_len,
                                     _ptr(self.skip), _ptr(self.match), _ptr(self.dist), _ptr(self.ws),
                                     self.ws.numel(), int(check), st), "lmap_fusion")

    def result(self):
        return (self.match[:self.n_out].cpu().numpy(), self.dist[:self.n_out].cpu().numpy(), self.off_np)


def fusion(ds: DeviceStore, pts: dict, queries, skip=None, check: bool = True, **params):
    """(match, dist, out_off) of the fusion candidate search, like the oracle's."""
    import torch
    job = Fusion(ds, pts, queries, skip)
    job.run(fuse_params(**params), check=check)
    torch.cuda.synchronize(ds.device)
    return job.result()


class Culling:
    """Device buffers of the culling counters of one problem (global indices)."""

    def __init__(self, n_kf: int, n_pt: int, obs_kf, obs_pt, obs_oct, n_levels: int = 8, active=None, protect=None,
                 device="cuda:0"):
        import torch
        dev = torch.device(device)
        self.device = dev
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a, dtype=dt)).to(dev)
        self.n_kf, self.n_pt, self.n_levels = int(n_kf), int(n_pt), int(n_levels)
        self.kf, self.pt, self.oct = t(obs_kf, np.int32), t(obs_pt, np.int32), t(obs_oct, np.uint8)
        self.n_obs = int(self.kf.numel())
        self.active = None if active is None else t(active, np.uint8)
        self.protect = None if protect is None else t(protect, np.uint8)
        self.counters = torch.empty(max(1, self.n_pt * self.n_levels), dtype=torch.int32, device=dev)
        self.kf_obs = torch.empty(max(1, self.n_kf), dtype=torch.int32, device=dev)
        self.kf_red = torch.empty(max(1, self.n_kf), dtype=torch.int32, device=dev)
        self.cull = torch.empty(max(1, self.n_kf), dtype=torch.uint8, device=dev)
        n = C.c_size_t()
        _check(library().lmap_cull_workspace_size(C.byref(n)), "lmap_cull_workspace_size")
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=dev)

    def run(self, params: CullParams | None = None, check: bool = True, stream=None):
        p = params or cull_params()
        st = C.c_void_p(stream.cuda_stream) if stream is not None else _stream(self.device)
        _check(library().lmap_culling(self.n_kf, self.n_pt, self.n_obs, self.n_levels, _ptr(self.kf), _ptr(self.pt),
                                      _ptr(self.oct), _ptr(self.active), _ptr(self.protect), C.byref(p),
                                      _ptr(self.counters), _ptr(self.kf_obs), _ptr(self.kf_red), _ptr(self.cull),
                                      _ptr(self.ws), self.ws.numel(), int(check), st), "lmap_culling")

    def result(self) -> dict:
        return dict(counters=self.counters[:self.n_pt * self.n_levels].cpu().numpy().reshape(self.n_pt, self.n_levels),
                    kf_obs=self.kf_obs[:self.n_kf].cpu().numpy(), kf_red=self.kf_red[:self.n_kf].cpu().numpy(),
                    cull=self.cull[:self.n_kf].cpu().numpy().astype(bool))


def culling(n_kf, n_pt, obs_kf, obs_pt, obs_oct, n_levels=8, active=None, protect=None, check=True, device="cuda:0",
            **params) -> dict:
    import torch
    job = Culling(n_kf, n_pt, obs_kf, obs_pt, obs_oct, n_levels, active, protect, device)
    job.run(cull_params(**params), check=check)
    torch.cuda.synchronize(job.device)
    return job.result()
