"""Python binding of liblba.so (the C ABI declared in include/lba.h).

Argument marshalling only: torch tensors provide device memory and the stream, ctypes
passes their pointers through the C ABI, and every step of the solve runs in the HIP
kernels of the library.  There is no fallback: if the library is missing or no GPU is
visible, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblba.so")

PREC_FP64 = 0
PREC_MIXED = 1
STATS_LEN = 12
STAT_NAMES = ["F_initial", "F_final", "iters_r1", "iters_r2", "trials", "lambda", "term_r1",
              "term_r2", "n_outliers", "F_end_r1", "F_start_r2", "Kopt"]

STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "HIP runtime error",
          -4: "workspace too small", -5: "unsupported problem size"}

# every symbol include/lba.h declares
EXPORTS = ["lba_abi_version", "lba_status_string", "lba_default_options", "lba_create",
           "lba_destroy", "lba_last_error", "lba_set_options", "lba_workspace_size", "lba_solve",
           "lba_solve_batch", "lba_profile_enable", "lba_profile_read"]

KERNEL_CLASSES = ["linearize", "linearize_init", "reduce", "cholesky", "update", "decide",
                  "init_reduce", "setup", "validate", "flags", "finalize"]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("iters_round1", C.c_int32), ("iters_round2", C.c_int32),
                ("max_trials", C.c_int32), ("round2_robust", C.c_int32), ("check_inputs", C.c_int32),
                ("huber2_mono", C.c_double), ("huber2_stereo", C.c_double),
                ("chi2_mono", C.c_double), ("chi2_stereo", C.c_double), ("tau", C.c_double),
                ("points_per_tile", C.c_int32), ("reserved", C.c_int32)]


class Intrinsics(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("bf", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("n_kf", C.c_int32), ("n_pt", C.c_int32), ("n_obs", C.c_int32),
                ("n_levels", C.c_int32), ("T_cw", C.c_void_p), ("fixed", C.c_void_p),
                ("X_w", C.c_void_p), ("obs_kf", C.c_void_p), ("obs_pt", C.c_void_p),
                ("obs_z", C.c_void_p), ("obs_z_f32", C.c_int32), ("reserved", C.c_int32),
                ("obs_type", C.c_void_p), ("obs_oct", C.c_void_p), ("sigma2", C.c_void_p),
                ("cam", Intrinsics)]


class Batch(C.Structure):
    _fields_ = [("n_windows", C.c_int32), ("reserved", C.c_int32), ("kf_off", C.c_void_p),
                ("pt_off", C.c_void_p), ("obs_off", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("T_out", C.c_void_p), ("X_out", C.c_void_p), ("outlier", C.c_void_p),
                ("stats", C.c_void_p)]


_lib = None


def library():
    """Load liblba.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_02036_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.lba_abi_version.restype = C.c_int32
        L.lba_status_string.restype = C.c_char_p
        L.lba_status_string.argtypes = [C.c_int]
        L.lba_default_options.argtypes = [C.POINTER(Options)]
        L.lba_create.argtypes = [C.POINTER(Options), C.c_int32, C.POINTER(C.c_void_p)]
        L.lba_create.restype = C.c_int
        L.lba_destroy.argtypes = [C.c_void_p]
        L.lba_last_error.argtypes = [C.c_void_p]
        L.lba_last_error.restype = C.c_char_p
        L.lba_set_options.argtypes = [C.c_void_p, C.POINTER(Options)]
        L.lba_set_options.restype = C.c_int
        L.lba_workspace_size.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(Batch),
                                         C.POINTER(C.c_size_t)]
        L.lba_workspace_size.restype = C.c_int
        L.lba_solve.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(Result), C.c_void_p,
                                C.c_size_t, C.c_void_p]
        L.lba_solve.restype = C.c_int
        L.lba_solve_batch.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(Batch),
                                      C.POINTER(Result), C.c_void_p, C.c_size_t, C.c_void_p]
        L.lba_solve_batch.restype = C.c_int
        L.lba_profile_enable.argtypes = [C.c_void_p, C.c_int32]
        L.lba_profile_enable.restype = C.c_int
        L.lba_profile_read.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int64),
                                       C.POINTER(C.c_double)]
        L.lba_profile_read.restype = C.c_int
        _lib = L
    return _lib


class LBAError(RuntimeError):
    pass


def default_options(**kw) -> Options:
    o = Options()
    library().lba_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": PREC_FP64, "mixed": PREC_MIXED}[v]
        setattr(o, k, v)
    return o


class Context:
    """Owns one lba_ctx (options + small pinned host staging)."""

    def __init__(self, device: int = 0, **options):
        self.lib = library()
        self.options = default_options(**options)
        h = C.c_void_p()
        st = self.lib.lba_create(C.byref(self.options), int(device), C.byref(h))
        if st != 0:
            raise LBAError(f"lba_create failed: {STATUS.get(st, st)}")
        self.handle = h
        self.device = device

    def set_options(self, **options):
        self.options = default_options(**options)
        self._check(self.lib.lba_set_options(self.handle, C.byref(self.options)), "lba_set_options")

    def _check(self, st, what):
        if st != 0:
            msg = self.lib.lba_last_error(self.handle).decode()
            raise LBAError(f"{what}: {STATUS.get(st, st)}: {msg}")

    def profile(self, enable: bool = True):
        """Enable (and reset) or disable per-kernel event timing."""
        self._check(self.lib.lba_profile_enable(self.handle, 1 if enable else 0), "lba_profile_enable")

    def profile_read(self) -> dict:
        """{kernel class: (launches, total ms)} accumulated since profiling was enabled."""
        out = {}
        for i, name in enumerate(KERNEL_CLASSES):
            n = C.c_int64()
            ms = C.c_double()
            self._check(self.lib.lba_profile_read(self.handle, i, C.byref(n), C.byref(ms)),
                        "lba_profile_read")
            out[name] = (n.value, ms.value)
        return out

    def close(self):
        if getattr(self, "handle", None):
            self.lib.lba_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceProblem:
    """A window or a batch of windows whose arrays live on the GPU (torch tensors).

    ``data`` is one window dict (as produced by ``synth``) or a concatenation with
    ``kf_off`` / ``pt_off`` / ``obs_off`` offsets (``synth.concat``)."""

    def __init__(self, data: dict, device="cuda", z_f32: bool = False):
        import torch
        dev = torch.device(device)
        self.torch = torch
        self.device = dev
        self.T_cw = torch.as_tensor(np.ascontiguousarray(data["T_cw"], dtype=np.float64).reshape(-1, 12),
                                    device=dev)
        self.X = torch.as_tensor(np.ascontiguousarray(data["X"], dtype=np.float64).reshape(-1, 3), device=dev)
        self.obs_kf = torch.as_tensor(np.ascontiguousarray(data["obs_kf"], dtype=np.int32), device=dev)
        self.obs_pt = torch.as_tensor(np.ascontiguousarray(data["obs_pt"], dtype=np.int32), device=dev)
        zdt = np.float32 if z_f32 else np.float64
        self.obs_z = torch.as_tensor(np.ascontiguousarray(data["obs_z"], dtype=zdt).reshape(3, -1), device=dev)
        self.obs_type = torch.as_tensor(np.ascontiguousarray(data["obs_type"], dtype=np.uint8), device=dev)
        self.obs_oct = torch.as_tensor(np.ascontiguousarray(data["obs_oct"], dtype=np.uint8), device=dev)
        self.fixed = np.ascontiguousarray(data["fixed"], dtype=np.uint8)
        self.sigma2 = np.ascontiguousarray(data["sigma2"], dtype=np.float64)
        self.cam = np.asarray(data["cam"], dtype=np.float64)
        self.z_f32 = z_f32
        n_kf, n_pt, n_obs = self.T_cw.shape[0], self.X.shape[0], self.obs_kf.shape[0]
        if "kf_off" in data:
            self.kf_off = np.ascontiguousarray(data["kf_off"], dtype=np.int32)
            self.pt_off = np.ascontiguousarray(data["pt_off"], dtype=np.int32)
            self.obs_off = np.ascontiguousarray(data["obs_off"], dtype=np.int32)
        else:
            self.kf_off = np.array([0, n_kf], dtype=np.int32)
            self.pt_off = np.array([0, n_pt], dtype=np.int32)
            self.obs_off = np.array([0, n_obs], dtype=np.int32)
        self.n_windows = len(self.kf_off) - 1
        self.problem = Problem(n_kf, n_pt, n_obs, len(self.sigma2), self.T_cw.data_ptr(),
                               self.fixed.ctypes.data, self.X.data_ptr(), self.obs_kf.data_ptr(),
                               self.obs_pt.data_ptr(), self.obs_z.data_ptr(), 1 if z_f32 else 0, 0,
                               self.obs_type.data_ptr(), self.obs_oct.data_ptr(),
                               self.sigma2.ctypes.data, Intrinsics(*[float(x) for x in self.cam]))
        self.batch = Batch(self.n_windows, 0, self.kf_off.ctypes.data, self.pt_off.ctypes.data,
                           self.obs_off.ctypes.data)


class Solver:
    """Reusable solve of one DeviceProblem: outputs and workspace are allocated once
    (torch caching allocator) and reused across calls."""

    def __init__(self, ctx: Context, prob: DeviceProblem):
        torch = prob.torch
        self.ctx = ctx
        self.prob = prob
        ws = C.c_size_t(0)
        ctx._check(ctx.lib.lba_workspace_size(ctx.handle, C.byref(prob.problem), C.byref(prob.batch),
                                              C.byref(ws)), "lba_workspace_size")
        self.ws_bytes = ws.value
        self.ws = torch.empty(max(self.ws_bytes, 256) + 256, dtype=torch.uint8, device=prob.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.T_out = torch.empty_like(prob.T_cw)
        self.X_out = torch.empty_like(prob.X)
        self.outlier = torch.empty(prob.obs_kf.shape[0], dtype=torch.uint8, device=prob.device)
        self.stats = np.zeros((prob.n_windows, STATS_LEN), dtype=np.float64)
        self.result = Result(self.T_out.data_ptr(), self.X_out.data_ptr(), self.outlier.data_ptr(),
                             self.stats.ctypes.data)

    def run(self, stream=None):
        torch = self.prob.torch
        if stream is None:
            stream = torch.cuda.current_stream(self.prob.device)
        st = self.ctx.lib.lba_solve_batch(self.ctx.handle, C.byref(self.prob.problem),
                                          C.byref(self.prob.batch), C.byref(self.result),
                                          C.c_void_p(self.ws_ptr), C.c_size_t(self.ws_bytes),
                                          C.c_void_p(stream.cuda_stream))
        self.ctx._check(st, "lba_solve_batch")
        return self

    def stats_dicts(self):
        return [dict(zip(STAT_NAMES, row.tolist())) for row in self.stats]


def solve(data: dict, device="cuda", z_f32: bool = False, **options) -> dict:
    """One-shot solve of a window (or a concatenated batch).  Returns host numpy copies of
    the refined poses (n_kf, 12), points (n_pt, 3), outlier flags and per-window stats."""
    import torch
    dev = torch.device(device)
    ctx = Context(device=dev.index or 0, **options)
    prob = DeviceProblem(data, device=dev, z_f32=z_f32)
    s = Solver(ctx, prob).run()
    out = dict(T=s.T_out.cpu().numpy(), X=s.X_out.cpu().numpy(),
               outlier=s.outlier.cpu().numpy().astype(bool), stats=s.stats_dicts())
    ctx.close()
    return out
