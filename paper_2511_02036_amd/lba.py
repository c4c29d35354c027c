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
TUNE_CLASSES = 9
STAT_NAMES = ["F_initial", "F_final", "iters_r1", "iters_r2", "trials", "lambda", "term_r1",
              "term_r2", "n_outliers", "F_end_r1", "F_start_r2", "Kopt"]

STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "HIP runtime error",
          -4: "workspace too small", -5: "unsupported problem size"}

# every symbol include/lba.h declares
EXPORTS = ["lba_abi_version", "lba_status_string", "lba_default_options", "lba_create",
           "lba_destroy", "lba_last_error", "lba_set_options", "lba_workspace_size", "lba_solve",
           "lba_solve_batch", "lba_profile_enable", "lba_profile_read", "lba_cost_workspace_size",
           "lba_cost_forward", "lba_cost_backward", "lba_tune", "lba_inertial_workspace_size",
           "lba_solve_inertial", "lba_tune_get", "lba_tune_set"]

KERNEL_CLASSES = ["linearize", "linearize_init", "reduce", "cholesky", "update", "decide",
                  "init_reduce", "setup", "validate", "flags", "finalize", "cost_forward",
                  "cost_backward", "order", "inertial"]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("iters_round1", C.c_int32), ("iters_round2", C.c_int32),
                ("max_trials", C.c_int32), ("round2_robust", C.c_int32), ("check_inputs", C.c_int32),
                ("huber2_mono", C.c_double), ("huber2_stereo", C.c_double),
                ("chi2_mono", C.c_double), ("chi2_stereo", C.c_double), ("tau", C.c_double),
                ("points_per_tile", C.c_int32), ("use_graphs", C.c_int32), ("trial_log", C.c_int32),
                ("schur_fp32_accum", C.c_int32), ("pair_cache", C.c_int32)]


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


class TrialRecord(C.Structure):
    _fields_ = [("round", C.c_int32), ("iter", C.c_int32), ("trial", C.c_int32),
                ("accepted", C.c_int32), ("solve_ok", C.c_int32), ("reserved", C.c_int32),
                ("lam", C.c_double), ("F", C.c_double), ("F_trial", C.c_double), ("gain", C.c_double)]


VI_ARRAYS = ["edge_i", "edge_j", "dt", "dR", "dv", "dp", "J_Rg", "J_vg", "J_va", "J_pg", "J_pa", "bg_bar",
             "ba_bar", "info", "info_bg", "info_ba", "v", "bg", "ba"]


class Inertial(C.Structure):
    _fields_ = [("n_edges", C.c_int32), ("reserved", C.c_int32), ("edge_off", C.c_void_p)] + \
        [(k, C.c_void_p) for k in VI_ARRAYS] + [("T_cb", C.c_double * 12), ("g", C.c_double * 3)]


class Result(C.Structure):
    _fields_ = [("T_out", C.c_void_p), ("X_out", C.c_void_p), ("outlier", C.c_void_p),
                ("stats", C.c_void_p), ("log", C.c_void_p)]


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
        L.lba_cost_workspace_size.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(Batch),
                                              C.POINTER(C.c_size_t)]
        L.lba_cost_workspace_size.restype = C.c_int
        L.lba_cost_forward.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(Batch), C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_size_t, C.c_void_p]
        L.lba_cost_forward.restype = C.c_int
        L.lba_cost_backward.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(Batch), C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.lba_cost_backward.restype = C.c_int
        L.lba_tune.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(Batch), C.c_void_p,
                               C.POINTER(C.c_int32)]
        L.lba_tune.restype = C.c_int
        L.lba_tune_get.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
        L.lba_tune_get.restype = C.c_int
        L.lba_tune_set.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
        L.lba_tune_set.restype = C.c_int
        L.lba_inertial_workspace_size.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(Batch),
                                                  C.POINTER(Inertial), C.POINTER(C.c_size_t)]
        L.lba_inertial_workspace_size.restype = C.c_int
        L.lba_solve_inertial.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(Batch), C.POINTER(Inertial),
                                         C.POINTER(Result), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_size_t, C.c_void_p]
        L.lba_solve_inertial.restype = C.c_int
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

    def tune(self, prob: "DeviceProblem", stream=None) -> list:
        """Run the tile tuner on this problem (see lba_tune); returns the points-per-tile
        table by window class (TUNE_CLASSES entries: 3 * keyframe class + point class)."""
        import torch
        stream = stream or torch.cuda.current_stream(prob.device)
        out = (C.c_int32 * TUNE_CLASSES)()
        self._check(self.lib.lba_tune(self.handle, C.byref(prob.problem), C.byref(prob.batch),
                                      C.c_void_p(stream.cuda_stream), out), "lba_tune")
        return list(out)

    def tune_table(self) -> list:
        """The context's tile table (lba_tune_get), to be stored by the caller."""
        out = (C.c_int32 * TUNE_CLASSES)()
        self._check(self.lib.lba_tune_get(self.handle, out), "lba_tune_get")
        return list(out)

    def set_tune_table(self, table) -> None:
        """Install a stored tile table (lba_tune_set); None forgets it."""
        arr = None if table is None else (C.c_int32 * TUNE_CLASSES)(*[int(x) for x in table])
        self._check(self.lib.lba_tune_set(self.handle, arr), "lba_tune_set")

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
        self.log_cap = int(ctx.options.trial_log)
        self.log = (TrialRecord * max(1, self.log_cap * prob.n_windows))()
        self.result = Result(self.T_out.data_ptr(), self.X_out.data_ptr(), self.outlier.data_ptr(),
                             self.stats.ctypes.data, C.addressof(self.log) if self.log_cap > 0 else None)

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

    def trial_logs(self):
        """Per window, the list of its recorded trials (as dicts), oldest first."""
        out = []
        for w in range(self.prob.n_windows):
            n = min(int(self.stats[w, 4]), self.log_cap)
            recs = self.log[w * self.log_cap: w * self.log_cap + n]
            out.append([dict(round=r.round, iter=r.iter, trial=r.trial, accepted=bool(r.accepted),
                             solve_ok=bool(r.solve_ok), lam=r.lam, F=r.F, F_trial=r.F_trial, gain=r.gain)
                        for r in recs])
        return out


class DeviceInertial:
    """The inertial measurements and initial velocities / biases of a window or a batch on
    the GPU.  ``vi`` is a dict of arrays as ``synth.vi_window`` returns (concatenated over
    windows with ``edge_off`` for a batch: window-local keyframe indices)."""

    def __init__(self, vi: dict, device="cuda"):
        import torch
        dev = torch.device(device)
        shapes = dict(edge_i=(np.int32, -1), edge_j=(np.int32, -1), dt=(np.float64, -1), dR=(np.float64, 9),
                      dv=(np.float64, 3), dp=(np.float64, 3), J_Rg=(np.float64, 9), J_vg=(np.float64, 9),
                      J_va=(np.float64, 9), J_pg=(np.float64, 9), J_pa=(np.float64, 9), bg_bar=(np.float64, 3),
                      ba_bar=(np.float64, 3), info=(np.float64, 81), info_bg=(np.float64, -1),
                      info_ba=(np.float64, -1), v=(np.float64, 3), bg=(np.float64, 3), ba=(np.float64, 3))
        self.t = {}
        for k, (dt, m) in shapes.items():
            a = np.ascontiguousarray(vi[k], dtype=dt)
            a = a.reshape(-1) if m == -1 else a.reshape(-1, m)
            self.t[k] = torch.as_tensor(a, device=dev)
        self.n_edges = int(self.t["edge_i"].shape[0])
        self.edge_off = None if "edge_off" not in vi else np.ascontiguousarray(vi["edge_off"], dtype=np.int32)
        ptr = lambda x: x.data_ptr() if x.numel() else None
        self.I = Inertial(self.n_edges, 0, None if self.edge_off is None else self.edge_off.ctypes.data,
                          *[ptr(self.t[k]) for k in VI_ARRAYS],
                          (C.c_double * 12)(*np.asarray(vi["T_cb"], dtype=np.float64).reshape(12).tolist()),
                          (C.c_double * 3)(*np.asarray(vi["g"], dtype=np.float64).reshape(3).tolist()))


class InertialSolver(Solver):
    """Reusable stereo-inertial solve of a DeviceProblem with its DeviceInertial."""

    def __init__(self, ctx: Context, prob: DeviceProblem, vi: DeviceInertial):
        torch = prob.torch
        self.ctx = ctx
        self.prob = prob
        self.vi = vi
        ws = C.c_size_t(0)
        batch = C.byref(prob.batch) if prob.n_windows > 1 else None
        ctx._check(ctx.lib.lba_inertial_workspace_size(ctx.handle, C.byref(prob.problem), batch, C.byref(vi.I),
                                                       C.byref(ws)), "lba_inertial_workspace_size")
        self.ws_bytes = ws.value
        self.ws = torch.empty(max(self.ws_bytes, 256) + 256, dtype=torch.uint8, device=prob.device)
        self.ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.T_out = torch.empty_like(prob.T_cw)
        self.X_out = torch.empty_like(prob.X)
        self.outlier = torch.empty(prob.obs_kf.shape[0], dtype=torch.uint8, device=prob.device)
        self.v_out = torch.empty_like(vi.t["v"])
        self.bg_out = torch.empty_like(vi.t["bg"])
        self.ba_out = torch.empty_like(vi.t["ba"])
        self.stats = np.zeros((prob.n_windows, STATS_LEN), dtype=np.float64)
        self.log_cap = int(ctx.options.trial_log)
        self.log = (TrialRecord * max(1, self.log_cap * prob.n_windows))()
        self.result = Result(self.T_out.data_ptr(), self.X_out.data_ptr(), self.outlier.data_ptr(),
                             self.stats.ctypes.data, C.addressof(self.log) if self.log_cap > 0 else None)

    def run(self, stream=None):
        torch = self.prob.torch
        if stream is None:
            stream = torch.cuda.current_stream(self.prob.device)
        batch = C.byref(self.prob.batch) if self.prob.n_windows > 1 else None
        st = self.ctx.lib.lba_solve_inertial(self.ctx.handle, C.byref(self.prob.problem), batch,
                                             C.byref(self.vi.I), C.byref(self.result), self.v_out.data_ptr(),
                                             self.bg_out.data_ptr(), self.ba_out.data_ptr(), C.c_void_p(self.ws_ptr),
                                             C.c_size_t(self.ws_bytes), C.c_void_p(stream.cuda_stream))
        self.ctx._check(st, "lba_solve_inertial")
        return self


def solve_inertial(data: dict, vi: dict, device="cuda", z_f32: bool = False, **options) -> dict:
    """One-shot stereo-inertial solve of a window (or a batch with ``edge_off``)."""
    import torch
    dev = torch.device(device)
    ctx = Context(device=dev.index or 0, **options)
    prob = DeviceProblem(data, device=dev, z_f32=z_f32)
    dvi = DeviceInertial(vi, device=dev)
    s = InertialSolver(ctx, prob, dvi).run()
    out = dict(T=s.T_out.cpu().numpy(), X=s.X_out.cpu().numpy(), V=s.v_out.cpu().numpy(),
               BG=s.bg_out.cpu().numpy(), BA=s.ba_out.cpu().numpy(),
               outlier=s.outlier.cpu().numpy().astype(bool), stats=s.stats_dicts(), log=s.trial_logs())
    ctx.close()
    return out


def solve(data: dict, device="cuda", z_f32: bool = False, **options) -> dict:
    """One-shot solve of a window (or a concatenated batch).  Returns host numpy copies of
    the refined poses (n_kf, 12), points (n_pt, 3), outlier flags and per-window stats."""
    import torch
    dev = torch.device(device)
    ctx = Context(device=dev.index or 0, **options)
    prob = DeviceProblem(data, device=dev, z_f32=z_f32)
    s = Solver(ctx, prob).run()
    out = dict(T=s.T_out.cpu().numpy(), X=s.X_out.cpu().numpy(),
               outlier=s.outlier.cpu().numpy().astype(bool), stats=s.stats_dicts(), log=s.trial_logs())
    ctx.close()
    return out


# ----------------------------------------------------------------------------------------
# differentiation form
# ----------------------------------------------------------------------------------------
class CostLayer:
    """The robust reprojection cost of every window of a batch as a differentiable
    function of FP32 pose perturbations xi (n_kf, 6), points X (n_pt, 3) and
    measurements z (3, n_obs); the topology, base poses, octaves and intrinsics come from
    ``data`` (one window dict or a concatenation, as for ``DeviceProblem``).

    ``forward`` and ``backward`` call lba_cost_forward / lba_cost_backward; use
    ``robust_cost`` for the autograd form."""

    def __init__(self, ctx: Context, data: dict, device="cuda"):
        import torch
        self.ctx = ctx
        self.prob = DeviceProblem(data, device=device, z_f32=True)
        self.torch = torch
        p = self.prob
        ws = C.c_size_t(0)
        ctx._check(ctx.lib.lba_cost_workspace_size(ctx.handle, C.byref(p.problem), C.byref(p.batch), C.byref(ws)),
                   "lba_cost_workspace_size")
        self.ws_bytes = ws.value
        self.ws = torch.empty(max(self.ws_bytes, 256) + 256, dtype=torch.uint8, device=p.device)
        self.ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.n_kf, self.n_pt, self.n_obs = p.T_cw.shape[0], p.X.shape[0], p.obs_kf.shape[0]
        self.n_windows = p.n_windows

    def _args(self, xi, X, z, mask):
        t = self.torch
        dev = self.prob.device

        def chk(x, shape, dtype, name):
            if x is None:
                return None
            if x.device != dev or x.dtype != dtype or tuple(x.shape) != shape or not x.is_contiguous():
                raise ValueError(f"{name}: expected contiguous {dtype} {shape} on {dev}, got "
                                 f"{x.dtype} {tuple(x.shape)} on {x.device}")
            return x
        xi = chk(xi, (self.n_kf, 6), t.float32, "xi")
        X = chk(X, (self.n_pt, 3), t.float32, "X")
        z = chk(z, (3, self.n_obs), t.float32, "z")
        mask = chk(mask, (self.n_obs,), t.uint8, "mask")
        ptr = lambda x: None if x is None else x.data_ptr()
        return xi, X, z, mask, ptr

    def forward(self, xi, X, z, mask=None, stream=None):
        """Cost per window (float64, (n_windows,))."""
        t = self.torch
        xi, X, z, mask, ptr = self._args(xi, X, z, mask)
        cost = t.empty(self.n_windows, dtype=t.float64, device=self.prob.device)
        stream = stream or t.cuda.current_stream(self.prob.device)
        st = self.ctx.lib.lba_cost_forward(self.ctx.handle, C.byref(self.prob.problem), C.byref(self.prob.batch),
                                           ptr(xi), ptr(X), ptr(z), ptr(mask), cost.data_ptr(),
                                           C.c_void_p(self.ws_ptr), C.c_size_t(self.ws_bytes),
                                           C.c_void_p(stream.cuda_stream))
        self.ctx._check(st, "lba_cost_forward")
        return cost

    def backward(self, xi, X, z, grad_cost, mask=None, stream=None):
        """Gradients (g_xi (n_kf, 6), g_X (n_pt, 3), g_z (3, n_obs)), all float32."""
        t = self.torch
        xi, X, z, mask, ptr = self._args(xi, X, z, mask)
        gc = grad_cost.to(device=self.prob.device, dtype=t.float64).contiguous()
        if tuple(gc.shape) != (self.n_windows,):
            raise ValueError(f"grad_cost: expected ({self.n_windows},), got {tuple(gc.shape)}")
        g_xi = t.empty((self.n_kf, 6), dtype=t.float32, device=self.prob.device)
        g_X = t.empty((self.n_pt, 3), dtype=t.float32, device=self.prob.device)
        g_z = t.empty((3, self.n_obs), dtype=t.float32, device=self.prob.device)
        stream = stream or t.cuda.current_stream(self.prob.device)
        st = self.ctx.lib.lba_cost_backward(self.ctx.handle, C.byref(self.prob.problem), C.byref(self.prob.batch),
                                            ptr(xi), ptr(X), ptr(z), ptr(mask), gc.data_ptr(), g_xi.data_ptr(),
                                            g_X.data_ptr(), g_z.data_ptr(), C.c_void_p(self.ws_ptr),
                                            C.c_size_t(self.ws_bytes), C.c_void_p(stream.cuda_stream))
        self.ctx._check(st, "lba_cost_backward")
        return g_xi, g_X, g_z


def _autograd_function():
    import torch

    class RobustReprojCost(torch.autograd.Function):
        """cost = RobustReprojCost.apply(layer, xi, X, z, mask): the robust reprojection
        cost per window; the backward pass is lba_cost_backward (Jacobians recomputed)."""

        @staticmethod
        def forward(fctx, layer, xi, X, z, mask):
            fctx.layer = layer
            fctx.mask = mask
            fctx.save_for_backward(xi, X, z)
            d = lambda x: None if x is None else x.detach()
            return layer.forward(d(xi), X.detach(), z.detach(), mask)

        @staticmethod
        def backward(fctx, grad_cost):
            xi, X, z = fctx.saved_tensors
            d = lambda x: None if x is None else x.detach()
            g_xi, g_X, g_z = fctx.layer.backward(d(xi), X.detach(), z.detach(), grad_cost, fctx.mask)
            return (None, g_xi if fctx.needs_input_grad[1] else None, g_X if fctx.needs_input_grad[2] else None,
                    g_z if fctx.needs_input_grad[3] else None, None)

    return RobustReprojCost


_RRC = None


def robust_cost(layer: CostLayer, xi, X, z, mask=None):
    """Differentiable cost per window (see CostLayer)."""
    global _RRC
    if _RRC is None:
        _RRC = _autograd_function()
    return _RRC.apply(layer, xi, X, z, mask)
