"""Seeded synthetic local-bundle-adjustment windows.

This module only *generates inputs*: camera trajectories, 3-D points, visibility-based
associations, octaves, pixel noise, injected outliers and initial perturbations.  It holds
none of the solver's arithmetic (no information weighting, robust kernel, Jacobians,
normal equations or damping).  To synthesise measurements it projects the noise-free
points with its own pinhole model, and it builds rotations and the initial pose
perturbation with SciPy's ``expm``.  Both the CPU oracle and the GPU path
consume its output; it imports neither.

The windows stand in for the stereo-inertial local maps of EuRoC / TUM-VI that the paper
evaluates on (Section V, Experimental Setup): keyframes carrying hundreds to thousands of
features, local maps with thousands to tens of thousands of points (Section IV-A).

Camera: pinhole 752x480, fx=fy=458, cx=367, cy=248, no distortion, frame x right / y down
/ z forward; stereo baseline 0.11 m (bf = 50.38 px*m).  Observation noise on u, v, uR is
N(0, (1.2^o)^2) for octave o ~ U{0..7}; exactly round(0.05 N) observations are replaced by
uniform outliers; optimisable keyframes start at Exp(w, v) * T_true with per-axis
w ~ N(0, 0.5 deg), v ~ N(0, 2 cm), points at X_true + N(0, 5 cm).

Draw order inside one window (one ``numpy.random.Generator``): trajectory, points
(rejection batches), octaves, stereo choice, pixel noise, outlier indices, outlier values,
pose perturbations, point perturbations.  Multi-window configurations draw each window
from ``SeedSequence(seed).spawn(n)``; a window's own size parameters come first.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import expm

FX = FY = 458.0
CX, CY = 367.0, 248.0
WIDTH, HEIGHT = 752, 480
BASELINE_M = 0.11
BF = BASELINE_M * FX
N_LEVELS = 8
SCALE_FACTOR = 1.2
MIN_DEPTH_VIS = 0.1
HUBER2_MONO = 5.991
HUBER2_STEREO = 7.815

CAM = np.array([FX, FY, CX, CY, BF], dtype=np.float64)
SIGMA2 = np.array([SCALE_FACTOR ** (2 * o) for o in range(N_LEVELS)], dtype=np.float64)


# ----------------------------------------------------------------------------------------
# geometry helpers (generation only)
# ----------------------------------------------------------------------------------------
def _look_rotation(z_axis: np.ndarray) -> np.ndarray:
    """Camera-to-world rotation whose optical axis is ``z_axis`` and whose y axis points
    as close to world +y (down) as possible."""
    z = z_axis / np.linalg.norm(z_axis)
    x = np.cross(np.array([0.0, 1.0, 0.0]), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    return np.stack([x, y, z], axis=1)


def _pose_from_center(R_wc: np.ndarray, c: np.ndarray) -> np.ndarray:
    R_cw = R_wc.T
    t_cw = -R_cw @ c
    return np.concatenate([R_cw, t_cw[:, None]], axis=1)


def _twist_exp(w: np.ndarray, v: np.ndarray) -> np.ndarray:
    """4x4 matrix exponential of the twist (rotation w, translation v) via SciPy."""
    A = np.zeros((4, 4))
    A[0, 1], A[0, 2], A[1, 2] = -w[2], w[1], -w[0]
    A[1, 0], A[2, 0], A[2, 1] = w[2], -w[1], w[0]
    A[:3, 3] = v
    return expm(A)


def _project(T: np.ndarray, X: np.ndarray):
    """Noise-free pinhole projection of points X (M,3) into poses T (K,3,4).

    Returns camera-frame depth (M,K), u, v, uR (M,K)."""
    R = T[:, :, :3]
    t = T[:, :, 3]
    Xc = np.einsum("kij,mj->mki", R, X) + t[None, :, :]
    z = Xc[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = FX * Xc[..., 0] / z + CX
        v = FY * Xc[..., 1] / z + CY
        ur = u - BF / z
    return z, u, v, ur


def _visible(z, u, v):
    return (z > MIN_DEPTH_VIS) & (u >= 0) & (u < WIDTH) & (v >= 0) & (v < HEIGHT)


# ----------------------------------------------------------------------------------------
# trajectories
# ----------------------------------------------------------------------------------------
def _arc_trajectory(K: int) -> tuple[np.ndarray, np.ndarray]:
    """K keyframes on a radius-2 m circle, evenly spaced over 1 rad (arc length 2 m),
    optical axis horizontal and pointing at the circle centre."""
    phis = np.linspace(-0.5, 0.5, K)
    poses, centers = [], []
    for phi in phis:
        c = np.array([2.0 * math.sin(phi), 0.0, -2.0 * math.cos(phi)])
        R_wc = _look_rotation(-c)
        poses.append(_pose_from_center(R_wc, c))
        centers.append(c)
    return np.array(poses), np.array(centers)


def _walk_trajectory(rng: np.random.Generator, K: int, length: float):
    """K keyframes along a random walk of the given length: heading yaw / pitch random
    walks N(0, 10 deg) / N(0, 2 deg) per step, look direction = heading yaw + N(0, 5 deg)."""
    step = length / max(K - 1, 1)
    yaw = pitch = 0.0
    p = np.zeros(3)
    poses, centers = [], []
    d2r = math.pi / 180.0
    for i in range(K):
        if i > 0:
            yaw += rng.normal(0.0, 10.0 * d2r)
            pitch += rng.normal(0.0, 2.0 * d2r)
            p = p + step * np.array([math.sin(yaw) * math.cos(pitch), -math.sin(pitch),
                                     math.cos(yaw) * math.cos(pitch)])
        look_yaw = yaw + rng.normal(0.0, 5.0 * d2r)
        d = np.array([math.sin(look_yaw) * math.cos(pitch), -math.sin(pitch),
                      math.cos(look_yaw) * math.cos(pitch)])
        poses.append(_pose_from_center(_look_rotation(d), p.copy()))
        centers.append(p.copy())
    return np.array(poses), np.array(centers)


# ----------------------------------------------------------------------------------------
# one window
# ----------------------------------------------------------------------------------------
def make_window(rng: np.random.Generator, *, trajectory: str, K: int, n_fixed: int, M: int,
                nobs: tuple[int, int], stereo_p: float, walk_length: float = 6.0,
                depth: tuple[float, float] = (1.0, 12.0), noise: bool = True,
                outlier_frac: float = 0.05) -> dict:
    """Build one window.  ``nobs=(lo, hi)`` draws each point's wanted observation count
    from U{lo..hi} (lo == hi for a fixed count); it is capped by visibility."""
    if trajectory == "arc":
        T_true, centers = _arc_trajectory(K)
    else:
        T_true, centers = _walk_trajectory(rng, K, walk_length)

    # --- points, redrawn until each is visible in >= 2 keyframes -----------------------
    pts = []
    have = 0
    while have < M:
        need = M - have
        nb = need + need // 4 + 16
        if trajectory == "arc":
            lo = np.array([-1.5, -1.0, 2.0])
            hi = np.array([1.5, 1.0, 8.0])
            P_c = rng.uniform(lo, hi, size=(nb, 3))
            mid = K // 2
            R_wc = T_true[mid, :, :3].T
            c = centers[mid]
            cand = P_c @ R_wc.T + c
        else:
            anchor = rng.integers(0, K, size=nb)
            uu = rng.uniform(0.0, WIDTH, size=nb)
            vv = rng.uniform(0.0, HEIGHT, size=nb)
            dd = rng.uniform(depth[0], depth[1], size=nb)
            P_c = np.stack([(uu - CX) / FX * dd, (vv - CY) / FY * dd, dd], axis=1)
            R_wc = np.transpose(T_true[anchor, :, :3], (0, 2, 1))
            cand = np.einsum("nij,nj->ni", R_wc, P_c) + centers[anchor]
        z, u, v, _ = _project(T_true, cand)
        ok = _visible(z, u, v).sum(axis=1) >= 2
        cand = cand[ok][:need]
        pts.append(cand)
        have += len(cand)
    X_true = np.concatenate(pts, axis=0)[:M]

    # --- association: each point seen by its n nearest visible keyframes ---------------
    z, u, v, ur = _project(T_true, X_true)
    vis = _visible(z, u, v)
    dist = np.linalg.norm(X_true[:, None, :] - centers[None, :, :], axis=2)
    dist = np.where(vis, dist, np.inf)
    order = np.argsort(dist, axis=1, kind="stable")
    if nobs[0] == nobs[1]:
        want = np.full(M, nobs[0])
    else:
        want = rng.integers(nobs[0], nobs[1] + 1, size=M)
    take = np.minimum(want, vis.sum(axis=1))
    sel = np.arange(K)[None, :] < take[:, None]
    pt_idx = np.repeat(np.arange(M), K).reshape(M, K)[sel]
    kf_idx = order[sel]
    # sort by point, then keyframe
    srt = np.lexsort((kf_idx, pt_idx))
    pt_idx = pt_idx[srt].astype(np.int32)
    kf_idx = kf_idx[srt].astype(np.int32)
    N = len(pt_idx)
    zz = z[pt_idx, kf_idx]
    u0 = u[pt_idx, kf_idx]
    v0 = v[pt_idx, kf_idx]
    ur0 = ur[pt_idx, kf_idx]

    # --- octaves, stereo choice, noise --------------------------------------------------
    octv = rng.integers(0, N_LEVELS, size=N).astype(np.uint8)
    stereo_ok = ur0 >= 0.0
    is_stereo = (rng.uniform(size=N) < stereo_p) & stereo_ok
    sig = SCALE_FACTOR ** octv.astype(np.float64)
    nz = rng.normal(size=(3, N)) * sig[None, :]
    if not noise:
        nz[:] = 0.0
    obs_z = np.empty((3, N))
    obs_z[0] = u0 + nz[0]
    obs_z[1] = v0 + nz[1]
    obs_z[2] = np.where(is_stereo, ur0 + nz[2], -1.0)

    # --- outliers ------------------------------------------------------------------------
    is_out = np.zeros(N, dtype=bool)
    n_out = int(round(outlier_frac * N)) if noise else 0
    if n_out > 0:
        idx = rng.choice(N, size=n_out, replace=False)
        uo = rng.uniform(0.0, WIDTH, size=n_out)
        vo = rng.uniform(0.0, HEIGHT, size=n_out)
        do = rng.uniform(0.0, BF / depth[0], size=n_out)
        obs_z[0, idx] = uo
        obs_z[1, idx] = vo
        obs_z[2, idx] = np.where(is_stereo[idx], uo - do, -1.0)
        is_out[idx] = True

    # --- initial perturbation ------------------------------------------------------------
    fixed = np.zeros(K, dtype=np.uint8)
    fixed[:n_fixed] = 1
    T_init = T_true.copy()
    d2r = math.pi / 180.0
    for k in range(K):
        if fixed[k]:
            continue
        w = rng.normal(0.0, 0.5 * d2r, size=3)
        vv = rng.normal(0.0, 0.02, size=3)
        E = _twist_exp(w, vv)
        T4 = np.vstack([T_true[k], [0, 0, 0, 1]])
        T_init[k] = (E @ T4)[:3]
    X_init = X_true + rng.normal(0.0, 0.05, size=X_true.shape)

    return {
        "T_cw": T_init.reshape(K, 12).copy(),
        "T_true": T_true.reshape(K, 12).copy(),
        "fixed": fixed,
        "X": X_init,
        "X_true": X_true,
        "obs_kf": kf_idx,
        "obs_pt": pt_idx,
        "obs_z": np.ascontiguousarray(obs_z),
        "obs_type": is_stereo.astype(np.uint8),
        "obs_oct": octv,
        "sigma2": SIGMA2.copy(),
        "cam": CAM.copy(),
        "is_outlier_true": is_out,
    }


# ----------------------------------------------------------------------------------------
# the five workload configurations
# ----------------------------------------------------------------------------------------
def c1_mono(seed: int = 0, noise: bool = True) -> dict:
    """Monocular window: 10 optimisable + 5 fixed keyframes on a 2 m arc, 1,500 points in
    a box 2-8 m deep, each seen by its 8 nearest visible keyframes (about 12k obs)."""
    rng = np.random.default_rng(seed)
    return make_window(rng, trajectory="arc", K=15, n_fixed=5, M=1500, nobs=(8, 8),
                       stereo_p=0.0, depth=(2.0, 8.0), noise=noise)


def c2_stereo(seed: int = 1, noise: bool = True) -> dict:
    """Stereo window: 20 optimisable + 10 fixed keyframes on a 6 m random walk, 8,000
    points 1-12 m deep, 8 observations per point (about 60k obs, 70% stereo)."""
    rng = np.random.default_rng(seed)
    return make_window(rng, trajectory="walk", K=30, n_fixed=10, M=8000, nobs=(8, 8),
                       stereo_p=0.7, walk_length=6.0, noise=noise)


def c3_precision(seed: int = 2, noise: bool = True) -> dict:
    """Large stereo window: 30 optimisable + 20 fixed keyframes over 10 m, 20,000 points,
    10 observations per point (about 200k obs)."""
    rng = np.random.default_rng(seed)
    return make_window(rng, trajectory="walk", K=50, n_fixed=20, M=20000, nobs=(10, 10),
                       stereo_p=0.7, walk_length=10.0, noise=noise)


def c4_windows(seed: int = 3, n_windows: int = 64, noise: bool = True) -> list[dict]:
    """64 windows of 10 keyframes (2 m walk) and 2,000 points, 8 obs per point; even
    windows monocular, odd windows 70/30 stereo/mono."""
    out = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(n_windows)):
        rng = np.random.default_rng(ss)
        out.append(make_window(rng, trajectory="walk", K=10, n_fixed=3, M=2000, nobs=(8, 8),
                               stereo_p=0.0 if i % 2 == 0 else 0.7, walk_length=2.0,
                               noise=noise))
    return out


def c5_window_sizes(seed: int = 4, n_windows: int = 256) -> list[tuple[int, int]]:
    """(K, M) of each batched window, drawn first from that window's own stream."""
    sizes = []
    for ss in np.random.SeedSequence(seed).spawn(n_windows):
        rng = np.random.default_rng(ss)
        sizes.append((int(rng.integers(5, 41)), int(rng.integers(500, 20001))))
    return sizes


def c5_windows(seed: int = 4, n_windows: int = 256, noise: bool = True,
               only: list[int] | None = None, max_points: int | None = None) -> list[dict]:
    """Batched windows: K ~ U{5..40} with floor(K/3) fixed, walk of 0.2 K m, points
    M ~ U{500..20,000}, 4-10 observations per point, 70/30 stereo/mono.  ``only`` builds
    a subset of the windows (same streams, so the same content); ``max_points`` caps M
    (smaller test batches with the same structure)."""
    out = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(n_windows)):
        if only is not None and i not in only:
            continue
        rng = np.random.default_rng(ss)
        K = int(rng.integers(5, 41))
        M = int(rng.integers(500, 20001))
        if max_points is not None:
            M = min(M, max_points)
        out.append(make_window(rng, trajectory="walk", K=K, n_fixed=K // 3, M=M, nobs=(4, 10),
                               stereo_p=0.7, walk_length=0.2 * K, noise=noise))
    return out


def tiny_window(seed: int, K: int = 4, n_fixed: int = 1, M: int = 20, stereo_p: float = 0.5,
                noise: bool = True, nobs: tuple[int, int] = (2, 4), outlier_frac: float = 0.05) -> dict:
    """Small window for brute-force checks (dense normal equations, finite differences)."""
    rng = np.random.default_rng(seed)
    return make_window(rng, trajectory="walk", K=K, n_fixed=n_fixed, M=M, nobs=nobs,
                       stereo_p=stereo_p, walk_length=0.3 * K, noise=noise,
                       outlier_frac=outlier_frac)


def concat(windows: list[dict]) -> dict:
    """Concatenate windows into one batch: arrays end to end, observation indices stay
    window-local, offsets give each window's keyframe / point / observation range."""
    kf_off = np.zeros(len(windows) + 1, dtype=np.int64)
    pt_off = np.zeros(len(windows) + 1, dtype=np.int64)
    ob_off = np.zeros(len(windows) + 1, dtype=np.int64)
    for i, w in enumerate(windows):
        kf_off[i + 1] = kf_off[i] + len(w["fixed"])
        pt_off[i + 1] = pt_off[i] + len(w["X"])
        ob_off[i + 1] = ob_off[i] + len(w["obs_kf"])
    cat = {
        "T_cw": np.concatenate([w["T_cw"] for w in windows]),
        "fixed": np.concatenate([w["fixed"] for w in windows]),
        "X": np.concatenate([w["X"] for w in windows]),
        "obs_kf": np.concatenate([w["obs_kf"] for w in windows]),
        "obs_pt": np.concatenate([w["obs_pt"] for w in windows]),
        "obs_z": np.concatenate([w["obs_z"] for w in windows], axis=1),
        "obs_type": np.concatenate([w["obs_type"] for w in windows]),
        "obs_oct": np.concatenate([w["obs_oct"] for w in windows]),
        "sigma2": windows[0]["sigma2"],
        "cam": windows[0]["cam"],
        "kf_off": kf_off, "pt_off": pt_off, "obs_off": ob_off,
    }
    return cat


# ----------------------------------------------------------------------------------------
# keyframe store for the correspondence and fusion searches
# ----------------------------------------------------------------------------------------
DESC_WORDS = 8   # 256-bit binary descriptors, eight 32-bit words


def _random_descriptors(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.integers(0, 1 << 32, size=(n, DESC_WORDS), dtype=np.uint64).astype(np.uint32)


def _flip_bits(rng: np.random.Generator, d: np.ndarray, p: float) -> np.ndarray:
    """Each of the 256 bits of each descriptor flipped independently with probability p."""
    bits = rng.uniform(size=(d.shape[0], DESC_WORDS, 32)) < p
    mask = (bits.astype(np.uint64) << np.arange(32, dtype=np.uint64)).sum(axis=2).astype(np.uint32)
    return d ^ mask


def keyframe_store(seed: int = 5, K: int = 80, M: int = 30000, kp_per_kf: int = 1200,
                   walk_length: float = 16.0, true_frac: float = 0.8, free_p: float = 0.6,
                   flip_p: float = 0.05, stereo_p: float = 0.7) -> dict:
    """Keyframes of a local map with their keypoints, as a GPU-resident keyframe store
    would hold them: poses, keypoint positions (left u, v and right uR or -1), octaves,
    256-bit descriptors and a 'free' flag (the keypoint has no map point yet).

    Each keyframe gets kp_per_kf keypoints: true_frac of them are projections of visible
    map points (octave U{0..7}, pixel noise N(0, 1.2^octave), the point's descriptor with
    each bit flipped with probability flip_p, a right coordinate with probability
    stereo_p when the point is stereo-visible), the rest distractors at uniform image
    positions with uniform random descriptors.  Keypoints are shuffled within their
    keyframe.  Draw order: trajectory, points, point descriptors, then per keyframe:
    selection, octaves, noise, stereo choice, flips, distractors, shuffle, free flags."""
    rng = np.random.default_rng(seed)
    T, centers = _walk_trajectory(rng, K, walk_length)
    anchor = rng.integers(0, K, size=M)
    uu = rng.uniform(0.0, WIDTH, size=M)
    vv = rng.uniform(0.0, HEIGHT, size=M)
    dd = rng.uniform(1.0, 12.0, size=M)
    P_c = np.stack([(uu - CX) / FX * dd, (vv - CY) / FY * dd, dd], axis=1)
    R_wc = np.transpose(T[anchor, :, :3], (0, 2, 1))
    X = np.einsum("nij,nj->ni", R_wc, P_c) + centers[anchor]
    pdesc = _random_descriptors(rng, M)
    z, u, v, ur = _project(T, X)
    vis = _visible(z, u, v)
    n_true = int(round(true_frac * kp_per_kf))
    cols = dict(u=[], v=[], ur=[], oct=[], free=[], desc=[], pt=[])
    kp_off = [0]
    for k in range(K):
        cand = np.nonzero(vis[:, k])[0]
        sel = np.sort(rng.choice(cand, size=min(n_true, len(cand)), replace=False))
        nt = len(sel)
        octv = rng.integers(0, N_LEVELS, size=nt)
        sig = SCALE_FACTOR ** octv
        nz = rng.normal(size=(3, nt)) * sig[None, :]
        st = (rng.uniform(size=nt) < stereo_p) & (ur[sel, k] >= 0.0)
        ku = u[sel, k] + nz[0]
        kv = v[sel, k] + nz[1]
        kur = np.where(st, ur[sel, k] + nz[2], -1.0)
        kd = _flip_bits(rng, pdesc[sel], flip_p)
        nd = kp_per_kf - nt
        du = rng.uniform(0.0, WIDTH, size=nd)
        dv = rng.uniform(0.0, HEIGHT, size=nd)
        doct = rng.integers(0, N_LEVELS, size=nd)
        dst = rng.uniform(size=nd) < stereo_p
        dur = np.where(dst, du - rng.uniform(0.0, BF / 1.0, size=nd), -1.0)
        ddesc = _random_descriptors(rng, nd)
        perm = rng.permutation(kp_per_kf)
        cols["u"].append(np.concatenate([ku, du])[perm])
        cols["v"].append(np.concatenate([kv, dv])[perm])
        cols["ur"].append(np.concatenate([kur, dur])[perm])
        cols["oct"].append(np.concatenate([octv, doct])[perm])
        cols["desc"].append(np.concatenate([kd, ddesc])[perm])
        cols["pt"].append(np.concatenate([sel, np.full(nd, -1)])[perm])
        cols["free"].append(rng.uniform(size=kp_per_kf) < free_p)
        kp_off.append(kp_off[-1] + kp_per_kf)
    return {
        "T_cw": T.reshape(K, 12).copy(),
        "centers": centers,
        "kp_off": np.array(kp_off, dtype=np.int32),
        "kp_u": np.concatenate(cols["u"]).astype(np.float32),
        "kp_v": np.concatenate(cols["v"]).astype(np.float32),
        "kp_ur": np.concatenate(cols["ur"]).astype(np.float32),
        "kp_oct": np.concatenate(cols["oct"]).astype(np.uint8),
        "kp_free": np.concatenate(cols["free"]).astype(np.uint8),
        "kp_desc": np.ascontiguousarray(np.concatenate(cols["desc"]), dtype=np.uint32),
        "kp_pt": np.concatenate(cols["pt"]).astype(np.int32),
        "X_true": X,
        "pt_desc": pdesc,
        "sigma2": SIGMA2.copy(),
        "scale": np.array([SCALE_FACTOR ** o for o in range(N_LEVELS)]),
        "cam": CAM.copy(),
        "width": WIDTH,
        "height": HEIGHT,
    }


def nearest_keyframes(store: dict, k: int, n: int) -> np.ndarray:
    """The n keyframes other than k with the closest camera centres (stable order)."""
    c = store["centers"]
    d = np.linalg.norm(c - c[k], axis=1)
    d[k] = np.inf
    return np.argsort(d, kind="stable")[:n].astype(np.int32)


def correspondence_queries(store: dict, n_cur: int = 64, n_nbr: int = 10):
    """(current, neighbour) keyframe pairs: each of the last n_cur keyframes with its
    n_nbr nearest keyframes."""
    K = len(store["kp_off"]) - 1
    cur, nbr = [], []
    for k in range(K - n_cur, K):
        for m in nearest_keyframes(store, k, n_nbr):
            cur.append(k)
            nbr.append(int(m))
    return np.array(cur, dtype=np.int32), np.array(nbr, dtype=np.int32)


def fusion_points(store: dict, seed: int = 6, n_cur: int = 64, n_nbr: int = 20, pos_sigma: float = 0.02,
                  flip_p: float = 0.02):
    """Map points of the last n_cur keyframes (the true points behind each keyframe's
    associated, i.e. non-free, keypoints), with what a map point carries for the fusion
    search: position (truth + N(0, pos_sigma) per axis), descriptor (the point's with
    bits flipped with probability flip_p), mean viewing direction over the store's
    keyframes that see it, and the distance range of scale invariance (the distance from
    the keyframe times 1.2^octave of its keypoint, down to that over 1.2^7).  Returns the
    points concatenated over keyframes and the queries (point range, neighbour keyframe):
    every keyframe's points against its n_nbr nearest keyframes."""
    rng = np.random.default_rng(seed)
    K = len(store["kp_off"]) - 1
    cen = store["centers"]
    kp_pt, kp_off = store["kp_pt"], store["kp_off"]
    seen_by = {}
    for k in range(K):
        for p in kp_pt[kp_off[k]:kp_off[k + 1]]:
            if p >= 0:
                seen_by.setdefault(int(p), []).append(k)
    X, D, Nrm, dmin, dmax = [], [], [], [], []
    q_p0, q_p1, q_nbr = [], [], []
    for k in range(K - n_cur, K):
        sl = slice(kp_off[k], kp_off[k + 1])
        pts = kp_pt[sl]
        octs = store["kp_oct"][sl]
        keep = (pts >= 0) & (store["kp_free"][sl] == 0)
        p0 = sum(len(x) for x in X)
        P = pts[keep]
        Xt = store["X_true"][P]
        nv = np.stack([np.mean([(Xt[i] - cen[m]) / np.linalg.norm(Xt[i] - cen[m]) for m in seen_by[int(p)]],
                               axis=0) for i, p in enumerate(P)]) if len(P) else np.zeros((0, 3))
        nv = nv / np.linalg.norm(nv, axis=1, keepdims=True) if len(P) else nv
        dist = np.linalg.norm(Xt - cen[k], axis=1)
        mx = dist * SCALE_FACTOR ** octs[keep].astype(np.float64)
        X.append(Xt + rng.normal(0.0, pos_sigma, size=Xt.shape))
        D.append(_flip_bits(rng, store["pt_desc"][P], flip_p))
        Nrm.append(nv)
        dmax.append(mx)
        dmin.append(mx / SCALE_FACTOR ** (N_LEVELS - 1))
        p1 = p0 + len(P)
        for m in nearest_keyframes(store, k, n_nbr):
            q_p0.append(p0)
            q_p1.append(p1)
            q_nbr.append(int(m))
    pts = {
        "X": np.concatenate(X),
        "desc": np.ascontiguousarray(np.concatenate(D), dtype=np.uint32),
        "normal": np.concatenate(Nrm),
        "dmin": np.concatenate(dmin),
        "dmax": np.concatenate(dmax),
    }
    q = (np.array(q_p0, dtype=np.int32), np.array(q_p1, dtype=np.int32), np.array(q_nbr, dtype=np.int32))
    return pts, q


# ----------------------------------------------------------------------------------------
# stereo-inertial windows
# ----------------------------------------------------------------------------------------
GRAVITY = np.array([0.0, 9.81, 0.0])   # world frame of the walks: y points down
# body (IMU) to camera: a small fixed rotation and a lever arm of a few centimetres
_R_CB = expm(np.array([[0.0, -0.03, -0.01], [0.03, 0.0, -0.02], [0.01, 0.02, 0.0]]))
T_CB = np.concatenate([_R_CB, np.array([[0.05], [-0.02], [0.01]])], axis=1)


def _so3(w):
    return expm(np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]]))


def vi_window(seed: int, K: int = 15, n_fixed: int = 5, M: int = 6000, nobs: tuple[int, int] = (8, 8),
              stereo_p: float = 0.7, walk_length: float = 4.0, noise: bool = True) -> tuple[dict, dict]:
    """A stereo-inertial window: the visual window of ``make_window`` (walk trajectory) and,
    between consecutive keyframes, a preintegrated inertial measurement consistent with the
    true body motion.

    Body frame: camera pose T_cw and body-to-camera T_CB give the body rotation
    R = R_cw^T R_cb and position p = R_cw^T (t_cb - t_cw).  Keyframes are dt ~ U[0.2, 0.3] s
    apart; true velocities are central differences of the body positions over time (one-
    sided at the ends); true biases bg ~ N(0, 2e-3) rad/s and ba ~ N(0, 2e-2) m/s^2 per axis
    at the first keyframe, then a random walk of N(0, 1e-4) / N(0, 1e-3) per edge.  Each
    measurement carries the biases it was integrated with (truth + N(0, 1e-3) / N(0, 1e-2))
    and bias Jacobians near their first-order values (J_Rg ~ -dt I, J_va ~ -dt I,
    J_pa ~ -dt^2/2 I, J_vg and J_pg small), plus N(0, 0.05 scale) perturbations; its
    (dR, dv, dp) give a zero inertial residual at the true states, then (noise only) are
    perturbed by a draw of the measurement's own covariance.  Information: the inverse of a
    correlated 9x9 covariance with standard deviations 2e-3 rad, 5e-3 m/s, 1e-3 m; bias
    random-walk information 1 / (1e-4^2 dt) and 1 / (1e-3^2 dt).  Optimisable keyframes
    start with velocities + N(0, 0.05) m/s, biases + N(0, 1e-3) / N(0, 1e-2).

    Draw order after the visual window (same generator): time steps, biases at the first
    keyframe, bias walks, per edge (integration biases, Jacobian perturbations, covariance
    factor, measurement noise), velocity and bias perturbations."""
    rng = np.random.default_rng(seed)
    w = make_window(rng, trajectory="walk", K=K, n_fixed=n_fixed, M=M, nobs=nobs, stereo_p=stereo_p,
                    walk_length=walk_length, noise=noise)
    T = w["T_true"].reshape(K, 3, 4)
    Rcb, tcb = T_CB[:, :3], T_CB[:, 3]
    Rb = np.einsum("kji,jl->kil", T[:, :, :3], Rcb)               # R_cw^T R_cb
    pb = np.einsum("kji,kj->ki", T[:, :, :3], tcb[None, :] - T[:, :, 3])
    dts = rng.uniform(0.2, 0.3, size=K - 1)
    t = np.concatenate([[0.0], np.cumsum(dts)])
    v = np.empty((K, 3))
    for k in range(K):
        a, b = max(k - 1, 0), min(k + 1, K - 1)
        v[k] = (pb[b] - pb[a]) / (t[b] - t[a])
    bg = np.empty((K, 3))
    ba = np.empty((K, 3))
    bg[0] = rng.normal(0.0, 2e-3, 3)
    ba[0] = rng.normal(0.0, 2e-2, 3)
    steps_g = rng.normal(0.0, 1e-4, (K - 1, 3))
    steps_a = rng.normal(0.0, 1e-3, (K - 1, 3))
    for k in range(1, K):
        bg[k] = bg[k - 1] + (steps_g[k - 1] if noise else 0.0)
        ba[k] = ba[k - 1] + (steps_a[k - 1] if noise else 0.0)
    sig = np.array([2e-3] * 3 + [5e-3] * 3 + [1e-3] * 3)
    E = dict(edge_i=[], edge_j=[], dt=[], dR=[], dv=[], dp=[], J_Rg=[], J_vg=[], J_va=[], J_pg=[], J_pa=[],
             bg_bar=[], ba_bar=[], info=[], info_bg=[], info_ba=[])
    I3 = np.eye(3)
    for e in range(K - 1):
        i, j, dt = e, e + 1, dts[e]
        bgb = bg[i] + rng.normal(0.0, 1e-3, 3)
        bab = ba[i] + rng.normal(0.0, 1e-2, 3)
        pert = rng.normal(0.0, 0.05, (5, 3, 3))
        J_Rg = -dt * (I3 + pert[0])
        J_vg = 0.5 * dt * dt * pert[1]
        J_va = -dt * (I3 + pert[2])
        J_pg = dt ** 3 / 6.0 * pert[3]
        J_pa = -0.5 * dt * dt * (I3 + pert[4])
        Lf = np.diag(sig) @ (np.eye(9) + 0.1 * np.tril(rng.normal(size=(9, 9)), -1))
        cov = Lf @ Lf.T
        n9 = Lf @ rng.normal(size=9) if noise else np.zeros(9)
        dbg, dba = bg[i] - bgb, ba[i] - bab
        # measurements that zero the residual at the true states, then the noise
        dR = Rb[i].T @ Rb[j] @ _so3(J_Rg @ dbg).T
        dv = Rb[i].T @ (v[j] - v[i] - GRAVITY * dt) - J_vg @ dbg - J_va @ dba
        dp = Rb[i].T @ (pb[j] - pb[i] - v[i] * dt - 0.5 * GRAVITY * dt * dt) - J_pg @ dbg - J_pa @ dba
        dR = dR @ _so3(-n9[:3])
        dv = dv + n9[3:6]
        dp = dp + n9[6:9]
        for k_, val in (("edge_i", i), ("edge_j", j), ("dt", dt), ("dR", dR), ("dv", dv), ("dp", dp),
                        ("J_Rg", J_Rg), ("J_vg", J_vg), ("J_va", J_va), ("J_pg", J_pg), ("J_pa", J_pa),
                        ("bg_bar", bgb), ("ba_bar", bab), ("info", np.linalg.inv(cov)),
                        ("info_bg", 1.0 / (1e-4 ** 2 * dt)), ("info_ba", 1.0 / (1e-3 ** 2 * dt))):
            E[k_].append(val)
    vi = {k: np.asarray(x) for k, x in E.items()}
    vi["edge_i"] = vi["edge_i"].astype(np.int32)
    vi["edge_j"] = vi["edge_j"].astype(np.int32)
    vi["T_cb"] = T_CB.copy()
    vi["g"] = GRAVITY.copy()
    vi["v_true"], vi["bg_true"], vi["ba_true"] = v.copy(), bg.copy(), ba.copy()
    v0, bg0, ba0 = v.copy(), bg.copy(), ba.copy()
    dv0 = rng.normal(0.0, 0.05, (K, 3))
    dg0 = rng.normal(0.0, 1e-3, (K, 3))
    da0 = rng.normal(0.0, 1e-2, (K, 3))
    opt = w["fixed"] == 0
    v0[opt] += dv0[opt]
    bg0[opt] += dg0[opt]
    ba0[opt] += da0[opt]
    vi["v"], vi["bg"], vi["ba"] = v0, bg0, ba0
    return w, vi


def vi_stereo(seed: int = 7, noise: bool = True) -> tuple[dict, dict]:
    """Stereo-inertial window: 10 optimisable + 5 fixed keyframes on a 4 m walk, 6,000
    points, 8 observations per point (70% stereo): a reduced system of 150 unknowns."""
    return vi_window(seed, K=15, n_fixed=5, M=6000, nobs=(8, 8), stereo_p=0.7, walk_length=4.0, noise=noise)


def concat_vi(pairs: list[tuple[dict, dict]]) -> tuple[dict, dict]:
    """Batch of stereo-inertial windows: the visual windows concatenated (``concat``) and
    their inertial measurements and states end to end, with ``edge_off`` (keyframe indices
    stay local to their window)."""
    w = concat([p[0] for p in pairs])
    vis = [p[1] for p in pairs]
    per_edge = ["edge_i", "edge_j", "dt", "dR", "dv", "dp", "J_Rg", "J_vg", "J_va", "J_pg", "J_pa", "bg_bar",
                "ba_bar", "info", "info_bg", "info_ba"]
    vi = {k: np.concatenate([np.asarray(x[k]) for x in vis]) for k in per_edge}
    for k in ("v", "bg", "ba", "v_true", "bg_true", "ba_true"):
        vi[k] = np.concatenate([x[k] for x in vis])
    vi["edge_off"] = np.concatenate([[0], np.cumsum([len(x["dt"]) for x in vis])]).astype(np.int32)
    vi["T_cb"] = vis[0]["T_cb"].copy()
    vi["g"] = vis[0]["g"].copy()
    return w, vi
