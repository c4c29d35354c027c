"""Comparison helpers shared by the GPU tests (GPU result vs the FP64 CPU oracle)."""
import numpy as np

CHI2 = {0: 5.991, 1: 7.815}


def weighted_sq_error(w, T, X):
    """s of every observation at (T, X), plus depth (NumPy, for flag bands)."""
    cam = w["cam"]
    Tk = np.asarray(T).reshape(-1, 3, 4)[w["obs_kf"]]
    Xj = np.asarray(X).reshape(-1, 3)[w["obs_pt"]]
    Xc = np.einsum("nij,nj->ni", Tk[:, :, :3], Xj) + Tk[:, :, 3]
    u = cam[0] * Xc[:, 0] / Xc[:, 2] + cam[2]
    v = cam[1] * Xc[:, 1] / Xc[:, 2] + cam[3]
    st = w["obs_type"].astype(bool)
    e2 = (w["obs_z"][0] - u) ** 2 + (w["obs_z"][1] - v) ** 2
    e2 = e2 + np.where(st, (w["obs_z"][2] - (u - cam[4] / Xc[:, 2])) ** 2, 0.0)
    return e2 / w["sigma2"][w["obs_oct"]], Xc[:, 2]


def projections(w, T, X):
    cam = w["cam"]
    Tk = np.asarray(T).reshape(-1, 3, 4)[w["obs_kf"]]
    Xj = np.asarray(X).reshape(-1, 3)[w["obs_pt"]]
    Xc = np.einsum("nij,nj->ni", Tk[:, :, :3], Xj) + Tk[:, :, 3]
    u = cam[0] * Xc[:, 0] / Xc[:, 2] + cam[2]
    v = cam[1] * Xc[:, 1] / Xc[:, 2] + cam[3]
    ur = u - cam[4] / Xc[:, 2]
    return np.stack([u, v, ur], axis=1)


def assert_fp64_parity(w, g_T, g_X, g_flags, g_stats, ref, cost_rel=1e-9, state_tol=1e-8):
    """Plain FP64 GPU vs oracle: final cost to 1e-9 relative, pose and point entries to
    1e-8 * max(1, |ref|), identical outlier flags except observations whose s lies
    within 1e-9 (relative) of the threshold at the oracle's final state."""
    Fr = ref["stats"]["F_final"]
    Fg = g_stats["F_final"]
    # relative bound, with an absolute floor at rounding level for windows the data fits
    # exactly (F ~ 1e-27 on both sides)
    floor = 1e-15 * max(1, len(w["obs_kf"]))
    assert abs(Fg - Fr) <= cost_rel * abs(Fr) + floor, (Fg, Fr)
    dT = np.abs(g_T - ref["T"]) / np.maximum(1.0, np.abs(ref["T"]))
    dX = np.abs(g_X - ref["X"]) / np.maximum(1.0, np.abs(ref["X"]))
    assert dT.max(initial=0.0) <= state_tol, ("pose", dT.max())
    assert dX.max(initial=0.0) <= state_tol, ("point", dX.max(), np.unravel_index(dX.argmax(), dX.shape))
    s, _ = weighted_sq_error(w, ref["T"], ref["X"])
    thr = np.where(w["obs_type"].astype(bool), CHI2[1], CHI2[0])
    band = np.abs(s - thr) <= 1e-9 * thr
    diff = (g_flags != ref["outlier"]) & ~band
    assert not diff.any(), ("flags", int(diff.sum()))
    # iteration counts are only comparable while no trial reached the rounding floor:
    # once |F - F'| is at the level of F's rounding, accept / reject is decided by noise
    if not schedule_is_noisy(w, ref):
        for k in ("iters_r1", "iters_r2", "n_outliers", "trials", "term_r1", "term_r2"):
            assert g_stats[k] == ref["stats"][k], (k, g_stats[k], ref["stats"][k])
        if any(l["round"] == 2 for l in ref["log"]):
            # the damping after the last trial: products of gain-dependent factors, each
            # gain carrying the relative error of F - F' (at most 1e-6 away from the floor)
            lr = ref["stats"]["lambda"]
            assert abs(g_stats["lambda"] - lr) <= 1e-6 * abs(lr), ("lambda", g_stats["lambda"], lr)


def schedule_is_noisy(w, ref):
    """True once any oracle trial reached the rounding floor: when |F - F'| is at the level
    of F's rounding, accept / reject (and every count after it) is decided by noise."""
    floor = 1e-15 * max(1, len(w["obs_kf"]))
    return any(np.isfinite(l["F_trial"]) and abs(l["F"] - l["F_trial"]) <= 1e-10 * abs(l["F"]) + floor
               for l in ref["log"])


def assert_trial_logs_match(w, g_log, r_log, rel=1e-9, cond_tau=None):
    """GPU per-trial log vs the oracle's, trial by trial: the same rounds, iterations, trial
    numbers, decisions and factorisation outcomes; lambda, F, F' and the gain ratio to
    `rel` (F' and gain only where the solve succeeded).  Stops at the first trial that
    reached the rounding floor (see schedule_is_noisy); returns the trials compared.

    A trial's step solves (H + lambda I) d = b, whose condition number is at most about
    max diag(H) / lambda; two correct solvers that round differently then differ in d, and
    so in F', by up to that factor times the rounding unit.  With the round's first damping
    lambda0 = tau * max diag(H), the bound of a trial is lambda0 / (tau * lambda).  A caller
    that starts the damping far below the curvature passes its tau as cond_tau, and F' is
    then held to rel + 1e-16 times that bound; by default it is held to rel."""
    floor = 1e-15 * max(1, len(w["obs_kf"]))
    n = 0
    lam0 = {}
    for g, r in zip(g_log, r_log):
        for k in ("round", "iter", "trial", "accepted", "solve_ok"):
            assert g[k] == r[k], (n, k, g, r)
        assert abs(g["lam"] - r["lam"]) <= 1e-6 * abs(r["lam"]), (n, "lambda", g, r)
        assert abs(g["F"] - r["F"]) <= rel * abs(r["F"]) + floor, (n, "F", g, r)
        lam0.setdefault(r["round"], r["lam"])
        n += 1
        if r["solve_ok"]:
            cond = lam0[r["round"]] / (cond_tau * r["lam"]) if cond_tau and r["lam"] > 0 else 0.0
            ftol = rel + 1e-16 * cond
            assert abs(g["F_trial"] - r["F_trial"]) <= ftol * abs(r["F_trial"]) + floor, (n, "F_trial", g, r)
            if abs(r["F"] - r["F_trial"]) <= 1e-10 * abs(r["F"]) + floor:
                return n
            # gain = (F - F') / den: relative error of F - F' is ~1e-16 F / |F - F'|, plus
            # the step's conditioning in F' and in the denominator
            tol = 1e-7 + (1e-13 + ftol) * abs(r["F"]) / abs(r["F"] - r["F_trial"])
            assert abs(g["gain"] - r["gain"]) <= tol * abs(r["gain"]), (n, "gain", g, r)
    assert len(g_log) == len(r_log), (len(g_log), len(r_log))
    return n


def reprojection_rms_diff(w, T_a, X_a, T_b, X_b, mask):
    pa = projections(w, T_a, X_a)
    pb = projections(w, T_b, X_b)
    st = w["obs_type"].astype(bool)
    d2 = ((pa[:, :2] - pb[:, :2]) ** 2).sum(axis=1) + np.where(st, (pa[:, 2] - pb[:, 2]) ** 2, 0.0)
    d2 = d2[mask]
    return float(np.sqrt(d2.mean())) if d2.size else 0.0


def window_slice(cat, i):
    """Arrays of window i of a concatenated batch."""
    k0, k1 = cat["kf_off"][i], cat["kf_off"][i + 1]
    p0, p1 = cat["pt_off"][i], cat["pt_off"][i + 1]
    o0, o1 = cat["obs_off"][i], cat["obs_off"][i + 1]
    return slice(k0, k1), slice(p0, p1), slice(o0, o1)


def pose_errors(T_a, T_b):
    """Largest camera-centre distance (m) and rotation angle (rad) between two pose sets."""
    A = np.asarray(T_a).reshape(-1, 3, 4)
    B = np.asarray(T_b).reshape(-1, 3, 4)
    ca = -np.einsum("kji,kj->ki", A[:, :, :3], A[:, :, 3])
    cb = -np.einsum("kji,kj->ki", B[:, :, :3], B[:, :, 3])
    dpos = np.linalg.norm(ca - cb, axis=1).max(initial=0.0)
    Rr = np.einsum("kij,klj->kil", A[:, :, :3], B[:, :, :3])
    # angle from both the skew and the symmetric part (arccos alone loses digits near 0)
    sk = np.stack([Rr[:, 2, 1] - Rr[:, 1, 2], Rr[:, 0, 2] - Rr[:, 2, 0], Rr[:, 1, 0] - Rr[:, 0, 1]], axis=1)
    ang = np.arctan2(0.5 * np.linalg.norm(sk, axis=1), 0.5 * (np.trace(Rr, axis1=1, axis2=2) - 1.0))
    return float(dpos), float(np.abs(ang).max(initial=0.0))


def mixed_metrics(w, g_T, g_X, g_stats, ref):
    """Errors of a mixed-precision (or batched) solve against the FP64 oracle."""
    Fr = ref["stats"]["F_final"]
    rel = abs(g_stats["F_final"] - Fr) / max(abs(Fr), 1e-30)
    rms = reprojection_rms_diff(w, g_T, g_X, ref["T"], ref["X"], ~ref["outlier"])
    dpos, dang = pose_errors(g_T, ref["T"])
    return dict(cost_rel=rel, rms_px=rms, pos_m=dpos, rot_rad=dang)


def assert_mixed_tolerances(w, g_T, g_X, g_stats, ref, cost_rel=1e-4, rms_px=0.01):
    m = mixed_metrics(w, g_T, g_X, g_stats, ref)
    assert m["cost_rel"] <= cost_rel, m
    assert m["rms_px"] <= rms_px, m
    return m


def round_z_f32(w):
    """The window with its measurements rounded to FP32 (what an FP32 upload holds)."""
    out = dict(w)
    out["obs_z"] = w["obs_z"].astype(np.float32).astype(np.float64)
    return out
