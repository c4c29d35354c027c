"""Pins of the stereo-inertial part of the CPU oracle against things other than itself:
SciPy's rotation vector and matrix exponential for the SO(3) logarithm and right
Jacobians, the input generator's own construction of the preintegrated measurements (zero
residual at the true states), central finite differences of the residual for every
Jacobian block, the dense normal equations of the whole window for the Schur-reduced
15-unknowns-per-keyframe step, convergence of noise-free windows to the truth, and the
visual-only solve when the inertial information is zero."""
import numpy as np
import pytest
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

from paper_2511_02036_amd import synth


@pytest.fixture(scope="module")
def ref():
    from oracle import lbaref
    lbaref.lib()
    return lbaref


def _hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def test_so3_log_matches_scipy_rotation_vectors(ref):
    rng = np.random.default_rng(0)
    for ang in (0.0, 1e-9, 1e-5, 3e-4, 0.1, 1.0, 2.5, np.pi - 1e-3, np.pi - 1e-6):
        for _ in range(5):
            ax = rng.normal(size=3)
            ax /= np.linalg.norm(ax)
            w = ang * ax
            R = expm(_hat(w))
            got = ref.so3_log(R)
            want = Rotation.from_matrix(R).as_rotvec()
            assert np.abs(got - want).max() <= 1e-8, (ang, got, want)
            np.testing.assert_allclose(expm(_hat(got)), R, atol=1e-12)


def test_right_jacobian_and_its_inverse(ref):
    """Exp(w + d) = Exp(w) Exp(Jr(w) d) to first order (central differences of SciPy's expm),
    and Jr^-1 Jr = I, at small and large angles."""
    rng = np.random.default_rng(1)
    for ang in (0.0, 1e-4, 5e-3, 0.3, 1.7, 3.0):
        ax = rng.normal(size=3)
        w = ang * ax / np.linalg.norm(ax)
        Jr = ref.so3_jr(w)
        R = expm(_hat(w))
        h = 1e-6
        for c in range(3):
            d = np.zeros(3)
            d[c] = h
            Rp, Rm = expm(_hat(w + d)), expm(_hat(w - d))
            # Log(R^T R(w + d)) / h -> Jr e_c
            fd = (Rotation.from_matrix(R.T @ Rp).as_rotvec() - Rotation.from_matrix(R.T @ Rm).as_rotvec()) / (2 * h)
            np.testing.assert_allclose(Jr[:, c], fd, atol=1e-8)
        np.testing.assert_allclose(ref.so3_jr_inv(w) @ Jr, np.eye(3), atol=1e-12)


def test_residual_is_zero_at_the_true_states(ref):
    """The generator builds each measurement from the true body motion (its own
    construction); the oracle's residual of every measurement vanishes there."""
    for seed in (3, 4):
        w, vi = synth.vi_window(seed, K=8, n_fixed=3, M=150, noise=False)
        for e in range(len(vi["dt"])):
            r = ref.vi_residual(w, vi, e, T=w["T_true"], V=vi["v_true"], BG=vi["bg_true"], BA=vi["ba_true"])
            assert np.abs(r).max() < 1e-12, (seed, e, r)
        assert ref.vi_cost(w, vi, T=w["T_true"], V=vi["v_true"], BG=vi["bg_true"], BA=vi["ba_true"]) < 1e-20


def _perturbed(T, V, BG, BA, k, c, h):
    T2, V2, G2, A2 = T.copy(), V.copy(), BG.copy(), BA.copy()
    if c < 6:
        xi = np.zeros(6)
        xi[c] = h
        A = np.zeros((4, 4))
        A[:3, :3] = _hat(xi[:3])
        A[:3, 3] = xi[3:]
        T2[k] = (expm(A) @ np.vstack([T[k].reshape(3, 4), [0, 0, 0, 1]]))[:3].reshape(12)
    elif c < 9:
        V2[k, c - 6] += h
    elif c < 12:
        G2[k, c - 9] += h
    else:
        A2[k, c - 12] += h
    return T2, V2, G2, A2


def test_jacobian_blocks_match_central_differences(ref):
    """Every column of the 15 x 30 Jacobian (twist along Exp(h e_c) T, velocity, biases of
    both keyframes) against central differences (h = 1e-6) to 1e-7 relative."""
    w, vi = synth.vi_window(5, K=6, n_fixed=2, M=120, noise=True)
    T = w["T_cw"].reshape(-1, 12).copy()
    V, BG, BA = vi["v"].copy(), vi["bg"].copy(), vi["ba"].copy()
    worst = 0.0
    for e in range(len(vi["dt"])):
        J = ref.vi_jacobian(w, vi, e, T=T, V=V, BG=BG, BA=BA)
        for side, k in enumerate((vi["edge_i"][e], vi["edge_j"][e])):
            for c in range(15):
                h = 1e-6
                rp = ref.vi_residual(w, vi, e, *_perturbed(T, V, BG, BA, k, c, h))
                rm = ref.vi_residual(w, vi, e, *_perturbed(T, V, BG, BA, k, c, -h))
                fd = (rp - rm) / (2 * h)
                an = J[:, 15 * side + c]
                err = np.abs(fd - an).max() / max(1e-6, np.abs(an).max())
                worst = max(worst, err)
                assert err < 1e-7, (e, side, c, fd, an)
    assert worst < 1e-7


def _dense_vi(ref, w, vi, lam):
    """The whole window's damped normal equations, dense, from the visual dense system and
    the inertial Jacobians: unknowns (twist, v, bg, ba) per optimisable keyframe, then the
    points; solved by numpy."""
    Hv, bv = ref.dense_system(w)
    fixed = w["fixed"].astype(bool)
    Kopt, M = int((~fixed).sum()), len(w["X"])
    opt = -np.ones(len(fixed), int)
    opt[~fixed] = np.arange(Kopt)
    n, D = 15 * Kopt, 15 * Kopt + 3 * M
    idx = np.concatenate([15 * k + np.arange(6) for k in range(Kopt)] + [n + np.arange(3 * M)])
    H = np.zeros((D, D))
    b = np.zeros(D)
    H[np.ix_(idx, idx)] = Hv
    b[idx] = bv
    for e in range(len(vi["dt"])):
        r = ref.vi_residual(w, vi, e)
        J = ref.vi_jacobian(w, vi, e)
        Om = np.zeros((15, 15))
        Om[:9, :9] = vi["info"][e].reshape(9, 9)
        Om[9:12, 9:12] = vi["info_bg"][e] * np.eye(3)
        Om[12:, 12:] = vi["info_ba"][e] * np.eye(3)
        cols, jc = [], []
        for side, k in enumerate((vi["edge_i"][e], vi["edge_j"][e])):
            if opt[k] >= 0:
                cols.append(15 * opt[k] + np.arange(15))
                jc.append(15 * side + np.arange(15))
        if not cols:
            continue
        cols, jc = np.concatenate(cols), np.concatenate(jc)
        Je = J[:, jc]
        H[np.ix_(cols, cols)] += Je.T @ Om @ Je
        b[cols] -= Je.T @ Om @ r
    return np.linalg.solve(H + lam * np.eye(D), b), n, H, b


@pytest.mark.parametrize("seed,lam", [(6, 1e-3), (7, 10.0)])
def test_schur_step_equals_dense_step(ref, seed, lam):
    w, vi = synth.vi_window(seed, K=5, n_fixed=2, M=25, nobs=(2, 4), noise=True)
    st = ref.vi_system_step(w, vi, lam)
    assert st["ok"]
    x, n, _, _ = _dense_vi(ref, w, vi, lam)
    np.testing.assert_allclose(st["d"], x[:n], rtol=1e-9, atol=1e-9 * np.abs(x).max())
    np.testing.assert_allclose(st["dl"].reshape(-1), x[n:], rtol=1e-9, atol=1e-9 * np.abs(x).max())


def test_noise_free_window_converges_to_the_truth(ref):
    w, vi = synth.vi_window(8, K=10, n_fixed=3, M=600, noise=False)
    r = ref.solve_vi(w, vi, iters_round1=10, iters_round2=40)
    assert r["stats"]["F_final"] <= 1e-12, r["stats"]
    assert np.abs(r["T"] - w["T_true"]).max() <= 1e-9
    assert np.abs(r["X"] - w["X_true"]).max() <= 1e-9
    assert np.abs(r["V"] - vi["v_true"]).max() <= 1e-9
    assert np.abs(r["BG"] - vi["bg_true"]).max() <= 1e-9
    assert np.abs(r["BA"] - vi["ba_true"]).max() <= 1e-9


def test_cost_is_non_increasing_and_fixed_states_hold(ref):
    w, vi = synth.vi_window(9, K=8, n_fixed=3, M=400, noise=True)
    r = ref.solve_vi(w, vi)
    acc = [l for l in r["log"] if l["accepted"]]
    assert len(acc) >= 10
    for l in acc:
        assert l["F_trial"] <= l["F"]
    fixed = w["fixed"].astype(bool)
    np.testing.assert_array_equal(r["T"][fixed], w["T_cw"].reshape(-1, 12)[fixed])
    np.testing.assert_array_equal(r["V"][fixed], vi["v"][fixed])
    np.testing.assert_array_equal(r["BG"][fixed], vi["bg"][fixed])
    np.testing.assert_array_equal(r["BA"][fixed], vi["ba"][fixed])
    # the inertial terms pull the velocities towards the truth
    opt = ~fixed
    assert np.abs(r["V"][opt] - vi["v_true"][opt]).mean() < 0.5 * np.abs(vi["v"][opt] - vi["v_true"][opt]).mean()


def test_zero_inertial_information_reduces_to_the_visual_solve(ref):
    """With every inertial information zero the joint cost is the reprojection cost: the
    poses and points follow the visual-only solve, and velocities and biases do not move."""
    w, vi = synth.vi_window(10, K=7, n_fixed=2, M=300, noise=True)
    vi0 = dict(vi)
    vi0["info"] = np.zeros_like(vi["info"])
    vi0["info_bg"] = np.zeros_like(vi["info_bg"])
    vi0["info_ba"] = np.zeros_like(vi["info_ba"])
    r = ref.solve_vi(w, vi0)
    v = ref.solve(w)
    assert abs(r["stats"]["F_final"] - v["stats"]["F_final"]) <= 1e-9 * v["stats"]["F_final"]
    np.testing.assert_allclose(r["T"], v["T"], atol=1e-9)
    np.testing.assert_allclose(r["X"], v["X"], atol=1e-8)
    np.testing.assert_array_equal(r["V"], vi["v"])
    np.testing.assert_array_equal(r["BG"], vi["bg"])
    np.testing.assert_array_equal(r["BA"], vi["ba"])
    assert [l["accepted"] for l in r["log"]] == [l["accepted"] for l in v["log"]]


def test_gain_ratio_tends_to_one_near_the_optimum(ref):
    """Close to the solution the joint cost is nearly quadratic, so the actual decrease of an
    accepted step matches the predicted decrease d^T (lambda d + b) (the gain ratio tends to
    1).  With measurement noise the reprojection and inertial gradients do not vanish one by
    one at the optimum, so a predicted decrease that misses either part is off at first
    order in the step."""
    w, vi = synth.vi_window(11, K=8, n_fixed=3, M=500, noise=True)
    r = ref.solve_vi(w, vi, iters_round1=8, iters_round2=10)
    late = [l for l in r["log"] if l["accepted"] and l["round"] == 2][-3:]
    assert len(late) == 3
    for l in late:
        assert abs(l["gain"] - 1.0) < 0.02, l


def test_initial_damping_includes_the_inertial_blocks(ref):
    """lambda0 = tau * the largest diagonal entry of the joint Gauss-Newton matrix: on a
    window where the inertial blocks dominate the diagonal, the first trial's lambda equals
    tau times the largest diagonal entry of the dense joint system (numpy)."""
    w, vi = synth.vi_window(12, K=5, n_fixed=2, M=25, nobs=(2, 4), noise=True)
    vi = dict(vi)
    vi["info"] = vi["info"] * 1e4
    r = ref.solve_vi(w, vi, iters_round1=1, iters_round2=0)
    Hv, _ = ref.dense_system(w)
    fixed = w["fixed"].astype(bool)
    Kopt = int((~fixed).sum())
    opt = -np.ones(len(fixed), int)
    opt[~fixed] = np.arange(Kopt)
    diag = np.zeros(15 * Kopt + 3 * len(w["X"]))
    idx = np.concatenate([15 * k + np.arange(6) for k in range(Kopt)] + [15 * Kopt + np.arange(3 * len(w["X"]))])
    diag[idx] = np.diag(Hv)
    for e in range(len(vi["dt"])):
        J = ref.vi_jacobian(w, vi, e)
        Om = np.zeros((15, 15))
        Om[:9, :9] = vi["info"][e].reshape(9, 9)
        Om[9:12, 9:12] = vi["info_bg"][e] * np.eye(3)
        Om[12:, 12:] = vi["info_ba"][e] * np.eye(3)
        H = J.T @ Om @ J
        for side, k in enumerate((vi["edge_i"][e], vi["edge_j"][e])):
            if opt[k] >= 0:
                diag[15 * opt[k] + np.arange(15)] += np.diag(H)[15 * side + np.arange(15)]
    lam0 = r["log"][0]["lam"]
    assert abs(lam0 - 1e-5 * diag.max()) <= 1e-9 * lam0
    assert diag[:15 * Kopt].max() > 10 * np.diag(Hv).max()   # the inertial part decides


def test_predicted_decrease_matches_the_dense_model(ref):
    """The gain ratio's denominator of the first trial, (F - F') / gain from the log, equals
    the decrease the damped Gauss-Newton model of the whole window predicts,
    d^T (lambda d + b) with (H + lambda I) d = b from the dense joint system (numpy)."""
    w, vi = synth.vi_window(13, K=5, n_fixed=2, M=30, nobs=(2, 4), noise=True)
    r = ref.solve_vi(w, vi, iters_round1=1, iters_round2=0)
    l0 = r["log"][0]
    den_log = (l0["F"] - l0["F_trial"]) / l0["gain"]
    d, n, H, b = _dense_vi(ref, w, vi, l0["lam"])
    den = d @ (l0["lam"] * d + b)
    assert abs(den_log - den) <= 1e-8 * abs(den), (den_log, den)
