"""Plain FP64 GPU local bundle adjustment vs the FP64 CPU oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import lbaref
from paper_2511_02036_amd import synth
from tests.parity import assert_fp64_parity, window_slice

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2511_02036_amd import lba  # noqa: E402


def _gpu(w, **opts):
    return lba.solve(w, device="cuda:0", **opts)


# Small windows with a well-posed gauge: at least one fixed keyframe with stereo, at
# least two for monocular windows (one fixed keyframe leaves the monocular scale free).
TINY = [  # seed, K, fixed, M, nobs, stereo_p
    (0, 3, 2, 5, (2, 3), 0.0),
    (1, 4, 1, 20, (2, 4), 0.5),
    (2, 5, 2, 63, (2, 5), 1.0),
    (3, 6, 2, 65, (3, 6), 0.3),
    (4, 8, 3, 200, (2, 8), 0.7),
    (5, 7, 2, 150, (3, 7), 0.5),
    (6, 12, 4, 700, (4, 10), 0.7),
]


@pytest.mark.parametrize("seed,K,nf,M,nobs,sp", TINY)
def test_small_windows_match_oracle(seed, K, nf, M, nobs, sp):
    w = synth.tiny_window(seed, K=K, n_fixed=nf, M=M, nobs=nobs, stereo_p=sp)
    print(f"case seed={seed} K={K} M={M} N={len(w['obs_kf'])}", flush=True)
    g = _gpu(w)
    r = lbaref.solve(w)
    assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)


@pytest.mark.parametrize("maker", [synth.c1_mono, synth.c2_stereo], ids=["c1_mono", "c2_stereo"])
def test_full_configs_match_oracle(maker):
    w = maker()
    print(f"case {maker.__name__} N={len(w['obs_kf'])}", flush=True)
    g = _gpu(w)
    r = lbaref.solve(w)
    assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)


def test_batch_of_uneven_windows_matches_per_window_oracle():
    ws = [synth.tiny_window(10 + i, K=3 + 2 * i, n_fixed=2 + i // 2, M=30 + 90 * i, nobs=(3, 3 + i),
                            stereo_p=0.25 * (i % 4)) for i in range(6)]
    cat = synth.concat(ws)
    g = lba.solve(cat, device="cuda:0")
    for i, w in enumerate(ws):
        ks, ps, os_ = window_slice(cat, i)
        r = lbaref.solve(w)
        assert_fp64_parity(w, g["T"][ks], g["X"][ps], g["outlier"][os_], g["stats"][i], r)


def test_window_without_fixed_keyframes_matches_in_gauge_invariant_terms():
    """No fixed keyframe: the 6-dof gauge is held by the damping alone, so the states
    themselves are not determined to rounding level; the cost and the reprojections are."""
    from tests.parity import reprojection_rms_diff
    w = synth.tiny_window(5, K=7, n_fixed=0, M=150, nobs=(3, 7), stereo_p=0.5)
    g = _gpu(w)
    r = lbaref.solve(w)
    Fr, Fg = r["stats"]["F_final"], g["stats"][0]["F_final"]
    assert abs(Fg - Fr) <= 1e-9 * Fr
    inl = ~r["outlier"]
    assert reprojection_rms_diff(w, g["T"], g["X"], r["T"], r["X"], inl) < 1e-6


def test_tile_size_does_not_change_the_solution():
    w = synth.tiny_window(21, K=8, n_fixed=2, M=900, nobs=(2, 8), stereo_p=0.6)
    a = _gpu(w, points_per_tile=64)
    b = _gpu(w, points_per_tile=4096)
    r = lbaref.solve(w)
    assert_fp64_parity(w, a["T"], a["X"], a["outlier"], a["stats"][0], r)
    assert_fp64_parity(w, b["T"], b["X"], b["outlier"], b["stats"][0], r)


def test_points_only_window():
    w = synth.tiny_window(22, K=5, n_fixed=5, M=120, nobs=(2, 5), stereo_p=0.5)
    g = _gpu(w)
    r = lbaref.solve(w)
    assert g["stats"][0]["Kopt"] == 0
    assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)
    np.testing.assert_array_equal(g["T"], w["T_cw"])


def test_window_without_observations():
    w = synth.tiny_window(23, K=3, n_fixed=1, M=4)
    for key in ("obs_kf", "obs_pt", "obs_type", "obs_oct"):
        w[key] = w[key][:0]
    w["obs_z"] = w["obs_z"][:, :0]
    g = _gpu(w)
    np.testing.assert_array_equal(g["T"], w["T_cw"])
    np.testing.assert_array_equal(g["X"], w["X"])
    assert g["stats"][0]["F_final"] == 0.0


def test_points_without_observations_keep_their_position():
    w = synth.tiny_window(24, K=5, n_fixed=2, M=40, nobs=(3, 4))
    # append 3 unobserved points and renumber nothing (they get no observations)
    w["X"] = np.concatenate([w["X"], np.array([[1.0, 2.0, 9.0], [0.0, 0.0, 5.0], [3.0, -1.0, 7.0]])])
    g = _gpu(w)
    r = lbaref.solve(w)
    assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)
    np.testing.assert_array_equal(g["X"][-3:], w["X"][-3:])


def test_zero_iterations_return_the_input_state():
    w = synth.tiny_window(25, K=5, n_fixed=1, M=50)
    g = _gpu(w, iters_round1=0, iters_round2=0)
    r = lbaref.solve(w, iters_round1=0, iters_round2=0)
    np.testing.assert_array_equal(g["T"], w["T_cw"])
    np.testing.assert_array_equal(g["X"], w["X"])
    np.testing.assert_array_equal(g["outlier"], r["outlier"])
    assert g["stats"][0]["F_initial"] == pytest.approx(r["stats"]["F_initial"], rel=1e-12)


def test_plain_least_squares_round_two():
    w = synth.tiny_window(26, K=6, n_fixed=2, M=150, nobs=(2, 6), stereo_p=0.5)
    g = _gpu(w, round2_robust=0)
    r = lbaref.solve(w, round2_robust=0)
    assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)


def test_float_measurements_are_accepted():
    w = synth.tiny_window(27, K=6, n_fixed=2, M=150, nobs=(2, 6), stereo_p=0.5)
    w32 = dict(w)
    w32["obs_z"] = w["obs_z"].astype(np.float32).astype(np.float64)
    g = lba.solve(w, device="cuda:0", z_f32=True)
    r = lbaref.solve(w32)
    assert_fp64_parity(w32, g["T"], g["X"], g["outlier"], g["stats"][0], r)


@pytest.mark.parametrize("breakage", ["unsorted", "kf_range", "pt_range", "octave", "type", "nan"])
def test_invalid_inputs_are_rejected_before_any_solve(breakage):
    w = synth.tiny_window(28, K=4, n_fixed=1, M=20)
    w = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in w.items()}
    if breakage == "unsorted":
        w["obs_pt"][[0, -1]] = w["obs_pt"][[-1, 0]]
    elif breakage == "kf_range":
        w["obs_kf"][3] = 4
    elif breakage == "pt_range":
        w["obs_pt"][-1] = 20
    elif breakage == "octave":
        w["obs_oct"][2] = 8
    elif breakage == "type":
        w["obs_type"][1] = 2
    elif breakage == "nan":
        w["obs_z"][0, 5] = np.nan
    with pytest.raises(lba.LBAError, match="invalid"):
        _gpu(w)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_tiles_split_across_update_blocks(precision):
    """One tile of 3,000 points: the update kernel then runs the tile as several blocks
    (parts of about 512 points) whose partial sums the decision adds."""
    w = synth.tiny_window(29, K=12, n_fixed=3, M=3000, nobs=(3, 8), stereo_p=0.6)
    g = _gpu(w, points_per_tile=4096, precision=precision)
    r = lbaref.solve(w)
    if precision == "fp64":
        assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)
    else:
        from tests.parity import assert_mixed_tolerances
        assert_mixed_tolerances(w, g["T"], g["X"], g["stats"][0], r)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_points_seen_once(precision):
    """Points 200..499 seen by one stereo observation each (the first 200, seen 3-6 times, hold
    the cameras): the update kernel's chunks then hold 64 points of one observation each, and
    every lane's point results overwrite observation terms that other lanes read just before
    (the two share one LDS staging area).  A window of only such points leaves the cameras to
    the damping alone, too ill-posed for the FP64 bar."""
    w = synth.tiny_window(40, K=6, n_fixed=2, M=500, nobs=(3, 6), stereo_p=1.0)
    pt = w["obs_pt"]
    first = np.r_[True, pt[1:] != pt[:-1]]
    # (a point seen once in mono is held along its ray by the damping only)
    keep = (pt < 200) | (first & (w["obs_type"] == 1))
    w = {k: (v[..., keep] if k.startswith("obs_") else v) for k, v in w.items()}
    once = np.bincount(w["obs_pt"], minlength=500)[200:]
    assert (once <= 1).all() and once.sum() > 256
    print(f"case points seen once precision={precision} N={len(w['obs_pt'])}", flush=True)
    g = _gpu(w, precision=precision)
    r = lbaref.solve(w)
    if precision == "fp64":
        assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)
    else:
        from tests.parity import assert_mixed_tolerances
        assert_mixed_tolerances(w, g["T"], g["X"], g["stats"][0], r)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_point_with_the_most_observations(precision):
    """A point with 64 observations, the most one wavefront takes (its first observation
    repeated): the update kernel's chunk then holds that one point in all 64 lanes, and the
    linearisation sums its block over 64 observations."""
    w = synth.tiny_window(32, K=5, n_fixed=2, M=40, nobs=(2, 4), stereo_p=0.5)
    first = np.flatnonzero(w["obs_pt"] == 0)
    rep = np.full(64 - len(first), first[0])
    idx = np.sort(np.concatenate([np.arange(len(w["obs_pt"])), rep]), kind="stable")
    w = {k: (v[..., idx] if k.startswith("obs_") else v) for k, v in w.items()}
    assert (w["obs_pt"] == 0).sum() == 64
    print(f"case point with 64 observations precision={precision} N={len(w['obs_pt'])}", flush=True)
    g = _gpu(w, precision=precision)
    r = lbaref.solve(w)
    if precision == "fp64":
        assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)
    else:
        from tests.parity import assert_mixed_tolerances
        assert_mixed_tolerances(w, g["T"], g["X"], g["stats"][0], r)


def test_size_limits_are_rejected_before_any_solve():
    """61 optimisable keyframes exceed the reduced system's limit of 60 (both
    precisions); a point with 65 observations exceeds one wavefront.  Both are refused
    with a message; the largest accepted case (60) is solved in
    tests/test_gpu_large_windows.py."""
    w = synth.tiny_window(30, K=63, n_fixed=2, M=120, nobs=(3, 6), stereo_p=0.5)
    for precision in ("fp64", "mixed"):
        with pytest.raises(lba.LBAError, match="61 optimisable keyframes"):
            _gpu(w, precision=precision)
    w = synth.tiny_window(31, K=5, n_fixed=2, M=20, nobs=(2, 4), stereo_p=0.5)
    first = np.flatnonzero(w["obs_pt"] == 0)[0]
    rep = np.full(63, first)
    idx = np.sort(np.concatenate([np.arange(len(w["obs_pt"])), rep]), kind="stable")
    w = {k: (v[..., idx] if k.startswith("obs_") else v) for k, v in w.items()}
    assert (w["obs_pt"] == 0).sum() > 64
    with pytest.raises(lba.LBAError, match="invalid"):
        _gpu(w)
