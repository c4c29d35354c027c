"""The Levenberg-Marquardt schedule on the GPU against the FP64 oracle: the per-trial log
(rounds, iterations, trials, decisions, damping, costs, gain ratios) compared trial by
trial, and the branches that only rejections reach (a reduced system that never
factorises, a budget of one trial per iteration)."""
import numpy as np
import pytest

from oracle import lbaref
from paper_2511_02036_amd import synth
from tests.parity import assert_fp64_parity, assert_trial_logs_match

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2511_02036_amd import lba  # noqa: E402

LOG = 256


def _gpu(w, **opts):
    return lba.solve(w, device="cuda:0", trial_log=LOG, **opts)


@pytest.mark.parametrize("seed,K,nf,M,nobs,sp", [
    (30, 4, 1, 40, (2, 4), 0.5),
    (31, 6, 2, 120, (3, 6), 0.0),
    (32, 8, 3, 300, (2, 8), 0.7),
])
def test_trial_log_matches_oracle_small(seed, K, nf, M, nobs, sp):
    w = synth.tiny_window(seed, K=K, n_fixed=nf, M=M, nobs=nobs, stereo_p=sp)
    print(f"case seed={seed} K={K} M={M} N={len(w['obs_kf'])}", flush=True)
    g = _gpu(w)
    r = lbaref.solve(w)
    n = assert_trial_logs_match(w, g["log"][0], r["log"])
    assert n >= 3


@pytest.mark.parametrize("maker", [synth.c1_mono, synth.c2_stereo], ids=["c1_mono", "c2_stereo"])
def test_trial_log_matches_oracle_full_configs(maker):
    w = maker()
    print(f"case {maker.__name__} N={len(w['obs_kf'])}", flush=True)
    g = _gpu(w)
    r = lbaref.solve(w)
    n = assert_trial_logs_match(w, g["log"][0], r["log"])
    assert n >= 10


def test_trial_log_of_a_batch_is_per_window():
    ws = [synth.tiny_window(40 + i, K=4 + i, n_fixed=2, M=60 + 40 * i, nobs=(2, 5), stereo_p=0.3 * i)
          for i in range(4)]
    cat = synth.concat(ws)
    g = lba.solve(cat, device="cuda:0", trial_log=LOG)
    for i, w in enumerate(ws):
        r = lbaref.solve(w)
        assert_trial_logs_match(w, g["log"][i], r["log"])


def _unobserved_keyframe_window():
    w = synth.tiny_window(10, K=4, n_fixed=1, M=15)
    keep = w["obs_kf"] != 3                      # keyframe 3 (optimisable) sees nothing
    for key in ("obs_kf", "obs_pt", "obs_type", "obs_oct"):
        w[key] = w[key][keep]
    w["obs_z"] = w["obs_z"][:, keep]
    return w


@pytest.mark.parametrize("max_trials", [1, 3, 10])
def test_every_trial_rejected_ends_each_round(max_trials):
    """tau = 0 with an optimisable keyframe that observes nothing: the reduced matrix keeps
    a zero block at lambda = 0, so every trial fails and each round ends after exactly
    max_trials trials with the state untouched."""
    w = _unobserved_keyframe_window()
    g = _gpu(w, tau=0.0, max_trials=max_trials)
    r = lbaref.solve(w, tau=0.0, max_trials=max_trials)
    st = g["stats"][0]
    assert st["trials"] == 2 * max_trials == r["stats"]["trials"]
    assert st["iters_r1"] == 0 and st["iters_r2"] == 0
    assert st["term_r1"] == 1 and st["term_r2"] == 1
    assert st["lambda"] == 0.0
    np.testing.assert_array_equal(g["T"], w["T_cw"])
    np.testing.assert_array_equal(g["X"], w["X"])
    assert [l["solve_ok"] for l in g["log"][0]] == [False] * (2 * max_trials)
    assert [(l["round"], l["trial"]) for l in g["log"][0]] == [(l["round"], l["trial"]) for l in r["log"]]
    np.testing.assert_array_equal(g["outlier"], r["outlier"])


@pytest.mark.parametrize("maker", [synth.c1_mono, synth.c2_stereo], ids=["c1_mono", "c2_stereo"])
def test_single_trial_budget_matches_oracle(maker):
    w = maker()
    g = _gpu(w, max_trials=1)
    r = lbaref.solve(w, max_trials=1)
    assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)
    assert_trial_logs_match(w, g["log"][0], r["log"])


def test_small_tau_rejections_match_oracle():
    """A damping start far below the curvature: early trials are rejected and lambda grows
    by nu = 2, 4, 8 ... before the first acceptance."""
    w = synth.tiny_window(33, K=6, n_fixed=2, M=150, nobs=(3, 6), stereo_p=0.5)
    g = _gpu(w, tau=1e-14)
    r = lbaref.solve(w, tau=1e-14)
    assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)
    assert_trial_logs_match(w, g["log"][0], r["log"], cond_tau=1e-14)
