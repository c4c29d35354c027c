"""Mixed-precision form (FP32 Jacobians / Hessian blocks / Schur, FP64 Cholesky, cost,
gain ratio, damping and states) and the batched form (many uneven windows per launch),
against the FP64 CPU oracle."""
import json
import os

import numpy as np
import pytest

from oracle import lbaref
from paper_2511_02036_amd import synth
from tests.parity import (assert_fp64_parity, assert_mixed_tolerances, mixed_metrics, round_z_f32,
                          window_slice)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2511_02036_amd import lba  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")


def _record(name, value):
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "precision_metrics.jsonl"), "a") as f:
        f.write(json.dumps({"case": name, **value}) + "\n")


@pytest.mark.parametrize("seed", [40, 41, 42])
def test_mixed_small_windows(seed):
    w = synth.tiny_window(seed, K=8, n_fixed=3, M=400, nobs=(3, 8), stereo_p=0.7)
    g = lba.solve(w, device="cuda:0", precision="mixed")
    r = lbaref.solve(w)
    assert_mixed_tolerances(w, g["T"], g["X"], g["stats"][0], r)


@pytest.mark.parametrize("z_f32", [False, True])
def test_mixed_c2(z_f32):
    w = synth.c2_stereo()
    wr = round_z_f32(w) if z_f32 else w
    g = lba.solve(w, device="cuda:0", precision="mixed", z_f32=z_f32)
    r = lbaref.solve(wr)
    m = assert_mixed_tolerances(wr, g["T"], g["X"], g["stats"][0], r)
    _record(f"c2_mixed_zf32={z_f32}", m)


@pytest.mark.parametrize("acc32", [0, 1], ids=["fp64_sums", "fp32_sums"])
def test_mixed_c3_precision_form(acc32):
    """C3 in the mixed form, with the Schur complement summed in FP64 (default) or, the
    literal precision form, in FP32."""
    w = synth.c3_precision()
    print(f"case c3 N={len(w['obs_kf'])} acc32={acc32}", flush=True)
    wr = round_z_f32(w)
    g = lba.solve(w, device="cuda:0", precision="mixed", z_f32=True, schur_fp32_accum=acc32)
    r = lbaref.solve(wr)
    m = assert_mixed_tolerances(wr, g["T"], g["X"], g["stats"][0], r)
    m["flags_differ"] = int((g["outlier"] != r["outlier"]).sum())
    _record(f"c3_mixed_acc32={acc32}", m)


def test_fp64_c3_matches_oracle():
    """The largest reduced system (180 unknowns) also runs in FP64 at oracle parity."""
    w = synth.c3_precision()
    g = lba.solve(w, device="cuda:0")
    r = lbaref.solve(w)
    assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)


def test_fp64_batch_of_c5_shaped_windows_matches_oracle():
    ws = synth.c5_windows(only=list(range(12)), max_points=1500)
    cat = synth.concat(ws)
    g = lba.solve(cat, device="cuda:0")
    for i, w in enumerate(ws):
        ks, ps, os_ = window_slice(cat, i)
        r = lbaref.solve(w)
        assert_fp64_parity(w, g["T"][ks], g["X"][ps], g["outlier"][os_], g["stats"][i], r)


def test_batch_equals_one_window_at_a_time():
    ws = synth.c5_windows(only=[3, 7, 11, 19], max_points=3000)
    cat = synth.concat(ws)
    g = lba.solve(cat, device="cuda:0")
    for i, w in enumerate(ws):
        ks, ps, os_ = window_slice(cat, i)
        s = lba.solve(w, device="cuda:0")
        np.testing.assert_allclose(g["T"][ks], s["T"], rtol=0, atol=1e-10)
        np.testing.assert_allclose(g["X"][ps], s["X"], rtol=0, atol=1e-9)
        assert g["stats"][i]["F_final"] == pytest.approx(s["stats"][0]["F_final"], rel=1e-11)


@pytest.fixture(scope="module")
def c5():
    ws = synth.c5_windows()
    return ws, synth.concat(ws)


def _oracle_all(ws, threads=16):
    """The FP64 oracle on every window, one window per thread (ctypes releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lbaref.solve, ws))


@pytest.fixture(scope="module")
def c5_refs(c5):
    ws, _ = c5
    wrs = [round_z_f32(w) for w in ws]
    return wrs, _oracle_all(wrs)


@pytest.mark.parametrize("acc32", [0, 1], ids=["fp64_sums", "fp32_sums"])
def test_c5_full_batch_mixed_every_window(c5, c5_refs, acc32):
    """All 256 windows of the batch, solved together in the mixed form on FP32
    measurements (Schur complement summed in FP64, or in FP32: the literal precision
    form), against the oracle on the same FP32-rounded measurements: final cost within
    1e-4 relative and RMS reprojection difference within 0.01 px in every window.
    Outlier flags may differ where an observation's s lies within the FP32 path's error of
    its threshold; their count is recorded with the other per-result errors."""
    ws, cat = c5
    print(f"case c5 mixed windows={len(ws)} N={len(cat['obs_kf'])} acc32={acc32}", flush=True)
    g = lba.solve(cat, device="cuda:0", precision="mixed", z_f32=True, schur_fp32_accum=acc32)
    st = g["stats"]
    assert all(s["iters_r1"] >= 1 and s["iters_r2"] >= 1 for s in st)
    wrs, refs = c5_refs
    rows = []
    for i, (wr, r) in enumerate(zip(wrs, refs)):
        ks, ps, os_ = window_slice(cat, i)
        m = mixed_metrics(wr, g["T"][ks], g["X"][ps], st[i], r)
        m["flags_differ"] = int((g["outlier"][os_] != r["outlier"]).sum())
        m["window"] = i
        m["N"] = len(wr["obs_kf"])
        rows.append(m)
    worst = max(rows, key=lambda m: m["cost_rel"])
    worst_px = max(rows, key=lambda m: m["rms_px"])
    _record(f"c5_mixed_all_windows_acc32={acc32}", dict(
        windows=len(rows), cost_rel_max=worst["cost_rel"], cost_rel_worst_window=worst,
        rms_px_max=worst_px["rms_px"], pos_m_max=max(m["pos_m"] for m in rows),
        rot_rad_max=max(m["rot_rad"] for m in rows), flags_differ_total=sum(m["flags_differ"] for m in rows),
        cost_rel_median=float(np.median([m["cost_rel"] for m in rows]))))
    for m in rows:
        assert m["cost_rel"] <= 1e-4, m
        assert m["rms_px"] <= 0.01, m


def test_c5_full_batch_fp64_every_window(c5):
    """The same 256 windows solved together in plain FP64 match the oracle window by
    window at the FP64 bar (1e-9 cost, 1e-8 states, flags outside the band)."""
    ws, cat = c5
    print(f"case c5 fp64 windows={len(ws)} N={len(cat['obs_kf'])}", flush=True)
    g = lba.solve(cat, device="cuda:0")
    refs = _oracle_all(ws)
    worst = 0.0
    for i, (w, r) in enumerate(zip(ws, refs)):
        ks, ps, os_ = window_slice(cat, i)
        assert_fp64_parity(w, g["T"][ks], g["X"][ps], g["outlier"][os_], g["stats"][i], r)
        Fr = r["stats"]["F_final"]
        worst = max(worst, abs(g["stats"][i]["F_final"] - Fr) / Fr)
    _record("c5_fp64_all_windows", dict(windows=len(ws), cost_rel_max=worst))
