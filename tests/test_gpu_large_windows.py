"""Windows beyond 30 optimisable keyframes against the FP64 CPU oracle, through the C ABI.

Above 30 optimisable keyframes the reduced system has more than 180 unknowns: it is
factorised in a copy in HBM instead of LDS, and the linearisation takes one pass per 476
camera blocks (31 keyframes: 496 blocks, two passes; 45: 1,035, three; 60: 1,830, four).
A batch that holds one such window factorises all its windows in HBM.  Such windows keep
one shared copy of the linearisation's camera sums (the per-wavefront copies do not fit
in LDS beside the rest), so their solves agree to rounding, not bit for bit."""
import pytest

from oracle import lbaref
from paper_2511_02036_amd import synth
from tests.parity import assert_fp64_parity, assert_mixed_tolerances, round_z_f32, window_slice

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2511_02036_amd import lba  # noqa: E402


def _window(kopt, seed, M=1500):
    return synth.tiny_window(seed, K=kopt + 5, n_fixed=5, M=M, nobs=(3, 8), stereo_p=0.6)


@pytest.mark.parametrize("kopt", [31, 45, 60])
def test_large_window_fp64_matches_oracle(kopt):
    w = _window(kopt, 40 + kopt)
    print(f"case large fp64 kopt={kopt} N={len(w['obs_kf'])}", flush=True)
    g = lba.solve(w, device="cuda:0")
    r = lbaref.solve(w)
    assert g["stats"][0]["Kopt"] == kopt
    assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)


@pytest.mark.parametrize("kopt", [31, 45])
def test_large_window_mixed_matches_oracle(kopt):
    w = _window(kopt, 60 + kopt)
    print(f"case large mixed kopt={kopt} N={len(w['obs_kf'])}", flush=True)
    g = lba.solve(w, device="cuda:0", precision="mixed", z_f32=True)
    r = lbaref.solve(round_z_f32(w))
    assert_mixed_tolerances(w, g["T"], g["X"], g["stats"][0], r)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_with_a_large_window_matches_per_window_oracle(precision):
    """Small and large windows in one batch, with tiles of 400 points: every window is
    factorised in HBM, the small ones end after their first linearisation pass, and the
    large one spreads its blocks over three passes per tile."""
    ws = [synth.tiny_window(70, K=8, n_fixed=2, M=300, nobs=(3, 6), stereo_p=0.6),
          _window(45, 71, M=1200),
          synth.tiny_window(72, K=26, n_fixed=4, M=900, nobs=(3, 8), stereo_p=0.6)]
    cat = synth.concat(ws)
    print(f"case large batch {precision} N={len(cat['obs_kf'])}", flush=True)
    mixed = precision == "mixed"
    g = lba.solve(cat, device="cuda:0", precision=precision, z_f32=mixed, points_per_tile=400)
    for i, w in enumerate(ws):
        ks, ps, os_ = window_slice(cat, i)
        if mixed:
            r = lbaref.solve(round_z_f32(w))
            assert_mixed_tolerances(w, g["T"][ks], g["X"][ps], g["stats"][i], r)
        else:
            r = lbaref.solve(w)
            assert_fp64_parity(w, g["T"][ks], g["X"][ps], g["outlier"][os_], g["stats"][i], r)

