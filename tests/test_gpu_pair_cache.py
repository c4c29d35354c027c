"""Chunk records of the linearisation kept for the rest of an LM round (pair_cache = 1, the
default) against the pair structure formed at every step (pair_cache = 0).

The first launch of a round forms each chunk's pairs, pieces and piece offsets and stores
them; the later launches load them.  The stored lists are the ones the kernel would form
again, so on windows whose camera sums are kept per wavefront the two solves agree bit
for bit (states, flags, statistics and the per-trial log).  Windows of more than 30
optimisable keyframes (several passes over the camera blocks, one shared copy of the
camera sums) agree to rounding; both are held to the FP64 oracle there."""
import numpy as np
import pytest

from oracle import lbaref
from paper_2511_02036_amd import synth
from tests.parity import assert_fp64_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2511_02036_amd import lba  # noqa: E402


def _same(a, b):
    assert np.array_equal(a["T"], b["T"])
    assert np.array_equal(a["X"], b["X"])
    assert np.array_equal(a["outlier"], b["outlier"])
    for sa, sb in zip(a["stats"], b["stats"]):
        _same_record(sa, sb)


def _same_record(ra, rb):
    assert ra.keys() == rb.keys()
    for k in ra:
        va, vb = ra[k], rb[k]
        assert va == vb or (isinstance(va, float) and np.isnan(va) and np.isnan(vb)), k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_records_give_the_same_batched_solve(precision):
    ws = synth.c5_windows(seed=4, only=list(range(0, 256, 16)), max_points=4000)
    cat = synth.concat(ws)
    print(f"case pair_cache batch precision={precision} windows={len(ws)} obs={len(cat['obs_kf'])}", flush=True)
    zf = precision == "mixed"
    a = lba.solve(cat, device="cuda:0", precision=precision, z_f32=zf, pair_cache=1, trial_log=64)
    b = lba.solve(cat, device="cuda:0", precision=precision, z_f32=zf, pair_cache=0, trial_log=64)
    _same(a, b)
    assert len(a["log"]) == len(b["log"])
    for la, lb in zip(a["log"], b["log"]):
        assert len(la) == len(lb) > 0
        for ra, rb in zip(la, lb):
            _same_record(ra, rb)


def test_records_on_a_single_window_repeat_bit_for_bit():
    w = synth.c2_stereo(seed=1)
    print(f"case pair_cache c2 obs={len(w['obs_kf'])}", flush=True)
    a = lba.solve(w, device="cuda:0", pair_cache=1)
    b = lba.solve(w, device="cuda:0", pair_cache=0)
    _same(a, b)


@pytest.mark.parametrize("kopt", [31, 45])
def test_records_with_several_passes_match_the_oracle(kopt):
    w = synth.tiny_window(70 + kopt, K=kopt + 5, n_fixed=5, M=1500, nobs=(3, 8), stereo_p=0.6)
    print(f"case pair_cache passes kopt={kopt} N={len(w['obs_kf'])}", flush=True)
    r = lbaref.solve(w)
    for cache in (1, 0):
        g = lba.solve(w, device="cuda:0", pair_cache=cache)
        assert_fp64_parity(w, g["T"], g["X"], g["outlier"], g["stats"][0], r)


def test_records_that_overflow_the_pool_fall_back_to_forming_them():
    """Points seen by about 24 of 25 optimisable keyframes (an arc facing inward) have about 11
    pairs per observation, more than the pool holds (8 words per observation and 256 per 256
    observations and per tile): the tiles whose records do not fit form them at every step,
    and the solve is the same as without records (25 optimisable keyframes: the camera sums
    keep one copy per wavefront, so both are bitwise-repeatable)."""
    w = synth.make_window(np.random.default_rng(91), trajectory="arc", K=26, n_fixed=1, M=500, nobs=(24, 26),
                          stereo_p=0.6)
    on = np.asarray(w["fixed"])[w["obs_kf"]] == 0
    m = np.bincount(w["obs_pt"][on], minlength=len(w["X"]))
    pairs, n = int((m * (m - 1) // 2).sum()), len(w["obs_kf"])
    print(f"case pair_cache overflow N={n} pairs={pairs}", flush=True)
    assert pairs > 8 * n + 256 * (n // 256 + 8)   # more pair words than the whole pool
    a = lba.solve(w, device="cuda:0", pair_cache=1)
    b = lba.solve(w, device="cuda:0", pair_cache=0)
    _same(a, b)
    r = lbaref.solve(w)
    assert_fp64_parity(w, a["T"], a["X"], a["outlier"], a["stats"][0], r)
