"""The correspondence search's no-allocation entry point (library-held scratch) against
the workspace entry point, through the C ABI: two calls in a row, the second smaller, and
a problem too large for the scratch refused."""
import numpy as np
import pytest

from paper_2511_02036_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2511_02036_amd import lmap
    lmap.library()
    return lmap


def _both(lm, ds, free, cur, nbr, **params):
    import torch
    job = lm.Correspondence(ds, cur, nbr)
    fr = ds.upload_free(free)
    p = lm.corr_params(**params)
    job.run(fr, p)
    torch.cuda.synchronize()
    want = job.result()
    job.match.fill_(7)
    job.dist.fill_(7)
    job.run_noalloc(fr, p)
    torch.cuda.synchronize()
    return job.result(), want


def test_noalloc_matches_workspace_entry_point_twice(lm):
    st = synth.keyframe_store(seed=31, K=20, M=8000, kp_per_kf=700, walk_length=4.0)
    ds = lm.DeviceStore(st)
    cur, nbr = synth.correspondence_queries(st, n_cur=10, n_nbr=6)
    print(f"no-alloc call 1: {len(cur)} queries", flush=True)
    got, want = _both(lm, ds, st["kp_free"], cur, nbr)
    for g, w in zip(got, want):
        np.testing.assert_array_equal(g, w)
    assert (got[0] >= 0).sum() > 0
    # second call, smaller, on the same scratch (what the first call left must not leak)
    print(f"no-alloc call 2: 5 queries", flush=True)
    got2, want2 = _both(lm, ds, st["kp_free"], cur[:5], nbr[:5], th_low=70)
    for g, w in zip(got2, want2):
        np.testing.assert_array_equal(g, w)


def test_noalloc_refuses_a_problem_beyond_the_scratch(lm):
    import ctypes as C
    st = synth.keyframe_store(seed=32, K=12, M=3000, kp_per_kf=300, walk_length=3.0)
    ds = lm.DeviceStore(st)
    n_q = (lm.NOALLOC_SCRATCH_BYTES // (4 * ds.max_kp)) + 64
    need = C.c_size_t()
    assert lm.library().lmap_corr_workspace_size(C.byref(ds.S), n_q, C.byref(need)) == 0
    assert need.value > lm.NOALLOC_SCRATCH_BYTES
    cur = np.zeros(n_q, np.int32)
    nbr = np.ones(n_q, np.int32)
    job = lm.Correspondence(ds, cur, nbr)
    with pytest.raises(lm.LMapError, match="workspace too small"):
        job.run_noalloc(ds.upload_free(st["kp_free"]))
