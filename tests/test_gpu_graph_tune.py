"""Batched form: LM steps replayed from HIP graphs against kernels launched one by one,
and the tile tuner (its table and a solve that uses it, against the FP64 oracle)."""
import numpy as np
import pytest

from paper_2511_02036_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2511_02036_amd import lba  # noqa: E402


def _windows():
    return synth.c5_windows(seed=4, only=list(range(0, 256, 32)), max_points=1500)


def _batch():
    return synth.concat(_windows())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_match_eager_launches(precision):
    """Three solves from captured step graphs (with the program's own GPU work and
    synchronisations between them) against one solve with kernels launched one by one,
    each replay held to the FP64 parity bar (cost 1e-9 relative, states 1e-8) or, in mixed
    precision, to 1e-6 relative cost and 1e-6 in the states (bitwise agreement is the next
    test's)."""
    cat = _batch()
    print(f"case graph precision={precision} obs={len(cat['obs_kf'])}", flush=True)
    dev = torch.device("cuda:0")
    eager_ctx = lba.Context(device=0, precision=precision, use_graphs=0)
    ep = lba.DeviceProblem(cat, device=dev, z_f32=precision == "mixed")
    e = lba.Solver(eager_ctx, ep).run()
    torch.cuda.synchronize()
    T0, X0, f0, s0 = e.T_out.cpu().numpy(), e.X_out.cpu().numpy(), e.outlier.cpu().numpy(), e.stats.copy()
    tol_c, tol_s = (1e-9, 1e-8) if precision == "fp64" else (1e-6, 1e-6)
    gctx = lba.Context(device=0, precision=precision, use_graphs=1)
    gp = lba.DeviceProblem(cat, device=dev, z_f32=precision == "mixed")
    g = lba.Solver(gctx, gp)
    for rep in range(3):
        g.run()
        torch.cuda.synchronize()
        T, X, f, st = g.T_out.cpu().numpy(), g.X_out.cpu().numpy(), g.outlier.cpu().numpy(), g.stats
        assert np.all(np.abs(st[:, 1] - s0[:, 1]) <= tol_c * np.abs(s0[:, 1])), rep
        assert np.max(np.abs(T - T0) / np.maximum(1.0, np.abs(T0))) <= tol_s, rep
        assert np.max(np.abs(X - X0) / np.maximum(1.0, np.abs(X0))) <= tol_s, rep
        assert np.mean(f != f0) <= 1e-4, rep
        # eager work of the program between replays
        x = torch.randn(1 << 20, device=dev)
        (x * 2.0 + 1.0).sum().item()
        torch.cuda.synchronize()



@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solves_repeat_bit_for_bit(precision):
    """Every sum of the solve is taken in a fixed order (no point of these windows is seen
    twice by one keyframe), so two eager solves in separate contexts and two graph
    replays return the same bits: final cost, iteration counts, poses, points and flags."""
    cat = _batch()
    print(f"case repeat precision={precision} obs={len(cat['obs_kf'])}", flush=True)
    dev = torch.device("cuda:0")
    runs = []
    for graphs, reps in ((0, 1), (0, 1), (1, 2)):
        ctx = lba.Context(device=0, precision=precision, use_graphs=graphs)
        prob = lba.DeviceProblem(cat, device=dev, z_f32=precision == "mixed")
        s = lba.Solver(ctx, prob)
        for _ in range(reps):
            s.run()
            torch.cuda.synchronize()
            runs.append((s.T_out.cpu().numpy(), s.X_out.cpu().numpy(), s.outlier.cpu().numpy(), s.stats.copy()))
    T0, X0, f0, s0 = runs[0]
    for i, (T, X, f, st) in enumerate(runs[1:], 1):
        assert np.array_equal(st, s0), i
        assert np.array_equal(T, T0), i
        assert np.array_equal(X, X0), i
        assert np.array_equal(f, f0), i

def test_tuner_table_and_tuned_solve(ref):
    ws = _windows()
    cat = synth.concat(ws)
    dev = torch.device("cuda:0")
    ctx = lba.Context(device=0, precision="fp64")
    prob = lba.DeviceProblem(cat, device=dev)
    table = ctx.tune(prob)
    print(f"tuned table {table}", flush=True)
    assert len(table) == lba.TUNE_CLASSES and all(v in (64, 128, 256, 512, 1024, 2048, 4096) for v in table)
    assert ctx.tune_table() == table
    s = lba.Solver(ctx, prob).run()
    from tests.parity import assert_fp64_parity, window_slice
    T, X, fl, st = s.T_out.cpu().numpy(), s.X_out.cpu().numpy(), s.outlier.cpu().numpy().astype(bool), s.stats_dicts()
    for i in (0, 3, 7):
        ks, ps, os_ = window_slice(cat, i)
        r = ref.solve(ws[i])
        assert_fp64_parity(ws[i], T[ks], X[ps], fl[os_], st[i], r)


def test_stored_tile_table_is_applied_and_mixed_batches_tune(ref):
    """A table stored with lba_tune_get and installed in a fresh context with
    lba_tune_set gives the same tile plan (the same workspace) and a solve at oracle
    parity; and a batch mixing one large window with many small ones tunes without running
    out of scratch (the candidate tables' workspaces differ in their update parts)."""
    ws = _windows()
    cat = synth.concat(ws)
    dev = torch.device("cuda:0")
    a = lba.Context(device=0, precision="fp64")
    prob = lba.DeviceProblem(cat, device=dev)
    table = a.tune(prob)
    b = lba.Context(device=0, precision="fp64")
    with pytest.raises(lba.LBAError):
        b.tune_table()
    b.set_tune_table(table)
    assert b.tune_table() == table
    sa = lba.Solver(a, prob).run()
    sb = lba.Solver(b, lba.DeviceProblem(cat, device=dev)).run()
    assert sa.ws_bytes == sb.ws_bytes
    from tests.parity import assert_fp64_parity, window_slice
    T, X = sb.T_out.cpu().numpy(), sb.X_out.cpu().numpy()
    fl, st = sb.outlier.cpu().numpy().astype(bool), sb.stats_dicts()
    for i in (1, 5):
        ks, ps, os_ = window_slice(cat, i)
        assert_fp64_parity(ws[i], T[ks], X[ps], fl[os_], st[i], ref.solve(ws[i]))
    b.set_tune_table(None)
    with pytest.raises(lba.LBAError):
        b.tune_table()
    with pytest.raises(lba.LBAError, match="points per tile"):
        b.set_tune_table([0] * lba.TUNE_CLASSES)
    # one window of 5,000 points among 40 of 60
    big = synth.c5_windows(only=[0], max_points=5000)
    small = [synth.tiny_window(300 + i, K=6, n_fixed=2, M=60, nobs=(2, 5)) for i in range(40)]
    mix = synth.concat(big + small)
    c = lba.Context(device=0, precision="mixed")
    t2 = c.tune(lba.DeviceProblem(mix, device=dev, z_f32=True))
    assert len(t2) == lba.TUNE_CLASSES
