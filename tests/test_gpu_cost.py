"""Differentiation form on the GPU: the robust-cost layer (lba_cost_forward /
lba_cost_backward) against the FP64 oracle's cost and analytic gradient at the same
FP32-rounded inputs, against central differences of the oracle cost (h = 1e-4, FP64),
through torch.autograd, and on edge cases.

Tolerances (FP32 arithmetic per observation, FP64 sums): the cost within 1e-5 relative;
each gradient array within |d| <= 1e-3 |ref| + 1e-4 max|ref| entrywise.  A residual is
a difference of two numbers below 1024 px, so FP32 leaves it an absolute error of a few
1e-4 px: relative to the gradient's scale that is the 1e-4 term; the 1e-3 term covers
the relative rounding of the products that follow."""
import numpy as np
import pytest

from paper_2511_02036_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _layer(data):
    from paper_2511_02036_amd import lba
    ctx = lba.Context(device=0)
    return lba.CostLayer(ctx, data, device="cuda:0"), lba


def _inputs(data, xi=None):
    dev = "cuda:0"
    X32 = np.ascontiguousarray(data["X"], dtype=np.float32).reshape(-1, 3)
    z32 = np.ascontiguousarray(data["obs_z"], dtype=np.float32).reshape(3, -1)
    tX = torch.tensor(X32, device=dev)
    tz = torch.tensor(z32, device=dev)
    txi = None if xi is None else torch.tensor(np.asarray(xi, dtype=np.float32), device=dev)
    return X32, z32, txi, tX, tz


def _oracle_window(ref, cat, i, X32, z32, xi32=None, keep=None):
    """Oracle cost and gradients of window i at the FP32-rounded inputs (keep: boolean
    mask of observations to include)."""
    from tests.parity import window_slice
    ks, ps, os_ = window_slice(cat, i)
    w = {k: cat[k] for k in ("cam", "sigma2")}
    w["T_cw"] = cat["T_cw"][ks]
    w["fixed"] = cat["fixed"][ks]
    w["X"] = X32[ps].astype(np.float64)
    sel = np.arange(os_.start, os_.stop)
    if keep is not None:
        sel = sel[keep[sel]]
    w["obs_kf"] = cat["obs_kf"][sel]
    w["obs_pt"] = cat["obs_pt"][sel]
    w["obs_z"] = z32[:, sel].astype(np.float64)
    w["obs_type"] = cat["obs_type"][sel]
    w["obs_oct"] = cat["obs_oct"][sel]
    xi = None if xi32 is None else xi32[ks].astype(np.float64)
    F, gxi, gX, gz = ref.cost_grad(w, xi=xi)
    return F, gxi, gX, gz, sel


def _close(a, b, what, rtol=1e-3, atol_frac=1e-4):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.abs(b).max(initial=0.0)
    err = np.abs(a - b)
    bound = rtol * np.abs(b) + atol_frac * scale + 1e-30
    worst = np.max(err / bound, initial=0.0)
    assert worst <= 1.0, f"{what}: worst error / bound = {worst:.3g} (max |ref| {scale:.3g})"


def test_c4_forward_backward_vs_oracle(ref):
    """All 64 windows of the differentiation workload (10 keyframes, 2,000 points, ~16k
    observations each, mono and 70/30 stereo windows)."""
    wins = synth.c4_windows(seed=3)
    cat = synth.concat(wins)
    layer, lba = _layer(cat)
    X32, z32, _, tX, tz = _inputs(cat)
    cost = layer.forward(None, tX, tz).cpu().numpy()
    g = torch.ones(layer.n_windows, dtype=torch.float64, device="cuda:0")
    gxi, gX, gz = [t.cpu().numpy() for t in layer.backward(None, tX, tz, g)]
    for i in range(len(wins)):
        F, rgxi, rgX, rgz, sel = _oracle_window(ref, cat, i, X32, z32)
        from tests.parity import window_slice
        ks, ps, os_ = window_slice(cat, i)
        assert abs(cost[i] - F) <= 1e-5 * abs(F), (i, cost[i], F)
        _close(gxi[ks], rgxi, f"window {i} g_xi")
        _close(gX[ps], rgX, f"window {i} g_X")
        _close(gz[:, os_], rgz, f"window {i} g_z")


def test_gradient_matches_central_differences(ref):
    """Directional derivatives of the oracle's FP64 cost (h = 1e-4) against the GPU
    gradient, along random directions in xi, X and z."""
    w = synth.c4_windows(seed=3, n_windows=2)[1]
    layer, lba = _layer(w)
    X32, z32, _, tX, tz = _inputs(w)
    g = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gxi, gX, gz = [t.cpu().numpy().astype(np.float64) for t in layer.backward(None, tX, tz, g)]
    base = dict(w, X=X32.astype(np.float64), obs_z=z32.astype(np.float64))
    rng = np.random.default_rng(11)
    h = 1e-4
    K = w["T_cw"].shape[0]
    for trial in range(3):
        dxi = rng.standard_normal((K, 6)) * np.array([1e-2] * 3 + [1e-2] * 3)
        dX = rng.standard_normal(X32.shape) * 1e-2
        dz = rng.standard_normal(z32.shape) * 0.5
        def F(t):
            wt = dict(base, X=base["X"] + t * dX, obs_z=base["obs_z"] + t * dz)
            return ref.cost_grad(wt, xi=t * dxi)[0]
        fd = (F(h) - F(-h)) / (2 * h)
        an = (gxi * dxi).sum() + (gX * dX).sum() + (gz * dz).sum()
        assert abs(an - fd) <= 2e-4 * max(abs(fd), 1.0), (trial, an, fd)


def test_nonzero_perturbation_uses_left_jacobian(ref):
    """xi != 0: poses Exp(xi) T and the pose gradient J_l(xi)^T (left-trivialised sum)."""
    wins = synth.c4_windows(seed=3, n_windows=4)
    cat = synth.concat(wins)
    rng = np.random.default_rng(5)
    xi = (rng.standard_normal((cat["T_cw"].shape[0], 6)) * np.array([0.05] * 3 + [0.05] * 3)).astype(np.float32)
    xi[0] = [0.4, -0.3, 0.2, 0.1, 0.0, -0.2]    # a large rotation as well
    layer, lba = _layer(cat)
    X32, z32, txi, tX, tz = _inputs(cat, xi)
    cost = layer.forward(txi, tX, tz).cpu().numpy()
    g = torch.tensor([1.0, -2.0, 0.5, 3.0], dtype=torch.float64, device="cuda:0")
    gxi, gX, gz = [t.cpu().numpy() for t in layer.backward(txi, tX, tz, g)]
    from tests.parity import window_slice
    for i in range(4):
        F, rgxi, rgX, rgz, _ = _oracle_window(ref, cat, i, X32, z32, xi32=xi)
        ks, ps, os_ = window_slice(cat, i)
        gi = float(g[i])
        assert abs(cost[i] - F) <= 1e-5 * abs(F)
        _close(gxi[ks], gi * rgxi, f"window {i} g_xi")
        _close(gX[ps], gi * rgX, f"window {i} g_X")
        _close(gz[:, os_], gi * rgz, f"window {i} g_z")


def test_mask_removes_observations(ref):
    wins = synth.c4_windows(seed=3, n_windows=2)
    cat = synth.concat(wins)
    rng = np.random.default_rng(9)
    N = cat["obs_kf"].shape[0]
    m = (rng.random(N) < 0.2).astype(np.uint8)
    layer, lba = _layer(cat)
    X32, z32, _, tX, tz = _inputs(cat)
    tm = torch.tensor(m, device="cuda:0")
    cost = layer.forward(None, tX, tz, tm).cpu().numpy()
    g = torch.ones(2, dtype=torch.float64, device="cuda:0")
    gxi, gX, gz = [t.cpu().numpy() for t in layer.backward(None, tX, tz, g, tm)]
    from tests.parity import window_slice
    keep = m == 0
    for i in range(2):
        F, rgxi, rgX, rgz, sel = _oracle_window(ref, cat, i, X32, z32, keep=keep)
        ks, ps, os_ = window_slice(cat, i)
        assert abs(cost[i] - F) <= 1e-5 * abs(F)
        _close(gxi[ks], rgxi, "masked g_xi")
        _close(gX[ps], rgX, "masked g_X")
        _close(gz[:, sel], rgz, "masked g_z")
        dropped = np.arange(os_.start, os_.stop)[m[os_] == 1]
        assert np.all(gz[:, dropped] == 0.0)


def test_autograd_function_and_determinism():
    wins = synth.c4_windows(seed=3, n_windows=3)
    cat = synth.concat(wins)
    layer, lba = _layer(cat)
    X32, z32, _, tX, tz = _inputs(cat)
    K = cat["T_cw"].shape[0]
    xi = torch.zeros((K, 6), dtype=torch.float32, device="cuda:0", requires_grad=True)
    X = tX.clone().requires_grad_(True)
    z = tz.clone().requires_grad_(True)
    cost = lba.robust_cost(layer, xi, X, z)
    wts = torch.tensor([0.5, 2.0, -1.0], dtype=torch.float64, device="cuda:0")
    (cost * wts).sum().backward()
    gxi, gX, gz = layer.backward(xi.detach(), tX, tz, wts)
    assert torch.equal(xi.grad, gxi) and torch.equal(X.grad, gX) and torch.equal(z.grad, gz)
    gxi2, gX2, gz2 = layer.backward(xi.detach(), tX, tz, wts)
    assert torch.equal(gxi, gxi2) and torch.equal(gX, gX2) and torch.equal(gz, gz2)
    c2 = layer.forward(xi.detach(), tX, tz)
    assert torch.equal(cost.detach(), c2)


def test_windows_without_observations(ref):
    """A window with points but no observations, between two ordinary ones: zero cost
    and zero gradients there, the neighbours unaffected."""
    a, b = synth.c4_windows(seed=3, n_windows=2)
    empty = dict(a)
    for k in ("obs_kf", "obs_pt", "obs_oct", "obs_type", "is_outlier_true"):
        if k in empty:
            empty[k] = empty[k][:0]
    empty["obs_z"] = a["obs_z"][:, :0]
    cat = synth.concat([a, empty, b])
    layer, lba = _layer(cat)
    X32, z32, _, tX, tz = _inputs(cat)
    cost = layer.forward(None, tX, tz).cpu().numpy()
    g = torch.ones(3, dtype=torch.float64, device="cuda:0")
    gxi, gX, gz = [t.cpu().numpy() for t in layer.backward(None, tX, tz, g)]
    from tests.parity import window_slice
    ks, ps, _ = window_slice(cat, 1)
    assert cost[1] == 0.0 and np.all(gxi[ks] == 0) and np.all(gX[ps] == 0)
    for i in (0, 2):
        F, rgxi, rgX, rgz, _ = _oracle_window(ref, cat, i, X32, z32)
        assert abs(cost[i] - F) <= 1e-5 * abs(F)
        ks, ps, os_ = window_slice(cat, i)
        _close(gX[ps], rgX, "neighbour g_X")


def test_invalid_index_is_rejected():
    w = synth.tiny_window(3, K=4, n_fixed=1, M=30)
    bad = dict(w)
    bad["obs_kf"] = w["obs_kf"].copy()
    bad["obs_kf"][3] = 99
    layer, lba = _layer(bad)
    X32, z32, _, tX, tz = _inputs(bad)
    with pytest.raises(lba.LBAError, match="keyframe index"):
        layer.forward(None, tX, tz)


@pytest.mark.parametrize("points_per_tile", [0, 37])
def test_many_keyframes_and_uneven_tiles(ref, points_per_tile):
    """A batch of a 50-keyframe window (its 300 pose-gradient entries exceed one reduce
    block, the per-entry path of the tile reduction) and a 5-keyframe window, at a
    nonzero perturbation; the default tile size and a small one that leaves ragged last
    tiles both match the oracle."""
    from paper_2511_02036_amd import lba
    rng = np.random.default_rng(21)
    big = synth.make_window(rng, trajectory="walk", K=50, n_fixed=20, M=1500, nobs=(4, 10), stereo_p=0.7,
                            walk_length=10.0)
    small = synth.make_window(rng, trajectory="walk", K=5, n_fixed=1, M=300, nobs=(3, 5), stereo_p=0.0,
                              walk_length=2.0)
    cat = synth.concat([big, small])
    xi = (rng.standard_normal((cat["T_cw"].shape[0], 6)) * 0.03).astype(np.float32)
    ctx = lba.Context(device=0, points_per_tile=points_per_tile)
    layer = lba.CostLayer(ctx, cat, device="cuda:0")
    X32, z32, txi, tX, tz = _inputs(cat, xi)
    cost = layer.forward(txi, tX, tz).cpu().numpy()
    g = torch.tensor([0.5, -1.5], dtype=torch.float64, device="cuda:0")
    gxi, gX, gz = [t.cpu().numpy() for t in layer.backward(txi, tX, tz, g)]
    from tests.parity import window_slice
    for i in range(2):
        F, rgxi, rgX, rgz, _ = _oracle_window(ref, cat, i, X32, z32, xi32=xi)
        ks, ps, os_ = window_slice(cat, i)
        gi = float(g[i])
        assert abs(cost[i] - F) <= 1e-5 * abs(F), (i, cost[i], F)
        _close(gxi[ks], gi * rgxi, f"window {i} g_xi")
        _close(gX[ps], gi * rgX, f"window {i} g_X")
        _close(gz[:, os_], gi * rgz, f"window {i} g_z")
