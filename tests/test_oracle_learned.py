"""Pins of the learned-estimator oracle (CPU only): GELU and the network
against torch's float64 reference layers, the backward pass against central
differences and autograd, Adam against torch.optim.Adam, and the feature
frame against its invariances."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_08222_amd.synth import range_windows  # noqa: E402

NIN, NH = 64, 128


def _split(th):
    t = torch.from_numpy(th)
    o = 0
    W1 = t[o:o + NH * NIN].view(NH, NIN); o += NH * NIN
    b1 = t[o:o + NH]; o += NH
    W2 = t[o:o + NH * NH].view(NH, NH); o += NH * NH
    b2 = t[o:o + NH]; o += NH
    W3 = t[o:o + 2 * NH].view(2, NH); o += 2 * NH
    b3 = t[o:o + 2]
    return W1, b1, W2, b2, W3, b3


def _torch_mlp(x, th):
    W1, b1, W2, b2, W3, b3 = _split(th)
    g = lambda z: torch.nn.functional.gelu(z, approximate="tanh")
    h1 = g(torch.from_numpy(x) @ W1.T + b1)
    h2 = g(h1 @ W2.T + b2)
    return (h2 @ W3.T + b3).numpy()


def _params(orc, seed=0, scale=0.2):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, orc.mlp_num_params())


def test_param_count(orc):
    assert orc.mlp_num_params() == 64 * 128 + 128 + 128 * 128 + 128 + 2 * 128 + 2


def test_forward_matches_torch(orc):
    th = _params(orc, 1)
    x = np.random.default_rng(2).normal(0, 1, (50, NIN))
    np.testing.assert_allclose(orc.mlp_forward(x, th), _torch_mlp(x, th), rtol=1e-12, atol=1e-12)


def test_backward_matches_autograd(orc):
    th = _params(orc, 3)
    rng = np.random.default_rng(4)
    x = rng.normal(0, 1, (40, NIN))
    tgt = rng.normal(0, 1, (40, 2))
    loss, grad, y = orc.mlp_backward(x, tgt, th)
    tt = torch.from_numpy(th.copy()).requires_grad_(True)
    W1, b1, W2, b2, W3, b3 = (None,) * 6
    o = 0
    parts = []
    for shape in [(NH, NIN), (NH,), (NH, NH), (NH,), (2, NH), (2,)]:
        n = int(np.prod(shape))
        parts.append(tt[o:o + n].view(*shape))
        o += n
    W1, b1, W2, b2, W3, b3 = parts
    g = lambda z: torch.nn.functional.gelu(z, approximate="tanh")
    out = g(g(torch.from_numpy(x) @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    ref = ((out - torch.from_numpy(tgt)) ** 2).sum(1).mean()
    ref.backward()
    assert abs(loss - ref.item()) < 1e-12
    np.testing.assert_allclose(grad, tt.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_backward_central_differences(orc):
    th = _params(orc, 5)
    rng = np.random.default_rng(6)
    x = rng.normal(0, 1, (8, NIN))
    tgt = rng.normal(0, 1, (8, 2))
    _, grad, _ = orc.mlp_backward(x, tgt, th)
    h = 1e-6
    for p in rng.choice(len(th), 60, replace=False):
        a, b = th.copy(), th.copy()
        a[p] += h
        b[p] -= h
        la, _, _ = orc.mlp_backward(x, tgt, a)
        lb, _, _ = orc.mlp_backward(x, tgt, b)
        assert abs((la - lb) / (2 * h) - grad[p]) <= 1e-6 * (1 + abs(grad[p]))


def test_adam_matches_torch(orc):
    rng = np.random.default_rng(7)
    th = rng.normal(0, 1, 300)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    tp = torch.from_numpy(th.copy()).requires_grad_(True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 8):
        g = rng.normal(0, 1, 300)
        orc.adam_step(th, g, m, v, step, lr=1e-2)
        opt.zero_grad()
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
        np.testing.assert_allclose(th, tp.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_features_invariance_and_round_trip(orc):
    win = range_windows(200, 16, seed=3).astype(np.float64)
    feat, frame = orc.window_features(win)
    # the network sees the same features after any rotation + translation
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    w2 = win.copy()
    w2[..., :2] = win[..., :2] @ R.T + np.array([123.0, -456.0])
    feat2, frame2 = orc.window_features(w2)
    np.testing.assert_allclose(feat2, feat, atol=1e-9)
    # newest-minus-oldest chord lies on +x in the window frame
    u0 = feat[:, 0:2] * 10
    ul = feat[:, 45:47] * 10
    chord = u0 - ul
    assert np.all(chord[:, 0] > 0) and np.allclose(chord[:, 1], 0, atol=1e-9)
    # zero-mean positions and ranges, mean range as the extra input
    np.testing.assert_allclose(feat[:, 0:48:3].sum(1), 0, atol=1e-9)
    np.testing.assert_allclose(feat[:, 2:48:3].sum(1), 0, atol=1e-9)
    np.testing.assert_allclose(feat[:, 48] * 1000, win[..., 2].mean(1), rtol=1e-12)
    assert (feat[:, 49:] == 0).all()
    # target encoding and decoding are inverse maps
    p = np.random.default_rng(1).uniform(-3000, 3000, (200, 2))
    np.testing.assert_allclose(orc.mlp_decode(frame, orc.mlp_target(frame, p)), p, atol=1e-9)


def test_residual_of_exact_point_is_zero(orc):
    rng = np.random.default_rng(8)
    a = rng.uniform(-50, 50, (5, 16, 2))
    p = rng.uniform(-1000, 1000, (5, 2))
    win = np.concatenate([a, np.hypot(a[..., 0] - p[:, None, 0], a[..., 1] - p[:, None, 1])[..., None]], -1)
    np.testing.assert_allclose(orc.residual_rms(win, p), 0, atol=1e-9)
    # moving the point 5 m along the line of sight changes every range by ~5 m
    d = p - a.mean(1)
    p2 = p + 5.0 * d / np.linalg.norm(d, axis=1, keepdims=True)
    assert (orc.residual_rms(win, p2) > 4.5).all()


def _bearing_setup(N=200, W=16, seed=3, noise=0.0):
    from paper_2505_08222_amd.synth import range_windows, window_targets
    win = range_windows(N, W, seed=seed, far=800.0).astype(np.float64)
    tgt = window_targets(N, W, seed=seed, far=800.0)
    if noise == 0.0:  # exact ranges
        win[..., 2] = np.hypot(win[..., 0] - tgt[:, None, 0], win[..., 1] - tgt[:, None, 1])
    centre = win[..., :2].mean(1)
    return win, tgt, centre


def test_range_refine_recovers_truth_from_exact_ranges(orc):
    """Noise-free ranges, the true bearing and a wrong start distance: the
    refined point is the target."""
    win, tgt, centre = _bearing_setup()
    u = tgt - centre
    start = centre + u * np.random.default_rng(0).uniform(0.7, 1.3, (len(u), 1))
    out = orc.range_refine(win, centre, start, iters=8)
    np.testing.assert_allclose(out, tgt, atol=1e-6)


def test_range_refine_matches_brute_force_line_search(orc):
    """Noisy ranges: the refined distance along the bearing is the minimiser of
    the range residual on a fine grid around it (brute force, 1 mm cells)."""
    win, tgt, centre = _bearing_setup(N=40, seed=5)
    rng = np.random.default_rng(1)
    start = tgt + rng.normal(0, 20.0, tgt.shape)
    out = orc.range_refine(win, centre, start, iters=20)
    for n in range(len(win)):
        e = (start[n] - centre[n]) / np.linalg.norm(start[n] - centre[n])
        d_ref = np.dot(out[n] - centre[n], e)
        grid = d_ref + np.arange(-2.0, 2.0, 1e-3)
        pts = centre[n] + grid[:, None] * e
        J = ((np.hypot(pts[:, None, 0] - win[n, None, :, 0], pts[:, None, 1] - win[n, None, :, 1])
              - win[n, None, :, 2]) ** 2).sum(1)
        assert abs(grid[np.argmin(J)] - d_ref) <= 2e-3
        # the refined point stays on the start's bearing
        v = out[n] - centre[n]
        assert abs(v[0] * e[1] - v[1] * e[0]) <= 1e-9 * max(1.0, np.linalg.norm(v))


def test_range_refine_edge_cases(orc):
    win, tgt, centre = _bearing_setup(N=10)
    same = orc.range_refine(win, centre, centre.copy(), iters=3)
    np.testing.assert_array_equal(same, centre)  # no bearing: returned as is
    w2 = win.copy()
    w2[:, 5:, 2] = np.nan  # missing entries are skipped
    out = orc.range_refine(w2, centre, centre + 0.9 * (tgt - centre), iters=8)
    np.testing.assert_allclose(out, tgt, atol=1e-6)
    zero = orc.range_refine(win, centre, centre + 0.9 * (tgt - centre), iters=0)
    np.testing.assert_allclose(zero, centre + 0.9 * (tgt - centre))
