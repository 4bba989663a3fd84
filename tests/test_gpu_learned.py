"""GPU checks of the learned estimator's kernels against the FP64 oracle:
features, forward (FP32 and BF16 operands), loss gradient, Adam, the
fallback-guarded inference and a short training run."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_08222_amd.synth import range_windows  # noqa: E402

pytestmark = pytest.mark.gpu


def _params(orc, seed=0, scale=0.15):
    return np.random.default_rng(seed).normal(0, scale, orc.mlp_num_params()).astype(np.float32)


def test_gemm_layout_forward_fp32(orc):
    """FP32-operand MFMA path equals the FP64 network to FP32 rounding; this
    also pins the MFMA lane layout assumed by the kernels."""
    from paper_2505_08222_amd import learned
    th = _params(orc, 1)
    x = np.random.default_rng(2).normal(0, 1, (333, 64)).astype(np.float32)
    y = learned.forward(torch.from_numpy(x).cuda(), torch.from_numpy(th).cuda(), "fp32")
    ref = orc.mlp_forward(x.astype(np.float64), th.astype(np.float64))
    np.testing.assert_allclose(y.cpu().numpy(), ref, rtol=1e-5, atol=1e-5)


def test_forward_bf16(orc):
    from paper_2505_08222_amd import learned
    th = _params(orc, 3)
    x = np.random.default_rng(4).normal(0, 1, (1000, 64)).astype(np.float32)
    y = learned.forward(torch.from_numpy(x).cuda(), torch.from_numpy(th).cuda(), "bf16").cpu().numpy()
    ref = orc.mlp_forward(x.astype(np.float64), th.astype(np.float64))
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err < 3e-2, err


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("bf16", 5e-2)])
def test_gradient(orc, precision, tol):
    from paper_2505_08222_amd import learned
    th = _params(orc, 5)
    rng = np.random.default_rng(6)
    N = 700
    x = rng.normal(0, 1, (N, 64)).astype(np.float32)
    tgt = rng.normal(0, 1, (N, 2)).astype(np.float32)
    idx = rng.permutation(N)[:512]
    loss, grad = learned.loss_and_grad(torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda(),
                                       torch.from_numpy(th).cuda(),
                                       index=torch.from_numpy(idx).cuda(), precision=precision)
    rl, rg, _ = orc.mlp_backward(x[idx].astype(np.float64), tgt[idx].astype(np.float64),
                                 th.astype(np.float64))
    g = grad.cpu().numpy()
    assert abs(loss.item() - rl) <= tol * abs(rl)
    rel = np.linalg.norm(g - rg) / np.linalg.norm(rg)
    assert rel < tol, rel
    if precision == "fp32":
        np.testing.assert_allclose(g, rg, rtol=1e-3, atol=1e-5 * np.abs(rg).max())


def test_adam(orc):
    from paper_2505_08222_amd import learned
    rng = np.random.default_rng(7)
    th = rng.normal(0, 1, 25090).astype(np.float32)
    p = torch.from_numpy(th.copy()).cuda()
    opt = learned.Adam(p, lr=1e-2)
    ref = th.astype(np.float64)
    m = np.zeros_like(ref)
    v = np.zeros_like(ref)
    for step in range(1, 6):
        g = rng.normal(0, 1, 25090).astype(np.float32)
        opt.step(torch.from_numpy(g).cuda())
        orc.adam_step(ref, g.astype(np.float64), m, v, step, lr=1e-2)
    np.testing.assert_allclose(p.cpu().numpy(), ref, rtol=1e-5, atol=1e-6)


def test_features(orc):
    from paper_2505_08222_amd import learned
    win = range_windows(3000, 16, seed=9)
    x, frame = learned.features(torch.from_numpy(win).cuda())
    rx, rframe = orc.window_features(win.astype(np.float64))
    np.testing.assert_allclose(x.cpu().numpy(), rx, atol=5e-5)
    np.testing.assert_allclose(frame.cpu().numpy()[:, :2], rframe[:, :2], rtol=1e-6, atol=1e-3)
    np.testing.assert_allclose(frame.cpu().numpy()[:, 2:4], rframe[:, 2:4], atol=1e-5)


def test_infer_fallback_rule(orc):
    """Every accepted network estimate passes the residual test; every other
    window gets exactly what est_exact gives."""
    from paper_2505_08222_amd import learned
    from paper_2505_08222_amd.env import est_exact
    win = range_windows(20000, 16, seed=11, missing=0.002)
    sigma = np.random.default_rng(1).uniform(0.5, 3.0, 20000).astype(np.float32)
    params = learned.init_params(3)
    w = torch.from_numpy(win).cuda()
    out, flag = learned.infer(w, params, torch.from_numpy(sigma).cuda(), k_sigma=3.0)
    ex, ev = est_exact(w)
    out, flag, ex, ev = (t.cpu().numpy() for t in (out, flag, ex, ev))
    acc = flag == 1
    rms = orc.residual_rms(win.astype(np.float64), out.astype(np.float64))
    assert (rms[acc] <= 3.0 * sigma[acc] * (1 + 1e-4) + 1e-3).all()
    assert not acc[np.isnan(win[..., 2]).any(1)].any()
    fb = ~acc
    np.testing.assert_array_equal(out[fb & (flag == 0)], ex[fb & (flag == 0)])
    np.testing.assert_array_equal((flag[fb] == 0), ev[fb].astype(bool))


def test_training_reduces_loss():
    """A few hundred Adam steps of the BF16 kernels cut the error on windows
    whose exact estimate lies within twice the mean range (ill-conditioned
    windows give arbitrarily far estimates; they are left to the fallback)."""
    from paper_2505_08222_amd import learned
    from paper_2505_08222_amd.env import est_exact
    win = torch.from_numpy(range_windows(60000, 16, seed=21, spread=1.0, far=800.0)).cuda()
    ex, ev = est_exact(win)
    x, frame = learned.features(win)
    y = learned.targets(frame, ex)
    keep = ev.bool() & (y.norm(dim=1) <= 2.0)
    x, y = x[keep].contiguous(), y[keep].contiguous()
    base = float((y - y.mean(0)).pow(2).sum(1).mean())
    params, hist = learned.train(x, y, epochs=6, batch=1024, lr=3e-3, lr_final=3e-4, seed=0)
    pred = learned.forward(x, params, "bf16")
    mse = float((pred - y).pow(2).sum(1).mean())
    assert mse < 0.3 * base, (mse, base, hist[-3:])


@pytest.fixture(scope="module")
def trained_params():
    from paper_2505_08222_amd import learned
    from paper_2505_08222_amd.env import est_exact
    win = torch.from_numpy(range_windows(60000, 16, seed=21, spread=1.0, far=800.0)).cuda()
    ex, ev = est_exact(win)
    x, frame = learned.features(win)
    y = learned.targets(frame, ex)
    keep = ev.bool() & (y.norm(dim=1) <= 2.0)
    params, _ = learned.train(x[keep].contiguous(), y[keep].contiguous(), epochs=6, batch=1024,
                              lr=3e-3, lr_final=3e-4, seed=0)
    return params


def test_infer_decode_fits_distance_along_bearing(orc, trained_params):
    """Every network estimate (all accepted here) sits at the distance along
    its bearing from the window centroid that best fits the ranges: the FP64
    oracle's line fit, started from the GPU's estimate, leaves it in place
    (to FP32 rounding of the residual sums)."""
    from paper_2505_08222_amd import learned
    win = range_windows(20000, 16, seed=13, far=800.0)
    sigma = np.random.default_rng(2).uniform(0.5, 3.0, 20000).astype(np.float32)
    out, flag = learned.infer(torch.from_numpy(win).cuda(), trained_params,
                              torch.from_numpy(sigma).cuda(), k_sigma=1e9)
    out = out.cpu().numpy().astype(np.float64)
    assert (flag.cpu().numpy() == 1).all()
    w64 = win.astype(np.float64)
    centre = w64[..., :2].mean(1)
    ref = orc.range_refine(w64, centre, out, iters=20)
    rbar = w64[..., 2].mean(1)
    moved = np.hypot(*(ref - out).T)
    frac = (moved <= 0.05 + 1e-4 * rbar).mean()
    assert frac >= 0.99, (frac, np.percentile(moved, [50, 99, 100]))


def test_infer_acceptance_with_trained_network(trained_params):
    """With the distance fitted to the ranges, most windows of the training
    distribution pass the 3-sigma residual test."""
    from paper_2505_08222_amd import learned
    win = range_windows(20000, 16, seed=17, far=800.0)
    sigma = np.random.default_rng(3).uniform(0.5, 3.0, 20000).astype(np.float32)
    _, flag = learned.infer(torch.from_numpy(win).cuda(), trained_params,
                            torch.from_numpy(sigma).cuda(), k_sigma=3.0)
    acc = (flag.cpu().numpy() == 1).mean()
    print("accepted fraction", acc)
    assert acc >= 0.5, acc


def test_trained_network_gains_over_exact_estimator(trained_params):
    """What the trained network gains over the estimator without it: on
    windows of the training distribution, the guarded learned estimates are
    closer to the true target positions (RMS) than the exact estimates."""
    from paper_2505_08222_amd import learned
    from paper_2505_08222_amd.env import est_exact
    from paper_2505_08222_amd.synth import window_targets
    N = 20000
    win = range_windows(N, 16, seed=29, far=800.0)
    truth = window_targets(N, 16, seed=29, far=800.0)
    sigma = np.random.default_rng(4).uniform(0.5, 3.0, N).astype(np.float32)
    w = torch.from_numpy(win).cuda()
    out, flag = learned.infer(w, trained_params, torch.from_numpy(sigma).cuda(), k_sigma=3.0)
    ex, ev = est_exact(w)
    v = ev.cpu().numpy().astype(bool) & (flag.cpu().numpy() != 2)
    err_l = np.hypot(*(out.cpu().numpy()[v] - truth[v]).T)
    err_x = np.hypot(*(ex.cpu().numpy()[v] - truth[v]).T)
    rms_l, rms_x = np.sqrt((err_l ** 2).mean()), np.sqrt((err_x ** 2).mean())
    print("RMS vs truth: learned (guarded)", rms_l, "exact", rms_x)
    assert rms_l < rms_x, (rms_l, rms_x)


def test_infer_full_size_sampled(orc, trained_params):
    """The learned configuration's inference size (1e6 windows of 16): on a
    sample of 20000 windows, accepted estimates pass the residual test and
    every other window carries exactly the exact estimator's output."""
    from paper_2505_08222_amd import learned
    from paper_2505_08222_amd.env import est_exact
    N = 1_000_000
    win = range_windows(N, 16, seed=31, far=3000.0)
    sigma = np.random.default_rng(5).uniform(0.5, 3.0, N).astype(np.float32)
    w = torch.from_numpy(win).cuda()
    out, flag = learned.infer(w, trained_params, torch.from_numpy(sigma).cuda(), k_sigma=3.0)
    ex, ev = est_exact(w)
    sel = np.sort(np.random.default_rng(6).choice(N, 20000, replace=False))
    out, flag = out.cpu().numpy()[sel], flag.cpu().numpy()[sel]
    ex, ev = ex.cpu().numpy()[sel], ev.cpu().numpy()[sel]
    acc = flag == 1
    rms = orc.residual_rms(win[sel].astype(np.float64), out.astype(np.float64))
    assert (rms[acc] <= 3.0 * sigma[sel][acc] * (1 + 1e-4) + 1e-3).all()
    fb = flag == 0
    np.testing.assert_array_equal(out[fb], ex[fb])
    np.testing.assert_array_equal(flag[~acc] == 0, ev[~acc].astype(bool))


def test_infer_empty():
    from paper_2505_08222_amd import learned
    out, flag = learned.infer(torch.zeros((0, 16, 3), device="cuda"), learned.init_params(0),
                              torch.zeros((0,), device="cuda"))
    assert out.shape == (0, 2) and flag.shape == (0,)
