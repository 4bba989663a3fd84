"""Pins of the learner oracle (oracle/ppo_oracle.py): GAE special cases with
closed forms, done handling, the clipped surrogate's values and its
gradient against torch's float64 autograd, entropy limits, the critic's
token layout, and the head gradient against finite differences of the
loss it feeds."""
import math

import numpy as np
import pytest

from oracle import ppo_oracle as po


def test_gae_closed_forms():
    rng = np.random.default_rng(0)
    T, E = 12, 5
    r = rng.normal(size=(T, E))
    v = rng.normal(size=(T + 1, E))
    d = np.zeros((T, E))
    g = 0.9
    # lambda = 0: the one-step TD residual
    a0, _ = po.gae(r, d, v, g, 0.0)
    np.testing.assert_allclose(a0, r + g * v[1:] - v[:T], atol=1e-12)
    # lambda = 1: the discounted return to the end, bootstrapped by V_T, minus V_t
    a1, ret1 = po.gae(r, d, v, g, 1.0)
    for t in range(T):
        disc = sum(g ** (k - t) * r[k] for k in range(t, T)) + g ** (T - t) * v[T]
        np.testing.assert_allclose(a1[t], disc - v[t], atol=1e-12)
        np.testing.assert_allclose(ret1[t], disc, atol=1e-12)
    # gamma = 0: reward minus value
    a2, _ = po.gae(r, d, v, 0.0, 0.7)
    np.testing.assert_allclose(a2, r - v[:T], atol=1e-12)


def test_gae_done_stops_bootstrap():
    T, E = 6, 1
    r = np.ones((T, E))
    v = np.full((T + 1, E), 10.0)
    d = np.zeros((T, E))
    d[2, 0] = 1.0
    a, _ = po.gae(r, d, v, 0.5, 1.0)
    # the step with done = 1 takes r - V only; the ones before it see nothing past it
    assert a[2, 0] == pytest.approx(1.0 - 10.0)
    assert a[1, 0] == pytest.approx(1.0 + 0.5 * 10.0 - 10.0 + 0.5 * a[2, 0])


def _sample(T=3, A=6, n_agents=2, na=5, seed=1):
    rng = np.random.default_rng(seed)
    ln = rng.normal(size=(T, A, 8))
    lo = ln + rng.normal(scale=0.3, size=(T, A, 8))
    act = rng.integers(0, na, size=(T, A))
    adv = rng.normal(size=(T, A // n_agents))
    v = rng.normal(size=(T, A // n_agents))
    R = rng.normal(size=(T, A // n_agents))
    return ln, lo, act, adv, v, R


def test_ratio_one_gives_advantage_and_policy_gradient():
    ln, _, act, adv, v, R = _sample()
    out = po.ppo_objective(ln, ln, act, adv, v, R, 2, 5, 0.2)
    N = act.size
    assert out["policy_loss"] == pytest.approx(-np.repeat(adv, 2, axis=1).mean())
    assert out["clip_frac"] == 0.0
    # rho = 1: d/dz of -A log-softmax(z)[k] / N = -A (onehot - p) / N
    t, a = 1, 3
    z = ln[t, a, :5]
    p = np.exp(z - z.max())
    p /= p.sum()
    oh = np.eye(5)[act[t, a]]
    np.testing.assert_allclose(out["dlogits"][t, a], -adv[t, a // 2] * (oh - p) / N, atol=1e-15)


def test_gradient_matches_autograd():
    torch = pytest.importorskip("torch")
    ln, lo, act, adv, v, R = _sample(T=4, A=8, n_agents=4, seed=3)
    eps = 0.15
    out = po.ppo_objective(ln, lo, act, adv, v, R, 4, 5, eps)
    z = torch.tensor(ln[..., :5], dtype=torch.float64, requires_grad=True)
    zo = torch.tensor(lo[..., :5], dtype=torch.float64)
    k = torch.tensor(act)
    lpn = torch.log_softmax(z, -1).gather(-1, k[..., None])[..., 0]
    lpo = torch.log_softmax(zo, -1).gather(-1, k[..., None])[..., 0]
    rho = torch.exp(lpn - lpo)
    A_ = torch.tensor(np.repeat(adv, 4, axis=1), dtype=torch.float64)
    loss = -torch.min(rho * A_, torch.clamp(rho, 1 - eps, 1 + eps) * A_).mean()
    loss.backward()
    assert out["policy_loss"] == pytest.approx(loss.item(), abs=1e-14)
    np.testing.assert_allclose(out["dlogits"], z.grad.numpy(), atol=1e-14)
    assert 0.0 < out["clip_frac"] < 1.0
    ent = -(torch.softmax(z, -1) * torch.log_softmax(z, -1)).sum(-1).mean()
    assert out["entropy"] == pytest.approx(ent.item(), abs=1e-14)


def test_entropy_limits_and_value_loss():
    T, A = 2, 4
    uni = np.zeros((T, A, 8))
    act = np.zeros((T, A), int)
    adv = np.zeros((T, A))
    v = np.array([[1.0, 2.0, 3.0, 4.0], [0.0, 0.0, 0.0, 0.0]])
    R = np.zeros((T, A))
    out = po.ppo_objective(uni, uni, act, adv, v, R, 1, 5, 0.2)
    assert out["entropy"] == pytest.approx(math.log(5))
    assert out["value_loss"] == pytest.approx((1 + 4 + 9 + 16) / 8)
    np.testing.assert_allclose(out["dvalues"], 2 * v / 8)
    peaked = np.zeros((T, A, 8))
    peaked[..., 0] = 60.0
    assert po.ppo_objective(peaked, peaked, act, adv, v, R, 1, 5, 0.2)["entropy"] < 1e-20


def test_critic_token_layout():
    g = np.array([[[100.0, -50.0, 0.0, 1.0, math.pi / 2, 0.0],
                   [300.0, 20.0, 0.0, 0.5, 0.0, 1.0]]])
    tok = po.critic_tokens(g, 1, 1, 1000.0)
    np.testing.assert_allclose(tok[0, 0], 0.0)
    np.testing.assert_allclose(tok[0, 1], [0.1, -0.05, 0.0, 1.0, 1.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(tok[0, 2], [0.3, 0.02, 0.5, 0.0, 0.0, 1.0], atol=1e-15)


def test_head_grad_matches_finite_differences():
    # a loss through the head: the PPO surrogate of logits W f + b; central
    # differences in each weight and bias against the analytic gradient
    rng = np.random.default_rng(7)
    T, A, na, n_agents = 2, 6, 5, 3
    feat = rng.normal(size=(T * A, 64))
    W = rng.normal(scale=0.2, size=(8, 64))
    b = rng.normal(scale=0.1, size=8)
    lo = rng.normal(size=(T, A, 8))
    act = rng.integers(0, na, size=(T, A))
    adv = rng.normal(size=(T, A // n_agents))
    v = R = np.zeros((T, A // n_agents))

    def loss(W_, b_):
        z = (feat @ W_.T + b_).reshape(T, A, 8)
        return po.ppo_objective(z, lo, act, adv, v, R, n_agents, na, 10.0)["policy_loss"]

    z = (feat @ W.T + b).reshape(T, A, 8)
    dl = po.ppo_objective(z, lo, act, adv, v, R, n_agents, na, 10.0)["dlogits"]
    dW, db = po.head_grad(feat, dl.reshape(T * A, na), na)
    assert (dW[na:] == 0).all() and (db[na:] == 0).all()
    h = 1e-6
    for k, d in ((0, 0), (2, 17), (4, 63), (1, 40)):
        Wp, Wm = W.copy(), W.copy()
        Wp[k, d] += h
        Wm[k, d] -= h
        assert dW[k, d] == pytest.approx((loss(Wp, b) - loss(Wm, b)) / (2 * h), abs=1e-8)
    for k in range(na):
        bp, bm = b.copy(), b.copy()
        bp[k] += h
        bm[k] -= h
        assert db[k] == pytest.approx((loss(W, bp) - loss(W, bm)) / (2 * h), abs=1e-8)
    # the head's rows past the actions carry no loss
    Wp = W.copy()
    Wp[6] += 1.0
    assert loss(Wp, b) == loss(W, b)


def test_head_grad_of_value_head():
    # value loss mean (w . f + c - R)^2: gradient 2 / N sum (V - R) f
    rng = np.random.default_rng(2)
    f = rng.normal(size=(9, 64))
    w = rng.normal(size=64)
    R = rng.normal(size=9)
    V = f @ w + 0.3
    dW, db = po.head_grad(f, (2.0 * (V - R) / 9)[:, None], 1)
    np.testing.assert_allclose(dW[0], 2.0 / 9 * ((V - R)[:, None] * f).sum(0), atol=1e-12)
    assert db[0] == pytest.approx(2.0 / 9 * (V - R).sum())
    assert not dW[1:].any() and not db[1:].any()
