"""Pins of the learner oracle (oracle/ppo_oracle.py): GAE special cases with
closed forms, done handling, the clipped surrogate's values and its
gradient against torch's float64 autograd, entropy limits, and the critic's
token layout."""
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
