"""Parity of the learner's forward half (critic values, GAE, clipped PPO
objective) with the FP64 oracle (oracle/ppo_oracle.py and the policy
oracle).

* Critic: the GPU's values of recorded global states against the oracle
  network on the oracle's tokens of the same states, within the BF16 bound of
  the policy logits (3e-2 of max(1, max |V|)).
* GAE: FP64 recurrence on both sides, FP32 output: 1e-6 relative.
* PPO objective: per-sample FP32 arithmetic summed in FP64 against FP64
  throughout: losses and entropy within 1e-5 of their scale; the logit
  gradient per element within 1e-5 of its largest entry, except samples whose
  ratio sits within 1e-5 of a clip edge (the clip decision may differ),
  which are counted and must stay rare; the value gradient 1e-6 relative.
* Head features: the input of each network's head (its final LayerNorm of
  the first token) against the oracle's, read out of the oracle's logits
  with heads whose rows are unit vectors (eight calls cover the 64
  features), within the BF16 bound; and the GPU's own outputs equal its
  features through the FP32 head.
* Head gradient: FP64 sums of FP32 products against the FP64 oracle, 1e-5
  of the largest entry; N = 0 gives zeros; an Adam step on the heads lowers
  the surrogate it was taken on.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_08222_amd.configs import env_config  # noqa: E402
from paper_2505_08222_amd.synth import policy_params, policy_tokens  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_agents,n_targets,E,T", [(5, 5, 61, 3), (2, 3, 40, 4), (1, 1, 33, 5),
                                                    (7, 8, 9, 2)])
def test_critic_values_match_oracle(orc, n_agents, n_targets, E, T):
    from oracle import ppo_oracle as po
    from paper_2505_08222_amd import policy, ppo
    from paper_2505_08222_amd.env import Env

    cfg = env_config("batched", n_agents=n_agents, n_targets=n_targets, episode_len=T)
    env = Env(cfg, E, seed=5)
    env.reset(0)
    gs = env.rollout(T, record=("gstate",))["gstate"]
    M = n_agents + n_targets
    params = policy.init_params(11)
    v = ppo.critic_forward(gs, n_agents, n_targets, params, pos_scale=1000.0).cpu().numpy()
    g = gs.cpu().numpy().astype(np.float64).reshape(T * E, M, 6)
    tok = po.critic_tokens(g, n_agents, n_targets, 1000.0)
    mask = np.ones(tok.shape[:2], np.uint8)
    want = orc.policy_forward(tok, mask, params.cpu().numpy().astype(np.float64))[:, 0]
    scale = max(1.0, float(np.abs(want).max()))
    err = np.abs(v - want).max()
    print(f"critic {n_agents}x{n_targets}: {T * E} states, max |V| {scale:.3f}, err {err:.2e}")
    assert err <= 3e-2 * scale
    env.close()


def test_gae_matches_oracle():
    from oracle import ppo_oracle as po
    from paper_2505_08222_amd import ppo

    rng = np.random.default_rng(0)
    T, E = 57, 301
    r = rng.normal(size=(T, E)).astype(np.float32)
    d = (rng.random((T, E)) < 0.05).astype(np.uint8)
    v = rng.normal(size=(T + 1, E)).astype(np.float32)
    for gamma, lam in ((0.99, 0.95), (1.0, 1.0), (0.9, 0.0)):
        a, R = ppo.gae(torch.tensor(r, device="cuda"), torch.tensor(d, device="cuda"),
                       torch.tensor(v, device="cuda"), gamma, lam)
        # the oracle in FP64 with the FP32 values of gamma and lambda the library gets
        wa, wR = po.gae(r, d, v, float(np.float32(gamma)), float(np.float32(lam)))
        np.testing.assert_allclose(a.cpu().numpy(), wa, rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(R.cpu().numpy(), wR, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("T,A,n_agents,n_actions", [(13, 505, 5, 5), (4, 96, 1, 8), (7, 62, 2, 3)])
def test_ppo_objective_matches_oracle(T, A, n_agents, n_actions):
    from oracle import ppo_oracle as po
    from paper_2505_08222_amd import ppo

    rng = np.random.default_rng(T * A)
    E = A // n_agents
    ln = rng.normal(size=(T, A, 8)).astype(np.float32)
    lo = (ln + rng.normal(scale=0.3, size=(T, A, 8))).astype(np.float32)
    act = rng.integers(0, n_actions, size=(T, A)).astype(np.int32)
    adv = rng.normal(size=(T, E)).astype(np.float32)
    val = rng.normal(size=(T, E)).astype(np.float32)
    ret = rng.normal(size=(T, E)).astype(np.float32)
    eps = 0.2
    dev = lambda x: torch.tensor(x, device="cuda")  # noqa: E731
    out, dl, dv = ppo.objective(dev(ln), dev(lo), dev(act), dev(adv), dev(val), dev(ret), n_agents,
                                n_actions, eps)
    out, dl, dv = out.cpu().numpy(), dl.cpu().numpy(), dv.cpu().numpy()
    want = po.ppo_objective(ln, lo, act, adv, val, ret, n_agents, n_actions, eps)
    # samples whose ratio sits on a clip edge (the decision may differ)
    lpn = ln[..., :n_actions] - np.log(np.exp(ln[..., :n_actions].astype(np.float64)).sum(-1,
                                                                                        keepdims=True))
    lpo = lo[..., :n_actions] - np.log(np.exp(lo[..., :n_actions].astype(np.float64)).sum(-1,
                                                                                        keepdims=True))
    k = act[..., None]
    rho = np.exp(np.take_along_axis(lpn, k, -1) - np.take_along_axis(lpo, k, -1))[..., 0]
    edge = (np.abs(rho - (1 + eps)) < 1e-5) | (np.abs(rho - (1 - eps)) < 1e-5)
    N = T * A
    mag = np.abs(rho * np.repeat(adv, n_agents, axis=1)).mean()
    assert abs(out[0] - want["policy_loss"]) <= 1e-5 * max(1.0, mag) + edge.sum() * 0.5 * mag / N
    assert abs(out[1] - want["value_loss"]) <= 1e-6 * max(1.0, want["value_loss"])
    assert abs(out[2] - want["entropy"]) <= 1e-5 * max(1.0, want["entropy"])
    assert abs(out[3] - want["clip_frac"]) <= edge.sum() / N + 1e-12
    assert 0.0 < want["clip_frac"] < 1.0
    gmax = np.abs(want["dlogits"]).max()
    diff = np.abs(dl[..., :n_actions] - want["dlogits"]).max(-1)
    bad = (diff > 1e-5 * gmax) & ~edge
    assert not bad.any(), (np.argwhere(bad)[:4], diff[bad][:4], gmax)
    assert (dl[..., n_actions:] == 0).all()
    np.testing.assert_allclose(dv, want["dvalues"], rtol=1e-6, atol=1e-9)
    print(f"ppo objective T={T} A={A}: out {out}, edge samples {int(edge.sum())}")


HEAD = 8 * 64 + 8


def _unit_head(params, j):
    """Parameters whose head outputs features 8j..8j+7 unchanged."""
    p = params.copy()
    W = np.zeros((8, 64))
    W[np.arange(8), 8 * j + np.arange(8)] = 1.0
    p[p.size - HEAD:p.size - 8] = W.reshape(-1)
    p[p.size - 8:] = 0.0
    return p


def _oracle_features(orc, tok, mask, params):
    return np.concatenate([orc.policy_forward(tok, mask, _unit_head(params, j))
                           for j in range(8)], axis=1)


def _check_features(feat, out, want, params, rows):
    """feat [N, 64] of the GPU against the oracle's; out [N, rows] the GPU's
    outputs of the same call against its own features through the head."""
    scale = max(1.0, float(np.abs(want).max()))
    err = np.abs(feat - want).max()
    assert err <= 3e-2 * scale, (err, scale)
    W = params[params.size - HEAD:params.size - 8].reshape(8, 64).astype(np.float64)
    b = params[params.size - 8:].astype(np.float64)
    through = feat.astype(np.float64) @ W[:rows].T + b[:rows]
    np.testing.assert_allclose(out, through, rtol=0, atol=2e-5 * max(1.0, np.abs(through).max()))
    return err


@pytest.mark.parametrize("n_agents,n_targets,n_envs", [(5, 5, 41), (2, 3, 29), (1, 1, 17)])
def test_policy_head_features(orc, n_agents, n_targets, n_envs):
    from paper_2505_08222_amd import ppo
    A = n_envs * n_agents
    x, mask = policy_tokens(A, n_agents, n_targets, seed=n_agents + 7 * n_targets)
    th = policy_params(orc.policy_num_params(), seed=4)
    n_tok = n_agents + n_targets
    logits, feat = ppo.policy_features(torch.from_numpy(x.reshape(-1, 6)).cuda(),
                                       torch.from_numpy(mask.reshape(-1)).cuda(),
                                       torch.from_numpy(th).cuda(), n_tok, n_agents)
    want = _oracle_features(orc, x.astype(np.float64), mask, th.astype(np.float64))
    err = _check_features(feat.cpu().numpy(), logits.cpu().numpy(), want, th, 8)
    print(f"policy features {n_agents}x{n_targets}: {A} agents, err {err:.2e}")


def test_critic_head_features(orc):
    from oracle import ppo_oracle as po
    from paper_2505_08222_amd import policy, ppo
    from paper_2505_08222_amd.env import Env

    na, nt, E, T = 3, 4, 37, 3
    cfg = env_config("batched", n_agents=na, n_targets=nt, episode_len=T)
    env = Env(cfg, E, seed=9)
    env.reset(0)
    gs = env.rollout(T, record=("gstate",))["gstate"]
    params = policy.init_params(12)
    v, feat = ppo.critic_forward(gs, na, nt, params, features=True)
    tok = po.critic_tokens(gs.cpu().numpy().astype(np.float64).reshape(T * E, na + nt, 6), na, nt,
                           1000.0)
    th = params.cpu().numpy()
    want = _oracle_features(orc, tok, np.ones(tok.shape[:2], np.uint8), th.astype(np.float64))
    _check_features(feat.cpu().numpy(), v.cpu().numpy()[:, None], want, th, 1)
    env.close()


@pytest.mark.parametrize("N,ld,n_out", [(1, 8, 5), (255, 8, 8), (1000, 8, 5), (70001, 8, 3),
                                        (4097, 1, 1)])
def test_head_grad_matches_oracle(N, ld, n_out):
    from oracle import ppo_oracle as po
    from paper_2505_08222_amd import ppo

    rng = np.random.default_rng(N + n_out)
    f = rng.normal(size=(N, 64)).astype(np.float32)
    d = rng.normal(scale=1e-3, size=(N, ld)).astype(np.float32)
    g = ppo.head_grad(torch.tensor(f, device="cuda"), torch.tensor(d, device="cuda"), n_out)
    g = g.cpu().numpy()
    dW, db = po.head_grad(f, d, n_out)
    want = np.concatenate([dW.reshape(-1), db])
    np.testing.assert_allclose(g, want, rtol=0, atol=1e-5 * np.abs(want).max())
    assert (g[n_out * 64:512] == 0).all() and (g[512 + n_out:] == 0).all()


def test_head_grad_empty():
    from paper_2505_08222_amd import ppo
    f = torch.empty((0, 64), dtype=torch.float32, device="cuda")
    d = torch.empty((0, 8), dtype=torch.float32, device="cuda")
    g = ppo.head_grad(f, d, 5)
    assert g.shape == (HEAD,) and (g == 0).all()


def test_head_step_lowers_surrogate(orc):
    # logits_old from the current parameters; one Adam step on the policy head
    # from the surrogate's gradient lowers the surrogate at the new logits
    from paper_2505_08222_amd import ppo
    na, nt, E = 5, 5, 64
    A = E * na
    x, mask = policy_tokens(A, na, nt, seed=3)
    th = torch.from_numpy(policy_params(orc.policy_num_params(), seed=5)).cuda()
    obs = torch.from_numpy(x.reshape(-1, 6)).cuda()
    msk = torch.from_numpy(mask.reshape(-1)).cuda()
    rng = np.random.default_rng(1)
    act = torch.tensor(rng.integers(0, 5, size=(1, A)).astype(np.int32), device="cuda")
    adv = torch.tensor(rng.normal(size=(1, E)).astype(np.float32), device="cuda")
    zero = torch.zeros((1, E), dtype=torch.float32, device="cuda")
    lo, feat = ppo.policy_features(obs, msk, th, na + nt, na)
    lo = lo.reshape(1, A, 8)
    out0, dl, _ = ppo.objective(lo, lo, act, adv, zero, zero, na, 5)
    g = ppo.head_grad(feat, dl.reshape(A, 8), 5)
    before = th.clone()
    opt = ppo.HeadAdam(th, lr=1e-3)
    opt.step(g)
    # only the head moved, each entry with a gradient by about lr
    assert torch.equal(th[:th.numel() - HEAD], before[:th.numel() - HEAD])
    step = (th - before)[th.numel() - HEAD:].cpu().numpy()
    gn = g.cpu().numpy()
    moved = np.abs(gn) > 1e-5  # Adam's first step: lr g / (|g| + eps)
    assert moved.sum() > 300
    np.testing.assert_allclose(np.abs(step[moved]), 1e-3, rtol=1e-2)
    assert (np.sign(step[moved]) == -np.sign(gn[moved])).all()
    assert np.abs(step).max() <= 1e-3 * (1 + 1e-4)
    assert not step[5 * 64:512].any() and not step[512 + 5:].any()  # unused action rows
    ln, _ = ppo.policy_features(obs, msk, th, na + nt, na)
    out1, _, _ = ppo.objective(ln.reshape(1, A, 8), lo, act, adv, zero, zero, na, 5)
    print(f"head step: surrogate {out0[0].item():.6f} -> {out1[0].item():.6f}")
    assert out1[0].item() < out0[0].item()
