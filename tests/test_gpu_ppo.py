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
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_08222_amd.configs import env_config  # noqa: E402

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
