"""GPU checks of the recurrent form of the attention networks (TransfMAPPO,
Fig. 3: a carried 64-wide state as the unmasked first row, read by the head,
its final LayerNorm the next state) against the FP64 oracle
(orc.policy_forward_rec).

* Actor, one step and the next: logits and the next state within the BF16
  bound of the plain policy (3e-2 of max(1, max |x|)), the second step fed
  the GPU's own first state (teacher-forced); the state updated in place
  equals the state written elsewhere bit for bit.
* Critic over a trajectory: every step's value and state teacher-forced on
  the GPU's previous state, and the oracle's free-running chain from zeros.
* Closed loop: graph replay equals the eager loop (with the carried state);
  the action of step t is the oracle's draw on the oracle's own chain of
  states over the loop's observations (>= 95% agreement, each disagreement
  near a CDF boundary); the final state matches the oracle's last step from
  the GPU's previous state (the free-running chain, whose BF16 rounding is
  fed back every step, within 0.1).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_08222_amd.configs import env_config  # noqa: E402
from paper_2505_08222_amd.synth import policy_params, policy_tokens  # noqa: E402

pytestmark = pytest.mark.gpu


def _close(got, want, what):
    scale = max(1.0, float(np.abs(want).max()))
    err = float(np.abs(got - want).max())
    assert err <= 3e-2 * scale, (what, err, scale)
    return err


@pytest.mark.parametrize("n_agents,n_targets,n_envs", [(5, 5, 41), (2, 3, 29), (1, 1, 17),
                                                       (7, 8, 9), (3, 4, 64)])
def test_actor_recurrent_matches_oracle(orc, n_agents, n_targets, n_envs):
    from paper_2505_08222_amd import policy
    A = n_envs * n_agents
    n_obs = n_agents + n_targets
    th = policy_params(orc.policy_num_params(), seed=6)
    x0, m0 = policy_tokens(A, n_agents, n_targets, seed=n_agents + 3 * n_targets)
    x1, m1 = policy_tokens(A, n_agents, n_targets, seed=n_agents + 3 * n_targets + 1)
    dev = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    pt = dev(th)
    l0, a0, h0 = policy.forward_rec(dev(x0.reshape(-1, 6)), dev(m0.reshape(-1)), None, pt, n_obs,
                                    n_agents, 5, seed=9, t=1)
    wl0, wh0 = orc.policy_forward_rec(x0.astype(np.float64), m0, None, th.astype(np.float64))
    e0 = _close(l0.cpu().numpy(), wl0, "logits 0")
    _close(h0.cpu().numpy(), wh0, "state 0")
    # second step from the GPU's own state, out of place and in place
    l1, a1, h1 = policy.forward_rec(dev(x1.reshape(-1, 6)), dev(m1.reshape(-1)), h0, pt, n_obs,
                                    n_agents, 5, seed=9, t=2)
    hin = h0.clone()
    l1b, a1b, h1b = policy.forward_rec(dev(x1.reshape(-1, 6)), dev(m1.reshape(-1)), hin, pt, n_obs,
                                       n_agents, 5, seed=9, t=2, hidden_out=hin)
    assert h1b.data_ptr() == hin.data_ptr()
    np.testing.assert_array_equal(h1b.cpu().numpy(), h1.cpu().numpy())
    np.testing.assert_array_equal(l1b.cpu().numpy(), l1.cpu().numpy())
    np.testing.assert_array_equal(a1b.cpu().numpy(), a1.cpu().numpy())
    wl1, wh1 = orc.policy_forward_rec(x1.astype(np.float64), m1,
                                      h0.cpu().numpy().astype(np.float64), th.astype(np.float64))
    e1 = _close(l1.cpu().numpy(), wl1, "logits 1")
    _close(h1.cpu().numpy(), wh1, "state 1")
    print(f"recurrent actor {n_agents}x{n_targets}: {A} agents, logit err {e0:.2e} / {e1:.2e}")


def test_critic_recurrent_matches_oracle(orc):
    from oracle import ppo_oracle as po
    from paper_2505_08222_amd import policy, ppo
    from paper_2505_08222_amd.env import Env
    na, nt, E, T = 3, 2, 45, 6
    cfg = env_config("batched", n_agents=na, n_targets=nt, episode_len=T)
    env = Env(cfg, E, seed=4)
    env.reset(0)
    gs = env.rollout(T, record=("gstate",))["gstate"]
    params = policy.init_params(13)
    v, s = ppo.critic_forward_rec(gs, na, nt, params)
    v, s = v.cpu().numpy(), s.cpu().numpy()
    th = params.cpu().numpy().astype(np.float64)
    g = gs.cpu().numpy().astype(np.float64).reshape(T, E, na + nt, 6)
    mask = np.ones((E, na + nt), np.uint8)
    chain = None
    for t in range(T):
        tok = po.critic_tokens(g[t], na, nt, 1000.0)[:, 1:]  # entities only
        prev = None if t == 0 else s[t - 1].astype(np.float64)
        wl, wh = orc.policy_forward_rec(tok, mask, prev, th)
        _close(v[t], wl[:, 0], f"value {t}")
        _close(s[t], wh, f"state {t}")
        cl, chain = orc.policy_forward_rec(tok, mask, chain, th)
        _close(v[t], cl[:, 0], f"chain value {t}")
    # a given first state: the same as running the first step separately
    v2, s2 = ppo.critic_forward_rec(gs[1:], na, nt, params, hidden=torch.from_numpy(s[0]).cuda())
    np.testing.assert_array_equal(v2.cpu().numpy(), v[1:])
    np.testing.assert_array_equal(s2.cpu().numpy(), s[1:])
    env.close()


def test_recurrent_policy_loop(orc):
    from paper_2505_08222_amd import policy
    from paper_2505_08222_amd.env import Env
    cfg = env_config("policy", episode_len=20, n_agents=3, n_targets=2)
    E, T, seed, episode = 80, 20, 5, 1
    params = policy.init_params(4)
    rec = ("obs", "obs_mask", "actions", "reward")
    a = Env(cfg, E, seed=seed)
    pa = policy.PolicyRollout(a, params, recurrent=True)
    ra, ma = pa.run(T, episode=episode, record=rec)
    # graph replay equals the eager loop, the carried state included
    b = Env(cfg, E, seed=seed)
    pb = policy.PolicyRollout(b, params, recurrent=True)
    gout, gm = pb.capture(T, episode=episode, record=rec)
    for _ in range(2):
        pb.hidden.fill_(7.0)
        pb.launch()
        torch.cuda.synchronize()
        for k in rec:
            np.testing.assert_array_equal(gout[k].cpu().numpy(), ra[k].cpu().numpy(), err_msg=k)
        np.testing.assert_array_equal(pb.hidden.cpu().numpy(), pa.hidden.cpu().numpy())
    # the plain form differs (the head reads another row)
    c = Env(cfg, E, seed=seed)
    rp, _ = policy.PolicyRollout(c, params).run(T, episode=episode, record=("actions",))
    assert (rp["actions"].cpu().numpy() != ra["actions"].cpu().numpy()).any()
    # actions against the oracle's chain of states on the loop's observations
    out = {k: v.cpu().numpy() for k, v in ra.items()}
    na, n_obs = cfg["n_agents"], cfg["n_agents"] + cfg["n_targets"]
    A = E * na
    th = params.cpu().numpy().astype(np.float64)
    env_of = a.order["env_ids"][np.arange(A) // na]
    # the step-0 input is the reset observation (a fresh batch of the same seed)
    d = Env(cfg, E, seed=seed)
    r0 = d.reset(episode)
    obs = [r0["obs"].cpu().numpy()] + list(out["obs"][:T - 1])
    msk = [r0["obs_mask"].cpu().numpy()] + list(out["obs_mask"][:T - 1])
    hid = None
    for t in range(T):
        logits, hid = orc.policy_forward_rec(obs[t].reshape(A, n_obs, 6).astype(np.float64),
                                             msk[t].reshape(A, n_obs), hid, th)
        if t not in (0, 1, 6, 13, T - 1):
            continue
        ctr = np.stack([np.full(A, t), env_of, np.arange(A) % na,
                        np.full(A, (episode << 4) | 4)], 1).astype(np.uint32)
        u = np.array([orc.u01(int(w)) for w in orc.philox(ctr, seed)[:, 0]])
        want = np.array([orc.policy_sample(logits[i], cfg["n_actions"], u[i]) for i in range(A)])
        got = out["actions"][t]
        agree = (got == want).mean()
        assert agree >= 0.95, (t, agree)
        for i in np.flatnonzero(got != want):
            p = np.exp(logits[i, :5] - logits[i, :5].max())
            cdf = np.cumsum(p / p.sum())
            assert np.min(np.abs(cdf - u[i])) < 0.05, (t, i)
    # the state left after the loop, teacher-forced: the oracle's last step
    # from the state a loop one step shorter leaves (same draws, same inputs)
    e = Env(cfg, E, seed=seed)
    pe = policy.PolicyRollout(e, params, recurrent=True)
    pe.run(T - 1, episode=episode, record=())
    _, want = orc.policy_forward_rec(obs[T - 1].reshape(A, n_obs, 6).astype(np.float64),
                                     msk[T - 1].reshape(A, n_obs),
                                     pe.hidden.cpu().numpy().astype(np.float64), th)
    err = _close(pa.hidden.cpu().numpy(), want, "final state")
    # the free-running chain drifts further: BF16 rounding fed back T times
    drift = np.abs(pa.hidden.cpu().numpy() - hid).max() / max(1.0, np.abs(hid).max())
    print(f"recurrent loop: final state err {err:.2e}, free-chain drift {drift:.2e}")
    assert drift < 0.1
