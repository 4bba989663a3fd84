"""GPU checks of the networks' training form (FP32 forward pass with its
tape, exact reverse pass) against the FP64 oracle (orc.policy_backward,
orc.policy_backward_rec, the forwards).

* Forward: logits (or values) within 1e-4 of max(1, max |logit|) of the
  oracle's (FP32 throughout: no BF16 operands here).
* Gradient: every parameter group (embedding, per layer the LayerNorms, the
  Q/K/V projection, attention output, feed-forward, and the final LayerNorm
  and head) within 2e-4 of that group's largest oracle entry; the carried
  state's gradient likewise. FP32 sums over up to a few thousand rows against
  FP64 give errors of order 1e-6 of the scale.
* Full updates (policy and critic, every parameter, Adam at a small step)
  lower the surrogate and the value loss at every step.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_08222_amd.configs import env_config  # noqa: E402
from paper_2505_08222_amd.synth import policy_params, policy_tokens  # noqa: E402

pytestmark = pytest.mark.gpu

D, F, L, NA = 64, 256, 2, 8
PER_LAYER = 2 * D + 3 * D * D + 3 * D + D * D + D + 2 * D + F * D + F + D * F + D
GROUPS = [("E", D * 6), ("e", D)] + [
    (f"{n}{l}", s) for l in range(L) for n, s in (
        ("ln1g", D), ("ln1b", D), ("Wqkv", 3 * D * D), ("bqkv", 3 * D), ("Wo", D * D),
        ("bo", D), ("ln2g", D), ("ln2b", D), ("W1", F * D), ("b1", F), ("W2", D * F),
        ("b2", D))] + [("lnfg", D), ("lnfb", D), ("Wh", NA * D), ("bh", NA)]


def _check_grad(got, want, tol=2e-4):
    off = 0
    worst = 0.0
    for name, size in GROUPS:
        g, w = got[off:off + size], want[off:off + size]
        scale = max(np.abs(w).max(), 1e-30)
        err = np.abs(g - w).max() / scale
        worst = max(worst, err)
        assert err <= tol or np.abs(w).max() < 1e-12, (name, err, scale)
        off += size
    assert off == got.size
    return worst


# the last case has 1001 agents x 9 tokens = 9009 rows: the weight gradients
# are summed over several row blocks in order, the last one ragged
@pytest.mark.parametrize("n_agents,n_targets,n_envs", [(5, 5, 41), (2, 3, 29), (1, 1, 17),
                                                       (7, 8, 9), (7, 2, 143)])
def test_policy_gradient_matches_oracle(orc, n_agents, n_targets, n_envs):
    from paper_2505_08222_amd import ppo
    A = n_envs * n_agents
    n_tok = n_agents + n_targets
    x, mask = policy_tokens(A, n_agents, n_targets, seed=2 * n_agents + n_targets)
    th = policy_params(orc.policy_num_params(), seed=8)
    dl = np.random.default_rng(A).normal(size=(A, 8)).astype(np.float32)
    dl[:, 5:] = 0.0
    tp = ppo.TrainPass(A, n_tok)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    logits, feat = tp.forward(dev(x.reshape(-1, 6)), dev(mask.reshape(-1)), dev(th))
    want = orc.policy_forward(x.astype(np.float64), mask, th.astype(np.float64))
    err = np.abs(logits.cpu().numpy() - want).max()
    assert err <= 1e-4 * max(1.0, np.abs(want).max()), err
    grad, _ = tp.backward(dev(th), dev(dl), 5)
    gw = orc.policy_backward(x.astype(np.float64), mask, th.astype(np.float64),
                             dl.astype(np.float64))
    worst = _check_grad(grad.cpu().numpy(), gw)
    print(f"train {n_agents}x{n_targets}: {A} agents, logit err {err:.1e}, grad err {worst:.1e}")


def test_recurrent_gradient_matches_oracle(orc):
    from paper_2505_08222_amd import ppo
    na, nt, E = 3, 4, 23
    A = E * na
    n_obs = na + nt
    x, mask = policy_tokens(A, na, nt, seed=31)
    th = policy_params(orc.policy_num_params(), seed=9)
    rng = np.random.default_rng(3)
    hid = rng.normal(size=(A, D)).astype(np.float32)
    dl = rng.normal(size=(A, 8)).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    tp = ppo.TrainPass(A, n_obs + 1, rec=1)
    logits, feat = tp.forward(dev(x.reshape(-1, 6)), dev(mask.reshape(-1)), dev(th), dev(hid))
    wl, wh = orc.policy_forward_rec(x.astype(np.float64), mask, hid.astype(np.float64),
                                    th.astype(np.float64))
    assert np.abs(logits.cpu().numpy() - wl).max() <= 1e-4 * max(1.0, np.abs(wl).max())
    assert np.abs(feat.cpu().numpy() - wh).max() <= 1e-4 * max(1.0, np.abs(wh).max())
    grad, dh = tp.backward(dev(th), dev(dl), 8)
    gw, dhw = orc.policy_backward_rec(x.astype(np.float64), mask, hid.astype(np.float64),
                                      th.astype(np.float64), dl.astype(np.float64))
    _check_grad(grad.cpu().numpy(), gw)
    assert np.abs(dh.cpu().numpy() - dhw).max() <= 2e-4 * np.abs(dhw).max()
    # no carried state: zeros
    tp.forward(dev(x.reshape(-1, 6)), dev(mask.reshape(-1)), dev(th), None)
    g0, _ = tp.backward(dev(th), dev(dl), 8)
    gz, _ = orc.policy_backward_rec(x.astype(np.float64), mask, None, th.astype(np.float64),
                                    dl.astype(np.float64))
    _check_grad(g0.cpu().numpy(), gz)


# the token-count limits: 16 rows per agent (recurrent, 15 observed tokens:
# every lane of the attention kernels busy, the largest LDS stage) and a
# single-token agent (one key, probability 1)
@pytest.mark.parametrize("na,nt,rec,E", [(7, 8, 1, 11), (1, 0, 0, 301)])
def test_gradient_at_token_count_limits(orc, na, nt, rec, E):
    from paper_2505_08222_amd import ppo
    A = E * na
    n_obs = na + nt
    x, mask = policy_tokens(A, na, nt, seed=41 + nt)
    th = policy_params(orc.policy_num_params(), seed=12)
    rng = np.random.default_rng(17)
    hid = rng.normal(size=(A, D)).astype(np.float32)
    dl = rng.normal(size=(A, 8)).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    tp = ppo.TrainPass(A, n_obs + rec, rec=rec)
    if rec:
        logits, _ = tp.forward(dev(x.reshape(-1, 6)), dev(mask.reshape(-1)), dev(th), dev(hid))
        want, _ = orc.policy_forward_rec(x.astype(np.float64), mask, hid.astype(np.float64),
                                         th.astype(np.float64))
        grad, dh = tp.backward(dev(th), dev(dl), 8)
        gw, dhw = orc.policy_backward_rec(x.astype(np.float64), mask, hid.astype(np.float64),
                                          th.astype(np.float64), dl.astype(np.float64))
        assert np.abs(dh.cpu().numpy() - dhw).max() <= 2e-4 * np.abs(dhw).max()
    else:
        logits, _ = tp.forward(dev(x.reshape(-1, 6)), dev(mask.reshape(-1)), dev(th))
        want = orc.policy_forward(x.astype(np.float64), mask, th.astype(np.float64))
        grad, _ = tp.backward(dev(th), dev(dl), 8)
        gw = orc.policy_backward(x.astype(np.float64), mask, th.astype(np.float64),
                                 dl.astype(np.float64))
    assert np.abs(logits.cpu().numpy() - want).max() <= 1e-4 * max(1.0, np.abs(want).max())
    worst = _check_grad(grad.cpu().numpy(), gw)
    print(f"train limits {n_obs + rec} rows: grad err {worst:.1e}")


@pytest.mark.parametrize("rec", [0, 1])
def test_critic_gradient_matches_oracle(orc, rec):
    from oracle import ppo_oracle as po
    from paper_2505_08222_amd import policy, ppo
    from paper_2505_08222_amd.env import Env
    na, nt, E, T = 3, 2, 37, 2
    cfg = env_config("batched", n_agents=na, n_targets=nt, episode_len=T)
    env = Env(cfg, E, seed=6)
    env.reset(0)
    gs = env.rollout(T, record=("gstate",))["gstate"][T - 1]
    params = policy.init_params(14)
    th = params.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(4)
    hid = torch.tensor(rng.normal(size=(E, D)).astype(np.float32), device="cuda") if rec else None
    dv = torch.tensor(rng.normal(size=E).astype(np.float32), device="cuda")
    tp = ppo.TrainPass(E, na + nt + 1, rec=rec)
    v, feat = tp.critic_forward(gs, na, nt, params, hidden=hid)
    tok = po.critic_tokens(gs.cpu().numpy().astype(np.float64).reshape(E, na + nt, 6), na, nt,
                           1000.0)
    dl = np.zeros((E, 8))
    dl[:, 0] = dv.cpu().numpy()
    if rec:
        tok = tok[:, 1:]
        h64 = hid.cpu().numpy().astype(np.float64)
        wl, _ = orc.policy_forward_rec(tok, np.ones(tok.shape[:2], np.uint8), h64, th)
        gw, _ = orc.policy_backward_rec(tok, np.ones(tok.shape[:2], np.uint8), h64, th, dl)
    else:
        wl = orc.policy_forward(tok, np.ones(tok.shape[:2], np.uint8), th)
        gw = orc.policy_backward(tok, np.ones(tok.shape[:2], np.uint8), th, dl)
    assert np.abs(v.cpu().numpy() - wl[:, 0]).max() <= 1e-4 * max(1.0, np.abs(wl[:, 0]).max())
    grad, _ = tp.backward(params, dv, 1)
    _check_grad(grad.cpu().numpy(), gw)
    env.close()


def test_full_update_lowers_losses(orc):
    # one PPO update of every parameter of the actor and the critic: the
    # surrogate at the new logits and the value loss at the new values fall
    from paper_2505_08222_amd import learned, policy, ppo
    na, nt, E = 3, 3, 96
    A, n_tok = E * na, na + nt
    x, mask = policy_tokens(A, na, nt, seed=5)
    obs = torch.from_numpy(x.reshape(-1, 6)).cuda()
    msk = torch.from_numpy(mask.reshape(-1)).cuda()
    actor = policy.init_params(30)
    critic = policy.init_params(31)
    rng = np.random.default_rng(8)
    act = torch.tensor(rng.integers(0, 5, size=(1, A)).astype(np.int32), device="cuda")
    adv = torch.tensor(rng.normal(size=(1, E)).astype(np.float32), device="cuda")
    ret = torch.tensor(rng.normal(size=(1, E)).astype(np.float32), device="cuda")
    gs = torch.randn(E, na + nt, 6, device="cuda",
                     generator=torch.Generator(device="cuda").manual_seed(9))
    gs[..., 5] = (torch.arange(na + nt, device="cuda") >= na).float()
    ta, tc = ppo.TrainPass(A, n_tok), ppo.TrainPass(E, na + nt + 1)
    # Adam's first steps move every one of the ~1e5 parameters by about lr
    # together: lr small enough for the first-order decrease to dominate
    oa, oc = learned.Adam(actor, lr=1e-5), learned.Adam(critic, lr=1e-5)
    lo, _ = ta.forward(obs, msk, actor)
    lo = lo.reshape(1, A, 8).clone()
    losses = []
    for it in range(3):
        ln, _ = ta.forward(obs, msk, actor)
        v, _ = tc.critic_forward(gs, na, nt, critic)
        out, dl, dv = ppo.objective(ln.reshape(1, A, 8), lo, act, adv, v.reshape(1, E), ret, na, 5)
        losses.append((out[0].item(), out[1].item()))
        ga, _ = ta.backward(actor, dl.reshape(A, 8), 5)
        gc, _ = tc.backward(critic, dv.reshape(E), 1)
        assert torch.isfinite(ga).all() and torch.isfinite(gc).all()
        oa.step(ga)
        oc.step(gc)
    print("update losses", losses)
    for k in range(1, len(losses)):
        assert losses[k][0] < losses[k - 1][0] and losses[k][1] < losses[k - 1][1], losses


def test_learner_iteration_on_closed_loop_experience():
    # one batch of closed-loop experience, then the learner's epochs: every
    # loss finite, both networks changed, and the batch's surrogate lower
    # after the update than before it
    from paper_2505_08222_amd import policy, ppo
    from paper_2505_08222_amd.env import Env
    na, nt, E, T, ep = 2, 2, 64, 16, 0
    cfg = env_config("policy", episode_len=T, n_agents=na, n_targets=nt)
    env = Env(cfg, E, seed=11)
    actor, critic = policy.init_params(40), policy.init_params(41)
    r0 = env.reset(ep, record=("obs", "obs_mask", "gstate"))
    out, _ = policy.PolicyRollout(env, actor).run(
        T, episode=ep, record=("obs", "obs_mask", "actions", "gstate", "reward", "done"))
    obs = torch.cat([r0["obs"][None], out["obs"][:T - 1]])
    mask = torch.cat([r0["obs_mask"][None], out["obs_mask"][:T - 1]])
    gs = torch.cat([r0["gstate"][None], out["gstate"]])
    a0, c0 = actor.clone(), critic.clone()
    lr = ppo.Learner(actor, critic, na, nt, lr=1e-4, behaviour="training")
    before = lr.logits(obs, mask)
    # the advantages the update itself uses (the critic before the update)
    vals = lr.values(gs.reshape(T + 1, E, na + nt, 6))
    adv, ret = ppo.gae(out["reward"], out["done"], vals, 0.99, 0.95)
    hist = lr.update(obs, mask, out["actions"], gs, out["reward"], out["done"], epochs=2,
                     minibatches=2)
    assert torch.isfinite(hist).all()
    assert not torch.equal(actor, a0) and not torch.equal(critic, c0)
    # the surrogate of the whole batch at the new logits against the old ones
    after = lr.logits(obs, mask)
    o0, _, _ = ppo.objective(before, before, out["actions"], adv, vals[:T].contiguous(), ret, na, 5)
    o1, _, _ = ppo.objective(after, before, out["actions"], adv, vals[:T].contiguous(), ret, na, 5)
    print("learner: minibatch losses", hist[:, :2].cpu().numpy().round(4).tolist(),
          "surrogate", o0[0].item(), "->", o1[0].item())
    assert o1[0].item() < o0[0].item()
    env.close()


def test_bptt_matches_oracle(orc):
    # three recurrent steps from zeros, differentiated through the carried
    # state: the GPU's chain against the oracle's (policy_bptt)
    from paper_2505_08222_amd import ppo
    na, nt, E, T = 2, 3, 21, 3
    A, n_obs = E * na, na + nt
    th = policy_params(orc.policy_num_params(), seed=12)
    seq = [policy_tokens(A, na, nt, seed=50 + t) for t in range(T)]
    rng = np.random.default_rng(5)
    dls = rng.normal(size=(T, A, 8)).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    params = dev(th)
    tp = ppo.TrainPass(A, n_obs + 1, rec=1)
    obs = [dev(x.reshape(-1, 6)) for x, _ in seq]
    msk = [dev(m.reshape(-1)) for _, m in seq]
    grad, states = ppo.bptt(tp, lambda t, h: tp.forward(obs[t], msk[t], params, h),
                            [dev(d) for d in dls], params, 8)
    want = orc.policy_bptt(np.stack([x.astype(np.float64) for x, _ in seq]),
                           np.stack([m for _, m in seq]), th.astype(np.float64),
                           dls.astype(np.float64))
    worst = _check_grad(grad.cpu().numpy(), want, tol=5e-4)
    print(f"bptt {T} steps x {A} agents: grad err {worst:.1e}")
    # accumulate: a second reverse pass of the last step adds its gradient
    tp.forward(obs[T - 1], msk[T - 1], params, states[T - 2])
    g_last, _ = tp.backward(params, dev(dls[T - 1]), 8)
    tp.forward(obs[T - 1], msk[T - 1], params, states[T - 2])
    g2, _ = tp.backward(params, dev(dls[T - 1]), 8, grad=g_last.clone(), accumulate=True)
    np.testing.assert_allclose(g2.cpu().numpy(), 2 * g_last.cpu().numpy(), rtol=1e-6,
                               atol=1e-6 * float(g_last.abs().max()))


def test_critic_bptt_matches_oracle(orc):
    from oracle import ppo_oracle as po
    from paper_2505_08222_amd import policy, ppo
    from paper_2505_08222_amd.env import Env
    na, nt, E, T = 2, 2, 29, 3
    cfg = env_config("batched", n_agents=na, n_targets=nt, episode_len=T)
    env = Env(cfg, E, seed=8)
    env.reset(0)
    gs = env.rollout(T, record=("gstate",))["gstate"]
    params = policy.init_params(15)
    rng = np.random.default_rng(6)
    dv = rng.normal(size=(T, E)).astype(np.float32)
    tc = ppo.TrainPass(E, na + nt + 1, rec=1)
    grad, _ = ppo.bptt(tc, lambda t, h: tc.critic_forward(gs[t], na, nt, params, hidden=h),
                       [torch.tensor(dv[t], device="cuda") for t in range(T)], params, 1)
    g = gs.cpu().numpy().astype(np.float64).reshape(T, E, na + nt, 6)
    tok = np.stack([po.critic_tokens(g[t], na, nt, 1000.0)[:, 1:] for t in range(T)])
    dl = np.zeros((T, E, 8))
    dl[..., 0] = dv
    want = orc.policy_bptt(tok, np.ones(tok.shape[:3], np.uint8),
                           params.cpu().numpy().astype(np.float64), dl)
    _check_grad(grad.cpu().numpy(), want, tol=5e-4)
    env.close()


def test_recurrent_learner_on_closed_loop_experience():
    # the recurrent closed loop's experience through the recurrent learner
    # (both networks differentiated through time over the batch's 12 steps,
    # minibatches of whole envs): finite losses, both networks changed, the
    # batch's surrogate lower afterwards
    from paper_2505_08222_amd import policy, ppo
    from paper_2505_08222_amd.env import Env
    na, nt, E, T, ep = 2, 2, 48, 12, 0
    cfg = env_config("policy", episode_len=T, n_agents=na, n_targets=nt)
    env = Env(cfg, E, seed=12)
    actor, critic = policy.init_params(42), policy.init_params(43)
    r0 = env.reset(ep, record=("obs", "obs_mask", "gstate"))
    out, _ = policy.PolicyRollout(env, actor, recurrent=True).run(
        T, episode=ep, record=("obs", "obs_mask", "actions", "gstate", "reward", "done"))
    obs = torch.cat([r0["obs"][None], out["obs"][:T - 1]])
    mask = torch.cat([r0["obs_mask"][None], out["obs_mask"][:T - 1]])
    gs = torch.cat([r0["gstate"][None], out["gstate"]])
    a0, c0 = actor.clone(), critic.clone()
    lr = ppo.Learner(actor, critic, na, nt, lr=1e-4, recurrent=True, behaviour="training")
    before = lr.logits(obs, mask)
    # the advantages the update itself uses (the critic before the update)
    vals = lr.values(gs.reshape(T + 1, E, na + nt, 6))
    adv, ret = ppo.gae(out["reward"], out["done"], vals, 0.99, 0.95)
    hist = lr.update(obs, mask, out["actions"], gs, out["reward"], out["done"], epochs=2,
                     minibatches=2)
    assert torch.isfinite(hist).all()
    assert not torch.equal(actor, a0) and not torch.equal(critic, c0)
    after = lr.logits(obs, mask)
    o0, _, _ = ppo.objective(before, before, out["actions"], adv, vals[:T].contiguous(), ret, na, 5)
    o1, _, _ = ppo.objective(after, before, out["actions"], adv, vals[:T].contiguous(), ret, na, 5)
    print("recurrent learner: minibatch losses", hist[:, :2].cpu().numpy().round(4).tolist(),
          "surrogate", o0[0].item(), "->", o1[0].item())
    assert o1[0].item() < o0[0].item()
    env.close()


def test_accumulate_on_the_row_block_path(orc):
    # 1001 agents x 9 rows (the recurrent form: 8 tokens + the state): the
    # weight gradients are summed over several row blocks, the last one
    # ragged; adding a second reverse pass of the same step gives twice the
    # first, and the first matches the oracle
    from paper_2505_08222_amd import ppo
    A = 1001
    x, m = policy_tokens(A, 1, 7, seed=19)
    th = policy_params(orc.policy_num_params(), seed=13)
    rng = np.random.default_rng(9)
    hid = rng.normal(size=(A, D)).astype(np.float32)
    dl = rng.normal(size=(A, 8)).astype(np.float32)
    dn = rng.normal(size=(A, D)).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    params = dev(th)
    tp = ppo.TrainPass(A, 9, rec=1)
    tp.forward(dev(x.reshape(-1, 6)), dev(m.reshape(-1)), params, dev(hid))
    g1, dh = tp.backward(params, dev(dl), 8, dnext=dev(dn))
    g2, _ = tp.backward(params, dev(dl), 8, dnext=dev(dn), grad=g1.clone(), accumulate=True)
    np.testing.assert_allclose(g2.cpu().numpy(), 2 * g1.cpu().numpy(), rtol=1e-6,
                               atol=1e-6 * float(g1.abs().max()))
    gw, dhw = orc.policy_backward_rec(x.astype(np.float64), m, hid.astype(np.float64),
                                      th.astype(np.float64), dl.astype(np.float64),
                                      dn.astype(np.float64))
    _check_grad(g1.cpu().numpy(), gw)
    assert np.abs(dh.cpu().numpy() - dhw).max() <= 2e-4 * np.abs(dhw).max()



@pytest.mark.parametrize("recurrent", [False, True])
def test_learner_behaviour_from_the_inference_kernels(recurrent):
    # the old logits are those of the policy that sampled the loop's actions
    # (the inference kernel on the loop's own observations, the recurrent
    # chain from zeros), the values the inference critic's, and an update
    # from them changes both networks with finite losses
    from paper_2505_08222_amd import policy, ppo
    from paper_2505_08222_amd.env import Env
    na, nt, E, T = 2, 2, 32, 8
    cfg = env_config("policy", episode_len=T, n_agents=na, n_targets=nt)
    env = Env(cfg, E, seed=13)
    actor, critic = policy.init_params(44), policy.init_params(45)
    r0 = env.reset(0, record=("obs", "obs_mask", "gstate"))
    out, _ = policy.PolicyRollout(env, actor, recurrent=recurrent).run(
        T, record=("obs", "obs_mask", "actions", "gstate", "reward", "done"))
    obs = torch.cat([r0["obs"][None], out["obs"][:T - 1]])
    mask = torch.cat([r0["obs_mask"][None], out["obs_mask"][:T - 1]])
    gs = torch.cat([r0["gstate"][None], out["gstate"]])
    lr = ppo.Learner(actor, critic, na, nt, lr=1e-4, recurrent=recurrent)
    vals, lo = lr._behaviour(obs, mask, gs.reshape(T + 1, E, na + nt, 6))
    A, n_tok = E * na, na + nt
    if recurrent:
        h = None
        for t in range(T):
            lg, _, h = policy.forward_rec(obs[t], mask[t], h, actor, n_tok, na)
            assert torch.equal(lg, lo[t])
        v_want = ppo.critic_forward_rec(gs, na, nt, critic)[0]
    else:
        for t in range(T):
            assert torch.equal(policy.forward(obs[t], mask[t], actor, n_tok, na)[0], lo[t])
        v_want = ppo.critic_forward(gs, na, nt, critic).reshape(T + 1, E)
    assert torch.equal(vals, v_want)
    # the training form's values and logits agree with them to the BF16 bound
    vt = lr.values(gs.reshape(T + 1, E, na + nt, 6))
    assert float((vt - vals).abs().max()) <= 3e-2 * max(1.0, float(vt.abs().max()))
    a0, c0 = actor.clone(), critic.clone()
    hist = lr.update(obs, mask, out["actions"], gs, out["reward"], out["done"], epochs=1,
                     minibatches=2)
    assert torch.isfinite(hist).all()
    assert not torch.equal(actor, a0) and not torch.equal(critic, c0)
    env.close()


def test_large_batch_gradient_is_reproducible_and_splits(orc):
    # 16384 agents x 10 tokens (the policy workload's minibatch scale): two
    # reverse passes give identical bits, and the gradient equals the sum of
    # the two halves' gradients (other row counts, so other GEMM shapes and
    # row-block partitions) to FP32 rounding
    from paper_2505_08222_amd import ppo
    A, H = 16384, 8192
    x, m = policy_tokens(A, 5, 5, seed=23)
    th = policy_params(orc.policy_num_params(), seed=29)
    rng = np.random.default_rng(31)
    dl = rng.normal(size=(A, 8)).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    params = dev(th)
    xs, ms, dls = dev(x.reshape(A, 10, 6)), dev(m.reshape(A, 10)), dev(dl)
    tp = ppo.TrainPass(A, 10)
    tp.forward(xs.reshape(-1, 6), ms.reshape(-1), params)
    g1, _ = tp.backward(params, dls, 8)
    g2, _ = tp.backward(params, dls, 8)
    assert torch.equal(g1, g2)
    th_ = ppo.TrainPass(H, 10)
    th_.forward(xs[:H].reshape(-1, 6), ms[:H].reshape(-1), params)
    gh, _ = th_.backward(params, dls[:H], 8)
    th_.forward(xs[H:].reshape(-1, 6), ms[H:].reshape(-1), params)
    gh, _ = th_.backward(params, dls[H:], 8, grad=gh, accumulate=True)
    _check_grad(gh.cpu().numpy(), g1.cpu().numpy().astype(np.float64), tol=1e-5)
