"""Pins of the oracle's paper-faithful variants (CPU only), Sec. IV-A-2/3:

* the follow reward, Eq. (2): worked values, its normalisation over the
  targets, its limits (threshold 0 and infinity) and the crash penalty;
* rudder-state actions: five rudder angles, only adjacent moves per step,
  heading change theta(gamma) per angle: a rudder held at a fixed angle is a
  constant turn (closed form), held at the middle a straight line, and a
  saturated rudder stays at its end;
* the 50-200 m pairwise spawn: every pair within the bounds, brute force
  over many envs, shapes and bounds, and the layout randomised;
* the 30 s step itself: closed forms at dt = 30 s.
"""
import math
import os

import numpy as np
import pytest

from paper_2505_08222_amd.configs import CONFIGS, env_config

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _run(orc, cfg, E, T, seed=0, actions=None, ids=None, records=None):
    ids = np.arange(E) if ids is None else np.asarray(ids)
    na, nt = orc.env_counts(cfg, seed, ids)
    kw = {} if records is None else {"records": records}
    return orc.rollout(cfg, ids, na, nt, seed, T, actions=actions, **kw), na, nt


# ------------------------------------------------------------------ Eq. (2)
def test_follow_reward_worked_values(orc):
    rows = np.loadtxt(os.path.join(GOLD, "follow_reward_eq2.txt"))
    for d, dmin, want in rows:
        assert orc.follow_reward(float(d), float(dmin)) == want, (d, dmin)


@pytest.mark.parametrize("d_follow,want", [(math.inf, 1.0), (0.0, 0.0)])
def test_follow_reward_limits(orc, d_follow, want):
    """Threshold infinity: every target followed (reward 1 unless a crash);
    threshold 0: none (entities never coincide)."""
    cfg = env_config("paper", d_follow=d_follow, episode_len=40, d_safe=0.0)
    out, _, _ = _run(orc, cfg, 30, 40)
    assert (out["reward"] == want).all()


def test_follow_reward_counts_followed_targets(orc):
    """Reward = (number of targets whose nearest agent is within d_min) / nT,
    with the crash penalty on top: the values lie on the grid k / nT, and -1
    exactly where two agents are closer than d_safe."""
    cfg = env_config("paper", episode_len=60, d_safe=25.0)
    out, na, nt = _run(orc, cfg, 60, 60)
    r = out["reward"]
    crash = out["crash"].astype(bool)
    assert crash.any() and (~crash).any()
    np.testing.assert_array_equal(r[crash], -1.0)
    k = r[~crash] * np.broadcast_to(nt, r.shape)[~crash]
    np.testing.assert_allclose(k, np.round(k), atol=1e-12)
    assert ((k >= 0) & (k <= np.broadcast_to(nt, r.shape)[~crash])).all()
    # the agents start 50-200 m from the targets and move 30 m per step: both
    # followed and unfollowed targets occur
    assert (k > 0).any() and (k < np.broadcast_to(nt, r.shape)[~crash]).any()


def test_follow_reward_from_recorded_positions(orc):
    """Against the recorded true positions of the same rollout: the number of
    targets with an agent within d_min (evaluated here by brute force over all
    pairs, with a margin so that rounding cannot matter)."""
    cfg = env_config("paper", episode_len=30)
    E, T = 40, 30
    out, na, nt = _run(orc, cfg, E, T)
    csr = out["csr"]
    checked = 0
    for e in range(E):
        for t in range(T):
            if out["crash"][t, e]:
                continue
            ag = out["agent"][t, csr["agent"][e]:csr["agent"][e + 1], :2]
            tg = out["target"][t, csr["target"][e]:csr["target"][e + 1], :2]
            d = np.hypot(ag[:, None, 0] - tg[None, :, 0], ag[:, None, 1] - tg[None, :, 1]).min(0)
            if (np.abs(d - cfg["d_follow"]) < 1e-6).any():
                continue
            assert out["reward"][t, e] == pytest.approx((d <= cfg["d_follow"]).mean(), abs=1e-15)
            checked += 1
    assert checked > E * T // 2


# ------------------------------------------------------------ rudder actions
def _rudder_cfg(**kw):
    return env_config("paper", ragged=0, n_agents=1, n_targets=1, agent_heading_sigma=0.0,
                      spawn_mode=0, reward_mode=0, **kw)


def test_rudder_held_in_the_middle_is_a_straight_line(orc):
    cfg = _rudder_cfg()
    T, E = 25, 6
    out, _, _ = _run(orc, cfg, E, T, actions=np.full((T, E), 1, np.int32))
    a0, aT = out["init_agent"], out["agent"][-1]
    want = a0[:, :2] + T * 30.0 * np.column_stack([np.cos(a0[:, 2]), np.sin(a0[:, 2])])
    np.testing.assert_allclose(aT[:, :2], want, rtol=0, atol=1e-8)


@pytest.mark.parametrize("action,end", [(2, 4), (0, 0)])
def test_rudder_saturates_and_turns_at_a_constant_rate(orc, action, end):
    """Always 'up' (or 'down') from the middle: the rudder reaches the end
    angle after two steps (adjacent moves only) and stays there, so from then
    on the heading turns by theta(+-0.24) per step: a constant-turn arc, whose
    closed form is p_n = p_2 + v dt sin(n d/2)/sin(d/2) (cos, sin)(psi_2 + (n+1) d/2)."""
    cfg = _rudder_cfg()
    T, E = 30, 5
    out, _, _ = _run(orc, cfg, E, T, actions=np.full((T, E), action, np.int32))
    theta = cfg["action_dpsi"]
    # the first two steps turn by theta at the intermediate, then the end angle
    mid = 3 if action == 2 else 1
    a0 = out["init_agent"]
    psi1 = a0[:, 2] + theta[mid]
    psi2 = psi1 + theta[end]
    dpsi = np.mod(out["agent"][1, :, 2] - psi2 + np.pi, 2 * np.pi) - np.pi
    np.testing.assert_allclose(dpsi, 0, atol=1e-12)
    d = theta[end]
    n = T - 2
    g = 30.0 * math.sin(n * d / 2) / math.sin(d / 2)
    ang = out["agent"][1, :, 2] + (n + 1) * d / 2
    want = out["agent"][1, :, :2] + g * np.column_stack([np.cos(ang), np.sin(ang)])
    np.testing.assert_allclose(out["agent"][-1, :, :2], want, rtol=0, atol=1e-7)


def test_rudder_moves_only_to_adjacent_angles(orc):
    """Random actions: the heading change of every step (noise off) is the
    theta of a rudder position that differs from the previous step's by at
    most one, starting next to the middle; invalid actions keep the rudder."""
    cfg = _rudder_cfg()
    T, E = 80, 20
    rng = np.random.default_rng(3)
    acts = rng.integers(0, 3, size=(T, E)).astype(np.int32)
    acts[10, 4] = 7  # invalid: keeps the rudder, still turns by its angle
    out, _, _ = _run(orc, cfg, E, T, actions=acts)
    theta = np.array(cfg["action_dpsi"])
    psi = np.concatenate([out["init_agent"][None, :, 2], out["agent"][:, :, 2]])
    step = np.mod(np.diff(psi, axis=0) + np.pi, 2 * np.pi) - np.pi
    pos = np.abs(step[..., None] - theta[None, None, :]).argmin(-1)
    assert np.abs(step - theta[pos]).max() < 1e-12
    prev = np.full(E, 2)
    for t in range(T):
        a = np.where((acts[t] >= 0) & (acts[t] <= 2), acts[t], 1)
        want = np.clip(prev + a - 1, 0, 4)
        np.testing.assert_array_equal(pos[t], want)
        prev = want
    assert out["actions"][10, 4] == -1


# --------------------------------------------------------------- the spawn
@pytest.mark.parametrize("smin,smax", [(50.0, 200.0), (30.0, 120.0), (10.0, 300.0)])
def test_pairwise_spawn_bounds_brute_force(orc, smin, smax):
    """Every pair of entities spawn_min to spawn_max apart, by brute force
    over every shape up to 13 entities and many envs; the tightest pairs come
    close to both bounds (the layout uses the range it is given)."""
    cfg = env_config("paper", spawn_min=smin, spawn_max=smax)
    worst_lo, worst_hi = np.inf, 0.0
    for na in range(1, 9):
        for nt in range(1, 9):
            if na + nt > 13:
                continue
            for env in range(25):
                x, y, rc = orc.spawn_pairwise(cfg, 7, 0, env * 31 + na * 5 + nt, na, nt)
                assert rc == 0
                d = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
                iu = np.triu_indices(na + nt, 1)
                worst_lo = min(worst_lo, d[iu].min())
                worst_hi = max(worst_hi, d[iu].max())
    assert worst_lo >= smin and worst_hi <= smax, (worst_lo, worst_hi)
    assert worst_lo < smin + 0.25 * (smax - smin) and worst_hi > 0.8 * smax
    x, y, rc = orc.spawn_pairwise(cfg, 7, 0, 0, 8, 6)
    assert rc == -1


def test_pairwise_spawn_is_randomised(orc):
    """Different envs and episodes get different layouts: every entity takes
    each of the 13 sites about equally often (chi-square), and the layout's
    orientation (angle of entity 0's site) spreads over the circle."""
    from scipy import stats
    cfg = env_config("paper")
    h = 0.9 * (200.0 - 2 * math.sqrt(3) * 50.0) / (2 * math.sqrt(2) * (2 * math.sqrt(3) + 1))
    s = 50.0 + 2 * math.sqrt(2) * h
    counts = np.zeros(3)
    for env in range(2600):
        x, y, _ = orc.spawn_pairwise(cfg, 3, env % 3, env, 1, 1)
        r = math.hypot(x[0], y[0])
        ring = 0 if r < s / 2 else (1 if r < (s + s * math.sqrt(3)) / 2 else 2)
        counts[ring] += 1
    # sites per ring: 1, 6, 6 of 13
    assert stats.chisquare(counts, 2600 * np.array([1, 6, 6]) / 13).pvalue > 1e-3


def test_rollout_uses_the_pairwise_spawn(orc):
    cfg = env_config("paper")
    out, na, nt = _run(orc, cfg, 12, 1, seed=5)
    csr = out["csr"]
    for e in range(12):
        x, y, _ = orc.spawn_pairwise(cfg, 5, 0, e, int(na[e]), int(nt[e]))
        ag = out["init_agent"][csr["agent"][e]:csr["agent"][e + 1]]
        tg = out["init_target"][csr["target"][e]:csr["target"][e + 1]]
        np.testing.assert_array_equal(ag[:, 0], x[:na[e]])
        np.testing.assert_array_equal(ag[:, 1], y[:na[e]])
        np.testing.assert_array_equal(tg[:, 0], x[na[e]:])
        np.testing.assert_array_equal(tg[:, 1], y[na[e]:])


# ------------------------------------------------------------ the 30 s step
def test_thirty_second_step_target_closed_form(orc):
    """Targets with zero heading jitter move v dt = 0.5 x 30 = 15 m per step in
    a straight line."""
    cfg = env_config("paper", target_heading_sigma=0.0, ragged=0, n_agents=2, n_targets=3)
    T = 20
    out, _, _ = _run(orc, cfg, 4, T)
    t0, tT = out["init_target"], out["target"][-1]
    want = t0[:, :2] + T * 15.0 * np.column_stack([np.cos(t0[:, 2]), np.sin(t0[:, 2])])
    np.testing.assert_allclose(tT[:, :2], want, rtol=0, atol=1e-8)


def test_paper_configuration_values():
    """The configuration carries the paper's numbers: five rudder angles
    -0.24..0.24, theta(0.24) = 1.45 rad at 1 m/s and 30 s, 450 m detection,
    1500 m communication, 50 m follow threshold, 50-200 m spawn."""
    c = CONFIGS["paper"]["env"]
    assert c["dt"] == 30.0 and c["agent_speed"] == 1.0 and c["n_rudder"] == 5
    np.testing.assert_allclose(c["action_dpsi"], [-1.45, -0.725, 0.0, 0.725, 1.45])
    assert (c["det_range"], c["comm_range"], c["d_follow"]) == (450.0, 1500.0, 50.0)
    assert (c["spawn_min"], c["spawn_max"]) == (50.0, 200.0)


# ----------------------------------------------------- pooled (communicated) LS
def test_pooled_without_reception_equals_own_windows(orc):
    """With nothing received (comm range 0) or one agent per env, the pooled
    tracker has only its own rows: every estimate equals the unpooled one."""
    for over in ({"comm_range": 0.0}, {"n_agents": 1, "ragged": 0}):
        cfg0 = env_config("ragged", episode_len=40, **over)
        cfg1 = dict(cfg0, pooled=1)
        a, _, _ = _run(orc, cfg0, 40, 40)
        b, _, _ = _run(orc, cfg1, 40, 40)
        np.testing.assert_array_equal(a["est"], b["est"])
        np.testing.assert_array_equal(a["est_valid"], b["est_valid"])


def test_pooled_exact_recovery_noise_free(orc):
    """Noise-free ranges and still targets: every pooled estimate is the true
    target position (the rows of all agents are consistent)."""
    cfg = env_config("ragged", episode_len=30, pooled=1, range_sigma_lo=0.0,
                     range_sigma_hi=0.0, target_speed_lo=0.0, target_speed_hi=0.0,
                     comm_range=5000.0)
    out, na, nt = _run(orc, cfg, 30, 30)
    csr = out["csr"]
    v = out["est_valid"][-1].astype(bool)
    assert v.mean() > 0.9
    for e in range(30):
        tg = out["target"][-1, csr["target"][e]:csr["target"][e + 1], :2]
        est = out["est"][-1, csr["pair"][e]:csr["pair"][e + 1]].reshape(na[e], nt[e], 2)
        ok = out["est_valid"][-1, csr["pair"][e]:csr["pair"][e + 1]].reshape(na[e], nt[e]) == 1
        d = np.abs(est - tg[None, :, :]).max(-1)
        assert (d[ok] < 1e-6).all()


def test_pooled_rows_are_the_received_windows(orc):
    """Each pooled estimate equals the linearised LS over the rows rebuilt from
    the rollout's own records: the agent's positions and ranges of the last W
    steps, plus those of each other agent at the steps where the observing
    agent's token for it was present (its broadcast was received)."""
    cfg = env_config("ragged", episode_len=25, pooled=1, comm_range=150.0, comm_loss_p=0.3)
    E, T, W = 30, 25, cfg["window"]
    out, na, nt = _run(orc, cfg, E, T)
    csr = out["csr"]
    checked = 0
    for e in range(E):
        A, N = na[e], nt[e]
        ag = out["agent"][:, csr["agent"][e]:csr["agent"][e + 1], :2]
        rg = out["ranges"][:, csr["pair"][e]:csr["pair"][e + 1]].reshape(T, A, N)
        tok = out["obs_mask"][:, csr["token"][e]:csr["token"][e + 1]].reshape(T, A, A + N)
        t = T - 1
        for i in range(A):
            others = [k for k in range(A) if k != i]
            for j in range(N):
                rows = []
                for k in [i] + others:
                    for s in range(t, max(-1, t - W), -1):
                        heard = k == i or tok[s, i, 1 + others.index(k)] == 1
                        if heard and not np.isnan(rg[s, k, j]):
                            rows.append((ag[s, k, 0], ag[s, k, 1], rg[s, k, j]))
                win = np.array(rows, np.float64)[None]
                q, ok = orc.ls_batch(win)
                p = csr["pair"][e] + i * N + j
                if ok[0] and out["est_fresh"][t, p]:
                    np.testing.assert_allclose(out["est"][t, p], q[0], rtol=0, atol=1e-9)
                    checked += 1
    assert checked > 40


def test_batch_solver_takes_long_pooled_windows(orc):
    """Pooled windows reach 8 agents x 16 entries: the batch solver uses every
    row of a 128-row window (equal to the single solve on the same rows, and
    different from the solve on its first 64)."""
    rng = np.random.default_rng(4)
    n = 128
    a = np.cumsum(rng.normal(0, 3, (n, 2)), 0)
    tgt = np.array([250.0, -90.0])
    r = np.hypot(*(a - tgt).T) + rng.normal(0, 1.0, n)
    win = np.column_stack([a, r])[None]
    q, ok = orc.ls_batch(win)
    okk, px, py = orc.ls_estimate(a[:, 0], a[:, 1], r)
    assert ok[0] and okk
    np.testing.assert_allclose(q[0], [px, py], rtol=0, atol=1e-9)
    q64, _ = orc.ls_batch(win[:, :64])
    assert np.abs(q64[0] - q[0]).max() > 1e-6
