"""Pins of the oracle's environment step (CPU only).

Closed forms of the kinematic surrogate (Sec. IV-A-3), noise-free ranges,
Eq. (1) worked values, the crash rule, and an end-to-end invariant: with
noise-free ranges and static targets every tracker recovers its target
exactly, so the tracking reward is 1 and each target token is the true offset.
"""
import math
import os

import numpy as np
import pytest

from paper_2505_08222_amd.configs import env_config

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _fixed_actions(T, A, a):
    return np.full((T, A), a, np.int32)


def _run(orc, cfg, E, T, seed=0, actions=None, episode=0, ids=None):
    ids = np.arange(E) if ids is None else np.asarray(ids)
    na, nt = orc.env_counts(cfg, seed, ids)
    return orc.rollout(cfg, ids, na, nt, seed, T, episode=episode, actions=actions), na, nt


def test_straight_line_closed_form(orc):
    """Zero turn and zero noise: p_T = p_0 + T v dt (cos psi_0, sin psi_0)."""
    cfg = env_config("plain", agent_heading_sigma=0.0, target_heading_sigma=0.0,
                     agent_speed=1.3, dt=2.0, target_speed_lo=0.7, target_speed_hi=0.7)
    T, E = 50, 8
    out, na, nt = _run(orc, cfg, E, T, actions=_fixed_actions(T, E, 2))
    a0, aT = out["init_agent"], out["agent"][-1]
    want = a0[:, :2] + T * 1.3 * 2.0 * np.column_stack([np.cos(a0[:, 2]), np.sin(a0[:, 2])])
    np.testing.assert_allclose(aT[:, :2], want, rtol=0, atol=1e-9)
    np.testing.assert_allclose(aT[:, 2], a0[:, 2], rtol=0, atol=0)
    t0, tT = out["init_target"], out["target"][-1]
    want_t = t0[:, :2] + T * 0.7 * 2.0 * np.column_stack([np.cos(t0[:, 2]), np.sin(t0[:, 2])])
    np.testing.assert_allclose(tT[:, :2], want_t, rtol=0, atol=1e-9)


@pytest.mark.parametrize("action,delta", [(4, 0.3), (0, -0.3), (3, 0.15)])
def test_constant_turn_closed_form(orc, action, delta):
    """Constant turn delta, heading first then move:
    p_T = p_0 + v dt sin(T delta/2)/sin(delta/2) (cos, sin)(psi_0 + (T+1) delta/2)."""
    cfg = env_config("plain", agent_heading_sigma=0.0)
    T, E = 37, 6
    out, _, _ = _run(orc, cfg, E, T, actions=_fixed_actions(T, E, action))
    a0, aT = out["init_agent"], out["agent"][-1]
    g = math.sin(T * delta / 2) / math.sin(delta / 2)
    ang = a0[:, 2] + (T + 1) * delta / 2
    want = a0[:, :2] + g * np.column_stack([np.cos(ang), np.sin(ang)])
    np.testing.assert_allclose(aT[:, :2], want, rtol=0, atol=1e-9)
    dpsi = np.mod(aT[:, 2] - (a0[:, 2] + T * delta) + np.pi, 2 * np.pi) - np.pi
    np.testing.assert_allclose(dpsi, 0, atol=1e-12)
    assert (np.abs(out["agent"][..., 2]) <= np.pi).all()  # headings stay angles


def test_noise_free_ranges_are_distances(orc):
    cfg = env_config("batched", range_sigma_lo=0.0, range_sigma_hi=0.0)
    T, E = 20, 5
    out, na, nt = _run(orc, cfg, E, T)
    csr = out["csr"]
    for e in range(E):
        for t in range(T):
            ag = out["agent"][t, csr["agent"][e]:csr["agent"][e + 1], :2]
            tg = out["target"][t, csr["target"][e]:csr["target"][e + 1], :2]
            d = np.hypot(ag[:, None, 0] - tg[None, :, 0], ag[:, None, 1] - tg[None, :, 1])
            got = out["ranges"][t, csr["pair"][e]:csr["pair"][e + 1]].reshape(d.shape)
            np.testing.assert_allclose(got, d, rtol=0, atol=1e-9)


def test_detection_range_marks_missing(orc):
    cfg = env_config("batched", det_range=1500.0)
    out, _, _ = _run(orc, cfg, 64, 5)
    csr = out["csr"]
    seen_missing = False
    for e in range(64):
        ag = out["agent"][0, csr["agent"][e]:csr["agent"][e + 1], :2]
        tg = out["target"][0, csr["target"][e]:csr["target"][e + 1], :2]
        d = np.hypot(ag[:, None, 0] - tg[None, :, 0], ag[:, None, 1] - tg[None, :, 1]).ravel()
        r = out["ranges"][0, csr["pair"][e]:csr["pair"][e + 1]]
        assert (np.isnan(r) == (d > 1500.0)).all()
        seen_missing |= bool(np.isnan(r).any())
    assert seen_missing


def test_static_targets_exact_tracking(orc):
    """Noise-free ranges + static targets: each window's ranges are exact
    distances to a fixed point, so every estimate the tracker produces is the
    true target (the guard may refuse near-collinear agent tracks). Where
    every target has an estimate, all tracking errors are ~0 and the reward is
    1 (or -1 on a crash); target tokens are the true offsets."""
    cfg = env_config("batched", range_sigma_lo=0.0, range_sigma_hi=0.0, target_speed_lo=0.0,
                     target_speed_hi=0.0, agent_heading_sigma=0.02, d_safe=1.0)
    T, E = 30, 16
    out, na, nt = _run(orc, cfg, E, T)
    csr = out["csr"]
    n_valid = n_all = n_full = 0
    for e in range(E):
        tg = out["init_target"][csr["target"][e]:csr["target"][e + 1], :2]
        for t in range(2, T):
            ps = slice(csr["pair"][e], csr["pair"][e + 1])
            est = out["est"][t, ps].reshape(na[e], nt[e], 2)
            valid = out["est_valid"][t, ps].reshape(na[e], nt[e]).astype(bool)
            err = np.hypot(est[..., 0] - tg[None, :, 0], est[..., 1] - tg[None, :, 1])
            assert (err[valid] < 1e-6).all()
            n_valid += valid.sum()
            n_all += valid.size
            ag = out["agent"][t, csr["agent"][e]:csr["agent"][e + 1], :2]
            toks = out["obs"][t, csr["token"][e]:csr["token"][e + 1]].reshape(na[e], na[e] + nt[e], 6)
            offs = tg[None, :, :] - ag[:, None, :]
            np.testing.assert_allclose(toks[:, na[e]:, :2][valid], offs[valid], atol=1e-6)
            if valid.any(axis=0).all() and not out["crash"][t, e]:
                n_full += 1
                assert out["reward"][t, e] == 1.0
                assert out["err"][t, csr["target"][e]:csr["target"][e + 1]].max() < 1e-6
    assert n_valid > 0.8 * n_all and n_full > 0.8 * E * (T - 2)


def test_estimates_wait_for_three_entries(orc):
    cfg = env_config("plain")
    out, _, _ = _run(orc, cfg, 16, 6)
    assert not out["est_valid"][0].any() and not out["est_valid"][1].any()
    assert out["est_fresh"][2].all()
    assert np.isinf(out["err"][:2]).all()
    assert (out["reward"][:2] == 0).all()


def _eq1_rows():
    rows = []
    for line in open(os.path.join(GOLD, "tracking_reward_eq1.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            e, num, den = line.split()
            rows.append((float(e), float(num), float(den)))
    return rows


def test_tracking_reward_worked_values(orc):
    for e, num, den in _eq1_rows():
        want = math.exp(-num / den) if math.isfinite(num) else 0.0
        assert abs(orc.tracking_reward(e) - want) < 1e-15
    # continuity at both thresholds and monotone decay in between
    assert abs(orc.tracking_reward(10.0 + 1e-9) - 1.0) < 1e-9
    assert orc.tracking_reward(50.0 - 1e-6) < 1e-20
    vals = [orc.tracking_reward(e) for e in np.linspace(0, 60, 601)]
    assert all(b <= a for a, b in zip(vals, vals[1:]))
    assert orc.tracking_reward(math.inf) == 0.0


def test_reward_structure_and_crash(orc):
    cfg = env_config("ragged", d_safe=40.0)
    E, T = 64, 40
    out, na, nt = _run(orc, cfg, E, T)
    csr = out["csr"]
    r = out["reward"]
    crash_seen = 0
    for e in range(E):
        for t in range(T):
            ag = out["agent"][t, csr["agent"][e]:csr["agent"][e + 1], :2]
            d = np.hypot(ag[:, None, 0] - ag[None, :, 0], ag[:, None, 1] - ag[None, :, 1])
            d[np.diag_indices(len(ag))] = np.inf
            crash = d.min() < 40.0
            assert bool(out["crash"][t, e]) == crash
            if crash:
                assert r[t, e] == -1.0
                crash_seen += 1
            else:
                assert 0.0 <= r[t, e] <= 1.0
                errs = out["err"][t, csr["target"][e]:csr["target"][e + 1]]
                want = np.mean([orc.tracking_reward(x) for x in errs])
                assert abs(r[t, e] - want) < 1e-12
    assert crash_seen > 0


def test_tracking_error_is_team_best(orc):
    cfg = env_config("ragged")
    out, na, nt = _run(orc, cfg, 32, 25)
    csr = out["csr"]
    t = 24
    for e in range(32):
        ps = slice(csr["pair"][e], csr["pair"][e + 1])
        est = out["est"][t, ps].reshape(na[e], nt[e], 2)
        valid = out["est_valid"][t, ps].reshape(na[e], nt[e]).astype(bool)
        tg = out["target"][t, csr["target"][e]:csr["target"][e + 1], :2]
        d = np.hypot(est[..., 0] - tg[None, :, 0], est[..., 1] - tg[None, :, 1])
        d[~valid] = np.inf
        np.testing.assert_array_equal(out["err"][t, csr["target"][e]:csr["target"][e + 1]],
                                      d.min(axis=0))


def test_reset_spawn_distribution(orc):
    cfg = env_config("ragged")
    E = 2000
    out, na, nt = _run(orc, cfg, E, 0)
    a = out["init_agent"]
    assert (np.hypot(a[:, 0], a[:, 1]) <= 200.0).all()
    assert (np.abs(a[:, 2]) <= np.pi).all()
    tg = out["init_target"]
    assert (np.abs(tg[:, :2]) <= 2000.0).all()
    assert (tg[:, 3] >= 0.2).all() and (tg[:, 3] <= 1.5).all()
    s = out["sigma_r"]
    assert (s >= 0.5).all() and (s <= 3.0).all()
    # the disk is filled uniformly: the squared radius is uniform
    from scipy import stats
    assert stats.kstest((np.hypot(a[:, 0], a[:, 1]) / 200.0) ** 2, "uniform").pvalue > 1e-3


def test_env_independence_and_determinism(orc):
    """Envs are keyed by their global id: simulating a subset gives the same
    numbers as simulating them inside a larger batch."""
    cfg = env_config("ragged")
    big, na, nt = _run(orc, cfg, 40, 15)
    sel = np.array([3, 17, 39])
    small, na2, nt2 = _run(orc, cfg, None, 15, ids=sel)
    cb, cs = big["csr"], small["csr"]
    for k, e in enumerate(sel):
        np.testing.assert_array_equal(
            big["agent"][:, cb["agent"][e]:cb["agent"][e + 1]],
            small["agent"][:, cs["agent"][k]:cs["agent"][k + 1]])
        np.testing.assert_array_equal(
            big["obs"][:, cb["token"][e]:cb["token"][e + 1]],
            small["obs"][:, cs["token"][k]:cs["token"][k + 1]])
        np.testing.assert_array_equal(big["reward"][:, e], small["reward"][:, k])
    again, _, _ = _run(orc, cfg, 40, 15)
    np.testing.assert_array_equal(again["obs"], big["obs"])
    other, _, _ = _run(orc, cfg, 40, 15, episode=1)
    assert not np.array_equal(other["agent"], big["agent"])


def test_done_only_on_last_step(orc):
    cfg = env_config("plain", episode_len=12)
    out, _, _ = _run(orc, cfg, 4, 12)
    assert (out["done"][:-1] == 0).all() and (out["done"][-1] == 1).all()


def test_observation_layout(orc):
    cfg = env_config("ragged", comm_range=150.0)
    out, na, nt = _run(orc, cfg, 50, 8)
    csr = out["csr"]
    t = 7
    saw_missing_agent = False
    for e in range(50):
        toks = out["obs"][t, csr["token"][e]:csr["token"][e + 1]].reshape(na[e], na[e] + nt[e], 6)
        mask = out["obs_mask"][t, csr["token"][e]:csr["token"][e + 1]].reshape(na[e], -1)
        ag = out["agent"][t, csr["agent"][e]:csr["agent"][e + 1], :2]
        for i in range(na[e]):
            np.testing.assert_array_equal(toks[i, 0], [0, 0, 0, 1, 0, 0])
            others = [k for k in range(na[e]) if k != i]
            for m, k in enumerate(others):
                tok = toks[i, 1 + m]
                assert tok[3:].tolist() == [0, 1, 0]
                d = ag[k] - ag[i]
                if np.hypot(*d) <= 150.0:
                    assert mask[i, 1 + m] == 1
                    np.testing.assert_allclose(tok[:2], d, atol=1e-9)
                else:
                    saw_missing_agent = True
                    assert mask[i, 1 + m] == 0 and (tok[:3] == 0).all()
            for j in range(nt[e]):
                tok = toks[i, na[e] + j]
                assert tok[3:].tolist() == [0, 0, 1] and tok[2] == 0.0
    assert saw_missing_agent


def test_comm_loss_drops_broadcasts(orc):
    cfg = env_config("batched", comm_loss_p=0.5)
    out, na, nt = _run(orc, cfg, 200, 3)
    m = out["obs_mask"][2].reshape(200, 2, 4)
    frac = 1.0 - m[:, :, 1].mean()  # token 1 of each agent is the other agent
    assert 0.4 < frac < 0.6


def test_env_metrics_consistent(orc):
    cfg = env_config("ragged")
    E, T = 20, 30
    out, na, nt = _run(orc, cfg, E, T)
    m = out["env_metrics"]
    np.testing.assert_allclose(m[:, 0], out["reward"].sum(0), rtol=1e-12)
    np.testing.assert_allclose(m[:, 4], out["crash"].sum(0))
    csr = out["csr"]
    for e in range(E):
        err = out["err"][:, csr["target"][e]:csr["target"][e + 1]]
        fin = np.isfinite(err)
        np.testing.assert_allclose(m[e, 1], err[fin].sum(), rtol=1e-12)
        assert m[e, 3] == fin.sum()


def test_invalid_action_is_no_turn(orc):
    cfg = env_config("plain", agent_heading_sigma=0.0)
    T, E = 5, 3
    acts = np.full((T, E), 9, np.int32)
    out, _, _ = _run(orc, cfg, E, T, actions=acts)
    np.testing.assert_array_equal(out["agent"][-1, :, 2], out["init_agent"][:, 2])
    assert (out["actions"] == -1).all()
