"""The five workload configurations of the batched tracking environment.

Each config is a plain dict of parameter values (SI units). The same dict is
handed to the GPU library and, in the tests, to the FP64 oracle; it holds no
arithmetic of the method.

Paper constants used as defaults (arXiv 2505.08222):
  * Eq. (1) thresholds eps_min = 10 m, eps_max = 50 m;
  * agent heading noise 0.02 rad (Sec. IV-A-3);
  * detection range 450 m and communication range 1500 m (Sec. IV-A-2). The
    batched workloads place targets uniformly in a square of 2-4 km with the
    agents near the centre, so the detection cut is lifted (det_range = inf)
    to keep every tracker busy; 450 m is kept as the "lost target" distance.
"""
import copy
import math

ACTIONS_DPSI = [-0.3, -0.15, 0.0, 0.15, 0.3]

BASE = dict(
    n_agents=1, n_targets=1, ragged=0, window=10, episode_len=200, n_actions=5,
    gn_iters=0, dt=1.0, area=2000.0, agent_speed=1.0, spawn_agent_radius=200.0,
    action_dpsi=ACTIONS_DPSI, agent_heading_sigma=0.02, target_heading_sigma=0.1,
    target_speed_lo=0.5, target_speed_hi=0.5, range_sigma_lo=1.0, range_sigma_hi=1.0,
    det_range=math.inf, comm_range=1500.0, comm_loss_p=0.0, eps_min=10.0, eps_max=50.0,
    d_safe=10.0, guard_tau=1e-4, lost_range=450.0,
    action_mode=0, n_rudder=5, reward_mode=0, spawn_mode=0, d_follow=50.0, spawn_min=50.0,
    spawn_max=200.0, pooled=0, est_kind=0, pf_q=1.0, pf_lik_sigma=2.0,
)


def _cfg(**kw):
    c = copy.deepcopy(BASE)
    c.update(kw)
    return c


# c0: plain step, 16 envs, 1 agent x 1 target, 200 steps, 2 km area.
PLAIN = dict(name="plain", num_envs=16, steps=200, seed=0,
             env=_cfg(n_agents=1, n_targets=1, episode_len=200, area=2000.0))
# c1: plain batched step, 4096 envs, 2x2, 500 steps, 4 km area, one graph.
BATCHED = dict(name="batched", num_envs=4096, steps=500, seed=0,
               env=_cfg(n_agents=2, n_targets=2, episode_len=500, area=4000.0))
# c2: ragged batch, 65536 envs, counts uniform 1..5 each, 1000 steps.
RAGGED = dict(name="ragged", num_envs=65536, steps=1000, seed=0,
              env=_cfg(n_agents=5, n_targets=5, ragged=1, episode_len=1000, area=4000.0,
                       target_speed_lo=0.2, target_speed_hi=1.5,
                       range_sigma_lo=0.5, range_sigma_hi=3.0))
# c3: learned estimator; windows of 16 from ragged-config rollouts.
LEARNED = dict(name="learned", num_envs=65536, steps=1000, seed=0, window=16,
               train_windows=10_000_000, infer_windows=1_000_000, hidden=128,
               env=_cfg(n_agents=5, n_targets=5, ragged=1, window=16, episode_len=1000,
                        area=4000.0, target_speed_lo=0.2, target_speed_hi=1.5,
                        range_sigma_lo=0.5, range_sigma_hi=3.0))
# c4: full rollout with the attention policy, 16384 envs, 5x5, 1000 steps.
POLICY = dict(name="policy", num_envs=16384, steps=1000, seed=0, d_model=64, heads=4,
              layers=2, ffn=256,
              env=_cfg(n_agents=5, n_targets=5, window=16, episode_len=1000, area=4000.0))

# The paper's own environment (Sec. IV-A-2, IV-A-3): 30 s steps at 1 m/s; the
# rudder takes five equidistant angles in [-0.24, 0.24] rad, moves only to an
# adjacent angle per step (actions: down, keep, up), and turns the heading by
# the linear theta(gamma) that maps 0.24 rad to 1.45 rad at this speed and
# step; targets at half the agents' speed; every entity spawned 50-200 m from
# every other; 450 m detection, 1500 m communication with dropped
# broadcasts; follow reward (Eq. (2), 50 m). A window of 10 ranges spans
# 300 s and a 300 m track.
RUDDER_ANGLES = [-0.24, -0.12, 0.0, 0.12, 0.24]
THETA_PER_RUDDER = 1.45 / 0.24  # rad of heading per rad of rudder, 1 m/s, 30 s
PAPER = dict(name="paper", num_envs=16384, steps=300, seed=0,
             env=_cfg(n_agents=5, n_targets=5, ragged=1, episode_len=300, dt=30.0,
                      agent_speed=1.0, area=4000.0, action_mode=1, n_actions=3, n_rudder=5,
                      action_dpsi=[THETA_PER_RUDDER * g for g in RUDDER_ANGLES],
                      target_speed_lo=0.5, target_speed_hi=0.5, det_range=450.0,
                      comm_range=1500.0, comm_loss_p=0.1, reward_mode=1, d_follow=50.0,
                      spawn_mode=1, spawn_min=50.0, spawn_max=200.0))

# The same with pooled trackers: each agent's tracker of a target also uses
# the ranges received from the other agents (Sec. IV-A-2).
PAPER_POOLED = dict(PAPER, name="paper_pooled", env=dict(PAPER["env"], pooled=1))

# The particle-filter tracker (Sec. II; the commented-out Sec. on the
# vectorised filter motivates it for moving targets) on the ragged batch, and
# on the paper's environment where every tracker also takes the ranges
# received from the other agents. The random walk's std is about a target's
# displacement per step; the likelihood's std adds 2 m (5 m) to the range
# noise so that 64 particles on a ring of a few hundred metres do not all
# collapse onto one.
RAGGED_PF = dict(RAGGED, name="ragged_pf",
                 env=dict(RAGGED["env"], est_kind=1, pf_q=1.0, pf_lik_sigma=2.0))
PAPER_PF = dict(PAPER, name="paper_pf",
                env=dict(PAPER["env"], pooled=1, est_kind=1, pf_q=15.0, pf_lik_sigma=5.0))

CONFIGS = {c["name"]: c for c in (PLAIN, BATCHED, RAGGED, LEARNED, POLICY, PAPER,
                                  PAPER_POOLED, RAGGED_PF, PAPER_PF)}


def env_config(name: str, **overrides) -> dict:
    """A copy of a workload's environment parameters with overrides applied."""
    c = copy.deepcopy(CONFIGS[name]["env"])
    c.update(overrides)
    return c
