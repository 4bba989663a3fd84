"""Curriculum hooks of TransfMAPPO (Sec. IV-B-2, Fig. 4): the stage sequence
and the parameter hand-over between stages. No arithmetic of the method
lives here; every stage runs the same GPU entry points with other
environment parameters, which the attention networks allow because they
take any number of entity tokens (Sec. IV-B-1).

Stages (readings of the paper's description):
  * pre-training: one agent, one erratic target at 0.6x its speed, the
    tracking reward (Eq. (1)), episodes of 128 steps;
  * horizon fine-tuning: the same at 256, 512 and 1024 steps;
  * two multi-agent branches from that base model, the horizon fixed at 256
    steps: "follow", n agents and n targets (n = 2..5) with the follow reward
    (Eq. (2)) and targets at 0.5x; "track", n agents (n = 2..3) and one very
    fast target at 0.8x with the tracking reward.
The actor's parameters carry over unchanged between all stages (every agent
runs a copy of the same network); the critic's are re-initialised once, at
the first multi-agent stage of each branch, and carried over after that.
Each stage runs the paper's environment (30 s steps, rudder-state actions,
450 m detection, dropped broadcasts) with fixed counts.
"""
import dataclasses

from .configs import env_config

PRETRAIN_HORIZON = 128
FINETUNE_HORIZONS = (256, 512, 1024)
MULTI_HORIZON = 256


@dataclasses.dataclass(frozen=True)
class Stage:
    name: str
    branch: str           # "single", "follow" or "track"
    n_agents: int
    n_targets: int
    episode_len: int
    reward_mode: int      # 0 tracking (Eq. (1)), 1 follow (Eq. (2))
    target_speed: float   # as a fraction of the agents' speed
    reset_critic: bool    # re-initialise the critic before this stage
    timesteps: float = None  # the paper's budget where it states one


def single_agent_stages():
    s = [Stage("pretrain", "single", 1, 1, PRETRAIN_HORIZON, 0, 0.6, False, 1e10)]
    for h in FINETUNE_HORIZONS:
        s.append(Stage(f"horizon{h}", "single", 1, 1, h, 0, 0.6, False))
    return s


def multi_agent_stages(branch: str):
    if branch == "follow":
        return [Stage(f"follow{n}v{n}", "follow", n, n, MULTI_HORIZON, 1, 0.5, n == 2)
                for n in range(2, 6)]
    if branch == "track":
        return [Stage(f"track{n}v1", "track", n, 1, MULTI_HORIZON, 0, 0.8, n == 2)
                for n in range(2, 4)]
    raise ValueError(f"unknown branch {branch!r}")


def stages(branch: str):
    """The full sequence of one branch: the single-agent stages, then the
    branch's multi-agent stages."""
    return single_agent_stages() + multi_agent_stages(branch)


def stage_env(stage: Stage, **overrides) -> dict:
    """Environment parameters of a stage (the paper's environment, fixed counts)."""
    c = env_config("paper", ragged=0, n_agents=stage.n_agents, n_targets=stage.n_targets,
                   episode_len=stage.episode_len, reward_mode=stage.reward_mode)
    v = c["agent_speed"] * stage.target_speed
    c.update(target_speed_lo=v, target_speed_hi=v)
    c.update(overrides)
    return c


def hand_over(stage: Stage, actor, critic, init_critic):
    """Parameters entering `stage`: the actor's unchanged; the critic's from
    init_critic() where the stage resets it, else unchanged."""
    return actor, (init_critic() if stage.reset_critic else critic)
