"""Seeded synthetic inputs shared by the GPU path's tests, the benchmark and the
oracle checks.

Holds no arithmetic of the method: it only draws agent tracks, target points
and noisy distances with numpy so that both sides can be fed identical
windows. The recipe mirrors the environment's workloads: an agent moving at
`spread` m per step with heading changes drawn from the five-action set plus
noise, a target 20 m - 3 km away, range noise std uniform in 0.5-3 m.
"""
import numpy as np

ACTIONS = np.array([-0.3, -0.15, 0.0, 0.15, 0.3])


def range_windows(N: int, W: int, seed: int = 0, missing: float = 0.0, spread: float = 1.0,
                  far: float = 3000.0, dtype=np.float32) -> np.ndarray:
    """Windows [N, W, 3] = (agent x, agent y, measured range); NaN = missing."""
    rng = np.random.default_rng(seed)
    psi0 = rng.uniform(-np.pi, np.pi, size=(N, 1))
    turns = ACTIONS[rng.integers(0, 5, size=(N, W))] + rng.normal(0, 0.02, size=(N, W))
    psi = psi0 + np.cumsum(turns, axis=1)
    start = rng.uniform(-1500, 1500, size=(N, 1, 2))
    steps = spread * np.stack([np.cos(psi), np.sin(psi)], axis=-1)
    a = start + np.cumsum(steps, axis=1)
    dist = rng.uniform(20.0, far, size=(N, 1))
    ang = rng.uniform(-np.pi, np.pi, size=(N, 1))
    tgt = a[:, :1, :] + np.stack([dist * np.cos(ang), dist * np.sin(ang)], axis=-1)
    sigma = rng.uniform(0.5, 3.0, size=(N, 1))
    r = np.hypot(a[..., 0] - tgt[..., 0], a[..., 1] - tgt[..., 1]) + sigma * rng.normal(size=(N, W))
    out = np.empty((N, W, 3), dtype=dtype)
    out[..., 0] = a[..., 0]
    out[..., 1] = a[..., 1]
    out[..., 2] = r
    if missing > 0:
        out[..., 2][rng.random((N, W)) < missing] = np.nan
    return out


def window_targets(N: int, W: int, seed: int = 0, **kw) -> np.ndarray:
    """The target points used by `range_windows` with the same arguments."""
    rng = np.random.default_rng(seed)
    psi0 = rng.uniform(-np.pi, np.pi, size=(N, 1))
    turns = ACTIONS[rng.integers(0, 5, size=(N, W))] + rng.normal(0, 0.02, size=(N, W))
    psi = psi0 + np.cumsum(turns, axis=1)
    start = rng.uniform(-1500, 1500, size=(N, 1, 2))
    spread = kw.get("spread", 1.0)
    steps = spread * np.stack([np.cos(psi), np.sin(psi)], axis=-1)
    a = start + np.cumsum(steps, axis=1)
    dist = rng.uniform(20.0, kw.get("far", 3000.0), size=(N, 1))
    ang = rng.uniform(-np.pi, np.pi, size=(N, 1))
    return (a[:, :1, :] + np.stack([dist * np.cos(ang), dist * np.sin(ang)], axis=-1))[:, 0, :]


def policy_tokens(A: int, n_agents: int, n_targets: int, seed: int = 0, p_missing: float = 0.2):
    """Observation tokens [A, n_agents + n_targets, 6] and masks of the entity
    layout (self, other agents, targets): random offsets (std 300 m), one-hot
    types, random missing entries (the self token is always present)."""
    rng = np.random.default_rng(seed)
    T = n_agents + n_targets
    x = np.zeros((A, T, 6), np.float32)
    x[:, :, :2] = rng.normal(0, 300.0, (A, T, 2))
    x[:, 0, :3] = 0
    x[:, 0, 3] = 1
    x[:, 1:n_agents, 4] = 1
    x[:, n_agents:, 5] = 1
    mask = (rng.random((A, T)) > p_missing).astype(np.uint8)
    mask[:, 0] = 1
    x[..., :3] *= mask[..., None]
    return x, mask


def policy_params(n: int, seed: int = 0, scale: float = 0.08) -> np.ndarray:
    """A random FP32 parameter vector of length n (normal, std `scale`)."""
    return np.random.default_rng(seed).normal(0, scale, n).astype(np.float32)
