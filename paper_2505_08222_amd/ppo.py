"""The learner's forward half (argument marshalling only): critic values of
global states, generalised advantage estimation and the clipped PPO
objective (MAPPO, Sec. III-B; TransformerCritic, Sec. IV-B-1). Every step
runs in the HIP library."""
import ctypes as C

import torch

from ._lib import check, lib, ptr


def _l():
    L = lib()
    if not getattr(L, "_ppo_registered", False):
        V, I32, I64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_float
        L.critic_workspace_bytes.argtypes = [I64, I32, I32]
        L.critic_workspace_bytes.restype = I64
        L.critic_forward.argtypes = [V, I64, I32, I32, F, V, V, V, I64, V]
        L.critic_forward.restype = C.c_int
        L.ppo_gae.argtypes = [V, V, V, I32, I64, F, F, V, V, V]
        L.ppo_gae.restype = C.c_int
        L.ppo_workspace_bytes.argtypes = []
        L.ppo_workspace_bytes.restype = I64
        L.ppo_objective.argtypes = [V, V, V, V, V, V, I32, I64, I32, I32, F, V, V, V, V, I64, V]
        L.ppo_objective.restype = C.c_int
        L._ppo_registered = True
    return L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def critic_forward(gstate, n_agents: int, n_targets: int, params, pos_scale: float = 1000.0):
    """gstate [N, n_agents + n_targets, 6] (or the rollout's [T, E*M, 6]) ->
    values [N]."""
    M = n_agents + n_targets
    g = gstate.reshape(-1, M, 6).contiguous()
    N = g.shape[0]
    L = _l()
    n = L.critic_workspace_bytes(N, n_agents, n_targets)
    buf = torch.empty(n + 256, dtype=torch.uint8, device=g.device)
    w = (buf.data_ptr() + 255) & ~255
    out = torch.empty(N, dtype=torch.float32, device=g.device)
    check(L.critic_forward(ptr(g), N, n_agents, n_targets, pos_scale, ptr(params), ptr(out),
                           C.c_void_p(w), n, _stream()))
    return out


def gae(rewards, dones, values, gamma: float, lam: float):
    """rewards [T, E], dones [T, E] (uint8), values [T + 1, E] -> (adv, ret)."""
    T, E = rewards.shape
    adv = torch.empty_like(rewards)
    ret = torch.empty_like(rewards)
    check(_l().ppo_gae(ptr(rewards.contiguous()), ptr(dones.contiguous()), ptr(values.contiguous()),
                       T, E, gamma, lam, ptr(adv), ptr(ret), _stream()))
    return adv, ret


def objective(logits_new, logits_old, actions, adv, values, returns, n_agents: int,
              n_actions: int, clip_eps: float = 0.2, grads: bool = True):
    """logits [T, A, 8], actions [T, A], adv / values / returns [T, E] ->
    (out [4] float64: policy loss, value loss, entropy, clip fraction;
    dlogits [T, A, 8] or None; dvalues [T, E] or None)."""
    T, A = actions.shape
    L = _l()
    work = torch.empty(L.ppo_workspace_bytes(), dtype=torch.uint8, device=actions.device)
    out = torch.empty(4, dtype=torch.float64, device=actions.device)
    dl = torch.empty_like(logits_new) if grads else None
    dv = torch.empty_like(values) if grads else None
    check(L.ppo_objective(ptr(logits_new.contiguous()), ptr(logits_old.contiguous()),
                          ptr(actions.contiguous()), ptr(adv.contiguous()), ptr(values.contiguous()),
                          ptr(returns.contiguous()), T, A, n_agents, n_actions, clip_eps, ptr(out),
                          ptr(dl), ptr(dv), ptr(work), work.numel(), _stream()))
    return out, dl, dv
