"""Attention policy of the full-rollout workload: argument marshalling for the
policy kernels in libmilrauv.so (see include/mi_lrauv.h, "Attention policy")."""
import ctypes as C

import torch

from ._lib import EnvOutputs, check, lib, ptr
from .env import Env, _stream

_SIG = {
    "policy_init": [C.c_void_p, C.c_uint64, C.c_void_p],
    "policy_forward": [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32,
                       C.c_void_p, C.c_int64, C.c_void_p],
    "policy_forward_rec": [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                           C.c_uint32, C.c_uint32, C.c_void_p, C.c_int64, C.c_void_p],
    "env_policy_rollout": [C.c_void_p, C.c_uint64, C.c_int32, C.c_void_p, C.c_void_p, C.c_float,
                           C.c_void_p, C.POINTER(EnvOutputs), C.c_void_p, C.c_int32, C.c_void_p,
                           C.c_int64, C.c_void_p],
}
_done = False


def _l():
    global _done
    L = lib()
    if not _done:
        for k, v in _SIG.items():
            getattr(L, k).argtypes = v
            getattr(L, k).restype = C.c_int
        L.policy_num_params.restype = C.c_int64
        L.policy_workspace_bytes.argtypes = [C.c_int64, C.c_int64]
        L.policy_workspace_bytes.restype = C.c_int64
        L.env_policy_workspace_bytes.argtypes = [C.c_void_p, C.c_int32]
        L.env_policy_workspace_bytes.restype = C.c_int64
        _done = True
    return L


def num_params() -> int:
    return int(_l().policy_num_params())


def _work(A, K, device):
    n = int(_l().policy_workspace_bytes(int(A), int(K)))
    buf = torch.empty(n + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, C.c_void_p(buf.data_ptr() + off), n


def init_params(seed=0, device="cuda") -> torch.Tensor:
    p = torch.empty(num_params(), dtype=torch.float32, device=device)
    check(_l().policy_init(ptr(p), C.c_uint64(seed), _stream()))
    return p


def forward(obs, mask, params, n_tok, n_agents, n_actions=5, seed=0, t=0, episode=0):
    """obs [A * n_tok, 6], mask [A * n_tok] -> (logits [A, 8], actions [A])."""
    A = obs.shape[0] // n_tok
    logits = torch.empty((A, 8), dtype=torch.float32, device=obs.device)
    actions = torch.empty((A,), dtype=torch.int32, device=obs.device)
    buf, w, n = _work(A, A * n_tok, obs.device)
    check(_l().policy_forward(A, n_tok, n_agents, n_actions, ptr(obs.contiguous()),
                              ptr(mask.contiguous()), ptr(params), ptr(logits), ptr(actions),
                              C.c_uint64(seed), t, episode, w, n, _stream()))
    del buf
    return logits, actions


def forward_rec(obs, mask, hidden, params, n_obs, n_agents, n_actions=5, seed=0, t=0, episode=0,
                hidden_out=None):
    """The recurrent form: obs [A * n_obs, 6], mask [A * n_obs], hidden [A, 64]
    or None (zeros) -> (logits [A, 8], actions [A], next hidden [A, 64]);
    hidden_out may be `hidden` itself (updated in place)."""
    A = obs.shape[0] // n_obs
    logits = torch.empty((A, 8), dtype=torch.float32, device=obs.device)
    actions = torch.empty((A,), dtype=torch.int32, device=obs.device)
    if hidden_out is None:
        hidden_out = torch.empty((A, 64), dtype=torch.float32, device=obs.device)
    buf, w, n = _work(A, A * (n_obs + 1), obs.device)
    check(_l().policy_forward_rec(A, n_obs, n_agents, n_actions, ptr(obs.contiguous()),
                                  ptr(mask.contiguous()), ptr(hidden), ptr(params), ptr(logits),
                                  ptr(actions), ptr(hidden_out), C.c_uint64(seed), t, episode, w,
                                  n, _stream()))
    del buf
    return logits, actions, hidden_out


class PolicyRollout:
    """Closed-loop rollouts of a fixed-count Env driven by the policy; with
    `mlp_params` the learned estimator (exact fallback at k_sigma * sigma_r)
    supplies the trackers' estimates inside the loop. With `recurrent` the
    actor runs in its recurrent form; `hidden` [A, 64] holds the carried state
    (the last step's after a run)."""

    def __init__(self, env: Env, params: torch.Tensor, mlp_params: torch.Tensor = None,
                 k_sigma: float = 3.0, recurrent: bool = False):
        self.env, self.params = env, params
        self.mlp_params, self.k_sigma = mlp_params, float(k_sigma)
        self.hidden = (torch.empty((env.A, 64), dtype=torch.float32, device=env.device)
                       if recurrent else None)
        n = int(_l().env_policy_workspace_bytes(env._h, int(mlp_params is not None)))
        assert n > 0, "the env must be bound"
        self._buf = torch.empty(n + 256, dtype=torch.uint8, device=env.device)
        off = (-self._buf.data_ptr()) % 256
        self._w, self._n = C.c_void_p(self._buf.data_ptr() + off), n

    def _call(self, T, episode, out, metrics, capture):
        check(_l().env_policy_rollout(self.env._h, C.c_uint64(episode), int(T), ptr(self.params),
                                      ptr(self.mlp_params), C.c_float(self.k_sigma),
                                      ptr(self.hidden), C.byref(Env._struct(out)), ptr(metrics),
                                      int(capture),
                                      self._w, self._n, _stream()))

    def run(self, T, episode=0, record=("reward", "done"), metrics=True):
        out = self.env._alloc(record, T)
        m = torch.zeros(8, dtype=torch.float64, device=self.env.device) if metrics else None
        self._call(T, episode, out, m, 0)
        return out, m

    def capture(self, T, episode=0, record=("reward", "done")):
        self.graph_out = self.env._alloc(record, T)
        self.graph_metrics = torch.zeros(8, dtype=torch.float64, device=self.env.device)
        torch.cuda.current_stream().synchronize()
        side = torch.cuda.Stream(device=self.env.device)
        with torch.cuda.stream(side):
            self._call(T, episode, self.graph_out, self.graph_metrics, 1)
        self._side = side
        return self.graph_out, self.graph_metrics

    def launch(self):
        self.env.launch_graph()
