"""Python face of the batched tracking environment (argument marshalling only).

Every step runs in the HIP library; torch supplies device memory and the
stream. Tensors follow the paper's definitions (arXiv 2505.08222):
  obs      [K, 6]  entity tokens (dx, dy, dz, is_self, is_agent, is_target) of
                   every agent, agent-major, env by env (Sec. IV-A-2 and the
                   TransfMAPPO caption)
  obs_mask [K]     1 where the offset is known
  reward   [E]     Eq. (1) tracking reward, normalised, -1 on a crash
  done     [E]     termination at the step limit
  gstate   [A+Tt, 6] global state (x, y, z, speed, heading, is_target)
Environments are in packed order (see `order`).
"""
import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import EnvLayout, EnvOutputs, check, lib, params_from_config, ptr

DEFAULT_RECORD = ("obs", "obs_mask", "reward", "done")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Env:
    """A batch of `num_envs` independent environments on the current GPU."""

    def __init__(self, cfg: dict, num_envs: int, seed: int = 0, counts=None, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("Env needs a ROCm GPU (torch.cuda.is_available() is False)")
        L = lib()
        self.cfg = dict(cfg)
        self.device = torch.device(device)
        self.seed = int(seed)
        self._params = params_from_config(cfg)
        h = C.c_void_p()
        cbuf = None
        if counts is not None:
            cbuf = np.ascontiguousarray(counts, dtype=np.int32).reshape(2, num_envs)
        check(L.env_create(C.byref(self._params), int(num_envs), C.c_uint64(self.seed),
                           None if cbuf is None else cbuf.ctypes.data_as(C.c_void_p),
                           C.byref(h)))
        self._h = h
        lay = EnvLayout()
        check(L.env_query_layout(h, C.byref(lay)))
        self.layout = lay
        self.E, self.A, self.Tt = lay.num_envs, lay.num_agents, lay.num_targets
        self.P, self.K = lay.num_pairs, lay.num_tokens
        n1 = self.E + 1
        self.order = {k: np.zeros(self.E if k == "env_ids" else n1, np.int64)
                      for k in ("env_ids", "agent", "target", "pair", "token")}
        o = self.order
        check(L.env_get_order(h, *(o[k].ctypes.data_as(C.c_void_p)
                                   for k in ("env_ids", "agent", "target", "pair", "token"))))
        self.n_agents = np.diff(o["agent"]).astype(np.int32)
        self.n_targets = np.diff(o["target"]).astype(np.int32)
        with torch.cuda.device(self.device):
            self._ws = torch.empty(lay.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            aligned = (base + 255) & ~255
            check(L.env_bind(h, C.c_void_p(aligned), lay.workspace_bytes, _stream()))

    # ------------------------------------------------------------------ io
    def _alloc(self, record, steps):
        T = steps
        shapes = {
            "obs": ((self.K, 6), torch.float32), "obs_mask": ((self.K,), torch.uint8),
            "reward": ((self.E,), torch.float32), "done": ((self.E,), torch.uint8),
            "est": ((self.P, 2), torch.float32), "est_valid": ((self.P,), torch.uint8),
            "gstate": ((self.A + self.Tt, 6), torch.float32),
            "actions": ((self.A,), torch.int32), "ranges": ((self.P,), torch.float32),
            "err": ((self.Tt,), torch.float32),
        }
        out = {}
        for name in record:
            shp, dt = shapes[name]
            full = shp if T is None else (T, *shp)
            out[name] = torch.empty(full, dtype=dt, device=self.device)
        return out

    @staticmethod
    def _struct(out):
        s = EnvOutputs()
        for name in _lib.OUTPUT_FIELDS:
            t = out.get(name)
            setattr(s, name, None if t is None else t.data_ptr())
        return s

    # ------------------------------------------------------------------ api
    def reset(self, episode: int = 0, record=("obs", "obs_mask")) -> dict:
        out = self._alloc([r for r in record if r in ("obs", "obs_mask", "gstate")], None)
        check(lib().env_reset(self._h, C.c_uint64(episode), C.byref(self._struct(out)), _stream()))
        return out

    def step(self, actions=None, record=DEFAULT_RECORD, out=None) -> dict:
        out = self._alloc(record, None) if out is None else out
        if actions is not None:
            actions = actions.to(device=self.device, dtype=torch.int32).contiguous()
            assert actions.numel() == self.A
        check(lib().env_step(self._h, ptr(actions), C.byref(self._struct(out)), _stream()))
        return out

    def rollout(self, T: int, actions=None, record=DEFAULT_RECORD, out=None) -> dict:
        out = self._alloc(record, T) if out is None else out
        if actions is not None:
            actions = actions.to(device=self.device, dtype=torch.int32).contiguous()
            assert actions.numel() == T * self.A
        check(lib().env_rollout(self._h, int(T), ptr(actions), C.byref(self._struct(out)),
                                _stream()))
        return out

    def capture_graph(self, T: int, episode: int = 0, record=DEFAULT_RECORD):
        """Capture reset + T-step rollout + metrics as one HIP graph."""
        self._graph_out = self._alloc(record, T)
        self._graph_metrics = torch.zeros(8, dtype=torch.float64, device=self.device)
        torch.cuda.current_stream().synchronize()
        # capture needs a non-legacy stream; replays go to the caller's stream
        side = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(side):
            check(lib().env_graph_capture(self._h, C.c_uint64(episode), int(T),
                                          C.byref(self._struct(self._graph_out)),
                                          ptr(self._graph_metrics), _stream()))
        self._capture_stream = side
        return self._graph_out, self._graph_metrics

    def launch_graph(self):
        check(lib().env_graph_launch(self._h, _stream()))

    def metrics(self) -> torch.Tensor:
        """[reward_sum, err_sum, err_sq_sum, err_count, crash_steps, lost_targets,
        env_steps, agent_steps] since the last reset."""
        m = torch.zeros(8, dtype=torch.float64, device=self.device)
        check(lib().env_metrics(self._h, ptr(m), _stream()))
        return m

    def status(self) -> int:
        flags = C.c_uint32()
        check(lib().env_status(self._h, C.byref(flags), _stream()))
        return int(flags.value)

    def state(self):
        a = torch.empty((self.A, 3), dtype=torch.float32, device=self.device)
        t = torch.empty((self.Tt, 4), dtype=torch.float32, device=self.device)
        check(lib().env_get_state(self._h, ptr(a), ptr(t), _stream()))
        return a, t

    def pf_state(self):
        """Particle-filter state (est_kind 1): particles [P, 64, 2] and the
        belief flags [P] as after the last step."""
        from ._lib import PF_PARTICLES
        xy = torch.empty((self.P, PF_PARTICLES, 2), dtype=torch.float32, device=self.device)
        b = torch.empty(self.P, dtype=torch.uint8, device=self.device)
        check(lib().env_pf_state(self._h, ptr(xy), ptr(b), _stream()))
        return xy, b

    def pf_update(self):
        """One more filter update with the last step's ranges (est_kind 1)."""
        check(lib().env_pf_update(self._h, _stream()))

    def set_mapping(self, lanes_per_agent: int, waves_per_block: int = 1):
        check(lib().env_set_mapping(self._h, int(lanes_per_agent), int(waves_per_block)))

    def get_mapping(self):
        g, w = C.c_int32(), C.c_int32()
        check(lib().env_get_mapping(self._h, C.byref(g), C.byref(w)))
        return g.value, w.value

    def set_schedule(self, chunk_steps: int):
        """-1 static, 0 automatic, > 0 dynamic with chunks of that many steps."""
        check(lib().env_set_schedule(self._h, int(chunk_steps)))

    def get_schedule(self) -> int:
        c = C.c_int32()
        check(lib().env_get_schedule(self._h, C.byref(c)))
        return c.value

    def autotune(self, probe_steps: int = 20, record=DEFAULT_RECORD, cache_path=None):
        out = self._alloc(record, probe_steps)
        check(lib().env_autotune(self._h, int(probe_steps), C.byref(self._struct(out)),
                                 None if cache_path is None else str(cache_path).encode(),
                                 _stream()))
        return self.get_mapping()

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().env_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def est_exact(win: torch.Tensor, gn_iters: int = 0, tau: float = 1e-4, accum: str = "fp64"):
    """Batched range-only estimator over windows win [N, W, 3] = (ax, ay, r)."""
    win = win.contiguous()
    assert win.dtype == torch.float32 and win.dim() == 3 and win.shape[2] == 3
    N, W, _ = win.shape
    out = torch.empty((N, 2), dtype=torch.float32, device=win.device)
    valid = torch.empty((N,), dtype=torch.uint8, device=win.device)
    check(lib().est_exact(ptr(win), N, W, gn_iters, tau, 0 if accum == "fp64" else 1, ptr(out),
                          ptr(valid), _stream()))
    return out, valid


def rng_philox(ctr: torch.Tensor, seed: int):
    """Philox4x32-10 words, uniforms and Box-Muller normals of counters [n, 4]."""
    ctr = ctr.to(torch.int32).contiguous()
    n = ctr.shape[0]
    words = torch.empty((n, 4), dtype=torch.int32, device=ctr.device)
    u = torch.empty((n, 4), dtype=torch.float32, device=ctr.device)
    z = torch.empty((n, 4), dtype=torch.float32, device=ctr.device)
    check(lib().rng_philox(ptr(ctr), n, C.c_uint64(seed), ptr(words), ptr(u), ptr(z), _stream()))
    return words, u, z
