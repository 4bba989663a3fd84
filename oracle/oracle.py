"""ctypes binding of the FP64 C oracle (liblrauv_oracle.so).

TEST INFRASTRUCTURE ONLY. Parameters arrive as a plain dict of values (the
same dict a test also hands to the GPU library); nothing here imports the
product package.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblrauv_oracle.so")
_lib = None


class OrcParams(C.Structure):
    _fields_ = [
        ("n_agents", C.c_int32), ("n_targets", C.c_int32), ("ragged", C.c_int32),
        ("window", C.c_int32), ("episode_len", C.c_int32), ("n_actions", C.c_int32),
        ("gn_iters", C.c_int32), ("pad_", C.c_int32),
        ("dt", C.c_double), ("area", C.c_double), ("agent_speed", C.c_double),
        ("spawn_agent_radius", C.c_double), ("action_dpsi", C.c_double * 8),
        ("agent_heading_sigma", C.c_double), ("target_heading_sigma", C.c_double),
        ("target_speed_lo", C.c_double), ("target_speed_hi", C.c_double),
        ("range_sigma_lo", C.c_double), ("range_sigma_hi", C.c_double),
        ("det_range", C.c_double), ("comm_range", C.c_double), ("comm_loss_p", C.c_double),
        ("eps_min", C.c_double), ("eps_max", C.c_double), ("d_safe", C.c_double),
        ("guard_tau", C.c_double), ("lost_range", C.c_double),
        ("action_mode", C.c_int32), ("n_rudder", C.c_int32), ("reward_mode", C.c_int32),
        ("spawn_mode", C.c_int32), ("d_follow", C.c_double), ("spawn_min", C.c_double),
        ("spawn_max", C.c_double), ("pooled", C.c_int32), ("pad2_", C.c_int32),
        ("est_kind", C.c_int32), ("pad3_", C.c_int32), ("pf_q", C.c_double),
        ("pf_lik_sigma", C.c_double),
    ]

PF_N = 64  # particles per tracker (ORC_PF_N)


_TRAJ_FIELDS = [
    ("init_agent", C.c_double), ("init_target", C.c_double), ("sigma_r", C.c_double),
    ("init_obs", C.c_double), ("init_mask", C.c_uint8),
    ("agent", C.c_double), ("target", C.c_double), ("ranges", C.c_double),
    ("est", C.c_double), ("est_valid", C.c_uint8), ("est_fresh", C.c_uint8),
    ("sens", C.c_double), ("err", C.c_double), ("reward", C.c_double),
    ("crash", C.c_uint8), ("done", C.c_uint8), ("obs", C.c_double),
    ("obs_mask", C.c_uint8), ("actions", C.c_int32), ("env_metrics", C.c_double),
]


class OrcTraj(C.Structure):
    _fields_ = [(n, C.POINTER(t)) for n, t in _TRAJ_FIELDS]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER
        L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_philox_bulk.argtypes = [C.c_int64, P(C.c_uint32), C.c_uint64, P(C.c_uint32)]
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_normal2.argtypes = [C.c_uint32, C.c_uint32, P(C.c_double), P(C.c_double)]
        L.orc_choice.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_choice.restype = C.c_uint32
        L.orc_env_counts.argtypes = [P(OrcParams), C.c_uint64, C.c_int64, P(C.c_int64),
                                     P(C.c_int32), P(C.c_int32)]
        L.orc_ls_estimate.argtypes = [C.c_int, P(C.c_double), P(C.c_double), P(C.c_double),
                                      C.c_int, C.c_double, P(C.c_double), P(C.c_double)]
        L.orc_ls_estimate.restype = C.c_int
        L.orc_ls_estimate_sens.argtypes = [C.c_int, P(C.c_double), P(C.c_double), P(C.c_double),
                                           C.c_int, C.c_double, P(C.c_double), P(C.c_double),
                                           P(C.c_double)]
        L.orc_ls_estimate_sens.restype = C.c_int
        L.orc_ls_batch.argtypes = [C.c_int64, C.c_int, P(C.c_double), C.c_int, C.c_double,
                                   P(C.c_double), P(C.c_uint8), C.c_int]
        L.orc_tracking_reward.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_tracking_reward.restype = C.c_double
        L.orc_follow_reward.argtypes = [C.c_double, C.c_double]
        L.orc_follow_reward.restype = C.c_double
        L.orc_spawn_pairwise.argtypes = [P(OrcParams), C.c_uint64, C.c_uint64, C.c_uint32,
                                         C.c_int, C.c_int, P(C.c_double), P(C.c_double)]
        L.orc_spawn_pairwise.restype = C.c_int
        L.orc_rollout.argtypes = [P(OrcParams), C.c_uint64, C.c_uint64, C.c_int64, P(C.c_int64),
                                  P(C.c_int32), P(C.c_int32), C.c_int32, P(C.c_int32),
                                  P(OrcTraj), C.c_int]
        L.orc_rollout.restype = C.c_int
        L.orc_pf_update.argtypes = [C.c_int, P(C.c_double), P(C.c_double), C.c_int, C.c_int,
                                    P(C.c_double), P(C.c_double), P(C.c_double), C.c_double,
                                    C.c_double, P(C.c_uint32), P(C.c_uint32), C.c_uint32,
                                    P(C.c_double), P(C.c_double), P(C.c_int32)]
        L.orc_pf_update.restype = C.c_int
        _register_learned(L)
        _lib = L
    return _lib


def _register_learned(L):
    """Declare the learned-part entry points when the library has them."""
    P, D, I64 = C.POINTER, C.c_double, C.c_int64
    if hasattr(L, "orc_mlp_forward"):
        L.orc_mlp_num_params.restype = I64
        L.orc_window_features.argtypes = [I64, C.c_int, P(D), P(D), P(D)]
        L.orc_mlp_target.argtypes = [I64, P(D), P(D), P(D)]
        L.orc_mlp_decode.argtypes = [I64, P(D), P(D), P(D)]
        L.orc_mlp_forward.argtypes = [I64, P(D), P(D), P(D)]
        L.orc_mlp_backward.argtypes = [I64, P(D), P(D), P(D), P(D), P(D)]
        L.orc_mlp_backward.restype = D
        L.orc_adam_step.argtypes = [I64, P(D), P(D), P(D), P(D), I64, D, D, D, D]
        L.orc_mlp_residual_rms.argtypes = [I64, C.c_int, P(D), P(D), P(D)]
        L.orc_range_refine.argtypes = [I64, C.c_int, P(D), P(D), P(D), C.c_int, P(D)]
    if hasattr(L, "orc_policy_forward"):
        L.orc_policy_num_params.restype = I64
        L.orc_policy_forward.argtypes = [I64, C.c_int, P(D), P(C.c_uint8), P(D), P(D)]
        L.orc_policy_forward_rec.argtypes = [I64, C.c_int, P(D), P(C.c_uint8), P(D), P(D), P(D),
                                             P(D)]
        L.orc_policy_backward.argtypes = [I64, C.c_int, P(D), P(C.c_uint8), P(D), P(D), P(D)]
        L.orc_policy_backward_rec.argtypes = [I64, C.c_int, P(D), P(C.c_uint8), P(D), P(D), P(D),
                                              P(D), P(D), P(D)]
        L.orc_policy_sample.argtypes = [P(D), C.c_int, D]
        L.orc_policy_sample.restype = C.c_int


def _p(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def make_params(cfg: dict) -> OrcParams:
    p = OrcParams()
    for name, _ in OrcParams._fields_:
        if name in ("pad_", "pad2_", "pad3_"):
            continue
        if name == "action_dpsi":
            vals = list(cfg["action_dpsi"]) + [0.0] * (8 - len(cfg["action_dpsi"]))
            p.action_dpsi = (C.c_double * 8)(*vals)
            continue
        setattr(p, name, cfg[name])
    return p


# ---------------------------------------------------------------- RNG pieces
def philox(ctr: np.ndarray, seed: int) -> np.ndarray:
    """Philox4x32-10 of counters [n,4] (uint32) with key = (seed lo, seed hi)."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().orc_philox_bulk(ctr.shape[0], _p(ctr, C.c_uint32), C.c_uint64(seed), _p(out, C.c_uint32))
    return out


def philox_key(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def u01(x: int) -> float:
    return lib().orc_u01(C.c_uint32(x))


def normal2(x0: int, x1: int):
    z0, z1 = C.c_double(), C.c_double()
    lib().orc_normal2(x0, x1, C.byref(z0), C.byref(z1))
    return z0.value, z1.value


def choice(x: int, n: int) -> int:
    return int(lib().orc_choice(x, n))


def env_counts(cfg: dict, seed: int, env_ids) -> tuple:
    ids = np.ascontiguousarray(env_ids, dtype=np.int64)
    na = np.empty(ids.shape[0], np.int32)
    nt = np.empty(ids.shape[0], np.int32)
    p = make_params(cfg)
    lib().orc_env_counts(C.byref(p), seed, ids.shape[0], _p(ids, C.c_int64), _p(na, C.c_int32),
                         _p(nt, C.c_int32))
    return na, nt


# ---------------------------------------------------------------- estimator
def ls_estimate(ax, ay, r, gn_iters=0, tau=1e-4, with_sens=False):
    ax = np.ascontiguousarray(ax, np.float64)
    ay = np.ascontiguousarray(ay, np.float64)
    r = np.ascontiguousarray(r, np.float64)
    px, py, s = C.c_double(), C.c_double(), C.c_double()
    if with_sens:
        ok = lib().orc_ls_estimate_sens(len(ax), _p(ax, C.c_double), _p(ay, C.c_double),
                                        _p(r, C.c_double), gn_iters, tau, C.byref(px),
                                        C.byref(py), C.byref(s))
        return (bool(ok), px.value, py.value, s.value)
    ok = lib().orc_ls_estimate(len(ax), _p(ax, C.c_double), _p(ay, C.c_double),
                               _p(r, C.c_double), gn_iters, tau, C.byref(px), C.byref(py))
    return (bool(ok), px.value, py.value)


def ls_batch(win: np.ndarray, gn_iters=0, tau=1e-4, n_threads=1):
    """win [N][W][3] = (ax, ay, r); r NaN marks a missing entry."""
    win = np.ascontiguousarray(win, np.float64)
    N, W, _ = win.shape
    out = np.zeros((N, 2), np.float64)
    valid = np.zeros(N, np.uint8)
    lib().orc_ls_batch(N, W, _p(win, C.c_double), gn_iters, tau, _p(out, C.c_double),
                       _p(valid, C.c_uint8), n_threads)
    return out, valid


def tracking_reward(e: float, eps_min=10.0, eps_max=50.0) -> float:
    return lib().orc_tracking_reward(e, eps_min, eps_max)


def follow_reward(d: float, d_follow=50.0) -> float:
    return lib().orc_follow_reward(d, d_follow)


def spawn_pairwise(cfg: dict, seed: int, episode: int, env_id: int, n_agents: int,
                   n_targets: int):
    """Pairwise spawn of one env: (x [n], y [n], status 0 or -1)."""
    n = n_agents + n_targets
    x = np.zeros(n)
    y = np.zeros(n)
    p = make_params(cfg)
    k = lib().orc_spawn_pairwise(C.byref(p), seed, episode, env_id, n_agents, n_targets,
                                 _p(x, C.c_double), _p(y, C.c_double))
    return x, y, int(k)


# ---------------------------------------------------------------- particle filter
PURPOSE_PF = 7
PURPOSE_PF_SEED = 8
ENT_PF_OFFSET = 2048


class PfWords:
    """Random inputs of one filter update: zw [n][2] (normal words of each
    particle), uw [n] (seeding-angle words), uoff (resampling-offset word)."""

    def __init__(self, zw, uw, uoff):
        self.zw = np.ascontiguousarray(zw, np.uint32).reshape(-1, 2)
        self.uw = np.ascontiguousarray(uw, np.uint32).reshape(-1)
        self.uoff = int(uoff)


def pf_words(seed: int, episode: int, t: int, env_id: int, agent: int, target: int,
             n: int = PF_N) -> PfWords:
    """The words tracker (agent, target) of env `env_id` draws at step t: one
    Philox block per particle pair h at (t, env, (8 agent + target) n/2 + h,
    7 | episode << 4) (words 0, 1: particle 2h's normals; 2, 3: 2h + 1's), the
    same counter with purpose 8 for the seeding angles (words 0 and 2), and
    word 0 of (t, env, 2048 + 8 agent + target, 7 | episode << 4) for the
    resampling offset."""
    code = 8 * agent + target
    ctr = np.zeros((n // 2, 4), np.uint32)
    ctr[:, 0] = t
    ctr[:, 1] = env_id
    ctr[:, 2] = code * (n // 2) + np.arange(n // 2)
    ctr[:, 3] = (episode << 4) | PURPOSE_PF
    z = philox(ctr, seed)
    ctr[:, 3] = (episode << 4) | PURPOSE_PF_SEED
    s = philox(ctr, seed)
    off = philox(np.array([[t, env_id, ENT_PF_OFFSET + code, (episode << 4) | PURPOSE_PF]],
                          np.uint32), seed)
    return PfWords(z.reshape(n, 2), s[:, [0, 2]].reshape(n), off[0, 0])


def pf_update(px, py, init: bool, rows, sigma_l: float, q: float, words: PfWords):
    """One particle-filter update (orc_pf_update). rows [m][3] = (ax, ay, r).
    Returns (ok, px, py, (ex, ey), src) with new particle arrays."""
    px = np.array(px, np.float64)
    py = np.array(py, np.float64)
    n = px.shape[0]
    rows = np.ascontiguousarray(np.asarray(rows, np.float64).reshape(-1, 3))
    ax = np.ascontiguousarray(rows[:, 0])
    ay = np.ascontiguousarray(rows[:, 1])
    r = np.ascontiguousarray(rows[:, 2])
    assert words.zw.shape[0] == n and words.uw.shape[0] == n
    src = np.empty(n, np.int32)
    ex, ey = C.c_double(), C.c_double()
    ok = lib().orc_pf_update(n, _p(px, C.c_double), _p(py, C.c_double), int(bool(init)),
                             rows.shape[0], _p(ax, C.c_double), _p(ay, C.c_double),
                             _p(r, C.c_double), sigma_l, q, _p(words.zw, C.c_uint32),
                             _p(words.uw, C.c_uint32), C.c_uint32(words.uoff), C.byref(ex),
                             C.byref(ey), _p(src, C.c_int32))
    return bool(ok), px, py, (ex.value, ey.value), src


# ---------------------------------------------------------------- rollout
ALL_RECORDS = ("init_agent", "init_target", "sigma_r", "init_obs", "init_mask", "agent",
               "target", "ranges", "est", "est_valid", "est_fresh", "sens", "err", "reward",
               "crash", "done", "obs", "obs_mask", "actions", "env_metrics")


def rollout(cfg: dict, env_ids, n_agents, n_targets, seed: int, T: int, episode: int = 0,
            actions=None, records=ALL_RECORDS, n_threads: int = 1) -> dict:
    """Reset then T steps of the selected envs (global ids `env_ids`)."""
    ids = np.ascontiguousarray(env_ids, np.int64)
    na = np.ascontiguousarray(n_agents, np.int32)
    nt = np.ascontiguousarray(n_targets, np.int32)
    E = ids.shape[0]
    A, Tt = int(na.sum()), int(nt.sum())
    P = int((na.astype(np.int64) * nt).sum())
    K = int((na.astype(np.int64) * (na + nt)).sum())
    shapes = {
        "init_agent": ((A, 3), np.float64), "init_target": ((Tt, 4), np.float64),
        "sigma_r": ((E,), np.float64), "init_obs": ((K, 6), np.float64),
        "init_mask": ((K,), np.uint8),
        "agent": ((T, A, 3), np.float64), "target": ((T, Tt, 4), np.float64),
        "ranges": ((T, P), np.float64), "est": ((T, P, 2), np.float64),
        "est_valid": ((T, P), np.uint8), "est_fresh": ((T, P), np.uint8),
        "sens": ((T, P), np.float64), "err": ((T, Tt), np.float64),
        "reward": ((T, E), np.float64), "crash": ((T, E), np.uint8),
        "done": ((T, E), np.uint8), "obs": ((T, K, 6), np.float64),
        "obs_mask": ((T, K), np.uint8), "actions": ((T, A), np.int32),
        "env_metrics": ((E, 6), np.float64),
    }
    if "init_obs" in records and "init_mask" not in records:
        records = tuple(records) + ("init_mask",)
    traj = OrcTraj()
    out = {}
    ctmap = dict(_TRAJ_FIELDS)
    for name in records:
        shp, dt = shapes[name]
        arr = np.zeros(shp, dt)
        out[name] = arr
        setattr(traj, name, _p(arr, ctmap[name]))
    act_p = None
    if actions is not None:
        actions = np.ascontiguousarray(actions, np.int32).reshape(T, A)
        act_p = _p(actions, C.c_int32)
    p = make_params(cfg)
    rc = lib().orc_rollout(C.byref(p), C.c_uint64(seed), C.c_uint64(episode), E,
                           _p(ids, C.c_int64), _p(na, C.c_int32), _p(nt, C.c_int32), T, act_p,
                           C.byref(traj), n_threads)
    if rc != 0:
        raise ValueError(f"oracle rollout rejected its arguments (rc={rc})")
    out["csr"] = {
        "agent": np.concatenate([[0], np.cumsum(na)]),
        "target": np.concatenate([[0], np.cumsum(nt)]),
        "pair": np.concatenate([[0], np.cumsum(na.astype(np.int64) * nt)]),
        "token": np.concatenate([[0], np.cumsum(na.astype(np.int64) * (na + nt))]),
    }
    return out


# ---------------------------------------------------------------- learned part
def mlp_num_params() -> int:
    return int(lib().orc_mlp_num_params())


def window_features(win: np.ndarray):
    """win [N, W, 3] -> features [N, 64], frame [N, 5]."""
    win = np.ascontiguousarray(win, np.float64)
    N, W, _ = win.shape
    feat = np.zeros((N, 64))
    frame = np.zeros((N, 5))
    lib().orc_window_features(N, W, _p(win, C.c_double), _p(feat, C.c_double),
                              _p(frame, C.c_double))
    return feat, frame


def mlp_target(frame, p):
    frame = np.ascontiguousarray(frame, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    y = np.zeros((frame.shape[0], 2))
    lib().orc_mlp_target(frame.shape[0], _p(frame, C.c_double), _p(p, C.c_double),
                         _p(y, C.c_double))
    return y


def mlp_decode(frame, y):
    frame = np.ascontiguousarray(frame, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    p = np.zeros((frame.shape[0], 2))
    lib().orc_mlp_decode(frame.shape[0], _p(frame, C.c_double), _p(y, C.c_double),
                         _p(p, C.c_double))
    return p


def mlp_forward(x, params):
    x = np.ascontiguousarray(x, np.float64)
    params = np.ascontiguousarray(params, np.float64)
    y = np.zeros((x.shape[0], 2))
    lib().orc_mlp_forward(x.shape[0], _p(x, C.c_double), _p(params, C.c_double),
                          _p(y, C.c_double))
    return y


def mlp_backward(x, target, params):
    """(loss, grad, y) of the mean-squared loss."""
    x = np.ascontiguousarray(x, np.float64)
    target = np.ascontiguousarray(target, np.float64)
    params = np.ascontiguousarray(params, np.float64)
    grad = np.zeros_like(params)
    y = np.zeros((x.shape[0], 2))
    loss = lib().orc_mlp_backward(x.shape[0], _p(x, C.c_double), _p(target, C.c_double),
                                  _p(params, C.c_double), _p(grad, C.c_double), _p(y, C.c_double))
    return loss, grad, y


def adam_step(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In place on float64 arrays."""
    lib().orc_adam_step(params.shape[0], _p(params, C.c_double), _p(grad, C.c_double),
                        _p(m, C.c_double), _p(v, C.c_double), step, lr, beta1, beta2, eps)


def range_refine(win, centre, p, iters=3):
    """The estimate moved along its bearing from `centre` to the distance that
    best fits the window's ranges (learned estimator decode step)."""
    win = np.ascontiguousarray(win, np.float64)
    centre = np.ascontiguousarray(centre, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    out = np.zeros_like(p)
    lib().orc_range_refine(p.shape[0], win.shape[1], _p(win, C.c_double), _p(centre, C.c_double),
                           _p(p, C.c_double), int(iters), _p(out, C.c_double))
    return out


def residual_rms(win, p):
    win = np.ascontiguousarray(win, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    N, W, _ = win.shape
    out = np.zeros(N)
    lib().orc_mlp_residual_rms(N, W, _p(win, C.c_double), _p(p, C.c_double), _p(out, C.c_double))
    return out


# ---------------------------------------------------------------- attention policy
def policy_num_params() -> int:
    return int(lib().orc_policy_num_params())


def policy_forward(tokens, mask, params):
    """tokens [A, n_tok, 6], mask [A, n_tok] -> logits [A, 8]."""
    tokens = np.ascontiguousarray(tokens, np.float64)
    mask = np.ascontiguousarray(mask, np.uint8)
    params = np.ascontiguousarray(params, np.float64)
    A, n_tok, _ = tokens.shape
    out = np.zeros((A, 8))
    lib().orc_policy_forward(A, n_tok, _p(tokens, C.c_double), _p(mask, C.c_uint8),
                             _p(params, C.c_double), _p(out, C.c_double))
    return out


def policy_forward_rec(tokens, mask, hidden, params):
    """The recurrent form: tokens [A, n_obs, 6], mask [A, n_obs], hidden
    [A, 64] or None (zeros) -> (logits [A, 8], next hidden [A, 64])."""
    tokens = np.ascontiguousarray(tokens, np.float64)
    mask = np.ascontiguousarray(mask, np.uint8)
    params = np.ascontiguousarray(params, np.float64)
    A, n_obs, _ = tokens.shape
    hin = None if hidden is None else np.ascontiguousarray(hidden, np.float64)
    out = np.zeros((A, 8))
    hout = np.zeros((A, 64))
    lib().orc_policy_forward_rec(A, n_obs, _p(tokens, C.c_double), _p(mask, C.c_uint8),
                                 None if hin is None else _p(hin, C.c_double),
                                 _p(params, C.c_double), _p(out, C.c_double),
                                 _p(hout, C.c_double))
    return out, hout


def policy_backward(tokens, mask, params, dlogits):
    """Gradient of sum_a dlogits[a] . logits[a] in every parameter (plain
    form) -> [P]."""
    tokens = np.ascontiguousarray(tokens, np.float64)
    mask = np.ascontiguousarray(mask, np.uint8)
    params = np.ascontiguousarray(params, np.float64)
    dl = np.ascontiguousarray(dlogits, np.float64).reshape(tokens.shape[0], 8)
    g = np.zeros(params.size)
    lib().orc_policy_backward(tokens.shape[0], tokens.shape[1], _p(tokens, C.c_double),
                              _p(mask, C.c_uint8), _p(params, C.c_double), _p(dl, C.c_double),
                              _p(g, C.c_double))
    return g


def policy_backward_rec(tokens, mask, hidden, params, dlogits, dnext=None):
    """The recurrent form -> (parameter gradient [P], gradient at the carried
    state [A, 64]); dnext [A, 64] (or None) is the loss gradient at the state
    this step passes on."""
    tokens = np.ascontiguousarray(tokens, np.float64)
    mask = np.ascontiguousarray(mask, np.uint8)
    params = np.ascontiguousarray(params, np.float64)
    A, n_obs, _ = tokens.shape
    dl = np.ascontiguousarray(dlogits, np.float64).reshape(A, 8)
    hin = None if hidden is None else np.ascontiguousarray(hidden, np.float64)
    dn = None if dnext is None else np.ascontiguousarray(dnext, np.float64).reshape(A, 64)
    g = np.zeros(params.size)
    dh = np.zeros((A, 64))
    lib().orc_policy_backward_rec(A, n_obs, _p(tokens, C.c_double), _p(mask, C.c_uint8),
                                  None if hin is None else _p(hin, C.c_double),
                                  _p(params, C.c_double), _p(dl, C.c_double),
                                  None if dn is None else _p(dn, C.c_double), _p(g, C.c_double),
                                  _p(dh, C.c_double))
    return g, dh


def policy_bptt(tokens_seq, masks_seq, params, dlogits_seq):
    """Gradient of sum_t dlogits_seq[t] . logits_t over a sequence of T steps
    of the recurrent form started from zeros (logits_t from the state the
    previous step passed on): the forward chain, then the steps' reverse
    passes in reverse order, each handing the gradient at its input state to
    the step before. tokens_seq [T][A][n_obs][6], masks_seq [T][A][n_obs],
    dlogits_seq [T][A][8] -> gradient [P]."""
    T = len(tokens_seq)
    states = [None]
    for t in range(T):
        _, h = policy_forward_rec(tokens_seq[t], masks_seq[t], states[-1], params)
        states.append(h)
    grad = np.zeros(np.asarray(params).size)
    dnext = None
    for t in range(T - 1, -1, -1):
        g, dh = policy_backward_rec(tokens_seq[t], masks_seq[t], states[t], params,
                                    dlogits_seq[t], dnext)
        grad += g
        dnext = dh
    return grad


def policy_sample(logits, n, u) -> int:
    lg = np.ascontiguousarray(logits, np.float64)
    return int(lib().orc_policy_sample(_p(lg, C.c_double), n, u))
