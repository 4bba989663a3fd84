"""ctypes declarations of the C ABI in include/mi_lrauv.h.

Loading fails loudly when libmilrauv.so has not been built: there is no
fallback implementation of any step of the path.
"""
import ctypes as C
import math
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmilrauv.so")
_lib = None

MIL_OK = 0
STATUS_BAD_ACTION = 0x1
STATUS_NONFINITE = 0x2
STATUS_SCHEDULE = 0x4


class MilError(RuntimeError):
    """A negative status returned by the library."""

    def __init__(self, code, msg):
        super().__init__(f"mi_lrauv error {code}: {msg}")
        self.code = code


class EnvParams(C.Structure):
    _fields_ = [
        ("n_agents", C.c_int32), ("n_targets", C.c_int32), ("ragged", C.c_int32),
        ("window", C.c_int32), ("episode_len", C.c_int32), ("n_actions", C.c_int32),
        ("gn_iters", C.c_int32), ("reserved0", C.c_int32),
        ("dt", C.c_float), ("area", C.c_float), ("agent_speed", C.c_float),
        ("spawn_agent_radius", C.c_float), ("action_dpsi", C.c_float * 8),
        ("agent_heading_sigma", C.c_float), ("target_heading_sigma", C.c_float),
        ("target_speed_lo", C.c_float), ("target_speed_hi", C.c_float),
        ("range_sigma_lo", C.c_float), ("range_sigma_hi", C.c_float),
        ("det_range", C.c_float), ("comm_range", C.c_float), ("comm_loss_p", C.c_float),
        ("eps_min", C.c_float), ("eps_max", C.c_float), ("d_safe", C.c_float),
        ("guard_tau", C.c_float), ("lost_range", C.c_float),
        ("action_mode", C.c_int32), ("n_rudder", C.c_int32), ("reward_mode", C.c_int32),
        ("spawn_mode", C.c_int32), ("d_follow", C.c_float), ("spawn_min", C.c_float),
        ("spawn_max", C.c_float), ("pooled", C.c_int32), ("est_kind", C.c_int32),
        ("pf_q", C.c_float), ("pf_lik_sigma", C.c_float),
    ]


PF_PARTICLES = 64  # MIL_PF_PARTICLES


class EnvLayout(C.Structure):
    _fields_ = [
        ("num_envs", C.c_int64), ("num_agents", C.c_int64), ("num_targets", C.c_int64),
        ("num_pairs", C.c_int64), ("num_tokens", C.c_int64), ("num_entities", C.c_int64),
        ("workspace_bytes", C.c_int64), ("window", C.c_int32), ("num_classes", C.c_int32),
    ]


OUTPUT_FIELDS = ("obs", "obs_mask", "reward", "done", "est", "est_valid", "gstate", "actions",
                 "ranges", "err")


class EnvOutputs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in OUTPUT_FIELDS]


def params_from_config(cfg: dict) -> EnvParams:
    p = EnvParams()
    for name, _ in EnvParams._fields_:
        if name == "reserved0":
            continue
        if name == "action_dpsi":
            vals = list(cfg["action_dpsi"]) + [0.0] * (8 - len(cfg["action_dpsi"]))
            p.action_dpsi = (C.c_float * 8)(*vals)
            continue
        v = cfg[name]
        setattr(p, name, float(v) if isinstance(v, float) or math.isinf(v) else v)
    return p


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIB_PATH)
    P, V, I32, I64, U64 = C.POINTER, C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    sig = {
        "env_create": [P(EnvParams), I64, U64, V, P(V)],
        "env_query_layout": [V, P(EnvLayout)],
        "env_get_order": [V, V, V, V, V, V],
        "env_bind": [V, V, I64, V],
        "env_reset": [V, U64, P(EnvOutputs), V],
        "env_step": [V, V, P(EnvOutputs), V],
        "env_rollout": [V, I32, V, P(EnvOutputs), V],
        "env_graph_capture": [V, U64, I32, P(EnvOutputs), V, V],
        "env_graph_launch": [V, V],
        "env_metrics": [V, V, V],
        "env_status": [V, P(C.c_uint32), V],
        "env_get_state": [V, V, V, V],
        "env_set_mapping": [V, I32, I32],
        "env_get_mapping": [V, P(I32), P(I32)],
        "env_set_schedule": [V, I32],
        "env_get_schedule": [V, P(I32)],
        "env_autotune": [V, I32, P(EnvOutputs), C.c_char_p, V],
        "env_destroy": [V],
        "est_exact": [V, I64, I32, I32, C.c_float, I32, V, V, V],
        "rng_philox": [V, I64, U64, V, V, V, V],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.env_last_error.argtypes = []
    L.env_last_error.restype = C.c_char_p
    _register_learned(L)
    _lib = L
    return L


def _register_learned(L):
    """Declare the learned-part entry points (MLP estimator, env windows)."""
    V, I32, I64, U64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_float
    table = {
        "mlp_init": [V, U64, V],
        "mlp_features": [V, I64, I32, V, V, V],
        "mlp_targets": [V, V, I64, V, V],
        "mlp_forward": [I64, V, V, V, I32, V, I64, V],
        "mlp_backward": [I64, V, V, V, V, V, V, I32, V, I64, V],
        "mlp_adam_step": [I64, V, V, V, V, F, F, F, F, I32, V],
        "mlp_train_step": [I64, V, V, V, V, V, V, F, F, F, F, I32, V, V, V, I64, V],
        "mlp_infer": [V, I64, I32, V, V, F, I32, F, V, V, V, I64, V],
        "mlp_infer_noalloc": [V, I64, I32, V, V, F, I32, F, V, V, V],
        "env_windows": [V, V, V, V, V],
        "env_pf_state": [V, V, V, V],
        "env_pf_update": [V, V],
    }
    for name, args in table.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.mlp_num_params.argtypes = []
    L.mlp_num_params.restype = I64
    L.mlp_workspace_bytes.argtypes = [I64, I32]
    L.mlp_workspace_bytes.restype = I64


def check(rc: int):
    if rc != MIL_OK:
        raise MilError(rc, lib().env_last_error().decode())
    return rc


def ptr(t):
    """Device (or host) address of a torch tensor, or None."""
    return None if t is None else C.c_void_p(t.data_ptr())
