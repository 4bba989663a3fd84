"""CPU checks of the C-ABI library: it loads, exports every symbol declared in
include/*.h, and its host-side entry points (creation, packing, layout,
argument validation) behave as documented. No GPU compute is called."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                             text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def milib():
    from paper_2505_08222_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmilrauv.so not built")
    return _lib


def test_exports_every_declared_symbol(milib):
    L = C.CDLL(milib.LIB_PATH)
    names = _declared_functions()
    assert len(names) >= 19
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2505_08222_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="build"):
        _lib.lib()


def _create(milib, cfg, E, seed=0, counts=None):
    L = milib.lib()
    p = milib.params_from_config(cfg)
    h = C.c_void_p()
    cbuf = None if counts is None else np.ascontiguousarray(counts, np.int32)
    rc = L.env_create(C.byref(p), E, C.c_uint64(seed),
                      None if cbuf is None else cbuf.ctypes.data_as(C.c_void_p), C.byref(h))
    return rc, h


def test_create_layout_and_packing(milib, orc):
    from paper_2505_08222_amd.configs import env_config
    cfg = env_config("ragged")
    E = 5000
    rc, h = _create(milib, cfg, E, seed=0)
    assert rc == 0
    L = milib.lib()
    lay = milib.EnvLayout()
    assert L.env_query_layout(h, C.byref(lay)) == 0
    ids = np.zeros(E, np.int64)
    offs = [np.zeros(E + 1, np.int64) for _ in range(4)]
    assert L.env_get_order(h, ids.ctypes.data_as(C.c_void_p),
                           *(o.ctypes.data_as(C.c_void_p) for o in offs)) == 0
    na, nt = np.diff(offs[0]), np.diff(offs[1])
    # counts drawn by the library equal the oracle's, env by env
    ona, ont = orc.env_counts(cfg, 0, ids)
    np.testing.assert_array_equal(na, ona)
    np.testing.assert_array_equal(nt, ont)
    # packed by shape: each (agents, targets) class is one contiguous run
    shapes = list(zip(na, nt))
    runs = [shapes[0]] + [s for a, s in zip(shapes, shapes[1:]) if s != a]
    assert len(runs) == len(set(runs)) == lay.num_classes == 25
    assert sorted(ids) == list(range(E))
    assert lay.num_agents == na.sum() and lay.num_pairs == (na * nt).sum()
    assert lay.num_tokens == (na * (na + nt)).sum()
    assert lay.workspace_bytes > 0 and lay.workspace_bytes % 256 == 0
    L.env_destroy(h)


def test_explicit_counts_and_validation(milib):
    from paper_2505_08222_amd.configs import env_config
    cfg = env_config("ragged")
    counts = np.array([[1, 2, 3], [5, 4, 3]], np.int32)
    rc, h = _create(milib, cfg, 3, counts=counts)
    assert rc == 0
    milib.lib().env_destroy(h)
    bad = counts.copy()
    bad[0, 1] = 9
    rc, _ = _create(milib, cfg, 3, counts=bad)
    assert rc == -1
    for key, val in [("window", 2), ("window", 17), ("n_agents", 9), ("n_actions", 0),
                     ("eps_max", 5.0), ("comm_loss_p", 1.5)]:
        c = dict(cfg)
        c[key] = val
        rc, _ = _create(milib, c, 4)
        assert rc == -1, key
        assert milib.lib().env_last_error()
    rc, _ = _create(milib, cfg, 0)
    assert rc == -1


def test_calls_out_of_order_are_rejected(milib):
    from paper_2505_08222_amd.configs import env_config
    rc, h = _create(milib, env_config("plain"), 4)
    L = milib.lib()
    out = milib.EnvOutputs()
    assert L.env_step(h, None, C.byref(out), None) == -5  # not bound
    assert L.env_reset(h, 0, C.byref(out), None) == -5
    assert L.env_set_mapping(h, 3, 1) == -1
    assert L.env_set_mapping(h, 2, 4) == 0
    g, w = C.c_int32(), C.c_int32()
    L.env_get_mapping(h, C.byref(g), C.byref(w))
    assert (g.value, w.value) == (2, 4)
    assert L.env_set_schedule(h, -2) == -1
    assert L.env_set_schedule(h, 7) == 0
    sc = C.c_int32()
    assert L.env_get_schedule(h, C.byref(sc)) == 0 and sc.value == 7
    assert L.env_bind(h, C.c_void_p(0x1001), 1 << 30, None) == -3  # misaligned
    L.env_destroy(h)
    assert L.est_exact(None, 10, 2, 0, C.c_float(1e-4), 0, None, None, None) == -1


def test_noalloc_inference_rejects_oversized_batches(milib):
    """The workspace-free inference refuses more windows than its static
    scratch holds, before touching any device."""
    L = milib.lib()
    too_many = (1 << 20) + 1
    rc = L.mlp_infer_noalloc(None, too_many, 16, None, None, 3.0, 0, 1e-4, None, None, None)
    assert rc == -1
    assert b"MIL_NOALLOC_MAX_WINDOWS" in L.env_last_error()
    assert L.mlp_infer_noalloc(None, 0, 16, None, None, 3.0, 0, 1e-4, None, None, None) == 0


def test_particle_filter_parameters_and_workspace(milib):
    """est_kind 1 validates its parameters, adds the particles (P x 64 x 8
    bytes and more) to the workspace, and env_pf_state refuses an
    environment without a filter before touching any device."""
    from paper_2505_08222_amd.configs import env_config
    L = milib.lib()
    cfg = env_config("ragged")
    rc, h0 = _create(milib, cfg, 64)
    assert rc == 0
    lay0 = milib.EnvLayout()
    L.env_query_layout(h0, C.byref(lay0))
    assert L.env_pf_state(h0, None, None, None) == -1
    L.env_destroy(h0)
    rc, h1 = _create(milib, dict(cfg, est_kind=1, pf_q=1.0, pf_lik_sigma=2.0), 64)
    assert rc == 0
    lay1 = milib.EnvLayout()
    L.env_query_layout(h1, C.byref(lay1))
    assert lay1.num_pairs == lay0.num_pairs
    # particles twice (state and its autotuning snapshot) plus per-tracker words
    assert lay1.workspace_bytes - lay0.workspace_bytes >= 2 * lay1.num_pairs * 64 * 8
    L.env_destroy(h1)
    for key, val in [("est_kind", 2), ("pf_q", -1.0), ("pf_lik_sigma", float("inf"))]:
        rc, _ = _create(milib, {**cfg, "est_kind": 1, key: val}, 4)
        assert rc == -1, key
        assert milib.lib().env_last_error()


def test_learner_entry_points_validate_before_any_device_call(milib):
    """The learner's entry points reject bad sizes, flags, workspaces and
    pointers with their documented codes before touching any device (so
    this runs without a GPU)."""
    pytest.importorskip("torch")
    from paper_2505_08222_amd import ppo
    L = ppo._l()
    EINVAL, ESHAPE, EALIGN = -1, -2, -3
    assert L.policy_train_workspace_bytes(0, 5) == -1
    assert L.policy_train_workspace_bytes(4, 17) == -1
    need = L.policy_train_workspace_bytes(4, 5)
    assert need > 4 * 5 * 2 * 1024 * 4  # the tape: over 2 K floats per row
    fake = C.c_void_p(1 << 20)  # aligned, never dereferenced
    args = lambda A, nt, rec, w, n: (A, nt, rec, None, None, None, None, None, None, w, n, None)  # noqa
    assert L.policy_train_forward(*args(0, 5, 0, fake, need)) == EINVAL
    assert L.policy_train_forward(*args(4, 17, 0, fake, need)) == EINVAL
    assert L.policy_train_forward(*args(4, 1, 1, fake, need)) == EINVAL  # no room for the state
    assert L.policy_train_forward(*args(4, 5, 2, fake, need)) == EINVAL
    assert L.policy_train_forward(*args(4, 5, 0, C.c_void_p((1 << 20) + 8), need)) == EALIGN
    assert L.policy_train_forward(*args(4, 5, 0, fake, need - 256)) == ESHAPE
    assert L.policy_train_forward(*args(4, 5, 0, fake, need)) == EINVAL  # null inputs
    bw = lambda n_out, ld: L.policy_train_backward(4, 5, 0, None, None, ld, n_out, None, 0, None,  # noqa
                                                   None, fake, need, None)
    assert bw(9, 9) == EINVAL and bw(0, 8) == EINVAL and bw(5, 4) == EINVAL
    assert bw(5, 8) == EINVAL  # null parameters
    cf = lambda na, nt, s: L.critic_train_forward(None, 4, na, nt, s, 0, None, None, None, None,  # noqa
                                                  fake, 1 << 40, None)
    assert cf(8, 8, 1000.0) == EINVAL and cf(2, 2, 0.0) == EINVAL and cf(2, 2, 1000.0) == EINVAL
    assert L.head_grad(-1, None, None, 8, 5, None, fake, 1 << 20, None) == EINVAL
    assert L.head_grad(4, None, None, 8, 0, None, fake, 1 << 20, None) == EINVAL
    assert L.head_grad(4, None, None, 4, 5, None, fake, 1 << 20, None) == EINVAL
    assert L.critic_forward_rec(None, -1, 4, 2, 2, 1000.0, None, None, None, None, fake, 1 << 30,
                                None) == EINVAL
    assert L.critic_forward_rec(None, 3, 4, 2, 2, 0.0, None, None, None, None, fake, 1 << 30,
                                None) == EINVAL
    assert L.critic_forward_rec(None, 0, 4, 2, 2, 1000.0, None, None, None, None, fake, 1 << 30,
                                None) == 0  # no steps: nothing to do
    assert L.policy_forward_rec(4, 16, 1, 5, None, None, None, None, None, None, fake,
                                C.c_uint64(0), 0, 0, fake, 1 << 30, None) == EINVAL
    assert L.policy_forward_rec(4, 5, 1, 5, None, None, None, None, None, None, None,
                                C.c_uint64(0), 0, 0, fake, 1 << 30, None) == EINVAL  # no state out
    obj = lambda T, eps: L.ppo_objective(None, None, None, None, None, None, T, 4, 1, 5, eps,  # noqa
                                         None, None, None, fake, 1 << 20, None)
    assert obj(0, 0.2) == EINVAL and obj(3, 1.0) == EINVAL and obj(3, 0.2) == EINVAL
    assert L.ppo_gae(None, None, None, -1, 4, 0.99, 0.95, None, None, None) == EINVAL
    assert L.ppo_gae(None, None, None, 3, 4, 1.5, 0.95, None, None, None) == EINVAL
