"""GPU parity of the HIP environment against the FP64 oracle (MI355X).

Every test calls the HIP library through its C ABI (via the thin binding)
and compares with the oracle on the same seeds and parameters.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_08222_amd.configs import CONFIGS, env_config  # noqa: E402

from parity_util import angle_diff, compare_rollout  # noqa: E402

pytestmark = pytest.mark.gpu

ALL = ("obs", "obs_mask", "reward", "done", "est", "est_valid", "gstate", "actions", "ranges",
       "err")


def _env(cfg, E, seed=0, **kw):
    from paper_2505_08222_amd.env import Env
    return Env(cfg, E, seed=seed, **kw)


def _oracle(orc, cfg, env, packed_idx, seed, T, episode=0, actions=None):
    ids = env.order["env_ids"][packed_idx]
    return orc.rollout(cfg, ids, env.n_agents[packed_idx], env.n_targets[packed_idx], seed, T,
                       episode=episode, actions=actions)


def _np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_rng_words_and_transforms(orc):
    from paper_2505_08222_amd.env import rng_philox
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:16] = 0
    ctr[:16, 0] = np.arange(16)
    seed = 0x1234_5678_9ABC_DEF0
    words, u, z = rng_philox(torch.from_numpy(ctr.view(np.int32)).cuda(), seed)
    w = words.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(w, orc.philox(ctr, seed))
    u = u.cpu().numpy()
    want_u = np.array([[orc.u01(int(x)) for x in row] for row in w[:512]])
    np.testing.assert_array_equal(u[:512].astype(np.float64), want_u)
    z = z.cpu().numpy()
    for k in range(512):
        z0, z1 = orc.normal2(int(w[k, 0]), int(w[k, 1]))
        z2, z3 = orc.normal2(int(w[k, 2]), int(w[k, 3]))
        # native log2/sqrt/sin/cos instructions: ~2 ulp each
        np.testing.assert_allclose(z[k], [z0, z1, z2, z3], rtol=1e-5, atol=1e-5)


def test_ragged_counts_match_oracle(orc):
    cfg = env_config("ragged")
    env = _env(cfg, 4096, seed=0)
    ids = env.order["env_ids"]
    na, nt = orc.env_counts(cfg, 0, ids)
    np.testing.assert_array_equal(env.n_agents, na)
    np.testing.assert_array_equal(env.n_targets, nt)
    # packed by shape, no padding
    assert env.A == na.sum() and env.P == (na * nt).sum()
    assert sorted(ids.tolist()) == list(range(4096))


@pytest.mark.parametrize("name", ["plain", "batched_small", "ragged_small", "window16_5x5",
                                  "gauss_newton", "detection_comm_loss", "fixed_8x8",
                                  "fixed_7x6", "ragged_w3", "ragged_w7", "ragged_w12",
                                  "paper", "paper_tracking", "paper_5x5", "pooled",
                                  "pooled_paper", "pooled_8x8"])
def test_rollout_parity(orc, name):
    if name == "plain":
        c = CONFIGS["plain"]
        cfg, E, T = env_config("plain"), c["num_envs"], c["steps"]
    elif name == "batched_small":
        cfg, E, T = env_config("batched"), 96, 120
    elif name == "window16_5x5":  # the policy / learned-estimator shape: W = 16, 5 x 5
        cfg, E, T = env_config("policy", episode_len=80), 64, 80
    elif name == "gauss_newton":  # refinement path of the tracker
        cfg, E, T = env_config("ragged", episode_len=60, gn_iters=4), 120, 60
    elif name == "detection_comm_loss":  # missing ranges and dropped broadcasts
        cfg, E, T = env_config("ragged", episode_len=60, det_range=1200.0, comm_range=120.0,
                               comm_loss_p=0.3), 150, 60
    elif name == "fixed_8x8":  # the largest shape class: 8 agents x 8 targets
        cfg, E, T = env_config("batched", episode_len=60, n_agents=8, n_targets=8), 40, 60
    elif name == "fixed_7x6":
        cfg, E, T = env_config("batched", episode_len=60, n_agents=7, n_targets=6), 50, 60
    elif name == "paper":  # Sec. IV-A-2/3: 30 s steps, rudder, follow reward, 450 m, spawn
        cfg, E, T = env_config("paper", episode_len=60), 300, 60
    elif name == "paper_tracking":  # the same with the tracking reward, Eq. (1)
        cfg, E, T = env_config("paper", episode_len=60, reward_mode=0), 300, 60
    elif name == "paper_5x5":
        cfg, E, T = env_config("paper", episode_len=60, ragged=0, window=16), 64, 60
    elif name == "pooled":  # trackers also use the ranges received from other agents
        cfg, E, T = env_config("ragged", episode_len=50, pooled=1, comm_range=300.0,
                               comm_loss_p=0.2, det_range=1500.0), 200, 50
    elif name == "pooled_paper":
        cfg, E, T = env_config("paper", episode_len=50, pooled=1), 200, 50
    elif name == "pooled_8x8":  # the largest rows: 8 agents x 16 entries
        cfg, E, T = env_config("batched", episode_len=40, n_agents=8, n_targets=8, window=16,
                               pooled=1, comm_range=2000.0, comm_loss_p=0.1), 24, 40
    elif name.startswith("ragged_w"):  # other window lengths (3..16 are accepted)
        W = int(name[len("ragged_w"):])
        cfg, E, T = env_config("ragged", episode_len=50, window=W), 200, 50
    else:
        cfg, E, T = env_config("ragged", episode_len=150), 300, 150
    seed = 0
    env = _env(cfg, E, seed=seed)
    env.reset(0)
    gpu = _np(env.rollout(T, record=ALL))
    sel = np.arange(E)
    ref = _oracle(orc, cfg, env, sel, seed, T)
    rep = compare_rollout(gpu, ref, env, sel, cfg, label=name)
    print(name, rep)


def test_full_size_batched_sampled(orc):
    """The 4096-env, 500-step workload, every step recorded, checked on 24
    sampled envs."""
    c = CONFIGS["batched"]
    cfg, E, T = env_config("batched"), c["num_envs"], c["steps"]
    env = _env(cfg, E, seed=c["seed"])
    env.reset(0)
    out = env.rollout(T, record=ALL)
    rng = np.random.default_rng(1)
    sel = np.sort(np.concatenate([[0, E - 1], rng.choice(np.arange(1, E - 1), 22, replace=False)]))
    gpu = {}
    o = env.order
    for k, v in out.items():
        a = v.cpu().numpy()
        gpu[k] = a
    ref = _oracle(orc, cfg, env, sel, c["seed"], T)
    rep = compare_rollout(gpu, ref, env, sel, cfg, label="batched-full")
    print("batched-full", rep)
    del o


def test_full_size_ragged_sampled(orc):
    """The 65536-env, 1000-step ragged workload in the benchmark's launch
    configuration: final state after 999 silent steps plus the last step's
    outputs, on 40 sampled envs covering every shape class."""
    c = CONFIGS["ragged"]
    cfg, E, T = env_config("ragged"), c["num_envs"], c["steps"]
    env = _env(cfg, E, seed=c["seed"])
    env.reset(0)
    env.rollout(T - 1, record=())
    last = _np(env.step(record=ALL))
    a_state, t_state = (x.cpu().numpy() for x in env.state())
    o = env.order
    rng = np.random.default_rng(2)
    cls_first = np.flatnonzero(np.r_[True, (np.diff(env.n_agents) != 0) | (np.diff(env.n_targets) != 0)])
    sel = np.unique(np.concatenate([cls_first, rng.choice(E, 15, replace=False)]))
    ref = _oracle(orc, cfg, env, sel, c["seed"], T)
    s = cfg["area"] / 2
    for n, k in enumerate(sel):
        ga = a_state[o["agent"][k]:o["agent"][k + 1]]
        ra = ref["agent"][-1][ref["csr"]["agent"][n]:ref["csr"]["agent"][n + 1]]
        assert np.abs(ga[:, :2] - ra[:, :2]).max() <= 1e-5 * s
        assert angle_diff(ga[:, 2], ra[:, 2]).max() <= 1e-5 * np.pi
        assert (np.abs(ga[:, 2]) <= np.pi + 1e-6).all()
        gt = t_state[o["target"][k]:o["target"][k + 1]]
        rt = ref["target"][-1][ref["csr"]["target"][n]:ref["csr"]["target"][n + 1]]
        assert np.abs(gt[:, :2] - rt[:, :2]).max() <= 1e-5 * s
    # last-step outputs of the sampled envs, through the same comparison
    one = {k: (v[None] if v.ndim >= 1 else v) for k, v in last.items()}
    ref1 = {k: (v[-1:] if isinstance(v, np.ndarray) and v.ndim >= 2 and k not in
                ("init_agent", "init_target", "init_obs", "env_metrics") else v)
            for k, v in ref.items()}
    ref1["reward"] = ref["reward"][-1:]
    ref1["crash"] = ref["crash"][-1:]
    ref1["done"] = ref["done"][-1:]
    rep = compare_rollout(one, ref1, env, sel, cfg, label="ragged-full-last")
    assert (last["done"] == 1).all()
    print("ragged-full", rep)


@pytest.mark.parametrize("cfgname,E,T", [("batched", 4096, 500), ("ragged", 3000, 120),
                                         ("ragged", 65536, 12), ("batched", 262144, 12)])
def test_lean_form_matches_full_bitwise(cfgname, E, T):
    """Recording only obs, obs_mask, reward and done (the benchmark's launch
    form, compiled without the other outputs' paths) gives the same bits,
    final state and metrics as the full form that the parity tests hold to
    the oracle. The two large batches take the staged, coalesced write of
    the observation block; the small ones write directly."""
    cfg = env_config(cfgname, episode_len=T)
    lean_env = _env(cfg, E, seed=0)
    full_env = _env(cfg, E, seed=0)
    lean_env.reset(0)
    full_env.reset(0)
    lean = _np(lean_env.rollout(T, record=("obs", "obs_mask", "reward", "done")))
    full = _np(full_env.rollout(T, record=ALL))
    for k in lean:
        np.testing.assert_array_equal(lean[k], full[k], err_msg=k)
    for a, b in zip(lean_env.state(), full_env.state()):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    np.testing.assert_array_equal(lean_env.metrics().cpu().numpy(),
                                  full_env.metrics().cpu().numpy())
    assert lean_env.status() == 0


def test_step_equals_rollout_bitwise():
    cfg = env_config("ragged", episode_len=40)
    E, T = 500, 40
    a = _env(cfg, E, seed=3)
    b = _env(cfg, E, seed=3)
    a.reset(2)
    b.reset(2)
    ra = _np(a.rollout(T, record=ALL))
    steps = [_np(b.step(record=ALL)) for _ in range(T)]
    for k in ALL:
        sb = np.stack([s[k] for s in steps])
        np.testing.assert_array_equal(ra[k], sb, err_msg=k)


def test_split_rollout_bitwise():
    cfg = env_config("batched", episode_len=60)
    a = _env(cfg, 700, seed=5)
    b = _env(cfg, 700, seed=5)
    a.reset(0)
    b.reset(0)
    ra = _np(a.rollout(60, record=ALL))
    r1 = _np(b.rollout(25, record=ALL))
    r2 = _np(b.rollout(35, record=ALL))
    for k in ALL:
        np.testing.assert_array_equal(ra[k], np.concatenate([r1[k], r2[k]]), err_msg=k)


@pytest.mark.parametrize("cfgname", ["batched", "ragged"])
def test_mapping_invariance_bitwise(cfgname):
    """Every env-to-wavefront mapping the autotuner may choose gives the same
    bits."""
    cfg = env_config(cfgname, episode_len=30)
    ref = None
    for G in (1, 2):
        for w in (1, 2, 4):
            env = _env(cfg, 1000, seed=9)
            env.set_mapping(G, w)
            env.reset(0)
            out = _np(env.rollout(30, record=ALL))
            if ref is None:
                ref = out
            else:
                for k in ALL:
                    np.testing.assert_array_equal(out[k], ref[k], err_msg=f"{k} G={G} w={w}")


@pytest.mark.parametrize("chunk,G,w", [(1, 1, 1), (7, 2, 4), (50, 1, 2)])
def test_dynamic_schedule_bitwise(chunk, G, w):
    """The dynamic schedule (chunks of steps handed from one wavefront to
    another through device-coherent memory, each waiting for its group's
    previous chunk) gives the same bits, final state and metrics as the
    static one, in the lean and the full form. Small chunks make many
    wavefronts wait on a predecessor that is still running."""
    cfg = env_config("ragged", episode_len=60)
    for record in (("obs", "obs_mask", "reward", "done"), ALL):
        envs = []
        for sched in (-1, chunk):
            env = _env(cfg, 3000, seed=4)
            env.set_mapping(G, w)
            env.set_schedule(sched)
            assert env.get_schedule() == sched
            env.reset(1)
            envs.append((env, _np(env.rollout(60, record=record))))
        (a, ra), (b, rb) = envs
        for k in ra:
            np.testing.assert_array_equal(rb[k], ra[k], err_msg=f"{k} chunk={chunk}")
        for x, y in zip(a.state(), b.state()):
            np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
        np.testing.assert_array_equal(a.metrics().cpu().numpy(), b.metrics().cpu().numpy())
        assert a.status() == 0 and b.status() == 0


@pytest.mark.parametrize("sched", [0, 48])
def test_dynamic_schedule_full_size_ragged(sched):
    """At the full ragged batch (65536 envs, more wavefront groups than the
    GPU holds at once) the automatic schedule, which the benchmark uses, and
    a finer forced one match the static schedule bit for bit."""
    cfg = env_config("ragged", episode_len=200)
    outs, mets, states = [], [], []
    for sc in (-1, sched):
        env = _env(cfg, 65536, seed=0)
        env.set_schedule(sc)
        env.reset(0)
        outs.append(env.rollout(200))
        mets.append(env.metrics())
        states.append(env.state())
        assert env.status() == 0
        env.close()
    for k in outs[0]:
        assert torch.equal(outs[0][k], outs[1][k]), k
    assert torch.equal(mets[0], mets[1])
    for x, y in zip(states[0], states[1]):
        assert torch.equal(x, y)


def test_dynamic_schedule_graph_replays():
    """Captured with a dynamic schedule, the graph clears its queue on every
    replay: each replay equals the eager static rollout."""
    cfg = env_config("ragged", episode_len=64)
    env = _env(cfg, 3000, seed=2)
    env.set_schedule(16)
    gout, gm = env.capture_graph(64, episode=0)
    eager = _env(cfg, 3000, seed=2)
    eager.set_schedule(-1)
    eager.reset(0)
    ref = _np(eager.rollout(64))
    ref_m = eager.metrics().cpu().numpy()
    for rep in range(3):
        for v in gout.values():
            v.zero_()
        gm.zero_()
        env.launch_graph()
        torch.cuda.synchronize()
        _ = torch.randn(1000, device="cuda").sum().item()
        got = _np(gout)
        for k in ref:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"replay {rep} {k}")
        np.testing.assert_array_equal(gm.cpu().numpy(), ref_m)
    assert env.status() == 0


def test_autotune_keeps_results_and_caches(tmp_path):
    cfg = env_config("ragged", episode_len=50)
    env = _env(cfg, 3000, seed=1)
    env.reset(0)
    cache = tmp_path / "tune.jsonl"
    g, w = env.autotune(probe_steps=10, cache_path=cache)
    assert g in (1, 2) and w in (1, 2, 4)
    assert cache.exists() and "lanes_per_agent" in cache.read_text()
    out = _np(env.rollout(50, record=ALL))  # state was restored by the tuner
    ref_env = _env(cfg, 3000, seed=1)
    ref_env.reset(0)
    ref = _np(ref_env.rollout(50, record=ALL))
    for k in ALL:
        np.testing.assert_array_equal(out[k], ref[k], err_msg=k)
    env2 = _env(cfg, 3000, seed=1)
    env2.reset(0)
    assert env2.autotune(probe_steps=10, cache_path=cache) == (g, w)


def test_graph_replay_matches_eager():
    cfg = env_config("batched", episode_len=80)
    env = _env(cfg, 2048, seed=0)
    gout, gm = env.capture_graph(80, episode=0)
    eager = _env(cfg, 2048, seed=0)
    eager.reset(0)
    ref = _np(eager.rollout(80))
    ref_m = eager.metrics().cpu().numpy()
    for rep in range(3):
        for v in gout.values():
            v.zero_()
        gm.zero_()
        env.launch_graph()
        torch.cuda.synchronize()
        _ = torch.randn(1000, device="cuda").sum().item()  # unrelated eager work between replays
        got = _np(gout)
        for k in ref:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"replay {rep} {k}")
        np.testing.assert_array_equal(gm.cpu().numpy(), ref_m)


def test_metrics_match_oracle(orc):
    """The reduction equals the sums of the per-step records it summarises;
    those records are held to the oracle's by the rollout parity tests."""
    cfg = env_config("ragged", episode_len=60)
    E, T = 400, 60
    env = _env(cfg, E, seed=0)
    env.reset(0)
    out = _np(env.rollout(T, record=ALL))
    m = env.metrics().cpu().numpy()
    sel = np.arange(E)
    ref = _oracle(orc, cfg, env, sel, 0, T)
    compare_rollout(out, ref, env, sel, cfg, label="metrics")
    np.testing.assert_allclose(m[0], out["reward"].astype(np.float64).sum(), rtol=1e-9)
    err = out["err"].astype(np.float64)
    fin = np.isfinite(err)
    np.testing.assert_allclose(m[1], err[fin].sum(), rtol=1e-9)
    np.testing.assert_allclose(m[2], (err[fin] ** 2).sum(), rtol=1e-6)
    assert m[3] == fin.sum()
    em = ref["env_metrics"].sum(0)
    assert m[4] == em[4] == (out["reward"] == -1).sum()  # crash steps
    # lost targets at the end, from the final positions
    a_state, t_state = (x.cpu().numpy() for x in env.state())
    o = env.order
    lost = 0
    for k in range(E):
        ag = a_state[o["agent"][k]:o["agent"][k + 1], :2]
        tg = t_state[o["target"][k]:o["target"][k + 1], :2]
        d = np.hypot(ag[:, None, 0] - tg[None, :, 0], ag[:, None, 1] - tg[None, :, 1]).min(0)
        lost += (d > cfg["lost_range"]).sum()
    assert m[5] == lost == em[5]
    assert m[6] == E * T and m[7] == env.A * T


@pytest.mark.parametrize("name", ["ragged", "paper"])
def test_reset_state_matches_oracle(orc, name):
    """Spawned positions, headings and target speeds right after reset: the
    disk and square of the plain workloads and the pairwise 50-200 m layout
    of the paper's (with every pair inside the bounds on the GPU too)."""
    cfg = env_config(name)
    E = 500
    env = _env(cfg, E, seed=8)
    out = _np(env.reset(2, record=("gstate",)))
    ref = _oracle(orc, cfg, env, np.arange(E), 8, 0, episode=2)
    o = env.order
    s = cfg["area"] / 2
    for k in range(E):
        na, nt = env.n_agents[k], env.n_targets[k]
        gb = o["agent"][k] + o["target"][k]
        gs = out["gstate"][gb:gb + na + nt]
        ra = ref["init_agent"][ref["csr"]["agent"][k]:ref["csr"]["agent"][k + 1]]
        rt = ref["init_target"][ref["csr"]["target"][k]:ref["csr"]["target"][k + 1]]
        assert np.abs(gs[:na, :2] - ra[:, :2]).max() <= 1e-5 * s
        assert np.abs(gs[na:, :2] - rt[:, :2]).max() <= 1e-5 * s
        assert angle_diff(gs[:na, 4], ra[:, 2]).max() <= 1e-5 * np.pi
        if cfg["spawn_mode"] == 1:
            xy = gs[:, :2].astype(np.float64)
            d = np.hypot(xy[:, None, 0] - xy[None, :, 0], xy[:, None, 1] - xy[None, :, 1])
            iu = np.triu_indices(na + nt, 1)
            assert (d[iu] >= cfg["spawn_min"] - 1e-3).all() and (d[iu] <= cfg["spawn_max"] + 1e-3).all()


def test_reset_observation(orc):
    cfg = env_config("ragged")
    env = _env(cfg, 200, seed=4)
    out = _np(env.reset(3, record=("obs", "obs_mask", "gstate")))
    sel = np.arange(200)
    ref = _oracle(orc, cfg, env, sel, 4, 0, episode=3)
    o = env.order
    ck = ref["csr"]["token"]
    for k in sel:
        g = out["obs"][o["token"][k]:o["token"][k + 1]]
        r = ref["init_obs"][ck[k]:ck[k + 1]]
        np.testing.assert_allclose(g, r, atol=1e-5 * 2000, rtol=0)
        np.testing.assert_array_equal(out["obs_mask"][o["token"][k]:o["token"][k + 1]],
                                      ref["init_mask"][ck[k]:ck[k + 1]])


def test_given_actions_and_bad_action_flag(orc):
    cfg = env_config("batched", episode_len=30)
    E, T = 64, 30
    env = _env(cfg, E, seed=2)
    env.reset(0)
    rng = np.random.default_rng(0)
    acts = rng.integers(0, 5, size=(T, env.A)).astype(np.int32)
    acts[7, 3] = 11  # out of range: no turn, status bit
    gpu = _np(env.rollout(T, actions=torch.from_numpy(acts).cuda(), record=ALL))
    assert env.status() & 0x1
    assert env.status() == 0  # cleared by the read
    ref = _oracle(orc, cfg, env, np.arange(E), 2, T, actions=acts)
    compare_rollout(gpu, ref, env, np.arange(E), cfg, label="given-actions")
    assert gpu["actions"][7, 3] == -1


def test_errors_are_reported():
    from paper_2505_08222_amd._lib import MilError
    cfg = env_config("plain", episode_len=5)
    env = _env(cfg, 8)
    with pytest.raises(MilError):
        env.step()  # before reset
    env.reset(0)
    env.rollout(5, record=())
    with pytest.raises(MilError):
        env.step()  # past the episode
    with pytest.raises(MilError):
        env.set_mapping(3, 1)


def test_env_windows_match_oracle(orc):
    """The exported tracker windows (entry k = the state k steps back: agent
    position and range) with each env's range sigma and the true target
    position, against the oracle's records of the same rollout."""
    from paper_2505_08222_amd import learned
    cfg = env_config("ragged", window=16, episode_len=40)
    E, T, W = 300, 40, 16
    env = _env(cfg, E, seed=6)
    env.reset(0)
    env.rollout(T, record=())
    win, sigma, truth = (x.cpu().numpy() for x in learned.env_windows(env))
    sel = np.arange(E)
    ref = _oracle(orc, cfg, env, sel, 6, T)
    o = env.order
    s = cfg["area"] / 2
    cp = np.concatenate([[0], np.cumsum(env.n_agents * env.n_targets)])
    for k in range(E):
        na, nt = env.n_agents[k], env.n_targets[k]
        for i in range(na):
            a = ref["csr"]["agent"][k] + i
            for j in range(nt):
                p = cp[k] + i * nt + j
                g = o["pair"][k] + i * nt + j
                for q in range(W):
                    t = T - 1 - q
                    assert np.abs(win[g, q, :2] - ref["agent"][t, a, :2]).max() <= 1e-5 * s
                    assert abs(win[g, q, 2] - ref["ranges"][t, p]) <= 1e-5 * s
                assert abs(sigma[g] - ref["sigma_r"][k]) <= 1e-6 * ref["sigma_r"][k]
                tg = ref["csr"]["target"][k] + j
                assert np.abs(truth[g] - ref["target"][T - 1, tg, :2]).max() <= 1e-5 * s
