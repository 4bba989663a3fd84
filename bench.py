#!/usr/bin/env python3
"""Benchmark of the batched range-only tracking environment on one MI355X.

One benchmark step = one replay of the captured HIP graph {reset, T-step
persistent rollout writing observations, masks, rewards and done flags,
metrics reduction} over the whole batch, inputs resident in HBM. Default
(`--workload all`): the ragged batch (65536 envs, agents and targets uniform
1..5 per env, 1000 steps) is the headline; the plain batched workload (4096
envs x 2x2 x 500 steps, with an env-count sweep), the learned estimator and
the closed loop with the attention policy follow as sections of the same JSON
line, then the paper's own environment (LS trackers, pooled LS, learned
estimator on its windows) and the particle-filter tracker on the ragged batch
and on the paper's environment. `--workload NAME` runs one of them alone.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "env-steps/s and HBM GB/s at 1 MI355X; learned vs exact estimator speedup at ≤1 m RMS"
HBM_PEAK_GBS = 8000.0
RECORD = ("obs", "obs_mask", "reward", "done")


def bytes_per_env_step(n_agents, n_targets):
    """Algorithmic HBM bytes one env-step must write: per observation token 6
    FP32 + 1 mask byte, reward FP32, done byte."""
    tokens = n_agents * (n_agents + n_targets)
    return 25 * tokens + 5


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Sources each dominant kernel is built from; the HBM traffic measured with
# rocprofv3 counters is reported only while their hash is the one it was
# measured on.
KERNEL_SOURCES = {
    "rollout_kernel": ["env_kernels.hip", "env_internal.h", "ls_device.h", "rng.h"],
    "policy_kernel": ["policy_kernels.hip", "policy_internal.h", "mfma_tile.h", "rng.h"],
    "pf_kernel": ["pf_kernels.hip", "env_internal.h", "rng.h"],
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_counters.md")
VALU_FILES = [os.path.join(ROOT, "profiles", n) for n in
              ("pf_kernel_valu_counters.md", "rollout_kernel_paper_valu_counters.md")]
# VALU issue capacity of the chip: 256 CUs x 4 SIMDs, each SIMD's vector unit
# busy for one cycle per cycle at 2.4 GHz (a full-rate wave64 instruction
# occupies it 4 cycles, a quarter-rate one 16)
VALU_PEAK_CYCLES = 256 * 4 * 2.4e9


def kernel_version(kernel):
    import hashlib
    h = hashlib.sha1()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2505_08222_amd", "csrc", name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:12]


def measured_traffic(kernel, workload):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, each scaled by the
    copy-kernel calibration) from the committed counter summary, or None when
    there is none for this workload or the kernel changed since."""
    import re
    if not os.path.exists(TRAFFIC_FILE):
        return None
    ver = kernel_version(kernel)
    pat = re.compile(r"^traffic\s+(\S+)\s+(\S+)\s+(\S+)\s+(\d+)\s+(\d+)\s*$")
    with open(TRAFFIC_FILE) as f:
        for line in f:
            m = pat.match(line.strip())
            if m and m.group(1) == kernel and m.group(2) == workload and m.group(3) == ver:
                return int(m.group(4)) + int(m.group(5))
    return None


def measured_valu(kernel, workload):
    """VALU-busy SIMD cycles per launch (4 x SQ_ACTIVE_INST_VALU, summed over
    the chip) and VALU instructions per launch from the committed counter
    summary, or None when there is none or the kernel changed since."""
    import re
    ver = kernel_version(kernel)
    pat = re.compile(r"^valu\s+(\S+)\s+(\S+)\s+(\S+)\s+(\d+)\s+(\d+)\s*$")
    for path in VALU_FILES:
        if not os.path.exists(path):
            continue
        with open(path) as f:
            for line in f:
                m = pat.match(line.strip())
                if m and m.group(1) == kernel and m.group(2) == workload and m.group(3) == ver:
                    return int(m.group(4)), int(m.group(5))
    return None


def pf_bytes_per_launch(env, cfg):
    """Algorithmic HBM bytes of one particle-filter launch: each tracker's 64
    particles read and written (1024 B), its rows read (16 B each: its own, or
    with pooling one per agent of its env), its descriptor (16 B), belief and
    estimate written (10 B) and belief read (1 B)."""
    import numpy as np
    na = env.n_agents.astype(np.int64)
    nt = env.n_targets.astype(np.int64)
    rows = na if cfg["pooled"] else np.ones_like(na)
    return float((na * nt * (1024 + 16 * rows + 27)).sum())


def pf_kernel_roofline(env, cfg, workload, full_size):
    """The particle-filter kernel timed alone: mid-episode (after 20 steps),
    event-timed repeats of the filter update on the stream it is launched on.
    Its bound is VALU issue (Philox rounds, Box-Muller, the cross-lane scans):
    the roofline reports the VALU-busy fraction from the committed counters
    over the live duration, with the HBM view beside it."""
    import numpy as np
    import torch

    stream = torch.cuda.current_stream()
    env.reset(0)
    env.rollout(20, record=())
    reps = 10
    durs = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            env.pf_update()
        b.record(stream)
        torch.cuda.synchronize()
        durs.append(a.elapsed_time(b) / reps)
    kern_ms = float(np.median(durs))
    alg = pf_bytes_per_launch(env, cfg)
    gbs = alg / (kern_ms / 1e3) / 1e9
    hbm = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": gbs / HBM_PEAK_GBS, "bytes_per_launch": alg}
    log(f"[bench] pf kernel {kern_ms*1e3:.1f} us/launch, {alg/1e6:.1f} MB algorithmic, "
        f"{gbs:.0f} GB/s")
    valu = measured_valu("pf_kernel", workload) if full_size else None
    traffic = measured_traffic("pf_kernel", workload) if full_size else None
    hbm["traffic"] = traffic
    roof = {"kernel": "pf_kernel", "kernel_ms": kern_ms, "trackers": int(env.P),
            "particles_per_tracker": 64,
            "particle_updates_per_s": env.P * 64 / (kern_ms / 1e3)}
    if valu is not None:
        busy, insts = valu
        ach = busy / (kern_ms / 1e3)
        roof.update({"bound": "alu", "achieved": ach, "peak": VALU_PEAK_CYCLES,
                     "unit": "VALU-busy SIMD cycles/s", "frac": ach / VALU_PEAK_CYCLES,
                     "valu_busy_cycles_per_launch": busy, "valu_insts_per_launch": insts,
                     "traffic": traffic, "hbm_view": hbm})
    else:
        roof.update(hbm)
    if traffic is not None:
        roof["traffic_unit"] = "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)"
        roof["traffic_gbps"] = traffic / (kern_ms / 1e3) / 1e9
    return roof


def copy_probe():
    """A plain 256 MiB device-to-device copy (the calibration kernel for the
    FETCH_SIZE / WRITE_SIZE counters): 3 launches."""
    import torch
    n = 64 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                      "launches": 3}), flush=True)


def host_cpu():
    """Cores the oracle may use on this host and what they are."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "usable_cores": usable}


def oracle_threads():
    """Every core this process may run on (the lease's share of the host)."""
    return host_cpu()["usable_cores"]


def cpu_baseline(cfg, env, T, budget_s):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    whole episodes of the envs in packed order, 256 envs per call, recording
    the same outputs as the GPU run; when every env is done it goes on with
    the next episode (a new reset draw) until the time budget is used."""
    from oracle import oracle as orc

    threads = oracle_threads()
    orc.lib()
    ids, na, nt = env.order["env_ids"], env.n_agents, env.n_targets
    # the filter does 64 particle updates per tracker: fewer envs per call
    chunk = (2 if cfg.get("est_kind", 0) == 1 else 64) * threads
    done_envsteps = 0
    calls = 0
    t0 = time.perf_counter()
    k, episode = 0, 0
    while time.perf_counter() - t0 < budget_s:
        sl = slice(k, min(k + chunk, len(ids)))
        orc.rollout(cfg, ids[sl], na[sl], nt[sl], env.seed, T, episode=episode,
                    records=("reward", "done", "obs", "obs_mask"), n_threads=threads)
        done_envsteps += (sl.stop - sl.start) * T
        calls += 1
        k = sl.stop
        if k >= len(ids):
            k, episode = 0, episode + 1
    el = time.perf_counter() - t0
    envs_run = done_envsteps // T
    return {"value": done_envsteps / el, "unit": "env-steps/s", "cores": threads,
            "kind": "oracle", **host_cpu(),
            "sample": f"{envs_run} env-episodes x {T} steps ({envs_run / len(ids):.2f} passes over "
                      f"the {len(ids)} envs, same seed and config, obs/mask/reward/done recorded), "
                      f"FP64 C with OpenMP over envs, {el:.1f} s"}


def cpu_baseline_policy(cfg, env, params, budget_s):
    """The oracle on a bounded sample of the policy workload: the first 16
    envs for 50 steps (oracle environment rollout, OpenMP over envs), then
    the oracle policy forward (single thread) on every agent's observation of
    every step, repeated until the budget is used; env-steps/s of the sum."""
    import numpy as np

    from oracle import oracle as orc

    threads = oracle_threads()
    orc.lib()
    E, T = 16, 50
    ids, na, nt = env.order["env_ids"][:E], env.n_agents[:E], env.n_targets[:E]
    n_tok = int(na[0] + nt[0])
    th = params.detach().cpu().numpy().astype(np.float64)
    t_env = t_pol = 0.0
    done = 0
    t_start = time.perf_counter()
    while time.perf_counter() - t_start < budget_s:
        t0 = time.perf_counter()
        ref = orc.rollout(cfg, ids, na, nt, env.seed, T, episode=done,
                          records=("obs", "obs_mask", "reward", "done"), n_threads=threads)
        t1 = time.perf_counter()
        for t in range(T):
            orc.policy_forward(ref["obs"][t].reshape(-1, n_tok, 6),
                               ref["obs_mask"][t].reshape(-1, n_tok), th)
        t2 = time.perf_counter()
        t_env += t1 - t0
        t_pol += t2 - t1
        done += 1
    return {"value": done * E * T / (t_env + t_pol), "unit": "env-steps/s", "cores": threads,
            "kind": "oracle", **host_cpu(),
            "sample": f"{done} x ({E} envs x {T} steps): oracle env rollout (FP64 C, OpenMP over "
                      f"envs, {t_env:.1f} s) + oracle policy forward on every agent-step (FP64 C, one "
                      f"thread, {t_pol:.1f} s)"}


def env_sweep(args, cfgname="batched", sizes=(4096, 16384, 65536, 262144, 1048576), T=100):
    """Env-count sweep of the rollout kernel at one shape (2 agents x 2
    targets): where the path turns from latency- to bandwidth-bound. Each
    point: autotuned mapping, T-step rollout recording obs/mask/reward/done,
    median of 5 event-timed launches."""
    import numpy as np
    import torch

    from paper_2505_08222_amd.configs import env_config
    from paper_2505_08222_amd.env import Env

    cfg = env_config(cfgname, episode_len=T)
    stream = torch.cuda.current_stream()
    cache = os.path.join(ROOT, "gpurun_out", "autotune_cache.jsonl")
    points = []
    for E in sizes:
        env = Env(cfg, E, seed=0)
        env.reset(0)
        if not args.no_autotune:
            env.autotune(probe_steps=20, cache_path=cache)
        out = env._alloc(RECORD, T)
        durs = []
        for _ in range(6):
            env.reset(0)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            env.rollout(T, record=RECORD, out=out)
            b.record(stream)
            torch.cuda.synchronize()
            durs.append(a.elapsed_time(b))
        ms = float(np.median(durs[1:]))
        alg = float(bytes_per_env_step(env.n_agents.astype(np.int64),
                                       env.n_targets.astype(np.int64)).sum()) * T
        gbs = alg / (ms / 1e3) / 1e9
        points.append({"envs": E, "steps": T, "kernel_ms": ms, "env_steps_per_s": E * T / (ms / 1e3),
                       "hbm_gbps_algorithmic": gbs, "frac": gbs / HBM_PEAK_GBS,
                       "lanes_per_agent": env.get_mapping()[0], "waves_per_block": env.get_mapping()[1]})
        log(f"[sweep] {E} envs: {ms:.3f} ms, {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.1%})")
        del out, env
        torch.cuda.empty_cache()
    return points


TRAIN_BATCH = 8192


def mlp_train_flops_per_sample(d_in=64, h=128, d_out=2):
    """Algorithmic FLOPs of one training sample: forward, the three weight
    gradients, and the input gradients of the second and output layers."""
    fwd = 2 * (d_in * h + h * h + h * d_out)
    return fwd + fwd + 2 * (h * d_out + h * h)


def mlp_infer_flops_per_window(d_in=64, h=128, d_out=2):
    return 2 * (d_in * h + h * h + h * d_out)


# Where the learned estimator's windows come from. "learned": the ragged
# configuration with W = 16 (1 s steps: a 16 m track per window); "paper": the
# paper's environment with W = 16 (30 s steps: a track of hundreds of metres,
# where the range-only solve is well posed), with the targets held still (the
# least-squares solve assumes a target that does not move within its window;
# at the paper's half speed a target moves 240 m in 16 steps and the window
# measures that model error instead) and no detection cut (complete windows).
WINDOW_SOURCES = {
    "learned": dict(env=None, num_envs=None, train=None, infer=None, train_first=100,
                    train_every=50, infer_first=125, infer_every=50, epochs=8),
    "paper": dict(env=dict(window=16, episode_len=300, ragged=1, target_speed_lo=0.0,
                           target_speed_hi=0.0, det_range=math.inf),
                  num_envs=16384, train=4_000_000, infer=1_000_000, train_first=16,
                  train_every=4, infer_first=18, infer_every=4, epochs=40),
}


def window_source(variant):
    """(env config, envs, train windows, inference windows, schedule)."""
    from paper_2505_08222_amd.configs import CONFIGS, env_config
    src = WINDOW_SOURCES[variant]
    if variant == "learned":
        c = CONFIGS["learned"]
        return (dict(c["env"]), c["num_envs"], c["train_windows"], c["infer_windows"], src)
    return (env_config("paper", **src["env"]), src["num_envs"], src["train"], src["infer"], src)


def train_estimator(args, variant="learned"):
    """The learned estimator's network, trained by the library's kernels on
    windows of ragged-configuration rollouts (W = 16): 1e7 windows, labels =
    exact estimates within 2x the mean range from tracks with condition
    number <= 1e3 (elsewhere the exact solve is noise, and those windows fall
    back to it anyway), 8 epochs of Adam. Then 20 further steps on the same
    data are timed with events (forward, backward, gradient reduction, Adam)
    for the training roofline. Returns (params, info)."""
    import numpy as np
    import torch

    from paper_2505_08222_amd import learned
    from paper_2505_08222_amd.configs import CONFIGS

    cfg, n_envs, n_train, _, src = window_source(variant)
    if args.envs:
        n_train = max(20000, int(n_train * args.envs / n_envs))
    E = args.envs or n_envs
    t0 = time.perf_counter()
    tr = learned.rollout_windows(cfg, E, n_train, seed=0, first_step=src["train_first"],
                                 every=src["train_every"])
    n_windows = int(tr["win"].shape[0])
    x, frame = learned.features(tr["win"])
    y = learned.targets(frame, tr["exact"])
    kap_tr = window_condition(tr["win"])
    keep = (y.norm(dim=1) <= 2.0) & (kap_tr <= 1e3)
    x, y = x[keep].contiguous(), y[keep].contiguous()
    del tr, frame, kap_tr, keep
    log(f"[learned] training set {x.shape[0]} of {n_windows} windows "
        f"({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    params, hist = learned.train(x, y, epochs=src["epochs"], batch=TRAIN_BATCH, lr=2e-3,
                                 lr_final=3e-5, seed=0, log=lambda m: None)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    log(f"[learned] trained {len(hist)} logged steps in {train_s:.1f} s, loss {hist[0][1]:.3e} -> "
        f"{hist[-1][1]:.3e}")
    # training step alone (the fused gradient + Adam step the training loop
    # runs): a copy of the weights, 20 steps timed with events
    p2 = params.clone()
    opt = learned.Adam(p2, lr=3e-5)
    work = learned._work(TRAIN_BATCH, "bf16", x.device)
    gen = torch.Generator(device=x.device)
    gen.manual_seed(1)
    idx = [torch.randperm(x.shape[0], generator=gen, device=x.device)[:TRAIN_BATCH]
           for _ in range(21)]
    learned.train_step(x, y, opt, index=idx[0], work=work)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for k in range(1, 21):
        learned.train_step(x, y, opt, index=idx[k], work=work)
    b.record(stream)
    torch.cuda.synchronize()
    step_ms = a.elapsed_time(b) / 20
    flops = mlp_train_flops_per_sample() * TRAIN_BATCH
    tflops = flops / (step_ms / 1e3) / 1e12
    info = {"seconds": train_s, "windows_generated": n_windows, "train_windows": int(x.shape[0]),
            "epochs": src["epochs"], "batch": TRAIN_BATCH, "loss_first": hist[0][1], "loss_last": hist[-1][1],
            "step_ms": step_ms, "samples_per_s": TRAIN_BATCH / (step_ms / 1e3),
            "mfma": {"bound": "mfma", "achieved": tflops, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": tflops / 2500.0, "flops_per_step": flops,
                     "kernels": "mlp_train_step: train_accum_kernel + reduce_step_kernel (gradient "
                                "reduction fused with Adam)"}}
    del x, y, work, idx
    torch.cuda.empty_cache()
    return params, info


def cpu_baseline_exact(win_cpu, budget_s):
    """The oracle's exact estimator (FP64 C, OpenMP over windows) on the
    inference windows, closed form and with 8 Gauss-Newton steps: windows per
    second, on as many windows as fit the time budget."""
    from oracle import oracle as orc

    threads = oracle_threads()
    orc.lib()
    out = {}
    for gn in (0, 8):
        n = min(len(win_cpu), 65536)
        done, t0 = 0, time.perf_counter()
        while True:
            orc.ls_batch(win_cpu[:n], gn_iters=gn, n_threads=threads)
            done += n
            el = time.perf_counter() - t0
            if el >= budget_s / 2 or done >= len(win_cpu) * 4:
                break
            n = min(len(win_cpu), n * 2)
        out[f"gauss_newton_{gn}"] = {"value": done / el, "unit": "windows/s"}
    return {"value": out["gauss_newton_0"]["value"], "unit": "windows/s (exact estimator, closed form)",
            "cores": threads, "kind": "oracle", **host_cpu(), "by_kind": out,
            "sample": f"the first windows of the inference set, FP64 C with OpenMP over windows, "
                      f"closed form and 8 Gauss-Newton steps, about {budget_s / 2:.0f} s each"}


def bench_learned(args, steps, cpu_seconds=None, trained=None, variant="learned"):
    """Learned estimator (the learned-estimator configuration): windows of 16
    from ragged-configuration rollouts (or, variant "paper", from the paper's
    30 s environment), Adam training of the BF16 MLP with the library's
    kernels, then guarded inference on a disjoint set, compared with the exact
    estimator on error (m) and throughput."""
    import numpy as np
    import torch

    from paper_2505_08222_amd import learned
    from paper_2505_08222_amd.configs import CONFIGS
    from paper_2505_08222_amd.env import est_exact

    cfg, n_envs, _, n_infer, src = window_source(variant)
    torch.cuda.set_device(0)
    if args.envs:  # smaller runs for quick checks
        n_infer = max(20000, int(n_infer * args.envs / n_envs))
    E = args.envs or n_envs
    params, train_info = trained if trained is not None else train_estimator(args, variant)
    t0 = time.perf_counter()
    te = learned.rollout_windows(cfg, E, n_infer, seed=1, first_step=src["infer_first"],
                                 every=src["infer_every"])
    log(f"[learned] inference windows {te['win'].shape[0]} ({time.perf_counter() - t0:.1f} s)")
    win, sigma, truth = te["win"], te["sigma"], te["truth"]
    N = win.shape[0]
    work = learned._work(N, "bf16", win.device)

    def timed(fn, reps=max(1, steps)):
        fn()
        torch.cuda.synchronize()
        evs = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            out = fn()
            b.record()
            torch.cuda.synchronize()
            evs.append(a.elapsed_time(b))
        return out, float(np.median(evs))

    (p_mlp, flag), ms_mlp = timed(lambda: learned.infer(win, params, sigma, 3.0, work=work))
    (p_ex, v_ex), ms_ex = timed(lambda: est_exact(win))
    (p_ex32, _), ms_ex32 = timed(lambda: est_exact(win, accum="fp32"))
    (p_gn, v_gn), ms_gn = timed(lambda: est_exact(win, gn_iters=8))
    xi, _ = learned.features(win)
    (_, _), ms_fwd = timed(lambda: (learned.forward(xi, params, "bf16"), None))
    flag = flag.cpu().numpy()
    pm, pe, pt = p_mlp.cpu().numpy(), p_ex.cpu().numpy(), truth.cpu().numpy()
    pg = p_gn.cpu().numpy()
    ve = v_ex.cpu().numpy().astype(bool)
    acc = flag == 1
    rng_ = np.hypot(*(pt - win[:, :, :2].mean(1).cpu().numpy()).T)
    kap = window_condition(win).cpu().numpy()
    d_me = np.hypot(*(pm - pe).T)
    d_et = np.hypot(*(pe - pt).T)
    bins = [(0, 50), (50, 100), (100, 200), (200, 500), (500, 1e9)]
    by_kappa = {}
    for lo, hi in [(1, 10), (10, 100), (100, 1e3), (1e3, np.inf)]:
        m = acc & ve & (kap >= lo) & (kap < hi)
        mt = ve & (kap >= lo) & (kap < hi)
        by_kappa[f"kappa {lo:g}-{hi:g}"] = {
            "windows": int(mt.sum()), "accepted_frac": float(m.sum() / max(mt.sum(), 1)),
            "rms_learned_vs_exact_m": float(np.sqrt(np.mean(d_me[m] ** 2))) if m.any() else None}
    by_bin = {}
    for lo, hi in bins:
        m = acc & ve & (rng_ >= lo) & (rng_ < hi)
        mt = ve & (rng_ >= lo) & (rng_ < hi)
        name = f"{int(lo)}-{int(hi) if hi < 1e8 else 'inf'} m"
        by_bin[name] = {
            "windows": int(mt.sum()), "accepted_frac": float(m.sum() / max(mt.sum(), 1)),
            "rms_learned_vs_exact_m": float(np.sqrt(np.mean(d_me[m] ** 2))) if m.any() else None,
            "rms_exact_vs_truth_m": float(np.sqrt(np.mean(d_et[mt] ** 2))) if mt.any() else None,
            "rms_final_vs_truth_m": float(np.sqrt(np.mean(np.hypot(*(pm[mt] - pt[mt]).T) ** 2))) if mt.any() else None,
        }
    # where the exact estimate is itself within 1 m of the truth (a well-posed
    # window), how far the accepted network estimates are from it
    wp = acc & ve & (d_et <= 1.0)
    well_posed = {"windows": int((ve & (d_et <= 1.0)).sum()), "accepted": int(wp.sum()),
                  "rms_learned_vs_exact_m": float(np.sqrt(np.mean(d_me[wp] ** 2))) if wp.any() else None}
    flops = mlp_infer_flops_per_window() * N
    res = {
        "metric": METRIC,
        "value": ms_ex / ms_mlp,
        "unit": "x (exact FP64 LS time / guarded learned time, same GPU, same windows)",
        "n_gpus": 1, "steps": max(1, steps), "warmup": 1, "ms_per_step": ms_mlp,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"learned estimator: 16-entry windows from "
                               + ("ragged-configuration" if variant == "learned" else
                                  "paper-environment (30 s step)")
                               + f" rollouts, train {train_info['train_windows']}, infer {N}",
                   "train_windows": train_info["train_windows"], "infer_windows": int(N)},
        "infer_ms": {"learned_guarded": ms_mlp, "mlp_forward_only": ms_fwd,
                     "exact_fp64": ms_ex, "exact_fp32": ms_ex32, "exact_gauss_newton8": ms_gn},
        "windows_per_s": {"learned_guarded": N / (ms_mlp / 1e3), "exact_fp64": N / (ms_ex / 1e3),
                          "exact_gauss_newton8": N / (ms_gn / 1e3)},
        "speedup_vs": {"exact_fp64": ms_ex / ms_mlp, "exact_fp32": ms_ex32 / ms_mlp,
                       "exact_gauss_newton8": ms_gn / ms_mlp},
        "accepted_frac": float(acc.mean()),
        "rms_learned_vs_exact_m_accepted": float(np.sqrt(np.mean(d_me[acc & ve] ** 2))),
        "median_learned_vs_exact_m_accepted": float(np.median(d_me[acc & ve])),
        "where_exact_within_1m_of_truth": well_posed,
        "by_range": by_bin,
        "by_condition": by_kappa,
        "train": train_info,
        "roofline": {"bound": "mfma", "achieved": flops / (ms_fwd / 1e3) / 1e12, "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": flops / (ms_fwd / 1e3) / 1e12 / 2500.0,
                     "kernel": "forward_kernel", "kernel_ms": ms_fwd, "flops_per_launch": flops},
        "guarded_inference_mfma_frac": flops / (ms_mlp / 1e3) / 1e12 / 2500.0,
        "gauss_newton_vs_truth_rms_m": float(np.sqrt(np.mean(np.hypot(*(pg[ve] - pt[ve]).T) ** 2))),
    }
    if cpu_seconds:
        log("[bench] cpu baseline (oracle), exact estimator on the inference windows")
        res["cpu_baseline"] = cpu_baseline_exact(win.cpu().numpy().astype(np.float64), cpu_seconds)
    del work, win, te
    torch.cuda.empty_cache()
    return res


def window_condition(win):
    """Condition number of S = sum_k u_k u_k^T (agent positions about their
    centroid) for each window [N, W, 3]."""
    import torch
    a = win[..., :2].double()
    u = a - a.mean(dim=1, keepdim=True)
    sxx = (u[..., 0] ** 2).sum(1)
    syy = (u[..., 1] ** 2).sum(1)
    sxy = (u[..., 0] * u[..., 1]).sum(1)
    tr, det = sxx + syy, sxx * syy - sxy * sxy
    disc = torch.sqrt(torch.clamp(tr * tr / 4 - det, min=0.0))
    lmax, lmin = tr / 2 + disc, tr / 2 - disc
    return (lmax / torch.clamp(lmin, min=1e-300)).float()


def policy_flops_per_agent_step(n_tok, d=64, heads=4, ffn=256, layers=2, n_out=8):
    """Algorithmic FLOPs of one agent's forward pass (dense layers + attention)."""
    per_layer = (2 * n_tok * d * 3 * d + 2 * 2 * heads * n_tok * n_tok * (d // heads)
                 + 2 * n_tok * d * d + 2 * 2 * n_tok * d * ffn)
    return 2 * n_tok * 6 * d + layers * per_layer + 2 * d * n_out


def bench_ppo(args, T=32, cpu_seconds=None):
    """The learner on the policy workload's shape (16384 envs x 5 agents x 5
    targets), one PPO batch of T steps: critic values of the T + 1 global
    states of every env, the policy re-evaluated on every agent's T
    observations, GAE, the clipped objective with its gradients, the heads'
    gradients and Adam steps; then the full update of every parameter (the
    training form's forward and reverse passes of actor and critic, Adam) on
    one minibatch. Inputs are synthetic tensors of the workload's shapes,
    resident in HBM (the learner's arithmetic does not depend on their
    values). Dominant kernel: the attention kernel (critic and policy
    forwards), MFMA roofline."""
    import numpy as np
    import torch

    from paper_2505_08222_amd import policy, ppo
    from paper_2505_08222_amd.configs import CONFIGS

    c = CONFIGS["policy"]
    E = args.envs or c["num_envs"]
    na = nt = 5
    M, n_tok, A = na + nt, na + na + nt, E * na
    g = torch.Generator(device="cuda").manual_seed(0)
    dev = "cuda"
    gs = torch.randn(T + 1, E * M, 6, device=dev, generator=g)
    gs[..., 0:2] *= 1000.0
    gs[..., 2] = 0.0
    gs[..., 5] = (torch.arange(E * M, device=dev) % M >= na).float()
    obs = torch.randn(T * A * n_tok, 6, device=dev, generator=g)
    mask = (torch.rand(T * A * n_tok, device=dev, generator=g) > 0.1).to(torch.uint8)
    actions = torch.randint(0, 5, (T, A), device=dev, dtype=torch.int32, generator=g)
    rewards = torch.rand(T, E, device=dev, generator=g)
    dones = torch.zeros(T, E, device=dev, dtype=torch.uint8)
    actor = policy.init_params(c["seed"])
    critic = policy.init_params(c["seed"] + 1)
    stream = torch.cuda.current_stream()

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            out = fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return float(np.median(ms)), out

    t_crit, (values, cfeat) = timed(lambda: ppo.critic_forward(gs, na, nt, critic, features=True))
    values = values.reshape(T + 1, E)
    t_pol, (logits, pfeat) = timed(lambda: ppo.policy_features(obs, mask, actor, n_tok, na))
    logits = logits.reshape(T, A, 8)
    logits_old = logits + 0.1 * torch.randn(logits.shape, device=dev, generator=g)
    t_gae, (adv, ret) = timed(lambda: ppo.gae(rewards, dones, values, 0.99, 0.95))
    t_obj, (out, dl, dv) = timed(lambda: ppo.objective(logits, logits_old, actions, adv,
                                                      values[:T].contiguous(), ret, na, 5))
    # the heads' gradients and Adam steps (the layers below them are not trained)
    t_hg, (ga, gc) = timed(lambda: (ppo.head_grad(pfeat, dl.reshape(T * A, 8), 5),
                                    ppo.head_grad(cfeat[:T * E], dv.reshape(-1), 1)))
    oa, oc = ppo.HeadAdam(actor), ppo.HeadAdam(critic)
    t_adam, _ = timed(lambda: (oa.step(ga), oc.step(gc)))
    total = t_crit + t_pol + t_gae + t_obj + t_hg + t_adam
    # the full update of every parameter on one minibatch: the training form
    # (FP32 forward with its tape, reverse pass) of the actor on mb_agents
    # agents and of the critic on their envs' states, then Adam on both
    from paper_2505_08222_amd import learned
    mb_envs = min(E, 8192)
    mb_agents = mb_envs * na
    ta, tc = ppo.TrainPass(mb_agents, n_tok), ppo.TrainPass(mb_envs, M + 1)
    mobs, mmask = obs[:mb_agents * n_tok], mask[:mb_agents * n_tok]
    mgs = gs[0, :mb_envs * M]
    dlm = dl.reshape(T * A, 8)[:mb_agents].contiguous()
    dvm = dv.reshape(-1)[:mb_envs].contiguous()
    fa, fc = learned.Adam(actor.clone(), lr=1e-5), learned.Adam(critic.clone(), lr=1e-5)

    def full_update():
        ta.forward(mobs, mmask, fa.params)
        g1, _ = ta.backward(fa.params, dlm, 5)
        tc.critic_forward(mgs, na, nt, fc.params)
        g2, _ = tc.backward(fc.params, dvm, 1)
        fa.step(g1)
        fc.step(g2)
        return g1, g2
    t_full, _ = timed(full_update)
    fl_full = 3 * (policy_flops_per_agent_step(n_tok) * mb_agents
                   + policy_flops_per_agent_step(M + 1) * mb_envs)
    fl_crit = policy_flops_per_agent_step(M + 1) * (T + 1) * E
    fl_pol = policy_flops_per_agent_step(n_tok) * T * A
    ach = fl_crit / (t_crit / 1e3) / 1e12
    log(f"[bench] ppo: critic {t_crit:.2f} ms, policy {t_pol:.2f} ms, gae {t_gae:.3f} ms, "
        f"objective {t_obj:.3f} ms, head gradients {t_hg:.3f} ms, Adam {t_adam:.3f} ms; "
        f"full update of {mb_agents} agents + {mb_envs} states {t_full:.2f} ms")
    o = out.cpu().numpy()
    res = {
        "metric": METRIC, "value": T * A / (total / 1e3), "unit": "agent-steps/s",
        "n_gpus": 1, "steps": 3, "dtype": "bf16 (MFMA, FP32 accumulate); FP64 GAE",
        "data": "synthetic tensors of the workload's shapes",
        "config": {"workload": f"PPO batch: {E} envs x {na} agents x {nt} targets x {T} steps: "
                               "critic on T + 1 states, policy on T steps (with the heads' "
                               "inputs), GAE, clipped objective, head gradients and Adam; the "
                               "full update of every parameter is timed under full_update",
                   "envs": E, "agents": A, "batch_steps": T},
        "ms": {"critic": t_crit, "policy": t_pol, "gae": t_gae, "objective": t_obj,
               "head_grad": t_hg, "adam": t_adam, "total": total},
        "full_update": {"minibatch_agents": mb_agents, "minibatch_states": mb_envs,
                        "ms": t_full, "agent_samples_per_s": mb_agents / (t_full / 1e3),
                        "tflops": fl_full / (t_full / 1e3) / 1e12,
                        # its dense products are FP32 GEMMs: the FP32 matrix peak bounds it
                        "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": 157.3,
                                     "achieved": fl_full / (t_full / 1e3) / 1e12,
                                     "frac": fl_full / (t_full / 1e3) / 1e12 / 157.3},
                        "note": "FP32 training form (forward with tape, exact backward; weight "
                                "gradients on the FP32 matrix cores, other products in "
                                "hipBLASLt/rocBLAS FP32 GEMMs) of actor and critic plus Adam on "
                                "every parameter; flops counted as 3x the forward's"},
        "objective": {"policy_loss": float(o[0]), "value_loss": float(o[1]),
                      "entropy": float(o[2]), "clip_frac": float(o[3])},
        "roofline": {"bound": "mfma", "kernel": "policy_kernel (critic tokens)", "achieved": ach,
                     "peak": 2500.0, "unit": "TFLOP/s", "frac": ach / 2500.0, "traffic": None,
                     "flops_per_state": policy_flops_per_agent_step(M + 1), "kernel_ms": t_crit,
                     "policy_forward_frac": fl_pol / (t_pol / 1e3) / 1e12 / 2500.0},
    }
    if cpu_seconds:
        res["cpu_baseline"] = cpu_baseline_ppo(critic, actor, cpu_seconds)
        res["full_update"]["cpu_oracle"] = cpu_oracle_gradient(actor, 2.0)
    return res


def cpu_oracle_gradient(actor, budget_s):
    """The oracle's gradient of the actor (FP64 C, one thread) on batches of
    20 agents of 5x5 envs until the budget is used; agent-samples/s."""
    import numpy as np

    from oracle import oracle as orc

    rng = np.random.default_rng(1)
    th = actor.detach().cpu().numpy().astype(np.float64)
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        x = rng.normal(size=(20, 10, 6))
        orc.policy_backward(x, np.ones((20, 10), np.uint8), th, rng.normal(size=(20, 8)))
        n += 20
    el = time.perf_counter() - t0
    return {"value": n / el, "unit": "agent-samples/s", "cores": 1,
            "sample": f"{n} agents of 10 tokens, {el:.1f} s"}


def bench_train_loop(args, T=32, epochs=1, minibatches=16):
    """End-to-end training on the policy workload's shape (16384 envs x 5 x 5):
    one PPO iteration is a closed-loop batch of T steps from an episode start
    (the attention policy driving the environment, exact estimator in the
    loop), then the learner over it (the critic's values of the T + 1 states
    and the behaviour policy's logits from the inference kernels, GAE, and
    `epochs` passes over `minibatches` groups of whole steps: training-form
    forward and reverse passes of actor and critic, Adam on every parameter). Reported: env-steps/s of training = T x envs over the
    iteration's time; the paper's own figure (1e10 single-agent timesteps of
    pre-training in 1.5 days on one H100, Sec. IV-B-2) is context only (another
    GPU, model and batch). One untimed iteration first."""
    import numpy as np
    import torch

    from paper_2505_08222_amd import policy, ppo
    from paper_2505_08222_amd.configs import CONFIGS, env_config
    from paper_2505_08222_amd.env import Env

    c = CONFIGS["policy"]
    E = args.envs or c["num_envs"]
    cfg = env_config("policy")
    na, nt = cfg["n_agents"], cfg["n_targets"]
    env = Env(cfg, E, seed=c["seed"])
    actor, critic = policy.init_params(c["seed"]), policy.init_params(c["seed"] + 1)
    learner = ppo.Learner(actor, critic, na, nt, lr=3e-4)
    roll = policy.PolicyRollout(env, actor)
    rec = ("obs", "obs_mask", "actions", "gstate", "reward", "done")

    def iteration(ep):
        t0 = time.perf_counter()
        r0 = env.reset(ep, record=("obs", "obs_mask", "gstate"))
        out, _ = roll.run(T, episode=ep, record=rec, metrics=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        obs = torch.cat([r0["obs"][None], out["obs"][:T - 1]])
        mask = torch.cat([r0["obs_mask"][None], out["obs_mask"][:T - 1]])
        gs = torch.cat([r0["gstate"][None], out["gstate"]])
        hist = learner.update(obs, mask, out["actions"], gs, out["reward"], out["done"],
                              epochs=epochs, minibatches=minibatches)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, hist

    iteration(0)
    t_roll, t_learn, hist = iteration(1)
    total = t_roll + t_learn
    h = hist.cpu().numpy()
    log(f"[bench] train loop: rollout {t_roll * 1e3:.1f} ms, learner {t_learn * 1e3:.1f} ms, "
        f"{T * E / total:.3g} env-steps/s of training")
    paper = 1e10 / (1.5 * 86400.0)
    return {
        "metric": METRIC, "value": T * E / total, "unit": "env-steps/s of PPO training",
        "n_gpus": 1, "steps": 1, "dtype": "bf16 rollout policy; fp32 learner",
        "data": "closed-loop experience from random-init networks",
        "config": {"workload": f"train loop: {E} envs x {na} agents x {nt} targets, batches of {T} "
                               f"steps from an episode start, {epochs} epoch(s) of {minibatches} "
                               "minibatches, every parameter of actor and critic updated",
                   "envs": E, "batch_steps": T, "epochs": epochs, "minibatches": minibatches},
        "agent_steps_per_s": T * E * na / total,
        "ms": {"rollout": t_roll * 1e3, "learner": t_learn * 1e3, "total": total * 1e3},
        "losses_first_last": [h[0].tolist(), h[-1].tolist()],
        "paper_pretraining_steps_per_s_context": paper,
    }


def cpu_baseline_ppo(critic, actor, budget_s):
    """The oracle's forward half on a bounded sample: 4 envs x 5x5 x 8 steps
    per round (critic and policy forwards in FP64 C, one thread; GAE and the
    objective in numpy), repeated until the budget is used; agent-steps/s."""
    import numpy as np

    from oracle import oracle as orc
    from oracle import ppo_oracle as po

    rng = np.random.default_rng(0)
    E, T, na, nt = 4, 8, 5, 5
    M, n_tok, A = na + nt, 2 * na + nt, E * na
    th_c = critic.detach().cpu().numpy().astype(np.float64)
    th_a = actor.detach().cpu().numpy().astype(np.float64)
    rounds = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        g = rng.normal(size=((T + 1) * E, M, 6))
        g[..., 5] = (np.arange(M) >= na)
        tok = po.critic_tokens(g, na, nt, 1000.0)
        v = orc.policy_forward(tok, np.ones(tok.shape[:2], np.uint8), th_c)[:, 0].reshape(T + 1, E)
        obs = rng.normal(size=(T * A, n_tok, 6))
        lg = orc.policy_forward(obs, np.ones((T * A, n_tok), np.uint8), th_a).reshape(T, A, 8)
        adv, ret = po.gae(rng.random((T, E)), np.zeros((T, E)), v, 0.99, 0.95)
        po.ppo_objective(lg, lg + 0.1, rng.integers(0, 5, (T, A)), adv, v[:T], ret, na, 5, 0.2)
        rounds += 1
    el = time.perf_counter() - t0
    return {"value": rounds * T * A / el, "unit": "agent-steps/s", "cores": 1, "kind": "oracle",
            **host_cpu(),
            "sample": f"{rounds} rounds of {E} envs x 5x5 x {T} steps (critic and policy forwards "
                      f"FP64 C, GAE and objective numpy), {el:.1f} s"}


def bench_policy(args, steps, warmup, mlp="train", cpu_seconds=None):
    """Full rollout with the attention policy: 16384 envs x 5 agents x 5
    targets x 1000 steps, each step = policy forward on every agent's
    observation, then the environment step, captured as one HIP graph.
    `mlp`: trained learned-estimator weights for the loop, "train" to train
    them here, None for the exact estimator."""
    import numpy as np
    import torch

    from paper_2505_08222_amd import policy
    from paper_2505_08222_amd.configs import CONFIGS, env_config
    from paper_2505_08222_amd.env import Env

    c = CONFIGS["policy"]
    cfg = env_config("policy")
    E = args.envs or c["num_envs"]
    T = c["steps"]
    torch.cuda.set_device(0)
    params = policy.init_params(c["seed"])
    if args.no_learned_loop:
        mlp = None
    elif isinstance(mlp, str):
        mlp = train_estimator(args)[0]

    def timed_loop(mlp_params):
        env = Env(cfg, E, seed=c["seed"])
        pr = policy.PolicyRollout(env, params, mlp_params=mlp_params, k_sigma=3.0)
        gout, gm = pr.capture(T, record=("reward", "done"))
        for _ in range(warmup):
            pr.launch()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            pr.launch()
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return env, gm, max(wall, ev0.elapsed_time(ev1) / 1e3)

    env, gm, elapsed = timed_loop(mlp)
    exact_loop = None
    if mlp is not None:
        _, gm_exact, el_exact = timed_loop(None)
        exact_loop = {"env_steps_per_s": E * T * steps / el_exact,
                      "agent_steps_per_s": env.A * T * steps / el_exact,
                      "ms_per_step": el_exact * 1e3 / steps,
                      "mean_reward": float(gm_exact[0] / max(float(gm_exact[6]), 1))}
    stream = torch.cuda.current_stream()
    # the policy kernel alone, on the final observation, timed with events
    n_tok = cfg["n_agents"] + cfg["n_targets"]
    env.reset(0)
    obs = env.rollout(1, record=("obs", "obs_mask"))
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    policy.forward(obs["obs"][0], obs["obs_mask"][0], params, n_tok, cfg["n_agents"])
    torch.cuda.synchronize()
    durs = []
    for _ in range(5):
        a.record(stream)
        policy.forward(obs["obs"][0], obs["obs_mask"][0], params, n_tok, cfg["n_agents"])
        b.record(stream)
        torch.cuda.synchronize()
        durs.append(a.elapsed_time(b))
    pol_ms = float(np.median(durs))
    flops = policy_flops_per_agent_step(n_tok) * env.A
    tflops = flops / (pol_ms / 1e3) / 1e12
    m = gm.cpu().numpy()
    extra = {}
    if cpu_seconds:
        log("[bench] cpu baseline (oracle), policy loop")
        extra["cpu_baseline"] = cpu_baseline_policy(cfg, env, params, cpu_seconds)
    return {
        "metric": METRIC, "value": E * T * steps / elapsed, "unit": "env-steps/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": elapsed * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"policy: {E} envs x 5 agents x 5 targets x {T} steps, attention "
                               "policy (d 64, 4 heads, 2 layers, FFN 256, random init) + env step "
                               + ("with the learned estimator (exact fallback at 3 sigma) in the loop"
                                  if mlp is not None else "with the exact estimator")
                               + " per step, one HIP graph", "envs": E, "episode_steps": T,
                   "estimator": "learned" if mlp is not None else "exact"},
        "exact_estimator_loop": exact_loop,
        "agent_steps_per_s": env.A * T * steps / elapsed,
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": tflops / 2500.0,
                     "traffic": measured_traffic("policy_kernel", "policy") if E == c["num_envs"] else None,
                     "kernel": "policy_kernel",
                     "kernel_ms": pol_ms, "flops_per_launch": flops},
        "episode_metrics": {"mean_reward": float(m[0] / max(m[6], 1)),
                            "crash_steps": float(m[4])},
        **extra,
    }


def bench_env(args, workload, steps, warmup, sweep=False, cpu_seconds=None):
    """A plain-step workload (plain, batched or ragged): the captured graph of
    reset + rollout + metrics, replayed `steps` times after `warmup` replays;
    the dominant kernel (the persistent rollout) timed alone with events on
    its stream for the roofline."""
    import numpy as np
    import torch

    from paper_2505_08222_amd.configs import CONFIGS, env_config
    from paper_2505_08222_amd.env import Env

    c = CONFIGS[workload]
    cfg = env_config(workload)
    E = args.envs or c["num_envs"]
    T = c["steps"]
    torch.cuda.set_device(0)
    log(f"[bench] workload={workload} envs={E} steps/episode={T}")
    env = Env(cfg, E, seed=c["seed"])
    mapping = env.get_mapping()
    if not args.no_autotune:
        env.reset(0)
        cache = os.path.join(ROOT, "gpurun_out", "autotune_cache.jsonl")
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        mapping = env.autotune(probe_steps=min(20, T), cache_path=cache)
        log(f"[bench] autotuned mapping lanes_per_agent={mapping[0]} waves_per_block={mapping[1]}")
    gout, gmetrics = env.capture_graph(T, episode=0, record=RECORD)
    for _ in range(warmup):
        env.launch_graph()
    torch.cuda.synchronize()
    log("[bench] warmup done")
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        env.launch_graph()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    log(f"[bench] timed {steps} graph replays: {gpu_ms:.3f} ms (events), {wall*1e3:.3f} ms wall")
    elapsed = max(wall, gpu_ms / 1e3)
    env_steps = E * T * steps
    value = env_steps / elapsed
    m = gmetrics.cpu().numpy()

    pf = cfg.get("est_kind", 0) == 1
    # dominant kernel: the persistent rollout (the particle filter when it is
    # the tracker), timed alone with events on the stream it is launched on
    out = {k: torch.empty_like(v) for k, v in gout.items()}
    durs = []
    for _ in range(3):
        env.reset(0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        env.rollout(T, record=RECORD, out=out)
        b.record(stream)
        torch.cuda.synchronize()
        durs.append(a.elapsed_time(b))
    kern_ms = float(np.mean(durs))
    bpe = bytes_per_env_step(env.n_agents.astype(np.int64), env.n_targets.astype(np.int64)).sum()
    alg_bytes = float(bpe) * T
    achieved = alg_bytes / (kern_ms / 1e3) / 1e9
    log(f"[bench] rollout {kern_ms:.3f} ms/launch, {alg_bytes/1e6:.1f} MB algorithmic, "
        f"{achieved:.1f} GB/s")

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": elapsed * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{workload}: {E} envs x {T} steps, "
                        + ("agents and targets uniform 1..5 per env"
                           if cfg["ragged"] else f"{cfg['n_agents']} agents x {cfg['n_targets']} targets")
                        + (f", particle filter (64 particles per tracker"
                           + (", pooled ranges" if cfg["pooled"] else "") + ")" if pf else
                           f", window {cfg['window']}")
                        + ", one HIP graph (reset + rollout + metrics)",
            "envs": E, "episode_steps": T, "agents": int(env.A), "targets": int(env.Tt),
            "tokens": int(env.K), "lanes_per_agent": mapping[0], "waves_per_block": mapping[1],
        },
        "agent_steps_per_s": float(env.A) * T * steps / elapsed,
        "hbm_gbps_algorithmic": achieved,
        "rollout_ms_per_launch": kern_ms,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic("rollout_kernel", workload) if E == c["num_envs"] else None,
            "kernel": "rollout_kernel", "kernel_ms": kern_ms, "bytes_per_launch": alg_bytes,
        } if not pf else pf_kernel_roofline(env, cfg, workload, E == c["num_envs"]),
        "episode_metrics": {
            "mean_reward": float(m[0] / max(m[6], 1)),
            "mean_tracking_error_m": float(m[1] / max(m[3], 1)),
            "crash_steps": float(m[4]), "lost_targets": float(m[5]),
        },
    }
    valu = measured_valu("rollout_kernel", workload) if not pf and E == c["num_envs"] else None
    if valu is not None:
        # the VALU view from the committed counters (paper environment: too few
        # wavefronts to fill the chip, so neither HBM nor VALU issue bounds it)
        busy, insts = valu
        ach = busy / (kern_ms / 1e3)
        result["roofline"]["alu_view"] = {
            "bound": "alu", "achieved": ach, "peak": VALU_PEAK_CYCLES,
            "unit": "VALU-busy SIMD cycles/s", "frac": ach / VALU_PEAK_CYCLES,
            "valu_busy_cycles_per_launch": busy, "valu_insts_per_launch": insts}
    if result["roofline"]["traffic"] is not None:
        result["roofline"]["traffic_unit"] = "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)"
        # the measured DRAM bytes over the live launch time, beside the algorithmic rate
        result["roofline"]["traffic_gbps"] = (result["roofline"]["traffic"] /
                                              (result["roofline"]["kernel_ms"] / 1e3) / 1e9)
    if sweep and E == c["num_envs"]:
        del out, gout
        torch.cuda.empty_cache()
        result["sweep"] = env_sweep(args)
    if cpu_seconds:
        log(f"[bench] cpu baseline (oracle), {workload}")
        result["cpu_baseline"] = cpu_baseline(cfg, env, T, cpu_seconds)
    env.close()
    return result


# Table I of the paper (JaxLrauv, its particle filter, 30 s steps; one H100
# by the paper's training setup): steps per second summed over envs, for n
# agents and n targets, n = 1..5.
PAPER_TABLE1_SPS = {128: [68508, 19712, 9128, 5180, 3469], 1024: [81686, 21534, 9786, 5450, 3574]}


def table1_grid(args, steps=5, T=300):
    """The paper's Table I grid on this build: the paper environment with the
    particle-filter tracker over pooled ranges, n agents x n targets, 128 and
    1024 envs; each point one captured graph of reset + T steps, replayed
    `steps` times (HIP events). The paper's SPS beside each point is context
    (another GPU, another filter implementation), not a target."""
    import torch

    from paper_2505_08222_amd.configs import env_config
    from paper_2505_08222_amd.env import Env

    stream = torch.cuda.current_stream()
    points = []
    for E in (128, 1024):
        for n in range(1, 6):
            cfg = env_config("paper_pf", n_agents=n, n_targets=n, ragged=0, episode_len=T)
            env = Env(cfg, E, seed=0)
            out, _ = env.capture_graph(T, episode=0, record=RECORD)
            env.launch_graph()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record(stream)
            for _ in range(steps):
                env.launch_graph()
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / steps
            sps = E * T / (ms / 1e3)
            paper = PAPER_TABLE1_SPS[E][n - 1]
            points.append({"envs": E, "agents": n, "targets": n, "sps": sps,
                           "ms_per_step": ms / T, "paper_sps_h100": paper,
                           "ratio_to_paper": sps / paper})
            log(f"[table1] {E} envs {n}A{n}T: {sps:.3g} SPS ({ms / T * 1e3:.1f} us/step), "
                f"paper {paper}")
            del out, env
    return points


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="all",
                    choices=["all", "plain", "batched", "ragged", "learned", "policy", "paper",
                             "paper_pooled", "learned_paper", "ragged_pf", "paper_pf", "ppo",
                             "train_loop"])
    ap.add_argument("--envs", type=int, default=None, help="override the number of envs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the env-count sweeps (the batched workload's; the Table I grid of "
                         "the paper_pf workload)")
    ap.add_argument("--no-learned-loop", action="store_true",
                    help="policy workload: keep the exact estimator in the loop")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the plain copy kernel used to calibrate HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(environments are independent: a multi-GPU run would shard env ranges)",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        copy_probe()
        return
    cpu_s = None if args.no_cpu_baseline else args.cpu_seconds
    if args.workload in ("learned", "learned_paper"):
        variant = "paper" if args.workload == "learned_paper" else "learned"
        print(json.dumps(bench_learned(args, args.steps, cpu_seconds=cpu_s, variant=variant)),
              flush=True)
        return
    if args.workload == "ppo":
        print(json.dumps(bench_ppo(args, cpu_seconds=cpu_s)), flush=True)
        return
    if args.workload == "train_loop":
        print(json.dumps(bench_train_loop(args)), flush=True)
        return
    if args.workload == "policy":
        print(json.dumps(bench_policy(args, args.steps, args.warmup, cpu_seconds=cpu_s)),
              flush=True)
        return
    if args.workload != "all":
        res = bench_env(args, args.workload, args.steps, args.warmup,
                        sweep=args.workload == "batched" and not args.no_sweep, cpu_seconds=cpu_s)
        if args.workload == "paper_pf" and not args.no_sweep:
            res["table1_grid"] = table1_grid(args)
        print(json.dumps(res), flush=True)
        return
    # headline: the ragged batch, the largest single-GPU configuration
    t_start = time.perf_counter()
    result = bench_env(args, "ragged", args.steps, args.warmup, cpu_seconds=cpu_s)
    # the other workloads, each with its own dominant kernel and CPU baseline;
    # fewer replays for the long closed loop
    sec_cpu = None if cpu_s is None else max(2.0, cpu_s / 2)
    result["batched"] = bench_env(args, "batched", args.steps, args.warmup,
                                  sweep=not args.no_sweep, cpu_seconds=sec_cpu)
    mlp, train_info = train_estimator(args)
    result["learned"] = bench_learned(args, args.steps, cpu_seconds=sec_cpu, trained=(mlp, train_info))
    result["policy"] = bench_policy(args, min(args.steps, 3), min(args.warmup, 1), mlp=mlp,
                                    cpu_seconds=sec_cpu)
    result["ppo"] = bench_ppo(args, cpu_seconds=None if sec_cpu is None else 4.0)
    result["train_loop"] = bench_train_loop(args)
    # the paper's own environment (30 s steps, rudder, follow reward, 450 m
    # detection, pairwise spawn) and the learned estimator on its windows
    result["paper"] = bench_env(args, "paper", args.steps, args.warmup, cpu_seconds=sec_cpu)
    result["paper_pooled"] = bench_env(args, "paper_pooled", args.steps, args.warmup,
                                       cpu_seconds=sec_cpu)
    result["learned_paper"] = bench_learned(args, args.steps, variant="paper")
    # the particle-filter tracker on the ragged batch and on the paper's
    # environment (pooled ranges); fewer replays: each step is three launches
    result["ragged_pf"] = bench_env(args, "ragged_pf", min(args.steps, 3), min(args.warmup, 1),
                                    cpu_seconds=sec_cpu)
    result["paper_pf"] = bench_env(args, "paper_pf", min(args.steps, 5), min(args.warmup, 1),
                                   cpu_seconds=sec_cpu)
    result["paper_pf"]["table1_grid"] = table1_grid(args)
    for k in ("batched", "learned", "policy", "ppo", "paper", "paper_pooled", "learned_paper",
              "ragged_pf", "paper_pf"):
        for key in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
            result[k].pop(key, None)
    result["bench_seconds"] = time.perf_counter() - t_start
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
