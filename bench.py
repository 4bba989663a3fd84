#!/usr/bin/env python3
"""Benchmark of the batched range-only tracking environment on one MI355X.

One benchmark step = one replay of the captured HIP graph {reset, T-step
persistent rollout writing observations, masks, rewards and done flags,
metrics reduction} over the whole batch, inputs resident in HBM. Default
workload: 4096 envs x 2 agents x 2 targets x 500 steps (the plain batched
configuration). Prints one JSON line.
"""
import argparse
import json
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


def cpu_baseline(cfg, env, T, budget_s):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload
    (whole episodes of the first envs in packed order, chunk by chunk, until
    the time budget is used)."""
    import numpy as np

    from oracle import oracle as orc

    threads = min(os.cpu_count() or 1, 16)
    orc.lib()
    ids, na, nt = env.order["env_ids"], env.n_agents, env.n_targets
    chunk = 256
    done_envsteps = 0
    done_envs = 0
    t0 = time.perf_counter()
    k = 0
    while k < len(ids) and time.perf_counter() - t0 < budget_s:
        sl = slice(k, min(k + chunk, len(ids)))
        orc.rollout(cfg, ids[sl], na[sl], nt[sl], env.seed, T,
                    records=("reward", "done", "obs", "obs_mask"), n_threads=threads)
        done_envs += sl.stop - sl.start
        done_envsteps += (sl.stop - sl.start) * T
        k = sl.stop
    el = time.perf_counter() - t0
    return {"value": done_envsteps / el, "unit": "env-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{done_envs} of {len(ids)} envs x {T} steps (whole episodes, same seed and "
                      f"config), FP64 C with OpenMP over envs, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched", choices=["plain", "batched", "ragged"])
    ap.add_argument("--envs", type=int, default=None, help="override the number of envs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(environments are independent: a multi-GPU run would shard env ranges, "
              "see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2505_08222_amd.configs import CONFIGS, env_config
    from paper_2505_08222_amd.env import Env

    c = CONFIGS[args.workload]
    cfg = env_config(args.workload)
    E = args.envs or c["num_envs"]
    T = c["steps"]
    torch.cuda.set_device(0)
    log(f"[bench] workload={args.workload} envs={E} steps/episode={T}")
    env = Env(cfg, E, seed=c["seed"])
    mapping = env.get_mapping()
    if not args.no_autotune:
        env.reset(0)
        cache = os.path.join(ROOT, "gpurun_out", "autotune_cache.jsonl")
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        mapping = env.autotune(probe_steps=min(20, T), cache_path=cache)
        log(f"[bench] autotuned mapping lanes_per_agent={mapping[0]} waves_per_block={mapping[1]}")
    gout, gmetrics = env.capture_graph(T, episode=0, record=RECORD)
    for _ in range(args.warmup):
        env.launch_graph()
    torch.cuda.synchronize()
    log("[bench] warmup done")
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        env.launch_graph()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    log(f"[bench] timed {args.steps} graph replays: {gpu_ms:.3f} ms (events), {wall*1e3:.3f} ms wall")
    elapsed = max(wall, gpu_ms / 1e3)
    env_steps = E * T * args.steps
    value = env_steps / elapsed
    m = gmetrics.cpu().numpy()

    # dominant kernel: the persistent rollout, timed alone with events on the
    # stream it is launched on
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
    log(f"[bench] rollout kernel {kern_ms:.3f} ms/launch, {alg_bytes/1e6:.1f} MB algorithmic, "
        f"{achieved:.1f} GB/s")

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {E} envs x {T} steps, "
                        + ("agents and targets uniform 1..5 per env"
                           if cfg["ragged"] else f"{cfg['n_agents']} agents x {cfg['n_targets']} targets")
                        + f", window {cfg['window']}, one HIP graph (reset + rollout + metrics)",
            "envs": E, "episode_steps": T, "agents": int(env.A), "targets": int(env.Tt),
            "tokens": int(env.K), "lanes_per_agent": mapping[0], "waves_per_block": mapping[1],
        },
        "agent_steps_per_s": float(env.A) * T * args.steps / elapsed,
        "hbm_gbps_algorithmic": achieved,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "rollout_kernel", "kernel_ms": kern_ms, "bytes_per_launch": alg_bytes,
        },
        "episode_metrics": {
            "mean_reward": float(m[0] / max(m[6], 1)),
            "mean_tracking_error_m": float(m[1] / max(m[3], 1)),
            "crash_steps": float(m[4]), "lost_targets": float(m[5]),
        },
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(cfg, env, T, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
