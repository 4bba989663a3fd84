"""Parity of the particle-filter tracker (est_kind 1) with the FP64 oracle.

Teacher-forced: the environment runs one step at a time; before and after
each step the GPU's particles and belief flags are exported through the C
ABI, and every tracker's update is recomputed by the oracle (orc_pf_update)
from the GPU's own particles before the step, the rows the GPU measured
(positions and ranges of its outputs; with pooling, the ranges of the agents
whose broadcast the observing agent received, read off its agent-token
masks), the env's range-noise std and the documented Philox words. Then:

* the belief flag after the step matches exactly; a tracker without belief
  and without a range keeps its particles, estimate and validity bit for bit;
* every particle after the step equals the oracle's moved (or seeded)
  particle that the systematic resampling selected, within the FP32 position
  tolerance below; a particle may instead equal a neighbouring source only
  where the oracle's cumulative weight sits within 1e-2 of the total from the
  resampling point (FP32 and FP64 weights order such near-ties differently),
  and such flips are rare;
* the estimate is the mean of the GPU's particles (an FP32 sum: 1e-5 of the
  largest particle coordinate) and agrees with the oracle's within the
  position tolerance plus the flips' share.

Position tolerance, from the arithmetic: the move x + q z rounds x (FP32,
2^-24 |x|) and takes z from FP32 Box-Muller (hardware log2, sqrt, sin, cos:
a few 1e-7 relative, times |z| <= 6), and the seed's angle 2 pi (k + u) / 64
rounds at 2^-25 revolutions; 4e-6 of (|x| + r + 6 (q + sigma_l)) bounds all of
them with margin.

End to end: a GPU rollout and the oracle's rollout of the same envs, seeds
and policy share every entity trajectory; their filters drift apart only
through near-tie flips, so their tracking-error distributions must agree
(median within 15%).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_08222_amd.configs import env_config  # noqa: E402

pytestmark = pytest.mark.gpu

PF = dict(est_kind=1)
CASES = {
    # name: (config, overrides, envs, steps)
    "ragged": ("ragged", dict(PF, pf_q=1.0, pf_lik_sigma=2.0), 150, 16),
    "ragged_detection": ("ragged", dict(PF, pf_q=1.0, pf_lik_sigma=2.0, det_range=900.0,
                                        comm_range=400.0, comm_loss_p=0.3), 150, 16),
    "paper": ("paper", dict(PF, pf_q=15.0, pf_lik_sigma=5.0), 200, 16),
    "paper_pooled": ("paper", dict(PF, pf_q=15.0, pf_lik_sigma=5.0, pooled=1), 200, 16),
    "fixed_8x8_pooled": ("batched", dict(PF, pf_q=1.0, pf_lik_sigma=2.0, pooled=1, n_agents=8,
                                         n_targets=8, comm_range=2000.0, comm_loss_p=0.2),
                         12, 12),
}
REC = ("gstate", "ranges", "est", "est_valid", "obs_mask")
MARGIN = 1e-2


def _rows(out, o, k, i, j, A, N, pooled):
    """Tracker (i, j) of packed env k: the rows the filter takes this step."""
    gb = o["agent"][k] + o["target"][k]
    others = [m for m in range(A) if m != i]
    rows = []
    for a in [i] + (others if pooled else []):
        heard = a == i or out["obs_mask"][o["token"][k] + i * (A + N) + 1 + others.index(a)] == 1
        r = out["ranges"][o["pair"][k] + a * N + j]
        if heard and r == r:
            rows.append((float(out["gstate"][gb + a, 0]), float(out["gstate"][gb + a, 1]),
                         float(r)))
    return np.array(rows, np.float64).reshape(-1, 3)


def _cum(px, py, rows, sl):
    lw = np.zeros(px.shape[0])
    for ax, ay, r in rows:
        lw -= (np.hypot(px - ax, py - ay) - r) ** 2 / (2 * sl * sl)
    return np.cumsum(np.exp(lw - lw.max()))


def _sigma(orc, env, cfg, episode):
    """Range-noise std of each env (packed order), drawn at reset: the
    oracle's value rounded to FP32, as the GPU computes it from the same word
    (the two may differ in the last bit, far below the tolerances)."""
    o = env.order
    r = orc.rollout(cfg, o["env_ids"], env.n_agents, env.n_targets, env.seed, 0,
                    episode=episode, records=("sigma_r",))
    return r["sigma_r"].astype(np.float32)


def _teacher_forced(orc, env, cfg, T, episode, sig):
    o = env.order
    na, nt, ids = env.n_agents, env.n_targets, o["env_ids"]
    q, pooled = float(cfg["pf_q"]), bool(cfg["pooled"])
    stats = dict(updates=0, resampled=0, flips=0, held=0, worst=0.0, worst_est=0.0)
    for t in range(T):
        bxy, bb = (x.cpu().numpy() for x in env.pf_state())
        out = {k: v.cpu().numpy() for k, v in env.step(record=REC).items()}
        axy, ab = (x.cpu().numpy() for x in env.pf_state())
        for k in range(env.E):
            A, N = int(na[k]), int(nt[k])
            sl = math.sqrt(float(sig[k]) ** 2 + cfg["pf_lik_sigma"] ** 2)
            for i in range(A):
                for j in range(N):
                    p = o["pair"][k] + i * N + j
                    rows = _rows(out, o, k, i, j, A, N, pooled)
                    belief = t > 0 and bb[p] == 1
                    words = orc.pf_words(env.seed, episode, t, int(ids[k]), i, j)
                    bx = bxy[p, :, 0].astype(np.float64)
                    by = bxy[p, :, 1].astype(np.float64)
                    ok, ox, oy, est, src = orc.pf_update(bx, by, belief, rows, sl, q, words)
                    assert bool(ab[p]) == ok, (t, k, i, j, belief, rows)
                    if not ok:
                        np.testing.assert_array_equal(axy[p], bxy[p])
                        stats["held"] += 1
                        continue
                    stats["updates"] += 1
                    first = 0 if belief else 1
                    _, px, py, _, _ = orc.pf_update(bx, by, belief, rows[:first], sl, q, words)
                    gx = axy[p, :, 0].astype(np.float64)
                    gy = axy[p, :, 1].astype(np.float64)
                    rmax = float(np.abs(rows[:, 2]).max()) if len(rows) else 0.0
                    tol = 4e-6 * (np.maximum(np.abs(px), np.abs(py)).max() + rmax + 6 * (q + sl))
                    if (src < 0).all():
                        d = np.maximum(np.abs(gx - px), np.abs(gy - py))
                        assert d.max() <= tol, (t, k, i, j, d.max(), tol)
                        stats["worst"] = max(stats["worst"], float(d.max() / tol))
                        share = 0.0
                    else:
                        stats["resampled"] += 64
                        cum = _cum(px, py, rows[first:], sl)
                        U = orc.u01(words.uoff)
                        share = 0.0
                        d = np.maximum(np.abs(gx - px[src]), np.abs(gy - py[src]))
                        good = d <= tol
                        if good.any():
                            stats["worst"] = max(stats["worst"], float(d[good].max() / tol))
                        for kk in np.flatnonzero(~good):
                            s = int(src[kk])
                            dd = np.maximum(np.abs(gx[kk] - px), np.abs(gy[kk] - py))
                            g = int(np.argmin(dd))
                            assert dd[g] <= tol, (t, k, i, j, kk, "no source matches", dd[g], tol)
                            point = (kk + U) / 64 * cum[-1]
                            lo, hi = min(g, s), max(g, s)
                            gap = np.abs(cum[lo:hi] - point).max() / cum[-1]
                            assert gap <= MARGIN, (t, k, i, j, kk, g, s, gap)
                            stats["flips"] += 1
                            share += math.hypot(px[g] - px[s], py[g] - py[s]) / 64
                    # estimate: the GPU's mean, and the oracle's up to the flips
                    e_gpu = out["est"][p].astype(np.float64)
                    assert out["est_valid"][p] == 1
                    cm = np.array([gx.mean(), gy.mean()])
                    # an FP32 sum of 64 terms: a few ulps of the terms' size
                    scale = max(np.abs(gx).max(), np.abs(gy).max()) + 1.0
                    assert np.abs(e_gpu - cm).max() <= 1e-5 * scale
                    de = np.abs(e_gpu - np.array(est)).max()
                    assert de <= tol + 1e-5 * scale + share, (t, k, i, j, de, tol, share)
                    stats["worst_est"] = max(stats["worst_est"], float(de / (tol + 1e-5 * scale)))
    return stats


@pytest.mark.parametrize("name", list(CASES))
def test_teacher_forced_particle_filter(orc, name):
    from paper_2505_08222_amd.env import Env

    base, over, E, T = CASES[name]
    cfg = env_config(base, episode_len=2 * T, **over)
    env = Env(cfg, E, seed=21)
    env.reset(0)
    st = _teacher_forced(orc, env, cfg, T, 0, _sigma(orc, env, cfg, 0))
    # a second episode: stale beliefs of the first must not carry over
    env.reset(1)
    st2 = _teacher_forced(orc, env, cfg, 3, 1, _sigma(orc, env, cfg, 1))
    for key in ("updates", "resampled", "flips", "held"):
        st[key] += st2[key]
    print(f"{name}: {st}")
    assert st["updates"] > 0
    assert st["flips"] <= max(4, st["resampled"] // 500), st
    env.close()


@pytest.mark.parametrize("name,over,E,T", [
    ("ragged", dict(pf_q=1.0, pf_lik_sigma=2.0), 512, 60),
    ("paper", dict(pf_q=15.0, pf_lik_sigma=5.0, pooled=1), 512, 40),
])
def test_rollout_tracking_error_matches_oracle(orc, name, over, E, T):
    from paper_2505_08222_amd.env import Env

    cfg = env_config(name, est_kind=1, episode_len=T, **over)
    env = Env(cfg, E, seed=4)
    env.reset(0)
    out = env.rollout(T, record=("err",))
    err_g = out["err"].cpu().numpy().astype(np.float64)  # [T, Tt] packed order
    o = env.order
    ref = orc.rollout(cfg, o["env_ids"], env.n_agents, env.n_targets, env.seed, T,
                      records=("err",), n_threads=8)
    err_o = ref["err"]  # same env order as given
    for lo, hi in ((0, T // 3), (T // 3, T)):
        g = err_g[lo:hi]
        r = err_o[lo:hi]
        assert np.isfinite(g).mean() == pytest.approx(np.isfinite(r).mean(), abs=0.02)
        mg = np.median(g[np.isfinite(g)])
        mr = np.median(r[np.isfinite(r)])
        print(f"{name} steps {lo}-{hi}: median error gpu {mg:.2f} oracle {mr:.2f}")
        assert abs(mg - mr) <= 0.15 * mr
    env.close()


def test_graph_replays_match_eager():
    """The captured rollout (reset, then per step: move half, filter, observe
    half) replays to the same bits as the eager calls, replay after replay."""
    from paper_2505_08222_amd.env import Env

    cfg = env_config("paper", est_kind=1, pf_q=15.0, pf_lik_sigma=5.0, pooled=1, episode_len=12)
    env = Env(cfg, 300, seed=8)
    env.reset(0)
    eager = env.rollout(12, record=("reward", "est", "est_valid", "obs"))
    eager = {k: v.clone() for k, v in eager.items()}
    out, _ = env.capture_graph(12, episode=0, record=("reward", "est", "est_valid", "obs"))
    for rep in range(3):
        env.launch_graph()
        torch.cuda.synchronize()
        for k in eager:
            assert torch.equal(out[k], eager[k]), (rep, k)
        # eager work between replays
        env.reset(0)
        env.rollout(5, record=("reward",))
        torch.cuda.synchronize()
    env.close()
