// Host runtime of the C ABI declared in include/mi_lrauv.h: batch packing,
// workspace layout, kernel dispatch, HIP graph capture and the mapping
// autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "env_internal.h"
#include "learned_internal.h"
#include "mi_lrauv.h"
#include "policy_internal.h"

#ifndef MIL_CODE_VERSION
#define MIL_CODE_VERSION "dev"
#endif

namespace {

thread_local std::string g_last_error = "no error";

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_CHECK(call)                                                                   \
  do {                                                                                    \
    hipError_t _e = (call);                                                               \
    if (_e != hipSuccess)                                                                 \
      return fail(MIL_EHIP, "%s failed: %s", #call, hipGetErrorString(_e));               \
  } while (0)

// Host copy of Philox4x32-10 (same definition as the device one, Salmon et
// al. SC'11) for the per-env counts drawn at creation time.
void philox_host(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

}  // namespace

struct mil_env {
  mil_env_params P{};
  int64_t E = 0;
  uint64_t seed = 0;
  int W = 0, max_a = 0, max_t = 0, size_class = 0, wcap = 0;
  std::vector<int64_t> env_ids;            // packed -> global id
  std::vector<uint8_t> na, nt;             // packed
  std::vector<int64_t> aoff, toff, poff, koff;
  struct Cls {
    int na, nt;
    int64_t env0, nenv;
  };
  std::vector<Cls> cls;
  int G = 1, wpb = 1;
  int32_t sched = 0;  // rollout schedule: -1 static, 0 automatic, > 0 chunk steps
  std::vector<mil::ClassInfo> cinfo;
  std::vector<uint8_t> wave_class;
  int num_waves = 0, max_waves = 0;
  // workspace
  char *ws = nullptr;
  int64_t ws_bytes = 0;
  struct {
    int64_t env_id, cnt_a, cnt_t, aoff, toff, poff, koff, classes, wave_class, queue, mpart;
    int64_t ax, ay, apsi, arud, tx, ty, tpsi, tv, sigma, hx, hy, hr, hrec, ex, ey, ev, macc, miacc;
    int64_t pmeta, pfxy, pfb, pfm;  // particle filter (est_kind 1)
    int64_t state_begin, state_end, status, snap, devstate, total;
  } off{};
  mil::DevParams dp{};
  mil::DevState ds{};
  int64_t t = -1;  // steps since reset; -1 before the first reset
  uint32_t episode = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int32_t graph_T = 0;
  // particle filter: the batch steps as two halves on two streams, so that
  // one half's filter (VALU-bound) overlaps the other half's rollout launches
  // (latency-bound)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int split_wave = 0;      // first wavefront group of the second half; 0: no split
  int64_t split_pair = 0;  // its first tracker
};

namespace {

bool valid_params(const mil_env_params *p, std::string &why) {
  auto bad = [&](const char *m) {
    why = m;
    return false;
  };
  if (p->n_agents < 1 || p->n_agents > MIL_MAX_AGENTS) return bad("n_agents must be in 1..8");
  if (p->n_targets < 1 || p->n_targets > MIL_MAX_TARGETS) return bad("n_targets must be in 1..8");
  if (p->ragged != 0 && p->ragged != 1) return bad("ragged must be 0 or 1");
  if (p->window < 3 || p->window > MIL_MAX_WINDOW) return bad("window must be in 3..16");
  if (p->episode_len < 1) return bad("episode_len must be >= 1");
  if (p->n_actions < 1 || p->n_actions > MIL_MAX_ACTIONS) return bad("n_actions must be in 1..8");
  if (p->gn_iters < 0 || p->gn_iters > 64) return bad("gn_iters must be in 0..64");
  if (!(p->dt > 0.f) || !(p->agent_speed >= 0.f)) return bad("dt must be > 0, agent_speed >= 0");
  if (!(p->area > 0.f) || !(p->spawn_agent_radius >= 0.f)) return bad("bad spawn geometry");
  if (!(p->target_speed_lo <= p->target_speed_hi) || !(p->range_sigma_lo <= p->range_sigma_hi))
    return bad("speed / range-sigma ranges need lo <= hi");
  if (!(p->range_sigma_lo >= 0.f) || !(p->target_speed_lo >= 0.f)) return bad("negative lo bound");
  if (!(p->eps_min < p->eps_max)) return bad("eps_min must be < eps_max");
  if (!(p->comm_loss_p >= 0.f && p->comm_loss_p <= 1.f)) return bad("comm_loss_p in [0,1]");
  if (!(p->guard_tau >= 0.f)) return bad("guard_tau must be >= 0");
  if (p->action_mode != 0 && p->action_mode != 1) return bad("action_mode must be 0 or 1");
  if (p->action_mode == 1 &&
      (p->n_actions != 3 || p->n_rudder < 1 || p->n_rudder > MIL_MAX_ACTIONS))
    return bad("rudder actions need n_actions = 3 and n_rudder in 1..8");
  if (p->reward_mode != 0 && p->reward_mode != 1) return bad("reward_mode must be 0 or 1");
  if (p->spawn_mode != 0 && p->spawn_mode != 1) return bad("spawn_mode must be 0 or 1");
  if (p->pooled != 0 && p->pooled != 1) return bad("pooled must be 0 or 1");
  if (p->pooled == 1 && p->gn_iters != 0)
    return bad("the pooled tracker is the linearised solve: gn_iters must be 0");
  if (p->est_kind != 0 && p->est_kind != 1) return bad("est_kind must be 0 or 1");
  if (p->est_kind == 1 && !(p->pf_q >= 0.f && p->pf_q < INFINITY && p->pf_lik_sigma >= 0.f &&
                            p->pf_lik_sigma < INFINITY))
    return bad("the particle filter needs finite pf_q >= 0 and pf_lik_sigma >= 0");
  if (p->spawn_mode == 1 &&
      (p->n_agents + p->n_targets > 13 || !(p->spawn_min >= 0.f) ||
       !((double)p->spawn_max >= 2.0 * std::sqrt(3.0) * (double)p->spawn_min)))
    return bad("pairwise spawn needs n_agents + n_targets <= 13 and "
               "spawn_max >= 2 sqrt(3) spawn_min");
  return true;
}

void build_waves(mil_env *h) {
  h->cinfo.clear();
  h->wave_class.clear();
  int wave = 0;
  for (size_t c = 0; c < h->cls.size(); ++c) {
    const auto &k = h->cls[c];
    const int epw = 64 / (k.na * h->G);
    const int64_t nw = (k.nenv + epw - 1) / epw;
    mil::ClassInfo ci{};
    ci.env0 = k.env0;
    ci.nenv = k.nenv;
    ci.aoff0 = h->aoff[k.env0];
    ci.toff0 = h->toff[k.env0];
    ci.poff0 = h->poff[k.env0];
    ci.koff0 = h->koff[k.env0];
    ci.na = k.na;
    ci.nt = k.nt;
    ci.wave0 = wave;
    ci.nwaves = (int32_t)nw;
    h->cinfo.push_back(ci);
    for (int64_t w = 0; w < nw; ++w) h->wave_class.push_back((uint8_t)c);
    wave += (int)nw;
  }
  h->num_waves = wave;
  // the filter's halves: the first wavefront group whose envs start at or
  // past half of the trackers
  h->split_wave = 0;
  h->split_pair = 0;
  if (h->P.est_kind == 1) {
    const int64_t P = h->poff[h->E];
    for (int w = 1; w < h->num_waves; ++w) {
      const auto &ci = h->cinfo[h->wave_class[w]];
      const int64_t e = ci.env0 + (int64_t)(w - ci.wave0) * (64 / (ci.na * h->G));
      if (2 * h->poff[e] >= P) {
        h->split_wave = w;
        h->split_pair = h->poff[e];
        break;
      }
    }
  }
}

int upload_mapping(mil_env *h, hipStream_t st) {
  build_waves(h);
  if (h->num_waves > h->max_waves) return fail(MIL_EINVAL, "wave table overflow");
  HIP_CHECK(hipMemcpyAsync(h->ws + h->off.classes, h->cinfo.data(),
                           h->cinfo.size() * sizeof(mil::ClassInfo), hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(h->ws + h->off.wave_class, h->wave_class.data(), h->wave_class.size(),
                           hipMemcpyHostToDevice, st));
  HIP_CHECK(hipStreamSynchronize(st));
  return MIL_OK;
}

void fill_dev_params(mil_env *h) {
  auto &d = h->dp;
  const auto &p = h->P;
  d.window = p.window;
  d.episode_len = p.episode_len;
  d.n_actions = p.n_actions;
  d.gn_iters = p.gn_iters;
  d.dt = p.dt;
  d.agent_speed = p.agent_speed;
  d.area = p.area;
  d.spawn_r = p.spawn_agent_radius;
  for (int k = 0; k < 8; ++k) d.dpsi[k] = p.action_dpsi[k];
  d.sig_a = p.agent_heading_sigma;
  d.sig_t = p.target_heading_sigma;
  d.tv_lo = p.target_speed_lo;
  d.tv_hi = p.target_speed_hi;
  d.sr_lo = p.range_sigma_lo;
  d.sr_hi = p.range_sigma_hi;
  d.det_range = p.det_range;
  d.comm_range = p.comm_range;
  d.comm_loss_p = p.comm_loss_p;
  d.eps_min = p.eps_min;
  d.eps_max = p.eps_max;
  d.d_safe = p.d_safe;
  d.tau = p.guard_tau;
  d.lost_range = p.lost_range;
  d.key0 = (uint32_t)h->seed;
  d.key1 = (uint32_t)(h->seed >> 32);
  d.action_mode = p.action_mode;
  d.n_rudder = p.n_rudder;
  d.reward_mode = p.reward_mode;
  d.spawn_mode = p.spawn_mode;
  d.d_follow = p.d_follow;
  d.spawn_min = p.spawn_min;
  d.spawn_max = p.spawn_max;
  d.pooled = p.pooled;
  // the filter takes only the newest entry: the kernels keep a window of one
  if (p.est_kind == 1) d.window = 1;
  d.est_kind = p.est_kind;
  d.pf_q = p.pf_q;
  d.pf_lik_sigma = p.pf_lik_sigma;
}

mil::DevOut dev_out(const mil_env_outputs *o) {
  mil::DevOut d{};
  if (!o) return d;
  d.obs = o->obs;
  d.obs_mask = o->obs_mask;
  d.reward = o->reward;
  d.done = o->done;
  d.est = o->est;
  d.est_valid = o->est_valid;
  d.gstate = o->gstate;
  d.actions = o->actions;
  d.ranges = o->ranges;
  d.err = o->err;
  return d;
}

int check_outputs(const mil_env_outputs *o) {
  if (!o) return MIL_OK;
  const void *fl[] = {o->obs, o->reward, o->est, o->gstate, o->actions, o->ranges, o->err};
  for (const void *q : fl)
    if (q && (((uintptr_t)q) & 7)) return fail(MIL_EALIGN, "output arrays must be 8-byte aligned");
  return MIL_OK;
}

// Step k's slice of step-major outputs [T][...].
mil::DevOut step_slice(const mil_env *h, const mil::DevOut &o, int64_t k) {
  const int64_t E = h->E, A = h->aoff[E], Tt = h->toff[E], P = h->poff[E], K = h->koff[E];
  auto at = [&](auto *q, int64_t per) { return q ? q + k * per : q; };
  mil::DevOut s = o;
  s.obs = at(o.obs, K * 6);
  s.obs_mask = at(o.obs_mask, K);
  s.reward = at(o.reward, E);
  s.done = at(o.done, E);
  s.est = at(o.est, P * 2);
  s.est_valid = at(o.est_valid, P);
  s.gstate = at(o.gstate, (A + Tt) * 6);
  s.actions = at(o.actions, A);
  s.ranges = at(o.ranges, P);
  s.err = at(o.err, Tt);
  return s;
}

// T steps from step t0 (outputs and actions step-major from the first). The
// least-squares trackers run inside the persistent rollout kernel; with the
// particle filter every step is the kernel's move half (which also hands each
// tracker's newest range to the filter), the filter, and the observe half.
int launch_steps(mil_env *h, int32_t t0, int32_t T, uint32_t episode, const int32_t *d_actions,
                 const mil::DevOut &o, hipStream_t st, int32_t sched) {
  const mil::DevState *dstate = (const mil::DevState *)(h->ws + h->off.devstate);
  if (h->P.est_kind == 0)
    return mil::launch_rollout(h->size_class, h->wcap, h->G, h->wpb, h->num_waves, h->dp, h->ds,
                               dstate, t0, T, episode, d_actions, o, st,
                               mil::DevExt{0, nullptr, nullptr}, sched);
  sched = -1;  // one or two steps per launch: the static schedule
  // per half: move(t0), filter(t0), then per step [observe(t), move(t + 1)]
  // in one launch and filter(t + 1), and observe(t0 + T - 1) last
  const int64_t A = h->aoff[h->E];
  auto act_at = [&](int32_t k) { return d_actions ? d_actions + (int64_t)k * A : nullptr; };
  const bool split = h->side && h->split_wave > 0;
  const int halves = split ? 2 : 1;
  hipStream_t sts[2] = {st, h->side};
  const int wave_begin[2] = {0, h->split_wave};
  const int wave_end[2] = {split ? h->split_wave : h->num_waves, h->num_waves};
  const int64_t pair_begin[2] = {0, h->split_pair};
  const int64_t pair_end[2] = {split ? h->split_pair : -1, -1};
  if (split) {
    if (hipEventRecord(h->ev_fork, st) != hipSuccess ||
        hipStreamWaitEvent(h->side, h->ev_fork, 0) != hipSuccess)
      return -1;
  }
  int rc = 0;
  for (int g = 0; g < halves && !rc; ++g) {
    mil::DevExt move{1, nullptr, nullptr};
    move.meas = h->ds.pfm;
    move.wave0 = wave_begin[g];
    mil::DevExt both{3, nullptr, nullptr};
    both.meas = h->ds.pfm;
    both.wave0 = wave_begin[g];
    mil::DevExt observe{2, nullptr, nullptr};
    observe.wave0 = wave_begin[g];
    auto roll = [&](int32_t t, int32_t n, int32_t k, const mil::DevExt &ext) {
      return mil::launch_rollout(h->size_class, h->wcap, h->G, h->wpb, wave_end[g], h->dp, h->ds,
                                 dstate, t, n, episode, act_at(k), step_slice(h, o, k), sts[g],
                                 ext, sched);
    };
    auto filter = [&](int32_t t) {
      return mil::launch_pf(h->dp, h->ds, t, episode, sts[g], pair_begin[g], pair_end[g]);
    };
    rc = roll(t0, 1, 0, move);
    if (!rc) rc = filter(t0);
    for (int32_t k = 0; k + 1 < T && !rc; ++k) {
      rc = roll(t0 + k, 2, k, both);
      if (!rc) rc = filter(t0 + k + 1);
    }
    if (!rc) rc = roll(t0 + T - 1, 1, T - 1, observe);
  }
  if (split) {
    // join even after a failed launch, so that a capture can end cleanly
    if (hipEventRecord(h->ev_join, h->side) != hipSuccess ||
        hipStreamWaitEvent(st, h->ev_join, 0) != hipSuccess)
      return -1;
  }
  return rc;
}

int run_rollout(mil_env *h, int32_t T, const int32_t *d_actions, const mil_env_outputs *outs,
                hipStream_t st, int32_t sched) {
  const int rc = launch_steps(h, (int32_t)h->t, T, h->episode, d_actions, dev_out(outs), st, sched);
  if (rc == -2) return fail(MIL_EINVAL, "no kernel for size class %d / window %d", h->size_class,
                            h->wcap);
  if (rc != 0) return fail(MIL_EHIP, "rollout launch failed: %s",
                           hipGetErrorString(hipGetLastError()));
  return MIL_OK;
}

std::string device_key(mil_env *h) {
  int dev = 0;
  hipGetDevice(&dev);
  hipDeviceProp_t prop{};
  hipGetDeviceProperties(&prop, dev);
  std::ostringstream k;
  k << prop.gcnArchName << "/" << prop.multiProcessorCount << "|E" << h->E << "|W" << h->W
    << "|gn" << h->P.gn_iters << "|S" << h->size_class;
  for (auto &c : h->cls) k << "|" << c.na << "x" << c.nt << ":" << c.nenv;
  k << "|" << MIL_CODE_VERSION;
  return k.str();
}

}  // namespace

extern "C" {

const char *env_last_error(void) { return g_last_error.c_str(); }

// Shared with the learned-part ABI in the same library.
int mil_set_error(int code, const char *msg) { return fail(code, "%s", msg); }

int env_create(const mil_env_params *params, int64_t num_envs, uint64_t seed,
               const int32_t *counts, mil_env **out) {
  if (!params || !out) return fail(MIL_EINVAL, "null argument");
  *out = nullptr;
  std::string why;
  if (!valid_params(params, why)) return fail(MIL_EINVAL, "%s", why.c_str());
  if (num_envs < 1 || num_envs > (int64_t(1) << 31))
    return fail(MIL_EINVAL, "num_envs must be in 1..2^31");
  mil_env *h = new (std::nothrow) mil_env();
  if (!h) return fail(MIL_ENOMEM, "out of host memory");
  h->P = *params;
  h->E = num_envs;
  h->seed = seed;
  h->W = params->window;
  // per-env counts (global id order)
  std::vector<uint8_t> ga(num_envs), gt(num_envs);
  for (int64_t e = 0; e < num_envs; ++e) {
    int a = params->n_agents, b = params->n_targets;
    if (counts) {
      a = counts[e];
      b = counts[num_envs + e];
      if (a < 1 || a > params->n_agents || b < 1 || b > params->n_targets) {
        delete h;
        return fail(MIL_EINVAL, "counts of env %lld outside 1..max", (long long)e);
      }
    } else if (params->ragged) {
      const uint32_t ctr[4] = {0u, (uint32_t)e, 0u, 3u /* config purpose */};
      uint32_t x[4];
      philox_host(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), x);
      a = 1 + (int)(((uint64_t)x[0] * (uint32_t)params->n_agents) >> 32);
      b = 1 + (int)(((uint64_t)x[1] * (uint32_t)params->n_targets) >> 32);
    }
    ga[e] = (uint8_t)a;
    gt[e] = (uint8_t)b;
  }
  // packing: classes by (targets desc, agents desc) -- heavier wavefronts are
  // dispatched first; inside a class, global id order
  std::vector<int64_t> order(num_envs);
  for (int64_t e = 0; e < num_envs; ++e) order[e] = e;
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    if (gt[x] != gt[y]) return gt[x] > gt[y];
    return ga[x] > ga[y];
  });
  h->env_ids = order;
  h->na.resize(num_envs);
  h->nt.resize(num_envs);
  h->aoff.assign(num_envs + 1, 0);
  h->toff.assign(num_envs + 1, 0);
  h->poff.assign(num_envs + 1, 0);
  h->koff.assign(num_envs + 1, 0);
  for (int64_t k = 0; k < num_envs; ++k) {
    const int a = ga[order[k]], b = gt[order[k]];
    h->na[k] = (uint8_t)a;
    h->nt[k] = (uint8_t)b;
    h->max_a = std::max(h->max_a, a);
    h->max_t = std::max(h->max_t, b);
    h->aoff[k + 1] = h->aoff[k] + a;
    h->toff[k + 1] = h->toff[k] + b;
    h->poff[k + 1] = h->poff[k] + (int64_t)a * b;
    h->koff[k + 1] = h->koff[k] + (int64_t)a * (a + b);
    if (h->cls.empty() || h->cls.back().na != a || h->cls.back().nt != b)
      h->cls.push_back({a, b, k, 0});
    h->cls.back().nenv += 1;
  }
  const int m = std::max(h->max_a, h->max_t);
  h->size_class = m <= 2 ? 2 : (m <= 5 ? 5 : 8);
  h->wcap = (h->W <= 10 && h->size_class < 8) ? 10 : 16;
  if (params->est_kind == 1) h->wcap = 1;  // the filter keeps only the newest entry
  // wave-table capacity: the largest count over the supported mappings
  for (int G = 1; G <= 2; ++G) {
    int64_t nw = 0;
    for (auto &c : h->cls) {
      const int epw = 64 / (c.na * G);
      nw += (c.nenv + epw - 1) / epw;
    }
    h->max_waves = (int)std::max<int64_t>(h->max_waves, nw);
  }
  h->G = 1;
  h->wpb = 1;
  build_waves(h);
  // workspace layout
  const int64_t E = num_envs, A = h->aoff[E], Tt = h->toff[E], P = h->poff[E];
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    const int64_t at = o;
    o = align256(o + bytes);
    return at;
  };
  auto &f = h->off;
  f.env_id = take(E * 4);
  f.cnt_a = take(E);
  f.cnt_t = take(E);
  f.aoff = take((E + 1) * 8);
  f.toff = take((E + 1) * 8);
  f.poff = take((E + 1) * 8);
  f.koff = take((E + 1) * 8);
  f.classes = take((int64_t)h->cls.size() * sizeof(mil::ClassInfo));
  f.wave_class = take(h->max_waves);
  f.queue = take(((int64_t)h->max_waves + 1) * 4);
  f.mpart = take((int64_t)mil::kMetricBlocks * 6 * 8);
  f.status = take(256);
  f.devstate = take(sizeof(mil::DevState));
  const bool pf = params->est_kind == 1;
  f.pmeta = take(pf ? P * 16 : 0);
  f.pfm = take(pf ? P * 16 : 0);
  f.state_begin = o;
  f.ax = take(A * 4);
  f.ay = take(A * 4);
  f.apsi = take(A * 4);
  f.arud = take(A * 4);
  f.tx = take(Tt * 4);
  f.ty = take(Tt * 4);
  f.tpsi = take(Tt * 4);
  f.tv = take(Tt * 4);
  f.sigma = take(E * 4);
  f.hx = take((int64_t)h->W * A * 4);
  f.hy = take((int64_t)h->W * A * 4);
  f.hr = take((int64_t)h->W * P * 4);
  f.hrec = take((int64_t)h->W * A);
  f.ex = take(P * 4);
  f.ey = take(P * 4);
  f.ev = take(P);
  f.macc = take(E * 3 * 8);
  f.miacc = take(E * 2 * 4);
  f.pfxy = take(pf ? P * mil::kPfParticles * 8 : 0);
  f.pfb = take(pf ? P : 0);
  f.state_end = o;
  f.snap = take(f.state_end - f.state_begin);
  f.total = o;
  fill_dev_params(h);
  *out = h;
  return MIL_OK;
}

int env_query_layout(const mil_env *h, mil_env_layout *out) {
  if (!h || !out) return fail(MIL_EINVAL, "null argument");
  out->num_envs = h->E;
  out->num_agents = h->aoff[h->E];
  out->num_targets = h->toff[h->E];
  out->num_pairs = h->poff[h->E];
  out->num_tokens = h->koff[h->E];
  out->num_entities = out->num_agents + out->num_targets;
  out->workspace_bytes = h->off.total;
  out->window = h->W;
  out->num_classes = (int32_t)h->cls.size();
  return MIL_OK;
}

int env_get_order(const mil_env *h, int64_t *env_ids, int64_t *agent_off, int64_t *target_off,
                  int64_t *pair_off, int64_t *token_off) {
  if (!h) return fail(MIL_EINVAL, "null handle");
  const size_t n1 = (size_t)h->E + 1;
  if (env_ids) std::copy(h->env_ids.begin(), h->env_ids.end(), env_ids);
  if (agent_off) std::copy(h->aoff.begin(), h->aoff.begin() + n1, agent_off);
  if (target_off) std::copy(h->toff.begin(), h->toff.begin() + n1, target_off);
  if (pair_off) std::copy(h->poff.begin(), h->poff.begin() + n1, pair_off);
  if (token_off) std::copy(h->koff.begin(), h->koff.begin() + n1, token_off);
  return MIL_OK;
}

int env_bind(mil_env *h, void *d_workspace, int64_t bytes, void *stream) {
  if (!h || !d_workspace) return fail(MIL_EINVAL, "null argument");
  if (((uintptr_t)d_workspace) & 255) return fail(MIL_EALIGN, "workspace must be 256-byte aligned");
  if (bytes < h->off.total)
    return fail(MIL_ESHAPE, "workspace has %lld bytes, %lld needed", (long long)bytes,
                (long long)h->off.total);
  hipStream_t st = (hipStream_t)stream;
  h->ws = (char *)d_workspace;
  h->ws_bytes = bytes;
  const int64_t E = h->E;
  std::vector<uint32_t> ids(E);
  for (int64_t k = 0; k < E; ++k) ids[k] = (uint32_t)h->env_ids[k];
  HIP_CHECK(hipMemcpyAsync(h->ws + h->off.env_id, ids.data(), E * 4, hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(h->ws + h->off.cnt_a, h->na.data(), E, hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(h->ws + h->off.cnt_t, h->nt.data(), E, hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(h->ws + h->off.aoff, h->aoff.data(), (E + 1) * 8, hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(h->ws + h->off.toff, h->toff.data(), (E + 1) * 8, hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(h->ws + h->off.poff, h->poff.data(), (E + 1) * 8, hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(h->ws + h->off.koff, h->koff.data(), (E + 1) * 8, hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemsetAsync(h->ws + h->off.status, 0, 256, st));
  auto &d = h->ds;
  auto F = [&](int64_t off) { return (float *)(h->ws + off); };
  d.env_id = (const uint32_t *)(h->ws + h->off.env_id);
  d.cnt_a = (const uint8_t *)(h->ws + h->off.cnt_a);
  d.cnt_t = (const uint8_t *)(h->ws + h->off.cnt_t);
  d.aoff = (const int64_t *)(h->ws + h->off.aoff);
  d.toff = (const int64_t *)(h->ws + h->off.toff);
  d.poff = (const int64_t *)(h->ws + h->off.poff);
  d.koff = (const int64_t *)(h->ws + h->off.koff);
  d.classes = (const mil::ClassInfo *)(h->ws + h->off.classes);
  d.wave_class = (const uint8_t *)(h->ws + h->off.wave_class);
  d.ax = F(h->off.ax);
  d.ay = F(h->off.ay);
  d.apsi = F(h->off.apsi);
  d.arud = (int32_t *)(h->ws + h->off.arud);
  d.tx = F(h->off.tx);
  d.ty = F(h->off.ty);
  d.tpsi = F(h->off.tpsi);
  d.tv = F(h->off.tv);
  d.sigma = F(h->off.sigma);
  d.hx = F(h->off.hx);
  d.hy = F(h->off.hy);
  d.hr = F(h->off.hr);
  d.hrec = (uint8_t *)(h->ws + h->off.hrec);
  d.ex = F(h->off.ex);
  d.ey = F(h->off.ey);
  d.ev = (uint8_t *)(h->ws + h->off.ev);
  d.macc = (double *)(h->ws + h->off.macc);
  d.miacc = (int32_t *)(h->ws + h->off.miacc);
  d.status = (uint32_t *)(h->ws + h->off.status);
  d.queue = (int32_t *)(h->ws + h->off.queue);
  d.mpart = (double *)(h->ws + h->off.mpart);
  const bool pf = h->P.est_kind == 1;
  if (pf && !h->side) {
    HIP_CHECK(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
    HIP_CHECK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
  }
  d.pmeta = pf ? (const uint32_t *)(h->ws + h->off.pmeta) : nullptr;
  d.pfxy = pf ? F(h->off.pfxy) : nullptr;
  d.pfb = pf ? (uint8_t *)(h->ws + h->off.pfb) : nullptr;
  d.pfm = pf ? F(h->off.pfm) : nullptr;
  if (pf) {
    // each tracker's env, (agent, target) code and counts, global agent index
    std::vector<uint32_t> meta((size_t)h->poff[E] * 4);
    for (int64_t k = 0; k < E; ++k)
      for (int i = 0; i < h->na[k]; ++i)
        for (int j = 0; j < h->nt[k]; ++j) {
          const int64_t q = h->poff[k] + (int64_t)i * h->nt[k] + j;
          meta[4 * q] = (uint32_t)k;
          meta[4 * q + 1] = (uint32_t)(8 * i + j) | ((uint32_t)h->na[k] << 8) |
                            ((uint32_t)h->nt[k] << 12);
          meta[4 * q + 2] = (uint32_t)(h->aoff[k] + i);
          meta[4 * q + 3] = 0u;
        }
    HIP_CHECK(hipMemcpyAsync(h->ws + h->off.pmeta, meta.data(), meta.size() * 4,
                             hipMemcpyHostToDevice, st));
    HIP_CHECK(hipStreamSynchronize(st));  // `meta` is a host temporary
  }
  d.E = E;
  d.A = h->aoff[E];
  d.Tt = h->toff[E];
  d.P = h->poff[E];
  d.K = h->koff[E];
  HIP_CHECK(hipMemcpyAsync(h->ws + h->off.devstate, &h->ds, sizeof(mil::DevState),
                           hipMemcpyHostToDevice, st));
  const int rc = upload_mapping(h, st);
  if (rc) return rc;
  h->t = -1;
  return MIL_OK;
}

int env_reset(mil_env *h, uint64_t episode, const mil_env_outputs *outs, void *stream) {
  if (!h) return fail(MIL_EINVAL, "null handle");
  if (!h->ws) return fail(MIL_ESTATE, "env_bind has not been called");
  if (episode >= (1ull << 28)) return fail(MIL_EINVAL, "episode must be < 2^28");
  int rc = check_outputs(outs);
  if (rc) return rc;
  h->episode = (uint32_t)episode;
  if (mil::launch_reset(h->dp, h->ds, h->episode, dev_out(outs), stream))
    return fail(MIL_EHIP, "reset launch failed: %s", hipGetErrorString(hipGetLastError()));
  h->t = 0;
  return MIL_OK;
}

int env_step(mil_env *h, const int32_t *d_actions, const mil_env_outputs *outs, void *stream) {
  return env_rollout(h, 1, d_actions, outs, stream);
}

int env_rollout(mil_env *h, int32_t T, const int32_t *d_actions, const mil_env_outputs *outs,
                void *stream) {
  if (!h) return fail(MIL_EINVAL, "null handle");
  if (!h->ws || h->t < 0) return fail(MIL_ESTATE, "env_reset has not been called");
  if (T < 0) return fail(MIL_EINVAL, "T must be >= 0");
  if (h->t + T > h->P.episode_len)
    return fail(MIL_ESTATE, "%d steps from step %lld pass the episode length %d", T,
                (long long)h->t, h->P.episode_len);
  int rc = check_outputs(outs);
  if (rc) return rc;
  if (T == 0) return MIL_OK;
  rc = run_rollout(h, T, d_actions, outs, (hipStream_t)stream, h->sched);
  if (rc) return rc;
  h->t += T;
  return MIL_OK;
}

int env_metrics(mil_env *h, double *d_metrics, void *stream) {
  if (!h || !d_metrics) return fail(MIL_EINVAL, "null argument");
  if (!h->ws || h->t < 0) return fail(MIL_ESTATE, "env_reset has not been called");
  if (mil::launch_metrics(h->dp, h->ds, (int32_t)h->t, d_metrics, stream))
    return fail(MIL_EHIP, "metrics launch failed");
  return MIL_OK;
}

int env_graph_capture(mil_env *h, uint64_t episode, int32_t T, const mil_env_outputs *outs,
                      double *d_metrics, void *stream) {
  if (!h) return fail(MIL_EINVAL, "null handle");
  if (!h->ws) return fail(MIL_ESTATE, "env_bind has not been called");
  if (T < 1 || T > h->P.episode_len) return fail(MIL_EINVAL, "T must be in 1..episode_len");
  if (episode >= (1ull << 28)) return fail(MIL_EINVAL, "episode must be < 2^28");
  int rc = check_outputs(outs);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (h->gexec) {
    hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  if (h->graph) {
    hipGraphDestroy(h->graph);
    h->graph = nullptr;
  }
  HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
  int lrc = mil::launch_reset(h->dp, h->ds, (uint32_t)episode, dev_out(outs), st);
  if (!lrc) lrc = launch_steps(h, 0, T, (uint32_t)episode, nullptr, dev_out(outs), st, h->sched);
  if (!lrc && d_metrics) lrc = mil::launch_metrics(h->dp, h->ds, T, d_metrics, st);
  hipGraph_t g = nullptr;
  hipError_t ec = hipStreamEndCapture(st, &g);
  if (lrc || ec != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return fail(MIL_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
  }
  h->graph = g;
  HIP_CHECK(hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0));
  h->graph_T = T;
  h->episode = (uint32_t)episode;
  h->t = -1;  // nothing has run yet
  return MIL_OK;
}

int env_graph_launch(mil_env *h, void *stream) {
  if (!h || !h->gexec) return fail(MIL_ESTATE, "no captured graph");
  HIP_CHECK(hipGraphLaunch(h->gexec, (hipStream_t)stream));
  h->t = h->graph_T;
  return MIL_OK;
}

int env_status(mil_env *h, uint32_t *host_flags, void *stream) {
  if (!h || !host_flags) return fail(MIL_EINVAL, "null argument");
  if (!h->ws) return fail(MIL_ESTATE, "env_bind has not been called");
  hipStream_t st = (hipStream_t)stream;
  HIP_CHECK(hipStreamSynchronize(st));
  HIP_CHECK(hipMemcpy(host_flags, h->ws + h->off.status, 4, hipMemcpyDeviceToHost));
  HIP_CHECK(hipMemset(h->ws + h->off.status, 0, 4));
  return MIL_OK;
}

int env_get_state(mil_env *h, float *d_agent, float *d_target, void *stream) {
  if (!h) return fail(MIL_EINVAL, "null handle");
  if (!h->ws || h->t < 0) return fail(MIL_ESTATE, "env_reset has not been called");
  if (mil::launch_get_state(h->ds, d_agent, d_target, stream))
    return fail(MIL_EHIP, "state copy launch failed");
  return MIL_OK;
}

int env_set_mapping(mil_env *h, int32_t lanes_per_agent, int32_t waves_per_block) {
  if (!h) return fail(MIL_EINVAL, "null handle");
  if (lanes_per_agent != 1 && lanes_per_agent != 2)
    return fail(MIL_EINVAL, "lanes_per_agent must be 1 or 2");
  if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
    return fail(MIL_EINVAL, "waves_per_block must be 1, 2 or 4");
  h->G = lanes_per_agent;
  h->wpb = waves_per_block;
  if (h->gexec) {  // a captured graph holds the old launch shape
    hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
    hipGraphDestroy(h->graph);
    h->graph = nullptr;
  }
  if (h->ws) return upload_mapping(h, nullptr);
  build_waves(h);
  return MIL_OK;
}

int env_get_mapping(const mil_env *h, int32_t *lanes_per_agent, int32_t *waves_per_block) {
  if (!h) return fail(MIL_EINVAL, "null handle");
  if (lanes_per_agent) *lanes_per_agent = h->G;
  if (waves_per_block) *waves_per_block = h->wpb;
  return MIL_OK;
}

int env_set_schedule(mil_env *h, int32_t chunk_steps) {
  if (!h) return fail(MIL_EINVAL, "null handle");
  if (chunk_steps < -1) return fail(MIL_EINVAL, "chunk_steps must be -1, 0 or positive");
  h->sched = chunk_steps;
  if (h->gexec) {  // a captured graph holds the old launch shape
    hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
    hipGraphDestroy(h->graph);
    h->graph = nullptr;
  }
  return MIL_OK;
}

int env_get_schedule(const mil_env *h, int32_t *chunk_steps) {
  if (!h || !chunk_steps) return fail(MIL_EINVAL, "null argument");
  *chunk_steps = h->sched;
  return MIL_OK;
}

int env_autotune(mil_env *h, int32_t probe_steps, const mil_env_outputs *outs,
                 const char *cache_path, void *stream) {
  if (!h) return fail(MIL_EINVAL, "null handle");
  if (!h->ws || h->t < 0) return fail(MIL_ESTATE, "env_reset has not been called");
  if (probe_steps < 1 || h->t + probe_steps > h->P.episode_len)
    return fail(MIL_EINVAL, "probe_steps must fit in the rest of the episode");
  hipStream_t st = (hipStream_t)stream;
  const std::string key = device_key(h);
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const auto kp = line.find("\"key\": \"" + key + "\"");
      if (kp == std::string::npos) continue;
      int G = 0, w = 0;
      const auto gp = line.find("\"lanes_per_agent\": ");
      const auto wp = line.find("\"waves_per_block\": ");
      if (gp != std::string::npos) G = std::atoi(line.c_str() + gp + 19);
      if (wp != std::string::npos) w = std::atoi(line.c_str() + wp + 19);
      if (env_set_mapping(h, G, w) == MIL_OK) return MIL_OK;
    }
  }
  const int64_t sbytes = h->off.state_end - h->off.state_begin;
  char *state = h->ws + h->off.state_begin;
  char *snap = h->ws + h->off.snap;
  HIP_CHECK(hipMemcpyAsync(snap, state, sbytes, hipMemcpyDeviceToDevice, st));
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  float best = 1e30f;
  int bestG = h->G, bestW = h->wpb;
  std::ostringstream trials;
  for (int G = 1; G <= 2; ++G) {
    for (int w : {1, 2, 4}) {
      int rc = env_set_mapping(h, G, w);
      if (rc) return rc;
      float ms_min = 1e30f;
      for (int rep = 0; rep < 2; ++rep) {
        HIP_CHECK(hipEventRecord(e0, st));
        // probed in the schedule a long rollout of this batch would get
        rc = run_rollout(h, probe_steps, nullptr, outs, st,
                         h->sched == 0 ? mil::kSchedProbe : h->sched);
        if (rc) return rc;
        HIP_CHECK(hipEventRecord(e1, st));
        HIP_CHECK(hipMemcpyAsync(state, snap, sbytes, hipMemcpyDeviceToDevice, st));
        HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        ms_min = std::min(ms_min, ms);
      }
      trials << (trials.tellp() ? ", " : "") << "\"" << G << "x" << w << "\": " << ms_min;
      if (ms_min < best) {
        best = ms_min;
        bestG = G;
        bestW = w;
      }
    }
  }
  HIP_CHECK(hipStreamSynchronize(st));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  int rc = env_set_mapping(h, bestG, bestW);
  if (rc) return rc;
  if (cache_path) {
    std::ofstream outf(cache_path, std::ios::app);
    outf << "{\"key\": \"" << key << "\", \"lanes_per_agent\": " << bestG
         << ", \"waves_per_block\": " << bestW << ", \"probe_steps\": " << probe_steps
         << ", \"ms\": " << best << ", \"trials_ms\": {" << trials.str() << "}}\n";
  }
  return MIL_OK;
}

int env_pf_state(mil_env *h, float *d_particles, uint8_t *d_belief, void *stream) {
  if (!h) return fail(MIL_EINVAL, "null handle");
  if (h->P.est_kind != 1) return fail(MIL_EINVAL, "the environment has no particle filter");
  if (!h->ws) return fail(MIL_ESTATE, "env_bind has not been called");
  hipStream_t st = (hipStream_t)stream;
  const int64_t P = h->poff[h->E];
  if (d_particles && P)
    HIP_CHECK(hipMemcpyAsync(d_particles, h->ds.pfxy, P * mil::kPfParticles * 8,
                             hipMemcpyDeviceToDevice, st));
  if (d_belief && P)
    HIP_CHECK(hipMemcpyAsync(d_belief, h->ds.pfb, P, hipMemcpyDeviceToDevice, st));
  return MIL_OK;
}

int env_pf_update(mil_env *h, void *stream) {
  if (!h) return fail(MIL_EINVAL, "null handle");
  if (h->P.est_kind != 1) return fail(MIL_EINVAL, "the environment has no particle filter");
  if (!h->ws || h->t < 1) return fail(MIL_ESTATE, "no step has been taken since the reset");
  if (mil::launch_pf(h->dp, h->ds, (int32_t)h->t - 1, h->episode, stream))
    return fail(MIL_EHIP, "particle-filter launch failed: %s", hipGetErrorString(hipGetLastError()));
  return MIL_OK;
}

int env_windows(mil_env *h, float *d_win, float *d_sigma, float *d_truth, void *stream) {
  if (!h || !d_win) return fail(MIL_EINVAL, "null argument");
  if (h->P.est_kind != 0) return fail(MIL_EINVAL, "the particle filter keeps no window");
  if (!h->ws || h->t < 0) return fail(MIL_ESTATE, "env_reset has not been called");
  if (mil::launch_env_windows(h->ds, h->W, h->P.n_agents * h->P.n_targets, d_win, d_sigma, d_truth,
                              stream))
    return fail(MIL_EHIP, "window copy launch failed");
  return MIL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Attention policy
// ---------------------------------------------------------------------------
namespace {

struct PolicyWork {
  int64_t prep, obs, mask, actions, total;
};

PolicyWork policy_work(int64_t A, int64_t K) {
  PolicyWork w{};
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    const int64_t at = o;
    o = align256(o + bytes);
    return at;
  };
  w.prep = take(mil::kPolPrepBytes);
  w.obs = take(K * 6 * 4);
  w.mask = take(K);
  w.actions = take(A * 4);
  w.total = o;
  return w;
}

int num_cus_env() {
  static int n = 0;
  if (n == 0) {
    int dev = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
  }
  return n;
}

void prepared_ptrs(char *prep, __bf16 **wq, __bf16 **wo, __bf16 **w1, __bf16 **w2) {
  __bf16 *b = (__bf16 *)prep;
  *wq = b;
  *wo = *wq + mil::kPolPrepWqkv;
  *w1 = *wo + mil::kPolPrepWo;
  *w2 = *w1 + mil::kPolPrepW1;
}

// env_policy_rollout's workspace: the policy's, then (learned estimator in
// the loop) windows [P][W][3], sigma [P], estimates [P][2], flags [P] and the
// estimator's workspace.
struct EnvPolicyWork {
  PolicyWork pol;
  int64_t win, sig, est, flag, mlp, mlp_bytes, total;
};

EnvPolicyWork env_policy_work(const mil_env *h, bool learned) {
  EnvPolicyWork w{};
  const int64_t A = h->aoff[h->E], K = h->koff[h->E], P = h->poff[h->E];
  w.pol = policy_work(A, K);
  int64_t o = w.pol.total;
  auto take = [&](int64_t bytes) {
    const int64_t at = o;
    o = align256(o + bytes);
    return at;
  };
  if (learned) {
    const int64_t W = h->P.window;
    w.win = take(P * W * 3 * 4);
    w.sig = take(P * 4);
    w.est = take(P * 2 * 4);
    w.flag = take(P);
    w.mlp_bytes = mlp_workspace_bytes(P, 0);
    w.mlp = take(w.mlp_bytes);
  }
  w.total = o;
  return w;
}

int policy_tile(int n_tok) {
  const int at = mil::kPolRows / n_tok;
  return at < mil::kPolMaxAgents ? at : mil::kPolMaxAgents;
}

}  // namespace

extern "C" {

int64_t policy_num_params(void) { return mil::kPolNumParams; }

int64_t policy_workspace_bytes(int64_t num_agents, int64_t num_tokens) {
  return policy_work(num_agents > 0 ? num_agents : 1, num_tokens > 0 ? num_tokens : 1).total;
}

int policy_init(float *d_params, uint64_t seed, void *stream) {
  if (!d_params) return fail(MIL_EINVAL, "null argument");
  if (mil::launch_policy_init(d_params, seed, stream)) return fail(MIL_EHIP, "init launch failed");
  return MIL_OK;
}

// One policy launch on caller tokens: n_tok rows per agent, the first the
// carried state when rec = 1 (then obs holds n_tok - 1 tokens per agent).
static int policy_run(int64_t A, int32_t n_tok, int rec, int32_t n_agents, int32_t n_actions,
                      const float *d_obs, const uint8_t *d_mask, const float *d_hidden_in,
                      const float *d_params, float *d_logits, int32_t *d_actions, float *d_feat,
                      uint64_t seed, uint32_t t, uint32_t episode, void *d_work,
                      int64_t work_bytes, void *stream) {
  if (A < 0 || n_tok < 1 + rec || n_tok > mil::kPolMaxTok || n_agents < 1 || n_actions < 1 ||
      n_actions > mil::kPolActions || (A % n_agents) != 0)
    return fail(MIL_EINVAL, rec ? "need n_obs in 1..15, n_actions in 1..8, A a multiple of n_agents"
                                : "need n_tok in 1..16, n_actions in 1..8, A a multiple of n_agents");
  if (A == 0) return MIL_OK;
  if (!d_obs || !d_mask || !d_params) return fail(MIL_EINVAL, "null argument");
  const PolicyWork w = policy_work(A, A * n_tok);
  if (!d_work || (((uintptr_t)d_work) & 255)) return fail(MIL_EALIGN, "workspace must be 256-byte aligned");
  if (work_bytes < w.prep + mil::kPolPrepBytes) return fail(MIL_ESHAPE, "workspace too small");
  char *ws = (char *)d_work;
  mil::PolicyArgs a{};
  __bf16 *wq, *wo, *w1, *w2;
  prepared_ptrs(ws + w.prep, &wq, &wo, &w1, &w2);
  if (mil::launch_policy_prepare(d_params, wq, wo, w1, w2, stream))
    return fail(MIL_EHIP, "policy prepare failed");
  a.A = A;
  a.n_tok = n_tok;
  a.agents_per_tile = policy_tile(n_tok);
  a.obs = d_obs;
  a.mask = d_mask;
  a.params = d_params;
  a.wqkv = wq; a.wo = wo; a.w1 = w1; a.w2 = w2;
  a.logits = d_logits;
  a.actions = d_actions;
  a.feat = d_feat;
  a.hidden_in = d_hidden_in;
  a.rec = rec;
  a.n_agents = n_agents;
  a.n_actions = n_actions;
  a.t = t;
  a.episode = episode;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  a.env_ids = nullptr;
  if (mil::launch_policy(a, num_cus_env(), stream)) return fail(MIL_EHIP, "policy launch failed");
  return MIL_OK;
}

int policy_forward(int64_t A, int32_t n_tok, int32_t n_agents, int32_t n_actions, const float *d_obs,
                   const uint8_t *d_mask, const float *d_params, float *d_logits,
                   int32_t *d_actions, uint64_t seed, uint32_t t, uint32_t episode, void *d_work,
                   int64_t work_bytes, void *stream) {
  return policy_run(A, n_tok, 0, n_agents, n_actions, d_obs, d_mask, nullptr, d_params, d_logits,
                    d_actions, nullptr, seed, t, episode, d_work, work_bytes, stream);
}

int policy_forward_feat(int64_t A, int32_t n_tok, int32_t n_agents, int32_t n_actions,
                        const float *d_obs, const uint8_t *d_mask, const float *d_params,
                        float *d_logits, int32_t *d_actions, float *d_feat, uint64_t seed,
                        uint32_t t, uint32_t episode, void *d_work, int64_t work_bytes,
                        void *stream) {
  return policy_run(A, n_tok, 0, n_agents, n_actions, d_obs, d_mask, nullptr, d_params, d_logits,
                    d_actions, d_feat, seed, t, episode, d_work, work_bytes, stream);
}

int policy_forward_rec(int64_t A, int32_t n_obs, int32_t n_agents, int32_t n_actions,
                       const float *d_obs, const uint8_t *d_mask, const float *d_hidden_in,
                       const float *d_params, float *d_logits, int32_t *d_actions,
                       float *d_hidden_out, uint64_t seed, uint32_t t, uint32_t episode,
                       void *d_work, int64_t work_bytes, void *stream) {
  if (A > 0 && !d_hidden_out) return fail(MIL_EINVAL, "null argument");
  if (n_obs < 1 || n_obs > mil::kPolMaxTok - 1)
    return fail(MIL_EINVAL, "need n_obs in 1..15 (the carried state takes one more row)");
  return policy_run(A, n_obs + 1, 1, n_agents, n_actions, d_obs, d_mask, d_hidden_in, d_params,
                    d_logits, d_actions, d_hidden_out, seed, t, episode, d_work, work_bytes,
                    stream);
}

// ---------------------------------------------------------------------------
// Learner's forward half: critic values, GAE, clipped PPO objective
// ---------------------------------------------------------------------------
static int64_t critic_logits_off(int64_t N, int nt) {
  return align256(policy_work(N, N * nt).total);
}

int64_t critic_workspace_bytes(int64_t N, int32_t n_agents, int32_t n_targets) {
  if (N < 0 || n_agents < 1 || n_targets < 1 || n_agents + n_targets + 1 > mil::kPolMaxTok) return -1;
  const int nt = n_agents + n_targets + 1;
  return critic_logits_off(N, nt) + align256(N * mil::kPolActions * 4);
}

int critic_forward(const float *d_gstate, int64_t N, int32_t n_agents, int32_t n_targets,
                   float pos_scale, const float *d_params, float *d_values, float *d_feat,
                   void *d_work, int64_t work_bytes, void *stream) {
  if (N < 0 || n_agents < 1 || n_targets < 1 || n_agents + n_targets + 1 > mil::kPolMaxTok)
    return fail(MIL_EINVAL, "need N >= 0 and 1 + n_agents + n_targets <= 16");
  if (!(pos_scale > 0.0f)) return fail(MIL_EINVAL, "pos_scale must be > 0");
  if (N == 0) return MIL_OK;
  if (!d_gstate || !d_params || !d_values) return fail(MIL_EINVAL, "null argument");
  if (!d_work || (((uintptr_t)d_work) & 255)) return fail(MIL_EALIGN, "workspace must be 256-byte aligned");
  if (work_bytes < critic_workspace_bytes(N, n_agents, n_targets))
    return fail(MIL_ESHAPE, "workspace too small (critic_workspace_bytes)");
  const int M = n_agents + n_targets, nt = M + 1;
  const PolicyWork w = policy_work(N, N * nt);
  char *ws = (char *)d_work;
  float *tokens = (float *)(ws + w.obs);
  uint8_t *mask = (uint8_t *)(ws + w.mask);
  float *logits = (float *)(ws + critic_logits_off(N, nt));
  __bf16 *wq, *wo, *w1, *w2;
  prepared_ptrs(ws + w.prep, &wq, &wo, &w1, &w2);
  if (mil::launch_critic_tokens(d_gstate, N, M, 1, pos_scale, tokens, mask, stream) ||
      mil::launch_policy_prepare(d_params, wq, wo, w1, w2, stream))
    return fail(MIL_EHIP, "critic set-up launch failed");
  mil::PolicyArgs a{};
  a.A = N;
  a.n_tok = nt;
  a.agents_per_tile = policy_tile(nt);
  a.obs = tokens;
  a.mask = mask;
  a.params = d_params;
  a.wqkv = wq; a.wo = wo; a.w1 = w1; a.w2 = w2;
  a.logits = logits;
  a.actions = nullptr;
  a.feat = d_feat;
  a.n_agents = 1;
  a.n_actions = 1;
  a.env_ids = nullptr;
  if (mil::launch_policy(a, num_cus_env(), stream) ||
      mil::launch_first_column(logits, N, d_values, stream))
    return fail(MIL_EHIP, "critic launch failed");
  return MIL_OK;
}

int critic_forward_rec(const float *d_gstate, int32_t T, int64_t N, int32_t n_agents,
                       int32_t n_targets, float pos_scale, const float *d_params,
                       const float *d_hidden_in, float *d_values, float *d_hidden_seq,
                       void *d_work, int64_t work_bytes, void *stream) {
  if (T < 0 || N < 0 || n_agents < 1 || n_targets < 1 || n_agents + n_targets + 1 > mil::kPolMaxTok)
    return fail(MIL_EINVAL, "need T >= 0, N >= 0 and 1 + n_agents + n_targets <= 16");
  if (!(pos_scale > 0.0f)) return fail(MIL_EINVAL, "pos_scale must be > 0");
  if (N == 0 || T == 0) return MIL_OK;
  if (!d_gstate || !d_params || !d_values || !d_hidden_seq) return fail(MIL_EINVAL, "null argument");
  if (!d_work || (((uintptr_t)d_work) & 255)) return fail(MIL_EALIGN, "workspace must be 256-byte aligned");
  if (work_bytes < critic_workspace_bytes(N, n_agents, n_targets))
    return fail(MIL_ESHAPE, "workspace too small (critic_workspace_bytes)");
  const int M = n_agents + n_targets, nt = M + 1;
  const PolicyWork w = policy_work(N, N * nt);
  char *ws = (char *)d_work;
  float *tokens = (float *)(ws + w.obs);
  uint8_t *mask = (uint8_t *)(ws + w.mask);
  float *logits = (float *)(ws + critic_logits_off(N, nt));
  __bf16 *wq, *wo, *w1, *w2;
  prepared_ptrs(ws + w.prep, &wq, &wo, &w1, &w2);
  if (mil::launch_policy_prepare(d_params, wq, wo, w1, w2, stream))
    return fail(MIL_EHIP, "critic set-up launch failed");
  // the steps in order: step t reads the state step t - 1 wrote
  for (int32_t t = 0; t < T; ++t) {
    mil::PolicyArgs a{};
    a.A = N;
    a.n_tok = nt;
    a.agents_per_tile = policy_tile(nt);
    a.obs = tokens;
    a.mask = mask;
    a.params = d_params;
    a.wqkv = wq; a.wo = wo; a.w1 = w1; a.w2 = w2;
    a.logits = logits;
    a.feat = d_hidden_seq + (int64_t)t * N * mil::kPolD;
    a.hidden_in = t == 0 ? d_hidden_in : d_hidden_seq + (int64_t)(t - 1) * N * mil::kPolD;
    a.rec = 1;
    a.n_agents = 1;
    a.n_actions = 1;
    if (mil::launch_critic_tokens(d_gstate + (int64_t)t * N * M * 6, N, M, 0, pos_scale, tokens,
                                  mask, stream) ||
        mil::launch_policy(a, num_cus_env(), stream) ||
        mil::launch_first_column(logits, N, d_values + (int64_t)t * N, stream))
      return fail(MIL_EHIP, "critic launch failed");
  }
  return MIL_OK;
}

int ppo_gae(const float *d_rewards, const uint8_t *d_dones, const float *d_values, int32_t T,
            int64_t E, float gamma, float lambda, float *d_adv, float *d_ret, void *stream) {
  if (T < 0 || E < 0) return fail(MIL_EINVAL, "need T >= 0, E >= 0");
  if (!(gamma >= 0.0f && gamma <= 1.0f && lambda >= 0.0f && lambda <= 1.0f))
    return fail(MIL_EINVAL, "gamma and lambda must be in [0, 1]");
  if (T == 0 || E == 0) return MIL_OK;
  if (!d_rewards || !d_dones || !d_values || !d_adv || !d_ret)
    return fail(MIL_EINVAL, "null argument");
  if (mil::launch_gae(d_rewards, d_dones, d_values, T, E, gamma, lambda, d_adv, d_ret, stream))
    return fail(MIL_EHIP, "gae launch failed");
  return MIL_OK;
}

int64_t ppo_workspace_bytes(void) {
  // the objective's partials, or the head gradient's (n_out <= 8)
  return (int64_t)mil::kPpoBlocks * mil::kPolActions * (mil::kPolD + 1) * 8;
}

int head_grad(int64_t N, const float *d_feat, const float *d_dout, int32_t ld, int32_t n_out,
              float *d_grad, void *d_work, int64_t work_bytes, void *stream) {
  if (N < 0 || n_out < 1 || n_out > mil::kPolActions || ld < n_out)
    return fail(MIL_EINVAL, "need N >= 0, n_out in 1..8, ld >= n_out");
  if (!d_grad || (N > 0 && (!d_feat || !d_dout))) return fail(MIL_EINVAL, "null argument");
  if (!d_work || (((uintptr_t)d_work) & 7) || work_bytes < ppo_workspace_bytes())
    return fail(MIL_ESHAPE, "workspace too small or misaligned (ppo_workspace_bytes, 8-byte aligned)");
  if (mil::launch_head_grad(d_feat, d_dout, N, ld, n_out, d_grad, (double *)d_work, stream))
    return fail(MIL_EHIP, "head gradient launch failed");
  return MIL_OK;
}

int ppo_objective(const float *d_logits_new, const float *d_logits_old, const int32_t *d_actions,
                  const float *d_adv, const float *d_values, const float *d_returns, int32_t T,
                  int64_t A, int32_t n_agents, int32_t n_actions, float clip_eps, double *d_out,
                  float *d_dlogits, float *d_dvalues, void *d_work, int64_t work_bytes,
                  void *stream) {
  if (T < 1 || A < 1 || n_agents < 1 || (A % n_agents) != 0 || n_actions < 1 ||
      n_actions > mil::kPolActions)
    return fail(MIL_EINVAL, "need T >= 1, A a positive multiple of n_agents, n_actions in 1..8");
  if (!(clip_eps >= 0.0f && clip_eps < 1.0f)) return fail(MIL_EINVAL, "clip_eps must be in [0, 1)");
  if (!d_logits_new || !d_logits_old || !d_actions || !d_adv || !d_values || !d_returns || !d_out)
    return fail(MIL_EINVAL, "null argument");
  if (!d_work || (((uintptr_t)d_work) & 7) || work_bytes < ppo_workspace_bytes())
    return fail(MIL_ESHAPE, "workspace too small or misaligned (ppo_workspace_bytes, 8-byte aligned)");
  if (mil::launch_ppo_objective(d_logits_new, d_logits_old, d_actions, d_adv, d_values, d_returns,
                                T, A, n_agents, n_actions, clip_eps, d_out, d_dlogits, d_dvalues,
                                (double *)d_work, stream))
    return fail(MIL_EHIP, "ppo objective launch failed");
  return MIL_OK;
}

int64_t env_policy_workspace_bytes(const mil_env *h, int32_t learned) {
  if (!h || !h->ws) return -1;
  return env_policy_work(h, learned != 0).total;
}

int env_policy_rollout(mil_env *h, uint64_t episode, int32_t T, const float *d_params,
                       const float *d_mlp_params, float k_sigma, float *d_hidden,
                       const mil_env_outputs *outs, double *d_metrics, int32_t capture,
                       void *d_work, int64_t work_bytes, void *stream) {
  if (!h || !d_params) return fail(MIL_EINVAL, "null argument");
  if (!h->ws) return fail(MIL_ESTATE, "env_bind has not been called");
  if (h->P.ragged) return fail(MIL_EINVAL, "the policy needs a batch with fixed counts");
  const int rec = d_hidden != nullptr;  // the recurrent form carries d_hidden across steps
  const int na = h->P.n_agents, n_tok = h->P.n_agents + h->P.n_targets + rec;
  if (n_tok > mil::kPolMaxTok || h->P.n_actions > mil::kPolActions)
    return fail(MIL_EINVAL, "the policy supports at most 16 rows per agent (tokens and the "
                            "carried state) and 8 actions");
  if (T < 1 || T > h->P.episode_len) return fail(MIL_EINVAL, "T must be in 1..episode_len");
  if (episode >= (1ull << 28)) return fail(MIL_EINVAL, "episode must be < 2^28");
  int rc = check_outputs(outs);
  if (rc) return rc;
  const bool learned = d_mlp_params != nullptr;
  if (learned && h->P.pooled)
    return fail(MIL_EINVAL, "the learned estimator in the loop takes one agent's own window: "
                            "pooled must be 0");
  if (learned && h->P.est_kind != 0)
    return fail(MIL_EINVAL, "the learned estimator replaces the least-squares tracker: "
                            "est_kind must be 0");
  if (learned && (h->P.window > 21 || !(k_sigma >= 0.0f)))
    return fail(MIL_EINVAL, "the learned estimator needs window <= 21 and k_sigma >= 0");
  const int64_t A = h->aoff[h->E], K = h->koff[h->E], Pn = h->poff[h->E];
  const EnvPolicyWork ew = env_policy_work(h, learned);
  const PolicyWork &w = ew.pol;
  if (!d_work || (((uintptr_t)d_work) & 255)) return fail(MIL_EALIGN, "workspace must be 256-byte aligned");
  if (work_bytes < ew.total) return fail(MIL_ESHAPE, "workspace too small (env_policy_workspace_bytes)");
  char *ws = (char *)d_work;
  float *wobs = (float *)(ws + w.obs);
  uint8_t *wmask = (uint8_t *)(ws + w.mask);
  int32_t *wact = (int32_t *)(ws + w.actions);
  __bf16 *wq, *wo, *w1, *w2;
  prepared_ptrs(ws + w.prep, &wq, &wo, &w1, &w2);
  hipStream_t st = (hipStream_t)stream;
  if (capture) {
    if (h->gexec) {
      hipGraphExecDestroy(h->gexec);
      h->gexec = nullptr;
    }
    if (h->graph) {
      hipGraphDestroy(h->graph);
      h->graph = nullptr;
    }
    HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
  }
  int lrc = mil::launch_policy_prepare(d_params, wq, wo, w1, w2, st);
  mil::DevOut r0{};
  r0.obs = wobs;
  r0.obs_mask = wmask;
  if (!lrc) lrc = mil::launch_reset(h->dp, h->ds, (uint32_t)episode, r0, st);
  const mil::DevOut full = dev_out(outs);
  const bool keep_obs = full.obs && full.obs_mask;
  for (int32_t t = 0; t < T && !lrc; ++t) {
    mil::PolicyArgs a{};
    a.A = A;
    a.n_tok = n_tok;
    a.agents_per_tile = policy_tile(n_tok);
    a.obs = (t == 0 || !keep_obs) ? wobs : full.obs + (int64_t)(t - 1) * K * 6;
    a.mask = (t == 0 || !keep_obs) ? wmask : full.obs_mask + (int64_t)(t - 1) * K;
    a.params = d_params;
    a.wqkv = wq; a.wo = wo; a.w1 = w1; a.w2 = w2;
    a.actions = wact;
    a.feat = d_hidden;  // this step's state, read back by the next (zeros at the reset)
    a.hidden_in = t == 0 ? nullptr : d_hidden;
    a.rec = rec;
    a.n_agents = na;
    a.n_actions = h->P.n_actions;
    a.t = (uint32_t)t;
    a.episode = (uint32_t)episode;
    a.key0 = h->dp.key0;
    a.key1 = h->dp.key1;
    a.env_ids = h->ds.env_id;
    lrc = mil::launch_policy(a, num_cus_env(), st);
    if (lrc) break;
    // this step's outputs: the caller's slice of step t, with the observation
    // kept in the workspace when the caller does not record it
    mil::DevOut o{};
    auto slice = [&](auto *p, int64_t per) { return p ? p + (int64_t)t * per : p; };
    o.obs = keep_obs ? slice(full.obs, K * 6) : wobs;
    o.obs_mask = keep_obs ? slice(full.obs_mask, K) : wmask;
    o.reward = slice(full.reward, h->E);
    o.done = slice(full.done, h->E);
    o.est = slice(full.est, h->poff[h->E] * 2);
    o.est_valid = slice(full.est_valid, h->poff[h->E]);
    o.gstate = slice(full.gstate, (A + h->toff[h->E]) * 6);
    o.actions = slice(full.actions, A);
    o.ranges = slice(full.ranges, h->poff[h->E]);
    o.err = slice(full.err, h->toff[h->E]);
    const mil::DevState *dstate = (const mil::DevState *)(h->ws + h->off.devstate);
    if (!learned) {
      lrc = launch_steps(h, t, 1, (uint32_t)episode, wact, o, st, h->sched);
    } else {
      // move, estimate every tracker from its window, then observe
      float *win = (float *)(ws + ew.win), *sig = (float *)(ws + ew.sig);
      float *est = (float *)(ws + ew.est);
      uint8_t *flag = (uint8_t *)(ws + ew.flag);
      // (phase 1 also writes every tracker's window and noise std for the network)
      lrc = mil::launch_rollout(h->size_class, h->wcap, h->G, h->wpb, h->num_waves, h->dp, h->ds,
                                dstate, t, 1, (uint32_t)episode, wact, o, st,
                                mil::DevExt{1, nullptr, nullptr, win, sig}, h->sched);
      if (!lrc)
        lrc = mlp_infer(win, Pn, h->P.window, d_mlp_params, sig, k_sigma, h->P.gn_iters,
                        h->P.guard_tau, est,
                        flag, ws + ew.mlp, ew.mlp_bytes, st) == MIL_OK
                  ? 0
                  : -1;
      if (!lrc)
        lrc = mil::launch_rollout(h->size_class, h->wcap, h->G, h->wpb, h->num_waves, h->dp,
                                  h->ds, dstate, t, 1, (uint32_t)episode, wact, o, st,
                                  mil::DevExt{2, est, flag}, h->sched);
    }
  }
  if (!lrc && d_metrics) lrc = mil::launch_metrics(h->dp, h->ds, T, d_metrics, st);
  if (capture) {
    hipGraph_t g = nullptr;
    hipError_t ec = hipStreamEndCapture(st, &g);
    if (lrc || ec != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return fail(MIL_EHIP, "policy graph capture failed: %s", hipGetErrorString(ec));
    }
    h->graph = g;
    HIP_CHECK(hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0));
    h->graph_T = T;
    h->episode = (uint32_t)episode;
    h->t = -1;
    return MIL_OK;
  }
  if (lrc) return fail(MIL_EHIP, "policy rollout launch failed: %s", hipGetErrorString(hipGetLastError()));
  h->episode = (uint32_t)episode;
  h->t = T;
  return MIL_OK;
}

int env_destroy(mil_env *h) {
  if (!h) return MIL_OK;
  if (h->gexec) hipGraphExecDestroy(h->gexec);
  if (h->graph) hipGraphDestroy(h->graph);
  if (h->side) {
    hipStreamSynchronize(h->side);
    hipStreamDestroy(h->side);
  }
  if (h->ev_fork) hipEventDestroy(h->ev_fork);
  if (h->ev_join) hipEventDestroy(h->ev_join);
  delete h;
  return MIL_OK;
}

int est_exact(const float *d_win, int64_t N, int32_t W, int32_t gn_iters, float tau, int32_t accum,
              float *d_out, uint8_t *d_valid, void *stream) {
  if (N < 0) return fail(MIL_EINVAL, "N must be >= 0");
  if (N == 0) return MIL_OK;
  if (!d_win || !d_out || !d_valid) return fail(MIL_EINVAL, "null argument");
  if (W < 3 || W > 64) return fail(MIL_EINVAL, "W must be in 3..64");
  if (gn_iters < 0 || gn_iters > 64) return fail(MIL_EINVAL, "gn_iters must be in 0..64");
  if (accum != 0 && accum != 1) return fail(MIL_EINVAL, "accum must be 0 or 1");
  if (((uintptr_t)d_win) & 3 || ((uintptr_t)d_out) & 7) return fail(MIL_EALIGN, "misaligned");
  if (mil::launch_est_exact(d_win, N, W, gn_iters, tau, accum, d_out, d_valid, stream))
    return fail(MIL_EHIP, "est_exact launch failed: %s", hipGetErrorString(hipGetLastError()));
  return MIL_OK;
}

int rng_philox(const uint32_t *d_ctr, int64_t n, uint64_t seed, uint32_t *d_out, float *d_u01,
               float *d_normal, void *stream) {
  if (n < 0) return fail(MIL_EINVAL, "n must be >= 0");
  if (n == 0) return MIL_OK;
  if (!d_ctr) return fail(MIL_EINVAL, "null counters");
  if (mil::launch_rng(d_ctr, n, (uint32_t)seed, (uint32_t)(seed >> 32), d_out, d_u01, d_normal,
                      stream))
    return fail(MIL_EHIP, "rng launch failed");
  return MIL_OK;
}

}  // extern "C"
