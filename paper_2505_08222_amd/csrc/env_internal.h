// Structures shared by the host runtime and the environment kernels.
#pragma once
#include <stdint.h>

namespace mil {

// Environment constants as the kernels see them (by value, kernel argument).
struct DevParams {
  int32_t window, episode_len, n_actions, gn_iters;
  float dt, agent_speed, area, spawn_r;
  float dpsi[8];
  float sig_a, sig_t;
  float tv_lo, tv_hi, sr_lo, sr_hi;
  float det_range, comm_range, comm_loss_p;
  float eps_min, eps_max, d_safe, tau, lost_range;
  uint32_t key0, key1;
  int32_t action_mode, n_rudder, reward_mode, spawn_mode;
  float d_follow, spawn_min, spawn_max;
  int32_t pooled;
  int32_t est_kind;  // 0 least squares, 1 particle filter
  float pf_q, pf_lik_sigma;
};

// One (agents, targets) shape. Environments of a shape are consecutive in
// packed order, so every per-env offset is an affine function of the env's
// index inside its class. wave0/nwaves depend on the lane mapping.
struct ClassInfo {
  int64_t env0, nenv;
  int64_t aoff0, toff0, poff0, koff0;
  int32_t na, nt;
  int32_t wave0, nwaves;
};

// Blocks of the metrics reduction (each sums a contiguous range of envs).
constexpr int kMetricBlocks = 256;

// Device pointers into the caller's workspace.
struct DevState {
  const uint32_t *env_id;  // [E] global id of each packed env
  const uint8_t *cnt_a;    // [E]
  const uint8_t *cnt_t;    // [E]
  const int64_t *aoff, *toff, *poff, *koff;  // [E+1]
  const ClassInfo *classes;                  // [num_classes]
  const uint8_t *wave_class;                 // [num_waves]
  float *ax, *ay, *apsi;                     // [A]
  int32_t *arud;                             // [A] rudder position (action_mode 1)
  float *tx, *ty, *tpsi, *tv;                // [Tt]
  float *sigma;                              // [E]
  float *hx, *hy;                            // [W][A], entry 0 = newest
  float *hr;                                 // [W][P]
  uint8_t *hrec;                             // [W][A] received-broadcast bits (pooled)
  float *ex, *ey;                            // [P]
  uint8_t *ev;                               // [P]
  double *macc;                              // [E][3] reward, err, err^2 sums
  int32_t *miacc;                            // [E][2] err count, crash steps
  uint32_t *status;                          // [1]
  int32_t *queue;                            // [1 + groups] dynamic-schedule counter, chunk flags
  double *mpart;                             // [kMetricBlocks][6] metrics partial sums
  // particle filter (est_kind 1; null otherwise)
  // [P][4] per tracker: packed env index; 8 * agent + target | n_agents << 8 |
  // n_targets << 12; global agent index; 0
  const uint32_t *pmeta;
  float *pfxy;            // [P][kPfParticles][2] particles
  uint8_t *pfb;           // [P] 1 when the tracker holds a belief
  float *pfm;             // [P][4] this step's agent x, y and range (move half's output)
  int64_t E, A, Tt, P, K;
};

// Particles per tracker: one per lane of a wavefront.
constexpr int kPfParticles = 64;

// Output pointers (mirrors mil_env_outputs) and the per-step strides of the
// step-major output arrays.
struct DevOut {
  int64_t E, A, Tt, P, K;
  float *obs;
  uint8_t *obs_mask;
  float *reward;
  uint8_t *done;
  float *est;
  uint8_t *est_valid;
  float *gstate;
  int32_t *actions;
  float *ranges;
  float *err;
};

// Split step of the full kernel, for an estimator that runs between its two
// halves: phase 1 moves the entities, draws the ranges and pushes the window,
// and (win not null) hands every tracker's window to the estimator: win
// [P][W][3] (agent x, agent y, range; entry 0 newest) and wsig [P] (the env's
// range-noise std); phase 2 takes each tracker's estimate from est [P][2] /
// flag [P] (flag 0 or 1: estimate present, 2: refused, hold the previous one)
// once its window is full, then computes reward, observation and outputs.
// With meas set, phase 1 also writes each tracker's newest entry to meas
// [P][4] (agent x, y, range, 0). Phase 2 with est null: the estimator has
// written the estimates into the state (ex, ey, ev) itself. Phase 3 (est
// null, T = 2): the observe half of the launch's first step, then the move
// half of its second, so that one launch sits between two filter updates.
// phase 0: whole step.
struct DevExt {
  int32_t phase;
  const float *est;
  const uint8_t *flag;
  float *win = nullptr;
  float *wsig = nullptr;
  float *meas = nullptr;
  // static schedule only: the launch covers wavefront groups wave0 ..
  // num_waves - 1 (a slice of the batch; the groups' envs are contiguous)
  int32_t wave0 = 0;
};

// Kernel launchers (env_kernels.hip). All enqueue on `stream`.
int launch_reset(const DevParams &p, const DevState &s, uint32_t episode, const DevOut &o,
                 void *stream);
// d_state: a device copy of `s` (the rollout reads it through this pointer so
// that the state pointers need not stay in scalar registers across steps).
// kSchedProbe: the automatic choice made as if T were long (two chunks of
// T/2 when a long rollout would be dynamic), for the autotuner's probes.
constexpr int32_t kSchedProbe = -2;
// sched: -1 static (one wavefront per group for all T steps), 0 automatic
// (dynamic when the groups number one to eight times the wavefronts the GPU
// holds at once and T spans two chunks), > 0 dynamic with chunks of that
// many steps.
int launch_rollout(int size_class, int wcap, int lanes_per_agent, int waves_per_block,
                   int num_waves, const DevParams &p, const DevState &s, const DevState *d_state,
                   int32_t t0, int32_t T, uint32_t episode, const int32_t *actions,
                   const DevOut &o, void *stream, const DevExt &ext = DevExt{0, nullptr, nullptr},
                   int32_t sched = 0);
int launch_metrics(const DevParams &p, const DevState &s, int32_t steps, double *d_metrics,
                   void *stream);
int launch_get_state(const DevState &s, float *d_agent, float *d_target, void *stream);

// pf_kernels.hip: one particle-filter update of every tracker for step t
// (after the move half of step t wrote s.pfm); writes the particles, the
// belief flags and, for trackers that hold a belief, ex / ey / ev.
// Trackers p_begin .. p_end - 1 (p_end < 0: to the last).
int launch_pf(const DevParams &p, const DevState &s, int32_t t, uint32_t episode, void *stream,
              int64_t p_begin = 0, int64_t p_end = -1);

// est_kernels.hip
int launch_est_exact(const float *d_win, int64_t N, int32_t W, int32_t gn_iters, float tau,
                     int32_t accum, float *d_out, uint8_t *d_valid, void *stream);
int launch_rng(const uint32_t *d_ctr, int64_t n, uint32_t key0, uint32_t key1, uint32_t *d_out,
               float *d_u01, float *d_normal, void *stream);

}  // namespace mil
