/*
 * mi_lrauv: MI355X (gfx950) library of the batched range-only tracking
 * environment of "Scaling Multi-Agent Reinforcement Learning for Underwater
 * Acoustic Tracking via Autonomous Vehicles" (arXiv 2505.08222).
 *
 * C ABI. Plain pointers and sizes only. Pointers named d_* are DEVICE
 * pointers (HIP global memory on the current device); all others are host.
 * Every call that takes a hipStream_t (passed as void*) only enqueues work on
 * that stream, in stream order, and never synchronises, unless stated. With
 * the particle filter (est_kind 1) a step also runs half of the batch on a
 * second stream of the handle's own, forked from and joined back into the
 * caller's stream by events within the same call (so stream order, and
 * graph capture, hold as for one stream).
 *
 * Ownership: the caller allocates every device buffer (its size comes from
 * env_query_layout) and keeps it alive while the handle uses it; the library
 * owns only the host-side handle, any HIP graph it instantiates and, with
 * the particle filter, that second stream and its two events (created by
 * env_bind, released by env_destroy).
 *
 * Errors: every int-returning call returns 0 (MIL_OK) or a negative
 * mil_status; env_last_error() then describes the last failure of the
 * calling thread. Device-side anomalies (an action index out of range, a
 * non-finite state) never trap: they set bits of a status word that
 * env_status() reads back.
 *
 * Layouts: struct-of-arrays, FP32 unless stated. Environments are stored in
 * PACKED order: sorted by (agents, targets) so that each wavefront holds
 * environments of one shape (identity order when the counts are fixed).
 * env_get_order() gives the global id of each packed environment and the
 * CSR offsets of its agents, targets, (agent,target) pairs and
 * observation tokens. Entities of one environment are contiguous:
 *   agents  [A]   A = sum n_agents
 *   targets [Tt]  Tt = sum n_targets
 *   pairs   [P]   P = sum n_agents*n_targets, pair (i,j) at i*n_targets + j
 *   tokens  [K]   K = sum n_agents*(n_agents+n_targets); agent i's tokens are
 *                 [self, the other agents in index order, the targets in
 *                 index order] (the TransfMAPPO entity tokens, Sec. IV-B-1).
 * A handle is not thread-safe; distinct handles are independent.
 */
#ifndef MI_LRAUV_H
#define MI_LRAUV_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MIL_MAX_AGENTS 8
#define MIL_MAX_TARGETS 8
#define MIL_MAX_WINDOW 16
#define MIL_MAX_ACTIONS 8

typedef enum mil_status {
  MIL_OK = 0,
  MIL_EINVAL = -1, /* a parameter is out of its documented range */
  MIL_ESHAPE = -2, /* a size does not match the handle or the layout */
  MIL_EALIGN = -3, /* a device pointer is not 256-byte aligned (workspace) or
                      not 8-byte aligned (outputs) */
  MIL_EHIP = -4,   /* a HIP runtime call failed; see env_last_error() */
  MIL_ESTATE = -5, /* call out of order (e.g. step before bind/reset, or past
                      the end of the episode) */
  MIL_ENOMEM = -6  /* host allocation failed */
} mil_status;

/* Device status bits reported by env_status(). */
#define MIL_STATUS_BAD_ACTION 0x1u /* an action index was outside 0..n_actions-1;
                                      that agent kept its heading */
#define MIL_STATUS_NONFINITE 0x2u  /* a position or heading became non-finite */
#define MIL_STATUS_SCHEDULE 0x4u   /* a dynamic-schedule chunk wait gave up (the rollout's
                                      results are then not to be trusted) */

/* Environment parameters (SI units). Meaning of each field, with the passage
 * of the paper it comes from:
 *  n_agents, n_targets  fixed counts, or the maxima (1..8) when ragged = 1;
 *                       ragged counts are drawn per env, uniform in 1..max.
 *  window               W, number of most recent range measurements each
 *                       (agent,target) tracker keeps (3..16); the particle
 *                       filter (est_kind 1) keeps only the newest.
 *  episode_len          steps per episode; done is set on the last one and
 *                       stepping past it is an error (termination only at the
 *                       step limit, Sec. IV-A-2 "Termination").
 *  n_actions, action_dpsi  heading change per discrete action (rad); the
 *                       paper's agents only steer at constant speed (Sec.
 *                       IV-A-2 "Actions Space").
 *  gn_iters             Gauss-Newton refinements after the linearised
 *                       least-squares solve (0 = plain LS, Sec. III-A).
 *  dt, agent_speed      step duration and constant agent speed; agents move
 *                       p += v dt (cos psi, sin psi) after turning (Sec.
 *                       IV-A-3).
 *  agent_heading_sigma  std of the Gaussian heading noise added each step
 *                       (0.02 rad in Sec. IV-A-3).
 *  target_heading_sigma std of the targets' random-walk heading jitter.
 *  target_speed_lo/hi   per-target constant speed, uniform in [lo, hi].
 *  range_sigma_lo/hi    per-env range-noise std, uniform in [lo, hi].
 *  area, spawn_agent_radius  targets spawn uniformly in the square
 *                       [-area/2, area/2]^2; agents uniformly in the disk of
 *                       this radius about the centre.
 *  det_range            true distances beyond this give no range (the
 *                       paper's 450 m detection limit, Sec. IV-A-2); INF
 *                       disables it.
 *  comm_range, comm_loss_p  an agent receives another agent's position only
 *                       within comm_range and when that agent's broadcast is
 *                       not dropped (probability comm_loss_p).
 *  eps_min, eps_max     Eq. (1) thresholds (10 m and 50 m in the paper).
 *  d_safe               crash distance: the reward is -1 when two agents are
 *                       closer (text after Eq. (2)).
 *  guard_tau            2x2 solves are refused when det <= tau * trace^2.
 *  lost_range           a target counts as lost at the end of a rollout when
 *                       every agent is farther than this.
 * Paper-faithful variants (Sec. IV-A-2 and IV-A-3):
 *  action_mode          0: action k turns the heading by action_dpsi[k];
 *                       1: rudder state: each agent's rudder sits at one of
 *                       n_rudder angles (starting at the middle one) and
 *                       actions 0, 1, 2 move it one angle down, keep it, move
 *                       it one angle up (only adjacent angles, "Actions
 *                       Space"); the heading turns by action_dpsi[rudder], the
 *                       linear theta(gamma) at that angle. Needs n_actions = 3;
 *                       an invalid action keeps the rudder.
 *  reward_mode          0: tracking reward, Eq. (1); 1: follow reward, Eq. (2):
 *                       a target scores 1 when its nearest agent (true
 *                       positions) is within d_follow.
 *  spawn_mode           0: as above; 1: every entity at least spawn_min and at
 *                       most spawn_max from every other: jittered sites of a
 *                       randomly rotated hexagonal patch about the centre, in
 *                       random order (needs n_agents + n_targets <= 13 and
 *                       spawn_max >= 2 sqrt(3) spawn_min).
 *  pooled               1: each agent's tracker of a target solves over its
 *                       own window and the entries of every other agent whose
 *                       broadcast of that step it received (not dropped,
 *                       within comm_range; Sec. IV-A-2: trackers are updated
 *                       with all the information received); needs gn_iters = 0
 *                       and the exact estimator in the loop.
 * Tracker model (Sec. II; Sec. IV-A-2: each agent keeps a least-squares or a
 * particle-filter model of each target):
 *  est_kind             0: least squares over the window (Sec. III-A);
 *                       1: particle filter of MIL_PF_PARTICLES particles per
 *                       (agent, target) tracker, updated every step with that
 *                       step's range (pooled: also the ranges received from
 *                       the other agents, own first, then in agent order).
 *                       Bootstrap filter: with no belief, the first range
 *                       seeds particle k on its ring (radius r + sigma_l z,
 *                       angle 2 pi (k + u) / 64); with a belief, each particle
 *                       moves by a random walk of std pf_q, the remaining
 *                       ranges weight it by the Gaussian range likelihood of
 *                       std sigma_l = sqrt(range_sigma^2 + pf_lik_sigma^2) and
 *                       systematic resampling draws the new set; the estimate
 *                       is the particles' mean. A tracker without a belief and
 *                       without a range keeps no estimate. Random words:
 *                       Philox(step, env id, (8 agent + target) * 64 + k,
 *                       7 | episode << 4) for particle k. Not with the learned
 *                       estimator in the loop.
 *  pf_q                 random-walk std per step (m), >= 0.
 *  pf_lik_sigma         added in quadrature to the env's range-noise std in
 *                       the likelihood (m), >= 0. */
typedef struct mil_env_params {
  int32_t n_agents, n_targets, ragged, window;
  int32_t episode_len, n_actions, gn_iters, reserved0;
  float dt, area, agent_speed, spawn_agent_radius;
  float action_dpsi[MIL_MAX_ACTIONS];
  float agent_heading_sigma, target_heading_sigma;
  float target_speed_lo, target_speed_hi;
  float range_sigma_lo, range_sigma_hi;
  float det_range, comm_range, comm_loss_p;
  float eps_min, eps_max, d_safe, guard_tau, lost_range;
  int32_t action_mode, n_rudder, reward_mode, spawn_mode;
  float d_follow, spawn_min, spawn_max;
  int32_t pooled;
  int32_t est_kind;
  float pf_q, pf_lik_sigma;
} mil_env_params;

/* Particles per tracker of the particle filter (one wavefront). */
#define MIL_PF_PARTICLES 64

/* Sizes of a created environment batch. */
typedef struct mil_env_layout {
  int64_t num_envs;        /* E */
  int64_t num_agents;      /* A */
  int64_t num_targets;     /* Tt */
  int64_t num_pairs;       /* P */
  int64_t num_tokens;      /* K */
  int64_t num_entities;    /* A + Tt (rows of the global state) */
  int64_t workspace_bytes; /* device workspace to pass to env_bind */
  int32_t window;          /* W */
  int32_t num_classes;     /* distinct (agents, targets) shapes */
} mil_env_layout;

/* Per-step outputs. Any pointer may be NULL (not written). For env_step each
 * array holds one step; for env_rollout it holds T steps, step-major
 * ([T][...]). Alignment: 8 bytes for float arrays.
 *  obs       [K][6] token = (dx, dy, dz, is_self, is_agent, is_target): the
 *            offset of the entity from the observing agent (other agents
 *            from what they broadcast, targets from the agent's own tracker)
 *            and a one-hot type (Sec. IV-A-2 "Observation Space", TransfMAPPO
 *            caption). A missing offset is written as zeros.
 *  obs_mask  [K] uint8, 1 if the offset is present.
 *  reward    [E] team reward: mean over targets of Eq. (1) on the best
 *            tracker's error, or -1 on a crash.
 *  done      [E] uint8.
 *  est       [P][2] each tracker's current (possibly held) estimate.
 *  est_valid [P] uint8, 1 once the tracker has an estimate.
 *  gstate    [A+Tt][6] global state (x, y, z, speed, heading, is_target); per
 *            env its agents then its targets; row offset of env e is
 *            agent_off[e] + target_off[e].
 *  actions   [A] int32, action applied (-1 when the input was invalid).
 *  ranges    [P] measured range (NaN when not detected).
 *  err       [Tt] tracking error e_j of the best tracker (+inf if none). */
typedef struct mil_env_outputs {
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
} mil_env_outputs;

typedef struct mil_env mil_env; /* opaque handle */

/* Create a batch of num_envs environments (host only; no device memory is
 * touched): the Gym-like tracking environment constructed from its agent and
 * target counts (the UTrackingEnv interface sketched in Sec. IV-A-1, with the
 * environment of Sec. IV-A-2 in its simplified GPU form of Sec. IV-A-3),
 * batched over independent environments; each environment is one instance
 * of the Dec-POMDP of Sec. III-B (n = agent count). seed keys every random draw (Philox4x32-10, key = seed): ragged
 * counts, spawns, noise and random actions. counts (optional, host [2][E]:
 * agents then targets) overrides the drawn ragged counts. */
int env_create(const mil_env_params *params, int64_t num_envs, uint64_t seed,
               const int32_t *counts, mil_env **out);
int env_query_layout(const mil_env *h, mil_env_layout *out);
/* Host arrays: env_ids [E] (global id of each packed env), agent_off,
 * target_off, pair_off, token_off [E+1]. Any pointer may be NULL. */
int env_get_order(const mil_env *h, int64_t *env_ids, int64_t *agent_off, int64_t *target_off,
                  int64_t *pair_off, int64_t *token_off);
/* Attach the caller's device workspace (>= workspace_bytes, 256-B aligned)
 * and upload the packed tables. Synchronous on `stream`. */
int env_bind(mil_env *h, void *d_workspace, int64_t bytes, void *stream);
/* Start episode `episode` in every env: reset() of the Gym-like interface
 * (Sec. IV-A-1), returning the first observation and the global state.
 * Spawn agents and targets, draw the per-env range noise, clear trackers
 * and metrics. outs may carry obs /
 * obs_mask / gstate for the initial observation (other fields ignored). */
int env_reset(mil_env *h, uint64_t episode, const mil_env_outputs *outs, void *stream);
/* One step of every env: step(actions) of the Gym-like interface (Sec.
 * IV-A-1), i.e. one transition P(s'|s,u) of the Dec-POMDP (Sec. III-B) with
 * its shared reward r(s,u) (Eq. (1), normalised, crash penalty; Sec.
 * IV-A-2) and per-agent observations O(s,a) (entity tokens, Sec. IV-A-2):
 * turn and move every vehicle (Sec. IV-A-3), draw noisy ranges, update each
 * tracker (Sec. III-A), observe, reward, done. d_actions [A] int32 (packed
 * agent order) or NULL for uniformly random actions drawn in the kernel. */
int env_step(mil_env *h, const int32_t *d_actions, const mil_env_outputs *outs, void *stream);
/* T steps of env_step in one persistent launch (the many-step simulation on
 * the GPU that Sec. IV-A-3 introduces; Table I measures its steps per
 * second); state stays in registers between steps. d_actions [T][A] or NULL
 * (random). Bit-identical to T calls of env_step. */
int env_rollout(mil_env *h, int32_t T, const int32_t *d_actions, const mil_env_outputs *outs,
                void *stream);
/* Capture reset(episode) + rollout(T) + metrics reduction as one HIP graph on
 * `stream` (capture mode: relaxed) and instantiate it; env_graph_launch
 * replays it. Outputs and d_metrics are baked into the graph. */
int env_graph_capture(mil_env *h, uint64_t episode, int32_t T, const mil_env_outputs *outs,
                      double *d_metrics, void *stream);
int env_graph_launch(mil_env *h, void *stream);
/* Reduce the per-env accumulators since the last reset into d_metrics[8]:
 * reward_sum, err_sum, err_sq_sum, err_count, crash_steps, lost_targets,
 * env_steps, agent_steps (sums over all envs; lost is evaluated on the
 * current positions). Deterministic order. */
int env_metrics(mil_env *h, double *d_metrics, void *stream);
/* Synchronise `stream`, read the device status word, clear it. */
int env_status(mil_env *h, uint32_t *host_flags, void *stream);
/* Copy the current state (packed order): d_agent [A][3] (x, y, heading),
 * d_target [Tt][4] (x, y, heading, speed). Either may be NULL. */
int env_get_state(mil_env *h, float *d_agent, float *d_target, void *stream);
/* Choose the env-to-wavefront mapping: `lanes_per_agent` 1 or 2 (targets of
 * an agent split over that many lanes) and `waves_per_block` 1, 2 or 4.
 * Every mapping gives bit-identical results. */
int env_set_mapping(mil_env *h, int32_t lanes_per_agent, int32_t waves_per_block);
int env_get_mapping(const mil_env *h, int32_t *lanes_per_agent, int32_t *waves_per_block);
/* Rollout schedule. chunk_steps = -1: static, one wavefront per group of
 * environments for all T steps. 0 (default): automatic, dynamic with chunks
 * of about 128 steps when the groups number between one and eight times the
 * wavefronts the GPU holds at once and T >= 192 (two chunks or more), else
 * static. > 0: dynamic with chunks of that many steps.
 * Dynamic: the rollout launch is preceded by a small kernel that clears the
 * queue in the workspace; the persistent wavefronts take (chunk, group) units
 * from an atomic counter, chunk-major, save the group's state after each
 * chunk and wait, before a group's next chunk, until the previous one has
 * published its state. Every schedule gives bit-identical results. Setting it
 * drops a captured graph. */
int env_set_schedule(mil_env *h, int32_t chunk_steps);
int env_get_schedule(const mil_env *h, int32_t *chunk_steps);
/* Time every mapping on probe_steps steps writing `outs` (buffers sized for
 * probe_steps steps; NULL = no outputs), with the state saved before and
 * restored after each probe, and keep the fastest. Under the automatic
 * schedule each mapping is probed in the schedule a long rollout of the
 * batch would get with it (dynamic ones in two chunks). If cache_path is not NULL
 * the choice is looked up in, and appended to, that JSON-lines file, keyed by
 * device, batch shape and code version. Needs a reset; synchronous. */
int env_autotune(mil_env *h, int32_t probe_steps, const mil_env_outputs *outs,
                 const char *cache_path, void *stream);
int env_destroy(mil_env *h);
/* Description of the last error on this thread (never NULL). */
const char *env_last_error(void);

/* Range-only localisation of N independent windows (Sec. III-A, linearised
 * least squares about the window centroid, then gn_iters Gauss-Newton steps
 * on the range residuals). d_win [N][W][3] = (agent x, agent y, range); a NaN
 * range marks a missing entry. Outputs d_out [N][2], d_valid [N] (0 when fewer
 * than 3 entries or det <= tau*trace^2). accum: 0 accumulates in FP64, 1 in
 * FP32 (faster, less accurate on ill-conditioned windows). W in 3..64. */
int est_exact(const float *d_win, int64_t N, int32_t W, int32_t gn_iters, float tau, int32_t accum,
              float *d_out, uint8_t *d_valid, void *stream);

/* Philox4x32-10 (Salmon et al., SC'11) on n counters d_ctr [n][4] with key
 * (seed lo, seed hi) -> d_out [n][4]; also the library's transforms of those
 * words: d_u01 [n][4] uniforms ((x>>9)+1/2)/2^23 and d_normal [n][4]
 * Box-Muller pairs of (w0,w1) and (w2,w3). Output pointers may be NULL. */
int rng_philox(const uint32_t *d_ctr, int64_t n, uint64_t seed, uint32_t *d_out, float *d_u01,
               float *d_normal, void *stream);


/* ---------------------------------------------------------------------------
 * Learned range-only estimator (stands in for the exact solve of Sec. III-A;
 * the exact estimator remains its fallback and the judge of its error).
 * Network: 64 -> 128 -> 128 -> 2, GELU (tanh form) after each hidden layer.
 * Parameters: one FP32 vector of mlp_num_params() floats, in this order:
 * W1 [128][64], b1 [128], W2 [128][128], b2 [128], W3 [2][128], b3 [2], each
 * weight matrix row-major (output, input).
 * Features of a window [W][3] = (agent x, agent y, range), W <= 21, all
 * entries present: with abar, rbar the means and theta the direction of the
 * chord from the oldest to the newest agent position (entry W-1 to entry 0),
 * u_k = R(-theta)(a_k - abar); x[3k..3k+2] = (u_k / 10 m, (r_k - rbar) / 10 m),
 * x[3W] = rbar / 1000 m, the rest 0. frame = (abar_x, abar_y, cos theta,
 * sin theta, rbar). The network predicts y = R(-theta)(p - abar) / rbar, so
 * p = abar + rbar R(theta) y.
 * precision: 0 = BF16 operands on MFMA with FP32 accumulation, 1 = FP32
 * operands (FP32 MFMA; for checks). Workspaces are caller-owned device
 * buffers of mlp_workspace_bytes(N, precision) bytes, 256-byte aligned.
 * ------------------------------------------------------------------------- */
int64_t mlp_num_params(void);
int64_t mlp_workspace_bytes(int64_t N, int32_t precision);
/* Glorot-uniform weights (Philox stream keyed by seed), zero biases. */
int mlp_init(float *d_params, uint64_t seed, void *stream);
/* d_win [N][W][3] -> d_x [N][64] (16-byte aligned), d_frame [N][5]. */
int mlp_features(const float *d_win, int64_t N, int32_t W, float *d_x, float *d_frame,
                 void *stream);
/* Normalised training target of estimates d_p [N][2]: d_y [N][2]. */
int mlp_targets(const float *d_frame, const float *d_p, int64_t N, float *d_y, void *stream);
/* d_y [N][2] = network(d_x). */
int mlp_forward(int64_t N, const float *d_x, const float *d_params, float *d_y, int32_t precision,
                void *d_work, int64_t work_bytes, void *stream);
/* Mean over the N samples of |y - target|^2 into *d_loss (may be NULL) and
 * its gradient into d_grad [mlp_num_params()]. Sample s reads row
 * d_index[s] of d_x and d_target (d_index NULL: row s). Deterministic.
 * Precision 0 needs d_x and d_params 16-byte aligned (MIL_EALIGN). */
int mlp_backward(int64_t N, const float *d_x, const int64_t *d_index, const float *d_target,
                 const float *d_params, float *d_grad, float *d_loss, int32_t precision,
                 void *d_work, int64_t work_bytes, void *stream);
/* One Adam step of the BF16 network on N samples: the gradient of
 * mlp_backward (precision 0, same sample selection, deterministic) and the
 * Adam update of mlp_adam_step applied to it, in two kernels: a persistent
 * kernel whose blocks each accumulate the weight gradients of several
 * 32-sample tiles in registers, then a fixed-order reduction that updates
 * d_params, d_m, d_v in place. d_grad (may be NULL) receives the gradient,
 * d_loss (may be NULL) the loss before the update. Workspace as for
 * mlp_backward with precision 0. */
int mlp_train_step(int64_t N, const float *d_x, const int64_t *d_index, const float *d_target,
                   float *d_params, float *d_m, float *d_v, float lr, float beta1, float beta2,
                   float eps, int32_t step, float *d_grad, float *d_loss, void *d_work,
                   int64_t work_bytes, void *stream);
/* Adam (Kingma and Ba) with bias correction on P parameters; step >= 1. */
int mlp_adam_step(int64_t P, float *d_params, const float *d_grad, float *d_m, float *d_v,
                  float lr, float beta1, float beta2, float eps, int32_t step, void *stream);
/* Estimates of N windows: the BF16 network gives the bearing p - c from the
 * window's centroid c; the distance along that bearing is fitted to the
 * window's ranges (three Gauss-Newton steps on the distance, each kept only if
 * the squared residual falls). The estimate is accepted when the RMS over the
 * window of (|p - a_k| - r_k) is <= k_sigma * d_sigma[n]; otherwise (or with a
 * missing entry) the exact solve of est_exact (gn_iters, tau). d_flag [N]:
 * 1 network, 0 exact fallback, 2 neither (exact solve refused). */
int mlp_infer(const float *d_win, int64_t N, int32_t W, const float *d_params,
              const float *d_sigma, float k_sigma, int32_t gn_iters, float tau, float *d_out,
              uint8_t *d_flag, void *d_work, int64_t work_bytes, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mlp_infer
 * with no workspace argument. Same kernels and results as mlp_infer (bit for
 * bit). Its scratch (BF16 weight copies, the fallback counter and list) is one
 * static device array of about 4.4 MB per GPU, held until the process ends;
 * N above MIL_NOALLOC_MAX_WINDOWS is rejected with MIL_EINVAL. Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller. Allocates nothing
 * (no hipMalloc, no hipFree); the array's address is looked up once per device
 * on first use. Errors: as mlp_infer, plus MIL_EHIP if the lookup fails. */
#define MIL_NOALLOC_MAX_WINDOWS (1 << 20)
int mlp_infer_noalloc(const float *d_win, int64_t N, int32_t W, const float *d_params,
                      const float *d_sigma, float k_sigma, int32_t gn_iters, float tau,
                      float *d_out, uint8_t *d_flag, void *stream);
/* Every tracker's current window of a bound environment: d_win [P][W][3]
 * (entry 0 = newest), d_sigma [P] its env's range-noise std, d_truth [P][2]
 * the true target position (either may be NULL). MIL_EINVAL with the
 * particle filter (est_kind 1), which keeps no window. */
int env_windows(mil_env *h, float *d_win, float *d_sigma, float *d_truth, void *stream);
/* The particle filter's state of a bound environment with est_kind = 1:
 * d_particles [P][MIL_PF_PARTICLES][2] (x, y) and d_belief [P] (1 when the
 * tracker holds a belief; either may be NULL), as after the last step. The
 * state is the filter's own (a step after a reset starts from no belief,
 * whatever the arrays hold). MIL_EINVAL when est_kind is 0. */
int env_pf_state(mil_env *h, float *d_particles, uint8_t *d_belief, void *stream);
/* One more particle-filter update of every tracker (est_kind = 1) with the
 * measurements of the last step taken, exactly as the step itself ran it
 * (same random words): the particles move and are weighted and resampled
 * again, and the estimates follow. For callers that time the filter alone or
 * iterate it on one step's ranges. MIL_ESTATE before the first step after a
 * reset, MIL_EINVAL when est_kind is 0. */
int env_pf_update(mil_env *h, void *stream);

/* ---------------------------------------------------------------------------
 * Attention policy: the per-agent transformer actor of Sec. IV-B-1
 * (TransfMAPPO), inference form (BF16 MFMA with FP32 accumulation), plain or
 * with its recurrent token (policy_forward_rec); the training form is with the
 * learner below. Each agent's tokens (its observation, [self, agents, targets],
 * n_tok = n_agents + n_targets <= 16) are embedded 6 -> 64, pass 2 pre-LN
 * layers of 4-head self-attention (keys with mask 0 excluded) and a 256-wide
 * GELU feed-forward block, and the self token's final LayerNorm gives 8
 * logits, of which the first n_actions define the action distribution.
 * Actions are inverse-CDF draws with u from Philox(counter = (step, global env
 * id, agent index, 4 | episode << 4), key = seed).
 * Parameters: one FP32 vector of policy_num_params() floats, in this order:
 * embedding W [64][6], b [64]; per layer: LN1 gain, offset [64], Wqkv
 * [192][64] (Q, K, V rows; head h uses features 16h..16h+15), bqkv [192], Wo
 * [64][64], bo [64], LN2 gain, offset [64], W1 [256][64], b1 [256], W2
 * [64][256], b2 [64]; final LN gain, offset [64]; Wh [8][64], bh [8].
 * ------------------------------------------------------------------------- */
int64_t policy_num_params(void);
/* Workspace for policy_forward / env_policy_rollout (256-byte aligned). */
int64_t policy_workspace_bytes(int64_t num_agents, int64_t num_tokens);
/* Glorot-uniform weights (Philox keyed by seed), LN gains 1, offsets/biases 0. */
int policy_init(float *d_params, uint64_t seed, void *stream);
/* Logits [A][8] (d_logits, may be NULL) and sampled actions [A] (d_actions,
 * may be NULL) of A agents, agent a being agent a % n_agents of env
 * a / n_agents; d_obs [A * n_tok][6], d_mask [A * n_tok]. */
int policy_forward(int64_t A, int32_t n_tok, int32_t n_agents, int32_t n_actions, const float *d_obs,
                   const uint8_t *d_mask, const float *d_params, float *d_logits,
                   int32_t *d_actions, uint64_t seed, uint32_t t, uint32_t episode, void *d_work,
                   int64_t work_bytes, void *stream);
/* policy_forward that also writes d_feat [A][64] (may be NULL): the head's
 * input of each agent, the final LayerNorm of its self token, for the head's
 * gradient (head_grad). */
int policy_forward_feat(int64_t A, int32_t n_tok, int32_t n_agents, int32_t n_actions,
                        const float *d_obs, const uint8_t *d_mask, const float *d_params,
                        float *d_logits, int32_t *d_actions, float *d_feat, uint64_t seed,
                        uint32_t t, uint32_t episode, void *d_work, int64_t work_bytes,
                        void *stream);
/* The recurrent form of the actor (TransfMAPPO, Fig. 3: an extra recurrent
 * embedding is transformed with the entity tokens and the action head reads
 * its output). A carried state d_hidden_in [A][64] (NULL: zeros, an
 * episode's start) enters each agent's residual stream as an unmasked first
 * row, not embedded, ahead of its n_obs <= 15 tokens (d_obs [A * n_obs][6],
 * d_mask [A * n_obs]); the head reads that row's final LayerNorm, which is
 * also written to d_hidden_out [A][64], the next step's state (may equal
 * d_hidden_in: each agent's row is read before it is written). Logits,
 * actions, draws, parameters and workspace as for policy_forward with
 * n_tok = n_obs + 1. Errors: MIL_EINVAL (sizes, null d_hidden_out),
 * MIL_ESHAPE, MIL_EALIGN, MIL_EHIP. */
int policy_forward_rec(int64_t A, int32_t n_obs, int32_t n_agents, int32_t n_actions,
                       const float *d_obs, const uint8_t *d_mask, const float *d_hidden_in,
                       const float *d_params, float *d_logits, int32_t *d_actions,
                       float *d_hidden_out, uint64_t seed, uint32_t t, uint32_t episode,
                       void *d_work, int64_t work_bytes, void *stream);
/* Workspace for env_policy_rollout on this bound batch (256-byte aligned):
 * the policy's, plus (learned != 0) every tracker's window, sigma, estimate
 * and flag and the learned estimator's own workspace. -1 on a bad handle. */
int64_t env_policy_workspace_bytes(const mil_env *h, int32_t learned);
/* Closed loop on a bound fixed-count batch: reset(episode), then T times
 * {policy on the latest observation -> actions; env step}, then (d_metrics
 * not NULL) the metrics reduction. outs as for env_rollout ([T][...]). With
 * capture = 1 the sequence is captured as the handle's HIP graph (replayed by
 * env_graph_launch) instead of run.
 * d_mlp_params (may be NULL): parameters of the learned estimator (mlp_*). When
 * given, each env step is split around it: the step moves the entities, draws
 * the ranges, pushes the windows and writes every tracker's window to the
 * workspace; they go through mlp_infer (residual test at k_sigma * sigma_r,
 * exact fallback); then the step
 * takes those estimates (for trackers whose window is full; shorter windows keep
 * the exact estimator) and computes reward and observation. Needs window <= 21.
 * d_hidden [A][64] (may be NULL): when given, the actor runs in its recurrent
 * form (policy_forward_rec) with the carried state kept there: zeros at the
 * reset, each step's state written over the last (the final one is left
 * there); n_agents + n_targets + 1 <= 16.
 * Errors: MIL_EINVAL (ragged batch, too many tokens or actions, bad T/episode,
 * window too long for the learned estimator), MIL_ESHAPE (workspace smaller
 * than env_policy_workspace_bytes), MIL_EALIGN, MIL_EHIP. */
int env_policy_rollout(mil_env *h, uint64_t episode, int32_t T, const float *d_params,
                       const float *d_mlp_params, float k_sigma, float *d_hidden,
                       const mil_env_outputs *outs, double *d_metrics, int32_t capture,
                       void *d_work, int64_t work_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * The learner's forward half (Sec. III-B: MAPPO updates the actors with the
 * PPO clipped surrogate objective and one centralised critic V(S) estimates
 * the value of the global state; Sec. IV-B-1, Fig. 3: the TransformerCritic
 * reads the full global state as entity tokens plus one embedding token whose
 * transformed output gives V; plain, or with that token recurrent), the
 * gradient of the two output heads, and the networks' training form (the
 * gradient of every parameter).
 * ------------------------------------------------------------------------- */
/* Workspace for critic_forward (256-byte aligned); -1 on bad sizes. */
int64_t critic_workspace_bytes(int64_t N, int32_t n_agents, int32_t n_targets);
/* V of N global states of fixed-count envs: d_gstate [N][n_agents +
 * n_targets][6], the rows env_rollout records in outs->gstate (x, y, z,
 * speed, heading, is_target; one step of a batch is N = num_envs states).
 * Each state becomes 1 + n_agents + n_targets <= 16 tokens: an all-zero token
 * (its embedding is the embedding bias; its output carries V), then each
 * agent and target as (x / pos_scale, y / pos_scale, v cos(heading),
 * v sin(heading), is_agent, is_target). The network is the policy's (same
 * parameter layout, policy_init, BF16 MFMA with FP32 accumulation) and V is
 * the first output of its head on the first token. d_values [N] (FP32);
 * d_feat [N][64] (may be NULL): the head's input of each state.
 * Errors: MIL_EINVAL (sizes, pos_scale <= 0), MIL_ESHAPE, MIL_EALIGN, MIL_EHIP. */
int critic_forward(const float *d_gstate, int64_t N, int32_t n_agents, int32_t n_targets,
                   float pos_scale, const float *d_params, float *d_values, float *d_feat,
                   void *d_work, int64_t work_bytes, void *stream);
/* The recurrent critic (Fig. 3: the TransformerCritic keeps a recurrent
 * embedding from which V is read) over T steps of N envs in order: at step t
 * the state carried from step t - 1 (d_hidden_in [N][64] at t = 0, NULL:
 * zeros) is the unmasked first row ahead of the n_agents + n_targets entity
 * tokens of d_gstate[t] ([T][N][n_agents + n_targets][6], tokens as for
 * critic_forward, no all-zero token); V_t = d_values[t] ([T][N]) is the
 * head's first output on that row's final LayerNorm, which is the next
 * state: d_hidden_seq [T][N][64] receives every step's (the head's inputs
 * for head_grad; the last is the state after the last step). Workspace
 * critic_workspace_bytes(N, ...) (one step's tokens). Errors as for
 * critic_forward. */
int critic_forward_rec(const float *d_gstate, int32_t T, int64_t N, int32_t n_agents,
                       int32_t n_targets, float pos_scale, const float *d_params,
                       const float *d_hidden_in, float *d_values, float *d_hidden_seq,
                       void *d_work, int64_t work_bytes, void *stream);
/* Training form of the networks (the gradient step of MAPPO, Sec. III-B,
 * through the TransfMAPPO actor and critic of Fig. 3): an FP32 forward pass
 * that records every intermediate in the workspace (the tape), then its
 * exact reverse pass into the gradient of every parameter. The per-row work
 * (embedding, LayerNorms, attention with its softmax and key mask, tanh
 * GELU, head), the weight gradients and the feed-forward up-projection
 * (FP32 matrix cores) run in the library's kernels, the other dense products in hipBLASLt and rocBLAS FP32
 * GEMMs; every sum is taken in a fixed order, so results do not depend on
 * the run. Rows as for policy_forward (n_tok per agent) or, with rec = 1,
 * the recurrent form of policy_forward_rec (n_tok - 1 observed tokens per
 * agent after the carried state). The library keeps one rocBLAS and one
 * hipBLASLt handle per device for these calls (made on the first call):
 * calls on one device must not overlap from several host threads. Within one call the carried state is an
 * input: its gradient is returned; a sequence is differentiated through the
 * state by chaining the calls (policy_train_backward). */
/* Workspace of the training form for A agents of n_tok rows (256-byte
 * aligned; about 11 KB per row plus 36 MB of partial sums); -1 on bad sizes. */
int64_t policy_train_workspace_bytes(int64_t A, int32_t n_tok);
/* Forward pass: d_obs [A * (n_tok - rec)][6], d_mask, d_hidden_in [A][64]
 * (rec = 1; NULL: zeros) -> d_logits [A][8] (may be NULL), d_feat [A][64]
 * (the head's inputs, may be NULL); the tape stays in d_work for
 * policy_train_backward. Errors: MIL_EINVAL (sizes, A < 1, null inputs),
 * MIL_ESHAPE, MIL_EALIGN, MIL_EHIP. */
int policy_train_forward(int64_t A, int32_t n_tok, int32_t rec, const float *d_obs,
                         const uint8_t *d_mask, const float *d_hidden_in, const float *d_params,
                         float *d_logits, float *d_feat, void *d_work, int64_t work_bytes,
                         void *stream);
/* The critic's forward pass on N global states (tokens as critic_forward;
 * rec = 1: the recurrent critic's step, entity tokens after the carried state
 * d_hidden_in) -> d_values [N], d_feat [N][64] (may be NULL); the tape is
 * that of policy_train_forward with A = N, n_tok = n_agents + n_targets + 1. */
int critic_train_forward(const float *d_gstate, int64_t N, int32_t n_agents, int32_t n_targets,
                         float pos_scale, int32_t rec, const float *d_hidden_in,
                         const float *d_params, float *d_values, float *d_feat, void *d_work,
                         int64_t work_bytes, void *stream);
/* Reverse pass of the last forward pass recorded in d_work (same A, n_tok,
 * rec, parameters): d_dout [A][ld] the loss gradient at the first n_out
 * outputs (ppo_objective's d_dlogits with ld 8; the critic's d_dvalues with
 * ld 1, n_out 1); d_dnext [A][64] (may be NULL) the loss gradient at the
 * head's input, which in the recurrent form is the state passed on to the
 * next step -> d_grad [policy_num_params()] (layout of the parameters;
 * overwritten, or added to with accumulate = 1), d_dhidden [A][64] (rec = 1,
 * may be NULL) the gradient at the carried state. Back-propagation through
 * time: the steps in reverse order, each forward pass taken again from its
 * input state, d_dnext = the following step's d_dhidden, accumulate = 1 after
 * the first. Errors as for policy_train_forward. */
int policy_train_backward(int64_t A, int32_t n_tok, int32_t rec, const float *d_params,
                          const float *d_dout, int32_t ld, int32_t n_out, const float *d_dnext,
                          int32_t accumulate, float *d_grad, float *d_dhidden, void *d_work,
                          int64_t work_bytes, void *stream);
/* Generalised advantage estimation (Schulman et al. 2016; the advantage
 * estimator of MAPPO) over T steps of E envs with the env's shared reward:
 * d_rewards [T][E], d_dones [T][E] (1: the step ends its episode, nothing is
 * bootstrapped past it), d_values [T + 1][E] (V of the state before step t,
 * row T the state after the last step). delta_t = r_t + gamma V_{t+1} (1 -
 * d_t) - V_t, A_t = delta_t + gamma lambda (1 - d_t) A_{t+1}; writes d_adv
 * [T][E] and the value targets d_ret [T][E] = A_t + V_t (FP64 recurrence,
 * FP32 output). gamma, lambda in [0, 1]. */
int ppo_gae(const float *d_rewards, const uint8_t *d_dones, const float *d_values, int32_t T,
            int64_t E, float gamma, float lambda, float *d_adv, float *d_ret, void *stream);
/* Bytes of the ppo_objective and head_grad workspace (8-byte aligned). */
int64_t ppo_workspace_bytes(void);
/* Gradient of the output head (the last linear layer of the policy or of the
 * critic) from the gradients at its outputs: d_feat [N][64] the head's inputs
 * (policy_forward_feat, critic_forward), d_dout [N][ld] the gradients at the
 * first n_out outputs (d_dlogits of ppo_objective with ld 8; d_dvalues with ld
 * 1, n_out 1). d_grad [8 * 64 + 8] in the head's parameter layout (Wh then
 * bh, the last 520 floats of the parameter vector): rows n_out..7 are 0, so
 * mlp_adam_step over those 520 floats updates the head. FP64 sums in a fixed
 * order; N = 0 gives a zero gradient (d_feat and d_dout may then be
 * NULL). The layers below the head are not differentiated here. Errors: MIL_EINVAL (N < 0, n_out outside 1..8,
 * ld < n_out, null pointer), MIL_ESHAPE (workspace), MIL_EHIP. */
int head_grad(int64_t N, const float *d_feat, const float *d_dout, int32_t ld, int32_t n_out,
              float *d_grad, void *d_work, int64_t work_bytes, void *stream);
/* The clipped PPO objective over T steps of A agents (agent a of env
 * a / n_agents, sharing its env's advantage): d_logits_new / d_logits_old
 * [T][A][8] (the first n_actions are the action logits: the policy at update
 * time and at sampling time), d_actions [T][A], d_adv [T][E], d_values and
 * d_returns [T][E] (critic output and targets). With rho = pi_new(a) /
 * pi_old(a), writes d_out [4] (FP64): policy loss -mean min(rho A, clip(rho,
 * 1 - clip_eps, 1 + clip_eps) A), value loss mean (V - R)^2, entropy mean
 * H(pi_new), and the fraction of samples where the clipped term is strictly
 * the smaller; d_dlogits [T][A][8] (may be NULL): d(policy loss)/d
 * logits_new (0 where the clipped term is the minimum; columns n_actions..7
 * are 0); d_dvalues [T][E] (may be NULL): d(value loss)/dV. Sums reduce in a
 * fixed order: results do not depend on the launch. */
int ppo_objective(const float *d_logits_new, const float *d_logits_old, const int32_t *d_actions,
                  const float *d_adv, const float *d_values, const float *d_returns, int32_t T,
                  int64_t A, int32_t n_agents, int32_t n_actions, float clip_eps, double *d_out,
                  float *d_dlogits, float *d_dvalues, void *d_work, int64_t work_bytes,
                  void *stream);

#ifdef __cplusplus
}
#endif
#endif
