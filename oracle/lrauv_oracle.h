/*
 * FP64 CPU oracle of the batched range-only tracking environment.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, plain reference that
 * the GPU path is checked against. Only the test suite, the package's smoke
 * check and the benchmark's CPU-baseline leg may load it. It shares no code,
 * header, table or helper with the HIP library; its only common ground with
 * the GPU side is the parameter values and seeds that a test passes to both.
 *
 * Paper: "Scaling Multi-Agent Reinforcement Learning for Underwater Acoustic
 * Tracking via Autonomous Vehicles" (arXiv 2505.08222).
 *   - kinematic surrogate and heading noise: Sec. IV-A-3 (JaxLrauv);
 *   - step structure, per-(agent,target) tracker, spawn: Sec. IV-A-2;
 *   - observation and global state: Sec. IV-A-2, "Observation Space" and the
 *     TransfMAPPO figure caption (Sec. IV-B-1);
 *   - tracking reward: Eq. (1); normalisation and crash penalty: text after
 *     Eq. (2);
 *   - range-only least-squares localisation: Sec. III-A;
 *   - partial observability limits (450 m detection, 1500 m comms): Sec.
 *     IV-A-2, "Why is UTracking a difficult environment?".
 * Where the paper is silent (RNG assignment, estimator guards, the multi-agent
 * tracking error) the oracle follows the readings stated at each function.
 *
 * Parity status per function is stated next to each declaration.
 */
#ifndef LRAUV_ORACLE_H
#define LRAUV_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Environment parameters, SI units, FP64. */
typedef struct orc_params {
  int32_t n_agents;        /* fixed count, or the maximum when ragged (<= 8) */
  int32_t n_targets;       /* fixed count, or the maximum when ragged (<= 8) */
  int32_t ragged;          /* 1: per-env counts drawn uniformly in 1..max */
  int32_t window;          /* W: length of the range history per pair */
  int32_t episode_len;     /* steps per episode; done is raised on the last */
  int32_t n_actions;       /* number of heading-change actions (<= 8) */
  int32_t gn_iters;        /* Gauss-Newton refinements after the linear LS */
  int32_t pad_;
  double dt;               /* step duration (s) */
  double area;             /* side of the square spawn area for targets (m) */
  double agent_speed;      /* constant agent speed v (m/s) */
  double spawn_agent_radius; /* agents spawn uniformly in this disk (m) */
  double action_dpsi[8];   /* heading change per action (rad) */
  double agent_heading_sigma;  /* std of the heading noise added per step */
  double target_heading_sigma; /* std of the target random-walk jitter */
  double target_speed_lo, target_speed_hi; /* per-target speed range */
  double range_sigma_lo, range_sigma_hi;   /* per-env range-noise std range */
  double det_range;        /* ranges beyond this true distance are missing */
  double comm_range;       /* agent positions beyond this are not received */
  double comm_loss_p;      /* probability an agent's broadcast is dropped */
  double eps_min, eps_max; /* Eq. (1) thresholds */
  double d_safe;           /* crash distance between agents */
  double guard_tau;        /* conditioning guard of the 2x2 solves */
  double lost_range;       /* a target is lost at episode end when every
                              agent is farther than this (m) */
  /* Paper-faithful variants (Sec. IV-A-2). */
  int32_t action_mode;     /* 0: action k turns the heading by action_dpsi[k];
                              1: rudder state: actions 0, 1, 2 move the rudder one
                              position down, keep it, move it one position up
                              ("Actions Space": only adjacent angles), and the
                              heading changes by action_dpsi[rudder], the paper's
                              linear theta(gamma) at each rudder angle */
  int32_t n_rudder;        /* rudder positions in action_mode 1 (<= 8); they
                              start at the middle one */
  int32_t reward_mode;     /* 0: tracking reward Eq. (1); 1: follow reward Eq. (2) */
  int32_t spawn_mode;      /* 0: agents in the disk, targets in the square;
                              1: every entity at least spawn_min from every other
                              and at most spawn_max apart (Sec. IV-A-2); needs
                              n_agents + n_targets <= 13 and
                              spawn_max >= 2 sqrt(3) spawn_min */
  double d_follow;         /* Eq. (2): a target is followed when some agent is
                              within this distance (m) */
  double spawn_min, spawn_max; /* pairwise spawn distances of spawn_mode 1 (m) */
  int32_t pooled;          /* 1: each agent's tracker of a target also uses the
                              ranges to it that the agent received from the other
                              agents (Sec. IV-A-2: every tracker is updated with
                              all the information received); 0: own ranges only */
  int32_t pad2_;
  /* Tracker model (Sec. II and Sec. IV-A-2: each agent keeps a least-squares
   * or a particle-filter model of each target). */
  int32_t est_kind;        /* 0: least squares over the window (Sec. III-A);
                              1: particle filter of ORC_PF_N particles, updated
                              with this step's ranges (see orc_pf_update) */
  int32_t pad3_;
  double pf_q;             /* std of each particle's random-walk move per step (m) */
  double pf_lik_sigma;     /* added in quadrature to the env's range-noise std to
                              give the likelihood's std (m) */
} orc_params;

/* Particles per tracker of the particle filter. */
#define ORC_PF_N 64

/* Per-step records of an oracle rollout. Every pointer may be NULL. Entity
 * arrays follow the selected envs in the order given, agents / targets /
 * (agent,target) pairs / observation tokens concatenated env by env (CSR).
 * T = number of steps recorded. */
typedef struct orc_traj {
  double  *init_agent;   /* [A][3]  x, y, psi right after reset */
  double  *init_target;  /* [Tt][4] x, y, psi, speed right after reset */
  double  *sigma_r;      /* [E] range-noise std of each env */
  double  *init_obs;     /* [K][6] observation right after reset */
  uint8_t *init_mask;    /* [K] */
  double  *agent;        /* [T][A][3] after each step */
  double  *target;       /* [T][Tt][4] after each step */
  double  *ranges;       /* [T][P] measured range, NaN when not detected */
  double  *est;          /* [T][P][2] current (possibly held) estimate */
  uint8_t *est_valid;    /* [T][P] 1 if an estimate exists */
  uint8_t *est_fresh;    /* [T][P] 1 if solved this step (not held) */
  double  *sens;         /* [T][P] sensitivity of the current estimate:
                            sum over window inputs of |d est / d input| (m/m) */
  double  *err;          /* [T][Tt] tracking error e_j, +inf when none */
  double  *reward;       /* [T][E] */
  uint8_t *crash;        /* [T][E] 1 if the crash penalty applied */
  uint8_t *done;         /* [T][E] */
  double  *obs;          /* [T][K][6] tokens (dx,dy,dz,is_self,is_agent,is_target) */
  uint8_t *obs_mask;     /* [T][K] */
  int32_t *actions;      /* [T][A] action index applied */
  double  *env_metrics;  /* [E][6] reward_sum, err_sum, err_sq_sum, err_count,
                            crash_steps, lost_targets_at_end */
} orc_traj;

/* ---- counter-based RNG (Salmon et al., SC'11, Philox4x32 with 10 rounds).
 * Pinned: published known-answer vectors and the rocRAND generator. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Bulk form used by tests: n counters [n][4] -> n outputs [n][4]. */
void orc_philox_bulk(int64_t n, const uint32_t *ctr, uint64_t seed, uint32_t *out);
/* Uniform in (0,1) from the top 23 bits, exact in binary32 and binary64. */
double orc_u01(uint32_t x);
/* Box-Muller (1958): two standard normals from two words. */
void orc_normal2(uint32_t x0, uint32_t x1, double *z0, double *z1);
/* floor(n * x / 2^32): uniform choice in 0..n-1. */
uint32_t orc_choice(uint32_t x, uint32_t n);

/* ---- per-env counts of a ragged batch (pinned: bounds and uniformity). */
void orc_env_counts(const orc_params *p, uint64_t seed, int64_t n,
                    const int64_t *env_ids, int32_t *n_agents, int32_t *n_targets);

/* ---- range-only localisation of one target from one agent's window
 * (Sec. III-A, linearised least squares, optional Gauss-Newton on the range
 * residuals). Inputs: n entries of agent position (ax, ay) and range r.
 * Returns 1 and writes (px, py) on success, 0 when fewer than 3 entries or
 * the conditioning guard fails. Pinned: exact recovery, numpy lstsq, grid
 * search, equivariance. */
int orc_ls_estimate(int n, const double *ax, const double *ay, const double *r,
                    int gn_iters, double tau, double *px, double *py);
/* Same solve, also returning the finite-difference sensitivity described for
 * orc_traj.sens (used to derive per-element parity tolerances). */
int orc_ls_estimate_sens(int n, const double *ax, const double *ay, const double *r,
                         int gn_iters, double tau, double *px, double *py, double *sens);
/* Batched form over windows [N][W][3] = (ax, ay, r), r NaN = missing entry,
 * W <= 512 rows (pooled windows of 8 agents x 64 entries). Entries are taken
 * in window order; out [N][2]; valid [N]. */
void orc_ls_batch(int64_t N, int W, const double *win, int gn_iters, double tau,
                  double *out, uint8_t *valid, int n_threads);

/* ---- Eq. (1): tracking reward of one target with error e. */
double orc_tracking_reward(double e, double eps_min, double eps_max);
/* ---- Eq. (2): follow reward of one target whose nearest agent is at
 * distance d. Pinned: worked values. */
double orc_follow_reward(double d, double d_follow);
/* ---- spawn_mode 1 placement of n <= 13 entities (agents first, then
 * targets, as in a reset) of env `env_id`: x, y [n]. Returns 0, or -1 with
 * more than 13 entities. Pinned: pairwise bounds by brute force. */
int orc_spawn_pairwise(const orc_params *p, uint64_t seed, uint64_t episode, uint32_t env_id,
                       int n_agents, int n_targets, double *x, double *y);

/* ---- one update of one tracker's particle filter (Sec. II: particles
 * moved by a motion model and resampled by the measurement likelihood; the
 * reading, a bootstrap filter with a random-walk move, a Gaussian range
 * likelihood and systematic resampling, is spelled out at the definition).
 * n <= 1024 particles (px, py), updated in place; init: 1 when they hold a
 * belief; m measurement rows (ax, ay, r), the first of which seeds the belief
 * when init is 0; sigma_l: likelihood std; q: move std. Random inputs:
 * zw [n][2] the two words particle k's normals come from (Box-Muller), uw [n]
 * the word of its seeding angle, uoff the word of the resampling offset.
 * Returns 1 with the estimate (the particles' mean) in (ex, ey) when the
 * tracker holds a belief afterwards, 0 when it has none (init 0 and no row;
 * nothing written). src [n] (may be NULL): the index each particle was copied
 * from by the resampling, -1 when there was none. Pinned: two-particle closed
 * form of the resampling decision, offspring counts of systematic
 * resampling, ring seeding geometry, translation equivariance, convergence
 * on a static target. */
int orc_pf_update(int n, double *px, double *py, int init, int m, const double *ax,
                  const double *ay, const double *r, double sigma_l, double q,
                  const uint32_t *zw, const uint32_t *uw, uint32_t uoff, double *ex, double *ey,
                  int32_t *src);

/* ---- full episode(s): reset then T steps for the selected envs.
 * env_ids: global env ids (they key the RNG); counts per selected env.
 * actions: [T][A] action indices, or NULL for the random policy.
 * Returns 0, or -1 on invalid arguments. */
int orc_rollout(const orc_params *p, uint64_t seed, uint64_t episode,
                int64_t n_sel, const int64_t *env_ids,
                const int32_t *n_agents, const int32_t *n_targets,
                int32_t T, const int32_t *actions, orc_traj *out, int n_threads);

#ifdef __cplusplus
}
#endif
#endif
