/*
 * FP64 CPU oracle of the batched range-only tracking environment.
 * TEST INFRASTRUCTURE ONLY (see lrauv_oracle.h): plain, slow, one env at a
 * time, written for checking by eye against the paper (arXiv 2505.08222).
 * Nothing here is blocked, fused or reordered for speed; the only
 * parallelism is an OpenMP loop over independent environments, used when the
 * oracle is timed as a CPU baseline.
 */
#include "lrauv_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OMAX 8   /* most agents / targets per env */
#define OWMAX 64 /* longest window */
#define OROWS (OMAX * OWMAX) /* most rows of one tracker's solve (pooled windows) */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, as defined by Salmon, Moraes, Dror and Shaw, "Parallel    */
/* random numbers: as easy as 1, 2, 3" (SC'11): a 4-word counter and a     */
/* 2-word key; each round multiplies words 0 and 2 by fixed odd constants,  */
/* swaps the halves of the 64-bit products with words 1 and 3 XOR the key,  */
/* and the key is bumped by the Weyl constants (golden ratio and sqrt(3)-1  */
/* scaled to 32 bits) between rounds.                                       */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = M0 * (uint64_t)c0;
    uint64_t p1 = M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_philox_bulk(int64_t n, const uint32_t *ctr, uint64_t seed, uint32_t *out) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

double orc_u01(uint32_t x) { return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0); }

void orc_normal2(uint32_t x0, uint32_t x1, double *z0, double *z1) {
  const double two_pi = 6.283185307179586476925286766559;
  double u0 = orc_u01(x0), u1 = orc_u01(x1);
  double rad = sqrt(-2.0 * log(u0));
  *z0 = rad * cos(two_pi * u1);
  *z1 = rad * sin(two_pi * u1);
}

uint32_t orc_choice(uint32_t x, uint32_t n) { return (uint32_t)(((uint64_t)x * n) >> 32); }

/* A heading is an angle: kept in [-pi, pi] after every update (one
 * correction suffices, a step turns by far less than pi). */
static double wrap_angle(double a) {
  const double pi = 3.14159265358979323846;
  if (a > pi) return a - 2.0 * pi;
  if (a < -pi) return a + 2.0 * pi;
  return a;
}

/* RNG counter words: (step or 0, global env id, entity code, purpose). */
enum {
  PURPOSE_DYNAMICS = 0,
  PURPOSE_MEASURE = 1,
  PURPOSE_RESET = 2,
  PURPOSE_CONFIG = 3,
  PURPOSE_PF = 7,     /* particle filter: normals of particle pair h at entity
                         (8 agent + target) * 32 + h; resampling offset at
                         ENT_PF_OFFSET + 8 agent + target */
  PURPOSE_PF_SEED = 8 /* particle filter: seeding angles, entity as the normals */
};
enum { ENT_TARGET_BLOCK = 16, ENT_RANGE_ROW = 64, ENT_ENV = 127, ENT_PF_OFFSET = 2048 };

static void draw(uint64_t seed, uint32_t c0, uint32_t env, uint32_t entity, uint32_t c3,
                 uint32_t out[4]) {
  uint32_t ctr[4] = {c0, env, entity, c3};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

void orc_env_counts(const orc_params *p, uint64_t seed, int64_t n, const int64_t *env_ids,
                    int32_t *n_agents, int32_t *n_targets) {
  for (int64_t k = 0; k < n; ++k) {
    if (!p->ragged) {
      n_agents[k] = p->n_agents;
      n_targets[k] = p->n_targets;
      continue;
    }
    uint32_t x[4];
    draw(seed, 0u, (uint32_t)env_ids[k], 0u, PURPOSE_CONFIG, x);
    n_agents[k] = 1 + (int32_t)orc_choice(x[0], (uint32_t)p->n_agents);
    n_targets[k] = 1 + (int32_t)orc_choice(x[1], (uint32_t)p->n_targets);
  }
}

/* ------------------------------------------------------------------------ */
/* Range-only localisation (Sec. III-A: trilateration linearised by least     */
/* squares). With a_k the agent positions and r_k the ranges, the squared    */
/* range equations |a_k - p|^2 = r_k^2 are written about the window centroid */
/* abar (p = abar + q, u_k = a_k - abar): 2 u_k.q - |q|^2 = |u_k|^2 - r_k^2. */
/* Treating |q|^2 as a free unknown and using sum u_k = 0, the least-squares */
/* q solves S q = g / 2 with S = sum u_k u_k^T and g = sum u_k c_k,          */
/* c_k = |u_k|^2 - (r_k^2 - rbar^2) (rbar^2 may be added because sum u_k = 0,*/
/* and r_k^2 - rbar^2 = d_k (2 rbar + d_k) with d_k = r_k - rbar).           */
/* Optional Gauss-Newton refinement minimises sum (|p - a_k| - r_k)^2.       */
/* ------------------------------------------------------------------------ */
static double range_cost(int n, const double *ax, const double *ay, const double *r, double px,
                         double py) {
  double J = 0.0;
  for (int k = 0; k < n; ++k) {
    double res = hypot(px - ax[k], py - ay[k]) - r[k];
    J += res * res;
  }
  return J;
}

int orc_ls_estimate(int n, const double *ax, const double *ay, const double *r, int gn_iters,
                    double tau, double *px, double *py) {
  if (n < 3) return 0;
  double mx = 0.0, my = 0.0, mr = 0.0;
  for (int k = 0; k < n; ++k) {
    mx += ax[k];
    my += ay[k];
    mr += r[k];
  }
  mx /= n;
  my /= n;
  mr /= n;
  double sxx = 0.0, sxy = 0.0, syy = 0.0, gx = 0.0, gy = 0.0;
  for (int k = 0; k < n; ++k) {
    double ux = ax[k] - mx, uy = ay[k] - my, d = r[k] - mr;
    double c = ux * ux + uy * uy - d * (2.0 * mr + d);
    sxx += ux * ux;
    sxy += ux * uy;
    syy += uy * uy;
    gx += ux * c;
    gy += uy * c;
  }
  double det = sxx * syy - sxy * sxy;
  double tr = sxx + syy;
  if (!(det > tau * tr * tr)) return 0;
  double qx = 0.5 * (syy * gx - sxy * gy) / det;
  double qy = 0.5 * (sxx * gy - sxy * gx) / det;
  double x = mx + qx, y = my + qy;

  for (int it = 0; it < gn_iters; ++it) {
    double hxx = 0.0, hxy = 0.0, hyy = 0.0, bx = 0.0, by = 0.0;
    for (int k = 0; k < n; ++k) {
      double dx = x - ax[k], dy = y - ay[k];
      double dist = hypot(dx, dy);
      if (dist <= 0.0) continue;
      double jx = dx / dist, jy = dy / dist, rho = dist - r[k];
      hxx += jx * jx;
      hxy += jx * jy;
      hyy += jy * jy;
      bx += jx * rho;
      by += jy * rho;
    }
    double dh = hxx * hyy - hxy * hxy, th = hxx + hyy;
    if (!(dh > tau * th * th)) break;
    double sx = -(hyy * bx - hxy * by) / dh;
    double sy = -(hxx * by - hxy * bx) / dh;
    double j0 = range_cost(n, ax, ay, r, x, y);
    double j1 = range_cost(n, ax, ay, r, x + sx, y + sy);
    if (!(j1 < j0)) break;
    x += sx;
    y += sy;
  }
  *px = x;
  *py = y;
  return 1;
}

int orc_ls_estimate_sens(int n, const double *ax, const double *ay, const double *r, int gn_iters,
                         double tau, double *px, double *py, double *sens) {
  int ok = orc_ls_estimate(n, ax, ay, r, gn_iters, tau, px, py);
  if (!ok) return 0;
  if (n > OROWS) return 0;
  double bx[OROWS], by[OROWS], br[OROWS];
  memcpy(bx, ax, sizeof(double) * n);
  memcpy(by, ay, sizeof(double) * n);
  memcpy(br, r, sizeof(double) * n);
  double total = 0.0;
  double *cols[3] = {bx, by, br};
  for (int c = 0; c < 3; ++c) {
    for (int k = 0; k < n; ++k) {
      double v = cols[c][k];
      double h = 1e-6 * (fabs(v) > 1.0 ? fabs(v) : 1.0);
      double xp, yp, xm, ym;
      cols[c][k] = v + h;
      int okp = orc_ls_estimate(n, bx, by, br, gn_iters, tau, &xp, &yp);
      cols[c][k] = v - h;
      int okm = orc_ls_estimate(n, bx, by, br, gn_iters, tau, &xm, &ym);
      cols[c][k] = v;
      if (!okp || !okm) {
        total = INFINITY;
        continue;
      }
      total += hypot(xp - xm, yp - ym) / (2.0 * h);
    }
  }
  *sens = total;
  return 1;
}

void orc_ls_batch(int64_t N, int W, const double *win, int gn_iters, double tau, double *out,
                  uint8_t *valid, int n_threads) {
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < N; ++i) {
    double ax[OROWS], ay[OROWS], r[OROWS];
    int n = 0;
    for (int k = 0; k < W && k < OROWS; ++k) {
      const double *e = win + (i * W + k) * 3;
      if (isnan(e[2])) continue;
      ax[n] = e[0];
      ay[n] = e[1];
      r[n] = e[2];
      ++n;
    }
    double x = 0.0, y = 0.0;
    int ok = orc_ls_estimate(n, ax, ay, r, gn_iters, tau, &x, &y);
    out[2 * i] = ok ? x : 0.0;
    out[2 * i + 1] = ok ? y : 0.0;
    valid[i] = (uint8_t)ok;
  }
}

/* ------------------------------------------------------------------------ */
/* Particle-filter tracker (Sec. II: a belief over the target's position held */
/* as particles, moved by a motion model and resampled by the likelihood of   */
/* the measured ranges). The paper names no variant; the reading is the       */
/* bootstrap filter:                                                          */
/*   seed   (no belief yet, first row (a, r)): particle k on the ring about a */
/*          of radius r + sigma_l z_k at angle 2 pi (k + u_k) / n (one        */
/*          particle per equal sector of the circle);                         */
/*   move   (belief held): x_k <- x_k + q (z_k, z'_k), a random walk;         */
/*   weight (rows not used to seed): w_k = prod_rows                          */
/*          exp(-(|x_k - a| - r)^2 / (2 sigma_l^2)), taken relative to the    */
/*          largest (the normalisation cancels in the resampling);            */
/*   resample (systematic, Kitagawa 1996): with C_m = w_0 + ... + w_m and one */
/*          offset U in [0, 1), output k copies particle                      */
/*          min{ m : C_m > (k + U) C_{n-1} / n } (the last one if none);      */
/*   estimate: the mean of the particles.                                     */
/* z_k, z'_k: Box-Muller of particle k's two normal words zw[2k], zw[2k+1];   */
/* u_k = u01(uw[k]); U = u01(uoff). How a step's words come from Philox is    */
/* the caller's (see the tracker in env_step).                                */
/* ------------------------------------------------------------------------ */
#define ORC_PF_MAX 1024

int orc_pf_update(int n, double *px, double *py, int init, int m, const double *ax,
                  const double *ay, const double *r, double sigma_l, double q,
                  const uint32_t *zw, const uint32_t *uw, uint32_t uoff, double *ex, double *ey,
                  int32_t *src) {
  const double two_pi = 6.283185307179586476925286766559;
  if (n < 1 || n > ORC_PF_MAX) return 0;
  if (!init && m < 1) return 0;
  int first = 0; /* rows before this one seeded the belief */
  if (!init) {
    for (int k = 0; k < n; ++k) {
      double z0, z1;
      orc_normal2(zw[2 * k], zw[2 * k + 1], &z0, &z1);
      const double ang = two_pi * ((double)k + orc_u01(uw[k])) / (double)n;
      const double rad = r[0] + sigma_l * z0;
      px[k] = ax[0] + rad * cos(ang);
      py[k] = ay[0] + rad * sin(ang);
    }
    first = 1;
  } else {
    for (int k = 0; k < n; ++k) {
      double z0, z1;
      orc_normal2(zw[2 * k], zw[2 * k + 1], &z0, &z1);
      px[k] += q * z0;
      py[k] += q * z1;
    }
  }
  if (src)
    for (int k = 0; k < n; ++k) src[k] = -1;
  if (m > first) {
    double lw[ORC_PF_MAX], cum[ORC_PF_MAX], ox[ORC_PF_MAX], oy[ORC_PF_MAX];
    double best = -INFINITY;
    for (int k = 0; k < n; ++k) {
      lw[k] = 0.0;
      for (int row = first; row < m; ++row) {
        const double res = hypot(px[k] - ax[row], py[k] - ay[row]) - r[row];
        lw[k] -= res * res / (2.0 * sigma_l * sigma_l);
      }
      if (lw[k] > best) best = lw[k];
    }
    double total = 0.0;
    for (int k = 0; k < n; ++k) {
      total += exp(lw[k] - best);
      cum[k] = total;
    }
    const double U = orc_u01(uoff);
    for (int k = 0; k < n; ++k) {
      const double point = ((double)k + U) / (double)n * total;
      int j = 0;
      while (j < n - 1 && !(cum[j] > point)) ++j;
      ox[k] = px[j];
      oy[k] = py[j];
      if (src) src[k] = j;
    }
    for (int k = 0; k < n; ++k) {
      px[k] = ox[k];
      py[k] = oy[k];
    }
  }
  double sx = 0.0, sy = 0.0;
  for (int k = 0; k < n; ++k) {
    sx += px[k];
    sy += py[k];
  }
  *ex = sx / (double)n;
  *ey = sy / (double)n;
  return 1;
}

/* Eq. (2): 1 when the nearest agent is within d_follow (inclusive). */
double orc_follow_reward(double d, double d_follow) { return d <= d_follow ? 1.0 : 0.0; }

/* Eq. (1). At e = eps_max the exponent tends to -inf, so the value is 0 and
 * the reward is continuous at both thresholds. */
double orc_tracking_reward(double e, double eps_min, double eps_max) {
  if (e < eps_min) return 1.0;
  if (!(e < eps_max)) return 0.0;
  double t = (e - eps_min) / (eps_max - eps_min);
  return exp(-2.0 * t / (1.0 - t));
}

/* ------------------------------------------------------------------------ */
/* One environment.                                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t env_id;
  int nA, nT, W, filled;
  double ax[OMAX], ay[OMAX], apsi[OMAX];
  double tx[OMAX], ty[OMAX], tpsi[OMAX], tv[OMAX];
  double sigma_r;
  /* window entry k = k-th most recent step */
  double hx[OMAX][OWMAX], hy[OMAX][OWMAX];
  double hr[OMAX][OMAX][OWMAX];
  double ex[OMAX][OMAX], ey[OMAX][OMAX], es[OMAX][OMAX];
  int ev[OMAX][OMAX];
  int comm_ok[OMAX];
  int rud[OMAX];  /* rudder position of each agent (action_mode 1) */
  /* rec[i][k][e]: agent i received agent k's broadcast (its position and
   * ranges) of window entry e; rec[i][i][e] = 1 */
  unsigned char rec[OMAX][OMAX][OWMAX];
  /* particle filter (est_kind 1): particles of tracker (i, j), belief flag */
  double ppx[OMAX][OMAX][ORC_PF_N], ppy[OMAX][OMAX][ORC_PF_N];
  int pinit[OMAX][OMAX];
} oenv;

/* Pairwise spawn (Sec. IV-A-2: every entity at least spawn_min and at most
 * spawn_max from every other; how the paper draws such a layout is not
 * stated). Reading: the entities take distinct sites of a hexagonal patch
 * about the centre of the area: the centre, the six sites of the first ring
 * at distance s, and the six sites of the second ring at distance s sqrt(3)
 * (each between two first-ring sites); 13 sites. Their order is a uniformly
 * random permutation, the patch is rotated by a uniform angle, and each
 * entity is moved off its site by a uniform offset in the square of
 * half-side h. Neighbouring sites are s apart and the farthest two 2 sqrt(3) s,
 * and an offset moves a pair's distance by at most 2 sqrt(2) h, so
 *   s = spawn_min + 2 sqrt(2) h   and   2 sqrt(3) s + 2 sqrt(2) h <= spawn_max
 * keep every pair within the bounds; h is 0.9 of the largest value that
 * satisfies both. Random words, in order, from Philox(1 + k, env, 127, reset),
 * k = 0, 1, ...: words 0..11 the Fisher-Yates choices (position i = 12 down
 * to 1 swaps with a uniform choice in 0..i), word 12 the rotation, words
 * 13 + 2n and 14 + 2n the offset of entity n (agents first, then targets).
 * Returns 0, or -1 with more than 13 entities. */
static int spawn_pairwise(const orc_params *p, uint64_t seed, uint64_t episode, uint32_t env_id,
                          int nA, int nT, double *xs, double *ys) {
  const int n = nA + nT;
  if (n > 13) return -1;
  const double two_pi = 6.283185307179586476925286766559, pi = two_pi / 2.0;
  const double r2 = sqrt(2.0), r3 = sqrt(3.0);
  const double h = 0.9 * (p->spawn_max - 2.0 * r3 * p->spawn_min) / (2.0 * r2 * (2.0 * r3 + 1.0));
  const double s = p->spawn_min + 2.0 * r2 * h;
  const uint32_t c3 = (uint32_t)((episode << 4) | PURPOSE_RESET);
  uint32_t w[40];
  for (int k = 0; k < 10; ++k) draw(seed, 1u + (uint32_t)k, env_id, ENT_ENV, c3, w + 4 * k);
  int perm[13];
  for (int i = 0; i < 13; ++i) perm[i] = i;
  for (int i = 12; i >= 1; --i) {
    int j = (int)orc_choice(w[12 - i], (uint32_t)(i + 1));
    int tmp = perm[i];
    perm[i] = perm[j];
    perm[j] = tmp;
  }
  const double phi = two_pi * orc_u01(w[12]);
  for (int m = 0; m < n; ++m) {
    int site = perm[m];
    double rad = 0.0, ang = 0.0;
    if (site >= 1 && site <= 6) {
      rad = s;
      ang = (site - 1) * pi / 3.0;
    } else if (site >= 7) {
      rad = s * r3;
      ang = pi / 6.0 + (site - 7) * pi / 3.0;
    }
    xs[m] = rad * cos(ang + phi) + h * (2.0 * orc_u01(w[13 + 2 * m]) - 1.0);
    ys[m] = rad * sin(ang + phi) + h * (2.0 * orc_u01(w[14 + 2 * m]) - 1.0);
  }
  return 0;
}

int orc_spawn_pairwise(const orc_params *p, uint64_t seed, uint64_t episode, uint32_t env_id,
                       int n_agents, int n_targets, double *x, double *y) {
  return spawn_pairwise(p, seed, episode, env_id, n_agents, n_targets, x, y);
}

/* Spawn (Sec. IV-A-2 spawns entities on the surface / at depth with
 * pairwise spacing, spawn_mode 1; the batched configurations instead place
 * agents in a disk about the centre of the area and targets uniformly in the
 * square, spawn_mode 0). Headings, target speeds and the range noise come
 * from the same draws in both modes. */
static void env_reset(const orc_params *p, uint64_t seed, uint64_t episode, oenv *E) {
  const double two_pi = 6.283185307179586476925286766559, pi = two_pi / 2.0;
  uint32_t c3 = (uint32_t)((episode << 4) | PURPOSE_RESET);
  uint32_t x[4];
  for (int i = 0; i < E->nA; ++i) {
    draw(seed, 0u, E->env_id, (uint32_t)i, c3, x);
    double rad = p->spawn_agent_radius * sqrt(orc_u01(x[0]));
    double ang = two_pi * orc_u01(x[1]);
    E->ax[i] = rad * cos(ang);
    E->ay[i] = rad * sin(ang);
    E->apsi[i] = -pi + two_pi * orc_u01(x[2]);
  }
  for (int j = 0; j < E->nT; ++j) {
    draw(seed, 0u, E->env_id, (uint32_t)(ENT_TARGET_BLOCK + j), c3, x);
    E->tx[j] = -0.5 * p->area + p->area * orc_u01(x[0]);
    E->ty[j] = -0.5 * p->area + p->area * orc_u01(x[1]);
    E->tpsi[j] = -pi + two_pi * orc_u01(x[2]);
    E->tv[j] = p->target_speed_lo + (p->target_speed_hi - p->target_speed_lo) * orc_u01(x[3]);
  }
  draw(seed, 0u, E->env_id, ENT_ENV, c3, x);
  E->sigma_r = p->range_sigma_lo + (p->range_sigma_hi - p->range_sigma_lo) * orc_u01(x[0]);
  if (p->spawn_mode == 1) {
    double xs[2 * OMAX], ys[2 * OMAX];
    spawn_pairwise(p, seed, episode, E->env_id, E->nA, E->nT, xs, ys);
    for (int i = 0; i < E->nA; ++i) {
      E->ax[i] = xs[i];
      E->ay[i] = ys[i];
    }
    for (int j = 0; j < E->nT; ++j) {
      E->tx[j] = xs[E->nA + j];
      E->ty[j] = ys[E->nA + j];
    }
  }
  E->filled = 0;
  for (int i = 0; i < OMAX; ++i) {
    E->rud[i] = (p->n_rudder - 1) / 2;
    E->comm_ok[i] = 1;
    for (int j = 0; j < OMAX; ++j) {
      E->ev[i][j] = 0;
      E->pinit[i][j] = 0;
      E->ex[i][j] = E->ey[i][j] = 0.0;
      E->es[i][j] = NAN;
    }
  }
}

/* Observation of agent i (Sec. IV-A-2 "Observation Space"; token layout of
 * the TransfMAPPO actor, Sec. IV-B-1): self, the other agents in index order,
 * the targets in index order. Each token is the relative 3D offset plus a
 * one-hot entity type. Other agents use what they broadcast (missing beyond
 * the comm range or when the broadcast was dropped); targets use agent i's
 * own tracker (missing when it has no estimate). Missing offsets are zero
 * with mask 0. */
static void env_obs(const orc_params *p, const oenv *E, double *obs, uint8_t *mask) {
  int k = 0;
  for (int i = 0; i < E->nA; ++i) {
    double *o = obs + 6 * k;
    o[0] = o[1] = o[2] = 0.0;
    o[3] = 1.0; o[4] = 0.0; o[5] = 0.0;
    mask[k++] = 1;
    for (int i2 = 0; i2 < E->nA; ++i2) {
      if (i2 == i) continue;
      o = obs + 6 * k;
      double dx = E->ax[i2] - E->ax[i], dy = E->ay[i2] - E->ay[i];
      int ok = E->comm_ok[i2] && hypot(dx, dy) <= p->comm_range;
      o[0] = ok ? dx : 0.0;
      o[1] = ok ? dy : 0.0;
      o[2] = 0.0;
      o[3] = 0.0; o[4] = 1.0; o[5] = 0.0;
      mask[k++] = (uint8_t)ok;
    }
    for (int j = 0; j < E->nT; ++j) {
      o = obs + 6 * k;
      int ok = E->ev[i][j];
      o[0] = ok ? E->ex[i][j] - E->ax[i] : 0.0;
      o[1] = ok ? E->ey[i][j] - E->ay[i] : 0.0;
      o[2] = 0.0;
      o[3] = 0.0; o[4] = 0.0; o[5] = 1.0;
      mask[k++] = (uint8_t)ok;
    }
  }
}

typedef struct {
  double *agent, *target, *ranges, *est, *sens, *obs, *err;
  uint8_t *est_valid, *est_fresh, *obs_mask;
  double reward;
  int crash, done;
  int32_t *actions;
} ostep_out;

/* One step t -> t+1 (Sec. IV-A-2 step structure, Sec. IV-A-3 kinematic
 * surrogate): agents turn then move, targets random-walk, ranges are measured
 * after the move, each (agent,target) tracker takes the new range into its
 * window and re-solves, then reward, observation and done are formed. */
static void env_step(const orc_params *p, uint64_t seed, uint64_t episode, uint32_t t, oenv *E,
                     const int32_t *actions_in, ostep_out *o) {
  uint32_t x[4];
  const uint32_t c3dyn = (uint32_t)((episode << 4) | PURPOSE_DYNAMICS);
  const uint32_t c3meas = (uint32_t)((episode << 4) | PURPOSE_MEASURE);
  const double vdt = p->agent_speed * p->dt;

  /* agents: heading change from the action plus noise, then straight move */
  for (int i = 0; i < E->nA; ++i) {
    draw(seed, t, E->env_id, (uint32_t)i, c3dyn, x);
    int a = actions_in ? actions_in[i] : (int)orc_choice(x[0], (uint32_t)p->n_actions);
    if (a < 0 || a >= p->n_actions) a = -1;
    double z0, z1;
    orc_normal2(x[1], x[2], &z0, &z1);
    double dpsi;
    if (p->action_mode == 1) {
      /* rudder: one position down / keep / one up, within the range; an
       * invalid action keeps the rudder */
      if (a >= 0) {
        int rr = E->rud[i] + a - 1;
        if (rr < 0) rr = 0;
        if (rr > p->n_rudder - 1) rr = p->n_rudder - 1;
        E->rud[i] = rr;
      }
      dpsi = p->action_dpsi[E->rud[i]];
    } else {
      dpsi = (a >= 0) ? p->action_dpsi[a] : 0.0;
    }
    E->apsi[i] = wrap_angle(E->apsi[i] + dpsi + p->agent_heading_sigma * z0);
    E->ax[i] = E->ax[i] + vdt * cos(E->apsi[i]);
    E->ay[i] = E->ay[i] + vdt * sin(E->apsi[i]);
    E->comm_ok[i] = !(orc_u01(x[3]) < p->comm_loss_p);
    if (o->actions) o->actions[i] = a;
  }
  /* targets: random walk of the heading, constant own speed */
  for (int q = 0; 2 * q < E->nT; ++q) {
    draw(seed, t, E->env_id, (uint32_t)(ENT_TARGET_BLOCK + q), c3dyn, x);
    double z[2];
    orc_normal2(x[0], x[1], &z[0], &z[1]);
    for (int m = 0; m < 2; ++m) {
      int j = 2 * q + m;
      if (j >= E->nT) break;
      E->tpsi[j] = wrap_angle(E->tpsi[j] + p->target_heading_sigma * z[m]);
      E->tx[j] = E->tx[j] + E->tv[j] * p->dt * cos(E->tpsi[j]);
      E->ty[j] = E->ty[j] + E->tv[j] * p->dt * sin(E->tpsi[j]);
    }
  }
  /* window shift: entry k -> k+1, the new step goes to entry 0 */
  for (int i = 0; i < E->nA; ++i) {
    for (int k = E->W - 1; k > 0; --k) {
      E->hx[i][k] = E->hx[i][k - 1];
      E->hy[i][k] = E->hy[i][k - 1];
      for (int j = 0; j < E->nT; ++j) E->hr[i][j][k] = E->hr[i][j][k - 1];
    }
    E->hx[i][0] = E->ax[i];
    E->hy[i][0] = E->ay[i];
  }
  if (E->filled < E->W) E->filled += 1;
  /* what each agent receives this step (the same rule as its observation of
   * the other agents): a broadcast that was not dropped, within comm_range */
  for (int i = 0; i < E->nA; ++i) {
    for (int k2 = 0; k2 < E->nA; ++k2) {
      for (int k = E->W - 1; k > 0; --k) E->rec[i][k2][k] = E->rec[i][k2][k - 1];
      const double dx = E->ax[k2] - E->ax[i], dy = E->ay[k2] - E->ay[i];
      E->rec[i][k2][0] = (unsigned char)(k2 == i || (E->comm_ok[k2] && hypot(dx, dy) <= p->comm_range));
    }
  }
  /* noisy ranges after the move; missing beyond the detection range */
  for (int i = 0; i < E->nA; ++i) {
    for (int q = 0; 4 * q < E->nT; ++q) {
      draw(seed, t, E->env_id, (uint32_t)(ENT_RANGE_ROW + 8 * i + q), c3meas, x);
      double z[4];
      orc_normal2(x[0], x[1], &z[0], &z[1]);
      orc_normal2(x[2], x[3], &z[2], &z[3]);
      for (int m = 0; m < 4; ++m) {
        int j = 4 * q + m;
        if (j >= E->nT) break;
        double dist = hypot(E->ax[i] - E->tx[j], E->ay[i] - E->ty[j]);
        double r = dist + E->sigma_r * z[m];
        E->hr[i][j][0] = (dist <= p->det_range) ? r : NAN;
      }
    }
  }
  /* est_kind 1: per-(agent,target) particle filter over this step's rows:
   * the agent's own range, then (pooled) the ranges received from the other
   * agents in index order; no belief and no row: no estimate (held) */
  if (p->est_kind == 1) {
    const uint32_t c3pf = (uint32_t)((episode << 4) | PURPOSE_PF);
    const uint32_t c3seed = (uint32_t)((episode << 4) | PURPOSE_PF_SEED);
    const double sl = sqrt(E->sigma_r * E->sigma_r + p->pf_lik_sigma * p->pf_lik_sigma);
    for (int i = 0; i < E->nA; ++i) {
      for (int j = 0; j < E->nT; ++j) {
        double wx[OMAX], wy[OMAX], wr[OMAX];
        int n = 0;
        for (int k2 = 0; k2 < E->nA; ++k2) {
          const int a = (k2 == 0) ? i : (k2 <= i ? k2 - 1 : k2);
          if (a != i && !p->pooled) break;
          if (isnan(E->hr[a][j][0]) || !E->rec[i][a][0]) continue;
          wx[n] = E->hx[a][0];
          wy[n] = E->hy[a][0];
          wr[n] = E->hr[a][j][0];
          ++n;
        }
        /* the step's words: one Philox block per particle pair (2h, 2h + 1),
         * words 0, 1 particle 2h's normals and 2, 3 particle 2h + 1's; a
         * second block per pair (purpose 8) gives the seeding angles from
         * words 0 and 2; the resampling offset is word 0 of the tracker's
         * own block (entity 2048 + code) */
        const uint32_t code = (uint32_t)(8 * i + j);
        uint32_t zw[2 * ORC_PF_N], uw[ORC_PF_N], blk[4];
        for (int h = 0; h < ORC_PF_N / 2; ++h) {
          draw(seed, t, E->env_id, code * (ORC_PF_N / 2) + (uint32_t)h, c3pf, blk);
          zw[4 * h] = blk[0];
          zw[4 * h + 1] = blk[1];
          zw[4 * h + 2] = blk[2];
          zw[4 * h + 3] = blk[3];
          draw(seed, t, E->env_id, code * (ORC_PF_N / 2) + (uint32_t)h, c3seed, blk);
          uw[2 * h] = blk[0];
          uw[2 * h + 1] = blk[2];
        }
        draw(seed, t, E->env_id, ENT_PF_OFFSET + code, c3pf, blk);
        double px, py;
        const int ok = orc_pf_update(ORC_PF_N, E->ppx[i][j], E->ppy[i][j], E->pinit[i][j], n, wx,
                                     wy, wr, sl, p->pf_q, zw, uw, blk[0], &px, &py, NULL);
        if (ok) {
          E->pinit[i][j] = 1;
          E->ex[i][j] = px;
          E->ey[i][j] = py;
          E->ev[i][j] = 1;
        }
        const int pidx = i * E->nT + j;
        if (o->ranges) o->ranges[pidx] = E->hr[i][j][0];
        if (o->est) {
          o->est[2 * pidx] = E->ev[i][j] ? E->ex[i][j] : 0.0;
          o->est[2 * pidx + 1] = E->ev[i][j] ? E->ey[i][j] : 0.0;
        }
        if (o->est_valid) o->est_valid[pidx] = (uint8_t)E->ev[i][j];
        if (o->est_fresh) o->est_fresh[pidx] = (uint8_t)ok;
        if (o->sens) o->sens[pidx] = NAN;
      }
    }
  }
  /* est_kind 0: per-(agent,target) least squares over the valid window
   * entries; hold on failure */
  for (int i = 0; i < E->nA && p->est_kind == 0; ++i) {
    for (int j = 0; j < E->nT; ++j) {
      double wx[OROWS], wy[OROWS], wr[OROWS];
      int n = 0;
      /* rows: agent i's own entries, then (pooled) those of every other agent
       * whose broadcast of that entry agent i received, agent by agent */
      for (int k2 = 0; k2 < E->nA; ++k2) {
        const int a = (k2 == 0) ? i : (k2 <= i ? k2 - 1 : k2);
        if (a != i && !p->pooled) break;
        for (int k = 0; k < E->filled; ++k) {
          if (isnan(E->hr[a][j][k]) || !E->rec[i][a][k]) continue;
          wx[n] = E->hx[a][k];
          wy[n] = E->hy[a][k];
          wr[n] = E->hr[a][j][k];
          ++n;
        }
      }
      double px, py, s = NAN;
      int ok = o->sens ? orc_ls_estimate_sens(n, wx, wy, wr, p->gn_iters, p->guard_tau, &px, &py, &s)
                       : orc_ls_estimate(n, wx, wy, wr, p->gn_iters, p->guard_tau, &px, &py);
      if (ok) {
        E->ex[i][j] = px;
        E->ey[i][j] = py;
        E->es[i][j] = s;
        E->ev[i][j] = 1;
      }
      int pidx = i * E->nT + j;
      if (o->ranges) o->ranges[pidx] = E->hr[i][j][0];
      if (o->est) {
        o->est[2 * pidx] = E->ev[i][j] ? E->ex[i][j] : 0.0;
        o->est[2 * pidx + 1] = E->ev[i][j] ? E->ey[i][j] : 0.0;
      }
      if (o->est_valid) o->est_valid[pidx] = (uint8_t)E->ev[i][j];
      if (o->est_fresh) o->est_fresh[pidx] = (uint8_t)ok;
      if (o->sens) o->sens[pidx] = E->es[i][j];
    }
  }
  /* reward: Eq. (1) per target on the team's best estimate, normalised by the
   * number of targets; crash penalty when two agents are closer than d_safe */
  double sum = 0.0;
  for (int j = 0; j < E->nT; ++j) {
    double e = INFINITY;
    for (int i = 0; i < E->nA; ++i) {
      if (!E->ev[i][j]) continue;
      double d = hypot(E->ex[i][j] - E->tx[j], E->ey[i][j] - E->ty[j]);
      if (d < e) e = d;
    }
    if (o->err) o->err[j] = e;
    if (p->reward_mode == 1) {
      /* Eq. (2): distance from the target to its nearest agent (true positions) */
      double dmin = INFINITY;
      for (int i = 0; i < E->nA; ++i) {
        double d = hypot(E->ax[i] - E->tx[j], E->ay[i] - E->ty[j]);
        if (d < dmin) dmin = d;
      }
      sum += orc_follow_reward(dmin, p->d_follow);
    } else {
      sum += orc_tracking_reward(e, p->eps_min, p->eps_max);
    }
  }
  double reward = sum / E->nT;
  int crash = 0;
  for (int i = 0; i < E->nA; ++i)
    for (int i2 = i + 1; i2 < E->nA; ++i2)
      if (hypot(E->ax[i] - E->ax[i2], E->ay[i] - E->ay[i2]) < p->d_safe) crash = 1;
  if (crash) reward = -1.0;
  o->reward = reward;
  o->crash = crash;
  o->done = (t + 1 == (uint32_t)p->episode_len);
  if (o->obs) env_obs(p, E, o->obs, o->obs_mask);
  for (int i = 0; i < E->nA; ++i) {
    if (o->agent) {
      o->agent[3 * i] = E->ax[i];
      o->agent[3 * i + 1] = E->ay[i];
      o->agent[3 * i + 2] = E->apsi[i];
    }
  }
  for (int j = 0; j < E->nT; ++j) {
    if (o->target) {
      o->target[4 * j] = E->tx[j];
      o->target[4 * j + 1] = E->ty[j];
      o->target[4 * j + 2] = E->tpsi[j];
      o->target[4 * j + 3] = E->tv[j];
    }
  }
}

int orc_rollout(const orc_params *p, uint64_t seed, uint64_t episode, int64_t n_sel,
                const int64_t *env_ids, const int32_t *n_agents, const int32_t *n_targets,
                int32_t T, const int32_t *actions, orc_traj *out, int n_threads) {
  if (!p || n_sel < 0 || T < 0 || p->window < 1 || p->window > OWMAX) return -1;
  if (p->n_actions < 1 || p->n_actions > 8) return -1;
  if (p->action_mode != 0 && p->action_mode != 1) return -1;
  if (p->action_mode == 1 && (p->n_rudder < 1 || p->n_rudder > 8 || p->n_actions != 3)) return -1;
  if (p->reward_mode != 0 && p->reward_mode != 1) return -1;
  if (p->spawn_mode != 0 && p->spawn_mode != 1) return -1;
  if (p->spawn_mode == 1 && !(p->spawn_min >= 0.0 && p->spawn_max >= 2.0 * sqrt(3.0) * p->spawn_min))
    return -1;
  if (p->spawn_mode == 1 && p->n_agents + p->n_targets > 13) return -1;
  if (p->pooled != 0 && p->pooled != 1) return -1;
  if (p->est_kind != 0 && p->est_kind != 1) return -1;
  if (p->est_kind == 1 && !(p->pf_q >= 0.0 && p->pf_lik_sigma >= 0.0)) return -1;
  for (int64_t k = 0; k < n_sel; ++k)
    if (n_agents[k] < 1 || n_agents[k] > OMAX || n_targets[k] < 1 || n_targets[k] > OMAX)
      return -1;
  /* CSR offsets over the selected envs */
  int64_t *ao = calloc((size_t)n_sel + 1, sizeof(int64_t));
  int64_t *to = calloc((size_t)n_sel + 1, sizeof(int64_t));
  int64_t *po = calloc((size_t)n_sel + 1, sizeof(int64_t));
  int64_t *ko = calloc((size_t)n_sel + 1, sizeof(int64_t));
  if (!ao || !to || !po || !ko) {
    free(ao); free(to); free(po); free(ko);
    return -1;
  }
  for (int64_t k = 0; k < n_sel; ++k) {
    ao[k + 1] = ao[k] + n_agents[k];
    to[k + 1] = to[k] + n_targets[k];
    po[k + 1] = po[k] + (int64_t)n_agents[k] * n_targets[k];
    ko[k + 1] = ko[k] + (int64_t)n_agents[k] * (n_agents[k] + n_targets[k]);
  }
  const int64_t A = ao[n_sel], Tt = to[n_sel], P = po[n_sel], K = ko[n_sel];

#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t k = 0; k < n_sel; ++k) {
    oenv *E = malloc(sizeof(oenv));
    memset(E, 0, sizeof(oenv));
    E->env_id = (uint32_t)env_ids[k];
    E->nA = n_agents[k];
    E->nT = n_targets[k];
    E->W = p->window;
    env_reset(p, seed, episode, E);
    if (out->init_agent)
      for (int i = 0; i < E->nA; ++i) {
        out->init_agent[3 * (ao[k] + i)] = E->ax[i];
        out->init_agent[3 * (ao[k] + i) + 1] = E->ay[i];
        out->init_agent[3 * (ao[k] + i) + 2] = E->apsi[i];
      }
    if (out->init_target)
      for (int j = 0; j < E->nT; ++j) {
        out->init_target[4 * (to[k] + j)] = E->tx[j];
        out->init_target[4 * (to[k] + j) + 1] = E->ty[j];
        out->init_target[4 * (to[k] + j) + 2] = E->tpsi[j];
        out->init_target[4 * (to[k] + j) + 3] = E->tv[j];
      }
    if (out->sigma_r) out->sigma_r[k] = E->sigma_r;
    if (out->init_obs) env_obs(p, E, out->init_obs + 6 * ko[k], out->init_mask + ko[k]);

    double m_rew = 0.0, m_err = 0.0, m_err2 = 0.0, m_cnt = 0.0, m_crash = 0.0;
    double errs[OMAX];
    for (int32_t t = 0; t < T; ++t) {
      ostep_out o;
      memset(&o, 0, sizeof(o));
#define SLICE(ptr, tot, off, w) ((ptr) ? (ptr) + ((int64_t)t * (tot) + (off)) * (w) : NULL)
      o.agent = SLICE(out->agent, A, ao[k], 3);
      o.target = SLICE(out->target, Tt, to[k], 4);
      o.ranges = SLICE(out->ranges, P, po[k], 1);
      o.est = SLICE(out->est, P, po[k], 2);
      o.est_valid = SLICE(out->est_valid, P, po[k], 1);
      o.est_fresh = SLICE(out->est_fresh, P, po[k], 1);
      o.sens = SLICE(out->sens, P, po[k], 1);
      o.obs = SLICE(out->obs, K, ko[k], 6);
      o.obs_mask = SLICE(out->obs_mask, K, ko[k], 1);
      o.actions = SLICE(out->actions, A, ao[k], 1);
#undef SLICE
      o.err = errs;
      const int32_t *act = actions ? actions + (int64_t)t * A + ao[k] : NULL;
      env_step(p, seed, episode, (uint32_t)t, E, act, &o);
      if (out->reward) out->reward[(int64_t)t * n_sel + k] = o.reward;
      if (out->crash) out->crash[(int64_t)t * n_sel + k] = (uint8_t)o.crash;
      if (out->done) out->done[(int64_t)t * n_sel + k] = (uint8_t)o.done;
      if (out->err)
        for (int j = 0; j < E->nT; ++j) out->err[(int64_t)t * Tt + to[k] + j] = errs[j];
      m_rew += o.reward;
      m_crash += o.crash;
      for (int j = 0; j < E->nT; ++j)
        if (isfinite(errs[j])) {
          m_err += errs[j];
          m_err2 += errs[j] * errs[j];
          m_cnt += 1.0;
        }
    }
    if (out->env_metrics) {
      double lost = 0.0;
      for (int j = 0; j < E->nT; ++j) {
        double dmin = INFINITY;
        for (int i = 0; i < E->nA; ++i) {
          double d = hypot(E->ax[i] - E->tx[j], E->ay[i] - E->ty[j]);
          if (d < dmin) dmin = d;
        }
        if (dmin > p->lost_range) lost += 1.0;
      }
      double *m = out->env_metrics + 6 * k;
      m[0] = m_rew; m[1] = m_err; m[2] = m_err2; m[3] = m_cnt; m[4] = m_crash; m[5] = lost;
    }
    free(E);
  }
  free(ao); free(to); free(po); free(ko);
  return 0;
}
