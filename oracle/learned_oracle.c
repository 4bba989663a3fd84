/*
 * FP64 oracle of the learned range-only estimator and of the attention
 * policy. TEST INFRASTRUCTURE ONLY (see lrauv_oracle.h).
 *
 * The learned estimator is not in the paper: it stands in for the per-target
 * range-only estimator of Sec. III-A. Its readings (features, output
 * parameterisation, loss) are listed in the design doc; this file writes them out
 * plainly in FP64.
 *
 *   features of a window of W entries (a_k, r_k), all present:
 *     abar = mean a_k, rbar = mean r_k; theta = direction of a_0 - a_{W-1}
 *     (0 when that chord is shorter than 1e-6 m); u_k = R(-theta)(a_k - abar)
 *     x[3k] = u_k.x / 10, x[3k+1] = u_k.y / 10, x[3k+2] = (r_k - rbar) / 10,
 *     x[3W] = rbar / 1000, remaining inputs up to 64 are 0.
 *   network: z1 = W1 x + b1, h1 = gelu(z1), z2 = W2 h1 + b2, h2 = gelu(z2),
 *     y = W3 h2 + b3 with gelu the tanh form of Hendrycks and Gimpel,
 *     W1 [128][64], W2 [128][128], W3 [2][128] stored row-major (out, in),
 *     parameter vector = W1, b1, W2, b2, W3, b3.
 *   estimate: p = abar + rbar * R(theta) y.
 *   loss: mean over samples of |y - y_target|^2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NIN 64
#define NH 128
#define NOUT 2
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NH * NIN)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NOUT * NH)
#define NPARAM (OFF_B3 + NOUT)

int64_t orc_mlp_num_params(void) { return NPARAM; }

static double gelu(double x) {
  const double c = 0.79788456080286535588; /* sqrt(2/pi) */
  return 0.5 * x * (1.0 + tanh(c * (x + 0.044715 * x * x * x)));
}

static double gelu_grad(double x) {
  const double c = 0.79788456080286535588;
  double u = c * (x + 0.044715 * x * x * x);
  double th = tanh(u);
  double du = c * (1.0 + 3.0 * 0.044715 * x * x);
  return 0.5 * (1.0 + th) + 0.5 * x * (1.0 - th * th) * du;
}

/* feat [N][64], frame [N][5] = (abar_x, abar_y, cos theta, sin theta, rbar) */
void orc_window_features(int64_t N, int W, const double *win, double *feat, double *frame) {
  for (int64_t n = 0; n < N; ++n) {
    const double *w = win + n * W * 3;
    double mx = 0.0, my = 0.0, mr = 0.0;
    for (int k = 0; k < W; ++k) {
      mx += w[3 * k];
      my += w[3 * k + 1];
      mr += w[3 * k + 2];
    }
    mx /= W;
    my /= W;
    mr /= W;
    double cx = w[0] - w[3 * (W - 1)], cy = w[1] - w[3 * (W - 1) + 1];
    double len = hypot(cx, cy);
    double c = 1.0, s = 0.0;
    if (len > 1e-6) {
      c = cx / len;
      s = cy / len;
    }
    double *f = feat + n * NIN;
    for (int i = 0; i < NIN; ++i) f[i] = 0.0;
    for (int k = 0; k < W; ++k) {
      double dx = w[3 * k] - mx, dy = w[3 * k + 1] - my;
      f[3 * k] = (c * dx + s * dy) / 10.0;
      f[3 * k + 1] = (-s * dx + c * dy) / 10.0;
      f[3 * k + 2] = (w[3 * k + 2] - mr) / 10.0;
    }
    f[3 * W] = mr / 1000.0;
    double *fr = frame + n * 5;
    fr[0] = mx;
    fr[1] = my;
    fr[2] = c;
    fr[3] = s;
    fr[4] = mr;
  }
}

/* Normalised target of an estimate p in a window's frame: R(-theta)(p - abar)/rbar. */
void orc_mlp_target(int64_t N, const double *frame, const double *p, double *y) {
  for (int64_t n = 0; n < N; ++n) {
    const double *fr = frame + n * 5;
    double dx = p[2 * n] - fr[0], dy = p[2 * n + 1] - fr[1];
    y[2 * n] = (fr[2] * dx + fr[3] * dy) / fr[4];
    y[2 * n + 1] = (-fr[3] * dx + fr[2] * dy) / fr[4];
  }
}

/* Estimate from a network output: abar + rbar R(theta) y. */
void orc_mlp_decode(int64_t N, const double *frame, const double *y, double *p) {
  for (int64_t n = 0; n < N; ++n) {
    const double *fr = frame + n * 5;
    double ux = fr[4] * y[2 * n], uy = fr[4] * y[2 * n + 1];
    p[2 * n] = fr[0] + fr[2] * ux - fr[3] * uy;
    p[2 * n + 1] = fr[1] + fr[3] * ux + fr[2] * uy;
  }
}

static void forward_one(const double *x, const double *th, double *z1, double *h1, double *z2,
                        double *h2, double *y) {
  for (int o = 0; o < NH; ++o) {
    double acc = th[OFF_B1 + o];
    for (int i = 0; i < NIN; ++i) acc += th[OFF_W1 + o * NIN + i] * x[i];
    z1[o] = acc;
    h1[o] = gelu(acc);
  }
  for (int o = 0; o < NH; ++o) {
    double acc = th[OFF_B2 + o];
    for (int i = 0; i < NH; ++i) acc += th[OFF_W2 + o * NH + i] * h1[i];
    z2[o] = acc;
    h2[o] = gelu(acc);
  }
  for (int o = 0; o < NOUT; ++o) {
    double acc = th[OFF_B3 + o];
    for (int i = 0; i < NH; ++i) acc += th[OFF_W3 + o * NH + i] * h2[i];
    y[o] = acc;
  }
}

void orc_mlp_forward(int64_t N, const double *x, const double *params, double *y) {
  double z1[NH], h1[NH], z2[NH], h2[NH];
  for (int64_t n = 0; n < N; ++n) forward_one(x + n * NIN, params, z1, h1, z2, h2, y + n * NOUT);
}

/* Mean-squared loss and its gradient (grad [NPARAM], overwritten). */
double orc_mlp_backward(int64_t N, const double *x, const double *target, const double *params,
                        double *grad, double *y_out) {
  for (int i = 0; i < NPARAM; ++i) grad[i] = 0.0;
  double loss = 0.0;
  double z1[NH], h1[NH], z2[NH], h2[NH], y[NOUT], dz2[NH], dz1[NH];
  for (int64_t n = 0; n < N; ++n) {
    const double *xn = x + n * NIN;
    forward_one(xn, params, z1, h1, z2, h2, y);
    if (y_out) {
      y_out[2 * n] = y[0];
      y_out[2 * n + 1] = y[1];
    }
    double dy[NOUT];
    for (int o = 0; o < NOUT; ++o) {
      double e = y[o] - target[n * NOUT + o];
      loss += e * e;
      dy[o] = 2.0 * e / (double)N;
    }
    for (int o = 0; o < NOUT; ++o) {
      grad[OFF_B3 + o] += dy[o];
      for (int i = 0; i < NH; ++i) grad[OFF_W3 + o * NH + i] += dy[o] * h2[i];
    }
    for (int i = 0; i < NH; ++i) {
      double dh = 0.0;
      for (int o = 0; o < NOUT; ++o) dh += dy[o] * params[OFF_W3 + o * NH + i];
      dz2[i] = dh * gelu_grad(z2[i]);
    }
    for (int o = 0; o < NH; ++o) {
      grad[OFF_B2 + o] += dz2[o];
      for (int i = 0; i < NH; ++i) grad[OFF_W2 + o * NH + i] += dz2[o] * h1[i];
    }
    for (int i = 0; i < NH; ++i) {
      double dh = 0.0;
      for (int o = 0; o < NH; ++o) dh += dz2[o] * params[OFF_W2 + o * NH + i];
      dz1[i] = dh * gelu_grad(z1[i]);
    }
    for (int o = 0; o < NH; ++o) {
      grad[OFF_B1 + o] += dz1[o];
      for (int i = 0; i < NIN; ++i) grad[OFF_W1 + o * NIN + i] += dz1[o] * xn[i];
    }
  }
  return loss / (double)N;
}

/* Adam (Kingma and Ba, 2015) with bias correction; step counts from 1. */
void orc_adam_step(int64_t P, double *params, const double *grad, double *m, double *v,
                   int64_t step, double lr, double beta1, double beta2, double eps) {
  double c1 = 1.0 - pow(beta1, (double)step), c2 = 1.0 - pow(beta2, (double)step);
  for (int64_t i = 0; i < P; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    params[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* RMS over a window of (|p - a_k| - r_k): the fallback test statistic. */
void orc_mlp_residual_rms(int64_t N, int W, const double *win, const double *p, double *rms) {
  for (int64_t n = 0; n < N; ++n) {
    const double *w = win + n * W * 3;
    double acc = 0.0;
    for (int k = 0; k < W; ++k) {
      double res = hypot(p[2 * n] - w[3 * k], p[2 * n + 1] - w[3 * k + 1]) - w[3 * k + 2];
      acc += res * res;
    }
    rms[n] = sqrt(acc / W);
  }
}

/* Distance along the network's bearing. The decoded point p fixes a
 * direction e from the window centroid c; the estimate is moved along it to
 * the distance d minimising J(d) = sum_k (|c + d e - a_k| - r_k)^2, by `iters`
 * Gauss-Newton steps on d from d0 = |p - c| (a step is kept only if J falls).
 * Missing ranges (NaN) are skipped. With p = c the point is returned as is. */
void orc_range_refine(int64_t N, int W, const double *win, const double *centre,
                      const double *p_in, int iters, double *p_out) {
  for (int64_t n = 0; n < N; ++n) {
    const double *w = win + n * W * 3;
    const double cx = centre[2 * n], cy = centre[2 * n + 1];
    double ex = p_in[2 * n] - cx, ey = p_in[2 * n + 1] - cy;
    double d = hypot(ex, ey);
    if (!(d > 0.0)) {
      p_out[2 * n] = p_in[2 * n];
      p_out[2 * n + 1] = p_in[2 * n + 1];
      continue;
    }
    ex /= d;
    ey /= d;
    for (int it = 0; it < iters; ++it) {
      double g = 0.0, h = 0.0, j0 = 0.0;
      for (int k = 0; k < W; ++k) {
        const double r = w[3 * k + 2];
        if (r != r) continue;
        const double dx = cx + d * ex - w[3 * k], dy = cy + d * ey - w[3 * k + 1];
        const double dist = hypot(dx, dy);
        const double rho = dist - r;
        j0 += rho * rho;
        if (dist > 0.0) {
          const double jd = (dx * ex + dy * ey) / dist; /* d rho / d d */
          g += jd * rho;
          h += jd * jd;
        }
      }
      if (!(h > 0.0)) break;
      const double dn = d - g / h;
      double j1 = 0.0;
      for (int k = 0; k < W; ++k) {
        const double r = w[3 * k + 2];
        if (r != r) continue;
        const double rho = hypot(cx + dn * ex - w[3 * k], cy + dn * ey - w[3 * k + 1]) - r;
        j1 += rho * rho;
      }
      if (!(j1 < j0)) break;
      d = dn;
    }
    p_out[2 * n] = cx + d * ex;
    p_out[2 * n + 1] = cy + d * ey;
  }
}

/* ------------------------------------------------------------------------ */
/* Attention policy (the TransfMAPPO actor of Sec. IV-B-1, without its        */
/* recurrent token; random initialisation, forward only). Tokens of one      */
/* agent: [self, other agents, targets], each (dx, dy, dz, one-hot type).    */
/* Pre-LN transformer: h = E x + e; for each layer: h += Wo MHA(LN1(h)) + bo,*/
/* h += W2 gelu(W1 LN2(h) + b1) + b2; logits = Wh LN_f(h_self) + bh.         */
/* Keys whose observation mask is 0 are excluded from attention.            */
/* Parameter order: E [64][6], e [64]; per layer: ln1 g,b [64], Wqkv [192][64]*/
/* (Q, K, V rows; head h uses features 16h..16h+15), bqkv [192], Wo [64][64],*/
/* bo, ln2 g,b, W1 [256][64], b1 [256], W2 [64][256], b2 [64]; lnf g,b [64]; */
/* Wh [8][64], bh [8] (the first n_actions rows are used).                   */
/* ------------------------------------------------------------------------ */
#define PD 64
#define PH 4
#define PDH 16
#define PF 256
#define PL 2
#define PA 8
#define P_LAYER (2 * PD + 3 * PD * PD + 3 * PD + PD * PD + PD + 2 * PD + PF * PD + PF + PD * PF + PD)
#define P_TOTAL (PD * 6 + PD + PL * P_LAYER + 2 * PD + PA * PD + PA)

int64_t orc_policy_num_params(void) { return P_TOTAL; }

static void layer_norm(const double *x, const double *g, const double *b, double *y) {
  double m = 0.0, v = 0.0;
  for (int i = 0; i < PD; ++i) m += x[i];
  m /= PD;
  for (int i = 0; i < PD; ++i) v += (x[i] - m) * (x[i] - m);
  v /= PD;
  double inv = 1.0 / sqrt(v + 1e-5);
  for (int i = 0; i < PD; ++i) y[i] = (x[i] - m) * inv * g[i] + b[i];
}

enum { P_MAXT = 32 };

/* The trunk and head on rows already in the residual stream: h[0..n_tok-1]
 * (modified in place), key mask mk; logits = Wh LN_f(h_0) + bh, and
 * feat = LN_f(h_0) when feat is not NULL. th points at the first layer's
 * parameters. */
static void policy_trunk(int n_tok, double h[][PD], const uint8_t *mk, const double *th,
                         double *logits, double *feat) {
  double a[P_MAXT][PD], q[P_MAXT][3 * PD], o[P_MAXT][PD], f[PF];
  const double *p = th;
  for (int l = 0; l < PL; ++l) {
    const double *g1 = p; p += PD;
    const double *b1n = p; p += PD;
    const double *Wqkv = p; p += 3 * PD * PD;
    const double *bqkv = p; p += 3 * PD;
    const double *Wo = p; p += PD * PD;
    const double *bo = p; p += PD;
    const double *g2 = p; p += PD;
    const double *b2n = p; p += PD;
    const double *W1 = p; p += PF * PD;
    const double *b1 = p; p += PF;
    const double *W2 = p; p += PD * PF;
    const double *b2 = p; p += PD;
    for (int t = 0; t < n_tok; ++t) layer_norm(h[t], g1, b1n, a[t]);
    for (int t = 0; t < n_tok; ++t)
      for (int r = 0; r < 3 * PD; ++r) {
        double acc = bqkv[r];
        for (int i = 0; i < PD; ++i) acc += Wqkv[r * PD + i] * a[t][i];
        q[t][r] = acc;
      }
    for (int hd = 0; hd < PH; ++hd)
      for (int t = 0; t < n_tok; ++t) {
        double s[P_MAXT], mx = -INFINITY;
        for (int u = 0; u < n_tok; ++u) {
          if (!mk[u]) { s[u] = -INFINITY; continue; }
          double acc = 0.0;
          for (int c = 0; c < PDH; ++c) acc += q[t][hd * PDH + c] * q[u][PD + hd * PDH + c];
          s[u] = acc / 4.0; /* sqrt(16) */
          if (s[u] > mx) mx = s[u];
        }
        double z = 0.0;
        for (int u = 0; u < n_tok; ++u) {
          s[u] = mk[u] ? exp(s[u] - mx) : 0.0;
          z += s[u];
        }
        for (int c = 0; c < PDH; ++c) {
          double acc = 0.0;
          for (int u = 0; u < n_tok; ++u) acc += s[u] * q[u][2 * PD + hd * PDH + c];
          o[t][hd * PDH + c] = acc / z;
        }
      }
    for (int t = 0; t < n_tok; ++t)
      for (int d = 0; d < PD; ++d) {
        double acc = bo[d];
        for (int i = 0; i < PD; ++i) acc += Wo[d * PD + i] * o[t][i];
        h[t][d] += acc;
      }
    for (int t = 0; t < n_tok; ++t) {
      layer_norm(h[t], g2, b2n, a[t]);
      for (int r = 0; r < PF; ++r) {
        double acc = b1[r];
        for (int i = 0; i < PD; ++i) acc += W1[r * PD + i] * a[t][i];
        f[r] = gelu(acc);
      }
      for (int d = 0; d < PD; ++d) {
        double acc = b2[d];
        for (int r = 0; r < PF; ++r) acc += W2[d * PF + r] * f[r];
        h[t][d] += acc;
      }
    }
  }
  const double *gf = p; p += PD;
  const double *bf = p; p += PD;
  const double *Wh = p; p += PA * PD;
  const double *bh = p; p += PA;
  double s0[PD];
  layer_norm(h[0], gf, bf, s0);
  for (int k = 0; k < PA; ++k) {
    double acc = bh[k];
    for (int i = 0; i < PD; ++i) acc += Wh[k * PD + i] * s0[i];
    logits[k] = acc;
  }
  if (feat)
    for (int i = 0; i < PD; ++i) feat[i] = s0[i];
}

/* Embedding of one token: E x + e. */
static void policy_embed(const double *th, const double *x, double *h) {
  const double *E = th, *e = th + PD * 6;
  for (int d = 0; d < PD; ++d) {
    double acc = e[d];
    for (int c = 0; c < 6; ++c) acc += E[d * 6 + c] * x[c];
    h[d] = acc;
  }
}

/* tokens [A][n_tok][6], mask [A][n_tok] -> logits [A][PA]; the head reads
 * the first token. */
void orc_policy_forward(int64_t A, int n_tok, const double *tokens, const uint8_t *mask,
                        const double *th, double *logits) {
  double h[P_MAXT][PD];
  for (int64_t ag = 0; ag < A; ++ag) {
    for (int t = 0; t < n_tok; ++t) policy_embed(th, tokens + (ag * n_tok + t) * 6, h[t]);
    policy_trunk(n_tok, h, mask + ag * n_tok, th + PD * 6 + PD, logits + ag * PA, NULL);
  }
}

/* The recurrent form (TransfMAPPO, Fig. 3): a carried 64-wide state enters
 * the residual stream as an extra first row, ahead of the n_obs embedded
 * tokens, and is never masked; the head reads that row, and its final
 * LayerNorm is the next state. tokens [A][n_obs][6], mask [A][n_obs],
 * hidden_in [A][64] (NULL: zeros, the start of an episode) -> logits [A][PA],
 * hidden_out [A][64] (may alias hidden_in). */
void orc_policy_forward_rec(int64_t A, int n_obs, const double *tokens, const uint8_t *mask,
                            const double *hidden_in, const double *th, double *logits,
                            double *hidden_out) {
  double h[P_MAXT][PD];
  uint8_t mk[P_MAXT];
  for (int64_t ag = 0; ag < A; ++ag) {
    for (int d = 0; d < PD; ++d) h[0][d] = hidden_in ? hidden_in[ag * PD + d] : 0.0;
    mk[0] = 1;
    for (int t = 0; t < n_obs; ++t) {
      policy_embed(th, tokens + (ag * n_obs + t) * 6, h[1 + t]);
      mk[1 + t] = mask[ag * n_obs + t];
    }
    policy_trunk(1 + n_obs, h, mk, th + PD * 6 + PD, logits + ag * PA, hidden_out + ag * PD);
  }
}

/* Inverse-CDF draw from softmax(logits[0..n-1]) with uniform u in (0,1):
 * the smallest k whose cumulative probability exceeds u. */
int orc_policy_sample(const double *logits, int n, double u) {
  double mx = -INFINITY, z = 0.0;
  for (int k = 0; k < n; ++k)
    if (logits[k] > mx) mx = logits[k];
  for (int k = 0; k < n; ++k) z += exp(logits[k] - mx);
  double c = 0.0;
  for (int k = 0; k < n; ++k) {
    c += exp(logits[k] - mx) / z;
    if (u < c) return k;
  }
  return n - 1;
}
