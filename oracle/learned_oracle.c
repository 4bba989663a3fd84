/*
 * FP64 oracle of the learned range-only estimator and of the attention
 * policy. TEST INFRASTRUCTURE ONLY (see lrauv_oracle.h).
 *
 * The learned estimator is not in the paper: it stands in for the per-target
 * range-only estimator of Sec. III-A. Its definitions (features, output
 * parameterisation, loss) are written out below, plainly, in FP64.
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
/* Attention policy (the TransfMAPPO actor of Sec. IV-B-1; the plain form   */
/* here, the recurrent form and the gradient further down). Tokens of one    */
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

/* ------------------------------------------------------------------------ */
/* Gradient of the attention network (the learner's backward pass, MAPPO's  */
/* gradient step of Sec. III-B through the TransfMAPPO networks of Fig. 3).  */
/* For a loss whose gradient at each agent's logits is dlogits, the exact   */
/* gradient in every parameter, summed over agents: the forward pass is     */
/* taken again with every intermediate kept, then each operation is         */
/* differentiated in reverse order (layer norm, attention with its softmax  */
/* and key mask, tanh GELU, the residual adds, the embedding). In the       */
/* recurrent form the carried state is an input: its gradient is returned   */
/* (dhidden, may be NULL) but not followed into earlier steps.              */
/* ------------------------------------------------------------------------ */
typedef struct {
  double hin[PL][P_MAXT][PD], a1[PL][P_MAXT][PD], q[PL][P_MAXT][3 * PD];
  double pr[PL][PH][P_MAXT][P_MAXT], o[PL][P_MAXT][PD], hmid[PL][P_MAXT][PD];
  double a2[PL][P_MAXT][PD], z[PL][P_MAXT][PF], hout[P_MAXT][PD];
} policy_tape;

static void ln_backward(const double *x, const double *g, const double *dy, double *dx,
                        double *dg, double *db) {
  double m = 0.0, v = 0.0;
  for (int i = 0; i < PD; ++i) m += x[i];
  m /= PD;
  for (int i = 0; i < PD; ++i) v += (x[i] - m) * (x[i] - m);
  v /= PD;
  const double r = 1.0 / sqrt(v + 1e-5);
  double xh[PD], dxh[PD], s1 = 0.0, s2 = 0.0;
  for (int i = 0; i < PD; ++i) {
    xh[i] = (x[i] - m) * r;
    dxh[i] = dy[i] * g[i];
    dg[i] += dy[i] * xh[i];
    db[i] += dy[i];
    s1 += dxh[i];
    s2 += dxh[i] * xh[i];
  }
  for (int i = 0; i < PD; ++i) dx[i] = r * (dxh[i] - s1 / PD - xh[i] * s2 / PD);
}

/* One agent: rows h[0..n_tok-1] already in the residual stream (embedded, or
 * the carried state first); the trunk's forward pass recorded on the tape. */
static void policy_trunk_taped(int n_tok, double h[][PD], const uint8_t *mk, const double *th,
                               policy_tape *tp) {
  double f[PF];
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
    for (int t = 0; t < n_tok; ++t) {
      memcpy(tp->hin[l][t], h[t], sizeof(double) * PD);
      layer_norm(h[t], g1, b1n, tp->a1[l][t]);
      for (int r = 0; r < 3 * PD; ++r) {
        double acc = bqkv[r];
        for (int i = 0; i < PD; ++i) acc += Wqkv[r * PD + i] * tp->a1[l][t][i];
        tp->q[l][t][r] = acc;
      }
    }
    for (int hd = 0; hd < PH; ++hd)
      for (int t = 0; t < n_tok; ++t) {
        double *s = tp->pr[l][hd][t], mx = -INFINITY, zs = 0.0;
        for (int u = 0; u < n_tok; ++u) {
          s[u] = -INFINITY;
          if (!mk[u]) continue;
          double acc = 0.0;
          for (int c = 0; c < PDH; ++c)
            acc += tp->q[l][t][hd * PDH + c] * tp->q[l][u][PD + hd * PDH + c];
          s[u] = acc / 4.0;
          if (s[u] > mx) mx = s[u];
        }
        for (int u = 0; u < n_tok; ++u) {
          s[u] = mk[u] ? exp(s[u] - mx) : 0.0;
          zs += s[u];
        }
        for (int u = 0; u < n_tok; ++u) s[u] /= zs;
        for (int c = 0; c < PDH; ++c) {
          double acc = 0.0;
          for (int u = 0; u < n_tok; ++u) acc += s[u] * tp->q[l][u][2 * PD + hd * PDH + c];
          tp->o[l][t][hd * PDH + c] = acc;
        }
      }
    for (int t = 0; t < n_tok; ++t) {
      for (int d = 0; d < PD; ++d) {
        double acc = bo[d];
        for (int i = 0; i < PD; ++i) acc += Wo[d * PD + i] * tp->o[l][t][i];
        h[t][d] += acc;
      }
      memcpy(tp->hmid[l][t], h[t], sizeof(double) * PD);
      layer_norm(h[t], g2, b2n, tp->a2[l][t]);
      for (int r = 0; r < PF; ++r) {
        double acc = b1[r];
        for (int i = 0; i < PD; ++i) acc += W1[r * PD + i] * tp->a2[l][t][i];
        tp->z[l][t][r] = acc;
        f[r] = gelu(acc);
      }
      for (int d = 0; d < PD; ++d) {
        double acc = b2[d];
        for (int r = 0; r < PF; ++r) acc += W2[d * PF + r] * f[r];
        h[t][d] += acc;
      }
    }
  }
  for (int t = 0; t < n_tok; ++t) memcpy(tp->hout[t], h[t], sizeof(double) * PD);
}

/* Reverse pass of one agent: dlogits [PA] and dfeat [PD] (may be NULL) the
 * loss gradients at the logits and at the head's input LN_f(h_0) -> the
 * parameter gradient added to gl (layers, final LN and head), dh [n_tok][PD]
 * the gradient at the rows entering the trunk. */
static void policy_trunk_backward(int n_tok, const uint8_t *mk, const double *th,
                                  const policy_tape *tp, const double *dlogits, const double *dfeat,
                                  double *gl, double dh[][PD]) {
  const double *p = th;
  const double *lay[PL];
  double *glay[PL];
  for (int l = 0; l < PL; ++l) {
    lay[l] = p + l * P_LAYER;
    glay[l] = gl + l * P_LAYER;
  }
  /* final LN and head (row 0) */
  const double *gf = p + PL * P_LAYER, *Wh = gf + 2 * PD;
  double *dgf = gl + PL * P_LAYER, *dbf = dgf + PD, *dWh = dgf + 2 * PD, *dbh = dWh + PA * PD;
  double s0[PD], ds0[PD];
  layer_norm(tp->hout[0], gf, gf + PD, s0);
  for (int i = 0; i < PD; ++i) ds0[i] = dfeat ? dfeat[i] : 0.0;
  for (int k = 0; k < PA; ++k) {
    dbh[k] += dlogits[k];
    for (int i = 0; i < PD; ++i) {
      dWh[k * PD + i] += dlogits[k] * s0[i];
      ds0[i] += dlogits[k] * Wh[k * PD + i];
    }
  }
  for (int t = 0; t < n_tok; ++t)
    for (int d = 0; d < PD; ++d) dh[t][d] = 0.0;
  ln_backward(tp->hout[0], gf, ds0, dh[0], dgf, dbf);
  double dz[PF], df[PF], da[PD], dx[PD];
  double dq[P_MAXT][3 * PD], dov[P_MAXT][PD];
  for (int l = PL - 1; l >= 0; --l) {
    const double *q = lay[l];
    const double *g1 = q; q += PD;
    q += PD; /* ln1 offset */
    const double *Wqkv = q; q += 3 * PD * PD;
    q += 3 * PD;
    const double *Wo = q; q += PD * PD;
    q += PD;
    const double *g2 = q; q += PD;
    q += PD;
    const double *W1 = q; q += PF * PD;
    q += PF;
    const double *W2 = q;
    double *w = glay[l];
    double *dg1 = w; w += PD;
    double *db1n = w; w += PD;
    double *dWqkv = w; w += 3 * PD * PD;
    double *dbqkv = w; w += 3 * PD;
    double *dWo = w; w += PD * PD;
    double *dbo = w; w += PD;
    double *dg2 = w; w += PD;
    double *db2n = w; w += PD;
    double *dW1 = w; w += PF * PD;
    double *db1 = w; w += PF;
    double *dW2 = w; w += PD * PF;
    double *db2 = w;
    /* feed-forward block: h = hmid + W2 gelu(z) + b2 */
    for (int t = 0; t < n_tok; ++t) {
      for (int r = 0; r < PF; ++r) df[r] = 0.0;
      for (int d = 0; d < PD; ++d) {
        db2[d] += dh[t][d];
        for (int r = 0; r < PF; ++r) {
          dW2[d * PF + r] += dh[t][d] * gelu(tp->z[l][t][r]);
          df[r] += W2[d * PF + r] * dh[t][d];
        }
      }
      for (int r = 0; r < PF; ++r) {
        dz[r] = df[r] * gelu_grad(tp->z[l][t][r]);
        db1[r] += dz[r];
      }
      for (int i = 0; i < PD; ++i) da[i] = 0.0;
      for (int r = 0; r < PF; ++r)
        for (int i = 0; i < PD; ++i) {
          dW1[r * PD + i] += dz[r] * tp->a2[l][t][i];
          da[i] += W1[r * PD + i] * dz[r];
        }
      ln_backward(tp->hmid[l][t], g2, da, dx, dg2, db2n);
      for (int d = 0; d < PD; ++d) dh[t][d] += dx[d];
    }
    /* attention block: hmid = hin + Wo o + bo */
    for (int t = 0; t < n_tok; ++t) {
      for (int i = 0; i < PD; ++i) dov[t][i] = 0.0;
      for (int d = 0; d < PD; ++d) {
        dbo[d] += dh[t][d];
        for (int i = 0; i < PD; ++i) {
          dWo[d * PD + i] += dh[t][d] * tp->o[l][t][i];
          dov[t][i] += Wo[d * PD + i] * dh[t][d];
        }
      }
      for (int r = 0; r < 3 * PD; ++r) dq[t][r] = 0.0;
    }
    for (int hd = 0; hd < PH; ++hd)
      for (int t = 0; t < n_tok; ++t) {
        const double *P = tp->pr[l][hd][t];
        double dP[P_MAXT], dot = 0.0;
        for (int u = 0; u < n_tok; ++u) {
          dP[u] = 0.0;
          for (int c = 0; c < PDH; ++c) {
            dP[u] += dov[t][hd * PDH + c] * tp->q[l][u][2 * PD + hd * PDH + c];
            dq[u][2 * PD + hd * PDH + c] += P[u] * dov[t][hd * PDH + c];
          }
          dot += P[u] * dP[u];
        }
        for (int u = 0; u < n_tok; ++u) {
          const double ds = P[u] * (dP[u] - dot) / 4.0; /* through s = q.k / sqrt(16) */
          if (!mk[u]) continue;
          for (int c = 0; c < PDH; ++c) {
            dq[t][hd * PDH + c] += ds * tp->q[l][u][PD + hd * PDH + c];
            dq[u][PD + hd * PDH + c] += ds * tp->q[l][t][hd * PDH + c];
          }
        }
      }
    for (int t = 0; t < n_tok; ++t) {
      for (int i = 0; i < PD; ++i) da[i] = 0.0;
      for (int r = 0; r < 3 * PD; ++r) {
        dbqkv[r] += dq[t][r];
        for (int i = 0; i < PD; ++i) {
          dWqkv[r * PD + i] += dq[t][r] * tp->a1[l][t][i];
          da[i] += Wqkv[r * PD + i] * dq[t][r];
        }
      }
      ln_backward(tp->hin[l][t], g1, da, dx, dg1, db1n);
      for (int d = 0; d < PD; ++d) dh[t][d] += dx[d];
    }
  }
}

/* grad [P] += the gradient of sum_a dlogits[a] . logits[a] (plain form:
 * tokens [A][n_tok][6], the head on the first token). */
void orc_policy_backward(int64_t A, int n_tok, const double *tokens, const uint8_t *mask,
                         const double *th, const double *dlogits, double *grad) {
  policy_tape *tp = (policy_tape *)malloc(sizeof(policy_tape));
  double h[P_MAXT][PD], dh[P_MAXT][PD];
  const double *tl = th + PD * 6 + PD;
  for (int64_t ag = 0; ag < A; ++ag) {
    const double *x = tokens + ag * n_tok * 6;
    for (int t = 0; t < n_tok; ++t) policy_embed(th, x + t * 6, h[t]);
    policy_trunk_taped(n_tok, h, mask + ag * n_tok, tl, tp);
    policy_trunk_backward(n_tok, mask + ag * n_tok, tl, tp, dlogits + ag * PA, NULL,
                          grad + PD * 6 + PD, dh);
    for (int t = 0; t < n_tok; ++t)
      for (int d = 0; d < PD; ++d) {
        grad[PD * 6 + d] += dh[t][d];
        for (int c = 0; c < 6; ++c) grad[d * 6 + c] += dh[t][d] * x[t * 6 + c];
      }
  }
  free(tp);
}

/* The recurrent form: the carried state hidden_in [A][64] (NULL: zeros) is
 * row 0; dnext [A][64] (may be NULL) is the loss gradient at the state this
 * step passes on (its head input, which the next step reads), so that a
 * sequence is differentiated by calling the steps in reverse order with
 * dnext = the following step's dhidden; dhidden [A][64] (may be NULL)
 * receives the gradient at hidden_in. */
void orc_policy_backward_rec(int64_t A, int n_obs, const double *tokens, const uint8_t *mask,
                             const double *hidden_in, const double *th, const double *dlogits,
                             const double *dnext, double *grad, double *dhidden) {
  policy_tape *tp = (policy_tape *)malloc(sizeof(policy_tape));
  double h[P_MAXT][PD], dh[P_MAXT][PD];
  uint8_t mk[P_MAXT];
  const double *tl = th + PD * 6 + PD;
  for (int64_t ag = 0; ag < A; ++ag) {
    const double *x = tokens + ag * n_obs * 6;
    for (int d = 0; d < PD; ++d) h[0][d] = hidden_in ? hidden_in[ag * PD + d] : 0.0;
    mk[0] = 1;
    for (int t = 0; t < n_obs; ++t) {
      policy_embed(th, x + t * 6, h[1 + t]);
      mk[1 + t] = mask[ag * n_obs + t];
    }
    policy_trunk_taped(1 + n_obs, h, mk, tl, tp);
    policy_trunk_backward(1 + n_obs, mk, tl, tp, dlogits + ag * PA, dnext ? dnext + ag * PD : NULL,
                          grad + PD * 6 + PD, dh);
    if (dhidden)
      for (int d = 0; d < PD; ++d) dhidden[ag * PD + d] = dh[0][d];
    for (int t = 0; t < n_obs; ++t)
      for (int d = 0; d < PD; ++d) {
        grad[PD * 6 + d] += dh[1 + t][d];
        for (int c = 0; c < 6; ++c) grad[d * 6 + c] += dh[1 + t][d] * x[t * 6 + c];
      }
  }
  free(tp);
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
