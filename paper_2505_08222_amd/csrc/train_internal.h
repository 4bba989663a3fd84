// Launchers of train_kernels.hip: the per-row and per-(agent, head) parts of
// the attention networks' FP32 training forward pass (with its tape) and of
// its reverse pass. Row-major arrays; an agent's n_tok rows are consecutive.
#pragma once
#include <stdint.h>

namespace mil {

// h [R][64] = embedding of each observed row, or the carried state (rec = 1,
// the first row of each agent; NULL hidden: zeros); xaug [R][8] = (x, 1, 0)
// or zeros for a carried row; mrow [R] = key mask (1 for a carried row).
int tr_embed(const float *obs, const uint8_t *mask, int64_t R, int nt, int rec,
             const float *hidden, const float *prm, float *h, float *xaug, uint8_t *mrow,
             void *stream);
int tr_layernorm(const float *x, const float *g, const float *b, float *y, int64_t R, void *stream);
// out [R][N] = base (NULL: 0) + bias broadcast over rows
int tr_bias_rows(const float *base, const float *bias, int64_t R, int N, float *out, void *stream);
// z [R][256] = x [R][64] W1^T + b1 (W1 [256][64]) and f = GELU(z), on the FP32
// matrix cores (x 16-byte aligned)
int tr_ffn_up(const float *x, const float *w1, const float *b1, float *z, float *f, int64_t R,
              void *stream);
// dz [R][256] *= GELU'(z) in place; bias_grad [256] (+)= its column sums
// (scratch: tr_colsum_scratch_doubles() doubles; 16-byte aligned arrays)
int tr_gelu_back_sums(float *dz, const float *z, int64_t R, double *scratch, int acc,
                      float *bias_grad, void *stream);
// qkv [R][192] -> P [A][4][nt][nt] (softmax over unmasked keys), o [R][64]
int tr_attention(const float *qkv, const uint8_t *mrow, int64_t A, int nt, float *P, float *o,
                 void *stream);
// dout [R][64] (gradient at o) -> dqkv [R][192]
int tr_attention_back(const float *qkv, const float *P, const uint8_t *mrow, const float *dout,
                      int64_t A, int nt, float *dqkv, void *stream);
// dxacc += LayerNorm input gradient; then gain_grad (+)= column sums of
// dy * xhat, bias_grad (+)= those of dy and next_grad (may be NULL) (+)= those
// of the updated dxacc (scratch as for tr_colsum; 16-byte aligned arrays)
int tr_layernorm_back_sums(const float *x, const float *g, const float *dy, float *dxacc,
                           int64_t R, double *scratch, int acc, float *gain_grad,
                           float *bias_grad, float *next_grad, void *stream);
// final LayerNorm of each agent's first row -> feat [A][64], logits [A][8] (may be NULL)
int tr_head(const float *h, int64_t A, int nt, const float *prm, float *logits, float *feat,
            void *stream);
// dnext [A][64] (may be NULL): an extra gradient at the head's input
int tr_head_back(const float *h, int64_t A, int nt, const float *prm, const float *dout, int ld,
                 int n_out, const float *dnext, float *dl8, float *dh, float *gfa, float *bfa,
                 void *stream);
// acc = 1: add into grad instead of writing (likewise for the two below)
int tr_embed_grad_scatter(const float *gaug, int acc, float *grad, void *stream);
int tr_first_rows(const float *dh, int64_t A, int nt, float *out, void *stream);
int tr_fill(float *p, float v, int64_t n, void *stream);
// out [N] = column sums of Y [R][N] (N <= 256), FP64 in a fixed order;
// scratch holds tr_colsum_scratch_doubles() doubles
int64_t tr_colsum_scratch_doubles();
int tr_colsum(const float *Y, int64_t R, int N, double *scratch, int acc, float *out,
              void *stream);
// dW [N][K] (+)= dY^T X over the R rows (dY [R][N], X [R][K]) on the FP32
// matrix cores, in up to kWgMaxBlocks row blocks whose partials (part holds
// kWgMaxBlocks * N * K floats) are then added in a fixed order. Shapes
// (N, K) in {(64, 64), (64, 256), (192, 64), (256, 64), (64, 8)}; -2 for any other
// (the caller uses a library GEMM), -1 if a launch failed.
constexpr int kWgMaxBlocks = 512;
int tr_wgrad(const float *dY, const float *X, int64_t R, int N, int K, float *part, int acc,
             float *out, void *stream);
// out [n] (+)= sum over b < nb of part[b][n], in order (FP64 sums)
int tr_sum_partials(const float *part, int nb, int64_t n, int acc, float *out, void *stream);

}  // namespace mil
