// Constants, parameter layout and launchers of the attention policy
// (policy_kernels.hip). The FP32 parameter vector is, in order: token
// embedding W [64][6], b [64]; per layer: ln1 gain, offset [64], Wqkv
// [192][64] (Q, K, V rows), bqkv [192], Wo [64][64], bo [64], ln2 gain,
// offset [64], W1 [256][64], b1 [256], W2 [64][256], b2 [64]; final
// LayerNorm gain, offset [64]; head Wh [8][64], bh [8]. Weight matrices are
// row-major (output, input).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mil {

constexpr int kPolD = 64, kPolHeads = 4, kPolDh = 16, kPolF = 256, kPolLayers = 2;
constexpr int kPolActions = 8;   // head rows (the first n_actions are used)
constexpr int kPolMaxTok = 16;   // tokens per agent (agents + targets of an env)
constexpr int kPolRows = 80;     // token rows per tile (two tiles' LDS fit one CU)
constexpr int kPolBlocksPerCU = 2;
constexpr int kPolMaxAgents = 16;
constexpr int kPolLdD = kPolD + 8, kPolLdF = kPolF + 8;
// offsets inside one layer
constexpr int kPolLn1G = 0, kPolLn1B = 64, kPolWqkv = 128, kPolBqkv = kPolWqkv + 3 * 64 * 64;
constexpr int kPolWo = kPolBqkv + 192, kPolBo = kPolWo + 64 * 64, kPolLn2G = kPolBo + 64;
constexpr int kPolLn2B = kPolLn2G + 64, kPolW1 = kPolLn2B + 64, kPolB1 = kPolW1 + 256 * 64;
constexpr int kPolW2 = kPolB1 + 256, kPolB2 = kPolW2 + 64 * 256;
constexpr int kPolLayerParams = kPolB2 + 64;
// offsets in the whole vector
constexpr int kPolOffEmbW = 0, kPolOffEmbB = 64 * 6, kPolOffLayer0 = kPolOffEmbB + 64;
constexpr int kPolOffFinal = kPolOffLayer0 + kPolLayers * kPolLayerParams;
constexpr int kPolLnfG = 0, kPolLnfB = 64, kPolWh = 128, kPolBh = kPolWh + kPolActions * 64;
constexpr int kPolNumParams = kPolOffFinal + kPolBh + kPolActions;
// LDS copy of the small FP32 parameters: embedding W [64][6] and b [64]; per
// layer ln1 gain/offset, bqkv, bo, ln2 gain/offset, b1, b2; the final
// LayerNorm and head exactly as in the vector.
constexpr int kSmEmbW = 0, kSmEmbB = 64 * 6, kSmLayer0 = kSmEmbB + 64;
constexpr int kSmLn1G = 0, kSmLn1B = 64, kSmBqkv = 128, kSmBo = kSmBqkv + 192, kSmLn2G = kSmBo + 64;
constexpr int kSmLn2B = kSmLn2G + 64, kSmB1 = kSmLn2B + 64, kSmB2 = kSmB1 + 256;
constexpr int kSmLayer = kSmB2 + 64;
constexpr int kSmFinal = kSmLayer0 + kPolLayers * kSmLayer;
constexpr int kSmTotal = kSmFinal + kPolBh + kPolActions;
// MFMA-ready BF16 weights (elements)
constexpr int64_t kPolPrepWqkv = (int64_t)kPolLayers * 3 * kPolD * kPolLdD;
constexpr int64_t kPolPrepWo = (int64_t)kPolLayers * kPolD * kPolLdD;
constexpr int64_t kPolPrepW1 = (int64_t)kPolLayers * kPolF * kPolLdD;
constexpr int64_t kPolPrepW2 = (int64_t)kPolLayers * kPolD * kPolLdF;
constexpr int64_t kPolPrepBytes = (kPolPrepWqkv + kPolPrepWo + kPolPrepW1 + kPolPrepW2) * 2;

struct PolicyArgs {
  int64_t A;                 // agents (fixed count per env)
  int32_t n_tok;             // tokens per agent
  int32_t agents_per_tile;
  const float *obs;          // [A * n_tok][6]
  const uint8_t *mask;       // [A * n_tok]
  const float *params;       // FP32 master parameters
  const __bf16 *wqkv, *wo, *w1, *w2;
  float *logits;             // [A][8] or null
  float *feat;               // [A][64] or null: the head's input (final LN of the first row)
  // recurrent form: rec = 1 puts a carried state ahead of each agent's
  // n_tok - 1 observed tokens as an unmasked first row (hidden_in [A][64], or
  // zeros when null; feat may alias it); rec = 0: n_tok observed tokens
  const float *hidden_in;
  int32_t rec;
  int32_t *actions;          // [A] or null
  int64_t n_agents;          // agents per env
  int32_t n_actions;
  uint32_t t, episode, key0, key1;
  const uint32_t *env_ids;   // packed env -> global id (null: identity)
};

int launch_policy_init(float *th, uint64_t seed, void *stream);
int launch_policy_prepare(const float *th, __bf16 *wqkv, __bf16 *wo, __bf16 *w1, __bf16 *w2,
                          void *stream);
int launch_policy(const PolicyArgs &args, int num_cus, void *stream);

// ppo_kernels.hip: the learner's forward half (critic tokens, GAE, clipped
// PPO objective); partial sums in kPpoBlocks blocks of four doubles.
constexpr int kPpoBlocks = 256;
int launch_critic_tokens(const float *gstate, int64_t N, int M, int lead, float pos_scale,
                         float *tokens, uint8_t *mask, void *stream);
int launch_first_column(const float *logits, int64_t N, float *out, void *stream);
int launch_gae(const float *rewards, const uint8_t *dones, const float *values, int32_t T, int64_t E,
               float gamma, float lambda, float *adv, float *ret, void *stream);
// Linear-head gradient in the head's layout (weights [8][64], biases [8]):
// grad[o][i] = sum_n dout[n * ld + o] feat[n][i], bias o = sum_n dout[n * ld + o]
// for o < n_out, 0 for the other rows; fixed-order sums.
int launch_head_grad(const float *feat, const float *dout, int64_t N, int ld, int n_out,
                     float *grad, double *part, void *stream);
int launch_ppo_objective(const float *lnew, const float *lold, const int32_t *actions,
                         const float *adv, const float *values, const float *returns, int32_t T,
                         int64_t A, int32_t n_agents, int32_t n_actions, float clip_eps,
                         double *out, float *dlogits, float *dvalues, double *part, void *stream);

}  // namespace mil
