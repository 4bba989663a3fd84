// C ABI of the attention networks' training form (declared in
// include/mi_lrauv.h, "learner"): the FP32 forward pass that records its
// tape in the caller's workspace, the reverse pass into the parameter
// gradient, and the critic's variant on global states. Per-row work runs in
// train_kernels.hip, and so do the layers' weight gradients (FP32 matrix
// cores, fixed-order partial sums), the feed-forward up-projection with its
// bias and GELU (FP32 matrix cores) and the column sums; the other dense
// products are plain FP32 GEMMs: the other forward ones in hipBLASLt with its
// bias epilogue, the input gradients into 64-wide rows in hipBLASLt, the rest in
// rocBLAS (atomics off). hipBLASLt runs without workspace, with the
// heuristic's first algorithm per shape, so results do not depend on the run.
#include <hip/hip_runtime.h>
#include <hipblaslt/hipblaslt.h>
#include <rocblas/rocblas.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "mi_lrauv.h"
#include "policy_internal.h"
#include "train_internal.h"

extern "C" int mil_set_error(int code, const char *msg);  // abi.cpp

namespace {

constexpr int D = mil::kPolD, F = mil::kPolF, L = mil::kPolLayers, NA = mil::kPolActions;
constexpr int kMaxSplit = 64;  // row chunks of a weight gradient's sum

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

// Workspace: the tape (per layer the inputs of every operation) and the
// reverse pass's scratch, all [rows][...] FP32 unless stated.
struct TrainWork {
  int64_t tok, tmask, xaug, mrow, h[L + 1], a1[L], qkv[L], P[L], o[L], hmid[L], a2[L], z[L], f[L],
      feat, dh, t64, dqkv, dz, dl8, gfa, bfa, gaug, csum, wpart, total;
};

TrainWork train_work(int64_t A, int nt) {
  const int64_t R = A * nt;
  TrainWork w{};
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    const int64_t at = o;
    o = align256(o + bytes);
    return at;
  };
  w.tok = take(R * 6 * 4);
  w.tmask = take(R);
  w.xaug = take(R * 8 * 4);
  w.mrow = take(R);
  for (int l = 0; l <= L; ++l) w.h[l] = take(R * D * 4);
  for (int l = 0; l < L; ++l) {
    w.a1[l] = take(R * D * 4);
    w.qkv[l] = take(R * 3 * D * 4);
    w.P[l] = take(A * mil::kPolHeads * nt * nt * 4);
    w.o[l] = take(R * D * 4);
    w.hmid[l] = take(R * D * 4);
    w.a2[l] = take(R * D * 4);
    w.z[l] = take(R * F * 4);
    w.f[l] = take(R * F * 4);
  }
  w.feat = take(A * D * 4);
  w.dh = take(R * D * 4);
  w.t64 = take(R * D * 4);
  w.dqkv = take(R * 3 * D * 4);
  w.dz = take(R * F * 4);
  w.dl8 = take(A * NA * 4);
  w.gfa = take(A * D * 4);
  w.bfa = take(A * D * 4);
  w.gaug = take(D * 8 * 4);
  w.csum = take(mil::tr_colsum_scratch_doubles() * 8);
  // weight-gradient partials; the largest weight is 256 x 64
  w.wpart = take((int64_t)(kMaxSplit + 1 > mil::kWgMaxBlocks ? kMaxSplit + 1 : mil::kWgMaxBlocks) *
                 F * D * 4);
  w.total = o;
  return w;
}

// One rocBLAS handle per device, made on first use (pointer mode host,
// atomics off so that every sum is taken in one order). The handle carries
// the stream of the call in progress: training-form calls on one device must
// not overlap from several host threads.
rocblas_handle blas_for_current_device() {
  static rocblas_handle handles[64] = {};
  static std::mutex made;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(made);
  if (!handles[dev]) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
    rocblas_set_pointer_mode(h, rocblas_pointer_mode_host);
    rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed);
    handles[dev] = h;
  }
  return handles[dev];
}

// hipBLASLt, per device: a handle and the plans (descriptors and algorithm)
// of the column-major products D [m][n] = op(A) B [k][n] (+ C) (+ bias [m]
// broadcast over columns) seen so far, made on first use; op(A) = A [m][k],
// or A^T for A [k][m] when trans. Same threading rule as the rocBLAS handle.
struct LtPlan {
  int64_t m, n, k;
  bool add, trans, bias;
  bool ok;  // the heuristic offered an algorithm that needs no workspace
  hipblasLtMatmulDesc_t desc = nullptr;
  hipblasLtMatrixLayout_t la = nullptr, lb = nullptr, lc = nullptr;
  hipblasLtMatmulAlgo_t algo;
};

struct LtDevice {
  hipblasLtHandle_t h = nullptr;
  std::vector<LtPlan> plans;
};

void lt_drop(LtPlan &p) {
  if (p.la) hipblasLtMatrixLayoutDestroy(p.la);
  if (p.lb) hipblasLtMatrixLayoutDestroy(p.lb);
  if (p.lc) hipblasLtMatrixLayoutDestroy(p.lc);
  if (p.desc) hipblasLtMatmulDescDestroy(p.desc);
}

// The plan for (m, n, k, add, trans, bias) on the current device; NULL if
// hipBLASLt is unavailable or offers no algorithm without workspace for it.
const LtPlan *lt_plan(int64_t m, int64_t n, int64_t k, bool add, bool trans, bool bias,
                      hipblasLtHandle_t *handle) {
  constexpr int kMaxPlans = 64;
  static LtDevice devs[64];
  static std::mutex made;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(made);
  LtDevice &d = devs[dev];
  if (!d.h && hipblasLtCreate(&d.h) != HIPBLAS_STATUS_SUCCESS) {
    d.h = nullptr;
    return nullptr;
  }
  *handle = d.h;
  for (const LtPlan &p : d.plans)
    if (p.m == m && p.n == n && p.k == k && p.add == add && p.trans == trans && p.bias == bias)
      return p.ok ? &p : nullptr;
  if ((int)d.plans.size() >= kMaxPlans) {  // many distinct batch sizes: start over
    for (LtPlan &p : d.plans) lt_drop(p);
    d.plans.clear();
  }
  d.plans.reserve(kMaxPlans);  // plans never move while in use
  LtPlan p{m, n, k, add, trans, bias, false};
  if (hipblasLtMatmulDescCreate(&p.desc, HIPBLAS_COMPUTE_32F, HIP_R_32F) != HIPBLAS_STATUS_SUCCESS)
    p.desc = nullptr;
  if (hipblasLtMatrixLayoutCreate(&p.la, HIP_R_32F, trans ? k : m, trans ? m : k, trans ? k : m) !=
      HIPBLAS_STATUS_SUCCESS)
    p.la = nullptr;
  if (hipblasLtMatrixLayoutCreate(&p.lb, HIP_R_32F, k, n, k) != HIPBLAS_STATUS_SUCCESS)
    p.lb = nullptr;
  if (hipblasLtMatrixLayoutCreate(&p.lc, HIP_R_32F, m, n, m) != HIPBLAS_STATUS_SUCCESS)
    p.lc = nullptr;
  if (!p.desc || !p.la || !p.lb || !p.lc) {  // out of host memory: rocBLAS serves this call
    lt_drop(p);
    return nullptr;
  }
  bool set = true;
  if (trans) {
    const int32_t op = HIPBLAS_OP_T;
    set = hipblasLtMatmulDescSetAttribute(p.desc, HIPBLASLT_MATMUL_DESC_TRANSA, &op, sizeof(op)) ==
          HIPBLAS_STATUS_SUCCESS;
  }
  if (bias && set) {
    const uint32_t epi = HIPBLASLT_EPILOGUE_BIAS;
    const int32_t bt = HIP_R_32F;
    set = hipblasLtMatmulDescSetAttribute(p.desc, HIPBLASLT_MATMUL_DESC_EPILOGUE, &epi,
                                          sizeof(epi)) == HIPBLAS_STATUS_SUCCESS &&
          hipblasLtMatmulDescSetAttribute(p.desc, HIPBLASLT_MATMUL_DESC_BIAS_DATA_TYPE, &bt,
                                          sizeof(bt)) == HIPBLAS_STATUS_SUCCESS;
  }
  if (!set) {
    lt_drop(p);
    return nullptr;
  }
  hipblasLtMatmulPreference_t pref;
  if (hipblasLtMatmulPreferenceCreate(&pref) == HIPBLAS_STATUS_SUCCESS) {
    uint64_t none = 0;
    hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &none,
                                          sizeof(none));
    hipblasLtMatmulHeuristicResult_t res[1];
    int got = 0;
    if (hipblasLtMatmulAlgoGetHeuristic(d.h, p.desc, p.la, p.lb, p.lc, p.lc, pref, 1, res, &got) ==
            HIPBLAS_STATUS_SUCCESS &&
        got > 0 && res[0].state == HIPBLAS_STATUS_SUCCESS && res[0].workspaceSize == 0) {
      p.algo = res[0].algo;
      p.ok = true;
    }
    hipblasLtMatmulPreferenceDestroy(pref);
  }
  d.plans.push_back(p);
  return d.plans.back().ok ? &d.plans.back() : nullptr;
}

struct Ctx {
  rocblas_handle h;
  void *stream;
  double *csum;  // column-sum scratch
  float *wpart;  // weight-gradient partials [kMaxSplit + 1][N * K]
  int acc = 0;   // parameter gradients: add into the output instead of writing
  bool ok = true;
  // Y [R][N] = X [R][K] W^T (W [N][K] row-major), added to Y when beta = 1
  void xwt(const float *X, const float *W, float *Y, int64_t R, int N, int K, float beta) {
    const float one = 1.0f;
    ok = ok && rocblas_sgemm(h, rocblas_operation_transpose, rocblas_operation_none, N, (int)R, K,
                             &one, W, K, X, K, &beta, Y, N) == rocblas_status_success;
  }
  // Y [R][N] = X [R][K] W^T + b (+ res [R][N], may be NULL): in hipBLASLt with
  // its bias epilogue (one pass over Y), else the bias rows then rocBLAS
  void linear(const float *X, const float *W, const float *b, const float *res, float *Y,
              int64_t R, int N, int K) {
    const float one = 1.0f, beta = res ? 1.0f : 0.0f;
    if (!ok) return;
    hipblasLtHandle_t lh = nullptr;
    const LtPlan *p = lt_plan(N, R, K, res != nullptr, true, true, &lh);
    if (p) {
      const void *bp = b;
      ok = hipblasLtMatmulDescSetAttribute(p->desc, HIPBLASLT_MATMUL_DESC_BIAS_POINTER, &bp,
                                           sizeof(bp)) == HIPBLAS_STATUS_SUCCESS &&
           hipblasLtMatmul(lh, p->desc, &one, W, p->la, X, p->lb, &beta, res ? res : Y, p->lc, Y,
                           p->lc, &p->algo, nullptr, 0, (hipStream_t)stream) ==
               HIPBLAS_STATUS_SUCCESS;
      return;
    }
    k(mil::tr_bias_rows(res, b, R, N, Y, stream));
    xwt(X, W, Y, R, N, K, 1.0f);
  }
  // dX [R][K] = dY [R][N] W [N][K] (+ dX when beta = 1); 64-wide outputs in
  // hipBLASLt (2.5-3x faster than rocBLAS on these shapes), others in rocBLAS
  void xw(const float *dY, const float *W, float *dX, int64_t R, int N, int K, float beta) {
    const float one = 1.0f;
    if (!ok) return;
    hipblasLtHandle_t lh = nullptr;
    const LtPlan *p = K == D ? lt_plan(K, R, N, beta != 0.0f, false, false, &lh) : nullptr;
    if (p) {
      ok = hipblasLtMatmul(lh, p->desc, &one, W, p->la, dY, p->lb, &beta, dX, p->lc, dX, p->lc,
                           &p->algo, nullptr, 0, (hipStream_t)stream) == HIPBLAS_STATUS_SUCCESS;
      return;
    }
    ok = rocblas_sgemm(h, rocblas_operation_none, rocblas_operation_none, K, (int)R, N, &one, W,
                       K, dY, N, &beta, dX, K) == rocblas_status_success;
  }
  // dW [N][K] = dY^T X summed over the R rows: on the matrix cores
  // (tr_wgrad) for the layers' shapes; otherwise the rows split into up to
  // kMaxSplit equal chunks (one batched GEMM, one product per chunk, plus the
  // remainder), the chunks' products then added in order
  void dw(const float *dY, const float *X, float *dW, int64_t R, int N, int K) {
    const float one = 1.0f, zero = 0.0f, beta = acc ? 1.0f : 0.0f;
    if (!ok) return;
    const int rc = mil::tr_wgrad(dY, X, R, N, K, wpart, acc, dW, stream);
    if (rc != -2) {  // the matrix-core kernel took it
      ok = rc == 0;
      return;
    }
    const int64_t nb = R / 4096 < kMaxSplit ? R / 4096 : kMaxSplit;
    if (nb <= 1) {
      ok = ok && rocblas_sgemm(h, rocblas_operation_none, rocblas_operation_transpose, K, N, (int)R,
                               &one, X, K, dY, N, &beta, dW, K) == rocblas_status_success;
      return;
    }
    const int64_t chunk = R / nb, rem = R - nb * chunk, nk = (int64_t)N * K;
    ok = ok && rocblas_sgemm_strided_batched(
                   h, rocblas_operation_none, rocblas_operation_transpose, K, N, (int)chunk, &one,
                   X, K, chunk * K, dY, N, chunk * N, &zero, wpart, K, nk, (int)nb) ==
                   rocblas_status_success;
    if (rem > 0)
      ok = ok && rocblas_sgemm(h, rocblas_operation_none, rocblas_operation_transpose, K, N,
                               (int)rem, &one, X + nb * chunk * K, K, dY + nb * chunk * N, N,
                               &zero, wpart + nb * nk, K) == rocblas_status_success;
    k(mil::tr_sum_partials(wpart, (int)(nb + (rem > 0)), nk, acc, dW, stream));
  }
  // out [N] = column sums of Y [R][N]
  void colsum(const float *Y, float *out, int64_t R, int N) {
    k(mil::tr_colsum(Y, R, N, csum, acc, out, stream));
  }
  void k(int rc) { ok = ok && rc == 0; }
};

int check_args(int64_t A, int32_t n_tok, int32_t rec, void *d_work, int64_t work_bytes) {
  if (A < 1 || rec < 0 || rec > 1 || n_tok < 1 + rec || n_tok > mil::kPolMaxTok)
    return mil_set_error(MIL_EINVAL, "need A >= 1, rec in {0, 1}, n_tok in 1 + rec..16");
  if (A * n_tok > INT32_MAX / (3 * D))
    return mil_set_error(MIL_EINVAL, "A * n_tok too large for one pass (split the batch)");
  if (!d_work || (((uintptr_t)d_work) & 255))
    return mil_set_error(MIL_EALIGN, "workspace must be 256-byte aligned");
  if (work_bytes < train_work(A, n_tok).total)
    return mil_set_error(MIL_ESHAPE, "workspace too small (policy_train_workspace_bytes)");
  return MIL_OK;
}

int train_forward(int64_t A, int nt, int rec, const float *obs, const uint8_t *mask,
                  const float *hidden, const float *prm, float *logits, float *feat_out,
                  char *ws, void *stream) {
  rocblas_handle bh = blas_for_current_device();
  if (!bh || rocblas_set_stream(bh, (hipStream_t)stream) != rocblas_status_success)
    return mil_set_error(MIL_EHIP, "rocBLAS handle unavailable");
  const TrainWork w = train_work(A, nt);
  const int64_t R = A * nt;
  auto fp = [&](int64_t off) { return (float *)(ws + off); };
  Ctx c{bh, stream, (double *)(ws + w.csum), fp(w.wpart)};
  uint8_t *mrow = (uint8_t *)(ws + w.mrow);
  c.k(mil::tr_embed(obs, mask, R, nt, rec, hidden, prm, fp(w.h[0]), fp(w.xaug), mrow, stream));
  for (int l = 0; l < L && c.ok; ++l) {
    const float *lp = prm + mil::kPolOffLayer0 + (int64_t)l * mil::kPolLayerParams;
    c.k(mil::tr_layernorm(fp(w.h[l]), lp + mil::kPolLn1G, lp + mil::kPolLn1B, fp(w.a1[l]), R,
                          stream));
    c.linear(fp(w.a1[l]), lp + mil::kPolWqkv, lp + mil::kPolBqkv, nullptr, fp(w.qkv[l]), R, 3 * D,
             D);
    c.k(mil::tr_attention(fp(w.qkv[l]), mrow, A, nt, fp(w.P[l]), fp(w.o[l]), stream));
    c.linear(fp(w.o[l]), lp + mil::kPolWo, lp + mil::kPolBo, fp(w.h[l]), fp(w.hmid[l]), R, D, D);
    c.k(mil::tr_layernorm(fp(w.hmid[l]), lp + mil::kPolLn2G, lp + mil::kPolLn2B, fp(w.a2[l]), R,
                          stream));
    c.k(mil::tr_ffn_up(fp(w.a2[l]), lp + mil::kPolW1, lp + mil::kPolB1, fp(w.z[l]), fp(w.f[l]), R,
                       stream));
    c.linear(fp(w.f[l]), lp + mil::kPolW2, lp + mil::kPolB2, fp(w.hmid[l]), fp(w.h[l + 1]), R, D,
             F);
  }
  c.k(mil::tr_head(fp(w.h[L]), A, nt, prm, logits, fp(w.feat), stream));
  if (feat_out && c.ok)
    c.ok = hipMemcpyAsync(feat_out, fp(w.feat), A * D * 4, hipMemcpyDeviceToDevice,
                          (hipStream_t)stream) == hipSuccess;
  return c.ok ? MIL_OK : mil_set_error(MIL_EHIP, "training forward launch failed");
}

}  // namespace

extern "C" {

int64_t policy_train_workspace_bytes(int64_t A, int32_t n_tok) {
  if (A < 1 || n_tok < 1 || n_tok > mil::kPolMaxTok) return -1;
  return train_work(A, n_tok).total;
}

int policy_train_forward(int64_t A, int32_t n_tok, int32_t rec, const float *d_obs,
                         const uint8_t *d_mask, const float *d_hidden_in, const float *d_params,
                         float *d_logits, float *d_feat, void *d_work, int64_t work_bytes,
                         void *stream) {
  int rc = check_args(A, n_tok, rec, d_work, work_bytes);
  if (rc) return rc;
  if (!d_obs || !d_mask || !d_params) return mil_set_error(MIL_EINVAL, "null argument");
  return train_forward(A, n_tok, rec, d_obs, d_mask, d_hidden_in, d_params, d_logits, d_feat,
                       (char *)d_work, stream);
}

int critic_train_forward(const float *d_gstate, int64_t N, int32_t n_agents, int32_t n_targets,
                         float pos_scale, int32_t rec, const float *d_hidden_in,
                         const float *d_params, float *d_values, float *d_feat, void *d_work,
                         int64_t work_bytes, void *stream) {
  if (n_agents < 1 || n_targets < 1 || n_agents + n_targets + 1 > mil::kPolMaxTok)
    return mil_set_error(MIL_EINVAL, "need 1 + n_agents + n_targets <= 16");
  if (!(pos_scale > 0.0f)) return mil_set_error(MIL_EINVAL, "pos_scale must be > 0");
  const int M = n_agents + n_targets, nt = M + 1;
  int rc = check_args(N, nt, rec, d_work, work_bytes);
  if (rc) return rc;
  if (!d_gstate || !d_params || !d_values) return mil_set_error(MIL_EINVAL, "null argument");
  char *ws = (char *)d_work;
  const TrainWork w = train_work(N, nt);
  float *tok = (float *)(ws + w.tok);
  uint8_t *tmask = (uint8_t *)(ws + w.tmask);
  // plain: the all-zero value token then the entities; recurrent: the
  // entities (the carried state takes the first row)
  if (mil::launch_critic_tokens(d_gstate, N, M, 1 - rec, pos_scale, tok, tmask, stream))
    return mil_set_error(MIL_EHIP, "critic token launch failed");
  float *logits = (float *)(ws + w.dz);  // free until the reverse pass
  rc = train_forward(N, nt, rec, tok, tmask, d_hidden_in, d_params, logits, d_feat, ws, stream);
  if (rc) return rc;
  if (mil::launch_first_column(logits, N, d_values, stream))
    return mil_set_error(MIL_EHIP, "critic value launch failed");
  return MIL_OK;
}

int policy_train_backward(int64_t A, int32_t n_tok, int32_t rec, const float *d_params,
                          const float *d_dout, int32_t ld, int32_t n_out, const float *d_dnext,
                          int32_t accumulate, float *d_grad, float *d_dhidden, void *d_work,
                          int64_t work_bytes, void *stream) {
  int rc = check_args(A, n_tok, rec, d_work, work_bytes);
  if (rc) return rc;
  if (n_out < 1 || n_out > NA || ld < n_out)
    return mil_set_error(MIL_EINVAL, "need n_out in 1..8 and ld >= n_out");
  if (!d_params || !d_dout || !d_grad) return mil_set_error(MIL_EINVAL, "null argument");
  rocblas_handle bh = blas_for_current_device();
  if (!bh || rocblas_set_stream(bh, (hipStream_t)stream) != rocblas_status_success)
    return mil_set_error(MIL_EHIP, "rocBLAS handle unavailable");
  char *ws = (char *)d_work;
  const int nt = n_tok;
  const TrainWork w = train_work(A, nt);
  const int64_t R = A * nt;
  auto fp = [&](int64_t off) { return (float *)(ws + off); };
  const uint8_t *mrow = (const uint8_t *)(ws + w.mrow);
  float *dh = fp(w.dh), *t64 = fp(w.t64);
  Ctx c{bh, stream, (double *)(ws + w.csum), fp(w.wpart), accumulate ? 1 : 0};
  float *gfin = d_grad + mil::kPolOffFinal;
  // head and final LayerNorm (each agent's first row)
  c.k(mil::tr_fill(dh, 0.0f, R * D, stream));
  c.k(mil::tr_head_back(fp(w.h[L]), A, nt, d_params, d_dout, ld, n_out, d_dnext, fp(w.dl8), dh,
                        fp(w.gfa), fp(w.bfa), stream));
  c.dw(fp(w.dl8), fp(w.feat), gfin + mil::kPolWh, A, NA, D);
  c.colsum(fp(w.dl8), gfin + mil::kPolBh, A, NA);
  c.colsum(fp(w.gfa), gfin + mil::kPolLnfG, A, D);
  c.colsum(fp(w.bfa), gfin + mil::kPolLnfB, A, D);
  for (int l = L - 1; l >= 0 && c.ok; --l) {
    const float *lp = d_params + mil::kPolOffLayer0 + (int64_t)l * mil::kPolLayerParams;
    float *gp = d_grad + mil::kPolOffLayer0 + (int64_t)l * mil::kPolLayerParams;
    // the bias b2 below this layer's output: summed by the LayerNorm pass of
    // the layer above, except for the last layer
    float *gprev = l > 0 ? gp - mil::kPolLayerParams : nullptr;
    // feed-forward block: h[l + 1] = hmid + W2 gelu(z) + b2
    if (l == L - 1) c.colsum(dh, gp + mil::kPolB2, R, D);
    c.dw(dh, fp(w.f[l]), gp + mil::kPolW2, R, D, F);
    c.xw(dh, lp + mil::kPolW2, fp(w.dz), R, D, F, 0.0f);
    c.k(mil::tr_gelu_back_sums(fp(w.dz), fp(w.z[l]), R, c.csum, c.acc, gp + mil::kPolB1, stream));
    c.dw(fp(w.dz), fp(w.a2[l]), gp + mil::kPolW1, R, F, D);
    c.xw(fp(w.dz), lp + mil::kPolW1, t64, R, F, D, 0.0f);
    c.k(mil::tr_layernorm_back_sums(fp(w.hmid[l]), lp + mil::kPolLn2G, t64, dh, R, c.csum, c.acc,
                                    gp + mil::kPolLn2G, gp + mil::kPolLn2B, gp + mil::kPolBo,
                                    stream));
    // attention block: hmid = h[l] + Wo attention(LN1(h[l])) + bo
    c.dw(dh, fp(w.o[l]), gp + mil::kPolWo, R, D, D);
    c.xw(dh, lp + mil::kPolWo, t64, R, D, D, 0.0f);
    c.k(mil::tr_attention_back(fp(w.qkv[l]), fp(w.P[l]), mrow, t64, A, nt, fp(w.dqkv), stream));
    c.colsum(fp(w.dqkv), gp + mil::kPolBqkv, R, 3 * D);
    c.dw(fp(w.dqkv), fp(w.a1[l]), gp + mil::kPolWqkv, R, 3 * D, D);
    c.xw(fp(w.dqkv), lp + mil::kPolWqkv, t64, R, 3 * D, D, 0.0f);
    c.k(mil::tr_layernorm_back_sums(fp(w.h[l]), lp + mil::kPolLn1G, t64, dh, R, c.csum, c.acc,
                                    gp + mil::kPolLn1G, gp + mil::kPolLn1B,
                                    gprev ? gprev + mil::kPolB2 : nullptr, stream));
  }
  // embedding (observed rows; a carried row's augmented input is zero)
  const int acc = c.acc;
  c.acc = 0;  // into the scratch matrix; the scatter then writes or adds
  c.dw(dh, fp(w.xaug), fp(w.gaug), R, D, 8);
  c.acc = acc;
  c.k(mil::tr_embed_grad_scatter(fp(w.gaug), c.acc, d_grad, stream));
  if (d_dhidden && rec) c.k(mil::tr_first_rows(dh, A, nt, d_dhidden, stream));
  return c.ok ? MIL_OK : mil_set_error(MIL_EHIP, "training backward launch failed");
}

}  // extern "C"
