// C-ABI entry points of the learned surrogate and of the tile-list exact
// fallback.  Shapes are validated on the host before any launch; the MLP's
// matrix dimensions must be multiples of the GEMM tile (64 for rows and all
// widths, the padded input width included), which the caller ensures by zero
// padding.

#include <stdio.h>

#include "../../include/qsvm.h"
#include "mlp.h"
#include "qsvm_internal.h"
#include "trace.h"
#include "sweep_common.h"

namespace qsvm {
qsvm_status api_fail(qsvm_status s, const char* msg);
qsvm_status api_ok();
qsvm_status api_hip(hipError_t e, const char* what);
bool api_injected_failure();
}  // namespace qsvm

namespace {

using qsvm::api_fail;
using qsvm::api_hip;
using qsvm::api_ok;

qsvm_status check_net(const qsvm_mlp* net, const char* what) {
  char msg[256];
  if (!net || !net->W1 || !net->W2 || !net->W3 || !net->b1 || !net->b2 || !net->b3) {
    snprintf(msg, sizeof msg, "%s: network or one of its weights is NULL", what);
    return api_fail(QSVM_ERR_INVALID_ARG, msg);
  }
  if (net->d_in < 64 || net->d_in % 64 || net->d_h1 < 64 || net->d_h1 % 64 || net->d_h2 < 64 ||
      net->d_h2 % 64 || net->d_out < 64 || net->d_out % 64) {
    snprintf(msg, sizeof msg, "%s: widths (%d, %d, %d, %d) must all be positive multiples of 64", what,
             net->d_in, net->d_h1, net->d_h2, net->d_out);
    return api_fail(QSVM_ERR_INVALID_ARG, msg);
  }
  return QSVM_OK;
}

qsvm_status check_rows(int64_t rows, const char* what) {
  char msg[160];
  if (rows < 64 || rows % 64 || rows > (int64_t(1) << 26)) {
    snprintf(msg, sizeof msg, "%s: rows = %lld must be a positive multiple of 64 (<= 2^26)", what, (long long)rows);
    return api_fail(QSVM_ERR_INVALID_ARG, msg);
  }
  return QSVM_OK;
}

qsvm_status injected(const char* what) {
  char msg[160];
  snprintf(msg, sizeof msg, "%s: injected launch failure (QSVM_FAULT_INJECT=launch)", what);
  return api_fail(QSVM_ERR_HIP, msg);
}

qsvm::GemmArgs gemm(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B, int64_t ldb,
                    void* C, void* C2, int64_t ldc, const float* bias = nullptr, const float* aux = nullptr) {
  qsvm::GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  g.C = C;
  g.C2 = C2;
  g.ldc = ldc;
  g.bias = bias;
  g.aux = aux;
  g.splits = 1;
  return g;
}

// Split-K factor of a weight-gradient GEMM with K = rows.
// Rows of the k-contiguous copy of a weight gradient's first operand (M
// activations x rows): M, one row of ones (its product row is the bias
// gradient, 1^T dH) and zeros up to a multiple of 128 where N allows the
// direct-to-LDS GEMM, else of 64.
int64_t padded_m(int64_t M, int64_t N) {
  const int64_t q = (N % 128 == 0) ? 128 : 64;
  return (M / q + 1) * q;
}

// Split-K of a weight gradient (Mp x N over K = rows): the smallest power of
// two that gives the GEMM at least 384 blocks, at most 32, each slab whole
// 64-deep steps and at least 256 rows.
int32_t grad_splits(int64_t Mp, int64_t N, int64_t rows) {
  const int64_t tiles = (Mp % 128 == 0 && N % 128 == 0) ? (Mp / 128) * (N / 128) : (Mp / 64) * (N / 64);
  int32_t s = 1;
  while (s < 32 && tiles * s < 384 && rows % (int64_t(2 * s) * 64) == 0 && rows / (2 * s) >= 256) s *= 2;
  return s;
}

// Floats of a weight gradient's scratch: its split-K slabs (Mp x N each),
// then the k-contiguous copies of its operands (Mp x rows and N x rows bf16).
int64_t grad_floats(int64_t M, int64_t N, int64_t rows) {
  const int64_t Mp = padded_m(M, N);
  return int64_t(grad_splits(Mp, N, rows)) * Mp * N + (Mp + N) * rows / 2;
}

int64_t workspace_floats(const qsvm_mlp* net, int64_t rows) {
  const int64_t din = net->d_in, h1 = net->d_h1, h2 = net->d_h2, dout = net->d_out;
  int64_t a = grad_floats(din, h1, rows);
  const int64_t b = grad_floats(h1, h2, rows), c = grad_floats(h2, dout, rows);
  if (b > a) a = b;
  if (c > a) a = c;
  return a;
}

// dW (M x N) = A^T dH and db (N) = 1^T dH over K = rows (A: rows x M,
// dH: rows x N, bf16, row-major).  Both operands are first copied
// k-contiguous, A's copy followed by a row of ones and zero rows (padded_m),
// so one product on the k-contiguous GEMMs (the direct-to-LDS kernel where
// the padded sizes are multiples of 128) gives dW in its first M rows and db
// in row M; it is split along K into slabs summed in a fixed order.
hipError_t grad_gemm(int64_t M, int64_t N, int64_t rows, const void* A, const void* B, float* dW, float* db,
                     float* ws, hipStream_t st) {
  const int64_t Mp = padded_m(M, N);
  const int32_t splits = grad_splits(Mp, N, rows);
  uint16_t* at = reinterpret_cast<uint16_t*>(ws + int64_t(splits) * Mp * N);  // 16-byte aligned: Mp, N % 64 == 0
  uint16_t* bt = at + Mp * rows;
  hipError_t e = qsvm::launch_transpose64_bf16({static_cast<const uint16_t*>(A), at, M, Mp},
                                                {static_cast<const uint16_t*>(B), bt, N, N}, rows, st);
  if (e != hipSuccess) return e;
  qsvm::GemmArgs g = gemm(Mp, N, rows, at, rows, bt, rows, ws, nullptr, N);
  g.splits = splits;
  e = qsvm::launch_gemm(0, 1, qsvm::EPI_F32, g, st);
  if (e == hipSuccess) e = qsvm::launch_sum_slabs(ws, splits, (M + 1) * N, Mp * N, dW, M * N, db, st);
  return e;
}

}  // namespace

extern "C" {

qsvm_status qsvm_gather_features(const double* X, int64_t N, int32_t n_qubits, const int32_t* idx, int64_t rows,
                                 int32_t d_pad, void* out, void* stream) {
  QSVM_TRACE_RANGE("qsvm_gather_features");
  const char* what = "qsvm_gather_features";
  if (!X || !idx || !out) return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_gather_features: NULL pointer");
  if (N < 1 || n_qubits < 1 || rows < 1 || d_pad < n_qubits)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_gather_features: need N, n_qubits, rows >= 1 and d_pad >= n_qubits");
  if (qsvm::api_injected_failure()) return injected(what);
  return api_hip(qsvm::launch_gather(X, N, n_qubits, idx, rows, d_pad, static_cast<uint16_t*>(out),
                                     static_cast<hipStream_t>(stream)),
                 what);
}

qsvm_status qsvm_mlp_forward(const qsvm_mlp* net, const void* X16, int64_t rows, const qsvm_mlp_acts* acts,
                             void* stream) {
  QSVM_TRACE_RANGE("qsvm_mlp_forward");
  const char* what = "qsvm_mlp_forward";
  qsvm_status s = check_net(net, what);
  if (s != QSVM_OK) return s;
  if ((s = check_rows(rows, what)) != QSVM_OK) return s;
  if (!X16 || !acts || !acts->A1 || !acts->A2 || !acts->E16)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_mlp_forward: input or a BF16 activation buffer is NULL");
  // inference: without the FP32 outputs (H1, H2, E all NULL) only the BF16
  // activations are written; the FP32 ones are needed by the backward pass
  const bool keep = acts->H1 || acts->H2 || acts->E;
  if (keep && (!acts->H1 || !acts->H2 || !acts->E))
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_mlp_forward: H1, H2 and E must be all given or all NULL");
  if (qsvm::api_injected_failure()) return injected(what);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // Each weight is first copied transposed (n x k, k contiguous: a
  // stream-ordered temporary of ~1.6 MB at 784-512-512-256), so the GEMMs
  // stage both operands into LDS with plain 16-byte stores instead of
  // transposing a weight slab in every block.
  const int64_t n1 = int64_t(net->d_in) * net->d_h1, n2 = int64_t(net->d_h1) * net->d_h2;
  const int64_t n3 = int64_t(net->d_h2) * net->d_out;
  uint16_t* wt = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&wt), size_t(n1 + n2 + n3) * sizeof(uint16_t), st);
  if (e != hipSuccess) return api_hip(e, what);
  uint16_t *wt1 = wt, *wt2 = wt + n1, *wt3 = wt + n1 + n2;
  qsvm::TransposeJobs tj{};
  tj.in[0] = static_cast<const uint16_t*>(net->W1);
  tj.in[1] = static_cast<const uint16_t*>(net->W2);
  tj.in[2] = static_cast<const uint16_t*>(net->W3);
  tj.out[0] = wt1;
  tj.out[1] = wt2;
  tj.out[2] = wt3;
  tj.R[0] = net->d_in, tj.C[0] = net->d_h1;
  tj.R[1] = net->d_h1, tj.C[1] = net->d_h2;
  tj.R[2] = net->d_h2, tj.C[2] = net->d_out;
  e = qsvm::launch_transpose_bf16(tj, 3, st);
  const int epi_gelu = keep ? qsvm::EPI_BIAS_GELU : qsvm::EPI_BIAS_GELU_BF16;
  const int epi_out = keep ? qsvm::EPI_BIAS : qsvm::EPI_BIAS_BF16;
  if (e == hipSuccess)
    e = qsvm::launch_gemm(0, 1, epi_gelu,
                          gemm(rows, net->d_h1, net->d_in, X16, net->d_in, wt1, net->d_in, acts->H1, acts->A1,
                               net->d_h1, net->b1),
                          st);
  if (e == hipSuccess)
    e = qsvm::launch_gemm(0, 1, epi_gelu,
                          gemm(rows, net->d_h2, net->d_h1, acts->A1, net->d_h1, wt2, net->d_h1, acts->H2, acts->A2,
                               net->d_h2, net->b2),
                          st);
  if (e == hipSuccess)
    e = qsvm::launch_gemm(0, 1, epi_out,
                          gemm(rows, net->d_out, net->d_h2, acts->A2, net->d_h2, wt3, net->d_h2, acts->E, acts->E16,
                               net->d_out, net->b3),
                          st);
  const hipError_t f = hipFreeAsync(wt, st);
  return api_hip(e != hipSuccess ? e : f, what);
}

qsvm_status qsvm_pair_head(const float* E, int64_t pairs, int32_t d, const float* target, const float* alpha_beta,
                           int32_t loss_kind, void* dE16, float* partial, float* out3, void* stream) {
  const char* what = "qsvm_pair_head";
  if (!E || !target || !alpha_beta || !dE16 || !partial || !out3)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_pair_head: NULL pointer");
  if (pairs < 1 || d < 1) return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_pair_head: pairs and d must be >= 1");
  if (loss_kind != 0 && loss_kind != 1) return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_pair_head: loss_kind must be 0 or 1");
  if (qsvm::api_injected_failure()) return injected(what);
  return api_hip(qsvm::launch_pair_head(E, pairs, d, target, alpha_beta, loss_kind, static_cast<uint16_t*>(dE16), partial,
                                        out3, static_cast<hipStream_t>(stream)),
                 what);
}

qsvm_status qsvm_pair_head_log(const void* X16, int32_t d_in, const float* E, int32_t d, int64_t pairs,
                               const float* target, const float* head, float scale, void* dE16, float* partial,
                               float* out3, float* pred, void* stream) {
  QSVM_TRACE_RANGE("qsvm_pair_head_log");
  const char* what = "qsvm_pair_head_log";
  if ((!X16 && d_in > 0) || !E || !target || !head || !dE16 || !partial || !out3)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_pair_head_log: NULL pointer");
  if (pairs < 1 || d_in < 0 || d < 1 || !(scale > 0.0f))
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_pair_head_log: need pairs >= 1, d_in >= 0, d >= 1, scale > 0");
  if (qsvm::api_injected_failure()) return injected(what);
  return api_hip(qsvm::launch_pair_head_log(static_cast<const uint16_t*>(X16), d_in, E, d, pairs, target, head, scale,
                                            static_cast<uint16_t*>(dE16), partial, out3, pred,
                                            static_cast<hipStream_t>(stream)),
                 what);
}

qsvm_status qsvm_mlp_backward(const qsvm_mlp* net, const void* X16, const qsvm_mlp_acts* acts, const void* dE16,
                              int64_t rows, const qsvm_mlp_grads* g, void* stream) {
  QSVM_TRACE_RANGE("qsvm_mlp_backward");
  const char* what = "qsvm_mlp_backward";
  qsvm_status s = check_net(net, what);
  if (s != QSVM_OK) return s;
  if ((s = check_rows(rows, what)) != QSVM_OK) return s;
  if (!X16 || !acts || !acts->H1 || !acts->A1 || !acts->H2 || !acts->A2 || !dE16 || !g || !g->dW1 || !g->db1 ||
      !g->dW2 || !g->db2 || !g->dW3 || !g->db3 || !g->dH1 || !g->dH2)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_mlp_backward: NULL pointer");
  if (!g->ws || g->ws_floats < workspace_floats(net, rows)) {
    char msg[200];
    snprintf(msg, sizeof msg, "%s: workspace of %lld floats < %lld needed (qsvm_mlp_workspace_floats)", what,
             (long long)g->ws_floats, (long long)workspace_floats(net, rows));
    return api_fail(QSVM_ERR_SIZE, msg);
  }
  if (qsvm::api_injected_failure()) return injected(what);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t din = net->d_in, h1 = net->d_h1, h2 = net->d_h2, dout = net->d_out;
  float* ws = g->ws;
  // dW3 = A2^T dE ; db3 = 1^T dE
  hipError_t e = grad_gemm(h2, dout, rows, acts->A2, dE16, g->dW3, g->db3, ws, st);
  // dH2 = (dE W3^T) * gelu'(H2)
  if (e == hipSuccess)
    e = qsvm::launch_gemm(0, 1, qsvm::EPI_GELU_BWD,
                          gemm(rows, h2, dout, dE16, dout, net->W3, dout, nullptr, g->dH2, h2, nullptr, acts->H2), st);
  // dW2 = A1^T dH2 ; db2 = 1^T dH2
  if (e == hipSuccess) e = grad_gemm(h1, h2, rows, acts->A1, g->dH2, g->dW2, g->db2, ws, st);
  // dH1 = (dH2 W2^T) * gelu'(H1)
  if (e == hipSuccess)
    e = qsvm::launch_gemm(0, 1, qsvm::EPI_GELU_BWD,
                          gemm(rows, h1, h2, g->dH2, h2, net->W2, h2, nullptr, g->dH1, h1, nullptr, acts->H1), st);
  // dW1 = X^T dH1 ; db1 = 1^T dH1
  if (e == hipSuccess) e = grad_gemm(din, h1, rows, X16, g->dH1, g->dW1, g->db1, ws, st);
  return api_hip(e, what);
}

int64_t qsvm_mlp_workspace_floats(const qsvm_mlp* net, int64_t rows) {
  if (check_net(net, "qsvm_mlp_workspace_floats") != QSVM_OK || check_rows(rows, "qsvm_mlp_workspace_floats") != QSVM_OK)
    return -1;
  return workspace_floats(net, rows);
}

qsvm_status qsvm_adamw(float* w, const float* grad, float* m, float* v, void* w16, int64_t count, float lr,
                       float beta1, float beta2, float eps, float weight_decay, int32_t step, void* stream) {
  QSVM_TRACE_RANGE("qsvm_adamw");
  const char* what = "qsvm_adamw";
  if (!w || !grad || !m || !v) return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_adamw: NULL pointer");
  if (count < 1 || step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps > 0.0f))
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_adamw: need count, step >= 1, lr >= 0, betas in [0, 1), eps > 0");
  if (qsvm::api_injected_failure()) return injected(what);
  qsvm::AdamArgs o{};
  o.lr = lr;
  o.beta1 = beta1;
  o.beta2 = beta2;
  o.eps = eps;
  o.weight_decay = weight_decay;
  o.bc1 = 1.0f - powf(beta1, float(step));
  o.bc2 = 1.0f - powf(beta2, float(step));
  return api_hip(qsvm::launch_adamw(w, grad, m, v, static_cast<uint16_t*>(w16), count, o, static_cast<hipStream_t>(stream)),
                 what);
}

qsvm_status qsvm_surrogate_gram(const void* E16, int64_t N, int64_t N_pad, int32_t d, const float* alpha_beta,
                                double* K, int64_t ldk, float* tile_max, void* stream) {
  const char* what = "qsvm_surrogate_gram";
  if (!E16 || !alpha_beta || !K || !tile_max) return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_surrogate_gram: NULL pointer");
  if (N < 1 || N_pad < N || N_pad % 64 || N_pad - N >= 64 || d < 32 || d % 32 || ldk < N)
    return api_fail(QSVM_ERR_INVALID_ARG,
                    "qsvm_surrogate_gram: need 1 <= N <= N_pad < N + 64, N_pad % 64 == 0, d % 32 == 0, ldk >= N");
  if (N_pad / 64 > 65535)  // launch grid: N_pad / 64 blocks across, half that down
    return api_fail(QSVM_ERR_UNSUPPORTED, "qsvm_surrogate_gram: N_pad above 64 * 65535");
  if (qsvm::api_injected_failure()) return injected(what);
  return api_hip(qsvm::launch_sigmoid_gram(static_cast<const uint16_t*>(E16), N_pad, d, alpha_beta, K, ldk, N, tile_max,
                                           static_cast<hipStream_t>(stream)),
                 what);
}

qsvm_status qsvm_surrogate_gram_log(const void* X16, int32_t d_in, const void* E16, int32_t d, int64_t N, int64_t N_pad,
                                    const float* head, double* K, int64_t ldk, float* tile_max, void* stream) {
  QSVM_TRACE_RANGE("qsvm_surrogate_gram_log");
  const char* what = "qsvm_surrogate_gram_log";
  if ((!X16 && d_in > 0) || !E16 || !head || !K || !tile_max)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_surrogate_gram_log: NULL pointer");
  if (N < 1 || N_pad < N || N_pad % 64 || N_pad - N >= 64 || d_in < 0 || d_in % 32 || d < 32 || d % 32 || ldk < N)
    return api_fail(QSVM_ERR_INVALID_ARG,
                    "qsvm_surrogate_gram_log: need 1 <= N <= N_pad < N + 64, N_pad % 64 == 0, d_in % 32 == 0, "
                    "d >= 32, d % 32 == 0, ldk >= N");
  if (N_pad > (int64_t(1) << 19))  // one block per 128 x 128 piece of the upper triangle, a 1-D grid
    return api_fail(QSVM_ERR_UNSUPPORTED, "qsvm_surrogate_gram_log: N_pad above 2^19");
  if (qsvm::api_injected_failure()) return injected(what);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  float* norms = nullptr;  // the rows' squared norms, stream-ordered workspace
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&norms), size_t(N_pad) * sizeof(float), st);
  if (e != hipSuccess) return api_hip(e, what);
  e = qsvm::launch_sat_log_gram(static_cast<const uint16_t*>(X16), d_in, static_cast<const uint16_t*>(E16), d, N_pad,
                                head, K, ldk, N, tile_max, norms, st);
  const hipError_t f = hipFreeAsync(norms, st);
  return api_hip(e != hipSuccess ? e : f, what);
}

qsvm_status qsvm_flag_pairs(const double* K, int64_t N, int64_t ldk, const int32_t* tiles, const int32_t* tile_count,
                            int64_t max_tiles, double cut, int32_t cap_per_tile, int32_t* pairs, int32_t* pair_count,
                            int64_t max_pairs, int32_t* dense_tiles, int32_t* dense_count, void* stream) {
  QSVM_TRACE_RANGE("qsvm_flag_pairs");
  const char* what = "qsvm_flag_pairs";
  if (!K || !tiles || !tile_count || !pairs || !pair_count || !dense_tiles || !dense_count)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_flag_pairs: NULL pointer");
  if (N < 1 || N > INT32_MAX || ldk < N)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_flag_pairs: need 1 <= N < 2^31 and ldk >= N");
  if (max_tiles < 0 || max_tiles > INT32_MAX || max_pairs < 0 || max_pairs > INT32_MAX)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_flag_pairs: max_tiles and max_pairs must lie in [0, 2^31)");
  if (cap_per_tile < 0 || cap_per_tile > 4096)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_flag_pairs: cap_per_tile outside [0, 4096]");
  if (max_tiles * int64_t(cap_per_tile) > INT32_MAX)
    return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_flag_pairs: max_tiles * cap_per_tile must stay below 2^31");
  if (qsvm::api_injected_failure()) return injected(what);
  return api_hip(qsvm::launch_flag_pairs(K, N, ldk, tiles, tile_count, max_tiles, cut, cap_per_tile, pairs, pair_count,
                                         max_pairs, dense_tiles, dense_count, static_cast<hipStream_t>(stream)),
                 what);
}

qsvm_status qsvm_flag_tiles(const float* tile_max, int32_t T, float tau, int32_t* tile_list, int32_t* count,
                            void* stream) {
  QSVM_TRACE_RANGE("qsvm_flag_tiles");
  const char* what = "qsvm_flag_tiles";
  if (!tile_max || !tile_list || !count) return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_flag_tiles: NULL pointer");
  if (T < 1 || T > 65536) return api_fail(QSVM_ERR_INVALID_ARG, "qsvm_flag_tiles: T outside [1, 65536]");
  if (qsvm::api_injected_failure()) return injected(what);
  return api_hip(qsvm::launch_flag_tiles(tile_max, T, tau, tile_list, count, static_cast<hipStream_t>(stream)), what);
}

}  // extern "C"
