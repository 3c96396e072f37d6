// Launch interface of the surrogate kernels (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsvm {

enum GemmEpilogue {
  EPI_F32 = 0,           // C (float) = acc
  EPI_BIAS_GELU = 1,     // C (float) = acc + bias (pre-activation); C2 (bf16) = gelu(C)
  EPI_BIAS = 2,          // C (float) = acc + bias; C2 (bf16) = C
  EPI_GELU_BWD = 3,      // C2 (bf16) = acc * gelu'(aux)
  EPI_BIAS_GELU_BF16 = 4, // C2 (bf16) = gelu(acc + bias) only (inference: no pre-activation kept)
  EPI_BIAS_BF16 = 5,      // C2 (bf16) = acc + bias only
};

struct GemmArgs {
  int64_t M, N, K;    // multiples of 64, 64, 32
  const void* A;      // bf16
  int64_t lda;
  const void* B;      // bf16
  int64_t ldb;
  void* C;            // float
  void* C2;           // bf16 output of some epilogues
  int64_t ldc;        // row stride of C, C2 and aux
  const float* bias;  // [N]
  const float* aux;   // pre-activation for EPI_GELU_BWD
  int32_t splits;     // split-K factor (>= 1; > 1 only with EPI_F32: C holds `splits` slabs of M x ldc)
};

struct AdamArgs {
  float lr, beta1, beta2, eps, weight_decay;
  float bc1, bc2;  // 1 - beta1^t, 1 - beta2^t
};

hipError_t launch_gemm(int ta, int tb, int epi, const GemmArgs& g, hipStream_t s);
// K = sigmoid(ab[0] E E^T + ab[1]), diagonal 1, per-64x64-tile off-diagonal maxima.
hipError_t launch_sigmoid_gram(const uint16_t* E, int64_t N_pad, int32_t d, const float* ab, double* K, int64_t ldk,
                               int64_t valid, float* tile_max, hipStream_t s);
// Up to three bf16 transposes (out_q = in_q^T, in_q R_q x C_q row-major) in
// one launch; first_block is filled in by the launcher.
struct TransposeJobs {
  const uint16_t* in[3];
  uint16_t* out[3];
  int64_t R[3], C[3];
  int32_t first_block[4];
};
hipError_t launch_transpose_bf16(TransposeJobs j, int32_t count, hipStream_t s);
// out (Cp x R) = in (R x C)^T for two bf16 matrices with R rows (R % 8 ==
// 0, C and Cp multiples of 64, Cp >= C); output rows C .. Cp - 1: a row of
// ones, then zeros.
struct T64Job {
  const uint16_t* in;
  uint16_t* out;
  int64_t C, Cp;
};
hipError_t launch_transpose64_bf16(T64Job j0, T64Job j1, int64_t R, hipStream_t s);
hipError_t launch_gather(const double* X, int64_t N, int32_t n, const int32_t* idx, int64_t rows, int32_t d_pad,
                         uint16_t* out, hipStream_t s);
// sum over z < n_slabs, in order, of slabs[z * stride + t], t < count, into
// out[t] for t < split and out2[t - split] above.
hipError_t launch_sum_slabs(const float* slabs, int32_t n_slabs, int64_t count, int64_t stride, float* out,
                            int64_t split, float* out2, hipStream_t s);

hipError_t launch_pair_head(const float* E, int64_t P, int32_t d, const float* target, const float* ab,
                            int32_t loss_kind, uint16_t* dE16, float* partial, float* out3, hipStream_t s);
// Log-domain head: per pair loss and gradient (pair_head_log + the fixed-order
// reduction into out3 = (loss, d/d log c, d/d log s)); the whole Gram.
hipError_t launch_pair_head_log(const uint16_t* X16, int32_t d_in, const float* E, int32_t d, int64_t P,
                                const float* target, const float* head, float scale, uint16_t* dE16, float* partial,
                                float* out3, float* pred, hipStream_t s);
// (norms: N_pad floats of workspace, the rows' squared norms times -s log2(e))
hipError_t launch_sat_log_gram(const uint16_t* X16, int32_t d_in, const uint16_t* E, int32_t d, int64_t N_pad,
                               const float* head, double* K, int64_t ldk, int64_t valid, float* tile_max,
                               float* norms, hipStream_t s);
hipError_t launch_adamw(float* w, const float* grad, float* m, float* v, uint16_t* w16, int64_t count,
                        const AdamArgs& o, hipStream_t s);
// Pairs (i < j) of the listed tiles with K[i][j] >= cut: at most cap per tile
// into the pair list, the other tiles into the dense list (counts cleared
// here first).
hipError_t launch_flag_pairs(const double* K, int64_t N, int64_t ldk, const int32_t* tiles, const int32_t* tile_count,
                             int64_t max_tiles, double cut, int32_t cap, int32_t* pairs, int32_t* pair_count,
                             int64_t max_pairs, int32_t* dense, int32_t* dense_count, hipStream_t s);
hipError_t launch_flag_tiles(const float* tile_max, int32_t T, float tau, int32_t* list, int32_t* count,
                             hipStream_t s);

}  // namespace qsvm
