/*
 * qsvm.h -- C ABI of libqsvm.so, an MI355X (gfx950) engine for quantum-kernel
 * Gram matrices computed by exact matrix-product-state (MPS) contraction.
 *
 * What is computed (paper §2, Eq. 3 and Eq. 4):
 *
 *     K[i][j] = |<psi(y_j)|psi(x_i)>|^2 ,   |psi(x)> = U(x)|0...0> ,
 *
 * for the ZZ feature map on a linear chain of n qubits: `reps` repetitions of
 * { H on every qubit; P(2 x_k) on qubit k; for k = 0..n-2 the block
 *   CNOT(k,k+1) P(theta_k)_{k+1} CNOT(k,k+1) }, theta_k = 2 (pi-x_k)(pi-x_{k+1}).
 * The paper encodes data with a parameterised circuit entangled by a linear
 * CNOT chain (§3.2) and obtains each entry as the all-zero amplitude of the
 * "U(x_i) then U(x_j)^dagger" circuit by tensor-network contraction with one
 * contraction order reused for every pair (§3.4.2, Alg. 2).  Here each data
 * point is first encoded once as an exact, untruncated MPS of bond dimension
 * chi = 2^reps (qsvm_encode_mps), and every entry is then the overlap of two
 * such MPS swept site by site (qsvm_gram, qsvm_gram_sym).  The symmetric call
 * computes the pairs i < j only and sets K[i][i] = 1 and K[j][i] = K[i][j],
 * the symmetrisation step of Alg. 1-3.  Alg. 1-3 store |amp|; this library
 * stores |amp|^2, the kernel of Eq. 3 (sqrt of an entry gives |amp|).
 *
 * Conventions shared by every call
 *   - All pointers named X, mps*, K, log_k are DEVICE pointers (memory from
 *     hipMalloc or a PyTorch CUDA tensor).  The caller owns every buffer; the
 *     library never keeps a pointer after a call returns and never frees one.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls only enqueue work and return without synchronising.
 *   - Arguments are validated on the host before any HIP call; on an error
 *     nothing is enqueued.  Errors inside a kernel cannot be detected by the
 *     call; they surface at the caller's next synchronisation.  Launch
 *     failures return QSVM_ERR_HIP.  qsvm_last_error() gives a message for
 *     the calling thread's most recent failure.
 *   - Supported: 1 <= n_qubits <= 65535, reps in {1, 2, 3} (chi = 2, 4, 8),
 *     1 <= N < 2^31.  Other reps return QSVM_ERR_UNSUPPORTED.
 *   - No call throws across the ABI.  Results are bitwise reproducible for the
 *     same inputs, arguments and device (no floating-point atomics).
 */
#ifndef QSVM_H
#define QSVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QSVM_OK = 0,
  QSVM_ERR_INVALID_ARG = -1, /* null pointer, non-positive size, ldk too small, bad option */
  QSVM_ERR_UNSUPPORTED = -2, /* valid request outside the supported range (e.g. reps > 3) */
  QSVM_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed */
  QSVM_ERR_SIZE = -4         /* a caller buffer is smaller than the call needs */
} qsvm_status;

/* Which sweep evaluates the overlaps.  Both compute the same MPS contraction
 * E <- sum_s B_s^dagger E A_s (the environment of <psi(y)|psi(x)>):
 *   DENSE      reads the dense site tensors and multiplies them as matrices;
 *   BUTTERFLY  reads the compact gauge generators of the same MPS (see the
 *              layout below) and applies each site tensor as a product of 2x2
 *              factors, 2-3x fewer operations.
 * AUTO currently selects BUTTERFLY. */
typedef enum {
  QSVM_SWEEP_AUTO = 0,
  QSVM_SWEEP_BUTTERFLY = 1,
  QSVM_SWEEP_DENSE = 2
} qsvm_sweep_kind;

/* Optional settings of qsvm_gram / qsvm_gram_sym.  Pass NULL for defaults;
 * a zero-initialised struct also means "defaults". */
typedef struct {
  int32_t renorm_every; /* sites between power-of-two renormalisations of the
                           environment (exact rescaling, exponent kept in an
                           integer log2 accumulator); 0 = default (4), else 1..16 */
  int32_t sweep;        /* qsvm_sweep_kind */
  int32_t diag_mode;    /* qsvm_gram_sym only: 0 = K[i][i] := 1 exactly (Alg. 1-3);
                           1 = compute the self-overlaps like any other pair */
  int32_t variant;      /* butterfly kernel variant: 0 = the tuned choice for this
                           reps and size (qsvm_autotune) or the built-in default;
                           1..4 = force variant 0..3 (ket points per lane and
                           register budget); the dense sweep ignores it */
  int64_t row_begin;    /* compute only rows i in [row_begin, row_end) of K;   */
  int64_t row_end;      /* 0,0 = all rows.  For qsvm_gram_sym a row i covers the
                           pairs (i, j > i) and writes K[i][j], K[j][i], and
                           K[i][i] by the diag_mode rule.  Lets a long Gram run
                           in resumable row blocks. */
  double* log_k;        /* optional device output: natural log of each entry,
                           same shape and ldk as K (-inf for an exact zero).
                           K itself underflows to 0 below ~1e-308; log_k does
                           not.  NULL = not written. */
} qsvm_gram_opts;

/*
 * Bytes of the MPS buffer that qsvm_encode_mps writes for N points of
 * n_qubits features: n*N*chi*chi*8 + n*N*16 with chi = 2^reps.  Returns 0 for
 * arguments outside the supported range.
 *
 * MPS buffer layout (site-major so that a sweep over site k reads the tensors
 * of consecutive points contiguously):
 *
 *  Section D, offset 0: dense site tensors, complex64 (re, im float pairs).
 *    Tensor of site k of point i, element [alpha][beta] at complex index
 *        ((k*N + i)*chi + alpha)*chi + beta .
 *    A_k[alpha][beta] = 2^(-reps/2) * sgn(beta)
 *                       * exp(i*(2 x_k |beta| + theta_{k-1} |alpha XOR beta|)),
 *    theta_{-1} = 0, |.| = number of set bits, and
 *    sgn(beta) = (-1)^(sum_{l=1}^{reps-1} beta_l beta_{l-1}) with beta_l the
 *    l-th bit of beta.  Bit l of a bond index is the value qubit k carries
 *    after repetition l+1; the physical index of A_k is s = bit (reps-1) of
 *    beta, so A_k^s[alpha][beta] = A_k[alpha][beta] if beta's top bit equals
 *    s and 0 otherwise.  The state is
 *        psi(s_0..s_{n-1}) = e_0^T A_0^{s_0} A_1^{s_1} ... A_{n-1}^{s_{n-1}} 1 ,
 *    with left boundary e_0 (row 0 of A_0) and right boundary all ones.
 *
 *  Section G, offset n*N*chi*chi*8: gauge generators, 4 floats per (k, i) at
 *    float4 index k*N + i.  With g_k = exp(i(2 x_k + theta_{k-1})):
 *      k >= 1: (a_k.re, a_k.im, b_k.re, b_k.im),
 *              a_k = exp(i theta_{k-1}) g_{k-1},  b_k = exp(-i theta_{k-1}) g_{k-1};
 *      k == 0: (g_{n-1}.re, g_{n-1}.im, 0, 0).
 *    In the diagonal gauge D_k = diag(1, g_k) per bond bit, every site tensor
 *    of Section D becomes 2^(-reps/2) * sgn(beta) * prod_l C_k[beta_l][alpha_l]
 *    with C_k = [[1, a_k], [1, b_k]] (row = new bit, column = old bit), the
 *    left boundary becomes sgn, and the right boundary becomes g_{n-1}^|beta|.
 */
size_t qsvm_mps_bytes(int64_t N, int32_t n_qubits, int32_t reps);

/*
 * Encode N feature vectors as exact MPS (the operand preparation of Alg. 2,
 * done once per point instead of once per pair).
 *   X          device, N x n_qubits float64, row-major (feature k of point i at
 *              X[i*n_qubits + k]); feature k drives qubit k.  Finite values
 *              expected (NaN/Inf propagate into the tensors).
 *   mps        device output buffer of at least qsvm_mps_bytes(N, n, reps)
 *              bytes, 16-byte aligned; layout above.
 *   mps_bytes  size of that buffer; smaller than needed -> QSVM_ERR_SIZE.
 * Phases are formed and reduced in FP64 and rounded once to FP32.
 */
qsvm_status qsvm_encode_mps(const double* X, int64_t N, int32_t n_qubits, int32_t reps,
                            void* mps, size_t mps_bytes, void* stream);

/*
 * Rectangular Gram: K[i*ldk + j] = |<psi(b_j)|psi(a_i)>|^2 for i < Na, j < Nb
 * (Alg. 2 over the index set of all (i, j); no symmetrisation, since the
 * "+ K^T + I" step is defined for square matrices only).
 *   mps_a, mps_b  device MPS buffers from qsvm_encode_mps with (Na, n, reps)
 *                 and (Nb, n, reps); may be the same buffer.
 *   K             device Na x Nb float64, row stride ldk >= Nb (elements).
 *   opts          NULL or settings above (diag_mode is ignored).
 * The environment is carried in FP32 with power-of-two renormalisation into
 * an integer log2 scale; the final modulus squared is formed in FP64.
 */
qsvm_status qsvm_gram(const void* mps_a, int64_t Na, const void* mps_b, int64_t Nb,
                      int32_t n_qubits, int32_t reps, double* K, int64_t ldk,
                      const qsvm_gram_opts* opts, void* stream);

/*
 * Symmetric Gram of one set (Alg. 1-3 with datasize1 = datasize2 = N): the
 * N(N-1)/2 pairs i < j are contracted; K[i*ldk + j] and K[j*ldk + i] both
 * receive the value, and K[i*ldk + i] = 1 (diag_mode 0) or the computed
 * self-overlap (diag_mode 1).
 *   mps  device MPS buffer from qsvm_encode_mps with (N, n, reps).
 *   K    device N x N float64, row stride ldk >= N.
 */
qsvm_status qsvm_gram_sym(const void* mps, int64_t N, int32_t n_qubits, int32_t reps,
                          double* K, int64_t ldk, const qsvm_gram_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * Batched jobs: many independent symmetric Grams in one persistent launch.
 * Every job is cut into the work items of the single-Gram sweep, the items of
 * all jobs are queued by decreasing cost (longest processing time first), and
 * one persistent kernel -- one block per resident slot of every compute unit
 * -- pops items with an atomic counter until the queue is empty (the
 * concurrent, host-free contraction stream of §4.1, batched over jobs).
 * ------------------------------------------------------------------------ */
typedef struct {
  const void* mps;   /* device MPS buffer of the job (qsvm_encode_mps with N, n_qubits, reps) */
  int64_t N;         /* points */
  int32_t n_qubits;
  int32_t reps;      /* 1..3; jobs may mix reps and sizes */
  double* K;         /* device N x N output, row stride ldk >= N; written as by qsvm_gram_sym */
  int64_t ldk;
  double* log_k;     /* optional device N x N output (same stride), or NULL */
} qsvm_job;

typedef struct {
  int32_t renorm_every; /* as in qsvm_gram_opts; 0 = default */
  int32_t diag_mode;    /* as in qsvm_gram_opts, for every job */
  int32_t use_graph;    /* 1: capture the launch (counter reset + persistent kernel)
                           into a hipGraph at plan creation and replay it */
  int32_t grid_blocks;  /* persistent blocks; 0 = compute units x resident blocks per unit */
} qsvm_batch_opts;

typedef struct qsvm_batch_plan qsvm_batch_plan; /* opaque */

/*
 * Build a plan for n_jobs jobs on the current device: validates every job
 * (errors name the job), orders the work queue, allocates and uploads the
 * job table and the queue counter (hipMalloc + a synchronous copy: call this
 * at set-up, not in a timed loop), and captures the graph if asked.  The
 * jobs' buffers must stay valid for every later launch.  *plan = NULL on error.
 */
qsvm_status qsvm_batch_plan_create(const qsvm_job* jobs, int32_t n_jobs, const qsvm_batch_opts* opts,
                                   qsvm_batch_plan** plan);

/* Enqueue one execution of the plan on `stream` (graph launch or the two
 * kernels).  Launches of one plan share its queue counter: keep them ordered
 * on one stream. */
qsvm_status qsvm_batch_plan_launch(qsvm_batch_plan* plan, void* stream);

/* Wait for the plan's last launch, then free it (NULL is a no-op). */
qsvm_status qsvm_batch_plan_destroy(qsvm_batch_plan* plan);

/* Work items in the queue, persistent grid size, and whether a graph is used. */
qsvm_status qsvm_batch_plan_info(const qsvm_batch_plan* plan, int64_t* total_items, int32_t* grid_blocks,
                                 int32_t* uses_graph);

/*
 * Autotune the butterfly sweep for (reps, n_qubits, N) on the current device:
 * every kernel variant (ket points per lane x register budget) is timed on a
 * synthetic symmetric Gram of that shape (features from a fixed hash, uniform
 * in [0, pi)), and the fastest is recorded in the per-process table that
 * launches with opts.variant == 0 consult, keyed by reps and floor(log2 n).
 * Allocates and frees its own device scratch (N x N doubles plus the MPS)
 * and synchronises `stream`; N <= 65536.
 *   best_variant  optional output: the chosen variant (0..3).
 *   variant_ms    optional output of n_variant_ms >= 4 floats: mean launch
 *                 time of each variant in milliseconds.
 */
qsvm_status qsvm_autotune(int32_t reps, int32_t n_qubits, int64_t N, void* stream, int32_t* best_variant,
                          float* variant_ms, int32_t n_variant_ms);

/* The variant (0..3) a launch with opts.variant == 0 uses for (reps, n_qubits). */
int32_t qsvm_get_tuned_variant(int32_t reps, int32_t n_qubits);

/* Record a variant for (reps, n_qubits) in the per-process table (e.g. from a
 * saved tuning cache).  No HIP call. */
qsvm_status qsvm_set_tuned_variant(int32_t reps, int32_t n_qubits, int32_t variant);

/* Static description of a status code (never NULL). */
const char* qsvm_status_string(qsvm_status s);

/* Message describing the calling thread's most recent non-OK status ("" if none). */
const char* qsvm_last_error(void);

/* ABI version of this header: 1. */
int32_t qsvm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QSVM_H */
