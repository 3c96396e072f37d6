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
 *   - Supported: 1 <= n_qubits <= 65535, reps in {1, ..., 6} (chi = 2 ..
 *     64), 1 <= N < 2^31.  Other reps return QSVM_ERR_UNSUPPORTED, as do the
 *     dense sweep at reps >= 4, dense tensors at reps >= 5, a device-resident
 *     tile count at reps >= 4 and a batch plan with a reps >= 4 job.  At
 *     reps >= 4 the butterfly sweep holds each pair's environment (128, 512
 *     or 2048 entries) in 2, 8 or 32 lanes, 64 entries per lane.
 *   - A Gram call issues its tiles as one or more kernel launches of whole
 *     rows of 64 x 64 tiles (a dispatch holds at most 2^24 - 8 blocks of 256
 *     threads), so one row of tiles must fit one launch: Nb <= 64 *
 *     floor((2^24 - 8) / b) with b = 16 blocks per tile (32, 128 and 512 for
 *     reps 4, 5 and 6, 1 for the state-vector Gram), i.e. Nb below about
 *     2^26 (2^25, 2^23, 2^21; 2^30).  Larger Nb is QSVM_ERR_UNSUPPORTED.
 *   - Tracing: with QSVM_ROCTX=1 in the environment, every entry point that
 *     enqueues work pushes a roctx range named after itself for the host side
 *     of the call (`rocprofv3 --marker-trace`); the marker library is opened
 *     at run time, so nothing links against it.
 *   - Precision: the sweep carries the environment in FP32 with an exact
 *     power-of-two log scale and forms |amp|^2 in FP64; every entry above
 *     an n-dependent threshold is then recomputed with an FP64 environment
 *     (qsvm_gram_opts.refine_above), so entries left in FP32 stay within
 *     ~5e-6 of the exact kernel and refined ones within ~1e-12.
 *   - No call throws across the ABI.  Results are bitwise reproducible for the
 *     same inputs, arguments and device (no floating-point atomics; the
 *     integer atomics that collect tile lists only order independent work).
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
  QSVM_ERR_UNSUPPORTED = -2, /* valid request outside the supported range (e.g. reps > 6) */
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
                           integer log2 accumulator); 0 = default (8), else 1..16 */
  int32_t sweep;        /* qsvm_sweep_kind */
  int32_t diag_mode;    /* qsvm_gram_sym only: 0 = K[i][i] := 1 exactly (Alg. 1-3);
                           1 = compute the self-overlaps like any other pair */
  int32_t variant;      /* butterfly kernel variant: 0 = the tuned choice for this
                           reps and size (qsvm_autotune) or the built-in default;
                           1..4 = force variant 0..3 (ket points per lane and
                           register budget; all agree bitwise); the dense
                           sweep ignores it */
  int64_t row_begin;    /* compute only rows i in [row_begin, row_end) of K;   */
  int64_t row_end;      /* 0,0 = all rows.  For qsvm_gram_sym a row i covers the
                           pairs (i, j > i) and writes K[i][j], K[j][i], and
                           K[i][i] by the diag_mode rule.  Lets a long Gram run
                           in resumable row blocks. */
  double* log_k;        /* optional device output: natural log of each entry,
                           same shape and ldk as K (-inf for an exact zero).
                           K itself underflows to 0 below ~1e-308; log_k does
                           not.  NULL = not written. */
  double refine_above;  /* FP64 refinement: after the FP32 sweep, every
                           computed entry above this value is recomputed with
                           an FP64 environment from FP64 generators (Sections
                           G + L): the 64 x 64 tiles whose largest entry
                           exceeds it are listed, and within them the waves
                           holding such an entry recompute it.  The FP32
                           sweep alone leaves up to ~1.3e-5 at 784 qubits for
                           K near 1 (measured bound 4e-6 + 2e-8 n at K = 1,
                           ~sqrt(K) times that below).  0 = automatic:
                           (5e-6 / (4e-6 + 2e-8 n))^2, so every entry left in
                           FP32 stays within 5e-6 (0.064 at 784 qubits; no
                           refinement and no scan at n <= 50); > 0 = that
                           threshold; negative = off.  Costs one read of the
                           written K plus the FP64 sweep of the listed tiles;
                           a 4-byte-per-tile list lives in a stream-ordered
                           temporary.  The state-vector Grams (FP64
                           throughout) ignore it. */
  const void* dense_a;  /* QSVM_SWEEP_DENSE only (required there, ignored
                           otherwise): the dense tensors (qsvm_encode_dense)
                           of the first set (mps_a, or the set of a symmetric
                           call) ... */
  const void* dense_b;  /* ... and of the second set of qsvm_gram (NULL =
                           dense_a, for mps_b == mps_a) */
} qsvm_gram_opts;

/*
 * Bytes of the MPS buffer that qsvm_encode_mps writes for N points of
 * n_qubits features: n*N*32 (Sections G and L, 16 bytes each per site and
 * point, whatever reps).  Returns 0 for arguments outside the supported range.
 *
 * MPS buffer layout (site-major so that a sweep over site k reads the data of
 * consecutive points contiguously).  With chi = 2^reps, the MPS of a point is
 *    psi(s_0..s_{n-1}) = e_0^T A_0^{s_0} A_1^{s_1} ... A_{n-1}^{s_{n-1}} 1 ,
 *    A_k[alpha][beta] = 2^(-reps/2) * sgn(beta)
 *                       * exp(i*(2 x_k |beta| + theta_{k-1} |alpha XOR beta|)),
 * theta_{-1} = 0, |.| = number of set bits, sgn(beta) =
 * (-1)^(sum_{l=1}^{reps-1} beta_l beta_{l-1}) with beta_l the l-th bit of
 * beta; bit l of a bond index is the value qubit k carries after repetition
 * l+1, the physical index of A_k is s = bit (reps-1) of beta
 * (A_k^s[alpha][beta] = A_k[alpha][beta] if beta's top bit equals s, else 0),
 * the left boundary is e_0 (row 0 of A_0) and the right boundary all ones.
 * The buffer holds this MPS in a diagonal gauge, compactly:
 *
 *  Section G, offset 0: gauge generators, 4 floats per (k, i) at float4 index
 *    k*N + i.  With g_k = exp(i(2 x_k + theta_{k-1})):
 *      k >= 1: (a_k.re, a_k.im, b_k.re, b_k.im),
 *              a_k = exp(i theta_{k-1}) g_{k-1},  b_k = exp(-i theta_{k-1}) g_{k-1};
 *      k == 0: (g_{n-1}.re, g_{n-1}.im, 0, 0).
 *    In the diagonal gauge D_k = diag(1, g_k) per bond bit, every site tensor
 *    A_k becomes 2^(-reps/2) * sgn(beta) * prod_l C_k[beta_l][alpha_l]
 *    with C_k = [[1, a_k], [1, b_k]] (row = new bit, column = old bit), the
 *    left boundary becomes sgn, and the right boundary becomes g_{n-1}^|beta|.
 *
 *  Section L, offset n*N*16: the FP32 residuals of Section G, same layout:
 *    each component is (float)(value - (double)G component), so G + L is the
 *    FP64 generator to ~2^-48 relative.  Read only by the FP64 refinement
 *    (qsvm_gram_opts.refine_above).
 *
 * The dense tensors A_k themselves are not part of the MPS buffer: only the
 * dense sweep (QSVM_SWEEP_DENSE, a cross-check that assumes nothing about
 * the tensors) reads them, from a separate buffer written by
 * qsvm_encode_dense and passed in qsvm_gram_opts.dense_a / dense_b.
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
 * Phases are formed and reduced in FP64 and rounded once to FP32 (Section G);
 * Section L keeps the rounding residual of each generator.
 */
qsvm_status qsvm_encode_mps(const double* X, int64_t N, int32_t n_qubits, int32_t reps,
                            void* mps, size_t mps_bytes, void* stream);

/*
 * Bytes of the dense site tensors of N points: n*N*chi*chi*8 (complex64).
 * 0 for arguments outside the supported range (dense tensors: reps <= 4).
 */
size_t qsvm_dense_bytes(int64_t N, int32_t n_qubits, int32_t reps);

/*
 * Write the dense site tensors A_k of the MPS above (complex64, re/im float
 * pairs), tensor of site k of point i, element [alpha][beta] at complex index
 * ((k*N + i)*chi + alpha)*chi + beta.  Only the dense sweep reads them.
 *   dense        device output of at least qsvm_dense_bytes(N, n, reps) bytes,
 *                16-byte aligned; dense_bytes its size (smaller -> QSVM_ERR_SIZE).
 * Other arguments as qsvm_encode_mps; each entry's phase is formed in FP64 and
 * rounded once to FP32.
 */
qsvm_status qsvm_encode_dense(const double* X, int64_t N, int32_t n_qubits, int32_t reps,
                              void* dense, size_t dense_bytes, void* stream);

/* The threshold qsvm_gram_opts.refine_above = 0 selects for n_qubits:
 * (5e-6 / (4e-6 + 2e-8 n))^2; a value >= 1 means no entry needs refining and
 * the Gram calls skip the refinement (n <= 50).  0 for n_qubits < 1.  No HIP
 * call. */
double qsvm_auto_refine_threshold(int32_t n_qubits);

/*
 * Rectangular Gram: K[i*ldk + j] = |<psi(b_j)|psi(a_i)>|^2 for i < Na, j < Nb
 * (Alg. 2 over the index set of all (i, j); no symmetrisation, since the
 * "+ K^T + I" step is defined for square matrices only).
 *   mps_a, mps_b  device MPS buffers from qsvm_encode_mps with (Na, n, reps)
 *                 and (Nb, n, reps); may be the same buffer.
 *   K             device Na x Nb float64, row stride ldk >= Nb (elements).
 *   opts          NULL or settings above (diag_mode is ignored).
 * The environment is carried in FP32 with power-of-two renormalisation into
 * an integer log2 scale; the final modulus squared is formed in FP64, and
 * large entries are recomputed in FP64 (opts->refine_above).
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

/*
 * qsvm_gram_sym for callers that cannot allocate device memory: work recorded
 * under stream capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results (bit for bit) as qsvm_gram_sym; no
 * hipMalloc, hipFree or other allocating call is made.  The FP64
 * refinement's tile list, a stream-ordered temporary in qsvm_gram_sym, is
 * kept instead in a static device array of QSVM_NOALLOC_SCRATCH_ENTRIES
 * uint32 entries (4 MiB, one per device, held until the process ends): one
 * entry for the count plus one per 64 x 64 tile of the call (at most 2^24 - 8
 * per launch chunk).  Calls whose refinement would need more -- more than
 * 1,048,575 tiles in the row range, e.g. N above about 92,600 for a full
 * symmetric Gram -- return QSVM_ERR_SIZE before anything is enqueued; calls
 * with the refinement off (opts->refine_above < 0, or n_qubits <= 50 with the
 * automatic threshold) do not touch the array and have no such limit.  Every
 * call on one device shares that device's array, and each call resets the
 * count it uses on the device before listing tiles: calls that overlap on one
 * device (different streams, or host threads) race and must be ordered by the
 * caller.
 */
#define QSVM_NOALLOC_SCRATCH_ENTRIES (1 << 20)
qsvm_status qsvm_gram_sym_noalloc(const void* mps, int64_t N, int32_t n_qubits, int32_t reps,
                                  double* K, int64_t ldk, const qsvm_gram_opts* opts, void* stream);

/*
 * Symmetric Gram restricted to a list of 64 x 64 tiles: for every (ti, tj) in
 * `tiles` (device int32 pairs, 0 <= ti <= tj < ceil(N/64)) the pairs
 * i < j with i in tile row ti and j in tile column tj are contracted and
 * written to K[i][j] and K[j][i], and diagonal tiles apply the diag_mode rule
 * -- exactly what qsvm_gram_sym writes for those tiles, bit for bit.  List
 * entries outside that range are skipped on the device.  Used as the exact
 * fallback of the surrogate.  opts row ranges must be 0,0.
 */
qsvm_status qsvm_gram_sym_tiles(const void* mps, int64_t N, int32_t n_qubits, int32_t reps, const int32_t* tiles,
                                int64_t n_tiles, double* K, int64_t ldk, const qsvm_gram_opts* opts, void* stream);

/*
 * qsvm_gram_sym_tiles with the list length in device memory: the number of
 * listed tiles is *tile_count (device int32, e.g. written by qsvm_flag_tiles
 * earlier on the same stream), read by the kernels when they run and clamped
 * to [0, max_tiles]; `tiles` holds room for max_tiles pairs.  The host never
 * reads the count, so a flag-then-recompute sequence (the surrogate's exact
 * fallback) needs no synchronisation between its steps.  Results equal qsvm_gram_sym_tiles over the
 * first *tile_count entries, bit for bit.  Butterfly sweep only (reps 1..3;
 * otherwise QSVM_ERR_UNSUPPORTED), max_tiles <= 2^24 - 8 (QSVM_ERR_UNSUPPORTED
 * above).  One persistent launch of the resident blocks strides over the
 * listed tiles (one fixed kernel variant per reps: opts->variant is
 * accepted and ignored), followed by the refinement of opts->refine_above.
 */
qsvm_status qsvm_gram_sym_tiles_dev(const void* mps, int64_t N, int32_t n_qubits, int32_t reps, const int32_t* tiles,
                                    const int32_t* tile_count, int64_t max_tiles, double* K, int64_t ldk,
                                    const qsvm_gram_opts* opts, void* stream);

/*
 * Exact entries of a symmetric Gram for a list of pairs: for each of the
 * first *pair_count (device int32, clamped to [0, max_pairs]) entries (i, j)
 * of `pairs` (device int32 pairs; (j, i) is taken as (i, j); entries with an
 * index outside [0, N) are skipped) K[i][j] and K[j][i] (and log K with
 * opts->log_k) are written with an FP64 environment from FP64 generators
 * (Sections G + L): the value the refinement (opts.refine_above) writes for
 * that entry, bit for bit.  i == j follows opts->diag_mode.  One pair per
 * group of 2 lanes (reps 1), 4 lanes (reps 2, 3) or per wave (reps >= 4),
 * the list's chunks spread over the blocks; the host never reads the count.  The exact fallback of the surrogate for
 * flagged pairs (qsvm_flag_pairs).  opts row ranges must be 0,0; sweep,
 * variant and refine_above are ignored.
 */
qsvm_status qsvm_gram_sym_pairs_dev(const void* mps, int64_t N, int32_t n_qubits, int32_t reps, const int32_t* pairs,
                                    const int32_t* pair_count, int64_t max_pairs, double* K, int64_t ldk,
                                    const qsvm_gram_opts* opts, void* stream);

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
  int32_t reps;      /* 1..3 (reps >= 4 is QSVM_ERR_UNSUPPORTED here: use
                        qsvm_gram / qsvm_gram_sym); jobs may mix reps and sizes */
  double* K;         /* device N x N output, row stride ldk >= N; written as by qsvm_gram_sym */
  int64_t ldk;
  double* log_k;     /* optional device N x N output (same stride), or NULL */
} qsvm_job;

typedef struct {
  int32_t renorm_every; /* as in qsvm_gram_opts; 0 = default */
  int32_t diag_mode;    /* as in qsvm_gram_opts, for every job */
  int32_t use_graph;    /* 1: capture the launch (counter reset + persistent kernel
                           + each job's refinement launches) into a hipGraph at
                           plan creation and replay it */
  int32_t grid_blocks;  /* persistent blocks, at most 2^24 - 8; 0 = compute units x resident blocks
                           per unit */
  double refine_above;  /* as in qsvm_gram_opts: after the persistent sweep, each
                           job's tiles with an entry above it are recomputed in
                           FP64 (0 = automatic per job from its n_qubits,
                           negative = off); the plan holds the list buffer */
  int32_t item_pi2;     /* work-item shape: ket points per lane of the reps = 2
                           items (2 or 4; 0 = from the tuned variant of the
                           plan's costliest reps = 2 job, see qsvm_autotune) */
  int32_t item_pi3;     /* the same for reps = 3 items (0 or 1: the persistent
                           kernel's register budget holds one reps = 3
                           environment per lane); reps = 1 items use 4.
                           Results do not depend on the shape. */
} qsvm_batch_opts;

typedef struct qsvm_batch_plan qsvm_batch_plan; /* opaque */

/*
 * Build a plan for n_jobs jobs on the current device: validates every job
 * (errors name the job), orders the work queue, allocates and uploads the
 * job table, the queue counter and the refinement's tile list (hipMalloc + a
 * synchronous copy: call this at set-up, not in a timed loop), and captures
 * the graph if asked.  The
 * jobs' buffers must stay valid for every later launch.  *plan = NULL on error.
 */
qsvm_status qsvm_batch_plan_create(const qsvm_job* jobs, int32_t n_jobs, const qsvm_batch_opts* opts,
                                   qsvm_batch_plan** plan);

/* Enqueue one execution of the plan on `stream` (graph launch, or the
 * counter reset, the persistent kernel and each job's refinement launches).
 * Launches of one plan share its queue counter and tile list: keep them
 * ordered on one stream. */
qsvm_status qsvm_batch_plan_launch(qsvm_batch_plan* plan, void* stream);

/* Wait for the plan's last launch, then free it (NULL is a no-op). */
qsvm_status qsvm_batch_plan_destroy(qsvm_batch_plan* plan);

/* Work items in the queue, persistent grid size, and whether a graph is used. */
qsvm_status qsvm_batch_plan_info(const qsvm_batch_plan* plan, int64_t* total_items, int32_t* grid_blocks,
                                 int32_t* uses_graph);

/* The plan's work-item shape: ket points per lane of its reps = 2 and reps = 3 items. */
qsvm_status qsvm_batch_plan_shape(const qsvm_batch_plan* plan, int32_t* item_pi2, int32_t* item_pi3);

/*
 * Autotune the butterfly sweep for (reps, n_qubits, N) on the current device:
 * every kernel variant (ket points per lane x register budget) is timed on a
 * synthetic symmetric Gram of that shape (features from a fixed hash, uniform
 * in [0, pi)), and the fastest is recorded in the table that Gram calls with
 * opts.variant == 0 and batch plans (their work-item shape) consult, keyed by
 * (GPU architecture, reps, floor(log2 n), floor(log2 N)).  The table is persisted: entries
 * are merged into a text cache file (qsvm_autotune_cache_path: the file named
 * by $QSVM_TUNE_CACHE, an empty value meaning no file, else
 * $XDG_CACHE_HOME/qsvm/autotune.txt or $HOME/.cache/qsvm/autotune.txt),
 * which a process reads on its first lookup for an architecture; a cache
 * that cannot be written leaves the in-process table in effect.
 * Allocates and frees its own device scratch (N x N doubles plus the MPS)
 * and synchronises `stream`; N <= 65536.
 *   best_variant  optional output: the chosen variant (0..3).
 *   variant_ms    optional output of n_variant_ms >= 4 floats: mean launch
 *                 time of each variant in milliseconds.
 */
qsvm_status qsvm_autotune(int32_t reps, int32_t n_qubits, int64_t N, void* stream, int32_t* best_variant,
                          float* variant_ms, int32_t n_variant_ms);

/* The variant (0..3) a launch with opts.variant == 0 uses for (reps, n_qubits)
 * on N points (a symmetric Gram of N points, or a rectangular Gram whose
 * pair count Na Nb equals N^2 / 2): the entry of the bucket
 * (floor(log2 n_qubits), floor(log2 N)), else 0 (the built-in default; a
 * variant tuned for another point count is not carried over). */
int32_t qsvm_get_tuned_variant(int32_t reps, int32_t n_qubits, int64_t N);

/* Record a variant for (reps, n_qubits, N) in the table of the current device's
 * architecture (in this process; qsvm_autotune_save writes it to the cache).
 * Queries the device's architecture; enqueues nothing. */
qsvm_status qsvm_set_tuned_variant(int32_t reps, int32_t n_qubits, int64_t N, int32_t variant);

/* Merge the table into the cache file now (the autotuner does so itself);
 * QSVM_ERR_INVALID_ARG with a message when the file cannot be written. */
qsvm_status qsvm_autotune_save(void);

/* The cache file in use ("" = persistence off).  The pointer stays valid until
 * the next call from the same thread. */
const char* qsvm_autotune_cache_path(void);

/* ------------------------------------------------------------------------
 * State-vector engine (the state-vector simulation method of §3.4.1 / Alg. 1,
 * rebuilt for whole Grams): every point's full 2^n-amplitude state is formed
 * once in FP64, and K = |Psi_a Psi_b^H|^2 is one dense complex product on the
 * FP64 matrix cores.  A second exact engine beside the MPS path, for
 * n_qubits <= 30 (memory 2^n * 16 B per point); its cost grows as 2^n where
 * the MPS path grows as n.
 * Layout: point i's state is 2^n complex128 values (re, im interleaved) at
 * element offset i * 2^n; amplitude b is the basis state whose bit k is
 * qubit k.
 * ------------------------------------------------------------------------ */

/* Bytes of the states of N points: N * 2^n * 16, or 0 when n_qubits is outside
 * 1..30, N < 1 or the size overflows int64. */
size_t qsvm_sv_bytes(int64_t N, int32_t n_qubits);

/*
 * Build psi(x_i) = U(x_i)|0^n> for the N rows of X (device N x n float64,
 * row-major): `reps` repetitions of H on every qubit followed by the
 * diagonal phase exp(i [sum_k 2 x_k b_k + sum_k theta_k (b_k XOR b_{k+1})]),
 * theta_k = 2 (pi - x_k)(pi - x_{k+1}) (the circuit of §3.2 read as the ZZ
 * map; the CNOT-P-CNOT block is that diagonal phase).  reps in 1..16.
 *   sv        device output of at least qsvm_sv_bytes(N, n) bytes, 16-byte
 *             aligned, caller-owned.
 * The phase factors come from per-point tables of 2^L + 2^(n-L+1) complex128
 * values, L = min(n, 11) (2^n + 2 values up to 11 qubits; beyond that
 * 2^11 + 2^(n-10), about 2^-9 of the states from 20 qubits on), held in a
 * stream-ordered temporary (hipMallocAsync / hipFreeAsync on `stream`).
 * QSVM_ERR_UNSUPPORTED for n_qubits outside 1..30; QSVM_ERR_SIZE for a short
 * buffer; QSVM_ERR_INVALID_ARG for other bad arguments; QSVM_ERR_HIP if the
 * temporary cannot be allocated.
 */
qsvm_status qsvm_encode_sv(const double* X, int64_t N, int32_t n_qubits, int32_t reps, void* sv,
                           size_t sv_bytes, void* stream);

/*
 * Rectangular Gram from states (Eq. 3 with the amplitudes of Alg. 1):
 * K[i*ldk + j] = |<psi(b_j)|psi(a_i)>|^2 for i < Na, j < Nb.  opts: NULL or
 * qsvm_gram_opts, of which log_k and row_begin/row_end are used (the MPS
 * sweep settings are validated and ignored).  K is FP64 and computed from
 * FP64 states with FP64 accumulation.
 */
qsvm_status qsvm_sv_gram(const void* sv_a, int64_t Na, const void* sv_b, int64_t Nb, int32_t n_qubits,
                         double* K, int64_t ldk, const qsvm_gram_opts* opts, void* stream);

/* Symmetric Gram from states: pairs i < j contracted and mirrored, the diagonal
 * by diag_mode as in qsvm_gram_sym.
 * Both Gram calls split the 2^n inner dimension across blocks when that fills
 * the device's resident blocks better (the split count depends on the tile
 * count, n and the device's compute units; at most 4096 partial tiles); the
 * partial products (tiles x splits x 64 KB, at most 256 MB) live in a
 * stream-ordered temporary (hipMallocAsync / hipFreeAsync on `stream`) and
 * are added in a fixed order, so results are reproducible on one device. */
qsvm_status qsvm_sv_gram_sym(const void* sv, int64_t N, int32_t n_qubits, double* K, int64_t ldk,
                             const qsvm_gram_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * Learned surrogate: an MLP embedding f: R^n -> R^d_out (layers
 * d_in -> d_h1 -> d_h2 -> d_out, GELU after the two hidden layers, BF16
 * weights and activations, FP32 accumulation on the matrix cores) with
 * K_hat(x, y) = sigmoid(alpha <f(x), f(y)> + beta), trained on exact kernel
 * entries; tiles where K_hat could exceed a threshold fall back to the exact
 * sweep (qsvm_gram_sym_tiles).  All widths and row counts are multiples of
 * 64 (pad features with zeros up to d_in; pad rows with zero rows).
 * Matrices are row-major; bf16 buffers are passed as void*.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t d_in, d_h1, d_h2, d_out;
  const void* W1; const float* b1; /* W1: d_in x d_h1 (bf16), b1: d_h1 (f32); layer: x W1 + b1 */
  const void* W2; const float* b2; /* W2: d_h1 x d_h2 */
  const void* W3; const float* b3; /* W3: d_h2 x d_out */
} qsvm_mlp;

typedef struct {   /* activations of `rows` inputs */
  float* H1; void* A1; /* rows x d_h1: pre-activation (f32), GELU output (bf16) */
  float* H2; void* A2; /* rows x d_h2 */
  float* E;  void* E16; /* rows x d_out embedding, f32 and bf16 */
} qsvm_mlp_acts;      /* H1, H2 and E may be NULL together (inference: only the
                         bf16 outputs are written, which the backward pass
                         cannot use) */

typedef struct {   /* gradients (f32, shaped like the parameters) and scratch */
  float* dW1; float* db1; float* dW2; float* db2; float* dW3; float* db3;
  void* dH1; void* dH2; /* bf16, rows x d_h1 and rows x d_h2 */
  float* ws;            /* f32 workspace of ws_floats >= qsvm_mlp_workspace_floats(net, rows):
                           k-contiguous copies of each weight gradient's operands
                           and its split-K partial products (weights and biases
                           in one product), reduced in a fixed order */
  int64_t ws_floats;
} qsvm_mlp_grads;

/* Workspace (floats) qsvm_mlp_backward needs for `rows` inputs; -1 for an
 * invalid network or row count.  No HIP call. */
int64_t qsvm_mlp_workspace_floats(const qsvm_mlp* net, int64_t rows);

/* out[r][c] = bf16(X[idx[r]][c]) for c < n_qubits; 0 for n_qubits <= c < d_pad
 * and for rows whose idx[r] is outside [0, N) (padding rows; checked on the
 * device).  X: N x n_qubits float64; idx: rows int32; out: rows x d_pad. */
qsvm_status qsvm_gather_features(const double* X, int64_t N, int32_t n_qubits, const int32_t* idx, int64_t rows,
                                 int32_t d_pad, void* out, void* stream);

/* Forward pass of `rows` inputs X16 (rows x d_in bf16) into acts.  The
 * weights are first copied transposed into a stream-ordered temporary
 * (hipMallocAsync / hipFreeAsync on `stream`, 2 (d_in d_h1 + d_h1 d_h2 +
 * d_h2 d_out) bytes) that the GEMMs read k-contiguously; the result does not
 * depend on it.  A layer with at least 256 output tiles of 256 x 256 runs on
 * a kernel that takes 128 KB of LDS per block: the first such launch on a
 * device raises that kernel's dynamic LDS limit (hipFuncSetAttribute, a
 * host call made once per device and epilogue), so under stream capture
 * make one uncaptured call of the same shape first; a failure of that call
 * is returned as QSVM_ERR_HIP. */
qsvm_status qsvm_mlp_forward(const qsvm_mlp* net, const void* X16, int64_t rows, const qsvm_mlp_acts* acts,
                             void* stream);

/* Pair head over E (2*pairs x d, f32): rows p and pairs + p are the two points
 * of pair p with exact kernel target[p].  K_hat = sigmoid(ab[0] <e, e'> + ab[1]);
 * loss_kind 0: loss = mean (K_hat - target)^2; 1: loss = mean soft-target
 * cross-entropy -t log K_hat - (1 - t) log(1 - K_hat) (its logit gradient
 * K_hat - t does not vanish for tiny kernels).  Writes dE16 (2*pairs x d,
 * bf16 gradient of the loss w.r.t. E), per-pair partials (3*pairs floats) and
 * out3 = (loss, dloss/dalpha, dloss/dbeta), reduced in a fixed order. */
qsvm_status qsvm_pair_head(const float* E, int64_t pairs, int32_t d, const float* target, const float* alpha_beta,
                           int32_t loss_kind, void* dE16, float* partial, float* out3, void* stream);

/* Log-domain pair head on the embedding z = [x, f(x)]: rows p and pairs + p of
 * X16 (2*pairs x d_in bf16, the gathered inputs; d_in may be 0, X16 then
 * may be NULL) and of E
 * (2*pairs x d f32, the MLP output) are the two points of pair p, and
 *   d2_p = ||z_p - z_{pairs+p}||^2,
 *   ln K_hat_p = -c (1 - exp(-s d2_p)),  c = exp(head[0]), s = exp(head[1]),
 * a kernel estimate that is exactly 1 for identical points, -c s d2 for
 * close ones and saturates at e^-c for unrelated ones (the concentration of
 * kernel values at many qubits, §4.2.1).  loss = mean_p ((ln K_hat_p - t_p) /
 * scale)^2 against the exact ln K (target[p], e.g. from qsvm_gram_opts.log_k).
 * Writes dE16 (2*pairs x d bf16, d loss / d E; the input part has no
 * parameters), per-pair partials (3*pairs floats) and out3 = (loss,
 * d loss / d head[0], d loss / d head[1]) reduced in a fixed order; pred
 * (optional, 2*pairs floats) receives (ln K_hat_p, d2_p). */
qsvm_status qsvm_pair_head_log(const void* X16, int32_t d_in, const float* E, int32_t d, int64_t pairs,
                               const float* target, const float* head, float scale, void* dE16, float* partial,
                               float* out3, float* pred, void* stream);

/* Backward pass given dE16 (rows x d_out bf16): parameter gradients into grads
 * (overwritten, not accumulated).  Each layer's weight and bias gradients are
 * one product [A, 1]^T dH (K = rows) on k-contiguous copies of the operands in
 * grads->ws, split along the rows into partial products summed in a fixed
 * order; a too-small workspace returns QSVM_ERR_SIZE. */
qsvm_status qsvm_mlp_backward(const qsvm_mlp* net, const void* X16, const qsvm_mlp_acts* acts, const void* dE16,
                              int64_t rows, const qsvm_mlp_grads* grads, void* stream);

/* AdamW step (decoupled weight decay, bias-corrected moments) on f32 master
 * weights w with moments m, v; step counts from 1; writes a bf16 copy to w16
 * when it is not NULL. */
qsvm_status qsvm_adamw(float* w, const float* grad, float* m, float* v, void* w16, int64_t count, float lr,
                       float beta1, float beta2, float eps, float weight_decay, int32_t step, void* stream);

/* Surrogate Gram: K[i][j] = sigmoid(ab[0] <e_i, e_j> + ab[1]) for i, j < N,
 * K[i][i] = 1 (the diagonal rule of Alg. 1-3), from E16 (N_pad x d bf16,
 * N_pad = N rounded up to 64, padding rows anything).  tile_max receives, per
 * 64 x 64 tile (row-major, (N_pad/64)^2 floats), the largest off-diagonal
 * K_hat (-inf for none). */
qsvm_status qsvm_surrogate_gram(const void* E16, int64_t N, int64_t N_pad, int32_t d, const float* alpha_beta,
                                double* K, int64_t ldk, float* tile_max, void* stream);

/* Log-domain surrogate Gram: K[i][j] = exp(ln K_hat(z_i, z_j)) with the head
 * of qsvm_pair_head_log on z = [X16 row, E16 row] (N_pad rows each, N_pad = N
 * rounded up to 64; d_in % 32 == 0 (0: no input part, X16 may be NULL),
 * d % 32 == 0), K[i][i] = 1, K row stride
 * ldk >= N.  The squared distances come from the BF16 inner products
 * (FP32 accumulation on the matrix cores) and the rows' squared norms;
 * ln K_hat is formed in FP32 once per pair (K is exactly symmetric).
 * tile_max receives per 64 x 64 tile ((N_pad/64)^2 floats, row-major) the
 * largest off-diagonal ln K_hat (-inf for none), for qsvm_flag_tiles with a
 * threshold in the log domain.  N_pad <= 2^19; N_pad floats of workspace are
 * taken stream-ordered (hipMallocAsync / hipFreeAsync on `stream`). */
qsvm_status qsvm_surrogate_gram_log(const void* X16, int32_t d_in, const void* E16, int32_t d, int64_t N, int64_t N_pad,
                                    const float* head, double* K, int64_t ldk, float* tile_max, void* stream);

/* Append every upper-triangular tile (ti <= tj) of a T x T tile_max array whose
 * value is >= tau to tile_list (int32 pairs, room for T(T+1)/2) and its count
 * to *count (device int32; cleared first).  The order of the list is not
 * specified. */
qsvm_status qsvm_flag_tiles(const float* tile_max, int32_t T, float tau, int32_t* tile_list, int32_t* count,
                            void* stream);

/* The pairs of flagged tiles that need the exact fallback (the surrogate's
 * fallback per pair; every buffer is the caller's).  For each of the first *tile_count (device int32,
 * clamped to [0, max_tiles]) entries (ti, tj) of `tiles` (as from
 * qsvm_flag_tiles), the pairs i < j of that tile with K[i][j] >= cut (K: the
 * N x N surrogate Gram, row stride ldk) are appended to `pairs` (int32
 * (i, j), room for max_pairs) when there are at most cap_per_tile of them
 * (0..4096); a tile with more, or whose pairs do not fit in max_pairs, is
 * appended to dense_tiles (int32 (ti, tj), room for max_tiles) instead.
 * *pair_count and *dense_count (device int32, cleared first) receive the
 * counts; *pair_count may exceed max_pairs, and list slots a tile reserved
 * but could not use hold (-1, -1) (qsvm_gram_sym_pairs_dev skips them).
 * max_tiles * cap_per_tile < 2^31.  The order of both lists is not
 * specified. */
qsvm_status qsvm_flag_pairs(const double* K, int64_t N, int64_t ldk, const int32_t* tiles, const int32_t* tile_count,
                            int64_t max_tiles, double cut, int32_t cap_per_tile, int32_t* pairs, int32_t* pair_count,
                            int64_t max_pairs, int32_t* dense_tiles, int32_t* dense_count, void* stream);

/* Static description of a status code (never NULL). */
const char* qsvm_status_string(qsvm_status s);

/* Message describing the calling thread's most recent non-OK status ("" if none). */
const char* qsvm_last_error(void);

/* ABI version of this header: 2 (2: the tuned-variant calls take the point
 * count N; batch options carry the work-item shape). */
int32_t qsvm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QSVM_H */
