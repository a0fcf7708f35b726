/*
 * rpod.h - C ABI of the MI355X randomized POD library (librpod.so).
 *
 * Randomized proper orthogonal decomposition (rPOD) of a snapshot matrix,
 * after Sec. 4.2 and Alg. 1 ("randomized POD with subspace iterations") of
 * Besabe, Girfoglio, Quaini, Rozza, arXiv 2504.15350: from an m x n snapshot
 * matrix S (m grid cells, n snapshots, one snapshot per column as in the
 * snapshot matrix of Sec. 4.1) and a target rank r, oversampling p and q
 * subspace iterations, compute
 *   Phi   (m x r)  the first r approximate left singular vectors (POD modes),
 *   sigma (r)      the matching approximate singular values, descending,
 *   A     (r x n)  the modal coefficients A = Phi^T S (Sec. 4.3, the matrix
 *                  whose column (k-1) N^t + p holds the coefficients of
 *                  snapshot (t_p, mu_k)).
 *
 * Every step runs on the GPU bound to the plan's stream: Gaussian sketch,
 * the products with S and S^T, CholeskyQR2 re-orthonormalisation after every
 * product (same span as step 3 of Alg. 1), T = Q^T S, the SVD of the small T,
 * the lift Phi = Q U_hat and the coefficients.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Device pointers are HIP device addresses on the current device; host
 *    pointers are marked "host". The caller owns every buffer (S, outputs,
 *    workspace); the library never allocates or frees device memory.
 *  - Matrices are column-major. S has leading dimension ld >= m (element
 *    (i, j) at S[j*ld + i]). Phi is m x r with leading dimension m; A is r x n
 *    with leading dimension r; sigma is r contiguous doubles.
 *  - Output element type: double when the S dtype is RPOD_F64, float for
 *    RPOD_F32, RPOD_BF16 and RPOD_F16. sigma is always double.
 *  - Calls that take a plan only enqueue work on the plan's stream and return
 *    at once. Errors found on the device (non-finite data, a rank-deficient
 *    sketch) are recorded in a device status word that rpod_status_query()
 *    reads after synchronising the stream.
 *  - Arguments are validated before anything is enqueued; on an error
 *    nothing is launched and rpod_last_error() describes the problem.
 *  - No C++ exception crosses this interface.
 *  - Results are deterministic: the same plan, seed and input give bitwise
 *    identical outputs (fixed-order reductions, no floating-point atomics).
 *  - Signs: every mode is flipped so that its entry of largest magnitude is
 *    positive (the lowest row index wins ties); the coefficient row follows.
 */
#ifndef RPOD_H
#define RPOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RPOD_OK = 0,
    RPOD_EINVAL = 1,        /* invalid argument; nothing was enqueued            */
    RPOD_EINVAL_DATA = 2,   /* NaN or Inf found in S (reported by status_query)  */
    RPOD_ENOMEM = 3,        /* workspace smaller than rpod_workspace_size()      */
    RPOD_EHIP = 4,          /* a HIP runtime call or kernel launch failed        */
    RPOD_EUNSUPPORTED = 5,  /* l = r + p > 128, or an unsupported dtype          */
    RPOD_EBREAKDOWN = 6     /* a sketch stayed rank-deficient after the shifted
                               CholeskyQR retry (e.g. S = 0, or l > rank(S) in
                               exact arithmetic); outputs are not meaningful     */
} rpod_status;

typedef enum {
    RPOD_F64 = 0,   /* S in double; all arithmetic FP64                           */
    RPOD_F32 = 1,   /* S in float; products on FP32 matrix cores, FP64 small ops  */
    RPOD_BF16 = 2,  /* S in bfloat16 (mixed precision; see rpod_desc.flags)       */
    RPOD_F16 = 3    /* S in IEEE half (mixed precision)                           */
} rpod_dtype;

/* Device status word bits (rpod_status_query). */
#define RPOD_FLAG_SHIFTED     0x1  /* a Cholesky needed the shifted retry (informational) */
#define RPOD_FLAG_BREAKDOWN   0x2  /* -> RPOD_EBREAKDOWN */
#define RPOD_FLAG_NONFINITE   0x4  /* -> RPOD_EINVAL_DATA */
#define RPOD_FLAG_JACOBI_SLOW 0x8  /* small SVD hit its sweep limit (informational) */
#define RPOD_FLAG_RANK_CUT    0x20 /* FP32/16-bit paths: the Gram matrix T T^T of step 6 was numerically
                                      rank-deficient (a pivot below l u times its largest diagonal entry,
                                      i.e. sigma_k below about sqrt(l u) sigma_1 = 1e-7 sigma_1); those
                                      singular values and their mode columns are returned as 0
                                      (informational; the FP64 path factors T^T itself and never cuts) */

/* Problem description.
 *   m, n   rows (grid cells) and columns (snapshots) of S, both >= 1.
 *   ld     leading dimension of S, >= m.
 *   dtype  an rpod_dtype value: storage type of S.
 *   r      target rank, >= 1;  p oversampling, >= 0;  q subspace iterations, >= 0.
 *          The sketch width l = r + p must satisfy l <= min(m, n) and l <= 128.
 *   flags  0, or RPOD_DESC_ENERGY: the plan also computes ||S||_F^2 (one
 *          more read of S per compute call, before the sketch) so that
 *          rpod_energy() can report the energy of the computed modes.
 *   block_cols  fluctuation snapshots (Sec. 4.1): 0 decomposes S as given;
 *          N^t >= 1 decomposes S' = S - [mean_1 1^T ... mean_M 1^T], where
 *          the columns form M = n / N^t consecutive blocks of N^t snapshots
 *          (one block per parameter, its N^t time instants) and mean_k is the
 *          mean of block k's columns (the time average of that parameter).
 *          Phi, sigma and A are then those of S' (A = Phi^T S'). S itself is
 *          read as given and never modified: the block sums come out of the
 *          first pass over S as M extra sketch columns and every product with
 *          S is corrected algebraically, so no pass is added. n must be a
 *          multiple of N^t and l <= n - M (every block of S' sums to zero, so
 *          rank(S') <= n - M; else RPOD_EINVAL); M <= 64 and roundup(l, 16) +
 *          roundup(M, 16) <= 128 (else RPOD_EUNSUPPORTED); not with warm plans.
 *          Accuracy: the correction subtracts terms of the size of the means,
 *          so with FP32 or 16-bit S the error relative to S' grows with the
 *          ratio of the means to the fluctuations. */
typedef struct {
    int64_t m, n, ld;
    int32_t dtype;
    int32_t r, p, q;
    uint32_t flags;
    int64_t block_cols;
} rpod_desc;

/* rpod_desc.flags bits. */
#define RPOD_DESC_ENERGY 0x1u  /* compute ||S||_F^2 for rpod_energy() */

typedef struct rpod_plan_s* rpod_plan;

/* Bytes of device workspace a plan for *desc needs (written to *bytes).
 * Returns RPOD_EINVAL / RPOD_EUNSUPPORTED for a description rpod_plan_create
 * would reject. */
rpod_status rpod_workspace_size(const rpod_desc* desc, size_t* bytes);

/* Create a plan bound to `hip_stream` (a hipStream_t; NULL = default stream).
 * `workspace` is a device buffer of at least rpod_workspace_size() bytes,
 * 256-byte aligned, owned by the caller and used exclusively by this plan
 * until rpod_plan_destroy(). The workspace is cleared and the plan's launch
 * program is uploaded into it on `hip_stream`; the call synchronises that
 * stream. The whole launch sequence of a compute call is captured once here
 * into a HIP graph (on private streams) that every compute call replays;
 * environment variable RPOD_NO_GRAPH=1 makes compute calls launch the kernels
 * one by one instead (same kernels, same results).
 * The plan object itself is host memory owned by the library. */
rpod_status rpod_plan_create(rpod_plan* plan, const rpod_desc* desc,
                             void* workspace, size_t workspace_bytes, void* hip_stream);

/* Release the host-side plan (the caller frees the workspace). Synchronises
 * the plan's stream first. */
rpod_status rpod_plan_destroy(rpod_plan plan);

/* Randomized POD of S (Alg. 1 of Sec. 4.2 with re-orthonormalisation after
 * every product with S or S^T), enqueued on the plan's stream.
 *   S      device, m x n column-major, leading dimension desc.ld, desc.dtype;
 *          16-byte aligned when ld is a multiple of 4 (FP64, FP32) or of 8
 *          (BF16, FP16), else aligned to its element size.
 *   seed   selects the Gaussian sketch (rpod_generate_omega with this seed).
 *   Phi    device, m x r column-major (ld = m), output.
 *   sigma  device, r doubles, output, descending.
 *   A      device, r x n column-major (ld = r), output, A = Phi^T S.
 * Buffers must not overlap each other or the workspace. */
rpod_status rpod_compute(rpod_plan plan, const void* S, uint64_t seed,
                         void* Phi, double* sigma, void* A);

/* Synchronise the plan's stream and read the device status word of the last
 * compute call (OR of RPOD_FLAG_* bits) into *device_flags (host, may be NULL).
 * Returns RPOD_EINVAL_DATA if RPOD_FLAG_NONFINITE is set, RPOD_EBREAKDOWN if
 * RPOD_FLAG_BREAKDOWN is set, RPOD_EHIP on a runtime error, else RPOD_OK. */
rpod_status rpod_status_query(rpod_plan plan, int32_t* device_flags);

/* Batches: several independent rPOD problems (Sec. 4.2 applied to each
 * snapshot matrix) in one plan. Matrices may differ in m, n, ld, r and p;
 * they must share dtype and q. Matrices whose padded sketch widths
 * (roundup(r + p, 16)) and padded ranks (roundup(r, 16)) agree form a class;
 * every step of Alg. 1 is one kernel launch per class, covering all its
 * matrices (each launch walks a per-matrix table of arguments and workgroup
 * offsets kept in the workspace), and the classes run as independent
 * branches of the plan's graph. Results equal those of single plans for the
 * same matrices and seeds, up to the row-split of the S^T Q products (the
 * split count is chosen per matrix from the batch size, which changes the
 * FP64 summation order of that product only).
 *   descs  host, `count` descriptions, 1 <= count <= 4096.
 * rpod_workspace_size_batched / rpod_plan_create_batched behave as their
 * single-matrix counterparts (which are the count = 1 case). */
rpod_status rpod_workspace_size_batched(const rpod_desc* descs, int32_t count, size_t* bytes);
rpod_status rpod_plan_create_batched(rpod_plan* plan, const rpod_desc* descs, int32_t count,
                                     void* workspace, size_t workspace_bytes, void* hip_stream);

/* Launch-shape knobs of a plan (0 = the library's default for the field).
 *   stq_workgroups   workgroups wanted per matrix for one S^T Q pass; the
 *                    row-split count of that split-K product follows from it
 *                    (at most 64 splits, at least 128 rows each).
 *   gram_workgroups  most workgroups per matrix of a tall Gram matrix, <= 256.
 *   reserved         must be 0.
 * Results depend on the knobs only through the FP64 summation order of the
 * split-K partial sums. */
typedef struct {
    int32_t stq_workgroups;
    int32_t gram_workgroups;
    int32_t reserved[6];
} rpod_tuning;

/* As rpod_workspace_size_batched / rpod_plan_create_batched with explicit
 * knobs (tuning may be NULL: defaults). */
rpod_status rpod_workspace_size_tuned(const rpod_desc* descs, int32_t count, const rpod_tuning* tuning,
                                      size_t* bytes);
rpod_status rpod_plan_create_tuned(rpod_plan* plan, const rpod_desc* descs, int32_t count,
                                   const rpod_tuning* tuning, void* workspace, size_t workspace_bytes,
                                   void* hip_stream);

/* Autotuner of the knobs for a batch (count = 1 for one matrix): times
 * whole compute calls (graph replays, HIP events on hip_stream) on the given
 * matrices for a coordinate search over stq_workgroups in {128, 256, ...,
 * 8192} and then gram_workgroups in {32, 64, 128, 256}, the defaults
 * included, and returns the fastest in *best (host) with its time per call
 * in milliseconds in *best_ms (host, may be NULL). Synchronous: returns
 * after the last trial.
 *   S          host array of `count` device pointers, as for rpod_compute_batched.
 *   workspace  device, at least rpod_autotune_workspace_size() bytes, 256-byte
 *              aligned; overwritten (trial plans and their outputs live there).
 *   repeats    timed calls per candidate (>= 1), after one untimed call.
 *   cache_path host string or NULL. If the file holds an entry for this batch
 *              (a hash of the descriptions, the device name and its compute
 *              unit count) it is returned without timing anything; otherwise
 *              the result is appended to the file as one text line
 *              "<key hex> <stq_workgroups> <gram_workgroups> <ms>". An
 *              unreadable or unwritable file is ignored. */
rpod_status rpod_autotune_workspace_size(const rpod_desc* descs, int32_t count, size_t* bytes);
rpod_status rpod_autotune(const rpod_desc* descs, int32_t count, const void* const* S, void* workspace,
                          size_t workspace_bytes, void* hip_stream, int32_t repeats, const char* cache_path,
                          rpod_tuning* best, double* best_ms);

/* Compute every matrix of a batched plan, enqueued on the plan's stream.
 * S, seeds, Phi, sigma, A: host arrays of `count` entries (the plan's
 * count), entry i being the argument of rpod_compute for matrix i (device
 * pointers, same layout, alignment and ownership rules). Also accepts a
 * plan of one matrix. */
rpod_status rpod_compute_batched(rpod_plan plan, const void* const* S, const uint64_t* seeds,
                                 void* const* Phi, double* const* sigma, void* const* A);

/* As rpod_status_query for every matrix: per_matrix_flags (host, `count`
 * entries, may be NULL) receives each matrix's status word; the return
 * value reflects the OR of all of them. */
rpod_status rpod_status_query_batched(rpod_plan plan, int32_t* per_matrix_flags);

/* Energy of the computed modes (Sec. 4.1, the energy criterion that picks the
 * number of modes from a threshold 0 < delta < 1), read with squared singular
 * values (the eigenvalue energy of the paper's tables): after a compute call
 * on a plan made with RPOD_DESC_ENERGY, energy (host, l = r + p values)
 * receives e_k = (sigma_1^2 + .. + sigma_k^2) / ||S||_F^2, k = 1..l, from the
 * l singular values of the sketched problem (each at most the true sigma_k, so
 * e_k never overstates the energy) and ||S||_F^2 computed on the GPU in FP64
 * (not with block_cols: RPOD_EUNSUPPORTED at plan creation). *rank (host, may be NULL) receives the
 * smallest k with e_k >= delta, or -1 when e_l < delta (a larger r + p is
 * needed). item selects the matrix of a batched plan (0 otherwise).
 * Synchronises the plan's stream. RPOD_EINVAL: NULL plan or energy, item out
 * of range, delta outside (0, 1), or a plan made without RPOD_DESC_ENERGY. */
rpod_status rpod_energy(rpod_plan plan, int32_t item, double delta, double* energy, int32_t* rank);

/* Reconstruction of the reduced-order fields (Sec. 4, the ROM approximation:
 * a field equals its zeroth-order time average plus the modes weighted by
 * their coefficients) and the relative L2 error of time-averaged fields
 * (Sec. 5, the error measure against the full-order solution).
 *   dtype  RPOD_F64 or RPOD_F32: element type of Phi, mean, alpha, out, ref.
 *   Phi    (device) m x r modes, leading dimension m; r in 1..128.
 *   mean   (device, may be NULL = zero) the zeroth-order field, m values.
 *   alpha  (device) r x T coefficients, leading dimension r (column t: time t).
 *   out    (device, may be NULL) receives the m x T fields mean + Phi alpha,
 *          leading dimension m.
 *   ref    (device, may be NULL) m x T full-order fields, leading dimension
 *          ld_ref >= m; with ref and eps non-NULL, *eps (host) receives
 *          ||avg_t ref - avg_t(mean + Phi alpha)|| / ||avg_t ref|| (Euclidean
 *          norms over the m cells: the L2 norm on a uniform grid up to the
 *          cell area, which cancels) and the call synchronises the stream;
 *          otherwise it only enqueues.
 * FP32 fields with m a multiple of 4 and out 16-byte aligned are formed on
 * the matrix cores with operands split exactly into BF16 parts (FP32-accurate
 * products, FP32 sums); other fields by fused multiply-adds in dtype. The
 * error's sums run in FP64, fixed order. workspace (device, 256-byte aligned) of at
 * least rpod_reconstruct_workspace_size(m, r) bytes, used only during the call. */
rpod_status rpod_reconstruct_workspace_size(int64_t m, int32_t r, size_t* bytes);
rpod_status rpod_reconstruct(int32_t dtype, int64_t m, int32_t r, int64_t T, const void* Phi, const void* mean,
                             const void* alpha, void* out, const void* ref, int64_t ld_ref, void* workspace,
                             size_t workspace_bytes, void* hip_stream, double* eps);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): rpod_reconstruct without
 * a workspace argument. Same arguments, meaning and results, except that the
 * fields are always formed by fused multiply-adds in dtype (never on the
 * matrix cores, whose operand staging needs a workspace), so FP32 fields may
 * differ from rpod_reconstruct's in the last bits; the error is the same
 * computation. Its scratch (the time-averaged coefficients, the partial sums
 * of the error) is a static device array of about 1 MB per GPU, kept until
 * the process ends; the call allocates nothing. m <= 2^24 (RPOD_EINVAL
 * beyond). Every call on one GPU shares that array: calls that overlap on
 * one GPU (different streams or threads) race and must be serialised by the
 * caller. */
rpod_status rpod_reconstruct_noalloc(int32_t dtype, int64_t m, int32_t r, int64_t T, const void* Phi,
                                     const void* mean, const void* alpha, void* out, const void* ref, int64_t ld_ref,
                                     void* hip_stream, double* eps);

/* The Gaussian sketch of Alg. 1 step 1 (entries N(0,1), Sec. 4.2), drawn on
 * the GPU: out (device) receives the n x l matrix column-major with leading
 * dimension ldo >= n, as double (dtype RPOD_F64) or float (RPOD_F32, the
 * double value rounded to nearest).
 * Definition: entry (j, c) uses Philox4x32-10 (Salmon et al., SC'11) with
 * key (seed mod 2^32, seed div 2^32) and counter (j mod 2^32, j div 2^32,
 * c div 2, 0), giving words x0..x3; a = (x0>>5)*2^26 + (x1>>6),
 * b = (x2>>5)*2^26 + (x3>>6), u1 = (a + 1/2) 2^-53, u2 = b 2^-53,
 * rho = sqrt(-2 ln u1), theta = 6.283185307179586 u2; even c takes
 * rho cos(theta), odd c takes rho sin(theta). Enqueued on hip_stream. */
rpod_status rpod_generate_omega(uint64_t seed, int64_t n, int32_t l, int32_t dtype,
                                void* out, int64_t ldo, void* hip_stream);

/* Raw Philox words behind the sketch: out (device, uint32) receives
 * n * ceil(l/2) * 4 words, element ((j * ceil(l/2) + t) * 4 + w) = word w of
 * the call for row j, column pair t. Enqueued on hip_stream. */
rpod_status rpod_sketch_bits(uint64_t seed, int64_t n, int32_t l, uint32_t* out,
                             void* hip_stream);

/* ------------------------------------------------------------------------
 * Learned warm start (an extension of Alg. 1 of Sec. 4.2; the paper has no
 * warm start). A small network maps the normalised parameter vector mu of a
 * snapshot matrix (4 components in [-1, 1]) to weights c over a bank of 8
 * orthonormal bases Phi_1..Phi_8 (m x r each, typically computed by rPOD at
 * other parameter values):
 *   c = softmax(W3 tanh(W2 tanh(W1 mu + b1) + b2) + b3),  4 -> 256 -> 256 -> 8,
 * FP32, 69,128 parameters packed in this order: W1 (256 x 4, row-major), b1
 * (256), W2 (256 x 256), b2 (256), W3 (8 x 256), b3 (8).
 * The predicted subspace is W = P(c)^j Phi_k*, P(c) = sum_k c_k Phi_k Phi_k^T,
 * k* = argmax c (lowest index on ties), j = 2: two steps of subspace
 * iteration on the weighted projector from the bank basis of largest weight
 * (a one-hot c gives Phi_k exactly; the result does not depend on the signs
 * or rotations of the bank bases). It is formed from the cached FP64 bank
 * Gram G_W = [Phi]^T [Phi] and one product with the bank.
 * Training loss of a pair (mu_i, Phi_i), mean over the pairs:
 *   L_i = ||Phi_i Phi_i^T - P(c)||_F^2 = r - 2 b_i^T c + c^T G8 c,
 *   b_ik = ||Phi_k^T Phi_i||_F^2 (rpod_warm_targets), G8_kl = ||Phi_k^T Phi_l||_F^2;
 * optimiser Adam with L2 weight decay added to the gradient. Every step
 * (forward, loss, backward, Adam, bank Grams) runs in the library's kernels.
 * ------------------------------------------------------------------------ */
#define RPOD_FLAG_RESIDUAL 0x10  /* warm start: result rejected, continuation ran (informational) */
#define RPOD_WARM_PARAMS 69128

typedef struct {
    int64_t m;          /* rows of the bank bases and of the snapshot matrices, >= 1 */
    int32_t r;          /* columns of each bank basis, 1..128 (= the rank of warm plans) */
    int32_t max_train;  /* largest batch of pairs for training / prediction, 1..4096 */
    uint64_t seed;      /* initial weights: Glorot-uniform from Philox4x32-10 */
} rpod_warm_desc;

/* Byte offsets into the model workspace (for reading or writing the
 * parameters and their gradient directly; FP32 arrays of RPOD_WARM_PARAMS). */
typedef struct {
    size_t params, grads, adam_m, adam_v;
    size_t bank;   /* FP32, column-major, leading dimension roundup(m, 256), 8 r columns */
    size_t gram;   /* FP64 G_W, 8r x 8r row-major */
    size_t gram8;  /* FP64 G8, 8 x 8 row-major */
    size_t total;  /* bytes of the model workspace */
} rpod_warm_layout;

typedef struct rpod_warm_s* rpod_warm;

rpod_status rpod_warm_layout_of(const rpod_warm_desc* desc, rpod_warm_layout* layout);

/* Create a model on `workspace` (device, layout.total bytes, 256-byte
 * aligned, owned by the caller): cleared, weights initialised from the seed,
 * Adam state zero. Every model call enqueues on hip_stream and those that
 * upload launch arguments (set_bank, targets) synchronise it. */
rpod_status rpod_warm_create(rpod_warm* model, const rpod_warm_desc* desc, void* workspace, size_t workspace_bytes,
                             void* hip_stream);
rpod_status rpod_warm_destroy(rpod_warm model);

/* Store the bank: bases = host array of 8 device pointers, each m x r FP32
 * column-major with leading dimension m (orthonormal columns expected); then
 * G_W and G8 in FP64. Synchronous. */
rpod_status rpod_warm_set_bank(rpod_warm model, const float* const* bases);

/* b (device, 8 doubles) = ||Phi_k^T basis||_F^2 for the m x r FP32 basis
 * (device, leading dimension m). Synchronous. */
rpod_status rpod_warm_targets(rpod_warm model, const float* basis, double* b);

/* Mean loss over N pairs (mu: device N x 4 FP32 row-major; b: device N x 8
 * FP64 targets) into *loss (device FP32, may be NULL) and its gradient into
 * the model's gradient array. N <= max_train. Enqueued. */
rpod_status rpod_warm_loss_grad(rpod_warm model, const float* mu, const double* b, int32_t N, float* loss);

/* `epochs` full-batch Adam steps on the N pairs (lr, beta1, beta2, eps,
 * weight_decay as in Adam with L2 decay); losses (device FP32, epochs
 * entries, may be NULL) receives the loss before each step. The step count
 * of the bias correction continues across calls. Enqueued. */
rpod_status rpod_warm_train(rpod_warm model, const float* mu, const double* b, int32_t N, int32_t epochs,
                            float lr, float beta1, float beta2, float eps, float weight_decay, float* losses);

/* c (device N x 8 FP32) = the network's weights for N parameter vectors. Enqueued. */
rpod_status rpod_warm_predict(rpod_warm model, const float* mu, int32_t N, float* c);

/* Warm plans. desc: dtype RPOD_F32, RPOD_BF16 or RPOD_F16, m = the model's
 * m, r = the model's r, p >= 1 Gaussian columns next to the predicted
 * subspace (l = r + p <= 128), q >= 0 subspace iterations after it. A
 * compute call runs Y = [W, S Omega_p] (Omega_p: the first p columns of the
 * sketch of `seed`), the CholeskyQR orthonormalisation, q iterations,
 * T = Q^T S and steps 6-7 of Alg. 1, then checks every returned triplet
 * (sigma_k, phi_k, v_k = a_k / sigma_k, a_k the k-th row of A):
 *   rho_k = ||S v_k - sigma_k phi_k|| / sigma_k,  rho = max_k rho_k,
 * S v_k from a product with FP64 arithmetic. The pair (phi_k, v_k) is then
 * an approximate singular pair: some singular value of S lies within
 * sigma_k rho_k of sigma_k. If rho <= tol the warm result stands; otherwise
 * (or if rho is not finite) q_fallback further subspace iterations continue
 * from the warm range basis Q and steps 5-7 run again, overwriting the
 * outputs (RPOD_FLAG_RESIDUAL is set in the status word). The decision is
 * taken on the device inside the same launch graph: no host round trip.
 * tol = +infinity accepts every warm result without the check: the residual
 * product (one more pass over S, with FP64 arithmetic) is not run, rho is
 * reported as NaN and q_fallback is unused.
 * A breakdown in either part is reported as by rpod_compute. The model must
 * outlive the plan; its weights and bank are read at every call. */
rpod_status rpod_workspace_size_warm(const rpod_desc* desc, rpod_warm model, int32_t q_fallback, size_t* bytes);
rpod_status rpod_plan_create_warm(rpod_plan* plan, const rpod_desc* desc, rpod_warm model, int32_t q_fallback,
                                  double tol, void* workspace, size_t workspace_bytes, void* hip_stream);

/* mu: host, 4 floats (normalised parameter vector). fell_back (1 if the
 * warm result was rejected and the continuation ran) and rho (of the warm
 * result): host, may be NULL; if either is non-NULL the call synchronises
 * the plan's stream to read them, else it only enqueues. */
rpod_status rpod_compute_warm(rpod_plan plan, const void* S, const float* mu, uint64_t seed, void* Phi,
                              double* sigma, void* A, int32_t* fell_back, double* rho);

/* rho_modes: host, r doubles: the rho_k of the warm result of the last
 * compute call. Synchronises the plan's stream. RPOD_EINVAL for a plan made
 * with tol = +infinity (nothing is computed). */
rpod_status rpod_warm_residuals(rpod_plan plan, double* rho_modes);

/* ------------------------------------------------------------------------
 * Adaptive rank (the energy rule of Sec. 4.1 chooses the number of modes;
 * Alg. 1 needs the sketch width before it starts). The sketch grows by
 * blocks of b columns with the blocked fixed-accuracy range finder of Yu,
 * Gu and Li (SIAM J. Matrix Anal. Appl. 39, 2018, randQB_EI):
 *   E = ||S||_F^2; for block i = 0, 1, ...:
 *     Q_i = orth(S Omega_i - Q (B Omega_i)); q times:
 *       Z_i = orth(S^T Q_i - B^T (Q^T Q_i)), Q_i = orth(S Z_i - Q (B Z_i));
 *     B_i = Q_i^T S; Q = [Q, Q_i]; B = [B; B_i]; E = E - ||B_i||_F^2
 *   until E <= (1 - delta) ||S||_F^2 or l = l_max,
 * E being the exact squared Frobenius error ||S - Q B||_F^2. The
 * orthonormalisations are CholeskyQR2 of [Q, block] (the Cholesky factor of
 * the joint Gram projects the block off Q; twice). Steps 6-7 of Alg. 1 then
 * run on B for all l columns, and the energy rank is the smallest r with
 * (sigma_1^2 + .. + sigma_r^2) / ||S||_F^2 >= delta (-1 if none). Omega_i
 * are columns i b .. i b + b - 1 of the sketch of `seed` (the columns
 * rpod_compute would use with l = l_max). With q = 0 the l columns of Q span
 * S Omega[:, :l], as in rpod_compute with that l. The whole loop, the stopping
 * test included, runs on the device in one launch graph: blocks after the
 * stop and the finishes for other widths are skipped launches.
 * desc: m, n, ld, dtype as for rpod_compute; r = l_max (a multiple of p, at
 * most 128 and at most min(m, n)); p = b (a positive multiple of 16); q
 * >= 0 power iterations per block; flags 0; block_cols 0. 0 < delta <= 1.
 * Per-pass timing records nothing for these plans. */
rpod_status rpod_workspace_size_adaptive(const rpod_desc* desc, double delta, size_t* bytes);
rpod_status rpod_plan_create_adaptive(rpod_plan* plan, const rpod_desc* desc, double delta, void* workspace,
                                      size_t workspace_bytes, void* hip_stream);

/* S as for rpod_compute. Outputs (device, room for l_max modes): Phi m x l
 * column-major (leading dimension m), sigma l values, A n x l row-major
 * (A[j l + k]), l = the sketch width used; storage types as for
 * rpod_compute. l_used, rank (the energy rank) and residual (E / ||S||_F^2
 * when the loop stopped): host, may be NULL; if any is non-NULL the call
 * synchronises the plan's stream to read them, else it only enqueues.
 * Errors as for rpod_compute (rpod_status_query). */
rpod_status rpod_compute_adaptive(rpod_plan plan, const void* S, uint64_t seed, void* Phi, double* sigma, void* A,
                                  int32_t* l_used, int32_t* rank, double* residual);

/* Per-pass timing, for measurement. With enable != 0 the plan records a
 * pair of HIP events on its stream around every pass over S issued by later
 * compute calls (pass 0: the products S X of Alg. 1 steps 2-3; pass 1: the
 * products S^T Q of steps 3 and 5; pass 2: on 16-bit storage, the product
 * S^T Q of step 5, which carries Q as hi + lo parts and is kept apart from
 * pass 1), resetting earlier records; enable = 0 stops recording. The first
 * call with enable != 0 creates the events. */
rpod_status rpod_plan_set_timing(rpod_plan plan, int32_t enable);

/* Synchronise the plan's stream and report the recorded launches of one
 * pass kind (0, 1 or 2): their number, summed duration in milliseconds, and the
 * algorithmic work of one launch: bytes = m n size(S) + n l size(S) + m l 4
 * (S once, the n x l operand once, the m x l result or operand once) and
 * flops = 2 m n l, summed over the matrices the launch covers (a batched
 * plan times its classes' launches; timing replays the kernels one by one
 * instead of the graph). Host pointers; any may be NULL. */
rpod_status rpod_plan_get_timing(rpod_plan plan, int32_t pass, int64_t* launches, double* total_ms,
                                 double* bytes_per_launch, double* flops_per_launch);

/* Human-readable description of the last error on the calling thread
 * (static storage, valid until the next call on that thread). */
const char* rpod_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RPOD_H */
