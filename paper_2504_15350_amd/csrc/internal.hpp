// Internal launch interface between the C ABI (rpod_abi.cpp) and the kernels.
//
// Every launcher takes a GroupLaunch: device arrays of per-matrix argument
// records and of tile offsets (see args.hpp), the call table, the number of
// matrices and the total number of workgroups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "args.hpp"

namespace rpod {

enum DT : int { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_F16 = 3 };

template <typename A>
struct GroupLaunch {
    const A* args;         // device, count records
    const int* tstart;     // device, count + 1 tile offsets
    const CallDesc* calls; // device call table
    int count;             // matrices in the group
    int tiles;             // workgroups of the launch
    const int* skip = nullptr;  // device; the launch does nothing unless (*skip & skip_mask)
    int skip_mask = 0;
};

// Streaming "skinny-right" product Y = S X on matrix cores (FP64/FP32 S).
//   S: m x n column-major (leading dim ldS); rows >= m and columns >= n read
//      as zero. X: n x 16*nt column-major (ldX >= roundup(n,16), multiple of
//      4), zero rows up to roundup(n,16). Y: mstore x 16*nt column-major (ldY
//      multiple of 4), type tout (F64, F32, or a 16-bit type when tin is F64,
//      converted through FP32); rows [0, mstore) are written, mstore <= ldY.
//   One workgroup per 256 rows of max(m, mstore). A record with cond set does
//   nothing unless (*cond & cond_mask). vec: S is 16-byte aligned with ldS a
//   multiple of 4 (vector loads). upper: X is upper triangular (16 x 16 tiles
//   below the diagonal skipped).
hipError_t launch_sx(int tin, int tout, int nt, bool vec, bool upper, const GroupLaunch<SxArgs>& L, hipStream_t st);
// The same product with X and Y in FP64 and S of any storage type tin,
// converted to FP64 in registers (FP64 matrix cores; vec: 8-byte-or-wider
// aligned vector loads as for launch_sx with that storage type).
hipError_t launch_sx_wide(int tin, int nt, bool vec, const GroupLaunch<SxArgs>& L, hipStream_t st);

// Split-K transposed product: slab s = S[rows of split s]^T Q[rows of split s]
// (FP64 slabs nP x 16*nt, column-major). S: m x n (ldS); Q: m x 16*nt (ldQ,
// zero rows up to roundup(m,64)). Tiles: ncb column blocks x nsplit.
//   FP64 S: ncb = nP / 256, split s covers rows [s*split_rows, ...).
//   FP32 S: ncb = nP / stq32_block_cols(), LDS-staged, splits interleaved in
//   steps of 64 rows (step t of split s: rows 64 (t nsplit + s) ..).
hipError_t launch_stq(int tin, int nt, bool vec, const GroupLaunch<StqArgs>& L, hipStream_t st);
int stq32_block_cols();

// 16-bit (tin = DT_BF16 or DT_F16) versions on the 16x16x32 matrix cores:
// Y (FP32) = S X with X in the same 16-bit type (ldX multiple of 8, zero rows
// up to roundup(n, 32)), one workgroup per 256 rows; slabs of S^T Q with Q
// given as 16-bit hi and lo parts (zero rows up to roundup(m, 128)), the lo
// product added when lo is set, written as FP32 slabs (the FP32
// accumulators). Splits are interleaved in steps of
// stq16_rows_per_step(lo) rows; tiles: ncb = nP / stq16_block_cols(lo) x
// nsplit. vec: S 16-byte aligned with ldS a multiple of 8.
hipError_t launch_sx16(int tin, int nt, bool vec, const GroupLaunch<SxArgs>& L, hipStream_t st);
hipError_t launch_stq16(int tin, int nt, bool lo, bool vec, const GroupLaunch<StqArgs>& L, hipStream_t st);
int stq16_block_cols(bool lo);
int stq16_rows_per_step(bool lo);
// hi = round16(Q), lo = round16(Q - hi) elementwise (count a multiple of 4;
// one workgroup per 1024 elements).
hipError_t launch_split16(int tin, const GroupLaunch<SplitArgs>& L, hipStream_t st);

// FP32 S on the BF16 matrix cores with every operand split exactly into three
// BF16 parts (six products per term, FP32-accurate dot products):
//   launch_sx_e6: Y = S X, X in FP32 (ldX x 16 nt, ldX a multiple of 4, zero
//   rows up to roundup(n, 32)), split as it is staged; 256 rows per workgroup.
//   launch_stq_e6: FP32 slabs of S^T Q, Q in FP32 (ldQ x 16 nt, ldQ a multiple
//   of 4, zero rows up to roundup(m, 32)), split as it is staged; tiles ncb =
//   nP / stq_e6_block_cols() x nsplit, splits interleaved in units of 64
//   rows (split s: rows 64 (k nsplit + s) .., k = 0, 1, ..), nP a multiple
//   of stq_e6_block_cols(); nsplit a multiple of 8 keeps each split's column
//   blocks on one XCD.
// en: also write each tile's sum of the squares of the S entries it read to fpart[tile]
// tall (with vec, not with en): products with few columns of S, the next step's loads issued early
hipError_t launch_sx_e6(int nt, bool vec, bool en, bool tall, const GroupLaunch<SxArgs>& L, hipStream_t st);
hipError_t launch_stq_e6(int nt, bool vec, const GroupLaunch<StqArgs>& L, hipStream_t st);
int stq_e6_block_cols();

// out[e] = sum over the nsplit slabs in FP64, fixed order (FP32 slabs when
// f32 is set, else FP64); one workgroup per 256 elements.
hipError_t launch_reduce_slabs(const GroupLaunch<ReduceArgs>& L, hipStream_t st);

// Fluctuation centring (K lp / 4 tiles for cprep: block k = t mod K, columns
// 4 (t / K) ..; 256 rows per tile for center_y; one tile per row chunk for
// cross; 256 entries per tile for center_z). tx: storage type of X; tacc: type of Y, M and Q.
hipError_t launch_center_prep(int tx, const GroupLaunch<CprepArgs>& L, hipStream_t st);
hipError_t launch_center_y(int tacc, const GroupLaunch<CenterYArgs>& L, hipStream_t st);
hipError_t launch_center_cross(int tacc, const GroupLaunch<CrossArgs>& L, hipStream_t st);
hipError_t launch_center_sum(const GroupLaunch<CrossSumArgs>& L, hipStream_t st);  // one tile per entry

// Reconstruction mean + Phi alpha (out may be NULL) and, with ref, the sums
// ||avg ref - avg recon||^2 and ||avg ref||^2 into out2[0], out2[1] (abar: r
// doubles, part: 2 ceil(m / 256) doubles of scratch). dt: DT_F64 or DT_F32.
// Static scratch of rpod_reconstruct_noalloc: layout and the device address of
// the current GPU's copy (looked up once per GPU).
constexpr int64_t RECON_NOALLOC_MAX_M = (int64_t)1 << 24;
constexpr int64_t RECON_NOALLOC_DOUBLES = 256 + 2 * (RECON_NOALLOC_MAX_M / 256);
hipError_t recon_scratch(double** ptr);
hipError_t launch_reconstruct(int dt, int64_t m, int r, int64_t T, const void* Phi, const void* mean,
                              const void* alpha, void* out, const void* ref, int64_t ld_ref, double* abar,
                              double* part, double* out2, hipStream_t st);
// FP32 fields on the matrix cores (m a multiple of 4, out 16-byte aligned):
// aug (lda x (r + 1), lda = roundup(m, 4)), x (ldx x 128, ldx = roundup(r + 1,
// 32)), one SxArgs record and two ints of tile table, all device scratch.
hipError_t launch_reconstruct_mfma(int64_t m, int r, int64_t T, const float* Phi, const float* mean,
                                   const float* alpha, float* out, float* aug, int64_t lda, float* x, int ldx,
                                   SxArgs* rec, int* tstart, hipStream_t st);

// ||S||_F^2 in FP64 (tin: storage type): nwg tiles of partial sums (columns
// strided over the tiles), then one tile adding them in order.
// sum_only: only the final sum (the partial sums came from the FP32 first pass).
hipError_t launch_frob(int tin, bool vec, bool sum_only, const GroupLaunch<FrobArgs>& P,
                       const GroupLaunch<FrobArgs>& F, hipStream_t st);
hipError_t launch_center_z(const GroupLaunch<CenterZArgs>& L, hipStream_t st);

// Gram matrix G = Y^T Y in FP64 of a tall M x 16*nt column-major matrix
// (ld multiple of 4, zero rows up to roundup(M,16)), type tin (F64/F32).
// Gpart holds gram_partial_count(nt) doubles; G is lp x lp row-major.
// L: gram_tiles(nt, nwg) workgroups per matrix (nwg = gram_nwg(M, cap, nt),
// at most one per 64 rows and at most cap; cap 0: about 512 workgroups over
// the pair groups); R: the reduction, gram_reduce_tiles(nt) workgroups per
// matrix.
int64_t gram_partial_count(int nt);
int gram_nwg(int64_t M, int cap, int nt);
int gram_tiles(int nt, int nwg);
int gram_reduce_tiles(int nt);
hipError_t launch_gram(int tin, int nt, const GroupLaunch<GramArgs>& L, const GroupLaunch<GramArgs>& R,
                       hipStream_t st);

// Cholesky G = R^T R (upper R) and its inverse, one workgroup per matrix, FP64.
//   l: live size, lp: padded size (<= 128); padding becomes identity.
//   On a non-positive pivot the factorisation is retried on G + s I with
//   the shift s = 11 (M l + l (l+1)) 2^-53 trace(G) (Fukaya et al., SISC
//   2020); *local and *flags get DEV_FLAG_SHIFTED. A failure of the retry
//   sets DEV_FLAG_BREAKDOWN; non-finite G sets DEV_FLAG_NONFINITE.
//   R64 / R32: R^-1, lp x lp column-major.
//   mode 0: first factorisation of an orthonormalisation (resets *local);
//   mode 1: unconditional; mode 2: run only if *local has DEV_FLAG_SHIFTED.
//   lp: the padded size shared by the launch's matrices (a multiple of 16;
//   lp / 16 waves per matrix, blocked).
hipError_t launch_chol_inv(int lp, const GroupLaunch<CholArgs>& L, hipStream_t st);

// Symmetric eigen-decomposition of the lp x lp FP64 Gram matrix G_B = B B^T
// (lp a multiple of 16, <= 128): diagonally pivoted Cholesky G_B = P L L^T P^T,
// then one-sided Jacobi (Hestenes) on the columns of L, preconditioned as
// by Drmac and Veselic; one workgroup of jacobi_threads(lp) threads per
// matrix (all matrices of a launch share lp).
//   UB: lp x lp column-major, column k = k-th eigenvector (= left singular
//   vector of B) by descending eigenvalue; sig[k] = sqrt(eigenvalue), the
//   k-th singular value of B, computed as a column norm. Directions beyond
//   the numerical rank of G_B (pivot below lp u max diag) get sig = 0 and a
//   zero UB column. A pair is rotated while |w_p . w_q| > tol |w_p| |w_q|.
int jacobi_threads(int lp);
hipError_t launch_jacobi(int lp, const GroupLaunch<JacobiArgs>& L, hipStream_t st);

// M = Rinv * UB[:, :r] (lp x rp, column-major) in FP64 and FP32, and
// Ur = UB[:, :r] zero-padded to lp x rp; one workgroup per 256 elements.
hipError_t launch_lift_coef(const GroupLaunch<LiftArgs>& L, hipStream_t st);

// Per-column argmax |Phi| partials over row chunks (tiles nchunk x r), then
// per-column signs (one 64-lane wave per column, tiles r).
hipError_t launch_signs(int tphi, const GroupLaunch<ColmaxArgs>& C, const GroupLaunch<SignArgs>& S, hipStream_t st);

// Phi_out (m x r, ld m) = Phi_int * sign; A_out (r x n, ld r) = sign * At^T;
// sigma_out = sig[:r]; the outputs come from the call table.
int fin_phi_tiles(int64_t m, int r, int tphi);  // tphi: type of Phi_int
int fin_a_tiles(int64_t n, int r);
hipError_t launch_finalize(int tphi, const GroupLaunch<FinArgs>& P, const GroupLaunch<FinArgs>& A, hipStream_t st);

// Gaussian sketch (n x l, column-major, ld ldo, zero columns [l, lpad) and
// zero rows [n, rows_pad)); tiles ceil(rows_pad / 256) x ceil(lpad / 2).
hipError_t launch_omega(int tout, const GroupLaunch<OmegaArgs>& L, hipStream_t st);
hipError_t launch_omega_direct(int tout, uint64_t seed, int64_t n, int l, void* out, int64_t ldo, hipStream_t st);
hipError_t launch_sketch_bits(uint64_t seed, int64_t n, int l, uint32_t* out, hipStream_t st);

hipError_t launch_zero_ints(const GroupLaunch<ZeroArgs>& L, hipStream_t st);

// ---- adaptive rank (small_kernels.hip) ----
// Status words of a matrix used by adaptive plans: bit k of ADAPT_ACTIVE lets
// block k run, bit k of ADAPT_STOP selects the finish for k blocks; the
// sketch width reached and the energy rank are published as plain words.
constexpr int ADAPT_ACTIVE = 3, ADAPT_STOP = 4, ADAPT_LUSED = 5, ADAPT_RANK = 6;
constexpr int ADAPT_MAX_BLOCKS = 8;
hipError_t launch_eye(const GroupLaunch<EyeArgs>& L, hipStream_t st);
// one thread: E_i, then either ADAPT_STOP |= 1 << (i + 1) and ADAPT_LUSED =
// (i + 1) b (E_i <= (1 - delta) ||S||_F^2, not finite, or the last block), or
// ADAPT_ACTIVE |= 1 << (i + 1)
hipError_t launch_adapt_decide(const GroupLaunch<AdaptDecideArgs>& L, hipStream_t st);
// one thread: ADAPT_RANK = the smallest r with (sigma_1^2 + .. + sigma_r^2) /
// ||S||_F^2 >= delta (cumulative sum in order), or -1
hipError_t launch_adapt_rank(const GroupLaunch<AdaptRankArgs>& L, hipStream_t st);

// ---- learned warm start (warm_kernels.hip) ----
// Network 4 -> 256 -> 256 -> K (tanh, tanh, softmax), FP32 parameters packed
// as W1 (256 x 4, row-major), b1, W2 (256 x 256), b2, W3 (K x 256), b3.
constexpr int WARM_IN = 4, WARM_H = 256, WARM_K = 8;
constexpr int WP_W1 = 0, WP_B1 = WP_W1 + WARM_H * WARM_IN, WP_W2 = WP_B1 + WARM_H,
              WP_B2 = WP_W2 + WARM_H * WARM_H, WP_W3 = WP_B2 + WARM_H, WP_B3 = WP_W3 + WARM_K * WARM_H,
              WP_COUNT = WP_B3 + WARM_K;
constexpr int DEV_FLAG_RESIDUAL = 0x10;

// Glorot-uniform weights from Philox4x32-10 (key = seed, counter = element
// index), zero biases.
hipError_t launch_warm_init(float* params, uint64_t seed, hipStream_t st);
// Forward of N parameter vectors (N x 4, row-major): hidden layers H1, H2
// (N x 256), softmax weights C (N x K).
hipError_t launch_warm_forward_batch(const float* params, const float* mu, int N, float* H1, float* H2, float* C,
                                     hipStream_t st);
// Loss of every pair (r - 2 b^T c + c^T G8 c) into loss_n, and dZ = dL/dz of
// the mean loss (N x K), from C; then the mean into *loss.
hipError_t launch_warm_loss(const float* C, const double* B, const double* G8, int N, int r, float* dZ,
                            double* loss_n, float* loss, hipStream_t st);
// Backward through the three layers into grads (same packing as params).
hipError_t launch_warm_backward(const float* params, const float* mu, int N, const float* H1, const float* H2,
                                const float* dZ, float* dA2, float* dA1, float* grads, hipStream_t st);
// One Adam step (L2 weight decay in the gradient); bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
hipError_t launch_warm_adam(float* params, const float* grads, float* m, float* v, float lr, float beta1,
                            float beta2, float eps, float wd, float bc1, float bc2, hipStream_t st);
// dst (ldd x cols_pad, FP32) = src (lds x cols) on rows < rows, zero on rows
// [rows, rows_pad) and columns [cols, cols_pad).
hipError_t launch_copy_pad(float* dst, int64_t ldd, const float* src, int64_t lds, int64_t rows, int64_t rows_pad,
                           int cols, int cols_pad, hipStream_t st);
// G[a][c0 + col] = Z[col * ldz + a] for a < Kr, col < ncol (G row-major, ld Kr).
hipError_t launch_gather_cols(double* G, int Kr, int c0, int ncol, const double* Z, int64_t ldz, hipStream_t st);
// out[k * KB + l] = sum over a in block k, b in block l (blocks of r) of
// src[a * sa + b * sb]^2; KA x KB outputs.
hipError_t launch_block_sumsq(const double* src, int64_t sa, int64_t sb, int r, int KA, int KB, double* out,
                              hipStream_t st);
// Plan steps (grouped): network forward of the call's parameter vector, the
// predicted subspace's coordinates (tiles: lp ceil(ldX / 64) per matrix,
// iters <= 2), and the residual of each returned singular triplet: per chunk
// of `rows` rows the squared norms of Y[:, k] - sig_k^2 Phi[:, k] (tiles:
// ceil(m / rows)), then rho_k = ||Y[:, k] - sig_k^2 Phi[:, k]|| / sig_k^2 and
// rho = max_k rho_k (one workgroup per matrix; rejection when rho > tol or
// not finite). r <= WARM_MAXLP.
constexpr int WARM_MAXLP = 128;
constexpr int WARM_RES_ROWS = 1024;  // rows per chunk of the residual sums
constexpr int WARM_DECISION = 2;     // status word of a matrix holding the warm start's decision
constexpr int WARM_PROJ_COLS = 256;  // column block of the FP64 S^T Q kernel (holds lp <= 128)
hipError_t launch_warm_plan_forward(const GroupLaunch<WarmFwdArgs>& L, hipStream_t st);
hipError_t launch_warm_z(const GroupLaunch<WarmZArgs>& L, hipStream_t st);
hipError_t launch_warm_mode_res(const GroupLaunch<ModeResArgs>& P, const GroupLaunch<ModeResFinalArgs>& F,
                                hipStream_t st);

// Write count call-table entries from host values (through kernel arguments).
hipError_t launch_set_calls(CallDesc* table, const CallDesc* host, int count, hipStream_t st);

}  // namespace rpod
