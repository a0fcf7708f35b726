// Internal launch interface between the C ABI (rpod_abi.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpod {

enum DT : int { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_F16 = 3 };

// Streaming "skinny-right" product Y = S X on matrix cores.
//   S: m x n column-major (leading dim ldS), element type tin (F64 or F32);
//      rows >= m and columns >= n read as zero.
//   X: n x 16*nt column-major (ldX >= roundup(n,16), multiple of 4), type tin,
//      zero-padded rows up to roundup(n,16).
//   Y: mstore x 16*nt column-major (ldY multiple of 4), type tout (F64, F32,
//      or a 16-bit type when tin is F64, converted through FP32); rows
//      [0, mstore) are written, mstore <= ldY.
//   If cond != nullptr the kernel does nothing unless (*cond & cond_mask).
//   upper: X is upper triangular (16 x 16 tiles below the diagonal skipped).
hipError_t launch_sx(int tin, int tout, int nt, const void* S, int64_t ldS, int64_t m, int64_t n,
                     const void* X, int64_t ldX, void* Y, int64_t ldY, int64_t mstore,
                     const int* cond, int cond_mask, hipStream_t st, bool upper = false);

// Split-K transposed product: partial[s] = S[rows of split s]^T Q[rows of split s].
//   S: m x n column-major (ldS), type tin; Q: m x 16*nt column-major (ldQ,
//   zero rows up to roundup(m,16)), type tin.
//   Zp: nsplit slabs of nP x 16*nt doubles (column-major, ld nP); nP is a
//   multiple of 256 >= n. Split s covers rows [s*split_rows, (s+1)*split_rows).
hipError_t launch_stq(int tin, int nt, const void* S, int64_t ldS, int64_t m, int64_t n,
                      const void* Q, int64_t ldQ, double* Zp, int64_t nP,
                      int64_t split_rows, int nsplit, hipStream_t st);

// 16-bit (tin = DT_BF16 or DT_F16) versions on the 16x16x32 matrix cores:
// Y (FP32) = S X with X in the same 16-bit type (ldX multiple of 8, zero rows
// up to roundup(n, 32)); partial Z = S^T Q with Q given as 16-bit hi and lo
// parts (zero rows up to roundup(m, 64)); the lo product is added when lo is
// set. split_rows must be a multiple of 64.
hipError_t launch_sx16(int tin, int nt, const void* S, int64_t ldS, int64_t m, int64_t n, const void* X,
                       int64_t ldX, float* Y, int64_t ldY, int64_t mstore, hipStream_t st);
hipError_t launch_stq16(int tin, int nt, bool lo, const void* S, int64_t ldS, int64_t m, int64_t n,
                        const unsigned short* Qh, const unsigned short* Ql, int64_t ldQ, double* Zp, int64_t nP,
                        int64_t split_rows, int nsplit, hipStream_t st);
// hi = round16(Q), lo = round16(Q - hi) elementwise (count a multiple of 4).
hipError_t launch_split16(int tin, const float* Q, int64_t count, unsigned short* hi, unsigned short* lo,
                          hipStream_t st);

// out[e] = sum_s Zp[s * count + e], fixed order.
hipError_t launch_reduce_slabs(const double* Zp, int nsplit, int64_t count, double* out, hipStream_t st);

// Gram matrix G = Y^T Y in FP64 of a tall M x 16*nt column-major matrix
// (ld multiple of 4, zero rows up to roundup(M,16)), type tin (F64/F32).
// Gpart must hold gram_partial_count(nt) doubles. G is lp x lp row-major.
int64_t gram_partial_count(int nt);
hipError_t launch_gram(int tin, int nt, const void* Y, int64_t ld, int64_t M, double* Gpart,
                       double* G, const int* cond, int cond_mask, hipStream_t st);

// Cholesky G = R^T R (upper R) and its inverse, one workgroup, FP64.
//   l: live size, lp: padded size (<= 128); padding becomes identity.
//   On a non-positive pivot the factorisation is retried on G + s I with
//   the shift s = 11 (M l + l (l+1)) 2^-53 trace(G) (Fukaya et al., SISC
//   2020); *local and *flags get DEV_FLAG_SHIFTED. A failure of the retry
//   sets DEV_FLAG_BREAKDOWN; non-finite G sets DEV_FLAG_NONFINITE.
//   Rinv64 / Rinv32: lp x lp column-major.
//   mode 0: first factorisation of an orthonormalisation (resets *local);
//   mode 1: unconditional; mode 2: run only if *local has DEV_FLAG_SHIFTED.
hipError_t launch_chol_inv(const double* G, int l, int lp, int64_t M, double* Rinv64, float* Rinv32,
                           int* flags, int* local, int mode, hipStream_t st);

// Symmetric eigen-decomposition of the lp x lp FP64 Gram matrix G_B = B B^T
// by one-sided Jacobi (Hestenes) on its columns, one workgroup.
//   UB: lp x lp column-major, column k = k-th eigenvector (= left singular
//   vector of B) by descending eigenvalue; sig[k] = sqrt(eigenvalue).
//   A pair is rotated while |w_p . w_q| > tol |w_p| |w_q|.
hipError_t launch_jacobi(const double* G, int l, int lp, double* UB, double* sig, int* flags, double tol,
                         hipStream_t st);

// M = Rinv * UB[:, :r] (lp x rp, column-major) in FP64 and FP32, and
// Ur = UB[:, :r] zero-padded to lp x rp.
hipError_t launch_lift_coef(const double* Rinv, const double* UB, int lp, int r, int rp,
                            double* M64, float* M32, double* Ur, hipStream_t st);

// Per-column argmax |Phi| partials over row chunks, then per-column sign.
hipError_t launch_signs(int tphi, const void* Phi, int64_t ld, int64_t m, int r, int nchunk,
                        double* part_val, int64_t* part_idx, double* signs, hipStream_t st);

// Phi_out (m x r, ld m) = Phi_int * sign; A_out (r x n, ld r) = sign * At^T;
// sigma_out = sig[:r].
hipError_t launch_finalize(int tphi, const void* Phi_int, int64_t ldP, int64_t m, int r,
                           const double* At, int64_t ldA, int64_t n, const double* signs,
                           const double* sig, void* Phi_out, void* A_out, double* sigma_out,
                           hipStream_t st);

// Gaussian sketch (n x l, column-major, ld ldo, zero columns [l, lpad) and
// zero rows [n, rows_pad)) and raw Philox words.
hipError_t launch_omega(int tout, uint64_t seed, int64_t n, int l, int lpad, int64_t rows_pad,
                        void* out, int64_t ldo, hipStream_t st);
hipError_t launch_sketch_bits(uint64_t seed, int64_t n, int l, uint32_t* out, hipStream_t st);

hipError_t launch_zero_ints(int* p, int count, hipStream_t st);

}  // namespace rpod
