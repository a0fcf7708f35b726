// Argument records of the grouped kernels (host and device).
//
// Every kernel is launched "grouped": one launch serves a group of matrices.
// The launch receives a device array of per-matrix argument records and a
// tile-offset table tstart[0..count]; workgroup b belongs to the matrix i with
// tstart[i] <= b < tstart[i+1] and handles local tile b - tstart[i]. A single
// matrix is a group of one. Per-call pointers (S, the outputs, the seed) live
// in a call table written before every compute call; records that need them
// say so (from_call) and carry the matrix's index into that table.
#pragma once

#include <stdint.h>

namespace rpod {

struct CallDesc {  // written per compute call
    const void* S;
    void* Phi;
    double* sigma;
    void* A;
    uint64_t seed;
    float mu[4];  // parameter vector of a warm-started call
};

struct SxArgs {  // Y = S X
    const void* S;
    int64_t ldS, m, n;
    const void* X;
    int64_t ldX;
    void* Y;
    int64_t ldY, mstore;
    const int* cond;
    int cond_mask;
    int call;  // >= 0: S comes from call table entry `call`
    int cmax;  // > 0: only output columns < cmax are stored
    double* fpart;  // FP32 first pass with the energy report: per-tile sums of S's squares
    int64_t col0;   // the product starts at column col0 of S (split-K over the columns; X already offset)
};

struct StqArgs {  // Z_s = S_s^T Q_s (split-K slabs)
    const void* S;
    int64_t ldS, m, n;
    const void* Q;   // FP32/FP64 Q, or the 16-bit hi part
    const void* Ql;  // 16-bit lo part
    int64_t ldQ;
    double* Zp;
    int64_t nP, split_rows;
    int nsplit, ncb;
    int call;
};

struct ReduceArgs {  // out = scale * (sum of nsplit slabs)
    const void* Zp;  // FP64 slabs, or FP32 ones when f32 is set
    int64_t count;
    void* out;       // FP64, or FP32 when out32 is set
    int nsplit;
    int f32;
    int out32;
    double scale = 1.0;  // a power of two (undoes the scale of an FP16 Q)
};

// Fluctuation snapshots (Sec. 4.1): S' = S - M E^T / N with M the block sums
// (m x K, columns lp .. lp + K - 1 of the first pass's output), E the n x K
// block indicator and N the block length. Column-major small matrices:
// C[k + c K].
struct CprepArgs {  // C = E^T X / N for the sketch-side operand X; optionally E itself
    void* X;        // storage type, ld rows, columns 0 .. lp - 1 read, lp .. lp + K - 1 written when ind
    int64_t ld, n, N;
    double* C;      // K x lp
    int lp, K, ind;
};

struct CenterYArgs {  // Y[:, c] -= sum_k M[:, k] C[k + c K], rows < m, c < lp
    void* Y;          // FP32/FP64, ld rows, lp + K columns (M after the first lp)
    int64_t ld, m;
    const double* C;
    int lp, K;
};

struct CrossArgs {  // partial sums of P = M^T Q over row chunks of `chunk` rows
    const void* M;  // FP32/FP64, ld rows, K columns
    const void* Q;  // FP32/FP64, ld rows, lp columns
    int64_t ld, m, chunk;
    double* Pp;     // entry-major: Pp[o * nchunk + chunk index], o = k + c K
    int lp, K, nchunk;
};

struct CrossSumArgs {  // P[o] = sum over the nchunk partial sums of entry o
    const double* Pp;
    double* P;
    int count, nchunk;
};

struct CenterZArgs {  // Z[j, c] -= P[j / N + c K] / N, j < n, c < lp
    double* Z;        // FP64, ld rows
    int64_t ld, n, N;
    const double* P;
    int lp, K;
};

struct FrobArgs {  // ||S||_F^2: per-workgroup partial sums, then their sum
    const void* S;    // storage type; from call table entry `call` when call >= 0
    int64_t ld, m, n;
    double* part;     // nwg partial sums
    double* out;      // the sum
    int nwg, call;
};

struct GramArgs {  // G = Y^T Y, FP64
    const void* Y;
    int64_t ld, M;
    double* Gpart;
    double* G;
    const int* cond;
    int cond_mask;
    int nwg;
};

struct CholArgs {  // Cholesky + inverse
    const double* G;
    int64_t M;
    double* R64;
    float* R32;
    int* flags;
    int* local;
    int l, lp, mode;
};

struct JacobiArgs {  // left singular vectors of the small T: from its Gram matrix, or from a factor C
    const double* G;   // Gram route: G = T T^T (lp x lp, row-major)
    double* UB;
    double* sig;
    int* flags;
    double tol;
    int l, lp;
    const double* C;   // non-NULL: factor route, C (l x l, column-major, leading dimension ldc) with
    int64_t ldc;       // C C^T = T T^T; one-sided Jacobi runs on the columns of C itself
};

struct LiftArgs {  // M = Rinv UB[:, :r], Ur = UB[:, :r]
    const double* Rinv;
    const double* UB;
    double* M64;
    float* M32;
    double* Ur;
    int lp, r, rp;
};

struct ColmaxArgs {  // per-chunk argmax |Phi|
    const void* Phi;
    int64_t ld, m, chunk;
    double* pval;
    int64_t* pidx;
    int r, nchunk;
};

struct SignArgs {
    const double* pval;
    const int64_t* pidx;
    double* signs;
    int r, nchunk;
};

struct FinArgs {  // outputs (Phi, A, sigma) from call table entry `call`
    const void* Phi_int;
    int64_t ldP, m;
    const double* At;
    int64_t ldA, n;
    const double* signs;
    const double* sig;
    int r, call;
};

struct OmegaArgs {  // Gaussian sketch; seed from call table entry `call` (or `seed` if call < 0)
    void* out;
    int64_t n, rows_pad, ldo;
    uint64_t seed;
    int l, lpad, call;
    uint32_t stream;  // counter word 3 (0: the sketch, 1: the residual probes)
};

struct SplitArgs {  // 16-bit hi/lo split of scale * Q
    const float* Q;
    int64_t count;
    unsigned short* hi;
    unsigned short* lo;
    float scale = 1.0f;  // a power of two
};

struct ZeroArgs {
    int* p;
    int count;
};

// ---- adaptive rank (blocked range finder) ----
struct EyeArgs {  // R (lp x lp, FP64) = I
    double* R;
    int lp;
};

struct AdaptDecideArgs {  // after block i: E_i = ||S||_F^2 - sum_{j <= i} cap[j], stop test
    const double* fro2;
    const double* cap;    // ||B_j||_F^2 of every finished block
    double* E;            // E_i, one per block
    int* flags;           // status words of the matrix
    double delta;
    int i, kmax, b;
};

struct AdaptRankArgs {  // the energy rank of the l computed singular values
    const double* sig;
    const double* fro2;
    int* flags;
    double delta;
    int l;
};

// ---- learned warm start ----
struct WarmFwdArgs {  // network forward of the call's parameter vector
    const float* params;
    double* c;     // K weights (FP64 copy of the FP32 softmax)
    int* kstar;    // argmax of c, lowest index on ties
    int call;
};

struct WarmZArgs {  // coordinates Z of the predicted subspace in the bank, FP32 out
    const double* GW;   // Kr x Kr row-major
    const double* c;
    const int* kstar;
    float* X;           // ldX x lp column-major
    int64_t ldX;
    int r, Kr, lp, iters;
};

struct ModeResArgs {  // per row chunk: sums over rows of (Y[:, k] - sig_k^2 Phi[:, k])^2, k < r
    const double* Y;      // m x r (ldY): S A^T with FP64 products
    int64_t ldY, m;
    const float* Phi;     // m x r (ldP): the returned modes before the sign convention
    int64_t ldP;
    const double* sig;    // r
    double* part;         // nchunk x r
    int64_t rows;         // rows per chunk (a multiple of 64)
    int r;
};

struct ModeResFinalArgs {  // rho_k = sqrt(sum of part[:, k]) / sig_k^2, rho = max_k rho_k
    const double* part;
    const double* sig;
    double* rho_modes;    // r
    double* rho;          // 1
    int* flags;           // status word: DEV_FLAG_RESIDUAL when the result is rejected
    int* decision;        // 1 when rejected (the continuation runs), else 0
    double tol;
    int r, nchunk;
};

// Workgroup -> (item, local tile) for grouped launches.
#ifdef __HIPCC__
__device__ __forceinline__ int group_item(const int* tstart, int count, int b) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {  // last i with tstart[i] <= b
        const int mid = (lo + hi + 1) >> 1;
        if (tstart[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}
#endif

// One grouped launch as seen by a kernel. skip (device, may be NULL): the
// whole launch does nothing unless (*skip & skip_mask) != 0 -- a step of a
// recorded program that runs only when an earlier kernel raised a flag.
template <typename A>
struct Group {
    const A* args;
    const int* tstart;
    const CallDesc* calls;
    int count;
    const int* skip = nullptr;
    int skip_mask = 0;
};

#ifdef __HIPCC__
template <typename A>
__device__ __forceinline__ bool group_skipped(const Group<A>& g) {
    return g.skip != nullptr && !(*g.skip & g.skip_mask);
}
#endif

}  // namespace rpod
