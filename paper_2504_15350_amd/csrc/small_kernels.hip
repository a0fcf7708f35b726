// Small FP64 linear algebra of the rPOD path and the Gaussian sketch.
//
//   k_omega        Gaussian sketch (Alg. 1 step 1) from Philox4x32-10
//   k_gram         FP64 Gram matrix Y^T Y of a tall matrix on FP64 MFMA
//   k_chol_inv     Cholesky + triangular inverse for CholeskyQR (step 4)
//   k_jacobi       SVD of the small T of step 6 via the eigenvectors of T T^T
//   k_lift_coef    the small factors of the lift (step 7) and the coefficients
//   k_colmax/...   deterministic sign convention and output packing
#include "device_common.hpp"
#include "internal.hpp"

namespace rpod {

template <typename T>
using V4 = typename vec4_of<T>::type;

__global__ void k_zero_ints(int* p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

hipError_t launch_zero_ints(int* p, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_ints, dim3((count + 255) / 256), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gaussian sketch. Thread per (row j, column pair t).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_omega(uint64_t seed, int64_t n, int l, int lpad, int64_t rows_pad, T* out, int64_t ldo) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;  // column pair
    if (j >= rows_pad) return;
    const int c0 = 2 * t, c1 = 2 * t + 1;
    double g0 = 0.0, g1 = 0.0;
    if (j < n && c0 < l) {
        const philox_out o = philox4x32_10((uint32_t)j, (uint32_t)((uint64_t)j >> 32), (uint32_t)t, 0u,
                                           (uint32_t)seed, (uint32_t)(seed >> 32));
        const uint64_t a = ((uint64_t)(o.x[0] >> 5) << 26) + (o.x[1] >> 6);
        const uint64_t b = ((uint64_t)(o.x[2] >> 5) << 26) + (o.x[3] >> 6);
        const double u1 = ((double)a + 0.5) * 0x1.0p-53;
        const double u2 = (double)b * 0x1.0p-53;
        const double rho = sqrt(-2.0 * log(u1));
        const double th = 6.283185307179586 * u2;
        g0 = rho * cos(th);
        g1 = rho * sin(th);
    }
    if (c0 < lpad) out[(int64_t)c0 * ldo + j] = narrow<T>(g0);
    if (c1 < lpad) out[(int64_t)c1 * ldo + j] = narrow<T>(c1 < l ? g1 : 0.0);
}

hipError_t launch_omega(int tout, uint64_t seed, int64_t n, int l, int lpad, int64_t rows_pad, void* out,
                        int64_t ldo, hipStream_t st) {
    dim3 grid((unsigned)((rows_pad + 255) / 256), (unsigned)((lpad + 1) / 2));
    if (tout == DT_F64)
        hipLaunchKernelGGL(k_omega<double>, grid, dim3(256), 0, st, seed, n, l, lpad, rows_pad, (double*)out, ldo);
    else if (tout == DT_F32)
        hipLaunchKernelGGL(k_omega<float>, grid, dim3(256), 0, st, seed, n, l, lpad, rows_pad, (float*)out, ldo);
    else if (tout == DT_BF16)
        hipLaunchKernelGGL(k_omega<__bf16>, grid, dim3(256), 0, st, seed, n, l, lpad, rows_pad, (__bf16*)out, ldo);
    else if (tout == DT_F16)
        hipLaunchKernelGGL(k_omega<_Float16>, grid, dim3(256), 0, st, seed, n, l, lpad, rows_pad, (_Float16*)out,
                           ldo);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

__global__ void k_sketch_bits(uint64_t seed, int64_t n, int npairs, uint32_t* out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    if (j >= n) return;
    const philox_out o = philox4x32_10((uint32_t)j, (uint32_t)((uint64_t)j >> 32), (uint32_t)t, 0u,
                                       (uint32_t)seed, (uint32_t)(seed >> 32));
    uint32_t* p = out + (j * npairs + t) * 4;
    p[0] = o.x[0]; p[1] = o.x[1]; p[2] = o.x[2]; p[3] = o.x[3];
}

hipError_t launch_sketch_bits(uint64_t seed, int64_t n, int l, uint32_t* out, hipStream_t st) {
    const int npairs = (l + 1) / 2;
    hipLaunchKernelGGL(k_sketch_bits, dim3((unsigned)((n + 255) / 256), (unsigned)npairs), dim3(256), 0, st, seed,
                       n, npairs, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gram matrix in FP64 on MFMA: G[16a + mm][16b + nn] = sum_i Y[i][16a+mm] Y[i][16b+nn]
// for tile pairs a <= b. Each wave walks row blocks of 16 (grid-stride); a
// lane loads rows 4*(l/16)..+3 of column 16a + l%16 for every tile a, and
// MFMA (pair, s) uses row slot s of that vector as the K index.
// Pairs [PLO, PHI) of the NT(NT+1)/2 upper-triangle tile pairs belong to one
// blockIdx.y group; partials are reduced over the 4 waves in LDS in a fixed
// order and written per workgroup.
// ---------------------------------------------------------------------------
constexpr int GRAM_WGS = 256;

__host__ __device__ constexpr int npairs_of(int nt) { return nt * (nt + 1) / 2; }
__host__ __device__ constexpr int gram_groups(int nt) { return nt <= 4 ? 1 : 3; }
__host__ __device__ constexpr int gram_pg(int nt) {
    return (npairs_of(nt) + gram_groups(nt) - 1) / gram_groups(nt);
}

int64_t gram_partial_count(int nt) { return (int64_t)GRAM_WGS * npairs_of(nt) * 256; }

template <typename Tin, int NT, int PLO, int PHI>
__device__ __forceinline__ void gram_body(const Tin* __restrict__ Y, int64_t ld, int64_t M,
                                          double* __restrict__ Gpart, double* red) {
    constexpr int PG = PHI - PLO;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kg = lane >> 4;
    f64x4 acc[PG];
#pragma unroll
    for (int p = 0; p < PG; ++p) acc[p] = f64x4{0, 0, 0, 0};

    const int64_t nrb = (M + 15) / 16;
    for (int64_t rb = (int64_t)blockIdx.x * 4 + wave; rb < nrb; rb += (int64_t)gridDim.x * 4) {
        const int64_t i0 = rb * 16 + 4 * kg;
        double x[NT][4];
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            const V4<Tin> v = *reinterpret_cast<const V4<Tin>*>(Y + (int64_t)(16 * a + r16) * ld + i0);
#pragma unroll
            for (int s = 0; s < 4; ++s) x[a][s] = (double)v[s];
        }
        int p = 0;
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
            for (int b = a; b < NT; ++b) {
                if (p >= PLO && p < PHI) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) acc[p - PLO] = mfma_16x16x4(x[a][s], x[b][s], acc[p - PLO]);
                }
                ++p;
            }
    }
    // fixed-order reduction over the 4 waves
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int p = 0; p < PG; ++p)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int idx = p * 256 + mfma_row<double>(kg, v) * 16 + r16;
                    red[idx] = (w == 0 ? 0.0 : red[idx]) + acc[p][v];
                }
        }
        __syncthreads();
    }
    constexpr int NP = npairs_of(NT);
    for (int e = threadIdx.x; e < PG * 256; e += 256) {
        const int p = PLO + e / 256;
        Gpart[((int64_t)blockIdx.x * NP + p) * 256 + (e % 256)] = red[e];
    }
}

template <typename Tin, int NT>
__global__ __launch_bounds__(256) void k_gram(const Tin* __restrict__ Y, int64_t ld, int64_t M,
                                              double* __restrict__ Gpart, const int* cond, int cond_mask) {
    if (cond != nullptr && !(*cond & cond_mask)) return;
    constexpr int NP = npairs_of(NT), PG = gram_pg(NT);
    __shared__ double red[PG * 256];
    if (blockIdx.y == 0) gram_body<Tin, NT, 0, (PG < NP ? PG : NP)>(Y, ld, M, Gpart, red);
    if constexpr (gram_groups(NT) > 1) {
        if (blockIdx.y == 1) gram_body<Tin, NT, PG, (2 * PG < NP ? 2 * PG : NP)>(Y, ld, M, Gpart, red);
        if (blockIdx.y == 2) gram_body<Tin, NT, 2 * PG, NP>(Y, ld, M, Gpart, red);
    }
}

__global__ void k_gram_reduce(const double* __restrict__ Gpart, int nt, int nwg, double* __restrict__ G,
                              const int* cond, int cond_mask) {
    if (cond != nullptr && !(*cond & cond_mask)) return;
    const int np = nt * (nt + 1) / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= np * 256) return;
    const int p = e / 256, mm = (e % 256) / 16, nn = e % 16;
    int a = 0, q = p;
    while (q >= nt - a) { q -= nt - a; ++a; }
    const int b = a + q;
    // eight independent partial sums (loads in flight together), combined in a fixed order
    double acc8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double* src = Gpart + (int64_t)p * 256 + (e % 256);
    const int64_t wstride = (int64_t)np * 256;
    int w = 0;
    for (; w + 8 <= nwg; w += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) acc8[u] += src[(w + u) * wstride];
    for (; w < nwg; ++w) acc8[0] += src[w * wstride];
    const double s = ((acc8[0] + acc8[1]) + (acc8[2] + acc8[3])) + ((acc8[4] + acc8[5]) + (acc8[6] + acc8[7]));
    const int lp = 16 * nt;
    G[(16 * a + mm) * lp + 16 * b + nn] = s;
    G[(16 * b + nn) * lp + 16 * a + mm] = s;
}

template <typename Tin, int NT>
static hipError_t gram_nt(const void* Y, int64_t ld, int64_t M, double* Gpart, double* G, const int* cond,
                          int cond_mask, hipStream_t st) {
    int64_t nrb = (M + 15) / 16;
    int nwg = (int)((nrb + 3) / 4);
    if (nwg > GRAM_WGS) nwg = GRAM_WGS;
    if (nwg < 1) nwg = 1;
    hipLaunchKernelGGL((k_gram<Tin, NT>), dim3(nwg, gram_groups(NT)), dim3(256), 0, st, (const Tin*)Y, ld, M,
                       Gpart, cond, cond_mask);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int cnt = npairs_of(NT) * 256;
    hipLaunchKernelGGL(k_gram_reduce, dim3((cnt + 255) / 256), dim3(256), 0, st, Gpart, NT, nwg, G, cond,
                       cond_mask);
    return hipGetLastError();
}

template <typename Tin>
static hipError_t gram_dispatch(int nt, const void* Y, int64_t ld, int64_t M, double* Gpart, double* G,
                                const int* cond, int cond_mask, hipStream_t st) {
    switch (nt) {
#define RPOD_GRAM_CASE(K) case K: return gram_nt<Tin, K>(Y, ld, M, Gpart, G, cond, cond_mask, st);
        RPOD_GRAM_CASE(1) RPOD_GRAM_CASE(2) RPOD_GRAM_CASE(3) RPOD_GRAM_CASE(4)
        RPOD_GRAM_CASE(5) RPOD_GRAM_CASE(6) RPOD_GRAM_CASE(7) RPOD_GRAM_CASE(8)
#undef RPOD_GRAM_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gram(int tin, int nt, const void* Y, int64_t ld, int64_t M, double* Gpart, double* G,
                       const int* cond, int cond_mask, hipStream_t st) {
    if (tin == DT_F64) return gram_dispatch<double>(nt, Y, ld, M, Gpart, G, cond, cond_mask, st);
    if (tin == DT_F32) return gram_dispatch<float>(nt, Y, ld, M, Gpart, G, cond, cond_mask, st);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Cholesky and triangular inverse, one workgroup of 256 threads, FP64 in LDS.
// A holds G; the factorisation overwrites its upper triangle with R
// (G = R^T R). The inverse X = R^-1 is built by Gauss-Jordan elimination
// from the last column backwards, storing X[i][j] (i < j) transposed in the
// strict lower triangle of A and its diagonal in xd.
// ---------------------------------------------------------------------------
constexpr int LPMAX = 128;
constexpr int LDA = LPMAX + 1;

__global__ __launch_bounds__(256) void k_chol_inv(const double* __restrict__ G, int l, int lp, int64_t M,
                                                  double* __restrict__ Rinv64, float* __restrict__ Rinv32,
                                                  int* flags, int* local, int mode) {
    __shared__ double A[LPMAX * LDA];
    __shared__ double xd[LPMAX];
    __shared__ double gdiag[LPMAX];
    __shared__ int s_fail, s_nonfinite;
    __shared__ double s_trace;
    const int tid = threadIdx.x;
    const int ti = tid & 15, tj = tid >> 4;  // 16 x 16 thread grid for the 2-D updates

    if (mode == 2 && !(*local & DEV_FLAG_SHIFTED)) return;
    if (tid == 0) {
        s_fail = 0;
        s_nonfinite = 0;
        if (mode == 0) *local = 0;
    }
    __syncthreads();
    for (int e = tid; e < lp * lp; e += 256) {
        const double g = G[e];
        if (!isfinite(g)) s_nonfinite = 1;
    }
    __syncthreads();
    bool ok = (s_nonfinite == 0);
    if (!ok && tid == 0) atomicOr(flags, DEV_FLAG_NONFINITE);

    if (ok) {
        if (tid == 0) {
            double tr = 0.0;
            for (int k = 0; k < l; ++k) tr += G[k * lp + k];
            s_trace = tr;
        }
        for (int k = tid; k < l; k += 256) gdiag[k] = G[k * lp + k];
        __syncthreads();
        for (int attempt = 0; attempt < 2; ++attempt) {
            const double shift =
                attempt == 0 ? 0.0 : 11.0 * ((double)M * l + (double)l * (l + 1)) * 0x1.0p-53 * s_trace;
            for (int i = tj; i < l; i += 16)
                for (int j = ti; j < l; j += 16) A[i * LDA + j] = G[i * lp + j] + (i == j ? shift : 0.0);
            if (tid == 0) s_fail = 0;
            __syncthreads();
            for (int k = 0; k < l; ++k) {
                const double d = A[k * LDA + k];
                const double tol = (double)l * 0x1.0p-52 * gdiag[k];
                if (!(d > tol) || !(d > 0.0)) {  // non-positive, tiny or NaN pivot (uniform)
                    if (tid == 0) s_fail = 1;
                    break;
                }
                const double rinv = 1.0 / sqrt(d);
                __syncthreads();  // everyone has read the pivot
                for (int j = k + tid; j < l; j += 256) A[k * LDA + j] *= rinv;  // row k of R
                __syncthreads();
                // trailing update of the upper triangle, rows/columns k+1..l-1
                for (int i = k + 1 + tj; i < l; i += 16) {
                    const double rki = A[k * LDA + i];
                    for (int j = i + ((ti - (i - k - 1)) % 16 + 16) % 16; j < l; j += 16)
                        A[i * LDA + j] -= rki * A[k * LDA + j];
                }
                __syncthreads();
            }
            __syncthreads();
            if (!s_fail) break;
            if (attempt == 0) {
                if (tid == 0) {
                    atomicOr(flags, DEV_FLAG_SHIFTED);
                    *local |= DEV_FLAG_SHIFTED;
                }
            } else {
                if (tid == 0) atomicOr(flags, DEV_FLAG_BREAKDOWN);
                ok = false;
            }
            __syncthreads();
        }
    }

    if (ok) {
        // X = R^-1 by Gauss-Jordan from the last column; X[i][j] (i < j) is
        // kept transposed in the strict lower triangle of A, X[k][k] in xd
        for (int i = tj; i < l; i += 16)
            for (int j = ti; j < i; j += 16) A[i * LDA + j] = 0.0;
        for (int k = tid; k < l; k += 256) xd[k] = 1.0;
        __syncthreads();
        for (int k = l - 1; k >= 0; --k) {
            const double inv = 1.0 / A[k * LDA + k];
            if (tid == 0) xd[k] *= inv;
            for (int j = k + 1 + tid; j < l; j += 256) A[j * LDA + k] *= inv;
            __syncthreads();
            // rows i < k, columns j >= k: X[i][j] -= R[i][k] X[k][j]
            for (int j = k + tj; j < l; j += 16) {
                const double xkj = (j == k) ? xd[k] : A[j * LDA + k];
                for (int i = ti; i < k; i += 16) A[j * LDA + i] -= A[i * LDA + k] * xkj;
            }
            __syncthreads();
        }
        for (int e = tid; e < lp * lp; e += 256) {
            const int k = e % lp, c = e / lp;  // element (k, c), column-major
            double v;
            if (k >= l || c >= l) v = (k == c) ? 1.0 : 0.0;
            else if (k == c) v = xd[k];
            else if (k < c) v = A[c * LDA + k];
            else v = 0.0;
            Rinv64[e] = v;
            Rinv32[e] = (float)v;
        }
    } else {
        for (int e = tid; e < lp * lp; e += 256) {
            const double v = (e % lp == e / lp) ? 1.0 : 0.0;
            Rinv64[e] = v;
            Rinv32[e] = (float)v;
        }
    }
}

hipError_t launch_chol_inv(const double* G, int l, int lp, int64_t M, double* Rinv64, float* Rinv32, int* flags,
                           int* local, int mode, hipStream_t st) {
    if (lp > LPMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(256), 0, st, G, l, lp, M, Rinv64, Rinv32, flags, local, mode);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One-sided Jacobi on the columns of the symmetric PSD G_B (lp x lp, FP64,
// in LDS, one workgroup). Rotations act on column pairs chosen by the
// round-robin (circle) schedule, lp/2 disjoint pairs per round, TPP threads
// per pair reducing with lane shuffles. At convergence the columns are
// w_k = lambda_k u_k with G_B = U diag(lambda) U^T; sigma_k = sqrt(lambda_k).
// ---------------------------------------------------------------------------
constexpr int JLD = LPMAX + 1;

__device__ __forceinline__ double shfl_xor_d(double v, int mask) {
    return __shfl_xor(v, mask, 64);
}

__global__ __launch_bounds__(1024) void k_jacobi(const double* __restrict__ G, int l, int lp,
                                                 double* __restrict__ UB, double* __restrict__ sig, int* flags,
                                                 double tol) {
    __shared__ double W[LPMAX * JLD];  // column c at W[c * JLD + row]
    __shared__ double nrm[LPMAX];
    __shared__ int s_rot;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int npair = lp / 2;
    const int tpp = nthr / npair;  // 16, 32 or 64 (power of two)

    for (int e = tid; e < lp * lp; e += nthr) {
        const int c = e / lp, row = e % lp;
        W[c * JLD + row] = (c < l && row < l) ? G[row * lp + c] : 0.0;
    }
    __syncthreads();

    const int pr = tid / tpp;     // pair slot
    const int sub = tid % tpp;    // lane within the pair group
    int sweep = 0;
    const int max_sweeps = 40;
    for (; sweep < max_sweeps; ++sweep) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int rnd = 0; rnd < lp - 1; ++rnd) {
            // circle method: element lp-1 fixed, others rotate
            int p, q;
            if (pr == 0) { p = lp - 1; q = rnd; }
            else { p = (rnd + pr) % (lp - 1); q = (rnd - pr + (lp - 1)) % (lp - 1); }
            if (p > q) { const int t = p; p = q; q = t; }
            double al = 0.0, be = 0.0, ga = 0.0;
            for (int row = sub; row < lp; row += tpp) {
                const double wp = W[p * JLD + row], wq = W[q * JLD + row];
                al += wp * wp; be += wq * wq; ga += wp * wq;
            }
            for (int off = tpp / 2; off > 0; off >>= 1) {
                al += shfl_xor_d(al, off);
                be += shfl_xor_d(be, off);
                ga += shfl_xor_d(ga, off);
            }
            if (al > 0.0 && be > 0.0 && fabs(ga) > tol * sqrt(al * be)) {
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int row = sub; row < lp; row += tpp) {
                    const double wp = W[p * JLD + row], wq = W[q * JLD + row];
                    W[p * JLD + row] = c * wp - s * wq;
                    W[q * JLD + row] = s * wp + c * wq;
                }
                if (sub == 0) s_rot = 1;
            }
            __syncthreads();
        }
        if (s_rot == 0) break;
        __syncthreads();
    }
    if (sweep == max_sweeps && tid == 0) atomicOr(flags, DEV_FLAG_JACOBI_SLOW);

    for (int c = tid; c < lp; c += nthr) {
        double s = 0.0;
        for (int row = 0; row < lp; ++row) s += W[c * JLD + row] * W[c * JLD + row];
        nrm[c] = sqrt(s);
    }
    __syncthreads();
    for (int c = tid; c < lp; c += nthr) {
        const double v = nrm[c];
        int rank = 0;
        for (int k = 0; k < lp; ++k) rank += (nrm[k] > v) || (nrm[k] == v && k < c);
        sig[rank] = sqrt(v);
        const double inv = v > 0.0 ? 1.0 / v : 0.0;
        for (int row = 0; row < lp; ++row) UB[(int64_t)rank * lp + row] = W[c * JLD + row] * inv;
    }
}

hipError_t launch_jacobi(const double* G, int l, int lp, double* UB, double* sig, int* flags, double tol,
                         hipStream_t st) {
    if (lp > LPMAX || lp % 16) return hipErrorInvalidValue;
    const int npair = lp / 2;
    int tpp = 64;  // threads per column pair: a power of two that divides the wave
    while (tpp * npair > 1024) tpp /= 2;
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(tpp * npair), 0, st, G, l, lp, UB, sig, flags, tol);
    return hipGetLastError();
}

// M = Rinv * UB[:, :r] and Ur = UB[:, :r], both lp x rp column-major (zero pad).
__global__ void k_lift_coef(const double* __restrict__ Rinv, const double* __restrict__ UB, int lp, int r, int rp,
                            double* __restrict__ M64, float* __restrict__ M32, double* __restrict__ Ur) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= lp * rp) return;
    const int k = e % lp, c = e / lp;
    double s = 0.0, u = 0.0;
    if (c < r) {
        for (int j = 0; j < lp; ++j) s += Rinv[(int64_t)j * lp + k] * UB[(int64_t)c * lp + j];
        u = UB[(int64_t)c * lp + k];
    }
    M64[e] = s;
    M32[e] = (float)s;
    Ur[e] = u;
}

hipError_t launch_lift_coef(const double* Rinv, const double* UB, int lp, int r, int rp, double* M64, float* M32,
                            double* Ur, hipStream_t st) {
    hipLaunchKernelGGL(k_lift_coef, dim3((lp * rp + 255) / 256), dim3(256), 0, st, Rinv, UB, lp, r, rp, M64, M32, Ur);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sign convention: per column, the entry of largest magnitude (lowest row on
// ties) is made positive. Partial argmax per (column, row chunk), then one
// thread per column combines chunks in order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_colmax(const T* __restrict__ Phi, int64_t ld, int64_t m, int64_t chunk,
                                                double* __restrict__ pval, int64_t* __restrict__ pidx) {
    const int c = blockIdx.y, ch = blockIdx.x;
    const int64_t i0 = (int64_t)ch * chunk;
    const int64_t i1 = (i0 + chunk < m) ? i0 + chunk : m;
    double best = -1.0, bval = 0.0;
    int64_t bidx = INT64_MAX;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const double v = (double)Phi[(int64_t)c * ld + i];
        const double a = fabs(v);
        if (a > best) { best = a; bidx = i; bval = v; }  // increasing i: strict > keeps first
    }
    __shared__ double sb[256], sv[256];
    __shared__ int64_t si[256];
    sb[threadIdx.x] = best; sv[threadIdx.x] = bval; si[threadIdx.x] = bidx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            const int o = threadIdx.x + off;
            if (sb[o] > sb[threadIdx.x] || (sb[o] == sb[threadIdx.x] && si[o] < si[threadIdx.x])) {
                sb[threadIdx.x] = sb[o]; sv[threadIdx.x] = sv[o]; si[threadIdx.x] = si[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t slot = (int64_t)c * gridDim.x + ch;
        pval[slot] = (sb[0] < 0.0) ? 0.0 : sv[0];
        pidx[slot] = si[0];
    }
}

__global__ void k_signs(const double* __restrict__ pval, const int64_t* __restrict__ pidx, int nchunk, int r,
                        double* __restrict__ signs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= r) return;
    double best = -1.0, bval = 0.0;
    int64_t bidx = INT64_MAX;
    for (int k = 0; k < nchunk; ++k) {
        const double v = pval[(int64_t)c * nchunk + k];
        const int64_t ix = pidx[(int64_t)c * nchunk + k];
        const double a = fabs(v);
        if (a > best || (a == best && ix < bidx)) { best = a; bval = v; bidx = ix; }
    }
    signs[c] = (bval < 0.0) ? -1.0 : 1.0;
}

hipError_t launch_signs(int tphi, const void* Phi, int64_t ld, int64_t m, int r, int nchunk, double* part_val,
                        int64_t* part_idx, double* signs, hipStream_t st) {
    const int64_t chunk = (m + nchunk - 1) / nchunk;
    dim3 grid(nchunk, r);
    if (tphi == DT_F64)
        hipLaunchKernelGGL(k_colmax<double>, grid, dim3(256), 0, st, (const double*)Phi, ld, m, chunk, part_val, part_idx);
    else
        hipLaunchKernelGGL(k_colmax<float>, grid, dim3(256), 0, st, (const float*)Phi, ld, m, chunk, part_val, part_idx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_signs, dim3((r + 63) / 64), dim3(64), 0, st, part_val, part_idx, nchunk, r, signs);
    return hipGetLastError();
}

template <typename T>
__global__ void k_fin_phi(const T* __restrict__ Pin, int64_t ldP, int64_t m, int r, const double* __restrict__ signs,
                          T* __restrict__ Pout) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= m) return;
    Pout[(int64_t)c * m + i] = (T)(signs[c] * (double)Pin[(int64_t)c * ldP + i]);
}

template <typename T>
__global__ void k_fin_a(const double* __restrict__ At, int64_t ldA, int64_t n, int r, const double* __restrict__ signs,
                        const double* __restrict__ sig, T* __restrict__ Aout, double* __restrict__ sigma_out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (int64_t)r && blockIdx.y == 0) sigma_out[e] = sig[e];
    if (e >= n * r) return;
    const int64_t j = e / r;
    const int k = (int)(e % r);
    Aout[e] = (T)(signs[k] * At[(int64_t)k * ldA + j]);
}

hipError_t launch_finalize(int tphi, const void* Phi_int, int64_t ldP, int64_t m, int r, const double* At,
                           int64_t ldA, int64_t n, const double* signs, const double* sig, void* Phi_out,
                           void* A_out, double* sigma_out, hipStream_t st) {
    dim3 gp((unsigned)((m + 255) / 256), r);
    const int64_t na = n * r > r ? n * r : r;
    dim3 ga((unsigned)((na + 255) / 256));
    if (tphi == DT_F64) {
        hipLaunchKernelGGL(k_fin_phi<double>, gp, dim3(256), 0, st, (const double*)Phi_int, ldP, m, r, signs,
                           (double*)Phi_out);
        hipLaunchKernelGGL(k_fin_a<double>, ga, dim3(256), 0, st, At, ldA, n, r, signs, sig, (double*)A_out, sigma_out);
    } else {
        hipLaunchKernelGGL(k_fin_phi<float>, gp, dim3(256), 0, st, (const float*)Phi_int, ldP, m, r, signs,
                           (float*)Phi_out);
        hipLaunchKernelGGL(k_fin_a<float>, ga, dim3(256), 0, st, At, ldA, n, r, signs, sig, (float*)A_out, sigma_out);
    }
    return hipGetLastError();
}

}  // namespace rpod
