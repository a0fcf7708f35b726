// Passes over a 16-bit snapshot matrix (bfloat16 or IEEE half) on the
// 16x16x32 matrix cores of gfx950, FP32 accumulation.
//
//   k_sx16   Y = S X    (X stored in the same 16-bit type)
//   k_stq16  Z = S^T Q  (Q stored in FP32, rounded to the 16-bit type on the
//                        fly; with LO the rounding remainder is applied as a
//                        second product, so Q carries ~16 significant bits:
//                        the refinement pass for T = Q^T S)
//
// MFMA operand layout (measured on gfx950 for 16x16x32 bf16/f16): lane l
// supplies A[l%16][8*(l/16) + i] and B[8*(l/16) + i][l%16], i = 0..7, and
// the result holds D[4*(l/16) + v][l%16] in component v.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace rpod {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

template <typename T16> struct mma16;
template <> struct mma16<__bf16> {
    typedef bf16x8 vec;
    static __device__ __forceinline__ f32x4 run(u16x8 a, u16x8 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
    static __device__ __forceinline__ unsigned short from_float(float x) {
        return __builtin_bit_cast(unsigned short, (__bf16)x);
    }
    static __device__ __forceinline__ float to_float(unsigned short h) {
        return (float)__builtin_bit_cast(__bf16, h);
    }
};
template <> struct mma16<_Float16> {
    typedef f16x8 vec;
    static __device__ __forceinline__ f32x4 run(u16x8 a, u16x8 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    }
    static __device__ __forceinline__ unsigned short from_float(float x) {
        return __builtin_bit_cast(unsigned short, (_Float16)x);
    }
    static __device__ __forceinline__ float to_float(unsigned short h) {
        return (float)__builtin_bit_cast(_Float16, h);
    }
};

// Eight consecutive rows i..i+7 of column j (16-bit), zero outside [0,lim) x [0,n).
template <bool VEC>
__device__ __forceinline__ u16x8 load_rows8(const unsigned short* S, int64_t ld, int64_t lim, int64_t n,
                                            int64_t i, int64_t j) {
    u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    if (j < n) {
        const unsigned short* p = S + j * ld + i;
        if (VEC && i + 7 < lim) {
            v = *reinterpret_cast<const u16x8*>(p);
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (i + t < lim) v[t] = p[t];
        }
    }
    return v;
}

// ---------------------------------------------------------------------------
// Y = S X, 16-bit S and X, FP32 Y. Workgroup: 256 rows, columns in chunks of
// 32 (one MFMA K). Each chunk of S is staged in LDS column-major (row runs
// of 16 bytes written by each thread, coalesced 512-byte column reads from
// HBM) and read back transposed: lane (r, kg) of m-tile mt gathers row
// 64 w + 16 mt + r of columns 8 kg .. 8 kg + 7. X is column-major, so its
// operand is one 16-byte load per output tile.
// ---------------------------------------------------------------------------
constexpr int SX16_BM = 256, SX16_BK = 32, SX16_LDR = SX16_BM + 4;  // LDS column stride (elements)

template <typename T16, int NT, bool VEC>
__global__ __launch_bounds__(256) void k_sx16(const unsigned short* __restrict__ S, int64_t ldS, int64_t m,
                                              int64_t n, const unsigned short* __restrict__ X, int64_t ldX,
                                              float* __restrict__ Y, int64_t ldY, int64_t mstore) {
    __shared__ unsigned short tile[SX16_BK * SX16_LDR];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, kg = lane >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * SX16_BM;
    const int rg = tid & 31, cc = tid >> 5;  // staging: rows 8 rg..+7 of columns cc + 8 q

    f32x4 acc[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[mt][c] = f32x4{0, 0, 0, 0};

    const bool active = i0 < m;
    for (int64_t j0 = 0; active && j0 < n; j0 += SX16_BK) {
        u16x8 st[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) st[q] = load_rows8<VEC>(S, ldS, m, n, i0 + 8 * rg, j0 + cc + 8 * q);
        u16x8 b[NT];
#pragma unroll
        for (int c = 0; c < NT; ++c)
            b[c] = *reinterpret_cast<const u16x8*>(X + (int64_t)(16 * c + r16) * ldX + j0 + 8 * kg);
        __syncthreads();  // previous chunk fully consumed
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned short* dst = tile + (cc + 8 * q) * SX16_LDR + 8 * rg;
            *reinterpret_cast<u16x4*>(dst) = u16x4{st[q][0], st[q][1], st[q][2], st[q][3]};
            *reinterpret_cast<u16x4*>(dst + 4) = u16x4{st[q][4], st[q][5], st[q][6], st[q][7]};
        }
        __syncthreads();
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const unsigned short* src = tile + (8 * kg) * SX16_LDR + wave * 64 + 16 * mt + r16;
            u16x8 a;
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = src[i * SX16_LDR];
#pragma unroll
            for (int c = 0; c < NT; ++c) acc[mt][c] = mma16<T16>::run(a, b[c], acc[mt][c]);
        }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const int64_t row = i0 + wave * 64 + 16 * mt + 4 * kg;
            float* py = Y + (int64_t)(16 * c + r16) * ldY + row;
            if (row + 3 < mstore) {
                *reinterpret_cast<f32x4*>(py) = acc[mt][c];
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (row + v < mstore) py[v] = acc[mt][c][v];
            }
        }
}

// ---------------------------------------------------------------------------
// Z_s = S_s^T Q_s, 16-bit S, FP32 Q. Workgroup: 256 columns (4 waves x 4
// tiles of 16), rows of split s in steps of 32 (one MFMA K):
//   A[mm][8 kg + i] = S[i0 + 8 kg + i][jw + 16 u + mm]  (one 16-byte load)
//   B[8 kg + i][nn] = round16(Q[i0 + 8 kg + i][16 c + nn])  (+ remainder if LO)
// ---------------------------------------------------------------------------
template <typename T16, int NT, bool VEC, bool LO>
__global__ __launch_bounds__(256) void k_stq16(const unsigned short* __restrict__ S, int64_t ldS, int64_t m,
                                               int64_t n, const float* __restrict__ Q, int64_t ldQ,
                                               double* __restrict__ Zp, int64_t nP, int64_t split_rows) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kg = lane >> 4;
    const int64_t jw = (int64_t)blockIdx.x * 256 + wave * 64;
    const int64_t ib = (int64_t)blockIdx.y * split_rows;
    const int64_t ie = (ib + split_rows < m) ? ib + split_rows : m;

    f32x4 acc[4][NT];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[u][c] = f32x4{0, 0, 0, 0};

    if (jw < n) {
        for (int64_t i0 = ib; i0 < ie; i0 += 32) {
            u16x8 a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = load_rows8<VEC>(S, ldS, ie, n, i0 + 8 * kg, jw + 16 * u + r16);
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const float* pq = Q + (int64_t)(16 * c + r16) * ldQ + i0 + 8 * kg;
                const f32x4 q0 = *reinterpret_cast<const f32x4*>(pq);
                const f32x4 q1 = *reinterpret_cast<const f32x4*>(pq + 4);
                u16x8 hi, lo;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float x = i < 4 ? q0[i] : q1[i - 4];
                    hi[i] = mma16<T16>::from_float(x);
                    if (LO) lo[i] = mma16<T16>::from_float(x - mma16<T16>::to_float(hi[i]));
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    acc[u][c] = mma16<T16>::run(a[u], hi, acc[u][c]);
                    if (LO) acc[u][c] = mma16<T16>::run(a[u], lo, acc[u][c]);
                }
            }
        }
    }
    double* zp = Zp + (int64_t)blockIdx.y * nP * (16 * NT);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            double* pz = zp + (int64_t)(16 * c + r16) * nP + jw + 16 * u + 4 * kg;
            typedef double d4 __attribute__((ext_vector_type(4)));
            *reinterpret_cast<d4*>(pz) = d4{acc[u][c][0], acc[u][c][1], acc[u][c][2], acc[u][c][3]};
        }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T16, int NT>
static hipError_t sx16_nt(const void* S, int64_t ldS, int64_t m, int64_t n, const void* X, int64_t ldX, void* Y,
                          int64_t ldY, int64_t mstore, hipStream_t st) {
    const int64_t rows = mstore > m ? mstore : m;
    dim3 grid((unsigned)((rows + SX16_BM - 1) / SX16_BM));
    const bool vec = (ldS % 8 == 0) && ((uintptr_t)S % 16 == 0);
    if (vec)
        hipLaunchKernelGGL((k_sx16<T16, NT, true>), grid, dim3(256), 0, st, (const unsigned short*)S, ldS, m, n,
                           (const unsigned short*)X, ldX, (float*)Y, ldY, mstore);
    else
        hipLaunchKernelGGL((k_sx16<T16, NT, false>), grid, dim3(256), 0, st, (const unsigned short*)S, ldS, m, n,
                           (const unsigned short*)X, ldX, (float*)Y, ldY, mstore);
    return hipGetLastError();
}

template <typename T16, int NT, bool LO>
static hipError_t stq16_nt(const void* S, int64_t ldS, int64_t m, int64_t n, const void* Q, int64_t ldQ, double* Zp,
                           int64_t nP, int64_t split_rows, int nsplit, hipStream_t st) {
    dim3 grid((unsigned)(nP / 256), (unsigned)nsplit);
    const bool vec = (ldS % 8 == 0) && ((uintptr_t)S % 16 == 0);
    if (vec)
        hipLaunchKernelGGL((k_stq16<T16, NT, true, LO>), grid, dim3(256), 0, st, (const unsigned short*)S, ldS, m,
                           n, (const float*)Q, ldQ, Zp, nP, split_rows);
    else
        hipLaunchKernelGGL((k_stq16<T16, NT, false, LO>), grid, dim3(256), 0, st, (const unsigned short*)S, ldS, m,
                           n, (const float*)Q, ldQ, Zp, nP, split_rows);
    return hipGetLastError();
}

template <typename T16>
static hipError_t sx16_dispatch(int nt, const void* S, int64_t ldS, int64_t m, int64_t n, const void* X,
                                int64_t ldX, void* Y, int64_t ldY, int64_t mstore, hipStream_t st) {
    switch (nt) {
#define RPOD_C(K) case K: return sx16_nt<T16, K>(S, ldS, m, n, X, ldX, Y, ldY, mstore, st);
        RPOD_C(1) RPOD_C(2) RPOD_C(3) RPOD_C(4) RPOD_C(5) RPOD_C(6) RPOD_C(7) RPOD_C(8)
#undef RPOD_C
        default: return hipErrorInvalidValue;
    }
}

template <typename T16, bool LO>
static hipError_t stq16_dispatch(int nt, const void* S, int64_t ldS, int64_t m, int64_t n, const void* Q,
                                 int64_t ldQ, double* Zp, int64_t nP, int64_t split_rows, int nsplit,
                                 hipStream_t st) {
    switch (nt) {
#define RPOD_C(K) case K: return stq16_nt<T16, K, LO>(S, ldS, m, n, Q, ldQ, Zp, nP, split_rows, nsplit, st);
        RPOD_C(1) RPOD_C(2) RPOD_C(3) RPOD_C(4) RPOD_C(5) RPOD_C(6) RPOD_C(7) RPOD_C(8)
#undef RPOD_C
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sx16(int tin, int nt, const void* S, int64_t ldS, int64_t m, int64_t n, const void* X,
                       int64_t ldX, float* Y, int64_t ldY, int64_t mstore, hipStream_t st) {
    if (tin == DT_BF16) return sx16_dispatch<__bf16>(nt, S, ldS, m, n, X, ldX, Y, ldY, mstore, st);
    if (tin == DT_F16) return sx16_dispatch<_Float16>(nt, S, ldS, m, n, X, ldX, Y, ldY, mstore, st);
    return hipErrorInvalidValue;
}

hipError_t launch_stq16(int tin, int nt, bool lo, const void* S, int64_t ldS, int64_t m, int64_t n, const float* Q,
                        int64_t ldQ, double* Zp, int64_t nP, int64_t split_rows, int nsplit, hipStream_t st) {
    if (tin == DT_BF16)
        return lo ? stq16_dispatch<__bf16, true>(nt, S, ldS, m, n, Q, ldQ, Zp, nP, split_rows, nsplit, st)
                  : stq16_dispatch<__bf16, false>(nt, S, ldS, m, n, Q, ldQ, Zp, nP, split_rows, nsplit, st);
    if (tin == DT_F16)
        return lo ? stq16_dispatch<_Float16, true>(nt, S, ldS, m, n, Q, ldQ, Zp, nP, split_rows, nsplit, st)
                  : stq16_dispatch<_Float16, false>(nt, S, ldS, m, n, Q, ldQ, Zp, nP, split_rows, nsplit, st);
    return hipErrorInvalidValue;
}

}  // namespace rpod
