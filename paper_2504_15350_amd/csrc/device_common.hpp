// Device-side helpers shared by the rPOD kernels (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float  f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct vec4_of;
template <> struct vec4_of<float>  { typedef f32x4 type; };
template <> struct vec4_of<double> { typedef f64x4 type; };
template <> struct vec4_of<__bf16> { typedef __bf16 type __attribute__((ext_vector_type(4))); };
template <> struct vec4_of<_Float16> { typedef _Float16 type __attribute__((ext_vector_type(4))); };

// Narrowing used for every store into a 16-bit operand: through FP32, each
// step rounding to nearest even.
// Global-memory (address space 1) pointers. Operands reached through
// argument records in memory are generic pointers to the compiler, which
// would access them with flat instructions; the hot kernels convert them once.
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* gbl(T* p) { return (GLOBAL T*)p; }

template <typename Tout, typename T>
__device__ __forceinline__ Tout narrow(T x) { return (Tout)(float)x; }
template <> __device__ __forceinline__ double narrow<double, double>(double x) { return x; }

// One 16x16x4 matrix-core step, D = A*B + C, wave64 operand layout:
//   lane l supplies A[l%16][l/16] and B[l/16][l%16];
//   the result holds D[mfma_row<T>(l/16, v)][l%16] in component v, where the
//   row is 4*(l/16)+v for the FP32 instruction and (l/16)+4*v for FP64
//   (both measured on gfx950).
__device__ __forceinline__ f32x4 mfma_16x16x4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma_16x16x4(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ int mfma_row(int kg, int v);
template <> __device__ __forceinline__ int mfma_row<float>(int kg, int v) { return 4 * kg + v; }
template <> __device__ __forceinline__ int mfma_row<double>(int kg, int v) { return kg + 4 * v; }

// Status word bits (mirror the public RPOD_FLAG_* values).
#define DEV_FLAG_SHIFTED     0x1
#define DEV_FLAG_BREAKDOWN   0x2
#define DEV_FLAG_NONFINITE   0x4
#define DEV_FLAG_JACOBI_SLOW 0x8
#define DEV_FLAG_RANK_CUT    0x20

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter c, key k.
struct philox_out { uint32_t x[4]; };

__device__ __forceinline__ philox_out philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                    uint32_t c3, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        if (rnd > 0) { k0 += W0; k1 += W1; }
        const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
        const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    philox_out o;
    o.x[0] = c0; o.x[1] = c1; o.x[2] = c2; o.x[3] = c3;
    return o;
}
