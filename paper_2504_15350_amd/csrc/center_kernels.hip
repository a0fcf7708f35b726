// Fluctuation snapshots (Sec. 4.1) without forming them.
//
// The snapshot matrix holds M = n / N blocks of N consecutive columns (one
// block per parameter, its N time instants); the fluctuation matrix is
// S' = S - Msum E^T / N, with Msum (m x M) the block sums of S's columns and
// E (n x M) the block indicator. The library never writes S' out:
//   - the first pass over S multiplies S by [Omega, E] (the indicator columns
//     written by k_center_prep after the sketch), so Msum comes out of that
//     pass as M extra output columns;
//   - S' X = S X - Msum (E^T X / N): k_center_prep forms C = E^T X / N from
//     the operand the pass used, k_center_y subtracts Msum C from the pass's
//     output (FP64 arithmetic, one rounding to the storage type);
//   - S'^T Q = S^T Q - E (Msum^T Q) / N: k_center_cross forms Msum^T Q in
//     FP64 (row-chunk slabs, summed by the slab reduction), k_center_z
//     subtracts it block by block from the reduced S^T Q.
// Every reduction has a fixed order, so results are deterministic.
#include "device_common.hpp"
#include "internal.hpp"

namespace rpod {

template <typename A>
static Group<A> mkgc(const GroupLaunch<A>& L) {
    Group<A> g;
    g.args = L.args;
    g.tstart = L.tstart;
    g.calls = L.calls;
    g.count = L.count;
    return g;
}

template <typename T>
__device__ __forceinline__ double to_d(T x) {
    if constexpr (sizeof(T) == 2) return (double)(float)x;
    else return (double)x;
}

// one workgroup per block k: C[k + c K] for c < lp (wave w: columns w, w + 4, ..),
// then (ind) column lp + k of X = the indicator of block k over all ld rows
template <typename T>
__global__ __launch_bounds__(256) void k_center_prep(Group<CprepArgs> g) {
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const CprepArgs& a = g.args[it];
    const int k = blockIdx.x - g.tstart[it];
    GLOBAL T* X = gbl((T*)a.X);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t j0 = (int64_t)k * a.N;
    for (int c = wave; c < a.lp; c += 4) {
        const GLOBAL T* col = X + (int64_t)c * a.ld + j0;
        double s = 0.0;
        for (int64_t j = lane; j < a.N; j += 64) s += to_d(col[j]);
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) a.C[k + (int64_t)c * a.K] = s / (double)a.N;
    }
    if (a.ind) {
        GLOBAL T* col = X + (int64_t)(a.lp + k) * a.ld;
        for (int64_t j = threadIdx.x; j < a.ld; j += 256) col[j] = (T)((j >= j0 && j < j0 + a.N) ? 1.0f : 0.0f);
    }
}

// 256 rows per tile: Y[i, c] -= sum_k Msum[i, k] C[k + c K], 16 columns at a time
template <typename T>
__global__ __launch_bounds__(256) void k_center_y(Group<CenterYArgs> g) {
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const CenterYArgs& a = g.args[it];
    __shared__ double cs[4096];  // K lp <= 4096
    for (int e = threadIdx.x; e < a.K * a.lp; e += 256) cs[e] = a.C[e];
    __syncthreads();
    const int64_t i = (int64_t)(blockIdx.x - g.tstart[it]) * 256 + threadIdx.x;
    if (i >= a.m) return;
    GLOBAL T* Y = gbl((T*)a.Y);
    const GLOBAL T* Ms = Y + (int64_t)a.lp * a.ld;
    for (int c0 = 0; c0 < a.lp; c0 += 16) {
        double acc[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[c] = 0.0;
        for (int k = 0; k < a.K; ++k) {
            const double mk = to_d(Ms[(int64_t)k * a.ld + i]);
#pragma unroll
            for (int c = 0; c < 16; ++c) acc[c] += mk * cs[k + (c0 + c) * a.K];
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            GLOBAL T* y = Y + (int64_t)(c0 + c) * a.ld + i;
            *y = (T)(to_d(*y) - acc[c]);
        }
    }
}

// one tile per chunk of rows: the chunk's slab of Msum^T Q (K x lp, FP64),
// 32-row steps staged in LDS; thread t owns outputs t, t + 256, ..
constexpr int CX_R = 32, CX_LD = CX_R + 1;
template <typename T>
__global__ __launch_bounds__(256) void k_center_cross(Group<CrossArgs> g) {
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const CrossArgs& a = g.args[it];
    const int ch = blockIdx.x - g.tstart[it];
    const int64_t i0 = (int64_t)ch * a.chunk;
    const int64_t i1 = (i0 + a.chunk < a.m) ? i0 + a.chunk : a.m;
    __shared__ double ms[CX_LD * 64], qs[CX_LD * 112];  // K <= 64, lp <= 112
    const GLOBAL T* M = gbl((const T*)a.M);
    const GLOBAL T* Q = gbl((const T*)a.Q);
    const int no = a.K * a.lp;  // <= 4096
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (int64_t r0 = i0; r0 < i1; r0 += CX_R) {
        __syncthreads();
        for (int e = threadIdx.x; e < CX_R * a.K; e += 256) {
            const int rr = e % CX_R, k = e / CX_R;
            const int64_t i = r0 + rr;
            ms[rr + CX_LD * k] = i < i1 ? to_d(M[(int64_t)k * a.ld + i]) : 0.0;
        }
        for (int e = threadIdx.x; e < CX_R * a.lp; e += 256) {
            const int rr = e % CX_R, c = e / CX_R;
            const int64_t i = r0 + rr;
            qs[rr + CX_LD * c] = i < i1 ? to_d(Q[(int64_t)c * a.ld + i]) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int o = threadIdx.x + 256 * u;
            if (o < no) {
                const int k = o % a.K, c = o / a.K;
                double s = acc[u];
                for (int rr = 0; rr < CX_R; ++rr) s += ms[rr + CX_LD * k] * qs[rr + CX_LD * c];
                acc[u] = s;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int o = threadIdx.x + 256 * u;
        if (o < no) a.Pp[(int64_t)ch * no + o] = acc[u];
    }
}

// 256 entries per tile over the ld x lp array Z
__global__ __launch_bounds__(256) void k_center_z(Group<CenterZArgs> g) {
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const CenterZArgs& a = g.args[it];
    const int64_t e = (int64_t)(blockIdx.x - g.tstart[it]) * 256 + threadIdx.x;
    const int64_t j = e % a.ld;
    const int64_t c = e / a.ld;
    if (c >= a.lp || j >= a.n) return;
    a.Z[c * a.ld + j] -= a.P[j / a.N + c * a.K] / (double)a.N;
}

hipError_t launch_center_prep(int tx, const GroupLaunch<CprepArgs>& L, hipStream_t st) {
    switch (tx) {
        case DT_F64: hipLaunchKernelGGL(k_center_prep<double>, dim3(L.tiles), dim3(256), 0, st, mkgc(L)); break;
        case DT_F32: hipLaunchKernelGGL(k_center_prep<float>, dim3(L.tiles), dim3(256), 0, st, mkgc(L)); break;
        case DT_BF16: hipLaunchKernelGGL(k_center_prep<__bf16>, dim3(L.tiles), dim3(256), 0, st, mkgc(L)); break;
        case DT_F16: hipLaunchKernelGGL(k_center_prep<_Float16>, dim3(L.tiles), dim3(256), 0, st, mkgc(L)); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_center_y(int tacc, const GroupLaunch<CenterYArgs>& L, hipStream_t st) {
    if (tacc == DT_F64)
        hipLaunchKernelGGL(k_center_y<double>, dim3(L.tiles), dim3(256), 0, st, mkgc(L));
    else
        hipLaunchKernelGGL(k_center_y<float>, dim3(L.tiles), dim3(256), 0, st, mkgc(L));
    return hipGetLastError();
}

hipError_t launch_center_cross(int tacc, const GroupLaunch<CrossArgs>& L, hipStream_t st) {
    if (tacc == DT_F64)
        hipLaunchKernelGGL(k_center_cross<double>, dim3(L.tiles), dim3(256), 0, st, mkgc(L));
    else
        hipLaunchKernelGGL(k_center_cross<float>, dim3(L.tiles), dim3(256), 0, st, mkgc(L));
    return hipGetLastError();
}

hipError_t launch_center_z(const GroupLaunch<CenterZArgs>& L, hipStream_t st) {
    hipLaunchKernelGGL(k_center_z, dim3(L.tiles), dim3(256), 0, st, mkgc(L));
    return hipGetLastError();
}

}  // namespace rpod
