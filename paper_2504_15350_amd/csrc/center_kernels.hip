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
//     FP64 (partial sums over row chunks, added up by k_center_sum), k_center_z
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
    g.skip = L.skip;
    g.skip_mask = L.skip_mask;
    return g;
}

template <typename T>
__device__ __forceinline__ double to_d(T x) {
    if constexpr (sizeof(T) == 2) return (double)(float)x;
    else return (double)x;
}

// tile t = (block k, quad cq): wave w sums column 4 cq + w of block k over its
// N rows (lanes over rows, a fixed butterfly); tiles with cq = 0 also write
// column lp + k of X = the indicator of block k over all ld rows (ind)
template <typename T>
__global__ __launch_bounds__(256) void k_center_prep(Group<CprepArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const CprepArgs& a = g.args[it];
    const int t = blockIdx.x - g.tstart[it];
    const int k = t % a.K, cq = t / a.K;
    GLOBAL T* X = gbl((T*)a.X);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t j0 = (int64_t)k * a.N;
    const int c = 4 * cq + wave;
    if (c < a.lp) {
        const GLOBAL T* col = X + (int64_t)c * a.ld + j0;
        double s = 0.0;
        for (int64_t j = lane; j < a.N; j += 64) s += to_d(col[j]);
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) a.C[k + (int64_t)c * a.K] = s / (double)a.N;
    }
    if (a.ind && cq == 0) {
        GLOBAL T* ind = X + (int64_t)(a.lp + k) * a.ld;
        for (int64_t j = threadIdx.x; j < a.ld; j += 256) ind[j] = (T)((j >= j0 && j < j0 + a.N) ? 1.0f : 0.0f);
    }
}

// 256 rows per tile, one per thread: Y[i, c] -= sum_k Msum[i, k] C[k + c K];
// the row's block sums are loaded once per group of 16 blocks, then the
// columns are corrected 16 at a time (their loads issued together)
template <typename T>
__global__ __launch_bounds__(256) void k_center_y(Group<CenterYArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const CenterYArgs& a = g.args[it];
    __shared__ double cs[4096];  // K lp <= 4096
    for (int e = threadIdx.x; e < a.K * a.lp; e += 256) cs[e] = a.C[e];
    __syncthreads();
    const int64_t i = (int64_t)(blockIdx.x - g.tstart[it]) * 256 + threadIdx.x;
    if (i >= a.m) return;
    GLOBAL T* Y = gbl((T*)a.Y);
    const GLOBAL T* Ms = Y + (int64_t)a.lp * a.ld;
    for (int k0 = 0; k0 < a.K; k0 += 16) {
        const int kn = a.K - k0 < 16 ? a.K - k0 : 16;
        double mk[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) mk[k] = k < kn ? to_d(Ms[(int64_t)(k0 + k) * a.ld + i]) : 0.0;
        for (int c0 = 0; c0 < a.lp; c0 += 16) {
            double acc[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) acc[c] = to_d(Y[(int64_t)(c0 + c) * a.ld + i]);
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (k < kn) {
                    const double* cr = cs + (k0 + k) + (int64_t)c0 * a.K;
#pragma unroll
                    for (int c = 0; c < 16; ++c) acc[c] -= mk[k] * cr[c * a.K];
                }
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) Y[(int64_t)(c0 + c) * a.ld + i] = (T)acc[c];
        }
    }
}

// one tile per chunk of rows: the chunk's slab of Msum^T Q (K x lp, FP64
// products and sums), 32-row steps staged in LDS in the storage type; register
// blocks of 1 x 4 outputs (row k, columns 4 cb .. 4 cb + 3), block b = k + K cb,
// thread t owning blocks t, t + 256, .. (K lp / 4 <= 1024 blocks)
constexpr int CX_R = 32, CX_LD = CX_R + 1;
template <typename T>
__global__ __launch_bounds__(256) void k_center_cross(Group<CrossArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const CrossArgs& a = g.args[it];
    const int ch = blockIdx.x - g.tstart[it];
    const int64_t i0 = (int64_t)ch * a.chunk;
    const int64_t i1 = (i0 + a.chunk < a.m) ? i0 + a.chunk : a.m;
    __shared__ T ms[CX_LD * 64], qs[CX_LD * 112];  // K <= 64, lp <= 112
    const GLOBAL T* M = gbl((const T*)a.M);
    const GLOBAL T* Q = gbl((const T*)a.Q);
    const int nb = a.K * (a.lp / 4);
    constexpr int BPT = 4;
    double acc[BPT][4];
#pragma unroll
    for (int u = 0; u < BPT; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    for (int64_t r0 = i0; r0 < i1; r0 += CX_R) {
        __syncthreads();
        for (int e = threadIdx.x; e < CX_R * a.K; e += 256) {
            const int rr = e % CX_R, k = e / CX_R;
            const int64_t i = r0 + rr;
            ms[rr + CX_LD * k] = i < i1 ? M[(int64_t)k * a.ld + i] : (T)0;
        }
        for (int e = threadIdx.x; e < CX_R * a.lp; e += 256) {
            const int rr = e % CX_R, c = e / CX_R;
            const int64_t i = r0 + rr;
            qs[rr + CX_LD * c] = i < i1 ? Q[(int64_t)c * a.ld + i] : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int b = threadIdx.x + 256 * u;
            if (b < nb) {
                const int k = b % a.K, cb = b / a.K;
                const T* m0 = ms + CX_LD * k;
                const T* q0 = qs + CX_LD * (4 * cb);
                for (int rr = 0; rr < CX_R; ++rr) {
                    const double x = to_d(m0[rr]);
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] += x * to_d(q0[rr + CX_LD * v]);
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int b = threadIdx.x + 256 * u;
        if (b < nb) {
            const int k = b % a.K, cb = b / a.K;
#pragma unroll
            for (int v = 0; v < 4; ++v) a.Pp[(k + (int64_t)(4 * cb + v) * a.K) * a.nchunk + ch] = acc[u][v];
        }
    }
}

// one tile per entry o: P[o] = the sum of its nchunk partial sums (contiguous);
// thread t adds chunks t, t + 256, .. in order, then a fixed tree in LDS
__global__ __launch_bounds__(256) void k_center_sum(Group<CrossSumArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const CrossSumArgs& a = g.args[it];
    const int o = blockIdx.x - g.tstart[it];
    const double* src = a.Pp + (int64_t)o * a.nchunk;
    double s = 0.0;
    for (int c = threadIdx.x; c < a.nchunk; c += 256) s += src[c];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.P[o] = red[0];
}

// 256 entries per tile over the ld x lp array Z
__global__ __launch_bounds__(256) void k_center_z(Group<CenterZArgs> g) {
    if (group_skipped(g)) return;
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

hipError_t launch_center_sum(const GroupLaunch<CrossSumArgs>& L, hipStream_t st) {
    hipLaunchKernelGGL(k_center_sum, dim3(L.tiles), dim3(256), 0, st, mkgc(L));
    return hipGetLastError();
}

hipError_t launch_center_z(const GroupLaunch<CenterZArgs>& L, hipStream_t st) {
    hipLaunchKernelGGL(k_center_z, dim3(L.tiles), dim3(256), 0, st, mkgc(L));
    return hipGetLastError();
}

}  // namespace rpod
