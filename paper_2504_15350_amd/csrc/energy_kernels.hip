// Frobenius norm of the snapshot matrix for the energy of the modes (Sec. 4.1,
// the energy criterion, read with squared singular values: sum sigma_i^2 =
// ||S||_F^2). Squares are summed in FP64 in a fixed order: tile w adds the
// columns w, w + nwg, .. (thread t rows V t, V t + 256 V, .. of each, V
// elements of 16 bytes per load when aligned), a tree in LDS; then one tile
// adds the nwg partial sums.
#include "device_common.hpp"
#include "internal.hpp"

namespace rpod {

template <typename A>
static Group<A> mkge(const GroupLaunch<A>& L) {
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
__device__ __forceinline__ double sq_d(T x) {
    double v;
    if constexpr (sizeof(T) == 2) v = (double)(float)x;
    else v = (double)x;
    return v * v;
}

__device__ __forceinline__ double block_sum256(double s, double* red) {
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    return red[0];
}

template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_frob_part(Group<FrobArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const FrobArgs& a = g.args[it];
    const int w = blockIdx.x - g.tstart[it];
    const GLOBAL T* S = gbl((const T*)(a.call >= 0 ? g.calls[a.call].S : a.S));
    constexpr int V = 16 / sizeof(T);
    typedef T TV __attribute__((ext_vector_type(V)));
    double s = 0.0;
    for (int64_t j = w; j < a.n; j += a.nwg) {
        const GLOBAL T* col = S + j * a.ld;
        for (int64_t i = (int64_t)threadIdx.x * V; i < a.m; i += 256 * V) {
            if (VEC && i + V <= a.m) {
                const TV v = __builtin_nontemporal_load(reinterpret_cast<const GLOBAL TV*>(col + i));
#pragma unroll
                for (int k = 0; k < V; ++k) s += sq_d(v[k]);
            } else {
                for (int64_t k = i; k < i + V && k < a.m; ++k) s += sq_d(col[k]);
            }
        }
    }
    __shared__ double red[256];
    const double tot = block_sum256(s, red);
    if (threadIdx.x == 0) a.part[w] = tot;
}

__global__ __launch_bounds__(256) void k_frob_sum(Group<FrobArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const FrobArgs& a = g.args[it];
    double s = 0.0;
    for (int w = threadIdx.x; w < a.nwg; w += 256) s += a.part[w];
    __shared__ double red[256];
    const double tot = block_sum256(s, red);
    if (threadIdx.x == 0) *a.out = tot;
}

template <typename T>
static void frob_t(bool vec, const GroupLaunch<FrobArgs>& P, hipStream_t st) {
    if (vec)
        hipLaunchKernelGGL((k_frob_part<T, true>), dim3(P.tiles), dim3(256), 0, st, mkge(P));
    else
        hipLaunchKernelGGL((k_frob_part<T, false>), dim3(P.tiles), dim3(256), 0, st, mkge(P));
}

hipError_t launch_frob(int tin, bool vec, bool sum_only, const GroupLaunch<FrobArgs>& P,
                       const GroupLaunch<FrobArgs>& F, hipStream_t st) {
    if (sum_only) {
        hipLaunchKernelGGL(k_frob_sum, dim3(F.tiles), dim3(256), 0, st, mkge(F));
        return hipGetLastError();
    }
    switch (tin) {
        case DT_F64: frob_t<double>(vec, P, st); break;
        case DT_F32: frob_t<float>(vec, P, st); break;
        case DT_BF16: frob_t<__bf16>(vec, P, st); break;
        case DT_F16: frob_t<_Float16>(vec, P, st); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_frob_sum, dim3(F.tiles), dim3(256), 0, st, mkge(F));
    return hipGetLastError();
}

}  // namespace rpod
