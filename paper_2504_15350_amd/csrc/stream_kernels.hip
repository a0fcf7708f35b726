// Passes over the snapshot matrix S on the matrix cores (gfx950).
//
//   k_sx   Y = S X   (sketch of Alg. 1 step 2, the S-products of step 3, and
//                     the small applications Y R^-1 / Q U_hat)
//   k_stq  Z = S^T Q (the S^T-products of step 3 and T^T = S^T Q of step 5)
//
// Both stream S column-major straight from HBM into registers in the
// operand layout of the 16x16x4 MFMA, so no LDS staging is needed: the row
// index of S is permuted inside an MFMA tile (free for the M and K
// dimensions as long as both operands agree), which turns every load into a
// 16-byte (FP32) or 32-byte (FP64) contiguous vector load.
#include "device_common.hpp"
#include "internal.hpp"

namespace rpod {

template <typename T>
using V4 = typename vec4_of<T>::type;

// Four consecutive rows i..i+3 of column j, rows >= lim or columns >= n read 0.
template <bool VEC, typename T>
__device__ __forceinline__ V4<T> load_rows4(const GLOBAL T* S, int64_t ld, int64_t lim, int64_t n,
                                            int64_t i, int64_t j) {
    V4<T> v = {0, 0, 0, 0};
    if (j < n) {
        const GLOBAL T* p = S + j * ld + i;
        if (VEC && i + 3 < lim) {
            v = *reinterpret_cast<const GLOBAL V4<T>*>(p);
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (i + t < lim) v[t] = p[t];
        }
    }
    return v;
}

template <typename Tout, typename T>
__device__ __forceinline__ void store4(GLOBAL Tout* p, T a, T b, T c, T d) {
    typedef typename vec4_of<Tout>::type VO;
    VO v = {narrow<Tout>(a), narrow<Tout>(b), narrow<Tout>(c), narrow<Tout>(d)};
    *reinterpret_cast<GLOBAL VO*>(p) = v;
}

// ---------------------------------------------------------------------------
// Y = S X. Workgroup = 4 waves = 256 rows of S; every wave owns 64 rows and
// all 16*NT output columns. Per 16-column step a lane loads rows
// 4*(l%16)..+3 of four columns (one vector each) and a 4-vector of X per
// output tile; MFMA (t, c, s) uses row slot t, output tile c, column slot s:
//   A[mm][k] = S[iw + 4 mm + t][j0 + 4 k + s],  B[k][nn] = X[j0 + 4 k + s][16 c + nn]
// so output row mm of MFMA t is global row iw + 4 mm + t.
// ---------------------------------------------------------------------------
// Tc: matrix-core type (X's type). S of a narrower storage type Tin is
// converted in registers (Tc = double: the FP64 residual products). Only
// output columns below cmax are stored.
template <typename Tin, typename Tc, typename Tout, int NT, bool VEC, bool UPPER>
__device__ __forceinline__ void sx_body(const GLOBAL Tin* S, int64_t ldS, int64_t m, int64_t n,
                                        const GLOBAL Tc* __restrict__ X, int64_t ldX, GLOBAL Tout* Y, int64_t ldY,
                                        int64_t mstore, int cmax, int64_t bx) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kg = lane >> 4;
    const int64_t iw = bx * 256 + wave * 64;
    const int64_t irow = iw + 4 * r16;

    V4<Tc> acc[4][NT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[t][c] = V4<Tc>{0, 0, 0, 0};

    if (iw < m) {
        for (int64_t j0 = 0; j0 < n; j0 += 16) {
            V4<Tc> a[4], b[NT];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const V4<Tin> raw = load_rows4<VEC>(S, ldS, m, n, irow, j0 + 4 * kg + s);
#pragma unroll
                for (int t = 0; t < 4; ++t) a[s][t] = (Tc)raw[t];
            }
#pragma unroll
            for (int c = 0; c < NT; ++c)
                b[c] = *reinterpret_cast<const GLOBAL V4<Tc>*>(X + (int64_t)(16 * c + r16) * ldX + j0 + 4 * kg);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int c = 0; c < NT; ++c) {
                        if (UPPER && j0 > 16 * c) continue;  // X upper triangular: tile is zero
                        acc[t][c] = mfma_16x16x4(a[s][t], b[c][s], acc[t][c]);
                    }
        }
    }
    // component v of acc[t][c] is MFMA row mm = mfma_row(kg, v), i.e. global
    // row iw + 4 mm + t: rows t = 0..3 are contiguous
#pragma unroll
    for (int c = 0; c < NT; ++c) {
        if (16 * c + r16 >= cmax) continue;
        GLOBAL Tout* py = Y + (int64_t)(16 * c + r16) * ldY;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = iw + 4 * mfma_row<Tc>(kg, v);
            if (row + 3 < mstore) {
                store4<Tout>(py + row, acc[0][c][v], acc[1][c][v], acc[2][c][v], acc[3][c][v]);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (row + t < mstore) py[row + t] = narrow<Tout>(acc[t][c][v]);
            }
        }
    }
}

template <typename Tin, typename Tout, int NT, bool VEC, bool UPPER>
__global__ __launch_bounds__(256) void k_sx(Group<SxArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const SxArgs& a = g.args[it];
    if (a.cond != nullptr && !(*a.cond & a.cond_mask)) return;
    const void* S = static_cast<const char*>(a.call >= 0 ? g.calls[a.call].S : a.S) +
                    a.col0 * a.ldS * (int64_t)sizeof(Tin);
    sx_body<Tin, Tin, Tout, NT, VEC, UPPER>(gbl((const Tin*)S), a.ldS, a.m, a.n, gbl((const Tin*)a.X), a.ldX,
                                            gbl((Tout*)a.Y), a.ldY, a.mstore, a.cmax > 0 ? a.cmax : 16 * NT,
                                            blockIdx.x - g.tstart[it]);
}

// Y (FP64) = S X with X in FP64 and S of any storage type, FP64 matrix cores.
template <typename Tin, int NT, bool VEC>
__global__ __launch_bounds__(256) void k_sx_wide(Group<SxArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const SxArgs& a = g.args[it];
    if (a.cond != nullptr && !(*a.cond & a.cond_mask)) return;
    const void* S = static_cast<const char*>(a.call >= 0 ? g.calls[a.call].S : a.S) +
                    a.col0 * a.ldS * (int64_t)sizeof(Tin);
    sx_body<Tin, double, double, NT, VEC, false>(gbl((const Tin*)S), a.ldS, a.m, a.n, gbl((const double*)a.X),
                                                 a.ldX, gbl((double*)a.Y), a.ldY, a.mstore,
                                                 a.cmax > 0 ? a.cmax : 16 * NT, blockIdx.x - g.tstart[it]);
}

// ---------------------------------------------------------------------------
// Z_s = S_s^T Q_s for row split s. Workgroup = 4 waves = 256 columns of S
// (each wave 4 tiles of 16 columns), streaming its split of rows 16 at a
// time. MFMA (u, c, s) with column tile u, output tile c, row slot s:
//   A[mm][k] = S[i0 + 4 k + s][jw + 16 u + mm],  B[k][nn] = Q[i0 + 4 k + s][16 c + nn].
// ---------------------------------------------------------------------------
template <typename Tin, int NT, bool VEC>
__device__ __forceinline__ void stq_body(const GLOBAL Tin* __restrict__ S, int64_t ldS, int64_t m, int64_t n,
                                         const GLOBAL Tin* __restrict__ Q, int64_t ldQ, GLOBAL double* __restrict__ Zp,
                                         int64_t nP,
                                         int64_t split_rows, int64_t bx, int64_t by) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kg = lane >> 4;
    const int64_t jw = bx * 256 + wave * 64;
    const int64_t ib = by * split_rows;
    const int64_t ie = (ib + split_rows < m) ? ib + split_rows : m;

    V4<Tin> acc[4][NT];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[u][c] = V4<Tin>{0, 0, 0, 0};

    if (jw < n) {
        for (int64_t i0 = ib; i0 < ie; i0 += 16) {
            V4<Tin> a[4], b[NT];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = load_rows4<VEC>(S, ldS, ie, n, i0 + 4 * kg, jw + 16 * u + r16);
#pragma unroll
            for (int c = 0; c < NT; ++c)
                b[c] = *reinterpret_cast<const GLOBAL V4<Tin>*>(Q + (int64_t)(16 * c + r16) * ldQ + i0 + 4 * kg);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int c = 0; c < NT; ++c) acc[u][c] = mfma_16x16x4(a[u][s], b[c][s], acc[u][c]);
        }
    }
    GLOBAL double* zp = Zp + by * nP * (16 * NT);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            GLOBAL double* pz = zp + (int64_t)(16 * c + r16) * nP + jw + 16 * u;
            if constexpr (sizeof(Tin) == 4) {
                store4<double>(pz + 4 * kg, acc[u][c][0], acc[u][c][1], acc[u][c][2], acc[u][c][3]);
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) pz[mfma_row<Tin>(kg, v)] = acc[u][c][v];
            }
        }
}

// grouped launch: local tile t covers column block t % ncb of split t / ncb
template <typename Tin, int NT, bool VEC>
__global__ __launch_bounds__(256) void k_stq(Group<StqArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const StqArgs& a = g.args[it];
    const int t = blockIdx.x - g.tstart[it];
    const void* S = a.call >= 0 ? g.calls[a.call].S : a.S;
    stq_body<Tin, NT, VEC>(gbl((const Tin*)S), a.ldS, a.m, a.n, gbl((const Tin*)a.Q), a.ldQ, gbl(a.Zp), a.nP,
                           a.split_rows, t % a.ncb, t / a.ncb);
}

// ---------------------------------------------------------------------------
// Z_s = S^T Q for FP32 S, LDS-staged. Workgroup: 64 HBU columns of S (HBU
// column tiles of 16 per wave, wave w owning columns 16 HBU w ..) over the
// rows of split s, 64 rows per step.
// Each step's S block (64 rows x 64 HBU columns) and Q block (64 rows x
// 16 NT columns) are staged in LDS column-major with a 68-float column
// stride (16-byte reads and writes without bank conflicts); the global
// reads cover 4 columns x 256 bytes per wave instruction. The next step's
// blocks are loaded into registers during the matrix-core work. MFMA
// (u, c, s) of row group k takes, in lane (r, g), rows 16 k + 4 g + s:
//   A[r][g] = S[i0 + 16 k + 4 g + s][j0 + 16 HBU w + 16 u + r],
//   B[g][r] = Q[i0 + 16 k + 4 g + s][16 c + r].
// Splits are interleaved: step t of split s covers rows 64 (t nsplit + s).
// ---------------------------------------------------------------------------
constexpr int STQ32_R = 64, STQ32_LDS = STQ32_R + 4;

template <int NT, bool VEC, int HBU>
__device__ __forceinline__ void stq32_body(const GLOBAL float* __restrict__ S, int64_t ldS, int64_t m, int64_t n,
                                           const GLOBAL float* __restrict__ Q, int64_t ldQ,
                                           GLOBAL double* __restrict__ Zp, int64_t nP, int nsplit, int ncb,
                                           int tile) {
    constexpr int R = STQ32_R, LD = STQ32_LDS, HB = 64 * HBU;
    constexpr int CPC = R / 4;                 // 16-byte chunks per column of a block
    constexpr int SPT = HB * CPC / 256;        // S chunks per thread
    constexpr int QPT = 16 * NT * CPC / 256;   // Q chunks per thread
    __shared__ __attribute__((aligned(16))) float ss[HB * LD];
    __shared__ __attribute__((aligned(16))) float qs[16 * NT * LD];
    const int cb = tile % ncb, sp = tile / ncb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, kg = lane >> 4;
    const int64_t j0 = (int64_t)cb * HB;
    const int64_t ib = (int64_t)sp * R, stride = (int64_t)nsplit * R;

    f32x4 acc[HBU][NT];
#pragma unroll
    for (int u = 0; u < HBU; ++u)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[u][c] = f32x4{0, 0, 0, 0};

    f32x4 sr[SPT], qr[QPT];
    auto fetch = [&](int64_t i0) {
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int ch = tid + 256 * q;
            sr[q] = load_rows4<VEC>(S, ldS, m, n, i0 + 4 * (ch % CPC), j0 + ch / CPC);
        }
#pragma unroll
        for (int q = 0; q < QPT; ++q) {
            const int ch = tid + 256 * q;
            qr[q] = *reinterpret_cast<const GLOBAL f32x4*>(Q + (int64_t)(ch / CPC) * ldQ + i0 + 4 * (ch % CPC));
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int ch = tid + 256 * q;
            *reinterpret_cast<f32x4*>(ss + (ch / CPC) * LD + 4 * (ch % CPC)) = sr[q];
        }
#pragma unroll
        for (int q = 0; q < QPT; ++q) {
            const int ch = tid + 256 * q;
            *reinterpret_cast<f32x4*>(qs + (ch / CPC) * LD + 4 * (ch % CPC)) = qr[q];
        }
    };
    if (ib < m) fetch(ib);
    for (int64_t i0 = ib; i0 < m; i0 += stride) {
        __syncthreads();  // previous step consumed
        put();
        __syncthreads();
        if (i0 + stride < m) fetch(i0 + stride);  // in flight during the matrix-core work
#pragma unroll
        for (int k = 0; k < R / 16; ++k) {
            f32x4 a[HBU], b[NT];
#pragma unroll
            for (int u = 0; u < HBU; ++u)
                a[u] = *reinterpret_cast<const f32x4*>(ss + (16 * HBU * wave + 16 * u + r16) * LD + 16 * k + 4 * kg);
#pragma unroll
            for (int c = 0; c < NT; ++c)
                b[c] = *reinterpret_cast<const f32x4*>(qs + (16 * c + r16) * LD + 16 * k + 4 * kg);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int u = 0; u < HBU; ++u)
#pragma unroll
                    for (int c = 0; c < NT; ++c) acc[u][c] = mfma_16x16x4(a[u][s], b[c][s], acc[u][c]);
        }
    }
    // D[4 g + v][r]: S column j0 + 16 HBU w + 16 u + 4 g + v, Q column 16 c + r
    GLOBAL double* zp = Zp + (int64_t)sp * nP * (16 * NT);
#pragma unroll
    for (int u = 0; u < HBU; ++u)
#pragma unroll
        for (int c = 0; c < NT; ++c)
            store4<double>(zp + (int64_t)(16 * c + r16) * nP + j0 + 16 * HBU * wave + 16 * u + 4 * kg, acc[u][c][0],
                           acc[u][c][1], acc[u][c][2], acc[u][c][3]);
}

template <int NT, bool VEC, int HBU>
__global__ __launch_bounds__(256) void k_stq32(Group<StqArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const StqArgs& a = g.args[it];
    const void* S = a.call >= 0 ? g.calls[a.call].S : a.S;
    stq32_body<NT, VEC, HBU>(gbl((const float*)S), a.ldS, a.m, a.n, gbl((const float*)a.Q), a.ldQ, gbl(a.Zp), a.nP,
                             a.nsplit, a.ncb, blockIdx.x - g.tstart[it]);
}

// out[e] = sum of the nsplit slabs in FP64, fixed order; 256 elements per workgroup
__global__ void k_reduce_slabs(Group<ReduceArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const ReduceArgs& a = g.args[it];
    const int64_t e = (int64_t)(blockIdx.x - g.tstart[it]) * blockDim.x + threadIdx.x;
    if (e >= a.count) return;
    // eight partial sums (slabs k = u mod 8: independent loads in flight), combined in a fixed order
    double p8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int ns = a.nsplit;
    int k = 0;
    if (a.f32) {
        const GLOBAL float* Zp = gbl((const float*)a.Zp) + e;
        for (; k + 8 <= ns; k += 8)
#pragma unroll
            for (int u = 0; u < 8; ++u) p8[u] += (double)Zp[(int64_t)(k + u) * a.count];
        for (; k < ns; ++k) p8[k & 7] += (double)Zp[(int64_t)k * a.count];
    } else {
        const GLOBAL double* Zp = gbl((const double*)a.Zp) + e;
        for (; k + 8 <= ns; k += 8)
#pragma unroll
            for (int u = 0; u < 8; ++u) p8[u] += Zp[(int64_t)(k + u) * a.count];
        for (; k < ns; ++k) p8[k & 7] += Zp[(int64_t)k * a.count];
    }
    const double v = (((p8[0] + p8[1]) + (p8[2] + p8[3])) + ((p8[4] + p8[5]) + (p8[6] + p8[7]))) * a.scale;
    if (a.out32)
        *gbl((float*)a.out + e) = (float)v;
    else
        *gbl((double*)a.out + e) = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename A>
static Group<A> mkgroup(const GroupLaunch<A>& L) {
    Group<A> g;
    g.args = L.args;
    g.tstart = L.tstart;
    g.calls = L.calls;
    g.count = L.count;
    g.skip = L.skip;
    g.skip_mask = L.skip_mask;
    return g;
}

template <typename Tin, typename Tout, int NT>
static hipError_t sx_nt(const GroupLaunch<SxArgs>& L, bool vec, bool upper, hipStream_t st) {
    const Group<SxArgs> g = mkgroup(L);
    if (upper)
        hipLaunchKernelGGL((k_sx<Tin, Tout, NT, true, true>), dim3(L.tiles), dim3(256), 0, st, g);
    else if (vec)
        hipLaunchKernelGGL((k_sx<Tin, Tout, NT, true, false>), dim3(L.tiles), dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL((k_sx<Tin, Tout, NT, false, false>), dim3(L.tiles), dim3(256), 0, st, g);
    return hipGetLastError();
}

template <typename Tin, typename Tout>
static hipError_t sx_dispatch(int nt, const GroupLaunch<SxArgs>& L, bool vec, bool upper, hipStream_t st) {
    switch (nt) {
#define RPOD_SX_CASE(K) case K: return sx_nt<Tin, Tout, K>(L, vec, upper, st);
        RPOD_SX_CASE(1) RPOD_SX_CASE(2) RPOD_SX_CASE(3) RPOD_SX_CASE(4)
        RPOD_SX_CASE(5) RPOD_SX_CASE(6) RPOD_SX_CASE(7) RPOD_SX_CASE(8)
#undef RPOD_SX_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename Tin, int NT>
static hipError_t sxw_nt(const GroupLaunch<SxArgs>& L, bool vec, hipStream_t st) {
    const Group<SxArgs> g = mkgroup(L);
    if (vec)
        hipLaunchKernelGGL((k_sx_wide<Tin, NT, true>), dim3(L.tiles), dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL((k_sx_wide<Tin, NT, false>), dim3(L.tiles), dim3(256), 0, st, g);
    return hipGetLastError();
}

template <typename Tin>
static hipError_t sxw_dispatch(int nt, const GroupLaunch<SxArgs>& L, bool vec, hipStream_t st) {
    switch (nt) {
#define RPOD_SXW_CASE(K) case K: return sxw_nt<Tin, K>(L, vec, st);
        RPOD_SXW_CASE(1) RPOD_SXW_CASE(2) RPOD_SXW_CASE(3) RPOD_SXW_CASE(4)
        RPOD_SXW_CASE(5) RPOD_SXW_CASE(6) RPOD_SXW_CASE(7) RPOD_SXW_CASE(8)
#undef RPOD_SXW_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sx_wide(int tin, int nt, bool vec, const GroupLaunch<SxArgs>& L, hipStream_t st) {
    if (tin == DT_F32) return sxw_dispatch<float>(nt, L, vec, st);
    if (tin == DT_BF16) return sxw_dispatch<__bf16>(nt, L, vec, st);
    if (tin == DT_F16) return sxw_dispatch<_Float16>(nt, L, vec, st);
    if (tin == DT_F64) return sxw_dispatch<double>(nt, L, vec, st);
    return hipErrorInvalidValue;
}

hipError_t launch_sx(int tin, int tout, int nt, bool vec, bool upper, const GroupLaunch<SxArgs>& L, hipStream_t st) {
    if (tin == DT_F64 && tout == DT_F64) return sx_dispatch<double, double>(nt, L, vec, upper, st);
    if (tin == DT_F64 && tout == DT_F32) return sx_dispatch<double, float>(nt, L, vec, upper, st);
    if (tin == DT_F32 && tout == DT_F32) return sx_dispatch<float, float>(nt, L, vec, upper, st);
    if (tin == DT_F64 && tout == DT_BF16) return sx_dispatch<double, __bf16>(nt, L, vec, upper, st);
    if (tin == DT_F64 && tout == DT_F16) return sx_dispatch<double, _Float16>(nt, L, vec, upper, st);
    return hipErrorInvalidValue;
}

template <typename Tin, int NT>
static hipError_t stq_nt(const GroupLaunch<StqArgs>& L, bool vec, hipStream_t st) {
    const Group<StqArgs> g = mkgroup(L);
    if constexpr (sizeof(Tin) == 4) {  // FP32: the LDS-staged kernel, two column tiles per wave
        if (vec)
            hipLaunchKernelGGL((k_stq32<NT, true, 2>), dim3(L.tiles), dim3(256), 0, st, g);
        else
            hipLaunchKernelGGL((k_stq32<NT, false, 2>), dim3(L.tiles), dim3(256), 0, st, g);
    } else {
        if (vec)
            hipLaunchKernelGGL((k_stq<Tin, NT, true>), dim3(L.tiles), dim3(256), 0, st, g);
        else
            hipLaunchKernelGGL((k_stq<Tin, NT, false>), dim3(L.tiles), dim3(256), 0, st, g);
    }
    return hipGetLastError();
}

int stq32_block_cols() { return 128; }

template <typename Tin>
static hipError_t stq_dispatch(int nt, const GroupLaunch<StqArgs>& L, bool vec, hipStream_t st) {
    switch (nt) {
#define RPOD_STQ_CASE(K) case K: return stq_nt<Tin, K>(L, vec, st);
        RPOD_STQ_CASE(1) RPOD_STQ_CASE(2) RPOD_STQ_CASE(3) RPOD_STQ_CASE(4)
        RPOD_STQ_CASE(5) RPOD_STQ_CASE(6) RPOD_STQ_CASE(7) RPOD_STQ_CASE(8)
#undef RPOD_STQ_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stq(int tin, int nt, bool vec, const GroupLaunch<StqArgs>& L, hipStream_t st) {
    if (tin == DT_F64) return stq_dispatch<double>(nt, L, vec, st);
    if (tin == DT_F32) return stq_dispatch<float>(nt, L, vec, st);
    return hipErrorInvalidValue;
}

hipError_t launch_reduce_slabs(const GroupLaunch<ReduceArgs>& L, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_slabs, dim3(L.tiles), dim3(256), 0, st, mkgroup(L));
    return hipGetLastError();
}

}  // namespace rpod
