// Small FP64 linear algebra of the rPOD path and the Gaussian sketch.
//
//   k_omega        Gaussian sketch (Alg. 1 step 1) from Philox4x32-10
//   k_gram         FP64 Gram matrix Y^T Y of a tall matrix on FP64 MFMA
//   k_chol_blk     Cholesky + triangular inverse for CholeskyQR (step 4)
//   k_jacobi       SVD of the small T of step 6 via the eigenvectors of T T^T
//                  (pivoted Cholesky, then preconditioned one-sided Jacobi)
//   k_lift_coef    the small factors of the lift (step 7) and the coefficients
//   k_colmax/...   deterministic sign convention and output packing
#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"

namespace rpod {

template <typename T>
using V4 = typename vec4_of<T>::type;

template <typename A>
static Group<A> mkg(const GroupLaunch<A>& L) {
    Group<A> g;
    g.args = L.args;
    g.tstart = L.tstart;
    g.calls = L.calls;
    g.count = L.count;
    g.skip = L.skip;
    g.skip_mask = L.skip_mask;
    return g;
}

__global__ void k_zero_ints(Group<ZeroArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const ZeroArgs& a = g.args[it];
    const int i = (blockIdx.x - g.tstart[it]) * blockDim.x + threadIdx.x;
    if (i < a.count) a.p[i] = 0;
}

hipError_t launch_zero_ints(const GroupLaunch<ZeroArgs>& L, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_ints, dim3(L.tiles), dim3(256), 0, st, mkg(L));
    return hipGetLastError();
}

// Per-call table: one entry per matrix, written from kernel arguments so
// that it needs no host staging buffer (and may precede a graph launch).
constexpr int CALLS_PER_LAUNCH = 16;
struct CallBatch {
    CallDesc d[CALLS_PER_LAUNCH];
    int first, count;
};

__global__ void k_set_calls(CallDesc* table, CallBatch b) {
    const int i = threadIdx.x;
    if (i < b.count) table[b.first + i] = b.d[i];
}

hipError_t launch_set_calls(CallDesc* table, const CallDesc* host, int count, hipStream_t st) {
    for (int first = 0; first < count; first += CALLS_PER_LAUNCH) {
        CallBatch b;
        b.first = first;
        b.count = count - first < CALLS_PER_LAUNCH ? count - first : CALLS_PER_LAUNCH;
        for (int i = 0; i < b.count; ++i) b.d[i] = host[first + i];
        hipLaunchKernelGGL(k_set_calls, dim3(1), dim3(CALLS_PER_LAUNCH), 0, st, table, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Gaussian sketch. Thread per (row j, column pair t).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void omega_body(uint64_t seed, int64_t n, int l, int lpad, int64_t rows_pad, GLOBAL T* out,
                                           int64_t ldo, int64_t bx, int t /* column pair */, uint32_t stream) {
    const int64_t j = bx * blockDim.x + threadIdx.x;
    if (j >= rows_pad) return;
    const int c0 = 2 * t, c1 = 2 * t + 1;
    double g0 = 0.0, g1 = 0.0;
    if (j < n && c0 < l) {
        const philox_out o = philox4x32_10((uint32_t)j, (uint32_t)((uint64_t)j >> 32), (uint32_t)t, stream,
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

// grouped: local tile t covers rows 256 (t % nb) .. and column pair t / nb
template <typename T>
__global__ void k_omega(Group<OmegaArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const OmegaArgs& a = g.args[it];
    const int t = blockIdx.x - g.tstart[it];
    const int nb = (int)((a.rows_pad + 255) / 256);
    const uint64_t seed = a.call >= 0 ? g.calls[a.call].seed : a.seed;
    omega_body<T>(seed, a.n, a.l, a.lpad, a.rows_pad, gbl((T*)a.out), a.ldo, t % nb, t / nb, a.stream);
}

template <typename T>
__global__ void k_omega_direct(uint64_t seed, int64_t n, int l, int64_t ldo, T* out) {
    omega_body<T>(seed, n, l, l, n, gbl(out), ldo, blockIdx.x, blockIdx.y, 0u);
}

hipError_t launch_omega(int tout, const GroupLaunch<OmegaArgs>& L, hipStream_t st) {
    if (tout == DT_F64)
        hipLaunchKernelGGL(k_omega<double>, dim3(L.tiles), dim3(256), 0, st, mkg(L));
    else if (tout == DT_F32)
        hipLaunchKernelGGL(k_omega<float>, dim3(L.tiles), dim3(256), 0, st, mkg(L));
    else if (tout == DT_BF16)
        hipLaunchKernelGGL(k_omega<__bf16>, dim3(L.tiles), dim3(256), 0, st, mkg(L));
    else if (tout == DT_F16)
        hipLaunchKernelGGL(k_omega<_Float16>, dim3(L.tiles), dim3(256), 0, st, mkg(L));
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_omega_direct(int tout, uint64_t seed, int64_t n, int l, void* out, int64_t ldo, hipStream_t st) {
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)((l + 1) / 2));
    if (tout == DT_F64)
        hipLaunchKernelGGL(k_omega_direct<double>, grid, dim3(256), 0, st, seed, n, l, ldo, (double*)out);
    else if (tout == DT_F32)
        hipLaunchKernelGGL(k_omega_direct<float>, grid, dim3(256), 0, st, seed, n, l, ldo, (float*)out);
    else if (tout == DT_BF16)
        hipLaunchKernelGGL(k_omega_direct<__bf16>, grid, dim3(256), 0, st, seed, n, l, ldo, (__bf16*)out);
    else if (tout == DT_F16)
        hipLaunchKernelGGL(k_omega_direct<_Float16>, grid, dim3(256), 0, st, seed, n, l, ldo, (_Float16*)out);
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
// pair group of the launch; partials are reduced over the 4 waves in LDS in a
// fixed order and written per workgroup.
// ---------------------------------------------------------------------------
constexpr int GRAM_WGS = 512;

__host__ __device__ constexpr int npairs_of(int nt) { return nt * (nt + 1) / 2; }
__host__ __device__ constexpr int gram_groups(int nt) { return nt <= 4 ? 1 : 3; }
__host__ __device__ constexpr int gram_pg(int nt) {
    return (npairs_of(nt) + gram_groups(nt) - 1) / gram_groups(nt);
}

int64_t gram_partial_count(int nt) { return (int64_t)GRAM_WGS * npairs_of(nt) * 256; }

template <typename Tin, int NT, int PLO, int PHI>
__device__ __forceinline__ void gram_body(const GLOBAL Tin* __restrict__ Y, int64_t ld, int64_t M,
                                          GLOBAL double* __restrict__ Gpart, double* red, int bx, int nwg) {
    constexpr int PG = PHI - PLO;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kg = lane >> 4;
    f64x4 acc[PG];
#pragma unroll
    for (int p = 0; p < PG; ++p) acc[p] = f64x4{0, 0, 0, 0};

    const int64_t nrb = (M + 15) / 16, rstride = (int64_t)nwg * 4;
    // the next row block is loaded while the matrix cores work on this one
    V4<Tin> vn[NT];
    auto load = [&](int64_t rb) {
#pragma unroll
        for (int a = 0; a < NT; ++a)
            vn[a] = *reinterpret_cast<const GLOBAL V4<Tin>*>(Y + (int64_t)(16 * a + r16) * ld + rb * 16 + 4 * kg);
    };
    int64_t rb = (int64_t)bx * 4 + wave;
    if (rb < nrb) load(rb);
    for (; rb < nrb; rb += rstride) {
        double x[NT][4];
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
            for (int s = 0; s < 4; ++s) x[a][s] = (double)vn[a][s];
        if (rb + rstride < nrb) load(rb + rstride);
        // row slot outermost: consecutive matrix-core instructions are independent
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            int p = 0;
#pragma unroll
            for (int a = 0; a < NT; ++a)
#pragma unroll
                for (int b = a; b < NT; ++b) {
                    if (p >= PLO && p < PHI) acc[p - PLO] = mfma_16x16x4(x[a][s], x[b][s], acc[p - PLO]);
                    ++p;
                }
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
        Gpart[((int64_t)bx * NP + p) * 256 + (e % 256)] = red[e];
    }
}

// grouped: local tile t is partial workgroup bx of pair group grp. With
// several pair groups, the groups of one row block sit 8 tiles apart (the
// same XCD when the item starts at a multiple of 8, at about the same time),
// so the second and third reads of the rows come from that XCD's L2.
template <typename Tin, int NT>
__global__ __launch_bounds__(256) void k_gram(Group<GramArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const GramArgs& a = g.args[it];
    if (a.cond != nullptr && !(*a.cond & a.cond_mask)) return;
    const int t = blockIdx.x - g.tstart[it];
    constexpr int NG = gram_groups(NT);
    int bx = t % a.nwg, grp = t / a.nwg;
    if (NG > 1 && (a.nwg & 7) == 0 && (g.tstart[it] & 7) == 0) {
        grp = (t >> 3) % NG;
        bx = (t / (8 * NG)) * 8 + (t & 7);
    }
    constexpr int NP = npairs_of(NT), PG = gram_pg(NT);
    __shared__ double red[PG * 256];
    const GLOBAL Tin* Y = gbl((const Tin*)a.Y);
    GLOBAL double* Gp = gbl(a.Gpart);
    if (grp == 0) gram_body<Tin, NT, 0, (PG < NP ? PG : NP)>(Y, a.ld, a.M, Gp, red, bx, a.nwg);
    if constexpr (gram_groups(NT) > 1) {
        if (grp == 1) gram_body<Tin, NT, PG, (2 * PG < NP ? 2 * PG : NP)>(Y, a.ld, a.M, Gp, red, bx, a.nwg);
        if (grp == 2) gram_body<Tin, NT, 2 * PG, NP>(Y, a.ld, a.M, Gp, red, bx, a.nwg);
    }
}

// grouped: npairs(nt) tiles of 256 elements per matrix
__global__ __launch_bounds__(256) void k_gram_reduce(Group<GramArgs> g, int nt) {
    if (group_skipped(g)) return;
    __shared__ double part[8][32];
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const GramArgs& ga = g.args[it];
    if (ga.cond != nullptr && !(*ga.cond & ga.cond_mask)) return;
    const int np = nt * (nt + 1) / 2;
    // 32 entries per workgroup, eight threads per entry: thread t sums the
    // partials w = t, t + 8, .. (independent loads in flight), and the eight
    // sums are combined in a fixed order
    const int el = threadIdx.x & 31, t = threadIdx.x >> 5;
    const int e = (blockIdx.x - g.tstart[it]) * 32 + el;
    const bool live = e < np * 256;
    double acc = 0.0;
    if (live) {
        const GLOBAL double* src = gbl(ga.Gpart) + e;  // entry e = pair e / 256, element e mod 256
        const int64_t wstride = (int64_t)np * 256;
        const int nwg = ga.nwg;
        double a4[4] = {0, 0, 0, 0};
        int w = t;
        for (; w + 24 < nwg; w += 32)
#pragma unroll
            for (int u = 0; u < 4; ++u) a4[u] += src[(int64_t)(w + 8 * u) * wstride];
        for (; w < nwg; w += 8) a4[0] += src[(int64_t)w * wstride];
        acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    }
    part[t][el] = acc;
    __syncthreads();
    if (t != 0 || !live) return;
    const double s = ((part[0][el] + part[1][el]) + (part[2][el] + part[3][el])) +
                     ((part[4][el] + part[5][el]) + (part[6][el] + part[7][el]));
    const int p = e / 256, mm = (e % 256) / 16, nn = e % 16;
    int a = 0, q = p;
    while (q >= nt - a) { q -= nt - a; ++a; }
    const int b = a + q;
    const int lp = 16 * nt;
    GLOBAL double* G = gbl(ga.G);
    G[(16 * a + mm) * lp + 16 * b + nn] = s;
    G[(16 * b + nn) * lp + 16 * a + mm] = s;
}

// Partial workgroups per pair group: one per 4 row blocks, at most `cap`;
// by default (cap 0) 256 for a single pair group (measured: more partials
// cost more in the reduction than they save) and about 512 workgroups over
// several pair groups (two waves per SIMD), rounded down to a multiple of 8.
int gram_nwg(int64_t M, int cap, int nt) {
    const int64_t nrb = (M + 15) / 16;
    int64_t nwg = (nrb + 3) / 4;
    if (cap < 1 || cap > GRAM_WGS) cap = gram_groups(nt) == 1 ? 256 : (GRAM_WGS / gram_groups(nt)) & ~7;
    if (nwg > cap) nwg = cap;
    if (nwg < 1) nwg = 1;
    return (int)nwg;
}

int gram_tiles(int nt, int nwg) { return nwg * gram_groups(nt); }
int gram_reduce_tiles(int nt) { return npairs_of(nt) * 8; }  // 32 entries per workgroup

template <typename Tin, int NT>
static hipError_t gram_nt(const GroupLaunch<GramArgs>& L, const GroupLaunch<GramArgs>& R, hipStream_t st) {
    hipLaunchKernelGGL((k_gram<Tin, NT>), dim3(L.tiles), dim3(256), 0, st, mkg(L));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_reduce, dim3(R.tiles), dim3(256), 0, st, mkg(R), NT);
    return hipGetLastError();
}

template <typename Tin>
static hipError_t gram_dispatch(int nt, const GroupLaunch<GramArgs>& L, const GroupLaunch<GramArgs>& R,
                                hipStream_t st) {
    switch (nt) {
#define RPOD_GRAM_CASE(K) case K: return gram_nt<Tin, K>(L, R, st);
        RPOD_GRAM_CASE(1) RPOD_GRAM_CASE(2) RPOD_GRAM_CASE(3) RPOD_GRAM_CASE(4)
        RPOD_GRAM_CASE(5) RPOD_GRAM_CASE(6) RPOD_GRAM_CASE(7) RPOD_GRAM_CASE(8)
#undef RPOD_GRAM_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gram(int tin, int nt, const GroupLaunch<GramArgs>& L, const GroupLaunch<GramArgs>& R,
                       hipStream_t st) {
    if (tin == DT_F64) return gram_dispatch<double>(nt, L, R, st);
    if (tin == DT_F32) return gram_dispatch<float>(nt, L, R, st);
    return hipErrorInvalidValue;
}

// 1 / sqrt(x) and 1 / x for x > 0 (finite): the hardware estimates refined by
// two Newton steps each (the error of the estimate squares at every step).
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    y = fma(y, fma(-x, y, 1.0), y);
    return y;
}

// v of lane `lane` (wave-uniform lane index), as a uniform value.
__device__ __forceinline__ double read_lane(double v, int lane) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// Blocked version for lp = 16 NB <= 128 with NB waves: lane j of wave p
// keeps rows 16 p .. 16 p + 15 of columns j and j + 64 (lp > 64) in
// registers. Step k: wave k / 16 reads the pivot from the lane holding
// column k, scales its row k into R[k][:] (1 / sqrt from the refined
// estimate) and updates its rows below k, A[i][j] -= R[k][i] R[k][j]
// (right-looking), the multipliers R[k][i] read from the lanes holding them;
// after its 16 rows the wave publishes them through LDS and, after one
// barrier per 16 steps, the waves below apply the 16 updates to their rows.
// (Factorisation 45 us at lp = 128 and 36 us at lp = 96, against 55 and 48 us
// with one barrier per step; bit-identical results.)
// The inverse X = R^-1 is formed by 16 x 16 blocks: the diagonal blocks by
// forward substitution on rows (lane t: x[c] = (delta_tc - sum_{k<c} x[k]
// R[k][c]) / R[c][c]), then the blocks at distance d = 1, 2, .. above the
// diagonal, X_ij = -X_ii sum_{k=i+1..j} R_ik X_kj, one wave per block. R and
// X are kept in LDS as their upper-triangular 16 x 16 blocks only (block
// (ib, jb), ib <= jb, at jb (jb + 1) / 2 + ib, column-major inside).
// Padding rows and columns of R become identity, so X has identity padding.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int blk(int ib, int jb) { return (jb * (jb + 1) / 2 + ib) * 256; }  // ib <= jb

template <int NB>
__global__ __launch_bounds__(64 * NB) void k_chol_blk(Group<CholArgs> gr) {
    if (group_skipped(gr)) return;
    constexpr int LP = 16 * NB, NTHR = 64 * NB, CPL = (LP + 63) / 64, NTRI = NB * (NB + 1) / 2 * 256;
    __shared__ __attribute__((aligned(16))) double Rs[NTRI];  // R, upper blocks
    __shared__ __attribute__((aligned(16))) double Xs[NTRI];  // R^-1, upper blocks
    __shared__ int s_fail;
    const CholArgs& a = gr.args[blockIdx.x];  // one workgroup per matrix
    const int tid = threadIdx.x, j = tid & 63, wave = tid >> 6;
    const int l = a.l, lp = a.lp;
    const double* __restrict__ G = a.G;
    if (a.mode == 2 && !(*a.local & DEV_FLAG_SHIFTED)) return;
    if (a.mode == 0 && tid == 0) *a.local = 0;

    double w[CPL][16];  // A[16 wave + r][j + 64 cc]
    double gd[CPL];
    bool fin = true;
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
        const int col = j + 64 * cc;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            w[cc][r] = col < LP ? G[(16 * wave + r) * lp + col] : 0.0;
            fin = fin && isfinite(w[cc][r]);
        }
        gd[cc] = col < LP ? G[col * lp + col] : 0.0;
    }
    bool ok = __syncthreads_and(fin) != 0;
    if (!ok && tid == 0) atomicOr(a.flags, DEV_FLAG_NONFINITE);
    if (ok) {
#pragma unroll 1
        for (int attempt = 0; attempt < 2; ++attempt) {
            if (attempt == 1) {
                double tr = 0.0;
                for (int k = 0; k < l; ++k) tr += G[k * lp + k];
                const double shift = 11.0 * ((double)a.M * l + (double)l * (l + 1)) * 0x1.0p-53 * tr;
#pragma unroll
                for (int cc = 0; cc < CPL; ++cc) {
                    const int col = j + 64 * cc;
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        w[cc][r] = (col < LP ? G[(16 * wave + r) * lp + col] : 0.0) +
                                   (16 * wave + r == col ? shift : 0.0);
                }
            }
            if (tid == 0) s_fail = 0;
            __syncthreads();
            bool fail = false;
            // Panel pb (rows and columns 16 pb .. 16 pb + 15): wave pb factorises its own 16 rows
            // without barriers (the multipliers R[k][16 pb + r] come from the lanes holding those
            // columns), publishes them through LDS (alternately in Xs and Rs, which hold R and its
            // inverse only afterwards), and after one barrier every wave below applies the panel's
            // 16 rank-1 updates to its rows, in the order of k as a step-by-step update would.
            for (int pb = 0; pb < NB; ++pb) {
                if (16 * pb >= l) break;
                double* rp = (pb & 1) ? Rs : Xs;  // R[16 pb + kk][col] at rp[kk * LP + col]
                if (wave == pb) {
#pragma unroll
                    for (int kk = 0; kk < 16; ++kk) {
                        const int k = 16 * pb + kk;
                        if (k >= l) continue;  // uniform; no break, so the loop unrolls
                        const bool khi = CPL > 1 && k >= 64;
                        const double d = read_lane(khi ? w[CPL - 1][kk] : w[0][kk], k & 63);
                        const double tol = (double)l * 0x1.0p-52 * read_lane(khi ? gd[CPL - 1] : gd[0], k & 63);
                        if (!(d > tol) || !(d > 0.0)) {  // non-positive, tiny or NaN pivot
                            // recorded once; the row becomes NaN, so every later pivot fails too
                            if (j == 0) s_fail = 1;
#pragma unroll
                            for (int cc = 0; cc < CPL; ++cc) w[cc][kk] = __builtin_nan("");
                        } else {
                            const double rinv = rsqrt_nr(d);
#pragma unroll
                            for (int cc = 0; cc < CPL; ++cc) {
                                const int col = j + 64 * cc;
                                w[cc][kk] = (col >= k) ? w[cc][kk] * rinv : 0.0;  // R[k][col]
                            }
                        }
#pragma unroll
                        for (int r = kk + 1; r < 16; ++r) {  // the panel's rows below row k
                            const int cr = 16 * pb + r;
                            const bool rhi = CPL > 1 && cr >= 64;
                            const double rk = read_lane(rhi ? w[CPL - 1][kk] : w[0][kk], cr & 63);  // R[k][cr]
#pragma unroll
                            for (int cc = 0; cc < CPL; ++cc) w[cc][r] -= rk * w[cc][kk];
                        }
                    }
#pragma unroll
                    for (int cc = 0; cc < CPL; ++cc) {
                        const int col = j + 64 * cc;
                        if (col < LP) {
#pragma unroll
                            for (int r = 0; r < 16; ++r) rp[r * LP + col] = w[cc][r];
                        }
                    }
                }
                __syncthreads();
                if (wave > pb) {
                    const int nk = min(16, l - 16 * pb);
                    for (int kk = 0; kk < nk; ++kk) {
                        double rkc[CPL];
#pragma unroll
                        for (int cc = 0; cc < CPL; ++cc) {
                            const int col = j + 64 * cc;
                            rkc[cc] = col < LP ? rp[kk * LP + col] : 0.0;
                        }
                        const double* ra = rp + kk * LP + 16 * wave;  // R[k][16 wave + r], the same in every lane
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const double a = ra[r];
#pragma unroll
                            for (int cc = 0; cc < CPL; ++cc) w[cc][r] -= a * rkc[cc];
                        }
                    }
                }
            }
            __syncthreads();
            fail = s_fail != 0;
            __syncthreads();  // every thread has read s_fail
            if (!fail) break;
            if (attempt == 0) {
                if (tid == 0) {
                    atomicOr(a.flags, DEV_FLAG_SHIFTED);
                    *a.local |= DEV_FLAG_SHIFTED;
                }
            } else {
                if (tid == 0) atomicOr(a.flags, DEV_FLAG_BREAKDOWN);
                ok = false;
            }
        }
    }
    if (ok) {
        // R (upper blocks; lower part of the diagonal blocks zero) with identity padding
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) {
            const int col = j + 64 * cc, cb = col >> 4;
            if (col < LP && wave <= cb) {
                double* dst = Rs + blk(wave, cb) + (col & 15) * 16;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int i = 16 * wave + r;
                    dst[r] = (i <= col) ? ((i < l && col < l) ? w[cc][r] : (i == col ? 1.0 : 0.0)) : 0.0;
                }
            }
        }
        __syncthreads();
        if (j < 16) {  // diagonal block of wave p: lane t = row t
            const double* Rd = Rs + blk(wave, wave);
            double x[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                double s0 = (c == j) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    if (k < c) {
                        const double rkc = Rd[c * 16 + k];
                        if (k & 1) s1 -= x[k] * rkc;
                        else s0 -= x[k] * rkc;
                    }
                }
                x[c] = (s0 + s1) * rcp_nr(Rd[c * 16 + c]);
            }
            double* Xd = Xs + blk(wave, wave);
#pragma unroll
            for (int c = 0; c < 16; ++c) Xd[c * 16 + j] = x[c];  // zero below the diagonal
        }
        __syncthreads();
        const int r = j & 15, cq = j >> 4;  // lane: row r, columns 4 cq .. 4 cq + 3 of a block
        for (int d = 1; d < NB; ++d) {
            const int ib = wave, jb = wave + d;
            if (jb < NB) {
                double tv[4] = {0.0, 0.0, 0.0, 0.0};  // T = sum_{kb=ib+1..jb} R_{ib,kb} X_{kb,jb}
                for (int kb = ib + 1; kb <= jb; ++kb) {
                    const double* Rb = Rs + blk(ib, kb);
                    const double* Xb = Xs + blk(kb, jb);
#pragma unroll
                    for (int m = 0; m < 16; ++m) {
                        const double rv = Rb[m * 16 + r];
#pragma unroll
                        for (int cc = 0; cc < 4; ++cc) tv[cc] = fma(rv, Xb[(4 * cq + cc) * 16 + m], tv[cc]);
                    }
                }
                // T goes through the (still unused) slot of X_{ib,jb}: written, read, then overwritten
                double* T = Xs + blk(ib, jb);
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) T[(4 * cq + cc) * 16 + r] = tv[cc];
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                const double* Xd = Xs + blk(ib, ib);
                double xv[4] = {0.0, 0.0, 0.0, 0.0};  // X_{ib,jb} = -X_{ib,ib} T
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const double xim = Xd[m * 16 + r];
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) xv[cc] = fma(-xim, T[(4 * cq + cc) * 16 + m], xv[cc]);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) T[(4 * cq + cc) * 16 + r] = xv[cc];
            }
            __syncthreads();
        }
        for (int e = tid; e < LP * LP; e += NTHR) {
            const int t = e % LP, c = e / LP;
            const double v = ((t >> 4) <= (c >> 4)) ? Xs[blk(t >> 4, c >> 4) + (c & 15) * 16 + (t & 15)] : 0.0;
            a.R64[e] = v;
            a.R32[e] = (float)v;
        }
    } else {
        for (int e = tid; e < LP * LP; e += NTHR) {
            const double v = (e % LP == e / LP) ? 1.0 : 0.0;
            a.R64[e] = v;
            a.R32[e] = (float)v;
        }
    }
}

hipError_t launch_chol_inv(int lp, const GroupLaunch<CholArgs>& L, hipStream_t st) {
    switch (lp) {
        case 16: hipLaunchKernelGGL(k_chol_blk<1>, dim3(L.count), dim3(64), 0, st, mkg(L)); break;
        case 32: hipLaunchKernelGGL(k_chol_blk<2>, dim3(L.count), dim3(128), 0, st, mkg(L)); break;
        case 48: hipLaunchKernelGGL(k_chol_blk<3>, dim3(L.count), dim3(192), 0, st, mkg(L)); break;
        case 64: hipLaunchKernelGGL(k_chol_blk<4>, dim3(L.count), dim3(256), 0, st, mkg(L)); break;
        case 80: hipLaunchKernelGGL(k_chol_blk<5>, dim3(L.count), dim3(320), 0, st, mkg(L)); break;
        case 96: hipLaunchKernelGGL(k_chol_blk<6>, dim3(L.count), dim3(384), 0, st, mkg(L)); break;
        case 112: hipLaunchKernelGGL(k_chol_blk<7>, dim3(L.count), dim3(448), 0, st, mkg(L)); break;
        case 128: hipLaunchKernelGGL(k_chol_blk<8>, dim3(L.count), dim3(512), 0, st, mkg(L)); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small SVD of step 6 (eigenvectors of G_B = T T^T), one workgroup per matrix.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double shfl_xor_d(double v, int mask) {
    return __shfl_xor(v, mask, 64);
}

// Value of lane (l ^ pattern) within rows of 16 by a DPP move (both halves).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
constexpr int DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140, DPP_QUAD_1032 = 0xB1, DPP_QUAD_2301 = 0x4E;

// Sum over each aligned group of 8 lanes, the same bits in all 8 lanes
// (the three steps pair commuting operands).
__device__ __forceinline__ double sum8(double x) {
    x += dpp_d<DPP_HALF_MIRROR>(x);
    x += dpp_d<DPP_QUAD_1032>(x);
    x += dpp_d<DPP_QUAD_2301>(x);
    return x;
}

// Maximum over the wave, returned uniformly.
__device__ __forceinline__ double wave_max(double x) {
    x = fmax(x, dpp_d<DPP_HALF_MIRROR>(x));
    x = fmax(x, dpp_d<DPP_QUAD_1032>(x));
    x = fmax(x, dpp_d<DPP_QUAD_2301>(x));
    x = fmax(x, dpp_d<DPP_MIRROR>(x));
    return fmax(fmax(read_lane(x, 0), read_lane(x, 16)), fmax(read_lane(x, 32), read_lane(x, 48)));
}

// Preconditioned one-sided Jacobi (Drmac and Veselic, SIMAX 2008): with the
// diagonally pivoted Cholesky factorisation G = P L L^T P^T, the left
// singular vectors of P L are the eigenvectors of G and its singular values
// the square roots of G's eigenvalues. One-sided Jacobi on the columns of
// P L (a row permutation does not change the column inner products) then
// needs few sweeps. Results: UB[:, k] = (P L V)[:, k] / sigma_k by
// descending sigma_k = ||(P L V)[:, k]||; factorisation stops at the first
// pivot below lp u times the largest diagonal entry of G (the remaining
// columns are zero, as are their sigma and UB columns).
// lp <= 64: the factorisation runs in one wave without moving data: lane i
// keeps row i of the Schur complement (original order) in registers, the
// pivot is the largest remaining diagonal entry (lowest index on ties), its
// row is published through LDS, and column j of P L is stored in original
// row order. lp > 64: the workgroup factorises with symmetric swaps in LDS.
// Sweeps: round-robin pairs, eight lanes per pair (each lane two pairs of
// adjacent rows per 16-row group, 16-byte LDS accesses), sums by DPP.
// Factor route (C non-NULL): the columns of C (C C^T = T T^T, from an
// orthonormal basis of T^T rather than from the Gram matrix) are loaded as
// they are, with no permutation, and the sweeps start at once.
template <int LP, int NTHR>
__device__ __forceinline__ void jacobi_chol_body(const double* __restrict__ G, int l, double* __restrict__ UB,
                                                 double* __restrict__ sig, int* flags, double tol, int* sweeps_out,
                                                 const double* __restrict__ C = nullptr, int64_t ldc = 0) {
    constexpr int NPAIR = LP / 2;
    constexpr int TPP = NTHR / NPAIR;
    constexpr int RPT = LP / TPP;
    static_assert(TPP == 8 && RPT * TPP == LP, "pair layout: eight lanes per pair");
    // column stride: the smallest >= LP that is 16 mod 64 doubles, so consecutive columns start
    // 128 bytes apart within the LDS's 512-byte window. The 32 lanes of one cycle are four column
    // pairs' 128-byte runs (eight lanes per pair), mostly of consecutive columns: with LP + 2 they
    // overlapped and 41 % of the LDS cycles were bank conflicts
    constexpr int LDW = LP + (((16 - LP) % 64) + 64) % 64;
    __shared__ __attribute__((aligned(16))) double W[LP * LDW];   // A[row][col] at W[col * LDW + row]
    __shared__ double nrm[LP];
    __shared__ int perm[LP];
    __shared__ int s_rank, s_rot;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (C != nullptr) {
        for (int e = tid; e < LP * LDW; e += NTHR) {
            const int c = e / LDW, row = e % LDW;
            W[e] = (c < l && row < l) ? C[(int64_t)c * ldc + row] : 0.0;
        }
        for (int c = tid; c < LP; c += NTHR) perm[c] = c;
        __syncthreads();
    } else if constexpr (LP <= 64) {
        __shared__ __attribute__((aligned(16))) double rowbuf[64];
        for (int e = tid; e < LP * LDW; e += NTHR) W[e] = 0.0;
        for (int c = tid; c < LP; c += NTHR) perm[c] = c;
        __syncthreads();
        if (wave == 0) {
            const int i = lane;
            const bool live = i < l;
            double a[LP];  // row i of the Schur complement, original column order
#pragma unroll
            for (int k = 0; k < LP; ++k) a[k] = (live && k < l) ? G[i * LP + k] : 0.0;
            double dg = live ? G[i * LP + i] : 0.0;
            const double thr = (double)LP * 0x1.0p-53 * wave_max(live ? dg : 0.0);
            bool done = !live;
            int rank = l;
            for (int j = 0; j < l; ++j) {
                const double v = done ? -1.0 : dg;
                const double vmax = wave_max(v);
                if (!(vmax > thr)) {  // remaining Schur complement negligible (or not finite)
                    rank = j;
                    break;
                }
                const int pv = __ffsll((unsigned long long)__ballot(!done && v == vmax)) - 1;
                if (i == pv) {
#pragma unroll
                    for (int k = 0; k < LP; ++k) rowbuf[k] = a[k];
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                const double app = rowbuf[pv];
                const double inv = rsqrt_nr(app), ljj = app * inv;
                double lij = done ? 0.0 : rowbuf[i] * inv;
                if (i == pv) {
                    lij = ljj;
                    done = true;
                }
                if (i < LP) W[j * LDW + i] = lij;
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                if (!done) {
#pragma unroll
                    for (int k = 0; k < LP; ++k) a[k] -= lij * W[j * LDW + k];
                    dg -= lij * lij;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            }
            if (lane == 0) s_rank = rank;
        }
        __syncthreads();
        if (tid == 0 && s_rank < l) atomicOr(flags, DEV_FLAG_RANK_CUT);
    } else {
        __shared__ double s_val[NTHR / 64];
        __shared__ int s_idx[NTHR / 64];
        __shared__ int s_piv;
        __shared__ double s_dmax;
        for (int e = tid; e < LP * LP; e += NTHR) {
            const int c = e / LP, row = e % LP;
            W[c * LDW + row] = (c < l && row < l) ? G[row * LP + c] : 0.0;
        }
        for (int c = tid; c < LP; c += NTHR) perm[c] = c;
        if (tid == 0) {
            double dm = 0.0;
            for (int i = 0; i < l; ++i) dm = fmax(dm, G[i * LP + i]);
            s_dmax = dm;
            s_rank = l;
        }
        __syncthreads();
        const double thr = (double)LP * 0x1.0p-53 * s_dmax;
        // diagonally pivoted Cholesky (right-looking, full symmetric storage)
        for (int j = 0; j < l; ++j) {
            // pivot: largest remaining diagonal entry, lowest index on ties
            double bv = -1.0;
            int bi = LP;
            for (int i = j + tid; i < l; i += NTHR) {
                const double v = W[i * LDW + i];
                if (v > bv) { bv = v; bi = i; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = shfl_xor_d(bv, off);
                const int oi = __shfl_xor(bi, off, 64);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            if (lane == 0) { s_val[wave] = bv; s_idx[wave] = bi; }
            __syncthreads();
            if (tid == 0) {
                double v = s_val[0];
                int ix = s_idx[0];
                for (int w = 1; w < NTHR / 64; ++w)
                    if (s_val[w] > v || (s_val[w] == v && s_idx[w] < ix)) { v = s_val[w]; ix = s_idx[w]; }
                s_piv = ix;
                if (!(v > thr)) s_rank = j;
            }
            __syncthreads();
            if (s_rank == j) break;
            const int pv = s_piv;
            if (pv != j) {  // symmetric swap of rows and columns j and pv
                for (int k = tid; k < LP; k += NTHR) {
                    const double a = W[k * LDW + j];
                    W[k * LDW + j] = W[k * LDW + pv];
                    W[k * LDW + pv] = a;
                }
                __syncthreads();
                for (int k = tid; k < LP; k += NTHR) {
                    const double a = W[j * LDW + k];
                    W[j * LDW + k] = W[pv * LDW + k];
                    W[pv * LDW + k] = a;
                }
                if (tid == 0) {
                    const int t = perm[j];
                    perm[j] = perm[pv];
                    perm[pv] = t;
                }
                __syncthreads();
            }
            const double ljj = sqrt(W[j * LDW + j]);
            const double inv = 1.0 / ljj;
            __syncthreads();
            for (int i = j + 1 + tid; i < l; i += NTHR) W[j * LDW + i] *= inv;   // column j below the diagonal
            if (tid == 0) W[j * LDW + j] = ljj;
            __syncthreads();
            // trailing update, both triangles: A[i][k] -= L[i][j] L[k][j]
            const int nt = l - j - 1;
            for (int e = tid; e < nt * nt; e += NTHR) {
                const int k = j + 1 + e / nt, i = j + 1 + e % nt;
                W[k * LDW + i] -= W[j * LDW + i] * W[j * LDW + k];
            }
            __syncthreads();
        }
        // L: lower triangle of the first `rank` columns; everything else zero
        const int rank = s_rank;
        if (tid == 0 && rank < l) atomicOr(flags, DEV_FLAG_RANK_CUT);
        for (int e = tid; e < LP * LP; e += NTHR) {
            const int c = e / LP, row = e % LP;
            if (c >= rank || row < c || row >= l) W[c * LDW + row] = 0.0;
        }
        __syncthreads();
    }
    // ---- one-sided Jacobi on the columns ----
    const int pr = tid / TPP, sub = tid % TPP;
    int sweep = 0;
    constexpr int max_sweeps = 40;
    for (; sweep < max_sweeps; ++sweep) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        bool rot = false;  // this lane's pair rotated during the sweep
        for (int rnd = 0; rnd < LP - 1; ++rnd) {
            int p, q;
            if (pr == 0) {
                p = LP - 1;
                q = rnd;
            } else {
                p = rnd + pr;
                if (p >= LP - 1) p -= LP - 1;
                q = rnd - pr;
                if (q < 0) q += LP - 1;
            }
            if (p > q) {
                const int t = p;
                p = q;
                q = t;
            }
            // lane sub: rows 16 k + 2 sub, 16 k + 2 sub + 1 (k < RPT / 2)
            typedef double d2 __attribute__((ext_vector_type(2)));
            d2 wp[RPT / 2], wq[RPT / 2];
#pragma unroll
            for (int k = 0; k < RPT / 2; ++k) {
                wp[k] = *reinterpret_cast<const d2*>(W + p * LDW + 16 * k + 2 * sub);
                wq[k] = *reinterpret_cast<const d2*>(W + q * LDW + 16 * k + 2 * sub);
            }
            double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
            for (int k = 0; k < RPT / 2; ++k)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    al += wp[k][h] * wp[k][h];
                    be += wq[k][h] * wq[k][h];
                    ga += wp[k][h] * wq[k][h];
                }
            al = sum8(al);
            be = sum8(be);
            ga = sum8(ga);
            if (al > 0.0 && be > 0.0 && ga * ga > (tol * tol) * (al * be)) {  // |ga| > tol sqrt(al be)
                // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta = (be - al) / (2 ga), written as
                // t = sign(zeta) |2 ga| / (|be - al| + sqrt((be - al)^2 + (2 ga)^2)); c = 1 / sqrt(1 + t^2)
                const double d = be - al, e2 = 2.0 * ga;
                const double sg = (d == 0.0 || ((d > 0.0) == (e2 > 0.0))) ? 1.0 : -1.0;
                const double h2 = fma(d, d, e2 * e2);
                const double t = sg * fabs(e2) * rcp_nr(fabs(d) + h2 * rsqrt_nr(h2));
                const double c = rsqrt_nr(fma(t, t, 1.0)), s = c * t;
#pragma unroll
                for (int k = 0; k < RPT / 2; ++k) {
                    *reinterpret_cast<d2*>(W + p * LDW + 16 * k + 2 * sub) = c * wp[k] - s * wq[k];
                    *reinterpret_cast<d2*>(W + q * LDW + 16 * k + 2 * sub) = s * wp[k] + c * wq[k];
                }
                rot = true;
            }
            __syncthreads();
        }
        // one flag write per wave and sweep (a shared write every round costs 7 %)
        if (__ballot(rot) != 0 && lane == 0) s_rot = 1;
        __syncthreads();
        if (s_rot == 0) break;
        __syncthreads();
    }
    if (sweep == max_sweeps && tid == 0) atomicOr(flags, DEV_FLAG_JACOBI_SLOW);
    if (sweeps_out != nullptr && tid == 0) *sweeps_out = sweep;
    for (int c = tid; c < LP; c += NTHR) {
        double s = 0.0;
        for (int row = 0; row < LP; ++row) s += W[c * LDW + row] * W[c * LDW + row];
        nrm[c] = sqrt(s);
    }
    __syncthreads();
    for (int c = tid; c < LP; c += NTHR) {
        const double v = nrm[c];
        int rank_c = 0;
        for (int k = 0; k < LP; ++k) rank_c += (nrm[k] > v) || (nrm[k] == v && k < c);
        sig[rank_c] = v;
        const double inv = v > 0.0 ? 1.0 / v : 0.0;
        for (int row = 0; row < LP; ++row) UB[(int64_t)rank_c * LP + perm[row]] = W[c * LDW + row] * inv;
    }
}

// eight lanes per column pair: 4 lp threads per workgroup
template <int LP>
__global__ __launch_bounds__(4 * LP) void k_jacobi(Group<JacobiArgs> g) {
    if (group_skipped(g)) return;
    const JacobiArgs& a = g.args[blockIdx.x];  // one workgroup per matrix
    jacobi_chol_body<LP, 4 * LP>(a.G, a.l, a.UB, a.sig, a.flags, a.tol, nullptr, a.C, a.ldc);
}

int jacobi_threads(int lp) { return 4 * lp; }

hipError_t launch_jacobi(int lp, const GroupLaunch<JacobiArgs>& L, hipStream_t st) {
    switch (lp) {
#define RPOD_JAC_CASE(K) \
    case K: hipLaunchKernelGGL(k_jacobi<K>, dim3(L.count), dim3(4 * K), 0, st, mkg(L)); break;
        RPOD_JAC_CASE(16) RPOD_JAC_CASE(32) RPOD_JAC_CASE(48) RPOD_JAC_CASE(64)
        RPOD_JAC_CASE(80) RPOD_JAC_CASE(96) RPOD_JAC_CASE(112) RPOD_JAC_CASE(128)
#undef RPOD_JAC_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// M = Rinv * UB[:, :r] and Ur = UB[:, :r], both lp x rp column-major (zero pad).
__global__ void k_lift_coef(Group<LiftArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const LiftArgs& la = g.args[it];
    const double* __restrict__ Rinv = la.Rinv;
    const double* __restrict__ UB = la.UB;
    double* __restrict__ M64 = la.M64;
    float* __restrict__ M32 = la.M32;
    double* __restrict__ Ur = la.Ur;
    const int lp = la.lp, r = la.r, rp = la.rp;
    const int e = (blockIdx.x - g.tstart[it]) * blockDim.x + threadIdx.x;
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

hipError_t launch_lift_coef(const GroupLaunch<LiftArgs>& L, hipStream_t st) {
    hipLaunchKernelGGL(k_lift_coef, dim3(L.tiles), dim3(256), 0, st, mkg(L));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sign convention: per column, the entry of largest magnitude (lowest row on
// ties) is made positive. Partial argmax per (column, row chunk), then one
// thread per column combines chunks in order.
// ---------------------------------------------------------------------------
// grouped: local tile t covers row chunk t % nchunk of column t / nchunk
template <typename T>
__global__ __launch_bounds__(256) void k_colmax(Group<ColmaxArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const ColmaxArgs& a = g.args[it];
    const int t = blockIdx.x - g.tstart[it];
    const int c = t / a.nchunk, ch = t % a.nchunk;
    const GLOBAL T* __restrict__ Phi = gbl((const T*)a.Phi);
    const int64_t i0 = (int64_t)ch * a.chunk;
    const int64_t i1 = (i0 + a.chunk < a.m) ? i0 + a.chunk : a.m;
    double best = -1.0, bval = 0.0;
    int64_t bidx = INT64_MAX;
    const GLOBAL T* col = Phi + (int64_t)c * a.ld;
    auto visit = [&](double v, int64_t i) {  // increasing i per thread: strict > keeps the first
        const double av = fabs(v);
        if (av > best) { best = av; bidx = i; bval = v; }
    };
    constexpr int V = 16 / sizeof(T);  // 16-byte loads when the chunk starts on one
    if ((a.ld % V) == 0 && (i0 % V) == 0) {
        typedef T TV __attribute__((ext_vector_type(V)));
        for (int64_t i = i0 + (int64_t)threadIdx.x * V; i < i1; i += 256 * V) {
            if (i + V <= i1) {
                const TV v = *reinterpret_cast<const GLOBAL TV*>(col + i);
#pragma unroll
                for (int k = 0; k < V; ++k) visit((double)v[k], i + k);
            } else {
                for (int64_t k = i; k < i1; ++k) visit((double)col[k], k);
            }
        }
    } else {
        for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) visit((double)col[i], i);
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
        const int64_t slot = (int64_t)c * a.nchunk + ch;
        a.pval[slot] = (sb[0] < 0.0) ? 0.0 : sv[0];
        a.pidx[slot] = si[0];
    }
}

// One wave per column: lane k takes chunks k, k + 64, .., then a butterfly
// keeps the largest magnitude, lowest row on ties (the same entry whatever
// the order of the comparisons).
__global__ __launch_bounds__(64) void k_signs(Group<SignArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const SignArgs& a = g.args[it];
    const int c = blockIdx.x - g.tstart[it];
    if (c >= a.r) return;  // uniform
    const int lane = threadIdx.x;
    double best = -1.0, bval = 0.0;
    int64_t bidx = INT64_MAX;
    for (int k = lane; k < a.nchunk; k += 64) {
        const double v = a.pval[(int64_t)c * a.nchunk + k];
        const int64_t ix = a.pidx[(int64_t)c * a.nchunk + k];
        const double av = fabs(v);
        if (av > best || (av == best && ix < bidx)) { best = av; bval = v; bidx = ix; }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const double ob = shfl_xor_d(best, off), ov = shfl_xor_d(bval, off);
        const unsigned long long ub = (unsigned long long)bidx;
        const unsigned lo = (unsigned)__shfl_xor((int)(unsigned)ub, off, 64);
        const unsigned hi = (unsigned)__shfl_xor((int)(unsigned)(ub >> 32), off, 64);
        const int64_t oi = (int64_t)(((unsigned long long)hi << 32) | lo);
        if (ob > best || (ob == best && oi < bidx)) { best = ob; bval = ov; bidx = oi; }
    }
    if (lane == 0) a.signs[c] = (bval < 0.0) ? -1.0 : 1.0;
}

hipError_t launch_signs(int tphi, const GroupLaunch<ColmaxArgs>& C, const GroupLaunch<SignArgs>& S, hipStream_t st) {
    if (tphi == DT_F64)
        hipLaunchKernelGGL(k_colmax<double>, dim3(C.tiles), dim3(256), 0, st, mkg(C));
    else
        hipLaunchKernelGGL(k_colmax<float>, dim3(C.tiles), dim3(256), 0, st, mkg(C));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_signs, dim3(S.tiles), dim3(64), 0, st, mkg(S));
    return hipGetLastError();
}

// grouped: Phi tiles (rows 256 V (t % nb).., column t / nb, V elements of 16 bytes per
// thread); outputs from the call table
template <typename T>
__global__ void k_fin_phi(Group<FinArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const FinArgs& a = g.args[it];
    const int t = blockIdx.x - g.tstart[it];
    constexpr int V = 16 / sizeof(T);  // elements per thread
    const int nb = (int)((a.m + 256 * V - 1) / (256 * V));
    const int c = t / nb;
    const int64_t i = ((int64_t)(t % nb) * 256 + threadIdx.x) * V;
    if (i >= a.m) return;
    GLOBAL T* Pout = gbl((T*)g.calls[a.call].Phi) + (int64_t)c * a.m;
    const GLOBAL T* Pin = gbl((const T*)a.Phi_int) + (int64_t)c * a.ldP;
    const double sg = a.signs[c];  // +1 or -1: the products are exact
    if (i + V <= a.m && (a.m % V) == 0 && (a.ldP % V) == 0 && ((uintptr_t)Pout % 16) == 0) {
        typedef T TV __attribute__((ext_vector_type(V)));
        const TV v = *reinterpret_cast<const GLOBAL TV*>(Pin + i);
        TV o;
#pragma unroll
        for (int k = 0; k < V; ++k) o[k] = (T)(sg * (double)v[k]);
        *reinterpret_cast<GLOBAL TV*>(Pout + i) = o;
    } else {
        for (int64_t k = i; k < i + V && k < a.m; ++k) Pout[k] = (T)(sg * (double)Pin[k]);
    }
}

template <typename T>
__global__ void k_fin_a(Group<FinArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const FinArgs& a = g.args[it];
    const int64_t e = (int64_t)(blockIdx.x - g.tstart[it]) * blockDim.x + threadIdx.x;
    const CallDesc& cd = g.calls[a.call];
    if (e < (int64_t)a.r) cd.sigma[e] = a.sig[e];
    if (e >= a.n * a.r) return;
    const int64_t j = e / a.r;
    const int k = (int)(e % a.r);
    gbl((T*)cd.A)[e] = (T)(a.signs[k] * gbl(a.At)[(int64_t)k * a.ldA + j]);
}

int fin_phi_tiles(int64_t m, int r, int tphi) {
    const int64_t span = 256 * (tphi == DT_F64 ? 2 : 4);
    return (int)((m + span - 1) / span) * r;
}
int fin_a_tiles(int64_t n, int r) { return (int)(((n * r > r ? n * r : r) + 255) / 256); }

hipError_t launch_finalize(int tphi, const GroupLaunch<FinArgs>& P, const GroupLaunch<FinArgs>& A, hipStream_t st) {
    if (tphi == DT_F64) {
        hipLaunchKernelGGL(k_fin_phi<double>, dim3(P.tiles), dim3(256), 0, st, mkg(P));
        hipLaunchKernelGGL(k_fin_a<double>, dim3(A.tiles), dim3(256), 0, st, mkg(A));
    } else {
        hipLaunchKernelGGL(k_fin_phi<float>, dim3(P.tiles), dim3(256), 0, st, mkg(P));
        hipLaunchKernelGGL(k_fin_a<float>, dim3(A.tiles), dim3(256), 0, st, mkg(A));
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adaptive rank: identity factor, stopping decision, energy rank
// ---------------------------------------------------------------------------
__global__ void k_eye(Group<EyeArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const EyeArgs& a = g.args[it];
    const int e = (blockIdx.x - g.tstart[it]) * 256 + threadIdx.x;
    if (e < a.lp * a.lp) a.R[e] = (e / a.lp == e % a.lp) ? 1.0 : 0.0;
}

hipError_t launch_eye(const GroupLaunch<EyeArgs>& L, hipStream_t st) {
    hipLaunchKernelGGL(k_eye, dim3(L.tiles), dim3(256), 0, st, mkg(L));
    return hipGetLastError();
}

__global__ void k_adapt_decide(Group<AdaptDecideArgs> g) {
    if (group_skipped(g)) return;
    const AdaptDecideArgs& a = g.args[blockIdx.x];
    if (threadIdx.x != 0) return;
    const double f = *a.fro2;
    double E = f;
    for (int j = 0; j <= a.i; ++j) E -= a.cap[j];
    a.E[a.i] = E;
    const bool stop = E <= (1.0 - a.delta) * f || !(E == E) || a.i + 1 >= a.kmax;
    if (stop) {
        a.flags[ADAPT_STOP] |= 1 << (a.i + 1);
        a.flags[ADAPT_LUSED] = (a.i + 1) * a.b;
    } else {
        a.flags[ADAPT_ACTIVE] |= 1 << (a.i + 1);
    }
}

hipError_t launch_adapt_decide(const GroupLaunch<AdaptDecideArgs>& L, hipStream_t st) {
    hipLaunchKernelGGL(k_adapt_decide, dim3(L.count), dim3(64), 0, st, mkg(L));
    return hipGetLastError();
}

__global__ void k_adapt_rank(Group<AdaptRankArgs> g) {
    if (group_skipped(g)) return;
    const AdaptRankArgs& a = g.args[blockIdx.x];
    if (threadIdx.x != 0) return;
    const double f = *a.fro2;
    double cum = 0.0;
    int r = -1;
    for (int k = 0; k < a.l; ++k) {
        cum += __dmul_rn(a.sig[k], a.sig[k]);  // no fused multiply-add: the host's rounding
        if (cum / f >= a.delta) {
            r = k + 1;
            break;
        }
    }
    a.flags[ADAPT_RANK] = r;
}

hipError_t launch_adapt_rank(const GroupLaunch<AdaptRankArgs>& L, hipStream_t st) {
    hipLaunchKernelGGL(k_adapt_rank, dim3(L.count), dim3(64), 0, st, mkg(L));
    return hipGetLastError();
}

}  // namespace rpod
