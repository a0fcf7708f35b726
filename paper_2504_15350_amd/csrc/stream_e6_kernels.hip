// Passes over an FP32 snapshot matrix on the BF16 matrix cores.
//
// Every FP32 value x is split exactly into three bfloat16 parts
//   x = h + m + l,  h = bf16(x), m = bf16(x - h), l = bf16(x - h - m)
// (each difference is exact in FP32). A product of two split operands keeps
// the six terms hh, hm, mh, hl, mm, lh, each an exact BF16 x BF16 product
// accumulated in FP32 by the 16x16x32 MFMA. With |m| <= 2^-8 |x| and
// |l| <= 2^-16 |x| the dropped terms ml, lm, ll weigh together about
// 2^-23 |x| |y|, the size of one FP32 rounding of the product, so a dot
// product is as accurate as one with FP32 products and FP32 accumulation.
// The BF16 matrix cores run 16 times the FP32 rate: with six products per
// term both passes stay bound by HBM, not by the FP32 matrix-core rate.
//
//   k_sx_e6   Y = S X   (X in FP32, split as it is staged)
//   k_stq_e6  slabs of Z = S^T Q (Q split as it is staged), interleaved row splits
//
// MFMA operand layout (16x16x32 bf16, gfx950): lane l supplies
// A[l%16][8(l/16) + i] and B[8(l/16) + i][l%16], i = 0..7; the result holds
// D[4(l/16) + v][l%16].
#include <hip/hip_bf16.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace rpod {

typedef __bf16 e6_bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short e6_u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mma_bf16(e6_u16x8 a, e6_u16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(e6_bf16x8, a), __builtin_bit_cast(e6_bf16x8, b),
                                                   c, 0, 0, 0);
}

typedef float e6_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 e6_bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned e6_u32x4 __attribute__((ext_vector_type(4)));

// Three-way split of two values; each result word packs the parts of a
// (low half) and b (high half). Rounding to nearest at every level.
__device__ __forceinline__ void split_pair(float a, float b, unsigned& h, unsigned& m, unsigned& l) {
    const e6_f32x2 x{a, b};
    h = __builtin_bit_cast(unsigned, __builtin_convertvector(x, e6_bf16x2));
    const e6_f32x2 r = x - e6_f32x2{__builtin_bit_cast(float, h << 16), __builtin_bit_cast(float, h & 0xffff0000u)};
    m = __builtin_bit_cast(unsigned, __builtin_convertvector(r, e6_bf16x2));
    const e6_f32x2 t = r - e6_f32x2{__builtin_bit_cast(float, m << 16), __builtin_bit_cast(float, m & 0xffff0000u)};
    l = __builtin_bit_cast(unsigned, __builtin_convertvector(t, e6_bf16x2));
}

// eight values (x0 then x1) -> the three BF16 operands
__device__ __forceinline__ void split8(f32x4 x0, f32x4 x1, e6_u16x8& ah, e6_u16x8& am, e6_u16x8& al) {
    e6_u32x4 h, m, l;
    unsigned a, b, c;
    split_pair(x0[0], x0[1], a, b, c); h[0] = a; m[0] = b; l[0] = c;
    split_pair(x0[2], x0[3], a, b, c); h[1] = a; m[1] = b; l[1] = c;
    split_pair(x1[0], x1[1], a, b, c); h[2] = a; m[2] = b; l[2] = c;
    split_pair(x1[2], x1[3], a, b, c); h[3] = a; m[3] = b; l[3] = c;
    ah = __builtin_bit_cast(e6_u16x8, h);
    am = __builtin_bit_cast(e6_u16x8, m);
    al = __builtin_bit_cast(e6_u16x8, l);
}

// acc += the six leading terms of (ah + am + al)(bh + bm + bl), small terms first
__device__ __forceinline__ void mma6(const e6_u16x8& ah, const e6_u16x8& am, const e6_u16x8& al, const e6_u16x8& bh,
                                     const e6_u16x8& bm, const e6_u16x8& bl, f32x4& acc) {
    f32x4 s = acc;
    s = mma_bf16(al, bh, s);
    s = mma_bf16(am, bm, s);
    s = mma_bf16(ah, bl, s);
    s = mma_bf16(am, bh, s);
    s = mma_bf16(ah, bm, s);
    acc = mma_bf16(ah, bh, s);
}

// Four consecutive rows i..i+3 of column j (FP32), rows >= lim or columns >= n read 0.
template <bool VEC>
__device__ __forceinline__ f32x4 e6_rows4(const GLOBAL float* S, int64_t ld, int64_t lim, int64_t n, int64_t i,
                                          int64_t j) {
    f32x4 v = {0, 0, 0, 0};
    if (j < n) {
        const GLOBAL float* p = S + j * ld + i;
        if (VEC && i + 3 < lim) {
            v = __builtin_nontemporal_load(reinterpret_cast<const GLOBAL f32x4*>(p));  // streamed once
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (i + t < lim) v[t] = p[t];
        }
    }
    return v;
}

// ---------------------------------------------------------------------------
// Y = S X. Workgroup = 4 waves = 256 rows. Per 32-column step lane (r, g)
// of a wave holds rows 4 r .. 4 r + 3 of columns j0 + 8 g + i, i = 0..7 (a
// wave instruction covers 4 columns x 256 bytes); element t of these is the
// A operand of row tile t (MFMA row r of tile t is row 4 r + t of the wave),
// K index 8 g + i. The step's block of X (32 rows x 16 NT columns, read in
// FP32 and split into its three BF16 parts as it is staged) is kept in LDS,
// double-buffered, and shared by the four waves. All four tiles are split before the matrix-core work, and the next
// step's S columns are loaded after it.
// ---------------------------------------------------------------------------
constexpr int E6_XLD = 40;  // halfwords per staged X column (32 rows + pad)

// TALL (products with few columns of S, K = 16 nt or r + 1: the tall R^-1 applications, the lift,
// the reconstruction): the next step's S columns are loaded as soon as the current ones are split,
// before the matrix-core work (with four steps per workgroup every exposed load latency counts:
// 1048576 x 128 times 128 x 128, 367 against 393 us); long passes over S keep the loads after the
// matrix-core work (262144 x 5000 with 64 columns: 1.07 against 1.12 ms).
template <int NT, bool VEC, bool EN = false, bool TALL = false>
__device__ __forceinline__ void sx_e6_body(const GLOBAL float* S, int64_t ldS, int64_t m, int64_t n,
                                           const GLOBAL float* __restrict__ X, int64_t ldX,
                                           GLOBAL float* Y, int64_t ldY, int64_t mstore, int cmax, int64_t bx,
                                           unsigned short* xs, double* ssq = nullptr) {
    constexpr int XPART = 16 * NT * E6_XLD;     // one staged part
    constexpr int XB = 3 * XPART;               // one staged X block (three parts)
    constexpr int XCH = 16 * NT * 8;            // 16-byte FP32 chunks of a block (4 rows each)
    constexpr int XPT = (XCH + 255) / 256;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int64_t iw = bx * 256 + wave * 64;
    const int64_t irow = iw + 4 * r16;
    const bool fast = VEC && iw + 64 <= m;  // whole wave in range: unguarded vector loads
    f32x4 acc[4][NT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[t][c] = f32x4{0, 0, 0, 0};
    f32x4 sv[8];
    auto load_s = [&](int64_t j0) {
        if (fast && j0 + 32 <= n) {
            const GLOBAL float* p = S + (j0 + 8 * g) * ldS + irow;
#pragma unroll
            for (int i = 0; i < 8; ++i)
                sv[i] = __builtin_nontemporal_load(reinterpret_cast<const GLOBAL f32x4*>(p + i * ldS));
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) sv[i] = e6_rows4<VEC>(S, ldS, m, n, irow, j0 + 8 * g + i);
        }
    };
    f32x4 xr[XPT];
    auto load_x = [&](int64_t j0) {
#pragma unroll
        for (int q = 0; q < XPT; ++q) {
            const int ch = tid + 256 * q;
            if (ch < XCH) xr[q] = *reinterpret_cast<const GLOBAL f32x4*>(X + (int64_t)(ch >> 3) * ldX + j0 + 4 * (ch & 7));
        }
    };
    // chunk (rows 4 k .. 4 k + 3 of a column) -> 8 bytes of each part
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    auto put_x = [&](int buf) {
#pragma unroll
        for (int q = 0; q < XPT; ++q) {
            const int ch = tid + 256 * q;
            if (ch < XCH) {
                unsigned h0, m0, l0, h1, m1, l1;
                split_pair(xr[q][0], xr[q][1], h0, m0, l0);
                split_pair(xr[q][2], xr[q][3], h1, m1, l1);
                unsigned short* d = xs + buf * XB + (ch >> 3) * E6_XLD + 4 * (ch & 7);
                *reinterpret_cast<u32x2*>(d) = u32x2{h0, h1};
                *reinterpret_cast<u32x2*>(d + XPART) = u32x2{m0, m1};
                *reinterpret_cast<u32x2*>(d + 2 * XPART) = u32x2{l0, l1};
            }
        }
    };
    load_s(0);  // rows >= m read as 0 (guarded path)
    load_x(0);
    put_x(0);
    int buf = 0;
    double sq = 0.0;  // EN: sum of the squares of this lane's S entries (FP32 per step, FP64 across steps)
    for (int64_t j0 = 0; j0 < n; j0 += 32) {  // uniform trip count: the barriers below are reached by all waves
        const bool more = j0 + 32 < n;
        if constexpr (EN) {
            float p = 0.0f;
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int t = 0; t < 4; ++t) p = fmaf(sv[i][t], sv[i][t], p);
            sq += (double)p;
        }
        e6_u16x8 ah[4], am[4], al[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            split8(f32x4{sv[0][t], sv[1][t], sv[2][t], sv[3][t]}, f32x4{sv[4][t], sv[5][t], sv[6][t], sv[7][t]}, ah[t],
                   am[t], al[t]);
        if (more) {
            load_x(j0 + 32);
            if (TALL) load_s(j0 + 32);  // sv is free once split
        }
        __syncthreads();  // block buf staged
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const unsigned short* xb = xs + buf * XB + (16 * c + r16) * E6_XLD + 8 * g;
            const e6_u16x8 bh = *reinterpret_cast<const e6_u16x8*>(xb);
            const e6_u16x8 bm = *reinterpret_cast<const e6_u16x8*>(xb + XPART);
            const e6_u16x8 bl = *reinterpret_cast<const e6_u16x8*>(xb + 2 * XPART);
#pragma unroll
            for (int t = 0; t < 4; ++t) mma6(ah[t], am[t], al[t], bh, bm, bl, acc[t][c]);
        }
        if (more) {
            if (!TALL) load_s(j0 + 32);
            put_x(buf ^ 1);  // block buf ^ 1 was last read before this step's barrier
            buf ^= 1;
        }
    }
    if constexpr (EN) *ssq = sq;
    // D[4 g + v][r] of tile t: row iw + 4 (4 g + v) + t, output column 16 c + r
#pragma unroll
    for (int c = 0; c < NT; ++c) {
        if (16 * c + r16 >= cmax) continue;
        GLOBAL float* py = Y + (int64_t)(16 * c + r16) * ldY;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = iw + 4 * (4 * g + v);
            if (row + 3 < mstore) {
                *reinterpret_cast<GLOBAL f32x4*>(py + row) =
                    f32x4{acc[0][c][v], acc[1][c][v], acc[2][c][v], acc[3][c][v]};
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (row + t < mstore) py[row + t] = acc[t][c][v];
            }
        }
    }
}

// EN: the energy report's variant (also each tile's sum of squares of S, in
// a fixed order: per lane, then a tree over the workgroup)
template <int NT, bool VEC, bool EN = false, bool TALL = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT <= 4 ? 2 : 1, 2))) void k_sx_e6(
    Group<SxArgs> g) {
    if (group_skipped(g)) return;
    __shared__ __attribute__((aligned(16))) unsigned short xs[2 * 3 * 16 * NT * E6_XLD];
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const SxArgs& a = g.args[it];
    if (a.cond != nullptr && !(*a.cond & a.cond_mask)) return;
    const void* S = static_cast<const char*>(a.call >= 0 ? g.calls[a.call].S : a.S) + a.col0 * a.ldS * 4;
    if constexpr (EN) {
        __shared__ double red[256];
        double sq = 0.0;
        sx_e6_body<NT, VEC, true>(gbl((const float*)S), a.ldS, a.m, a.n, gbl((const float*)a.X), a.ldX,
                                  gbl((float*)a.Y), a.ldY, a.mstore, a.cmax > 0 ? a.cmax : 16 * NT,
                                  blockIdx.x - g.tstart[it], xs, &sq);
        red[threadIdx.x] = sq;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0 && a.fpart != nullptr) a.fpart[blockIdx.x - g.tstart[it]] = red[0];
    } else {
        sx_e6_body<NT, VEC, false, TALL>(gbl((const float*)S), a.ldS, a.m, a.n, gbl((const float*)a.X), a.ldX,
                                         gbl((float*)a.Y), a.ldY, a.mstore, a.cmax > 0 ? a.cmax : 16 * NT,
                                         blockIdx.x - g.tstart[it], xs);
    }
}

// ---------------------------------------------------------------------------
// Z_s = S^T Q. Workgroup: 256 columns of S (four column tiles of 16 per
// wave), 32 rows per step; the step's S block (32 x 256, FP32) and the three
// BF16 parts of the Q block (32 x 16 NT, read as FP32 and split when staged)
// are staged in LDS column-major and the next step's blocks are loaded into
// registers during the matrix-core work. Lane (r, g) reads rows 8 g .. 8 g + 7
// of its S column (the A operand, split in registers) and of each Q column
// part (the B operand).
// Columns are stored unpadded with their 16-byte chunks XOR-swizzled (S
// column c: chunk k at k ^ ((c / 2) mod 8); Q column c: chunk k at
// k ^ ((c / 4) mod 4)), which keeps both the staging writes and the operand
// reads free of bank conflicts for every 16 lanes.
// Splits interleaved in units of 64 rows (256 bytes of an FP32 Q column):
// unit k of split s covers rows 64 (k nsplit + s) .. + 63, two steps. Each
// workgroup writes its FP32 accumulators as its split's slab (summed in FP64
// afterwards).
// Tiles go to the XCDs (workgroup b runs on XCD b mod 8) so that each XCD
// holds every column block of its splits: the Q rows of a split are then
// fetched into one L2 only.
// ---------------------------------------------------------------------------
constexpr int E6_R = 32, E6_LDS = E6_R, E6_LDQ = E6_R, E6_HB = 256;

template <int NT, bool VEC>
__device__ __forceinline__ void stq_e6_body(const GLOBAL float* __restrict__ S, int64_t ldS, int64_t m, int64_t n,
                                            const GLOBAL float* __restrict__ Q, int64_t ldQ,
                                            GLOBAL float* __restrict__ Zp, int64_t nP, int nsplit, int ncb,
                                            int tile, float* ss, unsigned short* qs) {
    constexpr int R = E6_R, LD = E6_LDS, LDQ = E6_LDQ, HB = E6_HB, U = HB / 64;
    constexpr int CPC = R / 4;                  // 16-byte S chunks per column
    constexpr int SPT = HB * CPC / 256;         // S chunks per thread
    constexpr int QCPC = R / 4;                 // 16-byte FP32 Q chunks per column
    constexpr int QCH = 16 * NT * QCPC;         // Q chunks per step
    constexpr int QPT = (QCH + 255) / 256;
    constexpr int QPART = 16 * NT * LDQ;        // halfwords per staged part
    const int cb = tile % ncb, sp = tile / ncb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int64_t j0 = (int64_t)cb * HB;
    const int64_t ib = (int64_t)sp * (2 * R), jump = (int64_t)nsplit * (2 * R) - R;
    // next step: the second half of the unit, or the first half of the next unit
    auto next = [&](int64_t i) { return ((i / R) & 1) ? i + jump : i + R; };

    f32x4 acc[U][NT];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[u][c] = f32x4{0, 0, 0, 0};

    f32x4 sr[SPT];
    f32x4 qr[QPT];
    // chunk q of a thread: column j0 + tid / CPC + q (256 / CPC), rows 4 (tid mod CPC) .. +3 of the step
    constexpr int CSTEP = 256 / CPC;
    const int64_t jt = j0 + tid / CPC;
    const GLOBAL float* sbase = S + jt * ldS + 4 * (tid % CPC);
    auto fetch = [&](int64_t i0) {
        if (VEC && i0 + R <= m) {  // whole step in range: one unguarded vector load per chunk
            const GLOBAL float* p = sbase + i0;
#pragma unroll
            for (int q = 0; q < SPT; ++q)
                sr[q] = (jt + CSTEP * q < n)
                            ? __builtin_nontemporal_load(reinterpret_cast<const GLOBAL f32x4*>(p + CSTEP * q * ldS))
                            : f32x4{0, 0, 0, 0};
        } else {
#pragma unroll
            for (int q = 0; q < SPT; ++q) {
                const int ch = tid + 256 * q;
                sr[q] = e6_rows4<VEC>(S, ldS, m, n, i0 + 4 * (ch % CPC), j0 + ch / CPC);
            }
        }
#pragma unroll
        for (int q = 0; q < QPT; ++q) {
            const int ch = tid + 256 * q;
            if (ch < QCH)
                qr[q] = *reinterpret_cast<const GLOBAL f32x4*>(Q + (int64_t)(ch / QCPC) * ldQ + i0 + 4 * (ch % QCPC));
        }
    };
    static_assert(CPC == 8 && QCPC == 8, "swizzle patterns assume 32-row steps");
    auto put = [&]() {
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int ch = tid + 256 * q, col = ch / CPC;
            *reinterpret_cast<f32x4*>(ss + col * LD + 4 * ((ch % CPC) ^ ((col >> 1) & 7))) = sr[q];
        }
        // Q chunk (rows 4 k .. 4 k + 3 of a column) -> 8 bytes of each part, in
        // half k mod 2 of the part's 16-byte chunk k / 2
        typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int q = 0; q < QPT; ++q) {
            const int ch = tid + 256 * q, col = ch / QCPC, k = ch % QCPC;
            if (ch < QCH) {
                unsigned h0, m0, l0, h1, m1, l1;
                split_pair(qr[q][0], qr[q][1], h0, m0, l0);
                split_pair(qr[q][2], qr[q][3], h1, m1, l1);
                const int o = col * LDQ + 8 * ((k >> 1) ^ ((col >> 2) & 3)) + 4 * (k & 1);
                *reinterpret_cast<u32x2*>(qs + o) = u32x2{h0, h1};
                *reinterpret_cast<u32x2*>(qs + QPART + o) = u32x2{m0, m1};
                *reinterpret_cast<u32x2*>(qs + 2 * QPART + o) = u32x2{l0, l1};
            }
        }
    };

    if (ib < m) fetch(ib);
    for (int64_t i0 = ib; i0 < m; i0 = next(i0)) {
        __syncthreads();  // previous step consumed
        put();
        __syncthreads();
        if (next(i0) < m) fetch(next(i0));  // in flight during the matrix-core work
        e6_u16x8 ah[U], am[U], al[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int col = 16 * U * wave + 16 * u + r16, sw = (col >> 1) & 7;
            const float* src = ss + col * LD;
            split8(*reinterpret_cast<const f32x4*>(src + 4 * ((2 * g) ^ sw)),
                   *reinterpret_cast<const f32x4*>(src + 4 * ((2 * g + 1) ^ sw)), ah[u], am[u], al[u]);
        }
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const int col = 16 * c + r16;
            const int o = col * LDQ + 8 * (g ^ ((col >> 2) & 3));
            const e6_u16x8 bh = *reinterpret_cast<const e6_u16x8*>(qs + o);
            const e6_u16x8 bm = *reinterpret_cast<const e6_u16x8*>(qs + QPART + o);
            const e6_u16x8 bl = *reinterpret_cast<const e6_u16x8*>(qs + 2 * QPART + o);
#pragma unroll
            for (int u = 0; u < U; ++u) mma6(ah[u], am[u], al[u], bh, bm, bl, acc[u][c]);
        }
    }
    // D[4 g + v][r]: S column j0 + 16 U w + 16 u + 4 g + v, Q column 16 c + r; the
    // slab keeps the FP32 accumulators as they are (summed in FP64 afterwards)
    GLOBAL float* zp = Zp + (int64_t)sp * nP * (16 * NT);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < NT; ++c)
            *reinterpret_cast<GLOBAL f32x4*>(zp + (int64_t)(16 * c + r16) * nP + j0 + 16 * U * wave + 16 * u + 4 * g) =
                acc[u][c];
}

template <int NT, bool VEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT <= 4 ? 2 : 1, 2))) void k_stq_e6(
    Group<StqArgs> g) {
    if (group_skipped(g)) return;
    __shared__ __attribute__((aligned(16))) float ss[E6_HB * E6_LDS];
    __shared__ __attribute__((aligned(16))) unsigned short qs[3 * 16 * NT * E6_LDQ];
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const StqArgs& a = g.args[it];
    const void* S = a.call >= 0 ? g.calls[a.call].S : a.S;
    // XCD-aware order: local tile b (XCD b mod 8 when the item starts at a
    // multiple of 8) takes tile (b mod 8) T / 8 + b / 8 of the item's T
    const int local = blockIdx.x - g.tstart[it], ntl = a.ncb * a.nsplit;
    const int tile = ((ntl & 7) == 0 && (g.tstart[it] & 7) == 0) ? (local & 7) * (ntl >> 3) + (local >> 3) : local;
    stq_e6_body<NT, VEC>(gbl((const float*)S), a.ldS, a.m, a.n, gbl((const float*)a.Q), a.ldQ, gbl((float*)a.Zp),
                         a.nP, a.nsplit, a.ncb, tile, ss, qs);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename A>
static Group<A> mke6(const GroupLaunch<A>& L) {
    Group<A> g;
    g.args = L.args;
    g.tstart = L.tstart;
    g.calls = L.calls;
    g.count = L.count;
    g.skip = L.skip;
    g.skip_mask = L.skip_mask;
    return g;
}

template <int NT>
static hipError_t sxe6_nt(const GroupLaunch<SxArgs>& L, bool vec, bool en, bool tall, hipStream_t st) {
    if (tall && vec && !en) {
        hipLaunchKernelGGL((k_sx_e6<NT, true, false, true>), dim3(L.tiles), dim3(256), 0, st, mke6(L));
        return hipGetLastError();
    }
    if (en) {
        if (vec)
            hipLaunchKernelGGL((k_sx_e6<NT, true, true>), dim3(L.tiles), dim3(256), 0, st, mke6(L));
        else
            hipLaunchKernelGGL((k_sx_e6<NT, false, true>), dim3(L.tiles), dim3(256), 0, st, mke6(L));
    } else if (vec) {
        hipLaunchKernelGGL((k_sx_e6<NT, true>), dim3(L.tiles), dim3(256), 0, st, mke6(L));
    } else {
        hipLaunchKernelGGL((k_sx_e6<NT, false>), dim3(L.tiles), dim3(256), 0, st, mke6(L));
    }
    return hipGetLastError();
}

template <int NT>
static hipError_t stqe6_nt(const GroupLaunch<StqArgs>& L, bool vec, hipStream_t st) {
    if (vec)
        hipLaunchKernelGGL((k_stq_e6<NT, true>), dim3(L.tiles), dim3(256), 0, st, mke6(L));
    else
        hipLaunchKernelGGL((k_stq_e6<NT, false>), dim3(L.tiles), dim3(256), 0, st, mke6(L));
    return hipGetLastError();
}

hipError_t launch_sx_e6(int nt, bool vec, bool en, bool tall, const GroupLaunch<SxArgs>& L, hipStream_t st) {
    switch (nt) {
#define RPOD_E6_CASE(K) case K: return sxe6_nt<K>(L, vec, en, tall, st);
        RPOD_E6_CASE(1) RPOD_E6_CASE(2) RPOD_E6_CASE(3) RPOD_E6_CASE(4)
        RPOD_E6_CASE(5) RPOD_E6_CASE(6) RPOD_E6_CASE(7) RPOD_E6_CASE(8)
#undef RPOD_E6_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stq_e6(int nt, bool vec, const GroupLaunch<StqArgs>& L, hipStream_t st) {
    switch (nt) {
#define RPOD_E6_CASE(K) case K: return stqe6_nt<K>(L, vec, st);
        RPOD_E6_CASE(1) RPOD_E6_CASE(2) RPOD_E6_CASE(3) RPOD_E6_CASE(4)
        RPOD_E6_CASE(5) RPOD_E6_CASE(6) RPOD_E6_CASE(7) RPOD_E6_CASE(8)
#undef RPOD_E6_CASE
        default: return hipErrorInvalidValue;
    }
}

int stq_e6_block_cols() { return E6_HB; }

}  // namespace rpod
