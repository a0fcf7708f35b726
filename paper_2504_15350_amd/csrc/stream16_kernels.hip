// Passes over a 16-bit snapshot matrix (bfloat16 or IEEE half) on the
// 16x16x32 matrix cores of gfx950, FP32 accumulation.
//
//   k_sx16    Y = S X    (X stored in the same 16-bit type)
//   k_stq16   Z = S^T Q  (Q given as 16-bit hi = round(Q) and, with LO, also
//                         lo = round(Q - hi) applied as a second product, so
//                         Q carries ~16 significant bits: the refinement pass
//                         for T = Q^T S)
//   k_split16 the hi/lo split of an FP32 Q
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
__device__ __forceinline__ u16x8 load_rows8(const GLOBAL unsigned short* S, int64_t ld, int64_t lim, int64_t n,
                                            int64_t i, int64_t j) {
    u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    if (j < n) {
        const GLOBAL unsigned short* p = S + j * ld + i;
        if (VEC && i + 7 < lim) {
            v = __builtin_nontemporal_load(reinterpret_cast<const GLOBAL u16x8*>(p));  // streamed once
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
// 32 (one MFMA K). Each chunk of S is staged in LDS column-major (every
// thread moves a 16-byte run of 8 rows; a column of the tile is one
// 512-byte coalesced read from HBM) and read back transposed by the LDS
// transpose reads of gfx950: lane (r, kg) of m-tile mt needs row
// 64 w + 16 mt + r of columns 8 kg .. 8 kg + 7, which two ds_read_b64_tr_b16
// deliver (below). The chunk of X (32 rows x 16 NT columns, column-major) is
// staged next to it and read as one 16-byte operand per output tile. The
// next chunk's global loads are issued before the current chunk's
// matrix-core work. (Two transpose reads per operand in place of eight
// 16-bit reads: 4.44 against 4.55 ms at 1048576 x 10000, lp = 128, with
// bit-identical results.)
// ---------------------------------------------------------------------------
constexpr int SX16_BM = 256, SX16_BK = 32;
// LDS strides. The LDS serves 32 lanes of a 16-byte access per cycle over a 512-byte window
// (measured on gfx950): the X operand reads (lanes: 16 columns x 2 chunks) need a stride of
// 16 (2 odd) bytes, 96 here; with 80 bytes they took two cycles. The S tile stride of 544 bytes
// with it: bank conflicts 40 % -> 25 % of the LDS cycles, S X 4.32 -> 4.27 and 4.34 -> 4.25 ms
// back to back, no measurable change inside the pipeline (4.30 ms), bit-identical.
constexpr int SX16_LDR = SX16_BM + 16;  // S tile column stride (elements; a multiple of 4 for 8-byte reads)
constexpr int SX16_LDX = SX16_BK + 16;  // X tile column stride (elements)

// LDS transpose read of 16-bit elements (gfx950 ds_read_b64_tr_b16), as
// measured on this part: within each group of 16 lanes, lane i receives
// element (i mod 4) of the 4-element (8-byte) runs addressed by lanes
// 4 j + i / 4 of the group, j = 0..3, in component j. With lane 4 j + q
// addressing rows 4 q .. 4 q + 3 of column j of a column-major tile, lane i
// receives row i of columns 0..3: one 16 x 4 transpose.
typedef short s16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ s16x4 lds_read_tr16(const unsigned short* p) {
    return __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4*)(p));
}

template <typename T16, int NT, bool VEC>
__device__ __forceinline__ void sx16_body(const GLOBAL unsigned short* __restrict__ S, int64_t ldS, int64_t m,
                                          int64_t n, const GLOBAL unsigned short* __restrict__ X, int64_t ldX,
                                          GLOBAL float* __restrict__ Y, int64_t ldY, int64_t mstore, int cmax,
                                          int64_t bx) {
    __shared__ __attribute__((aligned(16))) unsigned short tile[SX16_BK * SX16_LDR];
    __shared__ __attribute__((aligned(16))) unsigned short xt[16 * NT * SX16_LDX];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, kg = lane >> 4;
    const int64_t i0 = bx * SX16_BM;
    const int rg = tid & 31, cc = tid >> 5;  // S staging: rows 8 rg..+7 of columns cc + 8 q
    constexpr int XCH = 16 * NT * (SX16_BK / 8);  // 16-byte chunks of the X tile
    constexpr int XPT = (XCH + 255) / 256;

    f32x4 acc[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[mt][c] = f32x4{0, 0, 0, 0};

    if (i0 < m) {
        u16x8 st[4], xr[XPT];
        auto fetch = [&](int64_t j0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) st[q] = load_rows8<VEC>(S, ldS, m, n, i0 + 8 * rg, j0 + cc + 8 * q);
#pragma unroll
            for (int q = 0; q < XPT; ++q) {
                const int ch = tid + 256 * q;
                if (ch < XCH) {
                    const int c = ch / (SX16_BK / 8), part = ch % (SX16_BK / 8);
                    xr[q] = *reinterpret_cast<const GLOBAL u16x8*>(X + (int64_t)c * ldX + j0 + 8 * part);
                }
            }
        };
        fetch(0);
        // transpose-read source of lane (r16, kg): column 8 kg + r16 / 4 (and + 4), rows 4 (r16 % 4) ..
        // of the wave's m-tile
        const unsigned short* asrc = tile + (8 * kg + (r16 >> 2)) * SX16_LDR + wave * 64 + 4 * (r16 & 3);
        for (int64_t j0 = 0; j0 < n; j0 += SX16_BK) {
            __syncthreads();  // previous chunk fully consumed
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                unsigned short* dst = tile + (cc + 8 * q) * SX16_LDR + 8 * rg;
                *reinterpret_cast<u16x4*>(dst) = u16x4{st[q][0], st[q][1], st[q][2], st[q][3]};
                *reinterpret_cast<u16x4*>(dst + 4) = u16x4{st[q][4], st[q][5], st[q][6], st[q][7]};
            }
#pragma unroll
            for (int q = 0; q < XPT; ++q) {
                const int ch = tid + 256 * q;
                if (ch < XCH) {
                    const int c = ch / (SX16_BK / 8), part = ch % (SX16_BK / 8);
                    *reinterpret_cast<u16x8*>(xt + c * SX16_LDX + 8 * part) = xr[q];
                }
            }
            __syncthreads();
            if (j0 + SX16_BK < n) fetch(j0 + SX16_BK);  // in flight during the matrix-core work
            u16x8 b[NT];
#pragma unroll
            for (int c = 0; c < NT; ++c)
                b[c] = *reinterpret_cast<const u16x8*>(xt + (16 * c + r16) * SX16_LDX + 8 * kg);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const s16x4 lo = lds_read_tr16(asrc + 16 * mt), hi = lds_read_tr16(asrc + 16 * mt + 4 * SX16_LDR);
                const u16x8 a = {(unsigned short)lo[0], (unsigned short)lo[1], (unsigned short)lo[2], (unsigned short)lo[3],
                                 (unsigned short)hi[0], (unsigned short)hi[1], (unsigned short)hi[2], (unsigned short)hi[3]};
#pragma unroll
                for (int c = 0; c < NT; ++c) acc[mt][c] = mma16<T16>::run(a, b[c], acc[mt][c]);
            }
        }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            if (16 * c + r16 >= cmax) continue;
            const int64_t row = i0 + wave * 64 + 16 * mt + 4 * kg;
            GLOBAL float* py = Y + (int64_t)(16 * c + r16) * ldY + row;
            if (row + 3 < mstore) {
                *reinterpret_cast<GLOBAL f32x4*>(py) = acc[mt][c];
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (row + v < mstore) py[v] = acc[mt][c][v];
            }
        }
}

template <typename T16, int NT, bool VEC>
__global__ __launch_bounds__(256, 2) void k_sx16(Group<SxArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const SxArgs& a = g.args[it];
    const void* S = static_cast<const char*>(a.call >= 0 ? g.calls[a.call].S : a.S) + a.col0 * a.ldS * 2;
    sx16_body<T16, NT, VEC>(gbl((const unsigned short*)S), a.ldS, a.m, a.n, gbl((const unsigned short*)a.X), a.ldX,
                            gbl((float*)a.Y), a.ldY, a.mstore, a.cmax > 0 ? a.cmax : 16 * NT,
                            blockIdx.x - g.tstart[it]);
}

// ---------------------------------------------------------------------------
// Z_s = S_s^T Q_s, 16-bit S, Q given as 16-bit hi (and lo) parts.
// Workgroup: one per CU (its LDS), 4 x WN waves (stq16_grid), a block of
// 256 columns of S over the rows of split s, 128 rows per step. Per step the S block (128 x 256) and the Q block (128 x 16 NT, hi
// then lo) are staged in LDS; wave (wm, wn) multiplies S columns
// 64 wm .. 64 wm + 63 with the Q n-tiles wn NTW .. wn NTW + NTW - 1
// (NTW = ceil(NT / WN); tiles >= NT are skipped). Global reads cover
// 4 columns x 256 bytes per wave instruction (the shape that streams near the
// HBM peak) and are non-temporal; the next step's S and Q blocks are in
// flight during the matrix-core work. A step whose block lies wholly inside S
// loads without the per-lane bounds tests (measured: hi pass 4.83 -> 4.69 ms,
// hi + lo 6.18 -> 6.09 ms at 1048576 x 10000; the same change in S X was no
// faster). Operands are plain 16-byte LDS reads
// (K along rows):
//   A[mm][8 kg + i] = S[i0 + 32 k + 8 kg + i][j0 + 64 wm + 16 t + mm]
//   B[8 kg + i][nn] = Q[i0 + 32 k + 8 kg + i][16 c + nn]   (hi, then lo)
// so every accumulator sees its k steps in row order, hi before lo. Splits
// are interleaved (step t of split s covers rows 128 (t nsplit + s) .. +127),
// so the workgroups of one column block read neighbouring pieces of every
// column. Measured at 1048576 x 10000, lp = 128 (BF16, back to back): hi
// 4.71 ms against 5.15 ms for two 4-wave workgroups per CU on 128 x 128
// blocks (bit-identical slabs), hi + lo 6.27 ms against 7.41 ms (64-row steps
// there).
// ---------------------------------------------------------------------------
constexpr int STQ16_HB = 256;  // columns per block
constexpr int STQ16_R = 128;   // rows per step

// 4 x WN waves: hi 4 x 2; hi + lo 4 x 4, or 4 x 3 when that divides the Q tiles (96 columns), and
// 4 x 2 below 64 Q columns (16 waves would spill); 4 x 1 up to 32 Q columns (two workgroups per
// CU). A wave grid that divides the Q tiles keeps the matrix-core loop free of tile guards
// (measured: guards cost 0.5 ms of 5.3 at lp = 128).
template <bool LO, int NT> struct stq16_grid {
    static constexpr int WM = 4,
                         WN = NT <= 2 ? 1 : !(LO && NT >= 4) ? 2 : (NT % 4 != 0 && NT % 3 == 0) ? 3 : 4;
};

template <typename T16, int NT, bool VEC, bool LO>
__device__ __forceinline__ void stq16_body(const GLOBAL unsigned short* __restrict__ S, int64_t ldS, int64_t m,
                                           int64_t n, const GLOBAL unsigned short* __restrict__ Qh,
                                           const GLOBAL unsigned short* __restrict__ Ql, int64_t ldQ,
                                           GLOBAL float* __restrict__ Zp, int64_t nP, int nsplit, int ncb, int tile) {
    constexpr int WM = stq16_grid<LO, NT>::WM, WN = stq16_grid<LO, NT>::WN, NTHR = 64 * WM * WN;
    constexpr int R = STQ16_R, HB = STQ16_HB;
    // column stride of the LDS blocks: 288 bytes. The LDS serves 32 lanes of a 16-byte read per
    // cycle over a 512-byte window (measured on gfx950): lanes (column c, chunk kg < 2) then hit
    // 16-byte slot 18 c + kg mod 32, all distinct; a 272-byte stride (17 c + kg) put two lanes on
    // one slot and spent 36-40 % of the LDS cycles on bank conflicts (back to back: hi pass
    // 4.68 -> 4.57 ms, hi + lo 6.21 -> 6.09 ms; in the pipeline the call gains 0.1 ms;
    // bit-identical)
    constexpr int LDS_ = R + 16;
    constexpr int LPC = R / 8;    // 16-byte chunks per column of a block
    constexpr int NQ = LO ? 2 : 1;
    constexpr int MT = HB / WM / 16, NTW = (NT + WN - 1) / WN;
    __shared__ __attribute__((aligned(16))) unsigned short ss[HB * LDS_];
    __shared__ __attribute__((aligned(16))) unsigned short qs[NQ * 16 * NT * LDS_];
    const int cb = tile % ncb, sp = tile / ncb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, kg = lane >> 4, wm = wave % WM, wn = wave / WM;
    const int64_t j0 = (int64_t)cb * HB;
    const int64_t ib = (int64_t)sp * R, stride = (int64_t)nsplit * R;
    constexpr int SCHT = HB * LPC;                     // S chunks per block
    constexpr int SCH = (SCHT + NTHR - 1) / NTHR;      // ... per thread
    constexpr int QCH = 16 * NT * LPC;                 // Q chunks per block
    constexpr int QPT = (QCH + NTHR - 1) / NTHR;

    f32x4 acc[MT][NTW];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int c = 0; c < NTW; ++c) acc[t][c] = f32x4{0, 0, 0, 0};

    u16x8 sr[SCH], qr[NQ][QPT];
    auto fetch = [&](int64_t i0) {
#pragma unroll
        for (int q = 0; q < QPT; ++q) {
            const int ch = tid + NTHR * q;
            if (ch < QCH) {
                const int64_t off = (int64_t)(ch / LPC) * ldQ + i0 + 8 * (ch % LPC);
                qr[0][q] = *reinterpret_cast<const GLOBAL u16x8*>(Qh + off);
                if (LO) qr[NQ - 1][q] = *reinterpret_cast<const GLOBAL u16x8*>(Ql + off);
            }
        }
        if (VEC && i0 + R <= m && j0 + HB <= n) {   // whole block inside S: no per-lane bounds branches
#pragma unroll
            for (int q = 0; q < SCH; ++q) {
                const int ch = tid + NTHR * q;
                if (SCHT % NTHR == 0 || ch < SCHT)
                    sr[q] = __builtin_nontemporal_load(reinterpret_cast<const GLOBAL u16x8*>(
                        S + (j0 + ch / LPC) * ldS + i0 + 8 * (ch % LPC)));
            }
        } else {
#pragma unroll
            for (int q = 0; q < SCH; ++q) {
                const int ch = tid + NTHR * q;
                if (SCHT % NTHR == 0 || ch < SCHT) sr[q] = load_rows8<VEC>(S, ldS, m, n, i0 + 8 * (ch % LPC), j0 + ch / LPC);
            }
        }
    };
    if (ib < m) fetch(ib);
    for (int64_t i0 = ib; i0 < m; i0 += stride) {
        __syncthreads();  // previous step fully consumed
#pragma unroll
        for (int q = 0; q < SCH; ++q) {
            const int ch = tid + NTHR * q;
            if (SCHT % NTHR == 0 || ch < SCHT) *reinterpret_cast<u16x8*>(ss + (ch / LPC) * LDS_ + 8 * (ch % LPC)) = sr[q];
        }
#pragma unroll
        for (int q = 0; q < QPT; ++q) {
            const int ch = tid + NTHR * q;
            if (ch < QCH) {
#pragma unroll
                for (int h = 0; h < NQ; ++h)
                    *reinterpret_cast<u16x8*>(qs + (h * 16 * NT + ch / LPC) * LDS_ + 8 * (ch % LPC)) = qr[h][q];
            }
        }
        __syncthreads();
        if (i0 + stride < m) fetch(i0 + stride);  // next step, in flight during this one's work
#pragma unroll
        for (int k = 0; k < R / 32; ++k) {
            u16x8 b[NQ][NTW];
#pragma unroll
            for (int h = 0; h < NQ; ++h)
#pragma unroll
                for (int c = 0; c < NTW; ++c) {
                    const int nt = NTW * wn + c;
                    if (NT % WN == 0 || nt < NT)
                        b[h][c] = *reinterpret_cast<const u16x8*>(qs + (h * 16 * NT + 16 * nt + r16) * LDS_ + 32 * k +
                                                                  8 * kg);
                }
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                const u16x8 a = *reinterpret_cast<const u16x8*>(ss + (16 * MT * wm + 16 * t + r16) * LDS_ + 32 * k +
                                                                8 * kg);
#pragma unroll
                for (int h = 0; h < NQ; ++h)  // every accumulator: hi, then lo
#pragma unroll
                    for (int c = 0; c < NTW; ++c)
                        if (NT % WN == 0 || NTW * wn + c < NT) acc[t][c] = mma16<T16>::run(a, b[h][c], acc[t][c]);
            }
        }
    }
    GLOBAL float* zp = Zp + (int64_t)sp * nP * (16 * NT);  // FP32 slabs (summed in FP64 afterwards)
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int c = 0; c < NTW; ++c) {
            const int nt = NTW * wn + c;
            if (NT % WN == 0 || nt < NT)
                *reinterpret_cast<GLOBAL f32x4*>(zp + (int64_t)(16 * nt + r16) * nP + j0 + 16 * MT * wm + 16 * t +
                                                 4 * kg) = acc[t][c];
        }
}

// grouped launch: tile t covers column block t % ncb of split t / ncb. XCD-aware
// order (workgroup b runs on XCD b mod 8): when the item's tile count and its
// first workgroup are multiples of 8, local workgroup b takes tile
// (b mod 8) T / 8 + b / 8, so each XCD holds every column block of a range of
// splits and a split's Q rows are fetched into one L2 only.
template <typename T16, int NT, bool VEC, bool LO>
__global__ __launch_bounds__((64 * stq16_grid<LO, NT>::WM * stq16_grid<LO, NT>::WN)) void k_stq16(Group<StqArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const StqArgs& a = g.args[it];
    const void* S = a.call >= 0 ? g.calls[a.call].S : a.S;
    const int local = blockIdx.x - g.tstart[it], ntl = a.ncb * a.nsplit;
    const int tile = ((ntl & 7) == 0 && (g.tstart[it] & 7) == 0) ? (local & 7) * (ntl >> 3) + (local >> 3) : local;
    stq16_body<T16, NT, VEC, LO>(gbl((const unsigned short*)S), a.ldS, a.m, a.n, gbl((const unsigned short*)a.Q),
                                 gbl((const unsigned short*)a.Ql), a.ldQ, gbl((float*)a.Zp), a.nP, a.nsplit, a.ncb,
                                 tile);
}

// Split an FP32 tall matrix into 16-bit hi = round(c q) and lo = round(c q - hi), c a power of two.
template <typename T16>
__global__ void k_split16(Group<SplitArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const SplitArgs& sa = g.args[it];
    const GLOBAL float* __restrict__ Q = gbl(sa.Q);
    GLOBAL unsigned short* __restrict__ hi = gbl(sa.hi);
    GLOBAL unsigned short* __restrict__ lo = gbl(sa.lo);
    const int64_t e = ((int64_t)(blockIdx.x - g.tstart[it]) * blockDim.x + threadIdx.x) * 4;
    if (e >= sa.count) return;
    const f32x4 q = *reinterpret_cast<const GLOBAL f32x4*>(Q + e) * sa.scale;  // exact: a power of two
    u16x4 h, l;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        h[i] = mma16<T16>::from_float(q[i]);
        l[i] = mma16<T16>::from_float(q[i] - mma16<T16>::to_float(h[i]));
    }
    *reinterpret_cast<GLOBAL u16x4*>(hi + e) = h;
    *reinterpret_cast<GLOBAL u16x4*>(lo + e) = l;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename A>
static Group<A> mkgroup16(const GroupLaunch<A>& L) {
    Group<A> g;
    g.args = L.args;
    g.tstart = L.tstart;
    g.calls = L.calls;
    g.count = L.count;
    g.skip = L.skip;
    g.skip_mask = L.skip_mask;
    return g;
}

template <typename T16, int NT>
static hipError_t sx16_nt(const GroupLaunch<SxArgs>& L, bool vec, hipStream_t st) {
    if (vec)
        hipLaunchKernelGGL((k_sx16<T16, NT, true>), dim3(L.tiles), dim3(256), 0, st, mkgroup16(L));
    else
        hipLaunchKernelGGL((k_sx16<T16, NT, false>), dim3(L.tiles), dim3(256), 0, st, mkgroup16(L));
    return hipGetLastError();
}

template <typename T16, int NT, bool LO>
static hipError_t stq16_nt(const GroupLaunch<StqArgs>& L, bool vec, hipStream_t st) {
    const dim3 block(64 * stq16_grid<LO, NT>::WM * stq16_grid<LO, NT>::WN);
    if (vec)
        hipLaunchKernelGGL((k_stq16<T16, NT, true, LO>), dim3(L.tiles), block, 0, st, mkgroup16(L));
    else
        hipLaunchKernelGGL((k_stq16<T16, NT, false, LO>), dim3(L.tiles), block, 0, st, mkgroup16(L));
    return hipGetLastError();
}

template <typename T16>
static hipError_t sx16_dispatch(int nt, const GroupLaunch<SxArgs>& L, bool vec, hipStream_t st) {
    switch (nt) {
#define RPOD_C(K) case K: return sx16_nt<T16, K>(L, vec, st);
        RPOD_C(1) RPOD_C(2) RPOD_C(3) RPOD_C(4) RPOD_C(5) RPOD_C(6) RPOD_C(7) RPOD_C(8)
#undef RPOD_C
        default: return hipErrorInvalidValue;
    }
}

template <typename T16, bool LO>
static hipError_t stq16_dispatch(int nt, const GroupLaunch<StqArgs>& L, bool vec, hipStream_t st) {
    switch (nt) {
#define RPOD_C(K) case K: return stq16_nt<T16, K, LO>(L, vec, st);
        RPOD_C(1) RPOD_C(2) RPOD_C(3) RPOD_C(4) RPOD_C(5) RPOD_C(6) RPOD_C(7) RPOD_C(8)
#undef RPOD_C
        default: return hipErrorInvalidValue;
    }
}

int stq16_block_cols(bool) { return STQ16_HB; }
int stq16_rows_per_step(bool) { return STQ16_R; }

hipError_t launch_sx16(int tin, int nt, bool vec, const GroupLaunch<SxArgs>& L, hipStream_t st) {
    if (tin == DT_BF16) return sx16_dispatch<__bf16>(nt, L, vec, st);
    if (tin == DT_F16) return sx16_dispatch<_Float16>(nt, L, vec, st);
    return hipErrorInvalidValue;
}

hipError_t launch_stq16(int tin, int nt, bool lo, bool vec, const GroupLaunch<StqArgs>& L, hipStream_t st) {
    if (tin == DT_BF16)
        return lo ? stq16_dispatch<__bf16, true>(nt, L, vec, st) : stq16_dispatch<__bf16, false>(nt, L, vec, st);
    if (tin == DT_F16)
        return lo ? stq16_dispatch<_Float16, true>(nt, L, vec, st) : stq16_dispatch<_Float16, false>(nt, L, vec, st);
    return hipErrorInvalidValue;
}

hipError_t launch_split16(int tin, const GroupLaunch<SplitArgs>& L, hipStream_t st) {
    if (tin == DT_BF16)
        hipLaunchKernelGGL(k_split16<__bf16>, dim3(L.tiles), dim3(256), 0, st, mkgroup16(L));
    else if (tin == DT_F16)
        hipLaunchKernelGGL(k_split16<_Float16>, dim3(L.tiles), dim3(256), 0, st, mkgroup16(L));
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace rpod
