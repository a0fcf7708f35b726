// C ABI of the randomized POD library: validation, workspace layout, the
// recorded launch program of a plan (one matrix or a batch), its hipGraph,
// and the entry points. The program is the launch sequence of one rPOD call
// (Alg. 1 of Sec. 4.2), every launch grouped over the matrices of a class
// (same padded sketch width, rank tiles and storage type).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cmath>
#include <map>
#include <new>
#include <vector>

#include "../../include/rpod.h"
#include "internal.hpp"
#include "warm_model.hpp"

using namespace rpod;

namespace {

thread_local char g_err[512] = "no error";

rpod_status fail(rpod_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

int64_t roundup(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

}  // namespace

rpod_status rpod_internal_fail(rpod_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

namespace {

size_t dt_size(int dt) {
    switch (dt) {
        case DT_F64: return 8;
        case DT_F32: return 4;
        case DT_BF16: case DT_F16: return 2;
        default: return 0;
    }
}

bool is16(int dt) { return dt == DT_BF16 || dt == DT_F16; }
// FP16 storage of Q (hi and lo parts for the passes S^T Q): Q's entries are at most about 1 in
// magnitude (orthonormal columns), so its FP16 parts are taken of 2^14 Q and the slab sums scaled
// back by 2^-14 (both exact): hi stays below 2^15 and the lo part, about 2^-11 of hi, stays a
// normal FP16 number for entries down to about 2^-17 instead of 2^-3. BF16 has FP32's exponent
// range and needs no scale.
double q16_scale(int dt) { return dt == DT_F16 ? 0x1p14 : 1.0; }

// Buffers and sizes of one matrix, derived from its description.
struct Layout {
    int l, lp, nt, rp, ntr;
    int64_t mP, nP;
    int tin, tacc;
    int nsplit;
    int64_t split_rows;
    // split-K over the columns for S X on short, wide matrices (1: none)
    int nsplit_x;
    int64_t split_cols_x;
    // FP64 small SVD: C = Zw^T Q2 by split-K over the n rows (contiguous splits)
    int nsplit_c;
    int64_t split_rows_c;
    int nchunk;
    int gram_cap;
    // fluctuation centring (Sec. 4.1): K blocks of N columns; K = 0: none.
    // The first pass runs nta = lpa / 16 column tiles (lpa = lp + roundup(K, 16)).
    int K, lpa, nta, ncc;
    int64_t N, cchunk;
    // byte offsets into the matrix's workspace region
    size_t o_X, o_Y, o_Q1, o_Qh, o_Ql, o_Zp, o_Yp, o_Zt, o_Zw, o_Zw2, o_Gpart, o_G;
    size_t o_R64[3], o_R32[3], o_UB, o_sig, o_M64, o_M32, o_Ur, o_Phi, o_At, o_pval, o_pidx, o_signs;
    size_t o_Cb, o_Cp, o_Pc;  // centring: E^T X / N, slabs of Msum^T Q1 and their sum
    size_t o_Fp, o_Fro;       // energy: partial sums of ||S||_F^2 and the sum
    int nfro;                 // their count (0 without RPOD_DESC_ENERGY)
    size_t total;
};

rpod_status validate(const rpod_desc* d) {
    if (d == nullptr) return fail(RPOD_EINVAL, "desc is NULL");
    if (d->m < 1 || d->n < 1) return fail(RPOD_EINVAL, "m and n must be >= 1 (m=%lld, n=%lld)",
                                          (long long)d->m, (long long)d->n);
    if (d->ld < d->m) return fail(RPOD_EINVAL, "ld (%lld) must be >= m (%lld)", (long long)d->ld, (long long)d->m);
    if (d->r < 1) return fail(RPOD_EINVAL, "r must be >= 1 (r=%d)", d->r);
    if (d->p < 0) return fail(RPOD_EINVAL, "p must be >= 0 (p=%d)", d->p);
    if (d->q < 0) return fail(RPOD_EINVAL, "q must be >= 0 (q=%d)", d->q);
    if ((d->flags & ~RPOD_DESC_ENERGY) != 0) return fail(RPOD_EINVAL, "unknown flags 0x%x", d->flags);
    if (d->dtype < RPOD_F64 || d->dtype > RPOD_F16) return fail(RPOD_EINVAL, "unknown dtype %d", d->dtype);
    const int64_t l = (int64_t)d->r + d->p;
    const int64_t mn = d->m < d->n ? d->m : d->n;
    if (l > mn) return fail(RPOD_EINVAL, "l = r + p = %lld exceeds min(m, n) = %lld", (long long)l, (long long)mn);
    if (l > 128) return fail(RPOD_EUNSUPPORTED, "l = r + p = %lld exceeds 128", (long long)l);
    if (d->block_cols < 0) return fail(RPOD_EINVAL, "block_cols must be >= 0 (got %lld)", (long long)d->block_cols);
    if (d->block_cols > 0) {
        if (d->flags & RPOD_DESC_ENERGY)
            return fail(RPOD_EUNSUPPORTED, "RPOD_DESC_ENERGY is not available with block_cols");
        if (d->n % d->block_cols != 0)
            return fail(RPOD_EINVAL, "n (%lld) must be a multiple of block_cols (%lld)", (long long)d->n,
                        (long long)d->block_cols);
        const int64_t K = d->n / d->block_cols;
        if (l > d->n - K)  // each block of S' sums to zero: rank(S') <= n - K
            return fail(RPOD_EINVAL, "l = r + p = %lld exceeds n - blocks = %lld, the rank bound of the fluctuations",
                        (long long)l, (long long)(d->n - K));
        if (K > 64 || roundup(l, 16) + roundup(K, 16) > 128)
            return fail(RPOD_EUNSUPPORTED, "%lld blocks with l = %lld: needs at most 64 blocks and "
                        "roundup(l, 16) + roundup(blocks, 16) <= 128", (long long)K, (long long)l);
    }
    return RPOD_OK;
}

// wg_target: workgroups wanted for one S^T Q pass of this matrix (the row
// split count follows from it); gram_cap: most workgroups of a tall Gram.
Layout make_layout(const rpod_desc* d, int64_t wg_target, int gram_cap) {
    Layout L{};
    L.gram_cap = gram_cap;
    L.l = d->r + d->p;
    L.lp = (int)roundup(L.l, 16);
    L.nt = L.lp / 16;
    L.rp = (int)roundup(d->r, 16);
    L.ntr = L.rp / 16;
    L.mP = roundup(d->m, 256);
    L.nP = roundup(d->n, 256);
    L.tin = d->dtype;  // rpod_dtype and the internal codes coincide
    L.tacc = d->dtype == RPOD_F64 ? DT_F64 : DT_F32;
    // split-K over rows for S^T Q. FP64: blocks of 256 columns and
    // contiguous splits of >= 256 rows. FP32: blocks of 256 columns, splits
    // interleaved in units of 64 rows. 16-bit: blocks of 256 columns,
    // splits interleaved in steps of 128 rows.
    const bool s16 = is16(L.tin), f32 = L.tin == DT_F32;
    const int64_t ncb = s16 ? L.nP / stq16_block_cols(false) : f32 ? L.nP / stq_e6_block_cols() : L.nP / 256;
    const int64_t target = (s16 || f32) ? wg_target : std::max<int64_t>(64, wg_target / 4);
    int64_t ns = (target + ncb - 1) / ncb;
    // FP32: up to 128 splits (measured at 262144 x 5000: 64 splits 1.085 ms, 128 splits 1.03 ms
    // per pass, the 2560 tiles filling five rounds of two workgroups per CU; more are slower)
    const int64_t smax = f32 ? 128 : 64;
    if (ns > smax) ns = smax;
    // 16-bit: at least about 1365 rows per split (measured at 8192 x 90225, BF16: at p = 75
    // 6, 7 or 8 splits 2.97-2.99 ms per call, 12 splits 3.07 ms, 15 splits 3.40 ms; at p = 20
    // 6 splits 1.46 ms, 8 splits 1.50 ms; short splits cost more in slab traffic than they gain)
    const int64_t maxs = s16 ? std::max<int64_t>(1, d->m * 3 / 4096) : f32 ? (d->m + 63) / 64 : (d->m + 255) / 256;
    if (ns > maxs) ns = maxs;
    if (f32 && ns >= 8) ns -= ns % 8;  // whole XCD groups of splits
    if (ns < 1) ns = 1;
    L.split_rows = roundup((d->m + ns - 1) / ns, 64);
    L.nsplit = (s16 || f32) ? (int)ns : (int)((d->m + L.split_rows - 1) / L.split_rows);
    {   // at most as many splits as the main product (its slab buffer holds these), >= 256 rows each
        int64_t nsc = std::min<int64_t>(L.nsplit, (d->n + 255) / 256);
        if (nsc < 1) nsc = 1;
        L.split_rows_c = roundup((d->n + nsc - 1) / nsc, 64);
        L.nsplit_c = (int)((d->n + L.split_rows_c - 1) / L.split_rows_c);
    }
    {   // S X runs one workgroup per 256 rows; with fewer than 512 such tiles (a
        // single plan) the columns are split so that about 512 workgroups run,
        // each split at least 1024 columns, the slabs summed afterwards
        // (measured at 8192 x 90225, BF16, p = 75: 3.01 ms per call with 16
        // splits, 3.08 with 12, 3.15 with 63, 3.20 with 8: more splits cost
        // slab traffic, fewer leave CUs idle)
        const int64_t rt = L.mP / 256;
        int64_t nsx = 1;
        if (rt < 512 && wg_target >= 2048) {
            nsx = std::min<int64_t>((512 + rt - 1) / rt, std::max<int64_t>(1, d->n / 1024));
            nsx = std::min<int64_t>(nsx, 128);
        }
        L.split_cols_x = roundup((d->n + nsx - 1) / nsx, 32);
        L.nsplit_x = (int)((d->n + L.split_cols_x - 1) / L.split_cols_x);
    }
    int64_t nc = d->m / 2048;
    L.nchunk = (int)(nc < 1 ? 1 : (nc > 256 ? 256 : nc));
    L.N = d->block_cols;
    L.K = d->block_cols > 0 ? (int)(d->n / d->block_cols) : 0;
    L.lpa = L.lp + (int)roundup(L.K, 16);
    L.nta = L.lpa / 16;
    L.cchunk = roundup((d->m + 1023) / 1024, 32);  // rows per partial sum of Msum^T Q1 (up to 1024)
    L.ncc = L.K > 0 ? (int)((d->m + L.cchunk - 1) / L.cchunk) : 0;

    const size_t sa = dt_size(L.tacc), si = dt_size(L.tin);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t lp2 = (size_t)L.lp * L.lp;
    L.o_X = take((size_t)L.nP * L.lpa * si);  // centring: indicator columns after the first lp
    L.o_Y = take((size_t)L.mP * L.lpa * sa);  // centring: block sums after the first lp
    L.o_Q1 = take((size_t)L.mP * L.lp * sa);
    L.o_Qh = take(s16 ? (size_t)L.mP * L.lp * 2 : 0);
    L.o_Ql = take(s16 ? (size_t)L.mP * L.lp * 2 : 0);
    L.o_Zp = take((size_t)L.nsplit * L.nP * L.lp * (L.tin == DT_F64 ? 8 : 4));  // FP32 slabs off the FP64 path
    L.o_Yp = take(L.nsplit_x > 1 ? (size_t)L.nsplit_x * L.mP * L.lpa * sa : 0);   // slabs of a split S X
    L.o_Zt = take((size_t)L.nP * L.lp * 8);
    L.o_Zw = take((size_t)L.nP * L.lp * 8);
    L.o_Zw2 = take((size_t)L.nP * L.lp * 8);
    L.o_Gpart = take((size_t)gram_partial_count(L.nt) * 8);
    L.o_G = take(lp2 * 8);
    for (int k = 0; k < 3; ++k) {
        L.o_R64[k] = take(lp2 * 8);
        L.o_R32[k] = take(lp2 * 4);
    }
    L.o_UB = take(lp2 * 8);
    L.o_sig = take((size_t)L.lp * 8);
    L.o_M64 = take((size_t)L.lp * L.rp * 8);
    L.o_M32 = take((size_t)L.lp * L.rp * 4);
    L.o_Ur = take((size_t)L.lp * L.rp * 8);
    L.o_Phi = take((size_t)L.mP * L.rp * sa);
    L.o_At = take((size_t)L.nP * L.rp * 8);
    L.o_pval = take((size_t)L.rp * L.nchunk * 8);
    L.o_pidx = take((size_t)L.rp * L.nchunk * 8);
    L.o_signs = take((size_t)L.rp * 8);
    L.o_Cb = take((size_t)L.K * L.lp * 8);
    L.o_Cp = take((size_t)L.ncc * L.K * L.lp * 8);
    L.o_Pc = take((size_t)L.K * L.lp * 8);
    // FP32: the first pass's tiles (mP / 256) write the partial sums; otherwise a pass of 1024 tiles
    L.nfro = (d->flags & RPOD_DESC_ENERGY) ? (L.tin == DT_F32 ? (int)(L.mP / 256) : 1024) : 0;
    L.o_Fp = take((size_t)L.nfro * 8);
    L.o_Fro = take(8);
    L.total = off;
    return L;
}

// ---------------------------------------------------------------------------
// Recorded program
// ---------------------------------------------------------------------------
enum Kind { K_ZERO, K_OMEGA, K_SX, K_SXE6, K_SX16, K_STQ, K_STQE6, K_STQ16, K_REDUCE, K_GRAM, K_CHOL, K_JACOBI, K_LIFT,
            K_SIGNS, K_FIN, K_SPLIT, K_WFWD, K_WZ, K_SXW, K_MRES, K_CPREP, K_CY, K_CCROSS, K_CSUM, K_CZ, K_FROB,
            K_EYE, K_ADEC, K_ARANK };

struct Step {
    Kind kind;
    int tin = 0, tout = 0, nt = 0, lp = 0;  // lp: padded size (small SVD, Cholesky)
    bool vec = true, upper = false, lo = false;
    bool energy = false;  // K_SXE6: also the per-tile sums of squares; K_FROB: only the final sum
    bool tall = false;    // K_SXE6: a product with few columns of S (early loads)
    int pass = -1;  // 0: a pass S X over S, 1: a pass S^T Q over S, 2: the 16-bit refinement pass (timed)
    // conditional steps (warm and adaptive plans, one matrix): the launch does
    // nothing unless status word skip_word of the matrix has a bit of skip_mask
    int skip_word = -1, skip_mask = 0;
    size_t a1 = 0, t1 = 0, a2 = 0, t2 = 0;  // program-blob offsets of the argument / tile tables
    int count = 0, tiles1 = 0, tiles2 = 0;
    double bytes = 0, flops = 0;  // algorithmic work of the launch (passes over S)
};

struct Item {
    rpod_desc d;
    Layout L;
    size_t off;  // workspace offset of the matrix's region
    int idx;     // index in the batch (call table, flags region)
};

struct Builder {
    std::vector<char> blob;
    size_t put(const void* p, size_t bytes) {
        const size_t o = (size_t)roundup((int64_t)blob.size(), 16);
        blob.resize(o + bytes);
        std::memcpy(blob.data() + o, p, bytes);
        return o;
    }
    template <typename A>
    void add(Step& s, const std::vector<A>& args, const std::vector<int>& tiles, bool second = false) {
        std::vector<int> ts(args.size() + 1, 0);
        for (size_t i = 0; i < args.size(); ++i) ts[i + 1] = ts[i] + tiles[i];
        const size_t ao = put(args.data(), sizeof(A) * args.size());
        const size_t to = put(ts.data(), sizeof(int) * ts.size());
        s.count = (int)args.size();
        if (!second) {
            s.a1 = ao; s.t1 = to; s.tiles1 = ts.back();
        } else {
            s.a2 = ao; s.t2 = to; s.tiles2 = ts.back();
        }
    }
};

constexpr int FLAG_INTS = 64;  // status words per matrix (0: status, 1: orthonormalisation-local)

}  // namespace

struct rpod_plan_s {
    std::vector<Item> items;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t st = nullptr;
    size_t o_flags = 0, o_calls = 0, o_prog = 0;
    std::vector<std::vector<Step>> programs;  // one per class
    // graph of the whole program
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // per-pass event timing (measurement only)
    bool timing = false;
    std::vector<hipEvent_t> ev[3];
    std::vector<double> evbytes[3], evflops[3];
    size_t used[3] = {0, 0, 0};
    std::vector<CallDesc> host_calls;
    // warm plans: the model and the warm region (predicted coordinates, network
    // output, the residual product S A^T, its chunk sums, rho and rho_k)
    rpod_warm_s* model = nullptr;
    size_t o_warm = 0, w_Xw = 0, w_c = 0, w_kstar = 0, w_Yres = 0, w_part = 0, w_rho = 0, w_rhom = 0;
    int res_nchunk = 0;
    int64_t ldXw = 0;
    double tol = 0.0;
    int q_fb = 0;
    // adaptive plans: block width, block count, energy threshold, and the
    // adaptive region (||B_i||_F^2 and E_i per block, Frobenius partial sums)
    int adapt_b = 0, adapt_kmax = 0;
    double delta = 0.0;
    size_t o_adapt = 0;

    // Workspace addresses. The recorder also runs without a workspace (to size
    // one), so addresses are formed as integers: no arithmetic on a null pointer.
    template <typename T>
    T* addr(size_t off) const { return reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(ws) + off); }
    template <typename T>
    T* wat(size_t off) const { return addr<T>(o_warm + off); }
    double* adat(size_t k) const { return addr<double>(o_adapt + k * sizeof(double)); }
    int* flags(const Item& it) const { return flag(it, 0); }
    int* flag(const Item& it, int k) const { return addr<int>(o_flags + sizeof(int) * (FLAG_INTS * it.idx + k)); }
    template <typename T>
    T* at(const Item& it, size_t off) const { return addr<T>(it.off + off); }
    CallDesc* calls() const { return addr<CallDesc>(o_calls); }
    template <typename A>
    GroupLaunch<A> gl(const Step& s, bool second) const {
        GroupLaunch<A> g;
        g.args = addr<const A>(o_prog + (second ? s.a2 : s.a1));
        g.tstart = addr<const int>(o_prog + (second ? s.t2 : s.t1));
        g.calls = calls();
        g.count = s.count;
        g.tiles = second ? s.tiles2 : s.tiles1;
        if (s.skip_word >= 0) {  // plans with conditional steps hold one matrix
            g.skip = addr<const int>(o_flags + sizeof(int) * s.skip_word);
            g.skip_mask = s.skip_mask;
        }
        return g;
    }
};

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(RPOD_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

namespace {

// ---------------------------------------------------------------------------
// Recording one class (matrices sharing lp, rp, the storage type and q)
// ---------------------------------------------------------------------------
struct Recorder {
    const rpod_plan_s* P;
    Builder& B;
    std::vector<const Item*> C;
    std::vector<Step>& out;
    const Layout& L0() const { return C[0]->L; }

    template <typename F>
    auto each(F f) -> std::vector<decltype(f(*C[0]))> {
        std::vector<decltype(f(*C[0]))> v;
        for (const Item* it : C) v.push_back(f(*it));
        return v;
    }
    template <typename F>
    std::vector<int> tiles(F f) {
        std::vector<int> v;
        for (const Item* it : C) v.push_back(f(*it));
        return v;
    }

    // steps recorded since `first` run only if status word `word` has a bit of `mask`
    void only_if(size_t first, int word, int mask) {
        for (size_t k = first; k < out.size(); ++k) {
            out[k].skip_word = word;
            out[k].skip_mask = mask;
            out[k].pass = -1;  // not timed: skipped launches would distort the averages
        }
    }
    void zero() {
        Step s{K_ZERO};
        B.add(s, each([&](const Item& it) { return ZeroArgs{P->flags(it), FLAG_INTS}; }),
              tiles([](const Item&) { return 1; }));
        out.push_back(s);
    }
    void omega() {
        Step s{K_OMEGA};
        s.tout = L0().tin;
        B.add(s, each([&](const Item& it) {
                  OmegaArgs a{};
                  a.out = P->at<char>(it, it.L.o_X);
                  a.n = it.d.n; a.rows_pad = it.L.nP; a.ldo = it.L.nP;
                  a.seed = 0; a.l = it.L.l; a.lpad = it.L.lp; a.call = it.idx;
                  return a;
              }),
              tiles([](const Item& it) { return (int)((it.L.nP + 255) / 256) * ((it.L.lp + 1) / 2); }));
        out.push_back(s);
    }
    // generic tall x small product (internal operands)
    void sx(int tin, int tout, int nt, bool upper, std::vector<SxArgs> args) {
        Step s{K_SX};
        s.tin = tin; s.tout = tout; s.nt = nt; s.upper = upper; s.vec = true;
        std::vector<int> t;
        for (const SxArgs& a : args) t.push_back((int)((std::max(a.mstore, a.m) + 255) / 256));
        B.add(s, args, t);
        out.push_back(s);
    }
    // tall FP32 x small product on the BF16 matrix cores with split operands
    // (FP32-accurate), used when the small side's rows lp are a multiple of 32
    // (the kernel reads X rows up to a multiple of 32); FP64 or other lp: sx()
    void sx_tall(int tacc, int nt, bool upper, std::vector<SxArgs> args) {
        if (tacc != DT_F32 || L0().lp % 32 != 0) return sx(tacc, tacc, nt, upper, std::move(args));
        Step s{K_SXE6};
        s.tin = DT_F32; s.tout = DT_F32; s.nt = nt; s.vec = true; s.tall = true;
        std::vector<int> t;
        for (const SxArgs& a : args) t.push_back((int)((std::max(a.mstore, a.m) + 255) / 256));
        B.add(s, args, t);
        out.push_back(s);
    }
    // pass over S: Y = S X (first: with the centring indicator columns, if any)
    void pass_sx(bool first = false) {
        const bool s16 = is16(L0().tin), f32 = L0().tin == DT_F32;
        Step s{s16 ? K_SX16 : f32 ? K_SXE6 : K_SX};
        s.tin = L0().tin; s.tout = L0().tacc; s.nt = first ? L0().nta : L0().nt; s.pass = 0;
        s.vec = true;
        for (const Item* it : C) {
            s.vec = s.vec && (it->d.ld % (s16 ? 8 : 4) == 0);
            const double sz = (double)dt_size(it->L.tin);
            s.bytes += (double)it->d.m * it->d.n * sz + (double)it->d.n * it->L.l * sz + (double)it->d.m * it->L.l * 4.0;
            s.flops += 2.0 * it->d.m * it->d.n * it->L.l;
        }
        s.energy = first && f32 && L0().nfro > 0;  // FP32 energy report: sums of squares from this pass
        // one record per matrix, or per column split (short, wide matrices) into
        // slabs that a reduction then sums into Y; the energy pass is not split
        std::vector<SxArgs> args;
        std::vector<int> t;
        std::vector<ReduceArgs> red;
        std::vector<int> rt;
        const int w = 16 * s.nt;  // columns of Y written
        for (const Item* itp : C) {
            const Item& it = *itp;
            const int ns = s.energy ? 1 : it.L.nsplit_x;
            const size_t sa = dt_size(it.L.tacc);
            for (int k = 0; k < ns; ++k) {
                const int64_t c0 = (int64_t)k * it.L.split_cols_x;
                const int64_t nc = ns == 1 ? it.d.n : std::min<int64_t>(it.L.split_cols_x, it.d.n - c0);
                const size_t y = ns == 1 ? it.L.o_Y : it.L.o_Yp + (size_t)k * it.L.mP * w * sa;
                SxArgs a{nullptr, it.d.ld, it.d.m, nc, P->at<char>(it, it.L.o_X + (size_t)c0 * dt_size(it.L.tin)),
                         it.L.nP, P->at<char>(it, y), it.L.mP, it.L.mP, nullptr, 0, it.idx};
                a.col0 = c0;
                if (s.energy) a.fpart = P->at<double>(it, it.L.o_Fp);
                args.push_back(a);
                t.push_back((int)(it.L.mP / 256));
            }
            if (ns > 1) {
                const int o32 = it.L.tacc != DT_F64 ? 1 : 0;
                red.push_back(ReduceArgs{P->at<char>(it, it.L.o_Yp), it.L.mP * w, P->at<char>(it, it.L.o_Y), ns, o32, o32});
                rt.push_back((int)((it.L.mP * w + 255) / 256));
            }
        }
        B.add(s, args, t);
        out.push_back(s);
        if (!red.empty()) {
            Step r{K_REDUCE};
            B.add(r, red, rt);
            out.push_back(r);
        }
    }
    // pass over S: slabs of S^T Q1 (lo: Q1 carried as hi + lo on 16-bit paths), then their sum
    // into dst (Zt; Zw directly when Q1 needs no further factor)
    void pass_stq(bool lo, size_t Layout::*dst = &Layout::o_Zt) {
        const bool s16 = is16(L0().tin), f32 = L0().tin == DT_F32;
        Step s{s16 ? K_STQ16 : f32 ? K_STQE6 : K_STQ};
        s.tin = L0().tin; s.nt = L0().nt; s.lo = s16 && lo; s.pass = s.lo ? 2 : 1;
        s.vec = true;
        for (const Item* it : C) {
            s.vec = s.vec && (it->d.ld % (s16 ? 8 : 4) == 0);
            const double sz = (double)dt_size(it->L.tin);
            s.bytes += (double)it->d.m * it->d.n * sz + (double)it->d.n * it->L.l * sz + (double)it->d.m * it->L.l * 4.0;
            s.flops += 2.0 * it->d.m * it->d.n * it->L.l;
        }
        std::vector<StqArgs> args = each([&](const Item& it) {
            StqArgs a{};
            a.S = nullptr; a.ldS = it.d.ld; a.m = it.d.m; a.n = it.d.n;
            a.Q = P->at<char>(it, s16 ? it.L.o_Qh : it.L.o_Q1);  // FP32: split by the pass as it is staged
            a.Ql = s16 ? (const void*)P->at<char>(it, it.L.o_Ql) : nullptr;
            a.ldQ = it.L.mP; a.Zp = P->at<double>(it, it.L.o_Zp); a.nP = it.L.nP;
            a.split_rows = it.L.split_rows; a.nsplit = it.L.nsplit;
            a.ncb = s16 ? (int)(it.L.nP / stq16_block_cols(s.lo))
                        : f32 ? (int)(it.L.nP / stq_e6_block_cols()) : (int)(it.L.nP / 256);
            a.call = it.idx;
            return a;
        });
        std::vector<int> t;
        for (const StqArgs& a : args) t.push_back(a.ncb * a.nsplit);
        B.add(s, args, t);
        out.push_back(s);
        Step r{K_REDUCE};
        B.add(r, each([&](const Item& it) {
                  // the FP32 and 16-bit passes accumulate in FP32 and write FP32 slabs
                  ReduceArgs a{P->at<double>(it, it.L.o_Zp), it.L.nP * it.L.lp, P->at<double>(it, it.L.*dst),
                               it.L.nsplit, it.L.tin != DT_F64 ? 1 : 0};
                  a.scale = 1.0 / q16_scale(it.L.tin);
                  return a;
              }),
              tiles([](const Item& it) { return (int)((it.L.nP * it.L.lp + 255) / 256); }));
        out.push_back(r);
    }
    // ||S||_F^2 for the energy of the modes (plans with RPOD_DESC_ENERGY; a no-op otherwise)
    // after_first: FP32 plans add up the partial sums their first pass wrote (called after it);
    // the other types read S in a pass of their own (called before the sketch)
    void frob(bool after_first) {
        if (L0().nfro == 0 || after_first != (L0().tin == DT_F32)) return;
        Step s{K_FROB};
        s.tin = L0().tin;
        s.energy = after_first;
        s.vec = true;
        // 16-byte loads where rpod_compute requires S to be 16-byte aligned (ld a multiple of 4, or 8 for 16-bit)
        for (const Item* it : C) s.vec = s.vec && (it->d.ld % (is16(it->L.tin) ? 8 : 4) == 0);
        auto args = each([&](const Item& it) {
            return FrobArgs{nullptr, it.d.ld, it.d.m, it.d.n, P->at<double>(it, it.L.o_Fp), P->at<double>(it, it.L.o_Fro),
                            it.L.nfro, it.idx};
        });
        B.add(s, args, tiles([](const Item& it) { return it.L.nfro; }));
        B.add(s, args, tiles([](const Item&) { return 1; }), true);
        out.push_back(s);
    }
    // Fluctuation centring (Sec. 4.1) of the products with S; no-ops without blocks.
    bool centred() const { return L0().K > 0; }
    // C = E^T X / N for the operand of the next S X pass (ind: also write E)
    void center_prep(bool ind) {
        if (!centred()) return;
        Step s{K_CPREP};
        s.tin = L0().tin;
        B.add(s, each([&](const Item& it) {
                  return CprepArgs{P->at<char>(it, it.L.o_X), it.L.nP, it.d.n, it.L.N, P->at<double>(it, it.L.o_Cb),
                                   it.L.lp, it.L.K, ind ? 1 : 0};
              }),
              tiles([](const Item& it) { return it.L.K * (it.L.lp / 4); }));
        out.push_back(s);
    }
    // Y -= Msum C after an S X pass
    void center_y() {
        if (!centred()) return;
        Step s{K_CY};
        s.tin = L0().tacc;
        B.add(s, each([&](const Item& it) {
                  return CenterYArgs{P->at<char>(it, it.L.o_Y), it.L.mP, it.d.m, P->at<double>(it, it.L.o_Cb),
                                     it.L.lp, it.L.K};
              }),
              tiles([](const Item& it) { return (int)((it.d.m + 255) / 256); }));
        out.push_back(s);
    }
    // Z -= E (Msum^T Q1) / N after an S^T Q pass (Z: the pass's sum, Zt or Zw)
    void center_z(size_t Layout::*dst = &Layout::o_Zt) {
        if (!centred()) return;
        Step s{K_CCROSS};
        s.tin = L0().tacc;
        B.add(s, each([&](const Item& it) {
                  const size_t so = dt_size(it.L.tacc);
                  return CrossArgs{P->at<char>(it, it.L.o_Y + (size_t)it.L.lp * it.L.mP * so),
                                   P->at<char>(it, it.L.o_Q1), it.L.mP, it.d.m, it.L.cchunk,
                                   P->at<double>(it, it.L.o_Cp), it.L.lp, it.L.K, it.L.ncc};
              }),
              tiles([](const Item& it) { return it.L.ncc; }));
        out.push_back(s);
        Step r{K_CSUM};
        B.add(r, each([&](const Item& it) {
                  return CrossSumArgs{P->at<double>(it, it.L.o_Cp), P->at<double>(it, it.L.o_Pc), it.L.K * it.L.lp,
                                      it.L.ncc};
              }),
              tiles([](const Item& it) { return it.L.K * it.L.lp; }));
        out.push_back(r);
        Step z{K_CZ};
        B.add(z, each([&](const Item& it) {
                  return CenterZArgs{P->at<double>(it, it.L.*dst), it.L.nP, it.d.n, it.L.N,
                                     P->at<double>(it, it.L.o_Pc), it.L.lp, it.L.K};
              }),
              tiles([](const Item& it) { return (int)((it.L.nP * it.L.lp + 255) / 256); }));
        out.push_back(z);
    }
    void gram(int dt, std::vector<GramArgs> args) {
        Step s{K_GRAM};
        s.tin = dt; s.nt = L0().nt;
        std::vector<int> t1, t2;
        for (const GramArgs& a : args) {
            t1.push_back(gram_tiles(s.nt, a.nwg));
            t2.push_back(gram_reduce_tiles(s.nt));
        }
        B.add(s, args, t1);
        B.add(s, args, t2, true);
        out.push_back(s);
    }
    void chol(std::vector<CholArgs> args) {
        Step s{K_CHOL};
        s.lp = L0().lp;
        B.add(s, args, std::vector<int>(args.size(), 1));
        out.push_back(s);
    }
    // CholeskyQR2 of the tall In (ld, M rows, type dt) into Out; the final
    // factor R^-1 is left in R[kfin] so that Q = Out R^-1. Shifted CholeskyQR3
    // (Fukaya et al., SISC 2020) after a shifted first factorisation.
    void orth_tall(int kfin) {
        const int dt = L0().tacc;
        auto In = [&](const Item& it) { return (void*)P->at<char>(it, it.L.o_Y); };
        auto Out = [&](const Item& it) { return (void*)P->at<char>(it, it.L.o_Q1); };
        auto Rx = [&](const Item& it, int k) {
            return dt == DT_F64 ? (const void*)P->at<char>(it, it.L.o_R64[k]) : (const void*)P->at<char>(it, it.L.o_R32[k]);
        };
        auto gargs = [&](auto buf, bool cond) {
            return each([&](const Item& it) {
                return GramArgs{buf(it), it.L.mP, it.d.m, P->at<double>(it, it.L.o_Gpart), P->at<double>(it, it.L.o_G),
                                cond ? P->flag(it, 1) : nullptr, cond ? 1 : 0, gram_nwg(it.d.m, it.L.gram_cap, it.L.nt)};
            });
        };
        auto cargs = [&](int k, int mode) {
            return each([&](const Item& it) {
                return CholArgs{P->at<double>(it, it.L.o_G), it.d.m, P->at<double>(it, it.L.o_R64[k]),
                                P->at<float>(it, it.L.o_R32[k]), P->flags(it), P->flag(it, 1), it.L.l, it.L.lp, mode};
            });
        };
        auto apply = [&](auto src, auto dst, int k, bool cond) {
            return each([&](const Item& it) {
                return SxArgs{src(it), it.L.mP, it.d.m, it.L.lp, Rx(it, k), it.L.lp, dst(it), it.L.mP, it.L.mP,
                              cond ? P->flag(it, 1) : nullptr, cond ? 1 : 0, -1};
            });
        };
        gram(dt, gargs(In, false));
        chol(cargs(0, 0));
        sx_tall(dt, L0().nt, true, apply(In, Out, 0, false));
        gram(dt, gargs(Out, false));
        chol(cargs(kfin, 1));
        sx_tall(dt, L0().nt, true, apply(Out, Out, kfin, true));  // shifted retry, in place (no-op otherwise)
        gram(dt, gargs(Out, true));
        chol(cargs(kfin, 2));
        split_q();
    }
    // One CholeskyQR of the tall Y into Q1 = Y R^-1 for an iterate of which only
    // the span matters (the product S^T Q1 of a subspace iteration that is not
    // the last: the n-side basis and the next CholeskyQR2 follow), and a second
    // factorisation only after a shifted first one (CholeskyQR3 of Fukaya et
    // al.); no factor is left for the consumer: S^T Q1 itself is the iterate.
    // Q1's rounding in its storage type perturbs its span the same way whether
    // or not a second pass then orthonormalises it.
    void orth_tall_once() {
        const int dt = L0().tacc;
        auto In = [&](const Item& it) { return (void*)P->at<char>(it, it.L.o_Y); };
        auto Out = [&](const Item& it) { return (void*)P->at<char>(it, it.L.o_Q1); };
        auto Rx = [&](const Item& it, int k) {
            return dt == DT_F64 ? (const void*)P->at<char>(it, it.L.o_R64[k]) : (const void*)P->at<char>(it, it.L.o_R32[k]);
        };
        auto gargs = [&](auto buf, bool cond) {
            return each([&](const Item& it) {
                return GramArgs{buf(it), it.L.mP, it.d.m, P->at<double>(it, it.L.o_Gpart), P->at<double>(it, it.L.o_G),
                                cond ? P->flag(it, 1) : nullptr, cond ? 1 : 0, gram_nwg(it.d.m, it.L.gram_cap, it.L.nt)};
            });
        };
        auto cargs = [&](int k, int mode) {
            return each([&](const Item& it) {
                return CholArgs{P->at<double>(it, it.L.o_G), it.d.m, P->at<double>(it, it.L.o_R64[k]),
                                P->at<float>(it, it.L.o_R32[k]), P->flags(it), P->flag(it, 1), it.L.l, it.L.lp, mode};
            });
        };
        auto apply = [&](auto src, auto dst, int k, bool cond) {
            return each([&](const Item& it) {
                return SxArgs{src(it), it.L.mP, it.d.m, it.L.lp, Rx(it, k), it.L.lp, dst(it), it.L.mP, it.L.mP,
                              cond ? P->flag(it, 1) : nullptr, cond ? 1 : 0, -1};
            });
        };
        gram(dt, gargs(In, false));
        chol(cargs(0, 0));
        sx_tall(dt, L0().nt, true, apply(In, Out, 0, false));
        gram(dt, gargs(Out, true));                              // after a shift only
        chol(cargs(2, 2));
        sx_tall(dt, L0().nt, true, apply(Out, Out, 2, true));    // in place, after a shift only
        split_q();
    }
    // 16-bit storage: Q1 (FP32) as hi + lo BF16/FP16 parts for the passes S^T Q
    void split_q() {
        if (!is16(L0().tin)) return;
        Step s{K_SPLIT};
        s.tin = L0().tin;
        B.add(s, each([&](const Item& it) {
                  SplitArgs a{P->at<float>(it, it.L.o_Q1), it.L.mP * it.L.lp,
                              P->at<unsigned short>(it, it.L.o_Qh), P->at<unsigned short>(it, it.L.o_Ql)};
                  a.scale = (float)q16_scale(it.L.tin);
                  return a;
              }),
              tiles([](const Item& it) { return (int)((it.L.mP * it.L.lp / 4 + 255) / 256); }));
        out.push_back(s);
    }
    // Adaptive plans: explicit CholeskyQR2 of Q1[:, :lp] in place. The leading
    // columns hold the orthonormal basis so far and the trailing block the
    // newest product, so the Cholesky factor of the whole Gram also projects
    // the block off the basis (block Gram-Schmidt), and the second pass
    // repeats the projection. Shifted CholeskyQR3 after a breakdown as in
    // orth_tall; the last factor is applied, not left pending.
    void orth_joint() {
        const int dt = L0().tacc;
        auto Q = [&](const Item& it) { return (void*)P->at<char>(it, it.L.o_Q1); };
        auto Rx = [&](const Item& it, int k) {
            return dt == DT_F64 ? (const void*)P->at<char>(it, it.L.o_R64[k]) : (const void*)P->at<char>(it, it.L.o_R32[k]);
        };
        auto gargs = [&](bool cond) {
            return each([&](const Item& it) {
                return GramArgs{Q(it), it.L.mP, it.d.m, P->at<double>(it, it.L.o_Gpart), P->at<double>(it, it.L.o_G),
                                cond ? P->flag(it, 1) : nullptr, cond ? 1 : 0, gram_nwg(it.d.m, it.L.gram_cap, it.L.nt)};
            });
        };
        auto cargs = [&](int k, int mode) {
            return each([&](const Item& it) {
                return CholArgs{P->at<double>(it, it.L.o_G), it.d.m, P->at<double>(it, it.L.o_R64[k]),
                                P->at<float>(it, it.L.o_R32[k]), P->flags(it), P->flag(it, 1), it.L.l, it.L.lp, mode};
            });
        };
        auto apply = [&](int k, bool cond) {
            return each([&](const Item& it) {
                return SxArgs{Q(it), it.L.mP, it.d.m, it.L.lp, Rx(it, k), it.L.lp, Q(it), it.L.mP, it.L.mP,
                              cond ? P->flag(it, 1) : nullptr, cond ? 1 : 0, -1};
            });
        };
        gram(dt, gargs(false));
        chol(cargs(0, 0));
        sx_tall(dt, L0().nt, true, apply(0, false));
        gram(dt, gargs(false));
        chol(cargs(1, 1));
        sx_tall(dt, L0().nt, true, apply(1, true));   // shifted retry only
        gram(dt, gargs(true));
        chol(cargs(1, 2));
        sx_tall(dt, L0().nt, true, apply(1, false));  // the last factor
    }
    // *dst = ||Zt[:, :l]||_F^2 (FP64, n rows): adaptive plans, ||B_i||_F^2 of a block
    void frob_z(double* part, double* dst) {
        Step s{K_FROB};
        s.tin = DT_F64;
        s.vec = true;
        auto args = each([&](const Item& it) {
            return FrobArgs{P->at<double>(it, it.L.o_Zt), it.L.nP, it.d.n, it.L.l, part, dst, 64, -1};
        });
        B.add(s, args, tiles([](const Item&) { return 64; }));
        B.add(s, args, tiles([](const Item&) { return 1; }), true);
        out.push_back(s);
    }
    void adapt_decide(int i) {
        Step s{K_ADEC};
        B.add(s, each([&](const Item& it) {
                  return AdaptDecideArgs{P->at<double>(it, it.L.o_Fro), P->adat(0), P->adat(ADAPT_MAX_BLOCKS),
                                         P->flags(it), P->delta, i, P->adapt_kmax, P->adapt_b};
              }),
              tiles([](const Item&) { return 1; }));
        out.push_back(s);
    }
    void eye1() {  // R64[1] = I: the basis is explicit, step 7 lifts with Q1 itself
        Step s{K_EYE};
        B.add(s, each([&](const Item& it) { return EyeArgs{P->at<double>(it, it.L.o_R64[1]), it.L.lp}; }),
              tiles([](const Item& it) { return (it.L.lp * it.L.lp + 255) / 256; }));
        out.push_back(s);
    }
    void adapt_rank() {
        Step s{K_ARANK};
        B.add(s, each([&](const Item& it) {
                  return AdaptRankArgs{P->at<double>(it, it.L.o_sig), P->at<double>(it, it.L.o_Fro), P->flags(it),
                                       P->delta, it.L.l};
              }),
              tiles([](const Item&) { return 1; }));
        out.push_back(s);
    }
    // Zw = Zt R^-1 (R from the last tall orthonormalisation): Zw = S^T Q
    void small_from_slabs() {
        sx(DT_F64, DT_F64, L0().nt, true, each([&](const Item& it) {
               return SxArgs{P->at<char>(it, it.L.o_Zt), it.L.nP, it.d.n, it.L.lp, P->at<char>(it, it.L.o_R64[1]),
                             it.L.lp, P->at<char>(it, it.L.o_Zw), it.L.nP, it.L.nP, nullptr, 0, -1};
           }));
    }
    // Basis X of the n x l iterate Zw for the next product with S: one
    // CholeskyQR, X = Zw R^-1 (only its span matters; the CholeskyQR2 of the
    // next S X restores orthonormality); a second step after a shift.
    void basis_small() {
        const int tin = L0().tin;
        auto gargs = [&](bool second, bool cond) {
            return each([&](const Item& it) {
                return GramArgs{P->at<char>(it, second ? it.L.o_Zw2 : it.L.o_Zw), it.L.nP, it.d.n,
                                P->at<double>(it, it.L.o_Gpart), P->at<double>(it, it.L.o_G),
                                cond ? P->flag(it, 1) : nullptr, cond ? 1 : 0, gram_nwg(it.d.n, it.L.gram_cap, it.L.nt)};
            });
        };
        auto app = [&](size_t Layout::*src, size_t Layout::*dst, int k, bool cond) {
            return each([&](const Item& it) {
                return SxArgs{P->at<char>(it, it.L.*src), it.L.nP, it.d.n, it.L.lp, P->at<char>(it, it.L.o_R64[k]),
                              it.L.lp, P->at<char>(it, it.L.*dst), it.L.nP, it.L.nP, cond ? P->flag(it, 1) : nullptr,
                              cond ? 1 : 0, -1};
            });
        };
        auto cargs = [&](int k, int mode) {
            return each([&](const Item& it) {
                return CholArgs{P->at<double>(it, it.L.o_G), it.d.n, P->at<double>(it, it.L.o_R64[k]),
                                P->at<float>(it, it.L.o_R32[k]), P->flags(it), P->flag(it, 1), it.L.l, it.L.lp, mode};
            });
        };
        gram(DT_F64, gargs(false, false));
        chol(cargs(0, 0));
        sx(DT_F64, tin, L0().nt, true, app(&Layout::o_Zw, &Layout::o_X, 0, false));
        sx(DT_F64, DT_F64, L0().nt, true, app(&Layout::o_Zw, &Layout::o_Zw2, 0, true));
        gram(DT_F64, gargs(true, true));
        chol(cargs(2, 2));
        sx(DT_F64, tin, L0().nt, true, app(&Layout::o_Zw2, &Layout::o_X, 2, true));
    }
    // Orthonormal Q2 of the n x l iterate Zw = T^T by CholeskyQR2 (shifted
    // CholeskyQR3 after a breakdown), written explicitly into Zw2; factors in
    // R64[0] and R64[2] (R64[1] still holds the tall orthonormalisation's).
    void orth_small_explicit() {
        auto gargs = [&](size_t Layout::*src, bool cond) {
            return each([&](const Item& it) {
                return GramArgs{P->at<char>(it, it.L.*src), it.L.nP, it.d.n, P->at<double>(it, it.L.o_Gpart),
                                P->at<double>(it, it.L.o_G), cond ? P->flag(it, 1) : nullptr, cond ? 1 : 0,
                                gram_nwg(it.d.n, it.L.gram_cap, it.L.nt)};
            });
        };
        auto app = [&](size_t Layout::*src, int k, bool cond) {
            return each([&](const Item& it) {
                return SxArgs{P->at<char>(it, it.L.*src), it.L.nP, it.d.n, it.L.lp, P->at<char>(it, it.L.o_R64[k]),
                              it.L.lp, P->at<char>(it, it.L.o_Zw2), it.L.nP, it.L.nP,
                              cond ? P->flag(it, 1) : nullptr, cond ? 1 : 0, -1};
            });
        };
        auto cargs = [&](int k, int mode) {
            return each([&](const Item& it) {
                return CholArgs{P->at<double>(it, it.L.o_G), it.d.n, P->at<double>(it, it.L.o_R64[k]),
                                P->at<float>(it, it.L.o_R32[k]), P->flags(it), P->flag(it, 1), it.L.l, it.L.lp, mode};
            });
        };
        gram(DT_F64, gargs(&Layout::o_Zw, false));
        chol(cargs(0, 0));
        sx(DT_F64, DT_F64, L0().nt, true, app(&Layout::o_Zw, 0, false));
        gram(DT_F64, gargs(&Layout::o_Zw2, false));
        chol(cargs(2, 1));
        sx(DT_F64, DT_F64, L0().nt, true, app(&Layout::o_Zw2, 2, true));  // shifted retry, in place
        gram(DT_F64, gargs(&Layout::o_Zw2, true));
        chol(cargs(2, 2));
        sx(DT_F64, DT_F64, L0().nt, true, app(&Layout::o_Zw2, 2, false));  // Q2, in place
    }
    void finish() {
        const Layout& L = L0();
        Step j{K_JACOBI};
        j.lp = L.lp;
        // rotation threshold: FP64 rounding level on the FP64 path; elsewhere below
        // the FP32 storage error of Q (6e-8), which bounds the result anyway (1e-8
        // ends the iteration one sweep earlier than 1e-10 on the Fourier fields)
        const double jtol = L.tacc == DT_F64 ? (double)L.lp * 0x1.0p-53 : 1e-8;
        if (L.tacc == DT_F64) {
            // step 6 on the FP64 path, without squaring the condition number: T^T = Zw = Q2 R
            // (CholeskyQR2 on the n side), C = Zw^T Q2 = R^T, and one-sided Jacobi on the
            // columns of C gives the left singular vectors of T with errors of order
            // u sigma_1 / sigma_k (the Gram route below has u (sigma_1 / sigma_k)^2)
            orth_small_explicit();
            Step k{K_STQ};
            k.tin = DT_F64; k.nt = L.nt; k.vec = true;
            auto kargs = each([&](const Item& it) {
                StqArgs a{};
                a.S = P->at<double>(it, it.L.o_Zw); a.ldS = it.L.nP; a.m = it.d.n; a.n = it.L.lp;
                a.Q = P->at<double>(it, it.L.o_Zw2); a.Ql = nullptr; a.ldQ = it.L.nP;
                a.Zp = P->at<double>(it, it.L.o_Zp); a.nP = WARM_PROJ_COLS;
                a.split_rows = it.L.split_rows_c; a.nsplit = it.L.nsplit_c; a.ncb = 1; a.call = -1;
                return a;
            });
            B.add(k, kargs, tiles([](const Item& it) { return it.L.nsplit_c; }));
            out.push_back(k);
            Step rd{K_REDUCE};
            B.add(rd, each([&](const Item& it) {
                      return ReduceArgs{P->at<double>(it, it.L.o_Zp), (int64_t)WARM_PROJ_COLS * it.L.lp,
                                        P->at<double>(it, it.L.o_Zt), it.L.nsplit_c, 0};
                  }),
                  tiles([](const Item& it) { return (WARM_PROJ_COLS * it.L.lp + 255) / 256; }));
            out.push_back(rd);
            B.add(j, each([&](const Item& it) {
                      return JacobiArgs{nullptr, P->at<double>(it, it.L.o_UB), P->at<double>(it, it.L.o_sig),
                                        P->flags(it), jtol, it.L.l, it.L.lp, P->at<double>(it, it.L.o_Zt),
                                        (int64_t)WARM_PROJ_COLS};
                  }),
                  tiles([](const Item&) { return 1; }));
        } else {
            // step 6: SVD of T through the eigenvectors of T T^T
            gram(DT_F64, each([&](const Item& it) {
                     return GramArgs{P->at<char>(it, it.L.o_Zw), it.L.nP, it.d.n, P->at<double>(it, it.L.o_Gpart),
                                     P->at<double>(it, it.L.o_G), nullptr, 0, gram_nwg(it.d.n, it.L.gram_cap, it.L.nt)};
                 }));
            B.add(j, each([&](const Item& it) {
                      return JacobiArgs{P->at<double>(it, it.L.o_G), P->at<double>(it, it.L.o_UB),
                                        P->at<double>(it, it.L.o_sig), P->flags(it), jtol, it.L.l, it.L.lp,
                                        nullptr, 0};
                  }),
                  tiles([](const Item&) { return 1; }));
        }
        out.push_back(j);
        // step 7: Phi = Q U_hat[:, :r] = Q1 (R^-1 U_hat[:, :r]); A = U_hat_r^T T
        Step lf{K_LIFT};
        B.add(lf, each([&](const Item& it) {
                  return LiftArgs{P->at<double>(it, it.L.o_R64[1]), P->at<double>(it, it.L.o_UB),
                                  P->at<double>(it, it.L.o_M64), P->at<float>(it, it.L.o_M32),
                                  P->at<double>(it, it.L.o_Ur), it.L.lp, it.d.r, it.L.rp};
              }),
              tiles([](const Item& it) { return (it.L.lp * it.L.rp + 255) / 256; }));
        out.push_back(lf);
        sx_tall(L.tacc, L.ntr, false, each([&](const Item& it) {
               const void* Mx = it.L.tacc == DT_F64 ? (const void*)P->at<char>(it, it.L.o_M64)
                                                    : (const void*)P->at<char>(it, it.L.o_M32);
               return SxArgs{P->at<char>(it, it.L.o_Q1), it.L.mP, it.d.m, it.L.lp, Mx, it.L.lp,
                             P->at<char>(it, it.L.o_Phi), it.L.mP, it.L.mP, nullptr, 0, -1};
           }));
        sx(DT_F64, DT_F64, L.ntr, false, each([&](const Item& it) {
               return SxArgs{P->at<char>(it, it.L.o_Zw), it.L.nP, it.d.n, it.L.lp, P->at<char>(it, it.L.o_Ur), it.L.lp,
                             P->at<char>(it, it.L.o_At), it.L.nP, it.L.nP, nullptr, 0, -1};
           }));
        // sign convention and outputs
        Step sg{K_SIGNS};
        sg.tin = L.tacc;
        B.add(sg, each([&](const Item& it) {
                  return ColmaxArgs{P->at<char>(it, it.L.o_Phi), it.L.mP, it.d.m,
                                    (it.d.m + it.L.nchunk - 1) / it.L.nchunk, P->at<double>(it, it.L.o_pval),
                                    P->at<int64_t>(it, it.L.o_pidx), it.d.r, it.L.nchunk};
              }),
              tiles([](const Item& it) { return it.L.nchunk * it.d.r; }));
        B.add(sg, each([&](const Item& it) {
                  return SignArgs{P->at<double>(it, it.L.o_pval), P->at<int64_t>(it, it.L.o_pidx),
                                  P->at<double>(it, it.L.o_signs), it.d.r, it.L.nchunk};
              }),
              tiles([](const Item& it) { return it.d.r; }), true);  // one wave per column
        out.push_back(sg);
        Step fn{K_FIN};
        fn.tin = L.tacc;
        auto fargs = each([&](const Item& it) {
            return FinArgs{P->at<char>(it, it.L.o_Phi), it.L.mP, it.d.m, P->at<double>(it, it.L.o_At), it.L.nP,
                           it.d.n, P->at<double>(it, it.L.o_signs), P->at<double>(it, it.L.o_sig), it.d.r, it.idx};
        });
        B.add(fn, fargs, tiles([](const Item& it) { return fin_phi_tiles(it.d.m, it.d.r, it.L.tacc); }));
        B.add(fn, fargs, tiles([](const Item& it) { return fin_a_tiles(it.d.n, it.d.r); }), true);
        out.push_back(fn);
    }
    // Warm-started program (single matrix): Y = [W, S Omega_p], then as
    // record(), then the residual of the returned modes.
    void record_warm() {
        const Item& it = *C[0];
        const Layout& L = it.L;
        const rpod_warm_s* M = P->model;
        const bool s16 = is16(L.tin);
        const int p = it.d.p, r = it.d.r;
        const int lpad = (int)roundup(p, 16);
        zero();
        Step f{K_WFWD};
        B.add(f, std::vector<WarmFwdArgs>{{M->at<float>(M->L.params), P->wat<double>(P->w_c), P->wat<int>(P->w_kstar),
                                           it.idx}},
              std::vector<int>{1});
        out.push_back(f);
        Step z{K_WZ};
        B.add(z, std::vector<WarmZArgs>{{M->at<double>(M->L.gram), P->wat<double>(P->w_c), P->wat<int>(P->w_kstar),
                                         P->wat<float>(P->w_Xw), P->ldXw, r, M->Kr, L.lp, 2}},
              std::vector<int>{L.lp * (int)((P->ldXw + 63) / 64)});
        out.push_back(z);
        Step o{K_OMEGA};
        o.tout = L.tin;
        OmegaArgs oa{};
        oa.out = P->at<char>(it, L.o_X);
        oa.n = it.d.n; oa.rows_pad = L.nP; oa.ldo = L.nP; oa.seed = 0; oa.l = p; oa.lpad = lpad; oa.call = it.idx;
        B.add(o, std::vector<OmegaArgs>{oa}, std::vector<int>{(int)((L.nP + 255) / 256) * (lpad / 2)});
        out.push_back(o);
        // pass over S: the Gaussian columns, stored after the r predicted ones
        Step g{s16 ? K_SX16 : K_SX};
        g.tin = L.tin; g.tout = L.tacc; g.nt = lpad / 16; g.pass = 0;
        g.vec = it.d.ld % (s16 ? 8 : 4) == 0;
        const double sz = (double)dt_size(L.tin);
        g.bytes = (double)it.d.m * it.d.n * sz + (double)it.d.n * p * sz + (double)it.d.m * p * 4.0;
        g.flops = 2.0 * it.d.m * it.d.n * p;
        SxArgs ga{nullptr, it.d.ld, it.d.m, it.d.n, P->at<char>(it, L.o_X), L.nP,
                  P->at<char>(it, L.o_Y + (size_t)r * L.mP * dt_size(L.tacc)), L.mP, L.mP, nullptr, 0, it.idx, p};
        B.add(g, std::vector<SxArgs>{ga}, std::vector<int>{(int)(L.mP / 256)});
        out.push_back(g);
        // the predicted subspace W = bank Z into the first r columns
        sx(DT_F32, DT_F32, L.nt, false,
           std::vector<SxArgs>{{M->at<float>(M->L.bank), M->mP, it.d.m, M->Kr, P->wat<float>(P->w_Xw), P->ldXw,
                                P->at<char>(it, L.o_Y), L.mP, L.mP, nullptr, 0, -1, r}});
        // the iterates before the last product S^T Q need only their span
        if (it.d.q > 0) orth_tall_once(); else orth_tall(1);
        for (int i = 0; i < it.d.q; ++i) {
            pass_stq(false, &Layout::o_Zw);
            basis_small();
            pass_sx();
            if (i + 1 < it.d.q) orth_tall_once(); else orth_tall(1);
        }
        pass_stq(true);
        small_from_slabs();
        finish();
        if (std::isinf(P->tol)) return;  // accept every warm result: no residual, no continuation
        // residual of each returned triplet: Y = S A^T with FP64 products (A^T of
        // the internal FP64 coefficients, n x r), then rho_k and the decision
        Step w{K_SXW};
        w.tin = L.tin; w.nt = L.ntr;
        w.vec = it.d.ld % (s16 ? 8 : 4) == 0;
        B.add(w, std::vector<SxArgs>{{nullptr, it.d.ld, it.d.m, it.d.n, P->at<double>(it, L.o_At), L.nP,
                                      P->wat<double>(P->w_Yres), L.mP, L.mP, nullptr, 0, it.idx, r}},
              std::vector<int>{(int)(L.mP / 256)});
        out.push_back(w);
        Step rs{K_MRES};
        B.add(rs, std::vector<ModeResArgs>{{P->wat<double>(P->w_Yres), L.mP, it.d.m, P->at<float>(it, L.o_Phi), L.mP,
                                            P->at<double>(it, L.o_sig), P->wat<double>(P->w_part),
                                            (int64_t)WARM_RES_ROWS, r}},
              std::vector<int>{P->res_nchunk});
        B.add(rs, std::vector<ModeResFinalArgs>{{P->wat<double>(P->w_part), P->at<double>(it, L.o_sig),
                                                 P->wat<double>(P->w_rhom), P->wat<double>(P->w_rho), P->flags(it),
                                                 P->flag(it, WARM_DECISION), P->tol, r, P->res_nchunk}},
              std::vector<int>{1}, true);
        out.push_back(rs);
        // continuation after a rejection: q_fb more subspace iterations from the
        // warm range basis (Zw = S^T Q of the last pass is the first iterate's
        // n-side factor), then steps 5-7 again over the same buffers
        if (P->q_fb > 0) {
            const size_t first = out.size();
            basis_small();
            pass_sx();
            for (int i = 1; i < P->q_fb; ++i) {
                orth_tall_once();
                pass_stq(false, &Layout::o_Zw);
                basis_small();
                pass_sx();
            }
            orth_tall(1);
            pass_stq(true);
            small_from_slabs();
            finish();
            only_if(first, WARM_DECISION, 1);
        }
    }
    void record() {
        zero();
        frob(false);        // (energy: ||S||_F^2 in a pass of its own, non-FP32 types)
        omega();            // Alg. 1 step 1
        center_prep(true);  // (fluctuations: the indicator columns and E^T Omega / N)
        pass_sx(true);      // step 2 (and the block sums of S; FP32 energy: the partial sums of squares)
        frob(true);
        center_y();
        // step 4 (Q of the sketch); the iterates before the last product S^T Q need only their span
        const int q = C[0]->d.q;
        if (q > 0) orth_tall_once(); else orth_tall(1);
        for (int it = 0; it < q; ++it) {  // step 3, re-orthonormalised after every product
            pass_stq(false, &Layout::o_Zw);
            center_z(&Layout::o_Zw);
            basis_small();
            center_prep(false);
            pass_sx();
            center_y();
            if (it + 1 < q) orth_tall_once(); else orth_tall(1);
        }
        pass_stq(true);     // step 5 (refinement on 16-bit paths)
        center_z();
        small_from_slabs();
        finish();           // steps 6, 7 and the coefficients
    }
};

// Classes: matrices sharing the kernel template parameters of every step.
std::vector<std::vector<const Item*>> classes_of(const std::vector<Item>& items) {
    std::map<std::pair<int, int>, std::vector<const Item*>> m;
    for (const Item& it : items) m[{(it.L.nt * 256 + it.L.nta) * 2 + (it.L.nfro > 0), it.L.ntr}].push_back(&it);
    std::vector<std::vector<const Item*>> out;
    for (auto& kv : m) out.push_back(kv.second);
    return out;
}

hipError_t run_step(const rpod_plan_s* P, const Step& s, hipStream_t st) {
    switch (s.kind) {
        case K_ZERO: return launch_zero_ints(P->gl<ZeroArgs>(s, false), st);
        case K_OMEGA: return launch_omega(s.tout, P->gl<OmegaArgs>(s, false), st);
        case K_SX: return launch_sx(s.tin, s.tout, s.nt, s.vec, s.upper, P->gl<SxArgs>(s, false), st);
        case K_SXE6: return launch_sx_e6(s.nt, s.vec, s.energy, s.tall, P->gl<SxArgs>(s, false), st);
        case K_SX16: return launch_sx16(s.tin, s.nt, s.vec, P->gl<SxArgs>(s, false), st);
        case K_STQ: return launch_stq(s.tin, s.nt, s.vec, P->gl<StqArgs>(s, false), st);
        case K_STQE6: return launch_stq_e6(s.nt, s.vec, P->gl<StqArgs>(s, false), st);
        case K_STQ16: return launch_stq16(s.tin, s.nt, s.lo, s.vec, P->gl<StqArgs>(s, false), st);
        case K_REDUCE: return launch_reduce_slabs(P->gl<ReduceArgs>(s, false), st);
        case K_GRAM: return launch_gram(s.tin, s.nt, P->gl<GramArgs>(s, false), P->gl<GramArgs>(s, true), st);
        case K_CHOL: return launch_chol_inv(s.lp, P->gl<CholArgs>(s, false), st);
        case K_JACOBI: return launch_jacobi(s.lp, P->gl<JacobiArgs>(s, false), st);
        case K_LIFT: return launch_lift_coef(P->gl<LiftArgs>(s, false), st);
        case K_SPLIT: return launch_split16(s.tin, P->gl<SplitArgs>(s, false), st);
        case K_SIGNS: return launch_signs(s.tin, P->gl<ColmaxArgs>(s, false), P->gl<SignArgs>(s, true), st);
        case K_FIN: return launch_finalize(s.tin, P->gl<FinArgs>(s, false), P->gl<FinArgs>(s, true), st);
        case K_WFWD: return launch_warm_plan_forward(P->gl<WarmFwdArgs>(s, false), st);
        case K_WZ: return launch_warm_z(P->gl<WarmZArgs>(s, false), st);
        case K_SXW: return launch_sx_wide(s.tin, s.nt, s.vec, P->gl<SxArgs>(s, false), st);
        case K_MRES: return launch_warm_mode_res(P->gl<ModeResArgs>(s, false), P->gl<ModeResFinalArgs>(s, true), st);
        case K_CPREP: return launch_center_prep(s.tin, P->gl<CprepArgs>(s, false), st);
        case K_CY: return launch_center_y(s.tin, P->gl<CenterYArgs>(s, false), st);
        case K_CCROSS: return launch_center_cross(s.tin, P->gl<CrossArgs>(s, false), st);
        case K_CSUM: return launch_center_sum(P->gl<CrossSumArgs>(s, false), st);
        case K_CZ: return launch_center_z(P->gl<CenterZArgs>(s, false), st);
        case K_FROB:
            return launch_frob(s.tin, s.vec, s.energy, P->gl<FrobArgs>(s, false), P->gl<FrobArgs>(s, true), st);
        case K_EYE: return launch_eye(P->gl<EyeArgs>(s, false), st);
        case K_ADEC: return launch_adapt_decide(P->gl<AdaptDecideArgs>(s, false), st);
        case K_ARANK: return launch_adapt_rank(P->gl<AdaptRankArgs>(s, false), st);
    }
    return hipErrorInvalidValue;
}

// Record the start (begin=true) or stop event of one pass over S.
hipError_t mark(rpod_plan_s* P, const Step& s, bool begin, hipStream_t st) {
    if (!P->timing || s.pass < 0) return hipSuccess;
    const int kind = s.pass;
    std::vector<hipEvent_t>& v = P->ev[kind];
    const size_t idx = begin ? 2 * P->used[kind] : 2 * P->used[kind] + 1;
    if (idx >= v.size()) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        v.push_back(e);
    }
    hipError_t err = hipEventRecord(v[idx], st);
    if (!begin) {
        if (P->evbytes[kind].size() <= P->used[kind]) {
            P->evbytes[kind].push_back(0);
            P->evflops[kind].push_back(0);
        }
        P->evbytes[kind][P->used[kind]] = s.bytes;
        P->evflops[kind][P->used[kind]] = s.flops;
        ++P->used[kind];
    }
    return err;
}

hipError_t replay(rpod_plan_s* P, const std::vector<std::vector<Step>>& programs, hipStream_t st) {
    for (const std::vector<Step>& prog : programs)
        for (const Step& s : prog) {
            hipError_t e = mark(P, s, true, st);
            if (e == hipSuccess) e = run_step(P, s, st);
            if (e == hipSuccess) e = mark(P, s, false, st);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

// Capture the whole program into a hipGraph on private streams, one branch per
// class (branches are independent).
hipError_t capture(rpod_plan_s* P, const std::vector<std::vector<Step>>& programs, hipGraph_t* graph,
                   hipGraphExec_t* exec) {
    hipStream_t cs = nullptr;
    std::vector<hipStream_t> fs;
    std::vector<hipEvent_t> evs;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    const size_t nb = programs.size();
    for (size_t k = 0; e == hipSuccess && k < nb; ++k) {
        hipStream_t s;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) fs.push_back(s);
    }
    for (size_t k = 0; e == hipSuccess && k < nb + 1; ++k) {
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) evs.push_back(ev);
    }
    bool capturing = false;
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) capturing = true;
    if (e == hipSuccess) e = hipEventRecord(evs[nb], cs);
    for (size_t k = 0; e == hipSuccess && k < nb; ++k) {
        e = hipStreamWaitEvent(fs[k], evs[nb], 0);
        for (size_t i = 0; e == hipSuccess && i < programs[k].size(); ++i) e = run_step(P, programs[k][i], fs[k]);
        if (e == hipSuccess) e = hipEventRecord(evs[k], fs[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, evs[k], 0);
    }
    if (capturing) {
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
        if (e == hipSuccess) *graph = g;
        else if (g) (void)hipGraphDestroy(g);
    }
    for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
    for (hipStream_t s : fs) (void)hipStreamDestroy(s);
    if (cs) (void)hipStreamDestroy(cs);
    return e;
}

// Layout of a batch: flags, call table, matrix regions, then the program.
struct BatchLayout {
    std::vector<Item> items;
    size_t o_flags, o_calls, o_items_end;
};

rpod_status check_tuning(const rpod_tuning* t) {
    if (t == nullptr) return RPOD_OK;
    if (t->stq_workgroups < 0 || t->stq_workgroups > (1 << 20) || t->gram_workgroups < 0 ||
        t->gram_workgroups > 256)
        return fail(RPOD_EINVAL, "tuning values out of range (stq_workgroups %d, gram_workgroups %d)",
                    t->stq_workgroups, t->gram_workgroups);
    for (int k = 0; k < 6; ++k)
        if (t->reserved[k] != 0) return fail(RPOD_EINVAL, "tuning.reserved must be 0");
    return RPOD_OK;
}

rpod_status batch_layout(const rpod_desc* descs, int32_t count, const rpod_tuning* tune, BatchLayout& bl) {
    if (descs == nullptr) return fail(RPOD_EINVAL, "descs is NULL");
    if (count < 1 || count > 4096) return fail(RPOD_EINVAL, "count must be in [1, 4096] (got %d)", count);
    for (int i = 0; i < count; ++i) {
        rpod_status s = validate(&descs[i]);
        if (s != RPOD_OK) return s;
        if (descs[i].dtype != descs[0].dtype) return fail(RPOD_EINVAL, "all matrices of a batch must share dtype");
        if (descs[i].q != descs[0].q) return fail(RPOD_EINVAL, "all matrices of a batch must share q");
    }
    rpod_status ts = check_tuning(tune);
    if (ts != RPOD_OK) return ts;
    // single matrix: 5120 workgroups wanted (FP32 at 262144 x 5000: 20 column blocks x 128
    // splits, five rounds of two workgroups per CU; 16-bit at 1048576 x 10000: 40 column blocks
    // x 64 splits, ten rounds of one workgroup per CU)
    int64_t wg = count == 1 ? 5120 : std::max<int64_t>(256, 8192 / count);
    if (tune && tune->stq_workgroups > 0) wg = tune->stq_workgroups;
    const int gcap = (tune && tune->gram_workgroups > 0) ? tune->gram_workgroups : 0;  // 0: automatic
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    bl.o_flags = take((size_t)count * FLAG_INTS * sizeof(int));
    bl.o_calls = take((size_t)count * sizeof(CallDesc));
    bl.items.clear();
    for (int i = 0; i < count; ++i) {
        Item it;
        it.d = descs[i];
        it.L = make_layout(&descs[i], wg, gcap);
        it.off = take(it.L.total);
        it.idx = i;
        bl.items.push_back(it);
    }
    bl.o_items_end = off;
    return RPOD_OK;
}

// Record every class; returns the program blob.
std::vector<char> record_all(rpod_plan_s* P) {
    Builder B;
    P->programs.clear();
    for (const std::vector<const Item*>& cls : classes_of(P->items)) {
        P->programs.emplace_back();
        Recorder R{P, B, cls, P->programs.back()};
        R.record();
    }
    return B.blob;
}

rpod_status workspace_bytes(const rpod_desc* descs, int32_t count, const rpod_tuning* tune, size_t* bytes) {
    BatchLayout bl;
    rpod_status s = batch_layout(descs, count, tune, bl);
    if (s != RPOD_OK) return s;
    rpod_plan_s tmp;
    tmp.items = bl.items;
    tmp.o_flags = bl.o_flags;
    tmp.o_calls = bl.o_calls;
    tmp.o_prog = bl.o_items_end;
    const std::vector<char> blob = record_all(&tmp);
    *bytes = bl.o_items_end + (blob.size() + 255) / 256 * 256;
    return RPOD_OK;
}

void destroy_plan(rpod_plan_s* P) {
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    for (int k = 0; k < 3; ++k)
        for (hipEvent_t ev : P->ev[k]) (void)hipEventDestroy(ev);
    delete P;
}

rpod_status create_plan(rpod_plan* plan, const rpod_desc* descs, int32_t count, const rpod_tuning* tune,
                        void* workspace, size_t ws_bytes, void* hip_stream) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    *plan = nullptr;
    BatchLayout bl;
    rpod_status s = batch_layout(descs, count, tune, bl);
    if (s != RPOD_OK) return s;
    if (workspace == nullptr) return fail(RPOD_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % 256 != 0) return fail(RPOD_EINVAL, "workspace must be 256-byte aligned");
    size_t need = 0;
    s = workspace_bytes(descs, count, tune, &need);
    if (s != RPOD_OK) return s;
    if (ws_bytes < need) return fail(RPOD_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, need);
    rpod_plan_s* P = new (std::nothrow) rpod_plan_s;
    if (P == nullptr) return fail(RPOD_ENOMEM, "host allocation of the plan failed");
    P->items = bl.items;
    P->ws = static_cast<char*>(workspace);
    P->ws_bytes = ws_bytes;
    P->st = static_cast<hipStream_t>(hip_stream);
    P->o_flags = bl.o_flags;
    P->o_calls = bl.o_calls;
    P->o_prog = bl.o_items_end;
    P->host_calls.resize(count);
    const std::vector<char> blob = record_all(P);
    hipError_t e = hipMemsetAsync(workspace, 0, need, P->st);
    if (e == hipSuccess) e = hipMemcpyAsync(P->ws + P->o_prog, blob.data(), blob.size(), hipMemcpyHostToDevice, P->st);
    if (e == hipSuccess) e = hipStreamSynchronize(P->st);  // the blob is host memory of this frame
    if (e != hipSuccess) {
        destroy_plan(P);
        return fail(RPOD_EHIP, "initialising the workspace failed: %s", hipGetErrorString(e));
    }
    const char* ng = std::getenv("RPOD_NO_GRAPH");
    if (!(ng && ng[0] == '1')) {
        e = capture(P, P->programs, &P->graph, &P->exec);
        if (e != hipSuccess) {
            destroy_plan(P);
            return fail(RPOD_EHIP, "capturing the launch graph failed: %s", hipGetErrorString(e));
        }
    }
    *plan = P;
    return RPOD_OK;
}

rpod_status compute_impl(rpod_plan_s* P, const void* const* S, const uint64_t* seeds, void* const* Phi,
                         double* const* sigma, void* const* A, const float* mu = nullptr) {
    const int count = (int)P->items.size();
    for (int i = 0; i < count; ++i) {
        const Item& it = P->items[i];
        if (S[i] == nullptr || Phi[i] == nullptr || sigma[i] == nullptr || A[i] == nullptr)
            return fail(RPOD_EINVAL, "matrix %d: S, Phi, sigma and A must be non-NULL", i);
        // vector loads of S need 16-byte alignment when ld allows them
        const int64_t vq = is16(it.L.tin) ? 8 : 4;
        if (it.d.ld % vq == 0 && (uintptr_t)S[i] % 16 != 0)
            return fail(RPOD_EINVAL, "matrix %d: S must be 16-byte aligned when ld is a multiple of %lld", i,
                        (long long)vq);
        if ((uintptr_t)S[i] % dt_size(it.L.tin) != 0)
            return fail(RPOD_EINVAL, "matrix %d: S is not aligned to its element size", i);
        const size_t so = dt_size(it.L.tacc);
        if ((uintptr_t)Phi[i] % so || (uintptr_t)A[i] % so || (uintptr_t)sigma[i] % 8)
            return fail(RPOD_EINVAL, "matrix %d: Phi, A or sigma is not aligned to its element size", i);
        P->host_calls[i] = CallDesc{S[i], Phi[i], sigma[i], A[i], seeds[i], {0.f, 0.f, 0.f, 0.f}};
        if (mu != nullptr)
            for (int k = 0; k < 4; ++k) P->host_calls[i].mu[k] = mu[k];
    }
    HIP_TRY(launch_set_calls(P->calls(), P->host_calls.data(), count, P->st));
    if (P->exec != nullptr && !P->timing)
        HIP_TRY(hipGraphLaunch(P->exec, P->st));
    else
        HIP_TRY(replay(P, P->programs, P->st));
    return RPOD_OK;
}

// ---------------------------------------------------------------------------
// Adaptive plans (blocked range finder of Yu, Gu and Li 2018, randQB_EI, with
// the energy rule of Sec. 4.1 as its stopping test)
// ---------------------------------------------------------------------------
// An item of width l on the buffers of `base`: the layout scalars of an
// l-column plan (l a multiple of 16), the base's buffer offsets.
Item width_variant(const Item& base, int l) {
    Item v = base;
    v.d.r = l;
    v.d.p = 0;
    v.L.l = l;
    v.L.lp = l;
    v.L.nt = l / 16;
    v.L.rp = l;
    v.L.ntr = l / 16;
    v.L.lpa = l;
    v.L.nta = l / 16;
    return v;
}

// One program: the sketch, then block i = 0 .. kmax - 1, each of which runs
// only while the stopping test has not fired (block 0 always), then the
// finish for k = 1 .. kmax blocks, of which exactly one runs.
void record_adaptive(rpod_plan_s* P, Builder& B) {
    P->programs.assign(1, {});
    std::vector<Step>& out = P->programs[0];
    const Item& base = P->items[0];
    const int b = P->adapt_b, kmax = P->adapt_kmax, q = base.d.q;
    const size_t si = dt_size(base.L.tin), sa = dt_size(base.L.tacc);
    Recorder R0{P, B, {&base}, out};
    R0.zero();
    R0.frob(false);   // ||S||_F^2: a pass of its own off FP32
    R0.omega();       // all l_max columns; block i uses columns i b .. i b + b - 1
    for (int i = 0; i < kmax; ++i) {
        // the block's own operands: its sketch columns, its columns of Q1 (and
        // of the hi / lo parts), S^T Q_i of the power steps in Zt, B_i^T into Zw
        Item blk = width_variant(base, b);
        blk.L.o_X += (size_t)i * b * base.L.nP * si;
        blk.L.o_Q1 += (size_t)i * b * base.L.mP * sa;
        blk.L.o_Y = blk.L.o_Q1;
        blk.L.o_Qh += (size_t)i * b * base.L.mP * 2;
        blk.L.o_Ql += (size_t)i * b * base.L.mP * 2;
        blk.L.o_Zw = base.L.o_Zt;
        blk.L.o_Zt = base.L.o_Zw + (size_t)i * b * base.L.nP * 8;
        Item joint = width_variant(base, (i + 1) * b);  // [Q_0 .. Q_{i-1}, Y_i] in Q1
        Recorder Rb{P, B, {&blk}, out}, Rj{P, B, {&joint}, out};
        const size_t first = out.size();
        Rb.pass_sx(i == 0);   // Y_i = S Omega_i into Q1's block (block 0: FP32 energy partial sums)
        if (i == 0) R0.frob(true);
        Rj.orth_joint();      // Q_i = orth(Y_i - Q (Q^T Y_i)), twice
        for (int j = 0; j < q; ++j) {
            Rb.split_q();
            Rb.pass_stq(false, &Layout::o_Zw);  // S^T Q_i (Q_i is orthogonal to Q: B^T Q^T Q_i vanishes)
            Rb.basis_small();                   // Z_i = orth(S^T Q_i) into the block's sketch columns
            Rb.pass_sx();                       // S Z_i into Q1's block
            Rj.orth_joint();                    // Q_i = orth(S Z_i - Q (B Z_i)), twice
        }
        Rb.split_q();
        Rb.pass_stq(true, &Layout::o_Zt);       // B_i^T = S^T Q_i into Zw's block
        Rb.frob_z(P->adat(2 * ADAPT_MAX_BLOCKS), P->adat(i));
        Rb.adapt_decide(i);
        if (i > 0) Rb.only_if(first, ADAPT_ACTIVE, 1 << i);
    }
    for (int k = 1; k <= kmax; ++k) {
        Item fin = width_variant(base, k * b);  // Q1[:, :k b] explicit, B^T = Zw[:, :k b]
        Recorder Rf{P, B, {&fin}, out};
        const size_t first = out.size();
        Rf.eye1();
        Rf.finish();          // steps 6-7 of Alg. 1 on B, outputs of k b modes
        Rf.adapt_rank();
        Rf.only_if(first, ADAPT_STOP, 1 << k);
    }
    for (Step& st : out) st.pass = -1;  // per-pass timing is not kept for adaptive plans
}

rpod_status adaptive_build(rpod_plan_s* P, const rpod_desc* desc, double delta, std::vector<char>* blob_out,
                           size_t* bytes) {
    if (desc == nullptr) return fail(RPOD_EINVAL, "desc is NULL");
    if (desc->flags != 0) return fail(RPOD_EINVAL, "adaptive plans take flags = 0 (||S||_F^2 is always computed)");
    if (desc->block_cols != 0) return fail(RPOD_EUNSUPPORTED, "adaptive plans take block_cols = 0");
    const int b = desc->p, lmax = desc->r;
    if (b < 16 || b % 16 != 0) return fail(RPOD_EINVAL, "p (the block width) must be a positive multiple of 16 (got %d)", b);
    if (lmax < b || lmax % b != 0 || lmax > 128)
        return fail(RPOD_EINVAL, "r (the largest sketch width) must be a multiple of p and at most 128 (got %d)", lmax);
    if (!(delta > 0.0 && delta <= 1.0)) return fail(RPOD_EINVAL, "delta must lie in (0, 1]");
    rpod_desc d = *desc;
    d.r = lmax;
    d.p = 0;
    d.flags = RPOD_DESC_ENERGY;
    BatchLayout bl;
    rpod_status s = batch_layout(&d, 1, nullptr, bl);
    if (s != RPOD_OK) return s;
    P->items = bl.items;
    P->o_flags = bl.o_flags;
    P->o_calls = bl.o_calls;
    P->o_adapt = bl.o_items_end;
    P->o_prog = P->o_adapt + 1024;  // cap[8], E[8], 64 partial sums
    P->delta = delta;
    P->adapt_b = b;
    P->adapt_kmax = lmax / b;
    Builder B;
    record_adaptive(P, B);
    *bytes = P->o_prog + (B.blob.size() + 255) / 256 * 256;
    if (blob_out) *blob_out = B.blob;
    return RPOD_OK;
}

// ---------------------------------------------------------------------------
// Warm plans
// ---------------------------------------------------------------------------
rpod_status warm_check(const rpod_desc* d, const rpod_warm_s* M) {
    if (M == nullptr) return fail(RPOD_EINVAL, "model is NULL");
    rpod_status s = validate(d);
    if (s != RPOD_OK) return s;
    if (d->dtype == RPOD_F64) return fail(RPOD_EUNSUPPORTED, "warm plans take FP32, BF16 or FP16 matrices");
    if (d->m != M->d.m) return fail(RPOD_EINVAL, "desc.m (%lld) differs from the model's m (%lld)", (long long)d->m,
                                    (long long)M->d.m);
    if (d->r != M->d.r) return fail(RPOD_EINVAL, "desc.r (%d) differs from the model's r (%d)", d->r, M->d.r);
    if (d->p < 1) return fail(RPOD_EINVAL, "warm plans need p >= 1 Gaussian columns");
    return RPOD_OK;
}

// Warm region after the matrix region; returns its size.
size_t warm_region(rpod_plan_s* P) {
    const Item& it = P->items[0];
    const Layout& L = it.L;
    P->ldXw = roundup(P->model->Kr, 16);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    P->w_Xw = take((size_t)P->ldXw * L.lp * 4);
    P->w_c = take(WARM_K * 8);
    P->w_kstar = take(sizeof(int));
    P->w_Yres = take((size_t)L.mP * L.rp * 8);
    P->res_nchunk = (int)((it.d.m + WARM_RES_ROWS - 1) / WARM_RES_ROWS);
    P->w_part = take((size_t)P->res_nchunk * it.d.r * 8);
    P->w_rho = take(8);
    P->w_rhom = take((size_t)it.d.r * 8);
    return off;
}

// Lay out and record a warm plan (host only); returns the workspace bytes.
rpod_status warm_build(rpod_plan_s* P, const rpod_desc* desc, rpod_warm_s* M, int32_t q_fb, double tol,
                       std::vector<char>* blob_out, size_t* bytes) {
    rpod_status s = warm_check(desc, M);
    if (s != RPOD_OK) return s;
    if (desc->block_cols != 0) return fail(RPOD_EUNSUPPORTED, "warm plans take block_cols = 0");
    if (desc->flags != 0) return fail(RPOD_EUNSUPPORTED, "warm plans take flags = 0");
    if (q_fb < 0) return fail(RPOD_EINVAL, "q_fallback must be >= 0");
    if (!(tol >= 0.0)) return fail(RPOD_EINVAL, "tol must be >= 0");
    BatchLayout bl;
    s = batch_layout(desc, 1, nullptr, bl);
    if (s != RPOD_OK) return s;
    P->items = bl.items;
    P->o_flags = bl.o_flags;
    P->o_calls = bl.o_calls;
    P->model = M;
    P->tol = tol;
    P->q_fb = q_fb;
    P->o_warm = bl.o_items_end;
    const size_t wbytes = warm_region(P);
    P->o_prog = P->o_warm + wbytes;
    Builder B;
    P->programs.assign(1, {});
    {
        std::vector<const Item*> cls{&P->items[0]};
        Recorder R{P, B, cls, P->programs[0]};
        R.record_warm();
    }
    *bytes = P->o_prog + (B.blob.size() + 255) / 256 * 256;
    if (blob_out) *blob_out = B.blob;
    return RPOD_OK;
}

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------
const int STQ_CANDIDATES[] = {128, 256, 512, 1024, 2048, 4096, 8192};
const int GRAM_CANDIDATES[] = {32, 64, 128, 256};

// Output buffers of the trial calls, placed after the largest trial plan.
struct TrialOutputs {
    size_t plan_bytes;
    std::vector<size_t> phi, sig, a;
    size_t total;
};

rpod_status autotune_bytes(const rpod_desc* descs, int32_t count, size_t* bytes, TrialOutputs* to) {
    BatchLayout bl;
    rpod_status s = batch_layout(descs, count, nullptr, bl);
    if (s != RPOD_OK) return s;
    size_t pb = 0;
    s = workspace_bytes(descs, count, nullptr, &pb);
    if (s != RPOD_OK) return s;
    for (int c : STQ_CANDIDATES) {
        rpod_tuning t{};
        t.stq_workgroups = c;
        size_t b = 0;
        s = workspace_bytes(descs, count, &t, &b);
        if (s != RPOD_OK) return s;
        pb = std::max(pb, b);
    }
    TrialOutputs o;
    o.plan_bytes = (pb + 255) / 256 * 256;
    size_t off = o.plan_bytes;
    for (int i = 0; i < count; ++i) {
        const size_t so = descs[i].dtype == RPOD_F64 ? 8 : 4;
        o.phi.push_back(off);
        off += ((size_t)descs[i].m * descs[i].r * so + 255) / 256 * 256;
        o.sig.push_back(off);
        off += ((size_t)descs[i].r * 8 + 255) / 256 * 256;
        o.a.push_back(off);
        off += ((size_t)descs[i].r * descs[i].n * so + 255) / 256 * 256;
    }
    o.total = off;
    *bytes = off;
    if (to) *to = o;
    return RPOD_OK;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

bool cache_lookup(const char* path, uint64_t key, rpod_tuning* best, double* ms) {
    if (path == nullptr) return false;
    FILE* f = std::fopen(path, "r");
    if (f == nullptr) return false;
    unsigned long long k = 0;
    int a = 0, b = 0;
    double t = 0;
    bool found = false;
    while (std::fscanf(f, "%llx %d %d %lf", &k, &a, &b, &t) == 4) {
        if (k == key && a >= 0 && b >= 0 && b <= 256) {
            *best = rpod_tuning{};
            best->stq_workgroups = a;
            best->gram_workgroups = b;
            *ms = t;
            found = true;  // the last entry for a key wins
        }
    }
    std::fclose(f);
    return found;
}

rpod_status autotune(const rpod_desc* descs, int32_t count, const void* const* S, void* workspace, size_t ws_bytes,
                     hipStream_t st, int32_t repeats, const char* cache_path, rpod_tuning* best, double* best_ms) {
    if (best == nullptr || S == nullptr) return fail(RPOD_EINVAL, "S and best must be non-NULL");
    if (repeats < 1) return fail(RPOD_EINVAL, "repeats must be >= 1");
    TrialOutputs to;
    size_t need = 0;
    rpod_status s = autotune_bytes(descs, count, &need, &to);
    if (s != RPOD_OK) return s;
    if (workspace == nullptr || (uintptr_t)workspace % 256 != 0)
        return fail(RPOD_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < need) return fail(RPOD_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, need);
    int dev = 0;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    uint64_t key = fnv1a(1469598103934665603ull, descs, sizeof(rpod_desc) * (size_t)count);
    key = fnv1a(key, prop.gcnArchName, std::strlen(prop.gcnArchName));
    key = fnv1a(key, &prop.multiProcessorCount, sizeof(prop.multiProcessorCount));
    double ms = 0;
    if (cache_lookup(cache_path, key, best, &ms)) {
        if (best_ms) *best_ms = ms;
        return RPOD_OK;
    }
    char* ws = static_cast<char*>(workspace);
    std::vector<void*> Phi(count), A(count);
    std::vector<double*> sig(count);
    std::vector<uint64_t> seeds(count);
    for (int i = 0; i < count; ++i) {
        Phi[i] = ws + to.phi[i];
        A[i] = ws + to.a[i];
        sig[i] = reinterpret_cast<double*>(ws + to.sig[i]);
        seeds[i] = 0x5EED0000ull + (uint64_t)i;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(RPOD_EHIP, "hipEventCreate failed: %s", hipGetErrorString(he));
    }
    // time one candidate: ms per call, or a negative value on failure
    auto trial = [&](const rpod_tuning& t, rpod_status& err) -> double {
        rpod_plan p = nullptr;
        err = create_plan(&p, descs, count, &t, workspace, to.plan_bytes, st);
        if (err != RPOD_OK) return -1.0;
        err = compute_impl(p, S, seeds.data(), Phi.data(), sig.data(), A.data());
        hipError_t e = hipSuccess;
        for (int r = 0; err == RPOD_OK && e == hipSuccess && r < repeats; ++r) {
            if (r == 0) e = hipEventRecord(e0, st);
            if (e == hipSuccess) err = compute_impl(p, S, seeds.data(), Phi.data(), sig.data(), A.data());
        }
        if (err == RPOD_OK && e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float el = -1.f;
        if (err == RPOD_OK && e == hipSuccess) e = hipEventElapsedTime(&el, e0, e1);
        (void)hipStreamSynchronize(st);
        destroy_plan(p);
        if (err == RPOD_OK && e != hipSuccess) err = fail(RPOD_EHIP, "autotune timing failed: %s", hipGetErrorString(e));
        return err == RPOD_OK ? (double)el / repeats : -1.0;
    };
    rpod_tuning cur{};
    rpod_status err = RPOD_OK;
    double tbest = trial(cur, err);  // defaults
    if (err != RPOD_OK) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return err;
    }
    rpod_tuning bt = cur;
    for (int c : STQ_CANDIDATES) {
        rpod_tuning t{};
        t.stq_workgroups = c;
        const double v = trial(t, err);
        if (err != RPOD_OK) break;
        if (v < tbest) { tbest = v; bt = t; }
    }
    for (int g : GRAM_CANDIDATES) {
        if (err != RPOD_OK) break;
        rpod_tuning t = bt;
        t.gram_workgroups = g;
        const double v = trial(t, err);
        if (err != RPOD_OK) break;
        if (v < tbest) { tbest = v; bt = t; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != RPOD_OK) return err;
    *best = bt;
    if (best_ms) *best_ms = tbest;
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (f) {
            std::fprintf(f, "%016llx %d %d %.6f\n", (unsigned long long)key, bt.stq_workgroups, bt.gram_workgroups,
                         tbest);
            std::fclose(f);
        }
    }
    return RPOD_OK;
}

}  // namespace

extern "C" {

const char* rpod_last_error(void) { return g_err; }

rpod_status rpod_workspace_size(const rpod_desc* desc, size_t* bytes) {
    if (bytes == nullptr) return fail(RPOD_EINVAL, "bytes is NULL");
    return workspace_bytes(desc, 1, nullptr, bytes);
}

rpod_status rpod_workspace_size_batched(const rpod_desc* descs, int32_t count, size_t* bytes) {
    if (bytes == nullptr) return fail(RPOD_EINVAL, "bytes is NULL");
    return workspace_bytes(descs, count, nullptr, bytes);
}

rpod_status rpod_plan_create(rpod_plan* plan, const rpod_desc* desc, void* workspace, size_t workspace_bytes,
                             void* hip_stream) {
    return create_plan(plan, desc, 1, nullptr, workspace, workspace_bytes, hip_stream);
}

rpod_status rpod_plan_create_batched(rpod_plan* plan, const rpod_desc* descs, int32_t count, void* workspace,
                                     size_t workspace_bytes, void* hip_stream) {
    return create_plan(plan, descs, count, nullptr, workspace, workspace_bytes, hip_stream);
}

rpod_status rpod_workspace_size_tuned(const rpod_desc* descs, int32_t count, const rpod_tuning* tuning,
                                      size_t* bytes) {
    if (bytes == nullptr) return fail(RPOD_EINVAL, "bytes is NULL");
    return workspace_bytes(descs, count, tuning, bytes);
}

rpod_status rpod_plan_create_tuned(rpod_plan* plan, const rpod_desc* descs, int32_t count,
                                   const rpod_tuning* tuning, void* workspace, size_t workspace_bytes,
                                   void* hip_stream) {
    return create_plan(plan, descs, count, tuning, workspace, workspace_bytes, hip_stream);
}

rpod_status rpod_autotune_workspace_size(const rpod_desc* descs, int32_t count, size_t* bytes) {
    if (bytes == nullptr) return fail(RPOD_EINVAL, "bytes is NULL");
    return autotune_bytes(descs, count, bytes, nullptr);
}

rpod_status rpod_autotune(const rpod_desc* descs, int32_t count, const void* const* S, void* workspace,
                          size_t workspace_bytes, void* hip_stream, int32_t repeats, const char* cache_path,
                          rpod_tuning* best, double* best_ms) {
    return autotune(descs, count, S, workspace, workspace_bytes, static_cast<hipStream_t>(hip_stream), repeats,
                    cache_path, best, best_ms);
}

rpod_status rpod_workspace_size_warm(const rpod_desc* desc, rpod_warm model, int32_t q_fallback, size_t* bytes) {
    if (bytes == nullptr) return fail(RPOD_EINVAL, "bytes is NULL");
    rpod_plan_s tmp;
    return warm_build(&tmp, desc, model, q_fallback, 0.0, nullptr, bytes);
}

rpod_status rpod_plan_create_warm(rpod_plan* plan, const rpod_desc* desc, rpod_warm model, int32_t q_fallback,
                                  double tol, void* workspace, size_t workspace_bytes, void* hip_stream) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (workspace == nullptr || (uintptr_t)workspace % 256 != 0)
        return fail(RPOD_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    rpod_plan_s* P = new (std::nothrow) rpod_plan_s;
    if (P == nullptr) return fail(RPOD_ENOMEM, "host allocation of the plan failed");
    P->ws = static_cast<char*>(workspace);  // recorded arguments point into the workspace
    P->ws_bytes = workspace_bytes;
    P->st = static_cast<hipStream_t>(hip_stream);
    std::vector<char> blob;
    size_t need = 0;
    rpod_status s = warm_build(P, desc, model, q_fallback, tol, &blob, &need);
    if (s != RPOD_OK) {
        delete P;
        return s;
    }
    if (workspace_bytes < need) {
        delete P;
        return fail(RPOD_ENOMEM, "workspace has %zu bytes, %zu needed", workspace_bytes, need);
    }
    P->host_calls.resize(1);
    hipError_t e = hipMemsetAsync(workspace, 0, need, P->st);
    if (e == hipSuccess) e = hipMemcpyAsync(P->ws + P->o_prog, blob.data(), blob.size(), hipMemcpyHostToDevice, P->st);
    if (e == hipSuccess) e = hipStreamSynchronize(P->st);
    if (e != hipSuccess) {
        destroy_plan(P);
        return fail(RPOD_EHIP, "initialising the workspace failed: %s", hipGetErrorString(e));
    }
    const char* ng = std::getenv("RPOD_NO_GRAPH");
    if (!(ng && ng[0] == '1')) {
        e = capture(P, P->programs, &P->graph, &P->exec);
        if (e != hipSuccess) {
            destroy_plan(P);
            return fail(RPOD_EHIP, "capturing the launch graphs failed: %s", hipGetErrorString(e));
        }
    }
    *plan = P;
    return RPOD_OK;
}

rpod_status rpod_workspace_size_adaptive(const rpod_desc* desc, double delta, size_t* bytes) {
    if (bytes == nullptr) return fail(RPOD_EINVAL, "bytes is NULL");
    rpod_plan_s tmp;
    return adaptive_build(&tmp, desc, delta, nullptr, bytes);
}

rpod_status rpod_plan_create_adaptive(rpod_plan* plan, const rpod_desc* desc, double delta, void* workspace,
                                      size_t workspace_bytes, void* hip_stream) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (workspace == nullptr || (uintptr_t)workspace % 256 != 0)
        return fail(RPOD_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    rpod_plan_s* P = new (std::nothrow) rpod_plan_s;
    if (P == nullptr) return fail(RPOD_ENOMEM, "host allocation of the plan failed");
    P->ws = static_cast<char*>(workspace);
    P->ws_bytes = workspace_bytes;
    P->st = static_cast<hipStream_t>(hip_stream);
    std::vector<char> blob;
    size_t need = 0;
    rpod_status s = adaptive_build(P, desc, delta, &blob, &need);
    if (s != RPOD_OK) {
        delete P;
        return s;
    }
    if (workspace_bytes < need) {
        delete P;
        return fail(RPOD_ENOMEM, "workspace has %zu bytes, %zu needed", workspace_bytes, need);
    }
    P->host_calls.resize(1);
    hipError_t e = hipMemsetAsync(workspace, 0, need, P->st);
    if (e == hipSuccess) e = hipMemcpyAsync(P->ws + P->o_prog, blob.data(), blob.size(), hipMemcpyHostToDevice, P->st);
    if (e == hipSuccess) e = hipStreamSynchronize(P->st);
    if (e != hipSuccess) {
        destroy_plan(P);
        return fail(RPOD_EHIP, "initialising the workspace failed: %s", hipGetErrorString(e));
    }
    const char* ng = std::getenv("RPOD_NO_GRAPH");
    if (!(ng && ng[0] == '1')) {
        e = capture(P, P->programs, &P->graph, &P->exec);
        if (e != hipSuccess) {
            destroy_plan(P);
            return fail(RPOD_EHIP, "capturing the launch graph failed: %s", hipGetErrorString(e));
        }
    }
    *plan = P;
    return RPOD_OK;
}

rpod_status rpod_compute_adaptive(rpod_plan plan, const void* S, uint64_t seed, void* Phi, double* sigma, void* A,
                                  int32_t* l_used, int32_t* rank, double* residual) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    if (plan->adapt_kmax == 0) return fail(RPOD_EINVAL, "not an adaptive plan: use rpod_compute");
    rpod_status s = compute_impl(plan, &S, &seed, &Phi, &sigma, &A);
    if (s != RPOD_OK) return s;
    if (l_used == nullptr && rank == nullptr && residual == nullptr) return RPOD_OK;
    int w[8] = {0};
    double E[ADAPT_MAX_BLOCKS] = {0}, fro = 0.0;
    const Item& it = plan->items[0];
    HIP_TRY(hipMemcpyAsync(w, plan->flags(it), sizeof(w), hipMemcpyDeviceToHost, plan->st));
    HIP_TRY(hipMemcpyAsync(E, plan->adat(ADAPT_MAX_BLOCKS), sizeof(E), hipMemcpyDeviceToHost, plan->st));
    HIP_TRY(hipMemcpyAsync(&fro, plan->at<double>(it, it.L.o_Fro), sizeof(double), hipMemcpyDeviceToHost, plan->st));
    HIP_TRY(hipStreamSynchronize(plan->st));
    const int lu = w[ADAPT_LUSED];
    if (l_used) *l_used = lu;
    if (rank) *rank = w[ADAPT_RANK];
    if (residual) *residual = (lu > 0 && fro > 0.0) ? E[lu / plan->adapt_b - 1] / fro : std::nan("");
    return RPOD_OK;
}

rpod_status rpod_compute_warm(rpod_plan plan, const void* S, const float* mu, uint64_t seed, void* Phi,
                              double* sigma, void* A, int32_t* fell_back, double* rho) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    if (plan->model == nullptr) return fail(RPOD_EINVAL, "not a warm plan: use rpod_compute");
    if (mu == nullptr) return fail(RPOD_EINVAL, "mu is NULL");
    rpod_status s = compute_impl(plan, &S, &seed, &Phi, &sigma, &A, mu);
    if (s != RPOD_OK) return s;
    if (fell_back == nullptr && rho == nullptr) return RPOD_OK;
    if (std::isinf(plan->tol)) {  // no check was recorded
        if (fell_back) *fell_back = 0;
        if (rho) *rho = std::nan("");
        return RPOD_OK;
    }
    double rh = 0.0;
    int dec = 0;
    HIP_TRY(hipMemcpyAsync(&rh, plan->wat<double>(plan->w_rho), sizeof(double), hipMemcpyDeviceToHost, plan->st));
    HIP_TRY(hipMemcpyAsync(&dec, plan->flag(plan->items[0], WARM_DECISION), sizeof(int), hipMemcpyDeviceToHost,
                           plan->st));
    HIP_TRY(hipStreamSynchronize(plan->st));
    if (fell_back) *fell_back = dec;
    if (rho) *rho = rh;
    return RPOD_OK;
}

rpod_status rpod_warm_residuals(rpod_plan plan, double* rho_modes) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    if (plan->model == nullptr) return fail(RPOD_EINVAL, "not a warm plan");
    if (rho_modes == nullptr) return fail(RPOD_EINVAL, "rho_modes is NULL");
    if (std::isinf(plan->tol)) return fail(RPOD_EINVAL, "the plan was made with tol = +infinity: no residuals");
    HIP_TRY(hipMemcpyAsync(rho_modes, plan->wat<double>(plan->w_rhom), sizeof(double) * plan->items[0].d.r,
                           hipMemcpyDeviceToHost, plan->st));
    HIP_TRY(hipStreamSynchronize(plan->st));
    return RPOD_OK;
}

rpod_status rpod_plan_destroy(rpod_plan plan) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    hipError_t e = hipStreamSynchronize(plan->st);
    destroy_plan(plan);
    if (e != hipSuccess) return fail(RPOD_EHIP, "stream synchronisation failed: %s", hipGetErrorString(e));
    return RPOD_OK;
}

rpod_status rpod_compute(rpod_plan plan, const void* S, uint64_t seed, void* Phi, double* sigma, void* A) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    if (plan->items.size() != 1) return fail(RPOD_EINVAL, "plan holds a batch: use rpod_compute_batched");
    if (plan->model != nullptr) return fail(RPOD_EINVAL, "warm plan: use rpod_compute_warm");
    if (plan->adapt_kmax > 0) return fail(RPOD_EINVAL, "adaptive plan: use rpod_compute_adaptive");
    return compute_impl(plan, &S, &seed, &Phi, &sigma, &A);
}

rpod_status rpod_compute_batched(rpod_plan plan, const void* const* S, const uint64_t* seeds, void* const* Phi,
                                 double* const* sigma, void* const* A) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    if (S == nullptr || seeds == nullptr || Phi == nullptr || sigma == nullptr || A == nullptr)
        return fail(RPOD_EINVAL, "pointer arrays must be non-NULL");
    if (plan->model != nullptr) return fail(RPOD_EINVAL, "warm plan: use rpod_compute_warm");
    if (plan->adapt_kmax > 0) return fail(RPOD_EINVAL, "adaptive plan: use rpod_compute_adaptive");
    return compute_impl(plan, S, seeds, Phi, sigma, A);
}

rpod_status rpod_status_query_batched(rpod_plan plan, int32_t* per_matrix_flags) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    const size_t count = plan->items.size();
    std::vector<int> host(count * FLAG_INTS, 0);
    hipError_t e = hipMemcpyAsync(host.data(), plan->ws + plan->o_flags, host.size() * sizeof(int),
                                  hipMemcpyDeviceToHost, plan->st);
    if (e == hipSuccess) e = hipStreamSynchronize(plan->st);
    if (e != hipSuccess) return fail(RPOD_EHIP, "reading the status words failed: %s", hipGetErrorString(e));
    int all = 0;
    for (size_t i = 0; i < count; ++i) {
        all |= host[i * FLAG_INTS];
        if (per_matrix_flags) per_matrix_flags[i] = host[i * FLAG_INTS];
    }
    if (all & RPOD_FLAG_NONFINITE) return fail(RPOD_EINVAL_DATA, "non-finite values in S");
    if (all & RPOD_FLAG_BREAKDOWN) return fail(RPOD_EBREAKDOWN, "sketch rank-deficient after the shifted CholeskyQR retry");
    return RPOD_OK;
}

rpod_status rpod_energy(rpod_plan plan, int32_t item, double delta, double* energy, int32_t* rank) {
    if (plan == nullptr || energy == nullptr) return fail(RPOD_EINVAL, "plan and energy must be non-NULL");
    if (item < 0 || item >= (int32_t)plan->items.size())
        return fail(RPOD_EINVAL, "item %d out of range (the plan has %zu matrices)", item, plan->items.size());
    if (!(delta > 0.0 && delta < 1.0)) return fail(RPOD_EINVAL, "delta must lie in (0, 1)");
    if (plan->adapt_kmax > 0)
        return fail(RPOD_EINVAL, "adaptive plan: its energy rank comes from rpod_compute_adaptive");
    const Item& it = plan->items[item];
    if (it.L.nfro == 0) return fail(RPOD_EINVAL, "the plan was made without RPOD_DESC_ENERGY");
    std::vector<double> sig(it.L.lp, 0.0);
    double fro = 0.0;
    HIP_TRY(hipMemcpyAsync(sig.data(), plan->at<double>(it, it.L.o_sig), sizeof(double) * it.L.lp,
                           hipMemcpyDeviceToHost, plan->st));
    HIP_TRY(hipMemcpyAsync(&fro, plan->at<double>(it, it.L.o_Fro), sizeof(double), hipMemcpyDeviceToHost, plan->st));
    HIP_TRY(hipStreamSynchronize(plan->st));
    int32_t rk = -1;
    double acc = 0.0;
    for (int k = 0; k < it.L.l; ++k) {
        acc += sig[k] * sig[k];
        energy[k] = fro > 0.0 ? acc / fro : 0.0;
        if (rk < 0 && energy[k] >= delta) rk = k + 1;
    }
    if (rank) *rank = rk;
    return RPOD_OK;
}

// scratch of rpod_reconstruct: abar, the two sums, the error's partial sums,
// and for FP32 fields on the matrix cores the augmented modes, one chunk's
// operand and its launch record
struct ReconLayout {
    size_t abar, out2, part, aug, x, rec, tstart, total;
    int64_t lda;
    int ldx;
};
ReconLayout recon_layout(int64_t m, int r) {
    ReconLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    L.lda = roundup(m, 4);
    L.ldx = (int)roundup(r + 1, 32);
    L.abar = take((size_t)r * 8);
    L.out2 = take(16);
    L.part = take((size_t)2 * ((m + 255) / 256) * 8);
    L.aug = take((size_t)L.lda * (r + 1) * 4);
    L.x = take((size_t)L.ldx * 128 * 4);
    L.rec = take(sizeof(SxArgs));
    L.tstart = take(2 * sizeof(int));
    L.total = off;
    return L;
}

rpod_status rpod_reconstruct_workspace_size(int64_t m, int32_t r, size_t* bytes) {
    if (bytes == nullptr) return fail(RPOD_EINVAL, "bytes is NULL");
    if (m < 1 || r < 1 || r > 128) return fail(RPOD_EINVAL, "need m >= 1 and 1 <= r <= 128");
    *bytes = recon_layout(m, r).total;
    return RPOD_OK;
}

rpod_status rpod_reconstruct(int32_t dtype, int64_t m, int32_t r, int64_t T, const void* Phi, const void* mean,
                             const void* alpha, void* out, const void* ref, int64_t ld_ref, void* workspace,
                             size_t workspace_bytes, void* hip_stream, double* eps) {
    if (dtype != RPOD_F64 && dtype != RPOD_F32) return fail(RPOD_EINVAL, "dtype must be RPOD_F64 or RPOD_F32");
    if (T < 1) return fail(RPOD_EINVAL, "T must be >= 1");
    size_t need = 0;
    rpod_status s = rpod_reconstruct_workspace_size(m, r, &need);
    if (s != RPOD_OK) return s;
    if (Phi == nullptr || alpha == nullptr) return fail(RPOD_EINVAL, "Phi and alpha must be non-NULL");
    if (ref != nullptr && ld_ref < m) return fail(RPOD_EINVAL, "ld_ref (%lld) must be >= m", (long long)ld_ref);
    if (workspace == nullptr || (uintptr_t)workspace % 256 != 0)
        return fail(RPOD_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    if (workspace_bytes < need) return fail(RPOD_ENOMEM, "workspace has %zu bytes, %zu needed", workspace_bytes, need);
    char* ws = static_cast<char*>(workspace);
    const ReconLayout RL = recon_layout(m, r);
    double* abar = reinterpret_cast<double*>(ws + RL.abar);
    double* out2 = reinterpret_cast<double*>(ws + RL.out2);
    double* part = reinterpret_cast<double*>(ws + RL.part);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // FP32 fields on the matrix cores when the output allows 16-byte stores
    const bool mfma = dtype == RPOD_F32 && out != nullptr && m % 4 == 0 && (uintptr_t)out % 16 == 0;
    if (mfma)
        HIP_TRY(launch_reconstruct_mfma(m, r, T, static_cast<const float*>(Phi), static_cast<const float*>(mean),
                                        static_cast<const float*>(alpha), static_cast<float*>(out),
                                        reinterpret_cast<float*>(ws + RL.aug), RL.lda,
                                        reinterpret_cast<float*>(ws + RL.x), RL.ldx,
                                        reinterpret_cast<SxArgs*>(ws + RL.rec), reinterpret_cast<int*>(ws + RL.tstart),
                                        st));
    HIP_TRY(launch_reconstruct(dtype == RPOD_F64 ? DT_F64 : DT_F32, m, r, T, Phi, mean, alpha, mfma ? nullptr : out,
                               ref, ld_ref, abar, part, out2, st));
    if (ref != nullptr && eps != nullptr) {
        double h[2] = {0.0, 0.0};
        HIP_TRY(hipMemcpyAsync(h, out2, sizeof(h), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        *eps = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : 0.0;
    }
    return RPOD_OK;
}

rpod_status rpod_reconstruct_noalloc(int32_t dtype, int64_t m, int32_t r, int64_t T, const void* Phi,
                                     const void* mean, const void* alpha, void* out, const void* ref, int64_t ld_ref,
                                     void* hip_stream, double* eps) {
    if (dtype != RPOD_F64 && dtype != RPOD_F32) return fail(RPOD_EINVAL, "dtype must be RPOD_F64 or RPOD_F32");
    if (T < 1) return fail(RPOD_EINVAL, "T must be >= 1");
    if (m < 1 || r < 1 || r > 128) return fail(RPOD_EINVAL, "need m >= 1 and 1 <= r <= 128");
    if (m > RECON_NOALLOC_MAX_M)
        return fail(RPOD_EINVAL, "m = %lld exceeds the static scratch of this entry point (m <= %lld); "
                    "use rpod_reconstruct with a workspace", (long long)m, (long long)RECON_NOALLOC_MAX_M);
    if (Phi == nullptr || alpha == nullptr) return fail(RPOD_EINVAL, "Phi and alpha must be non-NULL");
    if (ref != nullptr && ld_ref < m) return fail(RPOD_EINVAL, "ld_ref (%lld) must be >= m", (long long)ld_ref);
    double* sc = nullptr;
    HIP_TRY(recon_scratch(&sc));
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // every scratch word the kernels read is written earlier in the same call: nothing to clear
    HIP_TRY(launch_reconstruct(dtype == RPOD_F64 ? DT_F64 : DT_F32, m, r, T, Phi, mean, alpha, out, ref, ld_ref, sc,
                               sc + 256, sc + 128, st));
    if (ref != nullptr && eps != nullptr) {
        double h[2] = {0.0, 0.0};
        HIP_TRY(hipMemcpyAsync(h, sc + 128, sizeof(h), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        *eps = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : 0.0;
    }
    return RPOD_OK;
}

rpod_status rpod_status_query(rpod_plan plan, int32_t* device_flags) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    std::vector<int32_t> f(plan->items.size(), 0);
    rpod_status s = rpod_status_query_batched(plan, f.data());
    if (device_flags) {
        int32_t all = 0;
        for (int32_t v : f) all |= v;
        *device_flags = all;
    }
    return s;
}

rpod_status rpod_plan_set_timing(rpod_plan plan, int32_t enable) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    plan->timing = enable != 0;
    plan->used[0] = plan->used[1] = plan->used[2] = 0;
    return RPOD_OK;
}

rpod_status rpod_plan_get_timing(rpod_plan plan, int32_t pass, int64_t* launches, double* total_ms,
                                 double* bytes_per_launch, double* flops_per_launch) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    if (pass < 0 || pass > 2) return fail(RPOD_EINVAL, "pass must be 0, 1 or 2");
    HIP_TRY(hipStreamSynchronize(plan->st));
    double tot = 0.0, b = 0.0, f = 0.0;
    for (size_t k = 0; k < plan->used[pass]; ++k) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, plan->ev[pass][2 * k], plan->ev[pass][2 * k + 1]));
        tot += ms;
        b += plan->evbytes[pass][k];
        f += plan->evflops[pass][k];
    }
    const double nl = (double)std::max<size_t>(plan->used[pass], 1);
    if (launches) *launches = (int64_t)plan->used[pass];
    if (total_ms) *total_ms = tot;
    if (bytes_per_launch) *bytes_per_launch = b / nl;
    if (flops_per_launch) *flops_per_launch = f / nl;
    return RPOD_OK;
}

rpod_status rpod_generate_omega(uint64_t seed, int64_t n, int32_t l, int32_t dtype, void* out, int64_t ldo,
                                void* hip_stream) {
    if (n < 1 || l < 1) return fail(RPOD_EINVAL, "n and l must be >= 1");
    if (ldo < n) return fail(RPOD_EINVAL, "ldo must be >= n");
    if (out == nullptr) return fail(RPOD_EINVAL, "out is NULL");
    if (dtype < RPOD_F64 || dtype > RPOD_F16) return fail(RPOD_EINVAL, "unknown dtype %d", dtype);
    HIP_TRY(launch_omega_direct(dtype, seed, n, l, out, ldo, static_cast<hipStream_t>(hip_stream)));
    return RPOD_OK;
}

rpod_status rpod_sketch_bits(uint64_t seed, int64_t n, int32_t l, uint32_t* out, void* hip_stream) {
    if (n < 1 || l < 1) return fail(RPOD_EINVAL, "n and l must be >= 1");
    if (out == nullptr) return fail(RPOD_EINVAL, "out is NULL");
    HIP_TRY(launch_sketch_bits(seed, n, l, out, static_cast<hipStream_t>(hip_stream)));
    return RPOD_OK;
}

}  // extern "C"
