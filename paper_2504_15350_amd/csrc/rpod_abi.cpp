// C ABI of the randomized POD library: validation, workspace layout, plans
// and the launch sequence of one rPOD call (Alg. 1 of Sec. 4.2).
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/rpod.h"
#include "internal.hpp"

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

size_t dt_size(int dt) {
    switch (dt) {
        case DT_F64: return 8;
        case DT_F32: return 4;
        case DT_BF16: case DT_F16: return 2;
        default: return 0;
    }
}

// Everything the launch sequence needs, derived from the description.
struct Layout {
    int l, lp, nt, rp, ntr;
    int64_t mP, nP;
    int tin, tacc;
    int nsplit;
    int64_t split_rows;
    int nchunk;
    // byte offsets into the workspace
    size_t o_flags, o_X, o_Y, o_Q1, o_Qh, o_Ql, o_Zp, o_Zt, o_Zw, o_Zw2, o_Gpart, o_G;
    size_t o_R64[3], o_R32[3], o_UB, o_sig, o_M64, o_M32, o_Ur, o_Phi, o_At, o_pval, o_pidx, o_signs;
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
    if (d->flags != 0) return fail(RPOD_EINVAL, "flags must be 0");
    if (d->dtype < RPOD_F64 || d->dtype > RPOD_F16) return fail(RPOD_EINVAL, "unknown dtype %d", d->dtype);
    const int64_t l = (int64_t)d->r + d->p;
    const int64_t mn = d->m < d->n ? d->m : d->n;
    if (l > mn) return fail(RPOD_EINVAL, "l = r + p = %lld exceeds min(m, n) = %lld", (long long)l, (long long)mn);
    if (l > 128) return fail(RPOD_EUNSUPPORTED, "l = r + p = %lld exceeds 128", (long long)l);
    return RPOD_OK;
}

Layout make_layout(const rpod_desc* d) {
    Layout L{};
    L.l = d->r + d->p;
    L.lp = (int)roundup(L.l, 16);
    L.nt = L.lp / 16;
    L.rp = (int)roundup(d->r, 16);
    L.ntr = L.rp / 16;
    L.mP = roundup(d->m, 256);
    L.nP = roundup(d->n, 256);
    L.tin = d->dtype == RPOD_F64 ? DT_F64 : d->dtype == RPOD_F32 ? DT_F32 : d->dtype == RPOD_BF16 ? DT_BF16 : DT_F16;
    L.tacc = d->dtype == RPOD_F64 ? DT_F64 : DT_F32;
    // split-K over rows for S^T Q. FP32/FP64: ~1024 workgroups of 256
    // columns, contiguous splits of >= 256 rows. 16-bit: ~4096 blocks of 128
    // columns (up to 64 splits), splits interleaved in steps of R rows.
    const bool s16k = d->dtype == RPOD_BF16 || d->dtype == RPOD_F16;
    const int64_t ncb = s16k ? L.nP / 128 : L.nP / 256;
    const int64_t target = s16k ? 4096 : 1024;
    int64_t ns = (target + ncb - 1) / ncb;
    if (ns > 64) ns = 64;
    const int64_t maxs = (d->m + (s16k ? 127 : 255)) / (s16k ? 128 : 256);
    if (ns > maxs) ns = maxs;
    if (ns < 1) ns = 1;
    L.split_rows = roundup((d->m + ns - 1) / ns, 64);
    L.nsplit = s16k ? (int)ns : (int)((d->m + L.split_rows - 1) / L.split_rows);
    int64_t nc = d->m / 2048;
    L.nchunk = (int)(nc < 1 ? 1 : (nc > 256 ? 256 : nc));

    const size_t sa = dt_size(L.tacc), si = dt_size(L.tin);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t lp2 = (size_t)L.lp * L.lp;
    L.o_flags = take(64 * sizeof(int));
    L.o_X = take((size_t)L.nP * L.lp * si);
    L.o_Y = take((size_t)L.mP * L.lp * sa);
    L.o_Q1 = take((size_t)L.mP * L.lp * sa);
    const bool s16 = L.tin == DT_BF16 || L.tin == DT_F16;
    L.o_Qh = take(s16 ? (size_t)L.mP * L.lp * 2 : 0);
    L.o_Ql = take(s16 ? (size_t)L.mP * L.lp * 2 : 0);
    L.o_Zp = take((size_t)L.nsplit * L.nP * L.lp * 8);
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
    L.total = off;
    return L;
}

}  // namespace

struct rpod_plan_s {
    rpod_desc d;
    Layout L;
    char* ws;
    hipStream_t st;
    // per-pass event timing (measurement only)
    bool timing = false;
    std::vector<hipEvent_t> ev[2];  // start/stop pairs, reused across resets
    size_t used[2] = {0, 0};
    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

// Record the start (begin=true) or stop event of one pass over S.
hipError_t mark(rpod_plan_s* P, int kind, bool begin) {
    if (!P->timing) return hipSuccess;
    std::vector<hipEvent_t>& v = P->ev[kind];
    const size_t idx = begin ? 2 * P->used[kind] : 2 * P->used[kind] + 1;
    if (idx >= v.size()) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        v.push_back(e);
    }
    hipError_t err = hipEventRecord(v[idx], P->st);
    if (!begin) ++P->used[kind];
    return err;
}

}  // namespace

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(RPOD_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

namespace {

// CholeskyQR2 of a tall matrix In (rows M, leading dim ld, type dt) into Out:
// Out = In R1^-1 is written, the final factor R2^-1 (or R3^-1 after the
// shifted retry) is left in R64[k]/R32[k] so that Q = Out R^-1 implicitly.
// If the first Cholesky needed a shift, a third pass Out <- Out R2^-1 runs
// (shifted CholeskyQR3, Fukaya et al., SISC 2020).
rpod_status orth(const rpod_plan_s* P, int dt, const void* In, void* Out, int64_t ld, int64_t M, int kfin) {
    const Layout& L = P->L;
    int* flags = P->at<int>(L.o_flags);
    int* local = flags + 1;
    double* Gp = P->at<double>(L.o_Gpart);
    double* G = P->at<double>(L.o_G);
    double* R64a = P->at<double>(L.o_R64[0]);
    float* R32a = P->at<float>(L.o_R32[0]);
    double* R64f = P->at<double>(L.o_R64[kfin]);
    float* R32f = P->at<float>(L.o_R32[kfin]);
    const void* Ra = dt == DT_F64 ? (const void*)R64a : (const void*)R32a;
    const void* Rf = dt == DT_F64 ? (const void*)R64f : (const void*)R32f;
    HIP_TRY(launch_gram(dt, L.nt, In, ld, M, Gp, G, nullptr, 0, P->st));
    HIP_TRY(launch_chol_inv(G, L.l, L.lp, M, R64a, R32a, flags, local, 0, P->st));
    HIP_TRY(launch_sx(dt, dt, L.nt, In, ld, M, L.lp, Ra, L.lp, Out, ld, ld, nullptr, 0, P->st, true));
    HIP_TRY(launch_gram(dt, L.nt, Out, ld, M, Gp, G, nullptr, 0, P->st));
    HIP_TRY(launch_chol_inv(G, L.l, L.lp, M, R64f, R32f, flags, local, 1, P->st));
    // shifted retry: Out <- Out R^-1 in place, then re-factor (no-ops unless flagged)
    HIP_TRY(launch_sx(dt, dt, L.nt, Out, ld, M, L.lp, Rf, L.lp, Out, ld, ld, local, 0x1, P->st, true));
    HIP_TRY(launch_gram(dt, L.nt, Out, ld, M, Gp, G, local, 0x1, P->st));
    HIP_TRY(launch_chol_inv(G, L.l, L.lp, M, R64f, R32f, flags, local, 2, P->st));
    return RPOD_OK;
}

// Basis of the n x l iterate Zw (FP64) for the next product with S, written
// to X in the S type: one CholeskyQR, X = Zw R^-1 (only the span matters
// here; the orthonormality that the method needs is restored by the
// CholeskyQR2 of the next S X). After a shifted factorisation a second
// CholeskyQR step runs (no-ops otherwise).
rpod_status basis_small(const rpod_plan_s* P, double* Zw, double* Zw2, void* X) {
    const Layout& L = P->L;
    int* flags = P->at<int>(L.o_flags);
    int* local = flags + 1;
    double* Gp = P->at<double>(L.o_Gpart);
    double* G = P->at<double>(L.o_G);
    double* Ra = P->at<double>(L.o_R64[0]);
    double* Rb = P->at<double>(L.o_R64[2]);
    hipStream_t st = P->st;
    HIP_TRY(launch_gram(DT_F64, L.nt, Zw, L.nP, P->d.n, Gp, G, nullptr, 0, st));
    HIP_TRY(launch_chol_inv(G, L.l, L.lp, P->d.n, Ra, P->at<float>(L.o_R32[0]), flags, local, 0, st));
    HIP_TRY(launch_sx(DT_F64, L.tin, L.nt, Zw, L.nP, P->d.n, L.lp, Ra, L.lp, X, L.nP, L.nP, nullptr, 0, st, true));
    // after a shift: Zw2 = Zw Ra^-1, refactor, X = Zw2 Rb^-1
    HIP_TRY(launch_sx(DT_F64, DT_F64, L.nt, Zw, L.nP, P->d.n, L.lp, Ra, L.lp, Zw2, L.nP, L.nP, local, 0x1, st, true));
    HIP_TRY(launch_gram(DT_F64, L.nt, Zw2, L.nP, P->d.n, Gp, G, local, 0x1, st));
    HIP_TRY(launch_chol_inv(G, L.l, L.lp, P->d.n, Rb, P->at<float>(L.o_R32[2]), flags, local, 2, st));
    HIP_TRY(launch_sx(DT_F64, L.tin, L.nt, Zw2, L.nP, P->d.n, L.lp, Rb, L.lp, X, L.nP, L.nP, local, 0x1, st, true));
    return RPOD_OK;
}

}  // namespace

extern "C" {

const char* rpod_last_error(void) { return g_err; }

rpod_status rpod_workspace_size(const rpod_desc* desc, size_t* bytes) {
    rpod_status s = validate(desc);
    if (s != RPOD_OK) return s;
    if (bytes == nullptr) return fail(RPOD_EINVAL, "bytes is NULL");
    *bytes = make_layout(desc).total;
    return RPOD_OK;
}

rpod_status rpod_plan_create(rpod_plan* plan, const rpod_desc* desc, void* workspace, size_t workspace_bytes,
                             void* hip_stream) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    *plan = nullptr;
    rpod_status s = validate(desc);
    if (s != RPOD_OK) return s;
    if (workspace == nullptr) return fail(RPOD_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % 256 != 0) return fail(RPOD_EINVAL, "workspace must be 256-byte aligned");
    Layout L = make_layout(desc);
    if (workspace_bytes < L.total)
        return fail(RPOD_ENOMEM, "workspace has %zu bytes, %zu needed", workspace_bytes, L.total);
    rpod_plan_s* P = new (std::nothrow) rpod_plan_s;
    if (P == nullptr) return fail(RPOD_ENOMEM, "host allocation of the plan failed");
    P->d = *desc;
    P->L = L;
    P->ws = static_cast<char*>(workspace);
    P->st = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipMemsetAsync(workspace, 0, L.total, P->st);
    if (e != hipSuccess) {
        delete P;
        return fail(RPOD_EHIP, "clearing the workspace failed: %s", hipGetErrorString(e));
    }
    *plan = P;
    return RPOD_OK;
}

rpod_status rpod_plan_destroy(rpod_plan plan) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    hipError_t e = hipStreamSynchronize(plan->st);
    for (int k = 0; k < 2; ++k)
        for (hipEvent_t ev : plan->ev[k]) (void)hipEventDestroy(ev);
    delete plan;
    if (e != hipSuccess) return fail(RPOD_EHIP, "stream synchronisation failed: %s", hipGetErrorString(e));
    return RPOD_OK;
}

rpod_status rpod_compute(rpod_plan plan, const void* S, uint64_t seed, void* Phi, double* sigma, void* A) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    if (S == nullptr || Phi == nullptr || sigma == nullptr || A == nullptr)
        return fail(RPOD_EINVAL, "S, Phi, sigma and A must be non-NULL");
    rpod_plan_s* P = plan;
    const Layout& L = P->L;
    const rpod_desc& d = P->d;
    if ((uintptr_t)S % dt_size(L.tin) != 0) return fail(RPOD_EINVAL, "S is not aligned to its element size");
    const size_t so = dt_size(L.tacc);
    if ((uintptr_t)Phi % so || (uintptr_t)A % so || (uintptr_t)sigma % 8)
        return fail(RPOD_EINVAL, "Phi, A or sigma is not aligned to its element size");
    hipStream_t st = P->st;
    int* flags = P->at<int>(L.o_flags);
    void* X = P->at<void>(L.o_X);
    void* Y = P->at<void>(L.o_Y);
    void* Q1 = P->at<void>(L.o_Q1);
    double* Zp = P->at<double>(L.o_Zp);
    double* Zt = P->at<double>(L.o_Zt);
    double* Zw = P->at<double>(L.o_Zw);
    double* Zw2 = P->at<double>(L.o_Zw2);
    double* R64t = P->at<double>(L.o_R64[1]);   // final factor of the tall orthonormalisation
    const int64_t m = d.m, n = d.n;
    const int lp = L.lp, nt = L.nt;

    HIP_TRY(launch_zero_ints(flags, 64, st));
    const bool s16 = L.tin == DT_BF16 || L.tin == DT_F16;
    // one pass Y = S X over S
    auto pass_sx = [&]() -> rpod_status {
        HIP_TRY(mark(P, 0, true));
        if (s16)
            HIP_TRY(launch_sx16(L.tin, nt, S, d.ld, m, n, X, L.nP, static_cast<float*>(Y), L.mP, L.mP, st));
        else
            HIP_TRY(launch_sx(L.tin, L.tacc, nt, S, d.ld, m, n, X, L.nP, Y, L.mP, L.mP, nullptr, 0, st));
        HIP_TRY(mark(P, 0, false));
        return RPOD_OK;
    };
    // one pass Z~ = S^T Q1 over S (lo: Q1 with ~16 significant bits on 16-bit paths)
    auto pass_stq = [&](bool lo) -> rpod_status {
        HIP_TRY(mark(P, 1, true));
        if (s16)
            HIP_TRY(launch_stq16(L.tin, nt, lo, S, d.ld, m, n, P->at<unsigned short>(L.o_Qh),
                                 P->at<unsigned short>(L.o_Ql), L.mP, Zp, L.nP, L.split_rows, L.nsplit, st));
        else
            HIP_TRY(launch_stq(L.tin, nt, S, d.ld, m, n, Q1, L.mP, Zp, L.nP, L.split_rows, L.nsplit, st));
        HIP_TRY(mark(P, 1, false));
        HIP_TRY(launch_reduce_slabs(Zp, L.nsplit, L.nP * lp, Zt, st));
        return RPOD_OK;
    };
    // CholeskyQR2 of Y into Q1; on 16-bit paths also the hi/lo parts of Q1
    auto orth_tall = [&]() -> rpod_status {
        rpod_status so = orth(P, L.tacc, Y, Q1, L.mP, m, 1);
        if (so != RPOD_OK) return so;
        if (s16)
            HIP_TRY(launch_split16(L.tin, static_cast<const float*>(Q1), L.mP * lp, P->at<unsigned short>(L.o_Qh),
                                   P->at<unsigned short>(L.o_Ql), st));
        return RPOD_OK;
    };
    rpod_status s;
    // Alg. 1 step 1: Gaussian sketch
    HIP_TRY(launch_omega(L.tin, seed, n, L.l, lp, L.nP, X, L.nP, st));
    // step 2: Y = S Omega, then Q by CholeskyQR2
    if ((s = pass_sx()) != RPOD_OK) return s;
    if ((s = orth_tall()) != RPOD_OK) return s;
    // step 3, one product at a time with re-orthonormalisation
    for (int it = 0; it < d.q; ++it) {
        if ((s = pass_stq(false)) != RPOD_OK) return s;
        HIP_TRY(launch_sx(DT_F64, DT_F64, nt, Zt, L.nP, n, lp, R64t, lp, Zw, L.nP, L.nP, nullptr, 0, st, true));
        if ((s = basis_small(P, Zw, Zw2, X)) != RPOD_OK) return s;
        if ((s = pass_sx()) != RPOD_OK) return s;
        if ((s = orth_tall()) != RPOD_OK) return s;
    }
    // step 5: T^T = S^T Q (Q = Q1 R^-1 applied on the small side); on 16-bit
    // paths this is the refinement pass with Q carried to ~16 bits
    if ((s = pass_stq(true)) != RPOD_OK) return s;
    HIP_TRY(launch_sx(DT_F64, DT_F64, nt, Zt, L.nP, n, lp, R64t, lp, Zw, L.nP, L.nP, nullptr, 0, st, true));
    // step 6: SVD of T through the eigenvectors of T T^T
    double* G = P->at<double>(L.o_G);
    double* UB = P->at<double>(L.o_UB);
    double* sig = P->at<double>(L.o_sig);
    HIP_TRY(launch_gram(DT_F64, nt, Zw, L.nP, n, P->at<double>(L.o_Gpart), G, nullptr, 0, st));
    // rotation threshold: FP64 rounding level on the FP64 path; elsewhere far
    // below the FP32 storage error of Q, which bounds the result anyway
    const double jtol = L.tacc == DT_F64 ? (double)lp * 0x1.0p-53 : 1e-10;
    HIP_TRY(launch_jacobi(G, L.l, lp, UB, sig, flags, jtol, st));
    // step 7: Phi = Q U_hat[:, :r] = Q1 (R^-1 U_hat[:, :r]); coefficients A = U_hat_r^T T
    double* M64 = P->at<double>(L.o_M64);
    float* M32 = P->at<float>(L.o_M32);
    double* Ur = P->at<double>(L.o_Ur);
    HIP_TRY(launch_lift_coef(R64t, UB, lp, d.r, L.rp, M64, M32, Ur, st));
    void* Phi_int = P->at<void>(L.o_Phi);
    const void* Mx = L.tacc == DT_F64 ? (const void*)M64 : (const void*)M32;
    HIP_TRY(launch_sx(L.tacc, L.tacc, L.ntr, Q1, L.mP, m, lp, Mx, lp, Phi_int, L.mP, L.mP, nullptr, 0, st));
    double* At = P->at<double>(L.o_At);
    HIP_TRY(launch_sx(DT_F64, DT_F64, L.ntr, Zw, L.nP, n, lp, Ur, lp, At, L.nP, L.nP, nullptr, 0, st));
    double* signs = P->at<double>(L.o_signs);
    HIP_TRY(launch_signs(L.tacc, Phi_int, L.mP, m, d.r, L.nchunk, P->at<double>(L.o_pval),
                         P->at<int64_t>(L.o_pidx), signs, st));
    HIP_TRY(launch_finalize(L.tacc, Phi_int, L.mP, m, d.r, At, L.nP, n, signs, sig, Phi, A, sigma, st));
    return RPOD_OK;
}

rpod_status rpod_status_query(rpod_plan plan, int32_t* device_flags) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    int host_flags = 0;
    hipError_t e = hipMemcpyAsync(&host_flags, plan->at<int>(plan->L.o_flags), sizeof(int), hipMemcpyDeviceToHost,
                                  plan->st);
    if (e == hipSuccess) e = hipStreamSynchronize(plan->st);
    if (e != hipSuccess) return fail(RPOD_EHIP, "reading the status word failed: %s", hipGetErrorString(e));
    if (device_flags) *device_flags = host_flags;
    if (host_flags & RPOD_FLAG_NONFINITE) return fail(RPOD_EINVAL_DATA, "non-finite values in S");
    if (host_flags & RPOD_FLAG_BREAKDOWN)
        return fail(RPOD_EBREAKDOWN, "sketch rank-deficient after the shifted CholeskyQR retry");
    return RPOD_OK;
}

rpod_status rpod_plan_set_timing(rpod_plan plan, int32_t enable) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    plan->timing = enable != 0;
    plan->used[0] = plan->used[1] = 0;
    return RPOD_OK;
}

rpod_status rpod_plan_get_timing(rpod_plan plan, int32_t pass, int64_t* launches, double* total_ms,
                                 double* bytes_per_launch, double* flops_per_launch) {
    if (plan == nullptr) return fail(RPOD_EINVAL, "plan is NULL");
    if (pass < 0 || pass > 1) return fail(RPOD_EINVAL, "pass must be 0 or 1");
    HIP_TRY(hipStreamSynchronize(plan->st));
    double tot = 0.0;
    for (size_t k = 0; k < plan->used[pass]; ++k) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, plan->ev[pass][2 * k], plan->ev[pass][2 * k + 1]));
        tot += ms;
    }
    const rpod_desc& d = plan->d;
    const double s = (double)dt_size(plan->L.tin), l = (double)plan->L.l;
    if (launches) *launches = (int64_t)plan->used[pass];
    if (total_ms) *total_ms = tot;
    if (bytes_per_launch) *bytes_per_launch = (double)d.m * d.n * s + (double)d.n * l * s + (double)d.m * l * 4.0;
    if (flops_per_launch) *flops_per_launch = 2.0 * d.m * d.n * l;
    return RPOD_OK;
}

rpod_status rpod_generate_omega(uint64_t seed, int64_t n, int32_t l, int32_t dtype, void* out, int64_t ldo,
                                void* hip_stream) {
    if (n < 1 || l < 1) return fail(RPOD_EINVAL, "n and l must be >= 1");
    if (ldo < n) return fail(RPOD_EINVAL, "ldo must be >= n");
    if (out == nullptr) return fail(RPOD_EINVAL, "out is NULL");
    if (dtype < RPOD_F64 || dtype > RPOD_F16) return fail(RPOD_EINVAL, "unknown dtype %d", dtype);
    const int dt = dtype;  // rpod_dtype and the internal codes coincide
    HIP_TRY(launch_omega(dt, seed, n, l, l, n, out, ldo, static_cast<hipStream_t>(hip_stream)));
    return RPOD_OK;
}

rpod_status rpod_sketch_bits(uint64_t seed, int64_t n, int32_t l, uint32_t* out, void* hip_stream) {
    if (n < 1 || l < 1) return fail(RPOD_EINVAL, "n and l must be >= 1");
    if (out == nullptr) return fail(RPOD_EINVAL, "out is NULL");
    HIP_TRY(launch_sketch_bits(seed, n, l, out, static_cast<hipStream_t>(hip_stream)));
    return RPOD_OK;
}

}  // extern "C"
