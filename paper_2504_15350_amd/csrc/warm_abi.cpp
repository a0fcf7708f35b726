// C ABI of the learned warm-start model: workspace layout, bank Grams,
// targets, training and prediction (every step in the library's kernels).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"
#include "warm_model.hpp"

using namespace rpod;

// error reporting lives with the rest of the ABI
rpod_status rpod_internal_fail(rpod_status s, const char* fmt, ...);

namespace {

int64_t rup(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

#define WFAIL(st, ...) rpod_internal_fail(st, __VA_ARGS__)
#define WHIP(expr)                                                                                     \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return WFAIL(RPOD_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

rpod_status check_desc(const rpod_warm_desc* d) {
    if (d == nullptr) return WFAIL(RPOD_EINVAL, "warm desc is NULL");
    if (d->m < 1) return WFAIL(RPOD_EINVAL, "warm model: m must be >= 1");
    if (d->r < 1 || d->r > 128) return WFAIL(RPOD_EINVAL, "warm model: r must be in [1, 128] (got %d)", d->r);
    if (d->r > d->m) return WFAIL(RPOD_EINVAL, "warm model: r must be <= m");
    if (d->max_train < 1 || d->max_train > 4096)
        return WFAIL(RPOD_EINVAL, "warm model: max_train must be in [1, 4096] (got %d)", d->max_train);
    return RPOD_OK;
}

// Fill the geometry and the layout of a model.
void geometry(rpod_warm_s& M) {
    const rpod_warm_desc& d = M.d;
    M.mP = rup(d.m, 256);
    M.Kr = WARM_K * d.r;
    M.bank_cols = (int)rup(M.Kr, 128);
    M.nPb = rup(M.Kr, 256);
    M.rpad = (int)rup(d.r, 16);
    // bank^T products use the FP32 split-K kernel: 128-column blocks, splits
    // interleaved in steps of 64 rows
    const int64_t ncb = M.nPb / stq32_block_cols();
    int64_t ns = (2048 + ncb - 1) / ncb;
    ns = std::min<int64_t>(ns, 64);
    ns = std::min<int64_t>(ns, (d.m + 63) / 64);
    ns = std::max<int64_t>(ns, 1);
    M.split_rows = rup((d.m + ns - 1) / ns, 64);
    M.nsplit = (int)ns;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t np = (size_t)WP_COUNT * 4;
    const size_t N = (size_t)d.max_train;
    M.L.params = take(np);
    M.L.grads = take(np);
    M.L.adam_m = take(np);
    M.L.adam_v = take(np);
    M.o_H1 = take(N * WARM_H * 4);
    M.o_H2 = take(N * WARM_H * 4);
    M.o_dA1 = take(N * WARM_H * 4);
    M.o_dA2 = take(N * WARM_H * 4);
    M.o_C = take(N * WARM_K * 4);
    M.o_dZ = take(N * WARM_K * 4);
    M.o_lossn = take(N * 8);
    M.o_loss = take(8);
    M.L.bank = take((size_t)M.mP * M.bank_cols * 4);
    M.L.gram = take((size_t)M.Kr * M.Kr * 8);
    M.L.gram8 = take(WARM_K * WARM_K * 8);
    M.o_stage = take((size_t)M.mP * std::max(M.rpad, 128) * 4);
    M.o_Zp = take((size_t)M.nsplit * M.nPb * 128 * 8);
    M.o_Zt = take((size_t)M.nPb * 128 * 8);
    M.args_bytes = 16384;
    M.o_args = take(M.args_bytes);
    M.L.total = off;
}

// Upload one grouped S^T Q launch (+ its slab reduction) over the bank and
// run it: Zt (nPb x 16 nt, column-major) = bank^T Q.
rpod_status bank_product(rpod_warm_s& M, const float* Q, int nt) {
    StqArgs a{};
    a.S = M.at<float>(M.L.bank);
    a.ldS = M.mP;
    a.m = M.d.m;
    a.n = M.Kr;
    a.Q = Q;
    a.Ql = nullptr;
    a.ldQ = M.mP;
    a.Zp = M.at<double>(M.o_Zp);
    a.nP = M.nPb;
    a.split_rows = M.split_rows;
    a.nsplit = M.nsplit;
    a.ncb = (int)(M.nPb / stq32_block_cols());
    a.call = -1;
    ReduceArgs ra{M.at<double>(M.o_Zp), M.nPb * 16 * nt, M.at<double>(M.o_Zt), M.nsplit, 0};
    const int tiles = a.ncb * a.nsplit;
    const int rtiles = (int)((ra.count + 255) / 256);
    struct Blob {
        StqArgs a;
        int ts[2];
        int pad[2];
        ReduceArgs ra;
        int rts[2];
    } blob;
    std::memset(&blob, 0, sizeof(blob));
    blob.a = a;
    blob.ts[0] = 0;
    blob.ts[1] = tiles;
    blob.ra = ra;
    blob.rts[0] = 0;
    blob.rts[1] = rtiles;
    char* dev = M.ws + M.o_args;
    WHIP(hipMemcpyAsync(dev, &blob, sizeof(blob), hipMemcpyHostToDevice, M.st));
    GroupLaunch<StqArgs> gs{reinterpret_cast<const StqArgs*>(dev + offsetof(Blob, a)),
                            reinterpret_cast<const int*>(dev + offsetof(Blob, ts)), nullptr, 1, tiles};
    GroupLaunch<ReduceArgs> gr{reinterpret_cast<const ReduceArgs*>(dev + offsetof(Blob, ra)),
                               reinterpret_cast<const int*>(dev + offsetof(Blob, rts)), nullptr, 1, rtiles};
    WHIP(launch_stq(DT_F32, nt, true, gs, M.st));
    WHIP(launch_reduce_slabs(gr, M.st));
    // the argument blob is reused by the next product: wait until this one ran
    WHIP(hipStreamSynchronize(M.st));
    return RPOD_OK;
}

}  // namespace

extern "C" {

rpod_status rpod_warm_layout_of(const rpod_warm_desc* desc, rpod_warm_layout* layout) {
    rpod_status s = check_desc(desc);
    if (s != RPOD_OK) return s;
    if (layout == nullptr) return WFAIL(RPOD_EINVAL, "layout is NULL");
    rpod_warm_s M;
    M.d = *desc;
    geometry(M);
    *layout = M.L;
    return RPOD_OK;
}

rpod_status rpod_warm_create(rpod_warm* model, const rpod_warm_desc* desc, void* workspace, size_t workspace_bytes,
                             void* hip_stream) {
    if (model == nullptr) return WFAIL(RPOD_EINVAL, "model is NULL");
    *model = nullptr;
    rpod_status s = check_desc(desc);
    if (s != RPOD_OK) return s;
    if (workspace == nullptr || (uintptr_t)workspace % 256 != 0)
        return WFAIL(RPOD_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    rpod_warm_s* M = new (std::nothrow) rpod_warm_s;
    if (M == nullptr) return WFAIL(RPOD_ENOMEM, "host allocation of the model failed");
    M->d = *desc;
    geometry(*M);
    if (workspace_bytes < M->L.total) {
        const size_t need = M->L.total;
        delete M;
        return WFAIL(RPOD_ENOMEM, "workspace has %zu bytes, %zu needed", workspace_bytes, need);
    }
    M->ws = static_cast<char*>(workspace);
    M->st = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipMemsetAsync(workspace, 0, M->L.total, M->st);
    if (e == hipSuccess) e = launch_warm_init(M->at<float>(M->L.params), desc->seed, M->st);
    if (e != hipSuccess) {
        delete M;
        return WFAIL(RPOD_EHIP, "initialising the model failed: %s", hipGetErrorString(e));
    }
    *model = M;
    return RPOD_OK;
}

rpod_status rpod_warm_destroy(rpod_warm model) {
    if (model == nullptr) return WFAIL(RPOD_EINVAL, "model is NULL");
    hipError_t e = hipStreamSynchronize(model->st);
    delete model;
    if (e != hipSuccess) return WFAIL(RPOD_EHIP, "stream synchronisation failed: %s", hipGetErrorString(e));
    return RPOD_OK;
}

rpod_status rpod_warm_set_bank(rpod_warm M, const float* const* bases) {
    if (M == nullptr || bases == nullptr) return WFAIL(RPOD_EINVAL, "model and bases must be non-NULL");
    for (int k = 0; k < WARM_K; ++k)
        if (bases[k] == nullptr) return WFAIL(RPOD_EINVAL, "bank basis %d is NULL", k);
    const int r = M->d.r;
    float* bank = M->at<float>(M->L.bank);
    for (int k = 0; k < WARM_K; ++k)
        WHIP(launch_copy_pad(bank + (int64_t)k * r * M->mP, M->mP, bases[k], M->d.m, M->d.m, M->mP, r, r, M->st));
    double* G = M->at<double>(M->L.gram);
    for (int c0 = 0; c0 < M->Kr; c0 += 128) {
        rpod_status s = bank_product(*M, bank + (int64_t)c0 * M->mP, 8);
        if (s != RPOD_OK) return s;
        WHIP(launch_gather_cols(G, M->Kr, c0, std::min(128, M->Kr - c0), M->at<double>(M->o_Zt), M->nPb, M->st));
        WHIP(hipStreamSynchronize(M->st));  // Zt is reused by the next chunk
    }
    WHIP(launch_block_sumsq(G, M->Kr, 1, r, WARM_K, WARM_K, M->at<double>(M->L.gram8), M->st));
    WHIP(hipStreamSynchronize(M->st));
    return RPOD_OK;
}

rpod_status rpod_warm_targets(rpod_warm M, const float* basis, double* b) {
    if (M == nullptr || basis == nullptr || b == nullptr) return WFAIL(RPOD_EINVAL, "model, basis and b must be non-NULL");
    const int r = M->d.r;
    float* stage = M->at<float>(M->o_stage);
    WHIP(launch_copy_pad(stage, M->mP, basis, M->d.m, M->d.m, M->mP, r, M->rpad, M->st));
    rpod_status s = bank_product(*M, stage, M->rpad / 16);
    if (s != RPOD_OK) return s;
    WHIP(launch_block_sumsq(M->at<double>(M->o_Zt), 1, M->nPb, r, WARM_K, 1, b, M->st));
    WHIP(hipStreamSynchronize(M->st));
    return RPOD_OK;
}

rpod_status rpod_warm_loss_grad(rpod_warm M, const float* mu, const double* b, int32_t N, float* loss) {
    if (M == nullptr || mu == nullptr || b == nullptr) return WFAIL(RPOD_EINVAL, "model, mu and b must be non-NULL");
    if (N < 1 || N > M->d.max_train) return WFAIL(RPOD_EINVAL, "N must be in [1, max_train] (got %d)", N);
    const float* P = M->at<float>(M->L.params);
    float* H1 = M->at<float>(M->o_H1);
    float* H2 = M->at<float>(M->o_H2);
    float* C = M->at<float>(M->o_C);
    float* dZ = M->at<float>(M->o_dZ);
    WHIP(launch_warm_forward_batch(P, mu, N, H1, H2, C, M->st));
    WHIP(launch_warm_loss(C, b, M->at<double>(M->L.gram8), N, M->d.r, dZ, M->at<double>(M->o_lossn),
                          loss ? loss : M->at<float>(M->o_loss), M->st));
    WHIP(launch_warm_backward(P, mu, N, H1, H2, dZ, M->at<float>(M->o_dA2), M->at<float>(M->o_dA1),
                              M->at<float>(M->L.grads), M->st));
    return RPOD_OK;
}

rpod_status rpod_warm_train(rpod_warm M, const float* mu, const double* b, int32_t N, int32_t epochs, float lr,
                            float beta1, float beta2, float eps, float weight_decay, float* losses) {
    if (M == nullptr) return WFAIL(RPOD_EINVAL, "model is NULL");
    if (epochs < 0) return WFAIL(RPOD_EINVAL, "epochs must be >= 0");
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) ||
        !(weight_decay >= 0.f))
        return WFAIL(RPOD_EINVAL, "Adam hyperparameters out of range");
    for (int32_t e = 0; e < epochs; ++e) {
        rpod_status s = rpod_warm_loss_grad(M, mu, b, N, losses ? losses + e : nullptr);
        if (s != RPOD_OK) return s;
        M->adam_t += 1;
        const double bc1 = 1.0 - std::pow((double)beta1, (double)M->adam_t);
        const double bc2 = 1.0 - std::pow((double)beta2, (double)M->adam_t);
        WHIP(launch_warm_adam(M->at<float>(M->L.params), M->at<float>(M->L.grads), M->at<float>(M->L.adam_m),
                              M->at<float>(M->L.adam_v), lr, beta1, beta2, eps, weight_decay, (float)bc1, (float)bc2,
                              M->st));
    }
    return RPOD_OK;
}

rpod_status rpod_warm_predict(rpod_warm M, const float* mu, int32_t N, float* c) {
    if (M == nullptr || mu == nullptr || c == nullptr) return WFAIL(RPOD_EINVAL, "model, mu and c must be non-NULL");
    if (N < 1 || N > M->d.max_train) return WFAIL(RPOD_EINVAL, "N must be in [1, max_train] (got %d)", N);
    WHIP(launch_warm_forward_batch(M->at<float>(M->L.params), mu, N, M->at<float>(M->o_H1), M->at<float>(M->o_H2), c,
                                   M->st));
    return RPOD_OK;
}

}  // extern "C"
