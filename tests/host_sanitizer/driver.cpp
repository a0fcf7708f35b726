// Drives the host side of the library through the C ABI with workspaces in
// host memory (see stubs.cpp): the autotuner over an uneven batch in every
// storage type (three calls each); single, batched, centred and adaptive
// plans created, computed twice and destroyed; a warm model with its bank and
// warm plans with and without the residual check. Exit status 0 when every
// call succeeds and every stream, event and graph was released.
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <vector>

#include "../../include/rpod.h"

int stub_report();

static void* host_ws(size_t bytes) { return aligned_alloc(256, (bytes + 255) / 256 * 256 + 256); }

static int run_plan(const rpod_desc* d, int count, const char* what) {
    size_t need = 0;
    if (rpod_workspace_size_batched(d, count, &need) != RPOD_OK) {
        printf("%s: workspace size failed: %s\n", what, rpod_last_error());
        return 1;
    }
    void* ws = host_ws(need);
    rpod_plan p = nullptr;
    int bad = rpod_plan_create_batched(&p, d, count, ws, need, nullptr) != RPOD_OK;
    std::vector<void*> S(count), Phi(count), A(count);
    std::vector<double*> sig(count);
    std::vector<uint64_t> seeds(count, 7);
    for (int i = 0; i < count && !bad; ++i) {
        S[i] = aligned_alloc(256, 256);   // never dereferenced on the host
        Phi[i] = aligned_alloc(256, 256);
        A[i] = aligned_alloc(256, 256);
        sig[i] = static_cast<double*>(aligned_alloc(256, 256));
    }
    for (int rep = 0; rep < 2 && !bad; ++rep)
        bad = rpod_compute_batched(p, S.data(), seeds.data(), Phi.data(), sig.data(), A.data()) != RPOD_OK;
    if (p) rpod_plan_destroy(p);
    for (int i = 0; i < count; ++i) {
        free(S[i]); free(Phi[i]); free(A[i]); free(sig[i]);
    }
    free(ws);
    printf("%s: %s%s\n", what, bad ? "FAILED " : "ok", bad ? rpod_last_error() : "");
    return bad;
}

int main() {
    int bad = 0;
    const long long shapes[3][4] = {{20000, 700, 25, 10}, {9000, 1200, 50, 10}, {30001, 500, 10, 10}};
    for (int dt : {2, 1, 3, 0}) {
        rpod_desc d[3];
        for (int i = 0; i < 3; ++i) {
            d[i] = rpod_desc{};
            d[i].m = shapes[i][0];
            d[i].n = shapes[i][1];
            d[i].ld = (shapes[i][0] + 7) / 8 * 8;
            d[i].dtype = dt;
            d[i].r = (int)shapes[i][2];
            d[i].p = (int)shapes[i][3];
            d[i].q = 2;
        }
        size_t need = 0;
        bad |= rpod_autotune_workspace_size(d, 3, &need) != RPOD_OK;
        void* ws = host_ws(need);
        std::vector<void*> S(3);
        for (int i = 0; i < 3; ++i) S[i] = aligned_alloc(256, 256);
        rpod_tuning best{};
        double ms = 0;
        for (int rep = 0; rep < 3; ++rep) {
            const rpod_status s = rpod_autotune(d, 3, (const void* const*)S.data(), ws, need, nullptr, 2, nullptr,
                                                &best, &ms);
            printf("dtype %d autotune %d: status %d best (%d, %d) %.3f\n", dt, rep, s, best.stq_workgroups,
                   best.gram_workgroups, ms);
            bad |= s != RPOD_OK;
        }
        for (int i = 0; i < 3; ++i) free(S[i]);
        free(ws);
        bad |= run_plan(d, 3, "batched plan");
        bad |= run_plan(d, 1, "single plan");
        rpod_desc c = d[1];
        c.block_cols = 100;   // 12 blocks of 100 snapshots
        bad |= run_plan(&c, 1, "centred plan");
        // adaptive: blocks of 16 up to 64 columns, one power step
        rpod_desc a = d[0];
        a.r = 64;
        a.p = 16;
        a.q = 1;
        size_t an = 0;
        bad |= rpod_workspace_size_adaptive(&a, 0.99, &an) != RPOD_OK;
        void* aws = host_ws(an);
        rpod_plan ap = nullptr;
        bad |= rpod_plan_create_adaptive(&ap, &a, 0.99, aws, an, nullptr) != RPOD_OK;
        void* buf = aligned_alloc(256, 256);
        int32_t lu = -1, rk = -1;
        double res = 0;
        for (int rep = 0; rep < 2 && ap; ++rep)
            bad |= rpod_compute_adaptive(ap, buf, 3, buf, static_cast<double*>(buf), buf, &lu, &rk, &res) != RPOD_OK;
        if (ap) rpod_plan_destroy(ap);
        free(buf);
        free(aws);
        printf("dtype %d adaptive plan: %s\n", dt, bad ? "FAILED" : "ok");
    }
    {   // warm model, bank and warm plans (checked with continuation, and unchecked)
        rpod_warm_desc wd{20001, 20, 16, 5};
        rpod_warm_layout wl{};
        bad |= rpod_warm_layout_of(&wd, &wl) != RPOD_OK;
        void* mws = host_ws(wl.total);
        rpod_warm model = nullptr;
        bad |= rpod_warm_create(&model, &wd, mws, wl.total, nullptr) != RPOD_OK;
        std::vector<float*> bank(8);
        for (auto& b : bank) b = static_cast<float*>(aligned_alloc(256, 256));
        bad |= model == nullptr || rpod_warm_set_bank(model, bank.data()) != RPOD_OK;
        for (double tol : {1e-3, std::numeric_limits<double>::infinity()}) {
            rpod_desc d{};
            d.m = 20001; d.n = 900; d.ld = 20008; d.dtype = 1; d.r = 20; d.p = 10; d.q = 1;
            size_t need = 0;
            bad |= rpod_workspace_size_warm(&d, model, 2, &need) != RPOD_OK;
            void* ws = host_ws(need);
            rpod_plan p = nullptr;
            bad |= rpod_plan_create_warm(&p, &d, model, 2, tol, ws, need, nullptr) != RPOD_OK;
            void* buf = aligned_alloc(256, 256);
            const float mu[4] = {0.1f, -0.2f, 0.3f, 0.0f};
            int32_t fb = -1;
            double rho = 0;
            for (int rep = 0; rep < 2 && p; ++rep)
                bad |= rpod_compute_warm(p, buf, mu, 11, buf, static_cast<double*>(buf), buf, &fb, &rho) != RPOD_OK;
            if (p) rpod_plan_destroy(p);
            free(buf);
            free(ws);
            printf("warm plan (tol %g): %s\n", tol, bad ? "FAILED" : "ok");
        }
        if (model) rpod_warm_destroy(model);
        for (auto& b : bank) free(b);
        free(mws);
    }
    bad |= stub_report();
    printf("%s\n", bad ? "FAILED" : "PASSED");
    return bad;
}
