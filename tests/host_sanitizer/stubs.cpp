// Host-only stand-ins for the HIP runtime calls and the kernel launchers that
// rpod_abi.cpp and warm_abi.cpp use, so that the plan recorder, the autotuner
// and the warm / adaptive bookkeeping run on a CPU under AddressSanitizer and
// UndefinedBehaviorSanitizer. Device memory is host memory here; no kernel
// runs. Every launcher checks that its launch record is well formed; the
// size helpers repeat the definitions in the kernel sources.
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../../paper_2504_15350_amd/csrc/internal.hpp"

static int g_streams = 0, g_events = 0, g_graphs = 0, g_execs = 0, g_bad = 0;

extern "C" {
hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t) { memset(p, v, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { memcpy(d, s, n); return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = (hipStream_t)malloc(64); ++g_streams; return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { free(s); --g_streams; return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t)malloc(64); ++g_events; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) { free(e); --g_events; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 1.0f + (float)(rand() % 100) * 0.01f; return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = (hipGraph_t)malloc(64); ++g_graphs; return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, hipGraphNode_t*, char*, size_t) {
    *e = (hipGraphExec_t)malloc(64); ++g_execs; return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) { free(g); --g_graphs; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { free(e); --g_execs; return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int) {
    memset(p, 0, sizeof(*p)); strcpy(p->gcnArchName, "gfx950"); p->multiProcessorCount = 256; return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "host stand-in"; }
hipError_t hipGetLastError(void) { return hipSuccess; }
}

int stub_report() {
    printf("[stubs] live streams %d events %d graphs %d execs %d, malformed launches %d\n", g_streams, g_events,
           g_graphs, g_execs, g_bad);
    return g_streams | g_events | g_graphs | g_execs | g_bad;
}

namespace rpod {
// size helpers (the same definitions as in the kernel sources)
constexpr int GRAM_WGS = 512;
constexpr int npairs_of(int nt) { return nt * (nt + 1) / 2; }
constexpr int gram_groups(int nt) { return nt <= 4 ? 1 : 3; }
int64_t gram_partial_count(int nt) { return (int64_t)GRAM_WGS * npairs_of(nt) * 256; }
int gram_nwg(int64_t M, int cap, int nt) {
    const int64_t nrb = (M + 15) / 16;
    int64_t nwg = (nrb + 3) / 4;
    if (cap < 1 || cap > GRAM_WGS) cap = gram_groups(nt) == 1 ? 256 : (GRAM_WGS / gram_groups(nt)) & ~7;
    if (nwg > cap) nwg = cap;
    if (nwg < 1) nwg = 1;
    return (int)nwg;
}
int gram_tiles(int nt, int nwg) { return nwg * gram_groups(nt); }
int gram_reduce_tiles(int nt) { return npairs_of(nt) * 8; }
int fin_phi_tiles(int64_t m, int r, int tphi) {
    const int64_t span = 256 * (tphi == DT_F64 ? 2 : 4);
    return (int)((m + span - 1) / span) * r;
}
int fin_a_tiles(int64_t n, int r) { return (int)(((n * r > r ? n * r : r) + 255) / 256); }
int stq16_block_cols(bool lo) { return (lo ? 2 : 1) * 128; }
int stq16_rows_per_step(bool lo) { return lo ? 64 : 128; }
int stq_e6_block_cols() { return 256; }
int stq32_block_cols() { return 128; }
int jacobi_threads(int lp) { return 4 * lp; }

// a launch record must name at least one matrix, a non-negative grid and, for
// grouped launches, a tile table whose last entry is the grid
template <typename A>
static hipError_t chk(const GroupLaunch<A>& L) {
    const bool ok = L.count > 0 && L.tiles >= 0 && L.args != nullptr && L.tstart != nullptr &&
                    L.tstart[0] == 0 && L.tstart[L.count] == L.tiles;
    if (!ok) ++g_bad;
    return ok ? hipSuccess : hipErrorInvalidValue;
}
static double g_scratch[RECON_NOALLOC_DOUBLES];

hipError_t launch_sx(int, int, int, bool, bool, const GroupLaunch<SxArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_sx_wide(int, int, bool, const GroupLaunch<SxArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_stq(int, int, bool, const GroupLaunch<StqArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_sx16(int, int, bool, const GroupLaunch<SxArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_stq16(int, int, bool, bool, const GroupLaunch<StqArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_split16(int, const GroupLaunch<SplitArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_sx_e6(int, bool, bool, bool, const GroupLaunch<SxArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_stq_e6(int, bool, const GroupLaunch<StqArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_reduce_slabs(const GroupLaunch<ReduceArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_center_prep(int, const GroupLaunch<CprepArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_center_y(int, const GroupLaunch<CenterYArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_center_cross(int, const GroupLaunch<CrossArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_center_sum(const GroupLaunch<CrossSumArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_center_z(const GroupLaunch<CenterZArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_frob(int, bool, bool, const GroupLaunch<FrobArgs>& P, const GroupLaunch<FrobArgs>& F, hipStream_t) {
    return chk(P) == hipSuccess ? chk(F) : hipErrorInvalidValue;
}
hipError_t launch_gram(int, int, const GroupLaunch<GramArgs>& L, const GroupLaunch<GramArgs>& R, hipStream_t) {
    return chk(L) == hipSuccess ? chk(R) : hipErrorInvalidValue;
}
hipError_t launch_chol_inv(int, const GroupLaunch<CholArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_jacobi(int, const GroupLaunch<JacobiArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_lift_coef(const GroupLaunch<LiftArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_signs(int, const GroupLaunch<ColmaxArgs>& C, const GroupLaunch<SignArgs>& S, hipStream_t) {
    return chk(C) == hipSuccess ? chk(S) : hipErrorInvalidValue;
}
hipError_t launch_finalize(int, const GroupLaunch<FinArgs>& P, const GroupLaunch<FinArgs>& A, hipStream_t) {
    return chk(P) == hipSuccess ? chk(A) : hipErrorInvalidValue;
}
hipError_t launch_omega(int, const GroupLaunch<OmegaArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_omega_direct(int, uint64_t, int64_t, int, void*, int64_t, hipStream_t) { return hipSuccess; }
hipError_t launch_sketch_bits(uint64_t, int64_t, int, uint32_t*, hipStream_t) { return hipSuccess; }
hipError_t launch_zero_ints(const GroupLaunch<ZeroArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_eye(const GroupLaunch<EyeArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_adapt_decide(const GroupLaunch<AdaptDecideArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_adapt_rank(const GroupLaunch<AdaptRankArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_set_calls(CallDesc*, const CallDesc*, int, hipStream_t) { return hipSuccess; }
hipError_t launch_warm_plan_forward(const GroupLaunch<WarmFwdArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_warm_z(const GroupLaunch<WarmZArgs>& L, hipStream_t) { return chk(L); }
hipError_t launch_warm_mode_res(const GroupLaunch<ModeResArgs>& P, const GroupLaunch<ModeResFinalArgs>& F,
                                hipStream_t) {
    return chk(P) == hipSuccess ? chk(F) : hipErrorInvalidValue;
}
hipError_t recon_scratch(double** ptr) { *ptr = g_scratch; return hipSuccess; }
hipError_t launch_reconstruct(int, int64_t, int, int64_t, const void*, const void*, const void*, void*, const void*,
                              int64_t, double*, double*, double*, hipStream_t) { return hipSuccess; }
hipError_t launch_reconstruct_mfma(int64_t, int, int64_t, const float*, const float*, const float*, float*, float*,
                                   int64_t, float*, int, SxArgs*, int*, hipStream_t) { return hipSuccess; }
hipError_t launch_warm_init(float*, uint64_t, hipStream_t) { return hipSuccess; }
hipError_t launch_warm_forward_batch(const float*, const float*, int, float*, float*, float*, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_warm_loss(const float*, const double*, const double*, int, int, float*, double*, float*,
                            hipStream_t) { return hipSuccess; }
hipError_t launch_warm_backward(const float*, const float*, int, const float*, const float*, const float*, float*,
                                float*, float*, hipStream_t) { return hipSuccess; }
hipError_t launch_warm_adam(float*, const float*, float*, float*, float, float, float, float, float, float, float,
                            hipStream_t) { return hipSuccess; }
hipError_t launch_copy_pad(float*, int64_t, const float*, int64_t, int64_t, int64_t, int, int, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_gather_cols(double*, int, int, int, const double*, int64_t, hipStream_t) { return hipSuccess; }
hipError_t launch_block_sumsq(const double*, int64_t, int64_t, int, int, int, double*, hipStream_t) {
    return hipSuccess;
}
}  // namespace rpod
