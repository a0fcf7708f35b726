// Learned warm start: the parameter network (forward, loss, backward, Adam),
// the bank's Gram helpers, the predicted subspace and the residual of the
// returned modes.
//
// Network: c = softmax(W3 tanh(W2 tanh(W1 mu + b1) + b2) + b3), FP32. Every
// hidden unit is one thread's dot product in a fixed order and every logit
// a fixed-order tree over 32 partial sums, the same code for training
// batches and for the single parameter vector of a plan, so both give the
// same weights bit for bit.
#include "device_common.hpp"
#include "internal.hpp"

namespace rpod {

template <typename A>
static Group<A> mkw(const GroupLaunch<A>& L) {
    Group<A> g;
    g.args = L.args;
    g.tstart = L.tstart;
    g.calls = L.calls;
    g.count = L.count;
    g.skip = L.skip;
    g.skip_mask = L.skip_mask;
    return g;
}

// ---------------------------------------------------------------------------
// forward pieces (one sample per 256-thread workgroup)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float unit1(const GLOBAL float* P, const float* x, int j) {
    float a = P[WP_B1 + j];
#pragma unroll
    for (int i = 0; i < WARM_IN; ++i) a = fmaf(P[WP_W1 + j * WARM_IN + i], x[i], a);
    return tanhf(a);
}

__device__ __forceinline__ float unit2(const GLOBAL float* P, const float* h1, int j) {
    float a = P[WP_B2 + j];
    for (int i = 0; i < WARM_H; ++i) a = fmaf(P[WP_W2 + j * WARM_H + i], h1[i], a);
    return tanhf(a);
}

// z[k] (LDS) for k < WARM_K: 32 threads per logit, fixed-order tree; red: 256 floats of LDS.
__device__ __forceinline__ void logits(const GLOBAL float* P, const float* h2, float* z, float* red) {
    const int t = threadIdx.x, k = t >> 5, l = t & 31;
    float a = 0.f;
    for (int i = l; i < WARM_H; i += 32) a = fmaf(P[WP_W3 + k * WARM_H + i], h2[i], a);
    red[t] = a;
    __syncthreads();
    for (int off = 16; off > 0; off >>= 1) {
        if (l < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (l == 0) z[k] = red[t] + P[WP_B3 + k];
    __syncthreads();
}

// softmax of z (thread 0), written to c; returns the argmax (lowest index on ties)
__device__ __forceinline__ int softmax8(const float* z, float* c) {
    float zm = z[0];
    for (int k = 1; k < WARM_K; ++k) zm = fmaxf(zm, z[k]);
    float e[WARM_K], s = 0.f;
    for (int k = 0; k < WARM_K; ++k) {
        e[k] = expf(z[k] - zm);
        s += e[k];
    }
    int best = 0;
    for (int k = 0; k < WARM_K; ++k) {
        c[k] = e[k] / s;
        if (c[k] > c[best]) best = k;
    }
    return best;
}

// ---------------------------------------------------------------------------
// initialisation
// ---------------------------------------------------------------------------
__global__ void k_warm_init(float* params, uint64_t seed) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= WP_COUNT) return;
    float a = 0.f;  // biases stay zero
    if (e < WP_B1) a = sqrtf(6.f / (WARM_IN + WARM_H));
    else if (e >= WP_W2 && e < WP_B2) a = sqrtf(6.f / (WARM_H + WARM_H));
    else if (e >= WP_W3 && e < WP_B3) a = sqrtf(6.f / (WARM_H + WARM_K));
    const philox_out o = philox4x32_10((uint32_t)e, 0u, 0u, 0x57A47u, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float u = (float)(o.x[0] >> 8) * 0x1.0p-24f;  // [0, 1)
    params[e] = a * (2.f * u - 1.f);
}

hipError_t launch_warm_init(float* params, uint64_t seed, hipStream_t st) {
    hipLaunchKernelGGL(k_warm_init, dim3((WP_COUNT + 255) / 256), dim3(256), 0, st, params, seed);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// training: forward, loss, backward, Adam
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_warm_fwd(const float* params, const float* mu, float* H1, float* H2,
                                                  float* C) {
    const GLOBAL float* P = gbl(params);
    const int n = blockIdx.x, j = threadIdx.x;
    __shared__ float x[WARM_IN], h1[WARM_H], h2[WARM_H], z[WARM_K], red[256];
    if (j < WARM_IN) x[j] = mu[n * WARM_IN + j];
    __syncthreads();
    h1[j] = unit1(P, x, j);
    H1[(int64_t)n * WARM_H + j] = h1[j];
    __syncthreads();
    h2[j] = unit2(P, h1, j);
    H2[(int64_t)n * WARM_H + j] = h2[j];
    __syncthreads();
    logits(P, h2, z, red);
    if (j == 0) {
        float c[WARM_K];
        softmax8(z, c);
        for (int k = 0; k < WARM_K; ++k) C[n * WARM_K + k] = c[k];
    }
}

hipError_t launch_warm_forward_batch(const float* params, const float* mu, int N, float* H1, float* H2, float* C,
                                     hipStream_t st) {
    hipLaunchKernelGGL(k_warm_fwd, dim3(N), dim3(256), 0, st, params, mu, H1, H2, C);
    return hipGetLastError();
}

// one thread per pair: loss_n and dL/dz of the mean loss
__global__ void k_warm_loss(const float* C, const double* B, const double* G8, int N, int r, float* dZ,
                            double* loss_n) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double c[WARM_K], dc[WARM_K];
    for (int k = 0; k < WARM_K; ++k) c[k] = (double)C[n * WARM_K + k];
    double L = (double)r, cdc = 0.0;
    for (int k = 0; k < WARM_K; ++k) {
        double gc = 0.0;
        for (int l = 0; l < WARM_K; ++l) gc += G8[k * WARM_K + l] * c[l];
        const double b = B[(int64_t)n * WARM_K + k];
        L += c[k] * gc - 2.0 * b * c[k];
        dc[k] = (2.0 / N) * (gc - b);
        cdc += c[k] * dc[k];
    }
    loss_n[n] = L;
    for (int k = 0; k < WARM_K; ++k) dZ[n * WARM_K + k] = (float)(c[k] * (dc[k] - cdc));
}

__global__ void k_warm_loss_mean(const double* loss_n, int N, float* loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int n = 0; n < N; ++n) s += loss_n[n];
    *loss = (float)(s / N);
}

hipError_t launch_warm_loss(const float* C, const double* B, const double* G8, int N, int r, float* dZ,
                            double* loss_n, float* loss, hipStream_t st) {
    hipLaunchKernelGGL(k_warm_loss, dim3((N + 63) / 64), dim3(64), 0, st, C, B, G8, N, r, dZ, loss_n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || loss == nullptr) return e;
    hipLaunchKernelGGL(k_warm_loss_mean, dim3(1), dim3(64), 0, st, loss_n, N, loss);
    return hipGetLastError();
}

// dA[n][i] = (sum_o dY[n][o] W[o][i]) (1 - H[n][i]^2), W: out x 256 row-major
__global__ __launch_bounds__(256) void k_warm_back_hidden(const float* dY, int out, const float* W, const float* H,
                                                          float* dA) {
    const int n = blockIdx.x, i = threadIdx.x;
    float s = 0.f;
    for (int o = 0; o < out; ++o) s = fmaf(dY[(int64_t)n * out + o], W[(int64_t)o * WARM_H + i], s);
    const float h = H[(int64_t)n * WARM_H + i];
    dA[(int64_t)n * WARM_H + i] = s * (1.f - h * h);
}

// dW[o][i] = sum_n dY[n][o] X[n][i] (e < out in), db[o] = sum_n dY[n][o] (next out elements)
__global__ void k_warm_wgrad(const float* dY, const float* X, int N, int out, int in, float* dW, float* db) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < out * in) {
        const int o = e / in, i = e % in;
        float s = 0.f;
        for (int n = 0; n < N; ++n) s = fmaf(dY[(int64_t)n * out + o], X[(int64_t)n * in + i], s);
        dW[e] = s;
    } else if (e < out * in + out) {
        const int o = e - out * in;
        float s = 0.f;
        for (int n = 0; n < N; ++n) s += dY[(int64_t)n * out + o];
        db[o] = s;
    }
}

hipError_t launch_warm_backward(const float* params, const float* mu, int N, const float* H1, const float* H2,
                                const float* dZ, float* dA2, float* dA1, float* grads, hipStream_t st) {
    hipLaunchKernelGGL(k_warm_wgrad, dim3((WARM_K * WARM_H + WARM_K + 255) / 256), dim3(256), 0, st, dZ, H2, N,
                       WARM_K, WARM_H, grads + WP_W3, grads + WP_B3);
    hipLaunchKernelGGL(k_warm_back_hidden, dim3(N), dim3(256), 0, st, dZ, WARM_K, params + WP_W3, H2, dA2);
    hipLaunchKernelGGL(k_warm_wgrad, dim3((WARM_H * WARM_H + WARM_H + 255) / 256), dim3(256), 0, st, dA2, H1, N,
                       WARM_H, WARM_H, grads + WP_W2, grads + WP_B2);
    hipLaunchKernelGGL(k_warm_back_hidden, dim3(N), dim3(256), 0, st, dA2, WARM_H, params + WP_W2, H1, dA1);
    hipLaunchKernelGGL(k_warm_wgrad, dim3((WARM_H * WARM_IN + WARM_H + 255) / 256), dim3(256), 0, st, dA1, mu, N,
                       WARM_H, WARM_IN, grads + WP_W1, grads + WP_B1);
    return hipGetLastError();
}

__global__ void k_warm_adam(float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                            float wd, float bc1, float bc2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= WP_COUNT) return;
    const float ge = g[e] + wd * p[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    p[e] -= lr * (me / bc1) / (sqrtf(ve / bc2) + eps);
}

hipError_t launch_warm_adam(float* params, const float* grads, float* m, float* v, float lr, float beta1,
                            float beta2, float eps, float wd, float bc1, float bc2, hipStream_t st) {
    hipLaunchKernelGGL(k_warm_adam, dim3((WP_COUNT + 255) / 256), dim3(256), 0, st, params, grads, m, v, lr, beta1,
                       beta2, eps, wd, bc1, bc2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// bank helpers
// ---------------------------------------------------------------------------
__global__ void k_copy_pad(float* dst, int64_t ldd, const float* src, int64_t lds, int64_t rows, int64_t rows_pad,
                           int cols, int cols_pad) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows_pad * cols_pad) return;
    const int64_t c = e / rows_pad, i = e % rows_pad;
    dst[c * ldd + i] = (c < cols && i < rows) ? src[c * lds + i] : 0.f;
}

hipError_t launch_copy_pad(float* dst, int64_t ldd, const float* src, int64_t lds, int64_t rows, int64_t rows_pad,
                           int cols, int cols_pad, hipStream_t st) {
    const int64_t total = rows_pad * cols_pad;
    hipLaunchKernelGGL(k_copy_pad, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, dst, ldd, src, lds, rows,
                       rows_pad, cols, cols_pad);
    return hipGetLastError();
}

__global__ void k_gather_cols(double* G, int Kr, int c0, int ncol, const double* Z, int64_t ldz) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)Kr * ncol) return;
    const int col = (int)(e / Kr), a = (int)(e % Kr);
    G[(int64_t)a * Kr + c0 + col] = Z[(int64_t)col * ldz + a];
}

hipError_t launch_gather_cols(double* G, int Kr, int c0, int ncol, const double* Z, int64_t ldz, hipStream_t st) {
    const int64_t total = (int64_t)Kr * ncol;
    hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, G, Kr, c0, ncol, Z,
                       ldz);
    return hipGetLastError();
}

// one workgroup per output block pair, fixed-order tree
__global__ __launch_bounds__(256) void k_block_sumsq(const double* src, int64_t sa, int64_t sb, int r, int KB,
                                                     double* out) {
    const int k = blockIdx.x / KB, l = blockIdx.x % KB;
    __shared__ double red[256];
    double s = 0.0;
    for (int e = threadIdx.x; e < r * r; e += 256) {
        const int a = k * r + e / r, b = l * r + e % r;
        const double v = src[(int64_t)a * sa + (int64_t)b * sb];
        s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

hipError_t launch_block_sumsq(const double* src, int64_t sa, int64_t sb, int r, int KA, int KB, double* out,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_block_sumsq, dim3(KA * KB), dim3(256), 0, st, src, sa, sb, r, KB, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// plan steps (grouped)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_warm_plan_fwd(Group<WarmFwdArgs> g) {
    if (group_skipped(g)) return;
    const WarmFwdArgs& a = g.args[blockIdx.x];  // one workgroup per matrix
    const GLOBAL float* P = gbl(a.params);
    const int j = threadIdx.x;
    __shared__ float x[WARM_IN], h1[WARM_H], h2[WARM_H], z[WARM_K], red[256];
    if (j < WARM_IN) x[j] = g.calls[a.call].mu[j];
    __syncthreads();
    h1[j] = unit1(P, x, j);
    __syncthreads();
    h2[j] = unit2(P, h1, j);
    __syncthreads();
    logits(P, h2, z, red);
    if (j == 0) {
        float c[WARM_K];
        const int best = softmax8(z, c);
        for (int k = 0; k < WARM_K; ++k) a.c[k] = (double)c[k];
        *a.kstar = best;
    }
}

hipError_t launch_warm_plan_forward(const GroupLaunch<WarmFwdArgs>& L, hipStream_t st) {
    hipLaunchKernelGGL(k_warm_plan_fwd, dim3(L.count), dim3(256), 0, st, mkw(L));
    return hipGetLastError();
}

// Z = (C G_W)^iters E_k* for iters <= 2, C = diag(c (x) 1_r), E_k* the
// columns of bank block k*. Tile (column i, rows 64 t .. 64 t + 63); four
// waves split the inner sum over the bank columns b and reduce in LDS:
//   iters 2: Z[e][i] = c_e sum_b G_W[e][b] c_b G_W[b][k* r + i]
// (G_W symmetric: read as G_W[b][e], coalesced over e).
__global__ __launch_bounds__(256) void k_warm_z(Group<WarmZArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const WarmZArgs& a = g.args[it];
    const int t = blockIdx.x - g.tstart[it];
    const int nrb = (int)((a.ldX + 63) / 64);
    const int i = t / nrb, rb = t % nrb;
    const int Kr = a.Kr, r = a.r;
    const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int64_t e = (int64_t)rb * 64 + lane;
    GLOBAL float* X = gbl(a.X) + (int64_t)i * a.ldX;
    const GLOBAL double* GW = gbl(a.GW);
    const int col = (*a.kstar) * r + i;
    __shared__ double red[256];
    double z = 0.0;
    if (i < r && e < Kr) {
        if (a.iters == 0) {
            z = (e == col) ? 1.0 : 0.0;
        } else if (a.iters == 1) {
            z = a.c[e / r] * GW[(int64_t)col * Kr + e];
        } else {
            double s = 0.0;
            const int b0 = part * ((Kr + 3) / 4), b1 = min(Kr, b0 + (Kr + 3) / 4);
            for (int b = b0; b < b1; ++b) s += GW[(int64_t)b * Kr + e] * (a.c[b / r] * GW[(int64_t)b * Kr + col]);
            red[threadIdx.x] = s;
        }
    }
    if (a.iters >= 2) {
        __syncthreads();
        if (part == 0 && i < r && e < Kr)
            z = a.c[e / r] * ((red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]));
    }
    if (part == 0 && e < a.ldX) X[e] = (float)z;
}

hipError_t launch_warm_z(const GroupLaunch<WarmZArgs>& L, hipStream_t st) {
    hipLaunchKernelGGL(k_warm_z, dim3(L.tiles), dim3(256), 0, st, mkw(L));
    return hipGetLastError();
}

// Residual of each returned singular triplet (sigma_k, phi_k, v_k), v_k =
// a_k / sigma_k with a_k the k-th coefficient row: S v_k - sigma_k phi_k =
// (S a_k - sigma_k^2 phi_k) / sigma_k, and Y = S A^T comes from an FP64
// product. Wave w of a workgroup takes the modes k = w mod 4; each lane sums
// the squares over rows lane, lane + 64, ... of the chunk, then a fixed
// butterfly over the wave. The error of sigma_k is at most sigma_k rho_k
// (the pair is an approximate eigenpair of the symmetric embedding
// [0 S; S^T 0] with residual norm sigma_k rho_k).
__global__ __launch_bounds__(256) void k_warm_mode_res(Group<ModeResArgs> g) {
    if (group_skipped(g)) return;
    const int it = group_item(g.tstart, g.count, blockIdx.x);
    const ModeResArgs& a = g.args[it];
    const int64_t i0 = (int64_t)(blockIdx.x - g.tstart[it]) * a.rows;
    const int64_t i1 = i0 + a.rows < a.m ? i0 + a.rows : a.m;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const GLOBAL double* Y = gbl(a.Y);
    const GLOBAL float* Phi = gbl(a.Phi);
    for (int k = wave; k < a.r; k += 4) {
        const double s2 = a.sig[k] * a.sig[k];
        double acc = 0.0;
        for (int64_t i = i0 + lane; i < i1; i += 64) {
            const double d = Y[(int64_t)k * a.ldY + i] - s2 * (double)Phi[(int64_t)k * a.ldP + i];
            acc = fma(d, d, acc);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) a.part[(int64_t)(blockIdx.x - g.tstart[it]) * a.r + k] = acc;
    }
}

__global__ __launch_bounds__(128) void k_warm_mode_final(Group<ModeResFinalArgs> g) {
    if (group_skipped(g)) return;
    const ModeResFinalArgs& a = g.args[blockIdx.x];  // one workgroup per matrix
    __shared__ double rk[WARM_MAXLP];
    const int k = threadIdx.x;
    if (k < a.r) {
        double s = 0.0;
        for (int c = 0; c < a.nchunk; ++c) s += a.part[(int64_t)c * a.r + k];
        const double sg = a.sig[k];
        rk[k] = sqrt(s) / (sg * sg);
        a.rho_modes[k] = rk[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = 0.0;
        bool bad = false;
        for (int c = 0; c < a.r; ++c) {
            bad = bad || !(rk[c] == rk[c]) || rk[c] > 1.0e308;
            mx = rk[c] > mx ? rk[c] : mx;
        }
        const double rho = bad ? __builtin_nan("") : mx;
        *a.rho = rho;
        const bool reject = !(rho <= a.tol);
        *a.decision = reject ? 1 : 0;
        if (reject) atomicOr(a.flags, DEV_FLAG_RESIDUAL);
    }
}

hipError_t launch_warm_mode_res(const GroupLaunch<ModeResArgs>& P, const GroupLaunch<ModeResFinalArgs>& F,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_warm_mode_res, dim3(P.tiles), dim3(256), 0, st, mkw(P));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_warm_mode_final, dim3(F.count), dim3(128), 0, st, mkw(F));
    return hipGetLastError();
}

}  // namespace rpod
