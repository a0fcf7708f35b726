// Reduced-order reconstruction (Sec. 4: a field is its zeroth-order time
// average plus the modes weighted by their time-dependent coefficients) and
// the relative L2 error of time-averaged fields against full-order ones
// (Sec. 5). Plain launches (no grouping): the caller's pointers are kernel
// arguments.
//   k_recon_abar  abar_k = (1/T) sum_t alpha[k, t], one wave per mode
//   k_recon_out   out[i, t] = mean[i] + sum_k Phi[i, k] alpha[k, t]
//                 (256 rows x 256 times per tile, 16 at a time, alpha block in
//                 LDS; arithmetic in the storage type)
//   k_recon_err   per tile of 256 rows: sums of (f - g)^2 and f^2 with
//                 f = avg_t ref[i, t] (eight interleaved sums, fixed order),
//                 g = mean[i] + sum_k Phi[i, k] abar_k
//   k_recon_sum   the tiles' sums, in order
#include <mutex>

#include "device_common.hpp"
#include "internal.hpp"

namespace rpod {

// Scratch of the entry point that allocates nothing (rpod_reconstruct_noalloc):
// abar (doubles 0..127), the two sums (128, 129) and the error's partial sums
// (from 256: two per 256-row tile, for m up to RECON_NOALLOC_MAX_M). Each GPU
// holds its own copy until the process ends; every call on a GPU shares it.
static __device__ __align__(256) double scratch[RECON_NOALLOC_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t recon_scratch(double** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        // the device address of this GPU's copy (the array's name in host code
        // is only a stand-in for the symbol)
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

template <typename T>
__global__ __launch_bounds__(64) void k_recon_abar(const T* __restrict__ alpha, int r, int64_t T_, double* abar) {
    const int k = blockIdx.x;
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < T_; t += 64) s += (double)alpha[t * r + k];
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) abar[k] = s / (double)T_;
}

template <typename T>
__global__ __launch_bounds__(256) void k_recon_out(const T* __restrict__ Phi, const T* __restrict__ mean,
                                                   const T* __restrict__ alpha, T* __restrict__ out, int64_t m, int r,
                                                   int64_t T_) {
    __shared__ T as[128 * 16];  // alpha[k, t0 .. t0 + 15], in the storage type
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const T base = (mean != nullptr && i < m) ? mean[i] : (T)0;
    const int64_t t1 = ((int64_t)blockIdx.y + 1) * 256 < T_ ? ((int64_t)blockIdx.y + 1) * 256 : T_;
    // 256 time steps per tile in chunks of 16; products and sums in the
    // storage type (the fields are stored in it), fused multiply-adds
    for (int64_t t0 = (int64_t)blockIdx.y * 256; t0 < t1; t0 += 16) {
        __syncthreads();
        for (int e = threadIdx.x; e < r * 16; e += 256) {
            const int k = e % r, tt = e / r;
            as[k + 128 * tt] = t0 + tt < T_ ? alpha[(t0 + tt) * r + k] : (T)0;
        }
        __syncthreads();
        if (i < m) {
            T acc[16];
#pragma unroll
            for (int tt = 0; tt < 16; ++tt) acc[tt] = base;
            for (int k = 0; k < r; ++k) {
                const T ph = Phi[(int64_t)k * m + i];
#pragma unroll
                for (int tt = 0; tt < 16; ++tt) acc[tt] = fma(ph, as[k + 128 * tt], acc[tt]);
            }
#pragma unroll
            for (int tt = 0; tt < 16; ++tt)
                if (t0 + tt < T_) out[(t0 + tt) * m + i] = acc[tt];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_recon_err(const T* __restrict__ Phi, const T* __restrict__ mean,
                                                   const double* __restrict__ abar, const T* __restrict__ ref,
                                                   int64_t ld_ref, int64_t m, int r, int64_t T_, double* part) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double d2 = 0.0, f2 = 0.0;
    if (i < m) {
        double fs[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // eight independent sums keep loads in flight
        int64_t t = 0;
        for (; t + 8 <= T_; t += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) fs[u] += (double)ref[(t + u) * ld_ref + i];
        }
        for (; t < T_; ++t) fs[0] += (double)ref[t * ld_ref + i];
        const double f = (((fs[0] + fs[1]) + (fs[2] + fs[3])) + ((fs[4] + fs[5]) + (fs[6] + fs[7]))) / (double)T_;
        double g = mean != nullptr ? (double)mean[i] : 0.0;
        for (int k = 0; k < r; ++k) g += (double)Phi[(int64_t)k * m + i] * abar[k];
        d2 = (f - g) * (f - g);
        f2 = f * f;
    }
    __shared__ double rd[256], rf[256];
    rd[threadIdx.x] = d2;
    rf[threadIdx.x] = f2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            rd[threadIdx.x] += rd[threadIdx.x + h];
            rf[threadIdx.x] += rf[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = rd[0];
        part[2 * blockIdx.x + 1] = rf[0];
    }
}

__global__ __launch_bounds__(256) void k_recon_sum(const double* part, int nt, double* out2) {
    double d = 0.0, f = 0.0;
    for (int w = threadIdx.x; w < nt; w += 256) {
        d += part[2 * w];
        f += part[2 * w + 1];
    }
    __shared__ double rd[256], rf[256];
    rd[threadIdx.x] = d;
    rf[threadIdx.x] = f;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            rd[threadIdx.x] += rd[threadIdx.x + h];
            rf[threadIdx.x] += rf[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out2[0] = rd[0];
        out2[1] = rf[0];
    }
}

// FP32 fields on the matrix cores: [Phi, mean] (m x (r + 1)) times the chunk's
// [alpha; 1] ((r + 1) x 128) by the split-operand S X kernel. k_recon_aug
// copies Phi and mean into the augmented matrix (leading dimension lda);
// k_recon_xchunk writes the chunk's operand (ldx rows, zero below r + 1 and
// past T) and the launch record of the chunk's S X product.
__global__ __launch_bounds__(256) void k_recon_aug(const float* __restrict__ Phi, const float* __restrict__ mean,
                                                   int64_t m, int r, float* __restrict__ aug, int64_t lda) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int k = blockIdx.y;  // 0 .. r
    if (i >= m) return;
    aug[(int64_t)k * lda + i] = k < r ? Phi[(int64_t)k * m + i] : (mean != nullptr ? mean[i] : 0.0f);
}

__global__ __launch_bounds__(256) void k_recon_xchunk(const float* __restrict__ alpha, int r, int64_t T_, int64_t t0,
                                                      float* __restrict__ x, int ldx, const float* aug, int64_t lda,
                                                      int64_t m, float* out, SxArgs* rec, int* tstart) {
    const int e = blockIdx.x * 256 + threadIdx.x;  // ldx x 128 entries
    if (e < ldx * 128) {
        const int k = e % ldx, c = e / ldx;
        const int64_t t = t0 + c;
        float v = 0.0f;
        if (t < T_) v = k < r ? alpha[t * r + k] : (k == r ? 1.0f : 0.0f);
        x[e] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        SxArgs a{};
        a.S = aug; a.ldS = lda; a.m = m; a.n = r + 1;
        a.X = x; a.ldX = ldx;
        a.Y = out + t0 * m; a.ldY = m; a.mstore = m;
        a.cond = nullptr; a.cond_mask = 0; a.call = -1;
        a.cmax = (int)(T_ - t0 < 128 ? T_ - t0 : 128);
        a.fpart = nullptr;
        *rec = a;
        tstart[0] = 0;
        tstart[1] = (int)((m + 255) / 256);
    }
}

hipError_t launch_reconstruct_mfma(int64_t m, int r, int64_t T_, const float* Phi, const float* mean,
                                   const float* alpha, float* out, float* aug, int64_t lda, float* x, int ldx,
                                   SxArgs* rec, int* tstart, hipStream_t st) {
    hipLaunchKernelGGL(k_recon_aug, dim3((unsigned)((m + 255) / 256), (unsigned)(r + 1)), dim3(256), 0, st, Phi, mean,
                       m, r, aug, lda);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int64_t t0 = 0; t0 < T_; t0 += 128) {
        hipLaunchKernelGGL(k_recon_xchunk, dim3((unsigned)((ldx * 128 + 255) / 256)), dim3(256), 0, st, alpha, r, T_,
                           t0, x, ldx, (const float*)aug, lda, m, out, rec, tstart);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        GroupLaunch<SxArgs> L;
        L.args = rec;
        L.tstart = tstart;
        L.calls = nullptr;
        L.count = 1;
        L.tiles = (int)((m + 255) / 256);
        e = launch_sx_e6(8, true, false, true, L, st);  // K = r + 1: a tall product
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
static hipError_t recon_t(int64_t m, int r, int64_t T_, const void* Phi, const void* mean, const void* alpha,
                          void* out, const void* ref, int64_t ld_ref, double* abar, double* part, double* out2,
                          hipStream_t st) {
    const unsigned rows = (unsigned)((m + 255) / 256);
    if (out != nullptr) {
        hipLaunchKernelGGL(k_recon_out<T>, dim3(rows, (unsigned)((T_ + 255) / 256)), dim3(256), 0, st, (const T*)Phi,
                           (const T*)mean, (const T*)alpha, (T*)out, m, r, T_);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (ref != nullptr) {
        hipLaunchKernelGGL(k_recon_abar<T>, dim3(r), dim3(64), 0, st, (const T*)alpha, r, T_, abar);
        hipLaunchKernelGGL(k_recon_err<T>, dim3(rows), dim3(256), 0, st, (const T*)Phi, (const T*)mean,
                           (const double*)abar, (const T*)ref, ld_ref, m, r, T_, part);
        hipLaunchKernelGGL(k_recon_sum, dim3(1), dim3(256), 0, st, (const double*)part, (int)rows, out2);
    }
    return hipGetLastError();
}

hipError_t launch_reconstruct(int dt, int64_t m, int r, int64_t T_, const void* Phi, const void* mean,
                              const void* alpha, void* out, const void* ref, int64_t ld_ref, double* abar,
                              double* part, double* out2, hipStream_t st) {
    if (dt == DT_F64) return recon_t<double>(m, r, T_, Phi, mean, alpha, out, ref, ld_ref, abar, part, out2, st);
    if (dt == DT_F32) return recon_t<float>(m, r, T_, Phi, mean, alpha, out, ref, ld_ref, abar, part, out2, st);
    return hipErrorInvalidValue;
}

}  // namespace rpod
