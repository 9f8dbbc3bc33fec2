// Image loss on the estimator's outputs, forward and backward in one pass
// (paper appendix A: L1 on tonemapped colours, T(x) = sRGB(log(x + 1)), and
// the light regulariser comparing the luminance of the tonemapped lighting
// with the HSV value of the tonemapped reference; composition c = kd*c_d + c_s
// from section 4.2).  HBM-bound: 48 B/px + 1 B mask in, 36 B/px out.
// Loss partial sums go per workgroup to FP64 scratch and are reduced in a
// fixed order, so the loss value is deterministic.
#include <hip/hip_runtime.h>
#include <math.h>

#include "mcdi_internal.h"

namespace mcdi {
namespace {

constexpr float kA = 0.055f, kLin = 0.0031308f;

__device__ __forceinline__ float srgb(float y) {
    return y <= kLin ? 12.92f * y : (1.0f + kA) * powf(y, 1.0f / 2.4f) - kA;
}
__device__ __forceinline__ float srgb_d(float y) {
    return y <= kLin ? 12.92f : ((1.0f + kA) / 2.4f) * powf(y, 1.0f / 2.4f - 1.0f);
}
__device__ __forceinline__ float tm(float x) { return srgb(log1pf(fmaxf(x, 0.0f))); }
__device__ __forceinline__ float tm_d(float x) { return x > 0.0f ? srgb_d(log1pf(x)) / (1.0f + x) : 0.0f; }
__device__ __forceinline__ float sgn(float x) { return x > 0.0f ? 1.0f : (x < 0.0f ? -1.0f : 0.0f); }

__global__ __launch_bounds__(256) void count_kernel(const uint8_t* mask, int64_t n, double* part) {
    __shared__ double s[256];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    s[threadIdx.x] = (k < n && mask[k]) ? 1.0 : 0.0;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// sequential sum of partials (fixed order); out[0] = sum
__global__ void sum_kernel(const double* part, int64_t nb, double* out) {
    double a = 0.0;
    for (int64_t i = 0; i < nb; ++i) a += part[i];
    *out = a;
}

__global__ __launch_bounds__(256) void loss_kernel(const float* kd, const float* cd, const float* cs,
                                                   const float* ref, const uint8_t* mask, int64_t n, float w_light,
                                                   const double* n_valid, double* part, float* g_kd, float* g_cd,
                                                   float* g_cs) {
    __shared__ double s_img[256], s_lit[256];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double nv = fmax(*n_valid, 1.0);
    const float inv3n = (float)(1.0 / (3.0 * nv)), invn = (float)(1.0 / nv);
    double li = 0.0, ll = 0.0;
    if (k < n) {
        const bool m = mask[k] != 0;
        float kdc[3], cdc[3], csc[3], gc[3], lsum_d[3];
        float ysum = 0.0f, vmax = -INFINITY;
        for (int c = 0; c < 3; ++c) {
            kdc[c] = kd[c * n + k];
            cdc[c] = cd[c * n + k];
            csc[c] = cs[c * n + k];
            const float r = ref[c * n + k];
            const float col = kdc[c] * cdc[c] + csc[c];
            const float d = tm(col) - tm(r);
            li += m ? (double)fabsf(d) : 0.0;
            gc[c] = m ? sgn(d) * tm_d(col) * inv3n : 0.0f;
            const float ls = cdc[c] + csc[c];
            ysum += tm(ls);
            lsum_d[c] = tm_d(ls);
            vmax = fmaxf(vmax, tm(r));
        }
        const float dl = ysum * (1.0f / 3.0f) - vmax;
        ll = m ? (double)fabsf(dl) : 0.0;
        const float gl = m ? sgn(dl) * invn * w_light * (1.0f / 3.0f) : 0.0f;
        for (int c = 0; c < 3; ++c) {
            if (g_kd) g_kd[c * n + k] = gc[c] * cdc[c];
            if (g_cd) g_cd[c * n + k] = gc[c] * kdc[c] + gl * lsum_d[c];
            if (g_cs) g_cs[c * n + k] = gc[c] + gl * lsum_d[c];
        }
    }
    s_img[threadIdx.x] = li;
    s_lit[threadIdx.x] = ll;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s_img[threadIdx.x] += s_img[threadIdx.x + o];
            s_lit[threadIdx.x] += s_lit[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s_img[0];
        part[2 * blockIdx.x + 1] = s_lit[0];
    }
}

__global__ void finish_kernel(const double* part, int64_t nb, const double* n_valid, float w_light, float* loss) {
    double a = 0.0, b = 0.0;
    for (int64_t i = 0; i < nb; ++i) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    const double nv = fmax(*n_valid, 1.0);
    const double li = a / (3.0 * nv), ll = b / nv;
    loss[0] = (float)li;
    loss[1] = (float)ll;
    loss[2] = (float)(li + (double)w_light * ll);
}

}  // namespace

// scratch: doubles, at least 3 * blocks + 1
hipError_t launch_image_loss(const float* kd, const float* cd, const float* cs, const float* ref,
                             const uint8_t* mask, int64_t n, float w_light, float* loss, float* g_kd, float* g_cd,
                             float* g_cs, double* scratch, hipStream_t s) {
    const int64_t nb = (n + 255) / 256;
    double* cnt_part = scratch;            // [nb]
    double* part = scratch + nb;           // [2 nb]
    double* n_valid = scratch + 3 * nb;    // [1]
    hipLaunchKernelGGL(count_kernel, dim3((unsigned)nb), dim3(256), 0, s, mask, n, cnt_part);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(1), 0, s, cnt_part, nb, n_valid);
    hipLaunchKernelGGL(loss_kernel, dim3((unsigned)nb), dim3(256), 0, s, kd, cd, cs, ref, mask, n, w_light, n_valid,
                       part, g_kd, g_cd, g_cs);
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(1), 0, s, part, nb, n_valid, w_light, loss);
    return hipGetLastError();
}

}  // namespace mcdi
