// Sampling tables of the lat-long probe (piecewise-constant 2D distribution,
// paper section 4.1 / appendix D), rebuilt whenever the probe changes.
//
// The weights and their running sums are FP64 and summed left to right, the
// order the tables are defined in, so every FP32 entry is the single rounding
// of the same FP64 value on any device; a row is one workgroup whose lanes
// compute the weights into LDS and whose first lane runs the scan (W <= 8192
// dependent FP64 adds, a few microseconds), rows run in parallel.
#include <hip/hip_runtime.h>
#include <math.h>

#include "device_common.h"

#pragma clang fp contract(off)

namespace mcdi {
namespace {

constexpr double kPiD = 3.14159265358979323846;

__device__ __forceinline__ double row_sin(int i, int H) { return sin(kPiD * ((double)i + 0.5) / (double)H); }

__device__ __forceinline__ double texel_weight(const float* env, int W, int i, int j, double srow) {
    const float* t = env + ((size_t)i * W + j) * 3;
    double y = ((double)t[0] + (double)t[1] + (double)t[2]) / 3.0;
    if (!(y > 0.0) || !isfinite(y)) y = 0.0;
    return y * srow;
}

__global__ __launch_bounds__(256) void rows_kernel(const float* env, int H, int W, float* cond, double* rowsum) {
    extern __shared__ double w[];  // [W]
    __shared__ double s_sum;
    const int i = blockIdx.x;
    const double srow = row_sin(i, H);
    for (int j = threadIdx.x; j < W; j += blockDim.x) w[j] = texel_weight(env, W, i, j, srow);
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int j = 0; j < W; ++j) {
            run += w[j];
            w[j] = run;  // inclusive prefix
        }
        s_sum = run;
        rowsum[i] = run;
    }
    __syncthreads();
    const double rs = s_sum;
    float* c = cond + (size_t)i * (W + 1);
    for (int k = threadIdx.x; k <= W; k += blockDim.x) {
        float v;
        if (k == 0) v = 0.0f;
        else if (k == W) v = 1.0f;
        else v = rs > 0.0 ? (float)(w[k - 1] / rs) : (float)((double)k / (double)W);
        c[k] = v;
    }
}

__global__ __launch_bounds__(256) void marginal_kernel(const double* rowsum, int H, float* marg, double* total_out,
                                                        int32_t* light_enabled) {
    extern __shared__ double pre[];  // [H]
    __shared__ double s_tot;
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int i = 0; i < H; ++i) {
            run += rowsum[i];
            pre[i] = run;
        }
        s_tot = run;
        *total_out = run;
        *light_enabled = run > 0.0 ? 1 : 0;
    }
    __syncthreads();
    const double tot = s_tot;
    for (int k = threadIdx.x; k <= H; k += blockDim.x) {
        float v;
        if (k == 0) v = 0.0f;
        else if (k == H) v = 1.0f;
        else v = tot > 0.0 ? (float)(pre[k - 1] / tot) : (float)((double)k / (double)H);
        marg[k] = v;
    }
}

__global__ void pdf_kernel(const float* env, int H, int W, const double* total, float* pdf) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)H * W) return;
    const int i = (int)(k / W), j = (int)(k - (int64_t)i * W);
    const double tot = *total;
    const double w = texel_weight(env, W, i, j, row_sin(i, H));
    pdf[k] = tot > 0.0 ? (float)((w / tot) * ((double)W * (double)H)) : 0.0f;
}

// Texels the light technique samples with probability above 1/kHotMax get a
// slot (at most kHotMax of them, since the probabilities sum to 1): the
// adjoint accumulates their gradient per workgroup in LDS before one global
// atomic per slot and workgroup.
__global__ void hot_init(int32_t* n_hot) { *n_hot = 0; }

__global__ void hot_kernel(const float* pdf, int H, int W, int32_t* hot_slot, int32_t* hot_texel,
                           int32_t* n_hot) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)H * W) return;
    const float p = pdf[k] / ((float)W * (float)H);
    int32_t slot = -1;
    if (p > 1.0f / (float)kHotMax) {
        slot = atomicAdd(n_hot, 1);
        if (slot < kHotMax) hot_texel[slot] = (int32_t)k;
        else slot = -1;
    }
    hot_slot[k] = slot;
}

__global__ __launch_bounds__(256) void guide_kernel(const float* cond, int W, int G, int32_t* guide) {
    const int i = blockIdx.x;
    const float* row = cond + (size_t)i * (W + 1);
    for (int g = threadIdx.x; g <= G; g += 256)
        guide[(size_t)i * (G + 1) + g] = cdf_find(row, W, (float)g / (float)G);
}

__global__ __launch_bounds__(256) void pack_kernel(const float* env, const float* pdf, int64_t n, float4* tex) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n) tex[k] = make_float4(env[3 * k], env[3 * k + 1], env[3 * k + 2], pdf[k]);
}

// Two bits per texel for ray generation, which only asks whether a light
// sample has a density: 0 none (pdf <= 0 or NaN: pdf / (2 pi^2 sin) is not
// > 0), 1 pdf >= 2^-100 (then pdf / (2 pi^2 sin) > 0 for every sin in
// (0, 1]: the quotient is at least 2^-100 / 19.8, or infinite), 2 a tiny
// positive pdf, whose quotient may round to 0 (read the pdf).  A quarter of a
// byte per texel stays in the L2 cache where the 4-byte densities do not.
__global__ __launch_bounds__(256) void dclass_kernel(const float* pdf, int64_t n, uint8_t* dclass) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;   // byte k: texels 4k .. 4k + 3
    if (4 * k >= n) return;
    uint32_t b = 0;
    for (int t = 0; t < 4; ++t) {
        const int64_t x = 4 * k + t;
        if (x >= n) break;
        const float p = pdf[x];
        const uint32_t c = !(p > 0.0f) ? 0u : (p >= 0x1p-100f ? 1u : 2u);
        b |= c << (2 * t);
    }
    dclass[k] = (uint8_t)b;
}

__global__ __launch_bounds__(256) void mix_kernel(const float4* rgb, const float4* dens, int64_t n, float4* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float4 a = rgb[k];
    out[k] = make_float4(a.x, a.y, a.z, dens[k].w);
}

}  // namespace

hipError_t launch_env_mix(const float4* rgb, const float4* dens, int64_t n, float4* out, hipStream_t s) {
    hipLaunchKernelGGL(mix_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rgb, dens, n, out);
    return hipGetLastError();
}

hipError_t launch_env_pack(const float* env, const float* pdf, int64_t n, float4* tex, hipStream_t s) {
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, env, pdf, n, tex);
    return hipGetLastError();
}

// Whether light draws read a cell's candidates in one go (cdf_find_row): for
// conditional tables larger than one XCD's L2 (4 MB), where a line read by
// one binary-search probe is often gone by the next.  A table that stays in
// the cache is searched faster by the binary search.
int env_row_window(int H, int W) {
    constexpr double kL2Bytes = 4 << 20;
    return (double)H * (W + 1) * sizeof(float) > kL2Bytes ? 1 : 0;
}

// Guide cells per row, at most 1024: about eight columns per cell for the
// binary search; sixteen with the candidate window, whose guide (a sixteenth
// of the rows' size) then stays in the L2 cache (on a 2048-column probe finer
// guides measured slower).
int env_guide_cells(int W, int win) {
    const int cols = win ? 16 : 8;
    int G = 1;
    while (cols * G <= W && G < 1024) G *= 2;
    return G;
}

hipError_t launch_env_dclass(const float* pdf, int64_t n, uint8_t* dclass, hipStream_t s) {
    const int64_t bytes = (n + 3) / 4;
    hipLaunchKernelGGL(dclass_kernel, dim3((unsigned)((bytes + 255) / 256)), dim3(256), 0, s, pdf, n, dclass);
    return hipGetLastError();
}

hipError_t launch_env_guide(const float* cond, int H, int W, int G, int32_t* guide, hipStream_t s) {
    hipLaunchKernelGGL(guide_kernel, dim3((unsigned)H), dim3(256), 0, s, cond, W, G, guide);
    return hipGetLastError();
}

hipError_t launch_env_hot(const float* pdf, int H, int W, int32_t* hot_slot, int32_t* hot_texel, int32_t* n_hot,
                          hipStream_t s) {
    const int64_t n = (int64_t)H * W;
    hipLaunchKernelGGL(hot_init, dim3(1), dim3(1), 0, s, n_hot);
    hipLaunchKernelGGL(hot_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pdf, H, W, hot_slot,
                       hot_texel, n_hot);
    return hipGetLastError();
}

// rowsum: device scratch of H + 1 doubles (the last holds the total)
hipError_t launch_env_cdf(const float* env, int H, int W, float* cond, float* marg, float* pdf, double* rowsum,
                          int32_t* light_enabled, hipStream_t s) {
    hipLaunchKernelGGL(rows_kernel, dim3(H), dim3(256), sizeof(double) * (size_t)W, s, env, H, W, cond, rowsum);
    hipLaunchKernelGGL(marginal_kernel, dim3(1), dim3(256), sizeof(double) * (size_t)H, s, rowsum, H, marg,
                       rowsum + H, light_enabled);
    const int64_t n = (int64_t)H * W;
    hipLaunchKernelGGL(pdf_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, env, H, W, rowsum + H, pdf);
    return hipGetLastError();
}

}  // namespace mcdi
