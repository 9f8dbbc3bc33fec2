// Differentiable cross-bilateral filter (paper appendix B, "Bilateral
// Denoiser"): the spatial part of SVGF evaluated densely over a (2R+1)^2
// footprint.  The weight of pixel q in the output of pixel p multiplies
//   a Gaussian in image distance, exp(-|p-q|^2 / (2 sigma^2)),
//   a depth edge-stop, exp(-|z(p)-z(q)| / (sigma_z |grad z(p).(p-q)| + eps)),
//   a normal term, max(0, n(p).n(q))^sigma_n,
// the output is the weight-normalised sum, and gradients go to the filtered
// colours only (the weights are constants of the backward pass).
//
// Layout: colours planar [n_chan][N], N = views*height*width, pixel
// v*H*W + y*W + x.  A workgroup owns a 16x16 tile: it stages the tile plus an
// R-pixel halo of guides (normalised normal and depth as one float4) and
// colours in LDS, then every lane walks its footprint out of LDS.  Each wave
// covers an 8x8 block and the LDS row stride is an odd multiple of 8 words,
// so the 64 lanes of one tap read 64 different banks.  Blocks are remapped so
// that consecutive tiles land on the same XCD and share halo lines in its L2.
//
// Precision: the depth gradient and the linear depth prediction are formed in
// FP64 from the FP32 depths (the differences of FP32 values and their products
// with the small integer offsets are exact there), so the prediction does not
// lose its digits when the two gradient components cancel along an iso-depth
// line.  The three weight factors are combined in one base-2 exponent and a
// single exp2; colours accumulate in FP32.
#include <hip/hip_runtime.h>
#include <math.h>

#include "mcdi_internal.h"

namespace mcdi {
namespace {

constexpr int kT = 16;          // tile side in pixels
constexpr double kEpsZ = 1e-5;  // added to the depth prediction (p = q gives 0 / eps)
constexpr double kLn2 = 0.69314718055994530942;

__host__ __device__ constexpr int lds_stride(int R) { return kT + 2 * R <= 24 ? 24 : 40; }

// Balanced block -> tile bijection: hardware places block b on XCD b % 8;
// XCD x gets the contiguous tile range starting at x*q + min(x, r).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Depth change per pixel along x and y at pixel (x, y) of a view: central
// difference where both neighbours are valid and inside the view, one-sided
// where one is, zero otherwise.  Exact in FP64.
__device__ __forceinline__ void depth_grad(const float* __restrict__ z, const uint8_t* __restrict__ m,
                                           int64_t base, int x, int y, int W, int H, double& gx, double& gy) {
    const int64_t i = base + (int64_t)y * W + x;
    const double zc = z[i];
    const bool xp = x + 1 < W && m[i + 1], xm = x > 0 && m[i - 1];
    const double zxp = xp ? (double)z[i + 1] : 0.0, zxm = xm ? (double)z[i - 1] : 0.0;
    gx = (xp && xm) ? (zxp - zxm) * 0.5 : (xp ? zxp - zc : (xm ? zc - zxm : 0.0));
    const bool yp = y + 1 < H && m[i + W], ym = y > 0 && m[i - W];
    const double zyp = yp ? (double)z[i + W] : 0.0, zym = ym ? (double)z[i - W] : 0.0;
    gy = (yp && ym) ? (zyp - zym) * 0.5 : (yp ? zyp - zc : (ym ? zc - zym : 0.0));
}

struct WeightConsts {
    float ks;     // -log2(e) / (2 sigma^2)
    float sn;     // sigma_n
    double szl;   // sigma_z * ln 2
    double epsl;  // eps * ln 2
};

// w(p, q) for guides p, q (normal xyz normalised or zero, depth w), the depth
// gradient at p, and the offset (dx, dy) = q - p.
__device__ __forceinline__ float tap_weight(const float4& p, const float4& q, double gx, double gy, int dx, int dy,
                                            const WeightConsts& c) {
    const float d = fmaf(p.x, q.x, fmaf(p.y, q.y, p.z * q.z));
    const float lg = __builtin_amdgcn_logf(fmaxf(d, 0.0f));  // log2, -inf at 0
    const double pr = fabs(fma(gx, (double)dx, gy * (double)dy));
    const float den = (float)__dadd_rn(__dmul_rn(c.szl, pr), c.epsl);
    const float az2 = fabsf(p.w - q.w) * __builtin_amdgcn_rcpf(den);  // |dz| / (pred + eps) * log2(e)
    const float e = fmaf(c.sn, lg, (float)(dx * dx + dy * dy) * c.ks - az2);
    return __builtin_amdgcn_exp2f(e);
}

__device__ __forceinline__ float4 load_guide(const BilatArgs& a, int64_t k) {
    float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
    if (a.mask[k]) {
        const float nx = a.nrm[k], ny = a.nrm[a.n + k], nz = a.nrm[2 * a.n + k];
        const float l2 = nx * nx + ny * ny + nz * nz;
        const float inv = l2 > 0.0f ? 1.0f / sqrtf(l2) : 0.0f;
        g = make_float4(nx * inv, ny * inv, nz * inv, a.depth[k]);
    }
    return g;
}

struct TileLoc {
    int64_t base;  // first pixel of the view
    int x0, y0;
};

__device__ __forceinline__ TileLoc tile_loc(const BilatArgs& a) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int per_view = a.tiles_x * a.tiles_y;
    const int v = t / per_view, r = t - v * per_view;
    return TileLoc{(int64_t)v * a.H * a.W, (r % a.tiles_x) * kT, (r / a.tiles_x) * kT};
}

// lane -> pixel inside the tile: wave w covers the 8x8 block (w&1, w>>1)
__device__ __forceinline__ void lane_pixel(int& px, int& py) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    px = (w & 1) * 8 + (l & 7);
    py = (w >> 1) * 8 + (l >> 3);
}

template <int R, int NC>
__global__ __launch_bounds__(256) void bilat_fwd_kernel(BilatArgs a, WeightConsts wc, const float* __restrict__ in,
                                                        float* __restrict__ out, float* __restrict__ wsum) {
    constexpr int S = lds_stride(R), RW = kT + 2 * R;
    __shared__ float4 geo[RW * S];
    __shared__ float col[NC][RW * S];
    const TileLoc t = tile_loc(a);
    for (int i = threadIdx.x; i < RW * RW; i += 256) {
        const int ly = i / RW, lx = i - ly * RW;
        const int gy = t.y0 - R + ly, gx = t.x0 - R + lx;
        float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
        float c[NC];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) c[ch] = 0.0f;
        if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
            const int64_t k = t.base + (int64_t)gy * a.W + gx;
            g = load_guide(a, k);
            if (a.mask[k]) {
#pragma unroll
                for (int ch = 0; ch < NC; ++ch) c[ch] = in[ch * a.n + k];
            }
        }
        geo[ly * S + lx] = g;
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) col[ch][ly * S + lx] = c[ch];
    }
    __syncthreads();
    int px, py;
    lane_pixel(px, py);
    const int x = t.x0 + px, y = t.y0 + py;
    if (x >= a.W || y >= a.H) return;
    const int64_t k = t.base + (int64_t)y * a.W + x;
    if (!a.mask[k]) {
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) out[ch * a.n + k] = 0.0f;
        if (wsum) wsum[k] = 0.0f;
        return;
    }
    double gx, gy;
    depth_grad(a.depth, a.mask, t.base, x, y, a.W, a.H, gx, gy);
    const float4 gp = geo[(py + R) * S + px + R];
    float acc[NC];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) acc[ch] = 0.0f;
    float den = 0.0f;
    for (int dy = -R; dy <= R; ++dy) {
        const int row = (py + R + dy) * S + px + R;
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
            const int j = row + dx;
            const float w = tap_weight(gp, geo[j], gx, gy, dx, dy, wc);
            den += w;
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) acc[ch] = fmaf(w, col[ch][j], acc[ch]);
        }
    }
    const float inv = den > 0.0f ? 1.0f / den : 0.0f;
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) out[ch * a.n + k] = acc[ch] * inv;
    if (wsum) wsum[k] = den;
}

// Adjoint: dL/dc(q) = sum_p dL/dout(p) w(p, q) / W(p) over the p whose
// footprint holds q, i.e. p = q - d for the same offsets d.  The staged
// region carries each p's guide, its FP64 depth gradient and its upstream
// gradient already divided by W(p).
template <int R, int NC>
__global__ __launch_bounds__(256) void bilat_bwd_kernel(BilatArgs a, WeightConsts wc, const float* __restrict__ g_out,
                                                        const float* __restrict__ wsum, float* __restrict__ g_in) {
    constexpr int S = lds_stride(R), RW = kT + 2 * R;
    __shared__ float4 geo[RW * S];
    __shared__ double2 grd[RW * S];
    __shared__ float gw[NC][RW * S];
    const TileLoc t = tile_loc(a);
    for (int i = threadIdx.x; i < RW * RW; i += 256) {
        const int ly = i / RW, lx = i - ly * RW;
        const int gy = t.y0 - R + ly, gx = t.x0 - R + lx;
        float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
        double2 d2 = make_double2(0.0, 0.0);
        float c[NC];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) c[ch] = 0.0f;
        if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
            const int64_t k = t.base + (int64_t)gy * a.W + gx;
            if (a.mask[k]) {
                g = load_guide(a, k);
                depth_grad(a.depth, a.mask, t.base, gx, gy, a.W, a.H, d2.x, d2.y);
                const float W = wsum[k];
                const float inv = W > 0.0f ? 1.0f / W : 0.0f;
#pragma unroll
                for (int ch = 0; ch < NC; ++ch) c[ch] = g_out[ch * a.n + k] * inv;
            }
        }
        geo[ly * S + lx] = g;
        grd[ly * S + lx] = d2;
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) gw[ch][ly * S + lx] = c[ch];
    }
    __syncthreads();
    int px, py;
    lane_pixel(px, py);
    const int x = t.x0 + px, y = t.y0 + py;
    if (x >= a.W || y >= a.H) return;
    const int64_t k = t.base + (int64_t)y * a.W + x;
    float acc[NC];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) acc[ch] = 0.0f;
    if (a.mask[k]) {
        const float4 gq = geo[(py + R) * S + px + R];
        for (int dy = -R; dy <= R; ++dy) {
            const int row = (py + R - dy) * S + px + R;
#pragma unroll
            for (int dx = -R; dx <= R; ++dx) {
                const int j = row - dx;
                const double2 gp = grd[j];
                const float w = tap_weight(geo[j], gq, gp.x, gp.y, dx, dy, wc);
#pragma unroll
                for (int ch = 0; ch < NC; ++ch) acc[ch] = fmaf(w, gw[ch][j], acc[ch]);
            }
        }
    }
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) g_in[ch * a.n + k] = acc[ch];
}

__global__ __launch_bounds__(256) void view_depth_kernel(GBufView g, float* __restrict__ depth) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= g.n) return;
    float d = 0.0f;
    if (g.mask[k]) {
        const int v = (int)(k / ((int64_t)g.height * g.width));
        const float ex = g.pos[k] - g.eye[3 * v], ey = g.pos[g.n + k] - g.eye[3 * v + 1],
                    ez = g.pos[2 * g.n + k] - g.eye[3 * v + 2];
        d = sqrtf(ex * ex + ey * ey + ez * ez);
    }
    depth[k] = d;
}

WeightConsts weight_consts(const BilatArgs& a) {
    const double s = a.sigma;
    return WeightConsts{(float)(-1.4426950408889634 / (2.0 * s * s)), a.sigma_n, (double)a.sigma_z * kLn2,
                        kEpsZ * kLn2};
}

template <int NC, bool BWD>
hipError_t dispatch(const BilatArgs& a, const float* x, const float* w, float* y, hipStream_t s) {
    const WeightConsts wc = weight_consts(a);
    const int nb = a.tiles_x * a.tiles_y * a.V;
#define MCDI_BILAT_CASE(RR)                                                                              \
    case RR:                                                                                             \
        if (BWD) bilat_bwd_kernel<RR, NC><<<nb, 256, 0, s>>>(a, wc, x, w, y);                           \
        else bilat_fwd_kernel<RR, NC><<<nb, 256, 0, s>>>(a, wc, x, y, const_cast<float*>(w));          \
        break;
    switch (a.R) {
        MCDI_BILAT_CASE(1)
        MCDI_BILAT_CASE(2)
        MCDI_BILAT_CASE(3)
        MCDI_BILAT_CASE(4)
        MCDI_BILAT_CASE(5)
        MCDI_BILAT_CASE(6)
        MCDI_BILAT_CASE(7)
        MCDI_BILAT_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef MCDI_BILAT_CASE
    return hipGetLastError();
}

}  // namespace

int bilateral_radius(float sigma) {
    const double r = ceil(3.0 * (double)sigma);
    return r < 1.0 ? 1 : (r > kBilatMaxR ? kBilatMaxR : (int)r);
}

void bilateral_tiles(BilatArgs& a) {
    a.tiles_x = (a.W + kT - 1) / kT;
    a.tiles_y = (a.H + kT - 1) / kT;
}

hipError_t launch_bilateral_fwd(const BilatArgs& a, int nc, const float* in, float* out, float* wsum,
                                hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    switch (nc) {
        case 1: return dispatch<1, false>(a, in, wsum, out, s);
        case 3: return dispatch<3, false>(a, in, wsum, out, s);
        case 6: return dispatch<6, false>(a, in, wsum, out, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bilateral_bwd(const BilatArgs& a, int nc, const float* g_out, const float* wsum, float* g_in,
                                hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    switch (nc) {
        case 1: return dispatch<1, true>(a, g_out, wsum, g_in, s);
        case 3: return dispatch<3, true>(a, g_out, wsum, g_in, s);
        case 6: return dispatch<6, true>(a, g_out, wsum, g_in, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_view_depth(const GBufView& g, float* depth, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    view_depth_kernel<<<(unsigned)((g.n + 255) / 256), 256, 0, s>>>(g, depth);
    return hipGetLastError();
}

}  // namespace mcdi
