// Per-pixel set-up and probe lookup shared by the shading kernels and the
// edge-sampled visibility gradient (FP64 frame set-up once per pixel, the
// bilinear taps of the probe, a wavefront sum).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "device_common.h"

namespace mcdi {

namespace {

struct Pixel {
    bool valid, nov_pos;
    float3 n, t, b;        // world frame
    float3 Vl;             // view in local frame (z = n.v)
    float3 o;              // shadow-ray origin
    float3 vh, t2v;        // visible-normal frame (stretched view, T2)
    float t1x, t1y;        // T1 (z = 0)
    float3 kd, F0;
    float m, r, a2, alpha, q, nov, lamV, G1V, nlen;
    float bsdf_w;          // 1: the BSDF technique is in use, 0: light sampling only
    bool r_active;
};

__device__ __forceinline__ bool finite3(float a, float b, float c) {
    return isfinite(a) && isfinite(b) && isfinite(c);
}

__device__ Pixel setup_pixel(const ShadeArgs& A, int64_t pix, bool& nonfinite) {
    const GBufView& g = A.g;
    const int64_t N = g.n;
    Pixel P;
    P.valid = false;
    P.nov_pos = false;
    nonfinite = false;
    if (!g.mask[pix]) return P;
    const int64_t hw = (int64_t)g.height * g.width;
    const int v = (int)(pix / hw);
    const float px = g.pos[pix], py = g.pos[N + pix], pz = g.pos[2 * N + pix];
    const float nxf = g.nrm[pix], nyf = g.nrm[N + pix], nzf = g.nrm[2 * N + pix];
    const float kx = g.kd[pix], ky = g.kd[N + pix], kz = g.kd[2 * N + pix];
    const float ko = g.korm[pix], kr = g.korm[N + pix], km = g.korm[2 * N + pix];
    const float ex = g.eye[3 * v], ey = g.eye[3 * v + 1], ez = g.eye[3 * v + 2];
    if (!(finite3(px, py, pz) && finite3(nxf, nyf, nzf) && finite3(kx, ky, kz) && finite3(ko, kr, km) &&
          finite3(ex, ey, ez))) {
        nonfinite = true;
        return P;
    }
    if (nxf == 0.0f && nyf == 0.0f && nzf == 0.0f) return P;
    const double wx = (double)ex - px, wy = (double)ey - py, wz = (double)ez - pz;
    if (wx == 0.0 && wy == 0.0 && wz == 0.0) return P;
    // FP64 setup
    const double nl = sqrt((double)nxf * nxf + (double)nyf * nyf + (double)nzf * nzf);
    const double nx = nxf / nl, ny = nyf / nl, nz = nzf / nl;
    const double wl = sqrt(wx * wx + wy * wy + wz * wz);
    const double Vx = wx / wl, Vy = wy / wl, Vz = wz / wl;
    const double nov = nx * Vx + ny * Vy + nz * Vz;
    const double sg = signbit(nzf) ? -1.0 : 1.0;
    const double fa = -1.0 / (sg + nz);
    const double fb = nx * ny * fa;
    const double tx = 1.0 + sg * nx * nx * fa, ty = sg * fb, tz = -sg * nx;
    const double bx = fb, by = sg + ny * ny * fa, bz = -ny;
    const double vlx = Vx * tx + Vy * ty + Vz * tz;
    const double vly = Vx * bx + Vy * by + Vz * bz;
    P.valid = true;
    P.nov_pos = nov > 0.0;
    P.nov = (float)nov;
    P.nlen = (float)nl;
    P.n = f3((float)nx, (float)ny, (float)nz);
    P.t = f3((float)tx, (float)ty, (float)tz);
    P.b = f3((float)bx, (float)by, (float)bz);
    P.Vl = f3((float)vlx, (float)vly, (float)nov);
    const double eps = (double)A.ray_eps;
    P.o = f3((float)(px + eps * nx), (float)(py + eps * ny), (float)(pz + eps * nz));
    P.kd = f3(kx, ky, kz);
    P.m = km;
    P.r = kr;
    P.r_active = kr > kRMin;
    const float rc = P.r_active ? kr : kRMin;
    const double al = (double)rc * (double)rc;
    P.alpha = (float)al;
    P.a2 = (float)(al * al);
    P.F0 = f3(0.04f * (1.0f - km) + kx * km, 0.04f * (1.0f - km) + ky * km, 0.04f * (1.0f - km) + kz * km);
    float q = 0.5f * (1.0f - km);
    q = fminf(fmaxf(q, 0.0f), 1.0f);
    if (!P.nov_pos || (A.flags & MCDI_FLAG_FORCE_COS)) q = 1.0f;
    else if (A.flags & MCDI_FLAG_FORCE_GGX) q = 0.0f;
    P.q = q;
    P.bsdf_w = (A.flags & MCDI_FLAG_BSDF_OFF) ? 0.0f : 1.0f;
    // Smith Lambda of the view and the visible-normal frame (FP64)
    if (P.nov_pos) {
        const double t2 = (1.0 - nov * nov) / (nov * nov);
        const double lam = 0.5 * (sqrt(1.0 + al * al * t2) - 1.0);
        P.lamV = (float)lam;
        P.G1V = (float)(1.0 / (1.0 + lam));
        double hx = al * vlx, hy = al * vly, hz = nov;
        const double hl = sqrt(hx * hx + hy * hy + hz * hz);
        hx /= hl; hy /= hl; hz /= hl;
        const double lensq = hx * hx + hy * hy;
        double t1x = 1.0, t1y = 0.0;
        if (lensq > 0.0) {
            const double il = 1.0 / sqrt(lensq);
            t1x = -hy * il;
            t1y = hx * il;
        }
        P.vh = f3((float)hx, (float)hy, (float)hz);
        P.t1x = (float)t1x;
        P.t1y = (float)t1y;
        P.t2v = f3((float)(-hz * t1y), (float)(hz * t1x), (float)(hx * t1y - hy * t1x));
    } else {
        P.lamV = 0.0f;
        P.G1V = 0.0f;
        P.vh = f3(0, 0, 1);
        P.t1x = 1.0f;
        P.t1y = 0.0f;
        P.t2v = f3(0, 1, 0);
    }
    return P;
}

// bilinear lookup: the four taps around (x, y) and their tent weights.
// Texel centres sit at half-integers; columns wrap across phi = 0, rows clamp
// at the poles.  Indices are clamped before use, so any coordinate (also a
// non-finite one) stays inside the probe.
struct Taps {
    int t[4];
    float w[4];
    int base;      // upper-left tap in the extended grid of H + 1 rows (row i0 + 1)
    float fx, fy;
};

__device__ __forceinline__ Taps bilinear_taps(const EnvView& e, float x, float y) {
    const int H = e.H, W = e.W;
    const float xs = x - 0.5f, ys = y - 0.5f;
    const float fj = floorf(xs), fi = floorf(ys);
    const float fx = xs - fj, fy = ys - fi;
    const int j0 = min(max((int)fj, -1), W - 1), i0 = min(max((int)fi, -1), H - 1);
    const int ja = j0 < 0 ? W - 1 : j0;
    const int jb = j0 + 1 >= W ? 0 : j0 + 1;
    const int ia = max(i0, 0), ib = min(i0 + 1, H - 1);
    Taps T;
    T.t[0] = ia * W + ja;
    T.t[1] = ia * W + jb;
    T.t[2] = ib * W + ja;
    T.t[3] = ib * W + jb;
    T.w[0] = (1.0f - fx) * (1.0f - fy);
    T.w[1] = fx * (1.0f - fy);
    T.w[2] = (1.0f - fx) * fy;
    T.w[3] = fx * fy;
    T.base = (i0 + 1) * W + ja;
    T.fx = fx;
    T.fy = fy;
    return T;
}

__device__ __forceinline__ float3 texel_rgb(const EnvView& e, int t) {
    const float4 p = e.tex[t];
    return f3(p.x, p.y, p.z);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

}  // namespace

}  // namespace mcdi
