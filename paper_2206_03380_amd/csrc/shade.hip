// Per-pixel Monte Carlo direct illumination on gfx950: forward (c_d, c_s and
// shadow-ray hit bits) and the adjoint of the detached estimator.
//
// One lane owns one pixel and loops over its samples; each sample draws one
// light-technique direction and one BSDF-technique direction (cosine or GGX
// visible normals, chosen with probability q), weights both with the balance
// heuristic over the three techniques and traces one shadow ray per
// direction above the horizon (paper: section 3.1, section 4.1, appendix D).
// The marginal CDF of the probe is staged in LDS; the per-pixel frame, view
// vector and visible-normal frame are set up in FP64 once per pixel (FP64
// FMA runs at the FP32 rate on CDNA, and it removes the ill-conditioning of
// the tangent frame when the view is close to the normal).
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

// visible-normal sample (Heitz 2018), local frame
__device__ __forceinline__ float3 sample_vndf(const Pixel& P, float u1, float u2) {
    const float r = sqrtf(u1);
    float sp, cp;
    sincospif(2.0f * u2, &sp, &cp);
    const float a1 = r * cp;
    float a2 = r * sp;
    const float s = 0.5f * (1.0f + P.vh.z);
    a2 = (1.0f - s) * sqrtf(fmaxf(0.0f, 1.0f - a1 * a1)) + s * a2;
    const float az = sqrtf(fmaxf(0.0f, 1.0f - a1 * a1 - a2 * a2));
    const float3 nh = f3(a1 * P.t1x + a2 * P.t2v.x + az * P.vh.x, a1 * P.t1y + a2 * P.t2v.y + az * P.vh.y,
                         a2 * P.t2v.z + az * P.vh.z);
    const float3 ne = normalize(f3(P.alpha * nh.x, P.alpha * nh.y, fmaxf(0.0f, nh.z)));
    const float vn = dot(P.Vl, ne);
    return (2.0f * vn) * ne - P.Vl;
}

struct Sample {
    float3 wl;     // local direction
    float3 w;      // world direction
    float pL;      // light-technique density
    int texel;     // probe texel index i*W + j
    float x, y;    // continuous texel coordinates (phi W / 2 pi, theta H / pi)
};

struct FwdAcc {
    float3 cd, cs;
};

struct BwdAcc {
    float3 gkd;
    float gm, gr;
    float3 gnl;  // d/dn in the local frame
};

// Light technique: piecewise-constant 2D distribution over the probe.
// Returns false when the sample has no density (direction at a pole).
__device__ __forceinline__ bool draw_light(const ShadeArgs& A, const Pixel& P, const float* s_marg, uint4 r0,
                                           Sample& S) {
    const int H = A.env.H, W = A.env.W;
    const float x0 = u01(r0.x), x1 = u01(r0.y);
    const int i = cdf_find(s_marg, H, x0);
    const float* crow = A.env.cond + (size_t)i * (W + 1);
    const int j = cdf_find_guided(crow, A.env.guide + (size_t)i * (A.env.G + 1), A.env.G, x1);
    const float m0 = s_marg[i], m1 = s_marg[i + 1];
    const float c0 = crow[j], c1 = crow[j + 1];
    S.y = (float)i + (x0 - m0) / (m1 - m0);
    S.x = (float)j + (x1 - c0) / (c1 - c0);
    const float v = S.y / (float)H;
    const float u = S.x / (float)W;
    float st, ct, sp, cp;
    sincospif(v, &st, &ct);
    sincospif(2.0f * u, &sp, &cp);
    S.w = f3(st * cp, ct, st * sp);
    S.texel = i * W + j;
    S.pL = st > 0.0f ? A.env.tex[S.texel].w / (2.0f * kPi * kPi * st) : 0.0f;
    S.wl = f3(dot(S.w, P.t), dot(S.w, P.b), dot(S.w, P.n));
    return S.pL > 0.0f;
}

// BSDF technique: cosine lobe with probability q, else GGX visible normals.
__device__ __forceinline__ bool draw_bsdf(const Pixel& P, uint4 r0, uint4 r1, Sample& S) {
    const float x2 = u01(r0.z), x4 = u01(r1.x), x5 = u01(r1.y);
    const bool cosl = x2 < P.q;
    if (cosl) {
        const float rr = sqrtf(x4);
        float sp, cp;
        sincospif(2.0f * x5, &sp, &cp);
        S.wl = f3(rr * cp, rr * sp, sqrtf(fmaxf(0.0f, 1.0f - x4)));
    } else {
        S.wl = sample_vndf(P, x4, x5);
    }
    S.w = normalize(S.wl.x * P.t + S.wl.y * P.b + S.wl.z * P.n);
    S.pL = 0.0f;
    S.texel = -1;
    return cosl;
}

// probe texel (nearest) of a BSDF-sampled direction and its light density
__device__ __forceinline__ void bsdf_texel(const ShadeArgs& A, bool light_on, Sample& S) {
    const int H = A.env.H, W = A.env.W;
    const float rho = sqrtf(S.w.x * S.w.x + S.w.z * S.w.z);
    const float th = atan2f(rho, S.w.y);
    float ph = atan2f(S.w.z, S.w.x);
    if (ph < 0.0f) ph += 2.0f * kPi;
    S.y = th * ((float)H * kInvPi);
    S.x = ph * ((float)W * (0.5f * kInvPi));
    const int ti = min((int)S.y, H - 1);
    const int tj = min((int)S.x, W - 1);
    S.texel = ti * W + tj;
    if (light_on && rho > 0.0f) S.pL = A.env.tex[S.texel].w / (2.0f * kPi * kPi * rho);
}

// where the adjoint puts probe-gradient records of non-hot texels: the tile's
// record region and its LDS fill counter (base NULL: direct global atomics)
struct RecSink {
    float4* base;
    uint32_t* count;
};

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

// one record (n float4s) appended to the tile's region: one LDS counter
// atomic per wave; the region holds every record the tile can make
template <int NQ>
__device__ __forceinline__ void append_record(const RecSink& rs, const float4 (&q)[NQ]) {
    const uint64_t act = __ballot(1);
    const int lane = (int)__lane_id();
    const int leader = __ffsll((unsigned long long)act) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(rs.count, (uint32_t)__popcll(act));
    base = (uint32_t)__shfl((int)base, leader);
    const uint32_t at = base + (uint32_t)__popcll(act & ((1ull << lane) - 1ull));
#pragma unroll
    for (int k = 0; k < NQ; ++k) rs.base[(size_t)NQ * at + k] = q[k];
}

// probe-gradient contribution (v0, v1, v2) of one texel: hot texels go to
// the workgroup's LDS copy, the rest to the tile's records (or straight to
// global memory when there are none)
// maybe_hot false: the texel's density rules it out of the hot set (its slot
// is not read)
__device__ __forceinline__ void scatter_texel(const ShadeArgs& A, int texel, float v0, float v1, float v2,
                                              float* s_hot, const RecSink& rs, bool maybe_hot = true) {
    const int slot = maybe_hot ? A.env.hot_slot[texel] : -1;
    if (slot >= 0) {
        atomicAdd(s_hot + 3 * slot + 0, v0);
        atomicAdd(s_hot + 3 * slot + 1, v1);
        atomicAdd(s_hot + 3 * slot + 2, v2);
    } else if (v0 == 0.0f && v1 == 0.0f && v2 == 0.0f) {
        // nothing to add (a shadowed sample with tau = 1, a zero tap weight)
    } else if (rs.base) {
        const float4 q[1] = {make_float4(__uint_as_float((uint32_t)texel), v0, v1, v2)};
        append_record<1>(rs, q);
    } else {
        float* ge = A.g_env + 3 * (size_t)texel;
        atomicAdd(ge + 0, v0);
        atomicAdd(ge + 1, v1);
        atomicAdd(ge + 2, v2);
    }
}

template <bool BWD, bool BIL>
__device__ __forceinline__ void eval_sample(const ShadeArgs& A, const Pixel& P, const Sample& S, float Hv,
                                            float invspp, FwdAcc& fa, BwdAcc& ba, float3 Ud, float3 Us,
                                            float* s_hot, const RecSink& rs) {
    const float NoL = S.wl.z;
    const float3 hl = normalize(P.Vl + S.wl);
    const float NoH = hl.z;
    const float s2 = hl.x * hl.x + hl.y * hl.y;
    const float VoH = dot(P.Vl, hl);
    const float D = ggx_D(NoH, s2, P.a2);
    const float pcos = NoL * kInvPi;
    const float pggx = P.nov_pos ? P.G1V * D / (4.0f * P.nov) : 0.0f;
    // balance heuristic over the techniques in use
    const float Pt = S.pL + P.bsdf_w * (P.q * pcos + (1.0f - P.q) * pggx);
    const float w = Hv / Pt;
    float3 L;
    float pdf_uv = 0.0f;   // nearest lookup: the texel's density (pdf table)
    if (BIL) {
        const Taps T = bilinear_taps(A.env, S.x, S.y);
        L = T.w[0] * texel_rgb(A.env, T.t[0]) + T.w[1] * texel_rgb(A.env, T.t[1]) +
            T.w[2] * texel_rgb(A.env, T.t[2]) + T.w[3] * texel_rgb(A.env, T.t[3]);
    } else {
        const float4 tx = A.env.tex[S.texel];
        L = f3(tx.x, tx.y, tx.z);
        pdf_uv = tx.w;
    }
    const float kdiff = (1.0f - P.m) * kInvPi * NoL;
    float S_ = 0.0f, Fw = 0.0f, G2 = 0.0f, lamL = 0.0f, t2L = 0.0f;
    float3 F = f3(0, 0, 0);
    if (P.nov_pos) {
        t2L = smith_t2(NoL);
        lamL = smith_lambda(t2L, P.a2);
        G2 = 1.0f / (1.0f + P.lamV + lamL);
        S_ = D * G2 / (4.0f * P.nov);
        const float omv = 1.0f - VoH;
        const float o2 = omv * omv;
        Fw = o2 * o2 * omv;
        F = f3(P.F0.x + (1.0f - P.F0.x) * Fw, P.F0.y + (1.0f - P.F0.y) * Fw, P.F0.z + (1.0f - P.F0.z) * Fw);
    }
    if (!BWD) {
        fa.cd = fa.cd + (kdiff * w) * L;
        fa.cs = fa.cs + (S_ * w) * f3(F.x * L.x, F.y * L.y, F.z * L.z);
        return;
    }
    const float K = w * invspp;
    // probe texel gradient: the coefficient of L_c, times the tap weight
    const float cdc = kdiff * K, csc = S_ * K;
    if (A.g_env) {
        const float v0 = Ud.x * cdc + Us.x * F.x * csc;
        const float v1 = Ud.y * cdc + Us.y * F.y * csc;
        const float v2 = Ud.z * cdc + Us.z * F.z * csc;
        if (BIL) {
            // taps recomputed from the coordinates: cheaper than keeping
            // them live across the BSDF terms
            const Taps T = bilinear_taps(A.env, S.x, S.y);
            if (rs.base) {
                // one record per sample (base, fractions, coefficient), split
                // into the four taps by the env-scatter pass; no LDS hot
                // sums here: twelve contended LDS float atomics per sample
                // cost more than the record
                if (v0 != 0.0f || v1 != 0.0f || v2 != 0.0f) {
                    const float4 q[2] = {make_float4(__uint_as_float((uint32_t)T.base), T.fx, T.fy, 0.0f),
                                         make_float4(v0, v1, v2, 0.0f)};
                    append_record<2>(rs, q);
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    scatter_texel(A, T.t[k], T.w[k] * v0, T.w[k] * v1, T.w[k] * v2, s_hot, rs);
            }
        } else {
            // hot texels have pdf > W H / kHotMax (the hot-set rule); half that
            // bound keeps the test free of rounding questions
            const bool maybe_hot = pdf_uv > 0.5f * ((float)A.env.W * (float)A.env.H / (float)kHotMax);
            scatter_texel(A, S.texel, v0, v1, v2, s_hot, rs, maybe_hot);
        }
    }
    const float udL = Ud.x * L.x + Ud.y * L.y + Ud.z * L.z;
    const float usL = Us.x * L.x + Us.y * L.y + Us.z * L.z;
    const float uskdL = Us.x * P.kd.x * L.x + Us.y * P.kd.y * L.y + Us.z * P.kd.z * L.z;
    const float usFL = Us.x * F.x * L.x + Us.y * F.y * L.y + Us.z * F.z * L.z;
    const float omF = 1.0f - Fw;
    ba.gkd = ba.gkd + (P.m * omF * S_ * K) * f3(Us.x * L.x, Us.y * L.y, Us.z * L.z);
    ba.gm += -NoL * kInvPi * K * udL + omF * S_ * K * (uskdL - 0.04f * usL);
    // diffuse part of d/dn: (1-m)/pi * udL * K * w_l
    float3 gn = ((1.0f - P.m) * kInvPi * udL * K) * S.wl;
    if (P.nov_pos) {
        const float a = P.alpha, a2 = P.a2;
        const float B = a2 * NoH * NoH + s2;
        const float dDda = D * (2.0f / a - 4.0f * a * NoH * NoH / B);
        const float t2V = smith_t2(P.nov);
        const float sqV = sqrtf(1.0f + a2 * t2V), sqL = sqrtf(1.0f + a2 * t2L);
        const float dlamV_da = a * t2V / (2.0f * sqV), dlamL_da = a * t2L / (2.0f * sqL);
        const float G2s = G2 * G2;
        const float dSda = (dDda * G2 - D * G2s * (dlamV_da + dlamL_da)) / (4.0f * P.nov);
        const float dSdr = P.r_active ? dSda * 2.0f * P.r : 0.0f;
        ba.gr += usFL * K * dSdr;
        const float dlamV_dx = -a2 / (2.0f * P.nov * P.nov * P.nov * sqV);
        const float dlamL_dx = -a2 / (2.0f * NoL * NoL * NoL * sqL);
        const float dSdV = -D * G2s * dlamV_dx / (4.0f * P.nov) - S_ / P.nov;
        const float dSdL = -D * G2s * dlamL_dx / (4.0f * P.nov);
        const float dSdH = D * 4.0f * (1.0f - a2) * NoH / B * G2 / (4.0f * P.nov);
        const float c = usFL * K;
        gn = gn + (c * dSdV) * P.Vl + (c * dSdL) * S.wl + (c * dSdH) * hl;
    }
    ba.gnl = ba.gnl + gn;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ void stage_marg(const ShadeArgs& A, float* s_marg) {
    for (int k = threadIdx.x; k <= A.env.H; k += blockDim.x) s_marg[k] = A.env.marg[k];
}

// ---------------------------------------------------------------------------
// The three stages work on one tile of kBlock pixels per workgroup.  The
// staged kernels run tile = blockIdx.x; the serving kernel pulls tiles of
// many requests from a queue and runs the stages back to back.
// ---------------------------------------------------------------------------

// 1) ray generation: the directions of every sample above the horizon,
//    compacted into the tile's ray region (LDS counter, no global atomics);
//    hit words of the tile's pixels are cleared; returns the ray count
//    (valid in thread 0 after the final barrier, in *s_cnt for all).
template <bool COUNT>
__device__ __forceinline__ void gen_tile(const ShadeArgs& A, int64_t tile, float4* region, uint32_t* hitbits,
                                         const float* s_marg, int* s_cnt) {
    const int64_t N = A.g.n;
    const int64_t pix = tile * kBlock + threadIdx.x;
    const bool active = pix < N;
    const int spp = A.spp;
    const int words = (2 * spp + 31) >> 5;
    const bool light_on = (*A.env.light_enabled != 0) && !(A.flags & MCDI_FLAG_LIGHT_OFF);
    const bool trace = A.tau != 0.0f && region != nullptr;
    bool nonfinite = false;
    Pixel P;
    P.valid = false;
    if (active) {
        for (int k = 0; k < words; ++k) hitbits[k * N + pix] = 0u;
        P = setup_pixel(A, pix, nonfinite);
        if (P.valid) A.origins[pix] = make_float4(P.o.x, P.o.y, P.o.z, 0.0f);
    }
    const bool go = P.valid && trace;
    const int64_t hw = (int64_t)A.g.height * A.g.width;
    const uint32_t view = active ? (uint32_t)(pix / hw) : 0u;
    const uint32_t piv = active ? (uint32_t)(pix - (int64_t)view * hw) : 0u;
    const uint32_t vid = (uint32_t)A.g.view_base + view;
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    const int lane = __lane_id();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t c_rays = 0, c_culled = 0;
    for (int s = 0; s < spp; ++s) {
        uint4 r0 = make_uint4(0, 0, 0, 0), r1 = r0;
        if (go) {
            r0 = philox10(make_uint4(piv, vid, (uint32_t)s, 0u), k0, k1);
            r1 = philox10(make_uint4(piv, vid, (uint32_t)s, 1u), k0, k1);
        }
        for (int tech = 0; tech < 2; ++tech) {
            bool want = false;
            Sample S;
            if (go) {
                bool has = true;
                if (tech == 0) has = light_on && draw_light(A, P, s_marg, r0, S);
                else if (P.bsdf_w != 0.0f) draw_bsdf(P, r0, r1, S);
                else has = false;
                want = has && S.wl.z > 0.0f;
                if (has && !want) ++c_culled;
            }
            const uint64_t bal = __ballot(want);
            if (bal == 0ull) continue;
            int base = 0;
            if (lane == 0) base = atomicAdd(s_cnt, (int)__popcll(bal));
            base = __shfl(base, 0);
            if (want) {
                const int slot = 2 * s + tech;
                const uint32_t tag = (uint32_t)threadIdx.x | ((uint32_t)slot << 8);
                region[base + (int)__popcll(bal & lt)] = make_float4(S.w.x, S.w.y, S.w.z, __uint_as_float(tag));
                ++c_rays;
            }
        }
    }
    if (COUNT) {
        const uint32_t a = wave_sum(c_rays), b = wave_sum(c_culled);
        const uint32_t v = wave_sum(P.valid ? 1u : 0u), nf = wave_sum(nonfinite ? 1u : 0u);
        if (lane == 0) {
            atomicAdd(&A.stats->rays_traced, (unsigned long long)a);
            atomicAdd(&A.stats->samples_culled, (unsigned long long)b);
            atomicAdd(&A.stats->valid_pixels, (unsigned long long)v);
            atomicAdd(&A.stats->invalid_pixels, (unsigned long long)nf);
        }
    }
}

// 2) any-hit traversal of the tile's ray region.  Lanes that finish a ray
//    take the next one from the region (one LDS atomic per wave per refill);
//    box steps and triangle steps run in separate phases so a wave keeps its
//    lanes on the same code (while-while traversal with dynamic fetch).
//
//    Per lane: the next node to test (n_total once the walk is over, or when
//    the lane holds no ray) and up to two postponed leaves, kept as their
//    packed payload words (first_triangle << 3 | count; 0 = none).  Testing
//    one triangle of a leaf advances its word by 7: the first index grows by
//    one and the count drops by one.  The second slot is only used while the
//    first is pending.
template <bool COUNT>
__device__ __forceinline__ void trace_tile(const ShadeArgs& A, int64_t tile, const float4* R, int count,
                                           uint32_t* hitbits, int* s_next) {
    const Scene& sc = A.scene;
    const int64_t N = A.g.n;
    const int64_t base_pix = tile * kBlock;
    const int n_total = sc.nodes[0].escape;
    const uint32_t n_tris = (uint32_t)sc.n_tris;
    const char* node_bytes = reinterpret_cast<const char*>(sc.nodes);
    const char* tri_bytes = reinterpret_cast<const char*>(sc.tris);
    const int lane = __lane_id();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    bool active = false, exhausted = false;
    Ray ray;
    int node = n_total;
    uint32_t p0 = 0u, p1 = 0u;
    int64_t pix = 0;
    int slot = 0;
    uint32_t c_hits = 0, c_box = 0, c_tri = 0, c_bstep = 0, c_tstep = 0;   // steps: lane 0 only
    // scheduling knobs: refill batch, node steps per phase check, and the
    // phase hand-over ratios (in halves)
    constexpr int kRefillMin = 32, kBoxSteps = 2, kBoxSwitch2 = 2, kTriSwitch2 = 2;
    while (true) {
        // refill when half of the wave is idle, or when nobody is busy
        const uint64_t need = __ballot(!active && !exhausted);
        const uint64_t busy = __ballot(active);
        if (need && (__popcll(need) >= kRefillMin || busy == 0ull)) {
            const int leader = __ffsll((unsigned long long)need) - 1;
            int b = 0;
            if (lane == leader) b = atomicAdd(s_next, (int)__popcll(need));
            b = __shfl(b, leader);
            if (!active && !exhausted) {
                const int idx = b + (int)__popcll(need & lt);
                if (idx < count) {
                    const float4 rr = R[idx];
                    const uint32_t tag = __float_as_uint(rr.w);
                    pix = base_pix + (tag & 255u);
                    slot = (int)(tag >> 8);
                    const float4 o = A.origins[pix];
                    ray = make_ray(f3(o.x, o.y, o.z), f3(rr.x, rr.y, rr.z));
                    node = 0;
                    p0 = p1 = 0u;
                    active = n_total > 0;
                } else {
                    exhausted = true;
                }
            }
        }
        if (!__any(active)) {
            if (!__any(!exhausted)) break;
            continue;
        }
        // box phase: a lane walks while its second leaf slot is free and the
        // tree is not finished (a leaf found with the first slot taken goes
        // to the second); the phase ends once the lanes that hold a leaf and
        // cannot walk are at least as many as the lanes still walking
        while (true) {
            if (!__any(node < n_total && p1 == 0u)) break;
#pragma unroll
            for (int step = 0; step < kBoxSteps; ++step) {
                const bool walking = node < n_total && p1 == 0u;
                if (COUNT && __any(walking) && lane == 0) ++c_bstep;
                if (walking) {
                    const uint32_t off = (uint32_t)node * 32u;
                    const float4 a = *reinterpret_cast<const float4*>(node_bytes + off);
                    const float4 b = *reinterpret_cast<const float4*>(node_bytes + off + 16u);
                    const uint32_t payload = __float_as_uint(b.w);
                    if (COUNT) ++c_box;
                    const bool hit = box_hit(ray, a, b);
                    // skip links point forward; max() keeps every walk finite
                    const int next = max(__float_as_int(a.w), node + 1);
                    node = (hit && payload == 0u) ? node + 1 : next;
                    const bool take = hit && payload != 0u;
                    const bool first_free = p0 == 0u;
                    p0 = (take && first_free) ? payload : p0;
                    p1 = (take && !first_free) ? payload : p1;
                }
            }
            const bool walk = node < n_total && p1 == 0u;
            const bool stuck = p0 != 0u && !walk;
            if (2 * __popcll(__ballot(stuck)) >= kBoxSwitch2 * __popcll(__ballot(walk))) break;
        }
        // triangle phase: one triangle of the first pending leaf per lane and
        // step; it ends when no leaf is pending, or when lanes that could walk
        // but hold no leaf outnumber the lanes testing
        while (true) {
            const bool test = p0 != 0u;
            if (!__any(test)) break;
            if (COUNT && lane == 0) ++c_tstep;
            if (test) {
                const uint32_t t = p0 >> 3;
                bool h = false;
                if (t < n_tris) {       // a payload past the triangle array tests nothing
                    const float4* tv = reinterpret_cast<const float4*>(tri_bytes + t * 48u);
                    if (COUNT) ++c_tri;
                    h = tri_anyhit(ray, tv[0], tv[1], tv[2]);
                }
                if (h) {
                    atomicOr(hitbits + (int64_t)(slot >> 5) * N + pix, 1u << (slot & 31));
                    ++c_hits;
                    active = false;
                    node = n_total;
                    p0 = p1 = 0u;
                } else {
                    p0 += 7u;
                    if ((p0 & 7u) == 0u) {
                        p0 = p1;
                        p1 = 0u;
                    }
                }
            }
            const bool testing = p0 != 0u;
            const bool idle = !testing && node < n_total;
            if (2 * __popcll(__ballot(idle)) > kTriSwitch2 * __popcll(__ballot(testing))) break;
        }
        if (active && p0 == 0u && node >= n_total) active = false;  // miss
    }
    if (COUNT) {
        const uint32_t h = wave_sum(c_hits), bx = wave_sum(c_box), tr = wave_sum(c_tri);
        if (lane == 0) {
            atomicAdd(&A.stats->rays_hit, (unsigned long long)h);
            atomicAdd(&A.stats->box_tests, (unsigned long long)bx);
            atomicAdd(&A.stats->tri_tests, (unsigned long long)tr);
            atomicAdd(&A.stats->box_slots, 64ull * c_bstep);
            atomicAdd(&A.stats->tri_slots, 64ull * c_tstep);
        }
    }
}

// 3) evaluation: forward values or the adjoint, from the hit bits.  For the
//    adjoint, s_hot must be zeroed before and flushed after (hot_flush).
//    BIL: bilinear probe lookup (MCDI_FLAG_BILINEAR) instead of the nearest
//    texel.
template <bool BWD, bool DUMP, bool BIL>
__device__ __forceinline__ void shade_tile(const ShadeArgs& A, int64_t tile, const float* s_marg, float* s_hot,
                                           const RecSink& rs) {
    const int64_t N = A.g.n;
    const int64_t pix = tile * kBlock + threadIdx.x;
    const int spp = A.spp;
    const bool light_on = (*A.env.light_enabled != 0) && !(A.flags & MCDI_FLAG_LIGHT_OFF);
    const bool trace = A.tau != 0.0f;
    if (pix >= N) return;
    bool nonfinite;
    const Pixel P = setup_pixel(A, pix, nonfinite);
    if (!P.valid) {
        if (!BWD) {
            for (int c = 0; c < 3; ++c) { A.c_d[c * N + pix] = 0.0f; A.c_s[c * N + pix] = 0.0f; }
        } else {
            for (int c = 0; c < 3; ++c) {
                A.g_kd[c * N + pix] = 0.0f; A.g_korm[c * N + pix] = 0.0f; A.g_nrm[c * N + pix] = 0.0f;
            }
        }
        if (DUMP) {
            uint32_t* d = A.decisions + (size_t)pix * spp * 3;
            for (int s = 0; s < spp; ++s) { d[3 * s] = kNone; d[3 * s + 1] = kNone; d[3 * s + 2] = 0u; }
        }
        return;
    }
    const int64_t hw = (int64_t)A.g.height * A.g.width;
    const uint32_t view = (uint32_t)(pix / hw), piv = (uint32_t)(pix - (int64_t)view * hw);
    const uint32_t vid = (uint32_t)A.g.view_base + view;
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    const float invspp = 1.0f / (float)spp;
    float3 Ud = f3(0, 0, 0), Us = f3(0, 0, 0);
    if (BWD) {
        Ud = f3(A.g_cd[pix], A.g_cd[N + pix], A.g_cd[2 * N + pix]);
        Us = f3(A.g_cs[pix], A.g_cs[N + pix], A.g_cs[2 * N + pix]);
    }
    FwdAcc fa{f3(0, 0, 0), f3(0, 0, 0)};
    BwdAcc ba{f3(0, 0, 0), 0.0f, 0.0f, f3(0, 0, 0)};
    uint32_t bits = 0;
    for (int s = 0; s < spp; ++s) {
        if (((2 * s) & 31) == 0) bits = A.hitbits_in[((2 * s) >> 5) * N + pix];
        const uint4 r0 = philox10(make_uint4(piv, vid, (uint32_t)s, 0u), k0, k1);
        const uint4 r1 = philox10(make_uint4(piv, vid, (uint32_t)s, 1u), k0, k1);
        uint32_t rec0 = kNone, rec1 = kNone;
        uint32_t rec2 = kDecValid | (P.nov_pos ? kDecNovPos : 0u);
        for (int tech = 0; tech < 2; ++tech) {
            Sample S;
            if (tech == 0) {
                if (!light_on) continue;
                const bool has = draw_light(A, P, s_marg, r0, S);
                rec0 = (uint32_t)S.texel;
                if (!has) { rec2 |= kDecLCull; continue; }
            } else {
                if (P.bsdf_w == 0.0f) continue;
                if (draw_bsdf(P, r0, r1, S)) rec2 |= kDecLobeCos;
            }
            if (!(S.wl.z > 0.0f)) { rec2 |= tech ? kDecBCull : kDecLCull; continue; }
            if (tech == 1) {
                bsdf_texel(A, light_on, S);
                rec1 = (uint32_t)S.texel;
            }
            float Hv = 1.0f;
            if (trace) {
                const int bitpos = 2 * s + tech;
                rec2 |= tech ? kDecBTraced : kDecLTraced;
                if ((bits >> (bitpos & 31)) & 1u) {
                    Hv = 1.0f - A.tau;
                    rec2 |= tech ? kDecBHit : kDecLHit;
                }
            }
            eval_sample<BWD, BIL>(A, P, S, Hv, invspp, fa, ba, Ud, Us, s_hot, rs);
        }
        if (DUMP) {
            uint32_t* d = A.decisions + ((size_t)pix * spp + s) * 3;
            d[0] = rec0; d[1] = rec1; d[2] = rec2;
        }
    }
    if (!BWD) {
        for (int c = 0; c < 3; ++c) {
            A.c_d[c * N + pix] = comp(fa.cd, c) * invspp;
            A.c_s[c * N + pix] = comp(fa.cs, c) * invspp;
        }
    } else {
        A.g_kd[pix] = ba.gkd.x; A.g_kd[N + pix] = ba.gkd.y; A.g_kd[2 * N + pix] = ba.gkd.z;
        A.g_korm[pix] = 0.0f; A.g_korm[N + pix] = ba.gr; A.g_korm[2 * N + pix] = ba.gm;
        const float il = 1.0f / P.nlen;
        const float3 gw = (ba.gnl.x * il) * P.t + (ba.gnl.y * il) * P.b;
        A.g_nrm[pix] = gw.x; A.g_nrm[N + pix] = gw.y; A.g_nrm[2 * N + pix] = gw.z;
    }
}

__device__ __forceinline__ void hot_zero(float* s_hot) {
    for (int k = threadIdx.x; k < 3 * kHotMax; k += blockDim.x) s_hot[k] = 0.0f;
}

// one global atomic per touched hot slot (call after a barrier)
__device__ __forceinline__ void hot_flush(const ShadeArgs& A, const float* s_hot) {
    if (!A.g_env) return;
    const int n_hot = min(*A.env.n_hot, kHotMax);
    for (int k = threadIdx.x; k < 3 * n_hot; k += blockDim.x) {
        const float v = s_hot[k];
        if (v != 0.0f) atomicAdd(A.g_env + 3 * (size_t)A.env.hot_texel[k / 3] + (k % 3), v);
    }
}

__device__ __forceinline__ float4* tile_region(const ShadeArgs& A, int64_t tile) {
    return A.rays ? A.rays + (size_t)tile * (size_t)(2 * A.spp * kBlock) : nullptr;
}

template <bool COUNT>
__global__ __launch_bounds__(kBlock) void gen_rays_kernel(ShadeArgs A, uint32_t* hitbits) {
    extern __shared__ float s_marg[];
    __shared__ int s_cnt;
    stage_marg(A, s_marg);
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    gen_tile<COUNT>(A, blockIdx.x, tile_region(A, blockIdx.x), hitbits, s_marg, &s_cnt);
    __syncthreads();
    if (threadIdx.x == 0) A.ray_count[blockIdx.x] = s_cnt;
}

// Traversal order of the tiles: a counting sort by ray count, most rays
// first, so that the longest workgroups start first and the short ones fill
// the end of the launch (longest-processing-time-first).  One workgroup;
// counts are bucketed by 8 rays (beyond 8184 rays a tile is just "long").
// The order of tiles within a bucket is arbitrary: traversal results do not
// depend on it.
constexpr int kOrderBuckets = 1024;

__global__ __launch_bounds__(1024) void order_tiles_kernel(const int32_t* __restrict__ cnt, int64_t n,
                                                           int32_t* __restrict__ order) {
    __shared__ int h[kOrderBuckets];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    auto bucket = [](int c) { return kOrderBuckets - 1 - min(max(c, 0) >> 3, kOrderBuckets - 1); };
    for (int64_t t = tid; t < n; t += 1024) atomicAdd(&h[bucket(cnt[t])], 1);
    __syncthreads();
    // exclusive scan over the buckets (bucket 0 = the most rays)
    int v = h[tid];
    for (int off = 1; off < kOrderBuckets; off <<= 1) {
        const int a = tid >= off ? h[tid - off] : 0;
        __syncthreads();
        h[tid] += a;
        __syncthreads();
    }
    h[tid] -= v;
    __syncthreads();
    for (int64_t t = tid; t < n; t += 1024) {
        const int pos = atomicAdd(&h[bucket(cnt[t])], 1);
        order[pos] = (int32_t)t;
    }
}

template <bool COUNT>
__global__ __launch_bounds__(kBlock) void trace_rays_kernel(ShadeArgs A, uint32_t* hitbits) {
    __shared__ int s_next;
    const int64_t tile = A.tile_order ? A.tile_order[blockIdx.x] : blockIdx.x;
    if (tile < 0 || tile >= (int64_t)gridDim.x) return;   // uniform: the whole workgroup reads the same entry
    if (threadIdx.x == 0) s_next = 0;
    __syncthreads();
    trace_tile<COUNT>(A, tile, tile_region(A, tile), A.ray_count[tile], hitbits, &s_next);
}

template <bool BWD, bool DUMP, bool BIL>
__device__ __forceinline__ void shade_body(const ShadeArgs& A) {
    extern __shared__ float smem[];
    __shared__ uint32_t s_rec;
    float* s_marg = smem;
    float* s_hot = smem + ((A.env.H + 1 + 3) & ~3);
    stage_marg(A, s_marg);
    if (BWD) hot_zero(s_hot);
    if (threadIdx.x == 0) s_rec = 0u;
    __syncthreads();
    const RecSink rs{(BWD && A.rec) ? A.rec + (size_t)blockIdx.x * A.rec_region * (BIL ? 2 : 1) : nullptr, &s_rec};
    shade_tile<BWD, DUMP, BIL>(A, blockIdx.x, s_marg, s_hot, rs);
    if (BWD) {
        __syncthreads();
        hot_flush(A, s_hot);
        if (A.rec && threadIdx.x == 0) A.rec_count[blockIdx.x] = s_rec;
    }
}

// Four waves per SIMD (at most 128 VGPRs) for every variant except the
// bilinear adjoint, which spills at that bound and runs faster at three.
template <bool BWD, bool DUMP, bool BIL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void shade_kernel(ShadeArgs A) {
    shade_body<BWD, DUMP, BIL>(A);
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void shade_bwd_bilinear_kernel(ShadeArgs A) {
    shade_body<true, false, true>(A);
}

// ---------------------------------------------------------------------------
// Serving: one persistent launch over the tiles of many requests.  Every
// workgroup takes the next tile from a global counter and runs generation,
// traversal, the forward evaluation and (for gradient requests) the adjoint
// on it; it stops when the tiles run out, so every wave exits.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void serve_kernel(const ServeItem* items, int n_items, int64_t total_tiles,
                                                       int* tile_counter, float4* scratch, int spp_max) {
    extern __shared__ float smem[];
    __shared__ int s_tile, s_item, s_cnt, s_next;
    float* s_hot = smem;                     // 3 * kHotMax
    float* s_marg = smem + 3 * kHotMax;      // H + 1 of the current item
    float4* region = scratch + (size_t)blockIdx.x * (size_t)(2 * spp_max * kBlock);
    while (true) {
        if (threadIdx.x == 0) {
            const int t = atomicAdd(tile_counter, 1);
            int lo = 0, hi = n_items;           // item with first_global <= t
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (items[mid].first_global <= t) lo = mid; else hi = mid;
            }
            s_tile = t;
            s_item = lo;
            s_cnt = 0;
            s_next = 0;
        }
        __syncthreads();
        const int64_t t = s_tile;
        if (t >= total_tiles) break;
        const ServeItem& it = items[s_item];
        const ShadeArgs& A = it.args;
        const int64_t tile = it.first_tile + (t - it.first_global);
        stage_marg(A, s_marg);
        __syncthreads();
        float4* reg = A.tau != 0.0f ? region : nullptr;
        gen_tile<false>(A, tile, reg, it.hitbits, s_marg, &s_cnt);
        __syncthreads();
        if (reg) trace_tile<false>(A, tile, reg, s_cnt, it.hitbits, &s_next);
        __syncthreads();
        const bool bil = (A.flags & MCDI_FLAG_BILINEAR) != 0;
        if (bil) shade_tile<false, false, true>(A, tile, s_marg, s_hot, RecSink{nullptr, nullptr});
        else shade_tile<false, false, false>(A, tile, s_marg, s_hot, RecSink{nullptr, nullptr});
        if (A.g_cd) {
            hot_zero(s_hot);
            __syncthreads();
            if (bil) shade_tile<true, false, true>(A, tile, s_marg, s_hot, RecSink{nullptr, nullptr});
            else shade_tile<true, false, false>(A, tile, s_marg, s_hot, RecSink{nullptr, nullptr});
            __syncthreads();
            hot_flush(A, s_hot);
        }
        __syncthreads();
    }
}

__global__ void serve_reset(int* tile_counter) { *tile_counter = 0; }

__global__ void trace_kernel(Scene sc, const float* o, const float* d, int64_t n, uint8_t* hit, int brute) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const Ray r = make_ray(f3(o[k], o[n + k], o[2 * n + k]), f3(d[k], d[n + k], d[2 * n + k]));
    const int n_total = sc.nodes[0].escape;
    uint32_t nb = 0, nt = 0;
    hit[k] = (brute ? brute_anyhit(sc, r) : bvh_anyhit(sc, r, n_total, nb, nt)) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Edge-sampled visibility gradient of the shadow term.  Seen from the ray
// origin o, a silhouette edge a-b bounds the directions its face blocks; as
// the vertices move, the arc through x(t) = a + t (b - a) moves along the
// unit normal mh of the plane (o, a, b) at mh . dx / r, r = |x - o|, and
// sweeps |(b - a) x w| / r of arc per unit t.  Across the arc the integrand
// drops from g to g (1 - tau) when nothing else blocks the out side, so a
// sample (edge e uniform over E, t uniform) adds
//   E s tau g(w) |(b - a) x w| / r^2 / n_es  x  ((1 - t) mh, t mh)
// to the gradients of a and b, s = +1 when the face lies on the +mh side.
// Silhouette: the edge's two faces lie on the same side of the plane (or it
// has one face).  g contracts the unshadowed integrand of c_d and c_s with
// the upstream gradients.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float3 load_vert(const float* v, int32_t i) {
    const float* p = v + 3 * (size_t)i;
    return f3(p[0], p[1], p[2]);
}

__device__ __forceinline__ float3 cross(float3 a, float3 b) {
    return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// probe radiance in direction w (nearest texel, or bilinear with BIL)
__device__ __forceinline__ float3 probe_radiance(const EnvView& e, float3 w, bool bil) {
    const int H = e.H, W = e.W;
    const float rho = sqrtf(w.x * w.x + w.z * w.z);
    const float th = atan2f(rho, w.y);
    float ph = atan2f(w.z, w.x);
    if (ph < 0.0f) ph += 2.0f * kPi;
    const float y = th * ((float)H * kInvPi);
    const float x = ph * ((float)W * (0.5f * kInvPi));
    if (bil) {
        const Taps T = bilinear_taps(e, x, y);
        return T.w[0] * texel_rgb(e, T.t[0]) + T.w[1] * texel_rgb(e, T.t[1]) + T.w[2] * texel_rgb(e, T.t[2]) +
               T.w[3] * texel_rgb(e, T.t[3]);
    }
    const int ti = min((int)y, H - 1), tj = min((int)x, W - 1);
    return texel_rgb(e, ti * W + tj);
}

// The face sides come from det(a - o, b - o, c - o) written as (a - o) .
// ((b - a) x (c - a)), free of the cancellation of differences from a
// distant o.  Returns false when the sample cannot carry a term: no
// silhouette, a degenerate arc, or the point at or below the horizon.
struct EdgeGeom {
    uint32_t e;          // edge row
    float t, s;          // point on the edge; +1 when the face lies on the +mh side
    float3 w, mh;        // unit direction to the point; unit arc normal
    float r2;            // squared distance to the point
    float3 eab;
};

__device__ __forceinline__ bool edge_geom(const EdgeArgs& E, const Pixel& P, uint32_t piv, uint32_t vid, int j,
                                          uint32_t ne, EdgeGeom& G) {
    const uint32_t k0 = (uint32_t)E.a.seed, k1 = (uint32_t)(E.a.seed >> 32);
    const uint4 r = philox10(make_uint4(piv, vid, (uint32_t)j, 2u), k0, k1);
    G.e = __umulhi(r.x, ne);
    G.t = u01(r.y);
    // the edge's corners, packed in one 64-byte line for this call
    const float4* q = E.egeo + 4 * (size_t)G.e;
    const float4 pa = q[0], pb = q[1], pc = q[2], pd = q[3];
    const float3 va = f3(pa.x, pa.y, pa.z);
    const float3 qa = va - P.o;
    G.eab = f3(pb.x, pb.y, pb.z) - va;
    const float3 m = cross(qa, G.eab);   // = (a - o) x (b - o)
    const float sc = dot(qa, cross(G.eab, f3(pc.x, pc.y, pc.z) - va));
    if (sc == 0.0f) return false;
    if (pd.w != 0.0f) {
        const float sd = dot(qa, cross(G.eab, f3(pd.x, pd.y, pd.z) - va));
        if ((sc > 0.0f && sd < 0.0f) || (sc < 0.0f && sd > 0.0f)) return false;   // both sides covered
    }
    const float ml2 = dot(m, m);
    if (!(ml2 > 0.0f)) return false;
    const float3 w = qa + G.t * G.eab;
    G.r2 = dot(w, w);
    G.w = (1.0f / sqrtf(G.r2)) * w;
    if (!(dot(G.w, P.n) > 0.0f)) return false;
    G.mh = (1.0f / sqrtf(ml2)) * m;
    G.s = sc > 0.0f ? 1.0f : -1.0f;
    return true;
}

// The part of setup_pixel the edge filter needs: validity (same rules), the
// shadow-ray origin and the unit normal, with the same FP64 arithmetic so
// that both are bit-identical to setup_pixel's.
__device__ __forceinline__ bool pixel_origin(const ShadeArgs& A, int64_t pix, Pixel& P, bool& nonfinite) {
    const GBufView& g = A.g;
    const int64_t N = g.n;
    nonfinite = false;
    if (!g.mask[pix]) return false;
    const int v = (int)(pix / ((int64_t)g.height * g.width));
    const float px = g.pos[pix], py = g.pos[N + pix], pz = g.pos[2 * N + pix];
    const float nxf = g.nrm[pix], nyf = g.nrm[N + pix], nzf = g.nrm[2 * N + pix];
    const float ex = g.eye[3 * v], ey = g.eye[3 * v + 1], ez = g.eye[3 * v + 2];
    if (!(finite3(px, py, pz) && finite3(nxf, nyf, nzf) &&
          finite3(g.kd[pix], g.kd[N + pix], g.kd[2 * N + pix]) &&
          finite3(g.korm[pix], g.korm[N + pix], g.korm[2 * N + pix]) && finite3(ex, ey, ez))) {
        nonfinite = true;
        return false;
    }
    if (nxf == 0.0f && nyf == 0.0f && nzf == 0.0f) return false;
    const double wx = (double)ex - px, wy = (double)ey - py, wz = (double)ez - pz;
    if (wx == 0.0 && wy == 0.0 && wz == 0.0) return false;
    const double nl = sqrt((double)nxf * nxf + (double)nyf * nyf + (double)nzf * nzf);
    const double nx = nxf / nl, ny = nyf / nl, nz = nzf / nl;
    const double eps = (double)A.ray_eps;
    P.n = f3((float)nx, (float)ny, (float)nz);
    P.o = f3((float)(px + eps * nx), (float)(py + eps * ny), (float)(pz + eps * nz));
    return true;
}

// 1) every edge sample of a pass of pixels; the candidates (silhouette, above
//    the horizon) go to the queue as (pixel in pass << 10 | sample).  Samples
//    are filtered 32 at a time into a bit mask before any append, so that
//    their loads overlap.
__global__ __launch_bounds__(kBlock) void edge_gen_kernel(EdgeArgs E) {
    const ShadeArgs& A = E.a;
    const int64_t local = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t pix = E.pix0 + local;
    const bool active = local < E.npix && pix < A.g.n;
    const uint32_t ne = *E.n_edges;
    bool nonfinite = false, valid = false;
    Pixel P;
    if (active) valid = pixel_origin(A, pix, P, nonfinite);
    const bool go = valid && ne > 0u && A.tau != 0.0f;
    const int64_t hw = (int64_t)A.g.height * A.g.width;
    const uint32_t view = active ? (uint32_t)(pix / hw) : 0u;
    const uint32_t piv = active ? (uint32_t)(pix - (int64_t)view * hw) : 0u;
    const uint32_t vid = (uint32_t)A.g.view_base + view;
    const int lane = __lane_id();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int j0 = 0; j0 < E.n_es; j0 += 32) {
        const int nj = E.n_es - j0 < 32 ? E.n_es - j0 : 32;
        uint32_t bits = 0u;
        if (go) {
            for (int jj = 0; jj < nj; ++jj) {
                EdgeGeom G;
                if (edge_geom(E, P, piv, vid, j0 + jj, ne, G)) bits |= 1u << jj;
            }
        }
        if (__ballot(bits != 0u) == 0ull) continue;
        for (int jj = 0; jj < nj; ++jj) {
            const bool emit = (bits >> jj) & 1u;
            const uint64_t bal = __ballot(emit);
            if (bal == 0ull) continue;
            const int leader = __ffsll((unsigned long long)bal) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(E.q_count, (uint32_t)__popcll(bal));
            base = (uint32_t)__shfl((int)base, leader);
            if (emit) {
                const uint32_t at = base + (uint32_t)__popcll(bal & lt);
                // the queue holds every sample of the pass; the check only
                // guards the bound
                if (at < E.q_cap) E.queue[at] = ((uint32_t)local << 10) | (uint32_t)(j0 + jj);
            }
        }
    }
    if (A.stats) {
        const uint32_t v = wave_sum(valid ? 1u : 0u), nf = wave_sum(nonfinite ? 1u : 0u);
        if (lane == 0) {
            atomicAdd(&A.stats->valid_pixels, (unsigned long long)v);
            atomicAdd(&A.stats->invalid_pixels, (unsigned long long)nf);
        }
    }
}

// Any-hit query of one ray by a whole wavefront.  Lane k descends six levels
// from the root along the bits of k to one of up to 64 disjoint subtrees (the
// first child of an internal node i is i + 1, the second is the first child's
// skip link; a leaf reached early belongs to the lane whose remaining bits are
// zero) and walks its subtree with the skip links, bounded by the subtree's
// end.  A missed ancestor box implies missed descendants, so testing each
// subtree root's own box suffices.  The walk stops as soon as any lane finds
// a hit.  The ray must be the same in every lane; the result is uniform.
__device__ __forceinline__ bool wave_anyhit(const Scene& sc, const Ray& r, int n_total) {
    if (n_total <= 0) return false;
    const float4* nodes = reinterpret_cast<const float4*>(sc.nodes);
    constexpr int kDepth = 6;
    const int lane = __lane_id();
    int node = 0;
    bool mine = true;
    for (int lvl = 0; lvl < kDepth; ++lvl) {
        const int payload = __float_as_int(nodes[2 * node + 1].w);
        int right = -1;
        if (payload == 0 && node + 1 < n_total) right = __float_as_int(nodes[2 * (node + 1)].w);
        // a leaf (or a malformed link) ends the descent here
        if (payload != 0 || right <= node + 1 || right >= n_total) {
            mine = (lane >> lvl) == 0;
            break;
        }
        node = ((lane >> lvl) & 1) ? right : node + 1;
    }
    const int esc = __float_as_int(nodes[2 * node].w);
    const int end = (esc > node && esc <= n_total) ? esc : n_total;
    int i = mine ? node : end;
    bool hit = false;
    while (__any(i < end)) {
        if (i < end) {
            const float4 a = nodes[2 * i];
            const float4 b = nodes[2 * i + 1];
            const int escape = __float_as_int(a.w);
            const int payload = __float_as_int(b.w);
            const int next = (escape > i && escape <= end) ? escape : end;
            if (!box_hit(r, a, b)) {
                i = next;
            } else if (payload == 0) {
                ++i;
            } else {
                const int first = payload >> 3;
                const int cnt = (first + (payload & 7) <= sc.n_tris) ? (payload & 7) : 0;
                for (int k = 0; k < cnt && !hit; ++k) {
                    const float4* t = sc.tris + 3 * (first + k);
                    hit = tri_anyhit(r, t[0], t[1], t[2]);
                }
                i = next;
            }
        }
        if (__any(hit)) return true;
    }
    return false;
}

// 2) the queued candidates, one per wavefront: the sample is recomputed (in
//    every lane alike), its term evaluated and its out-side ray traced by the
//    whole wavefront; a ray that reaches the probe adds the term to both
//    vertices of the edge
__global__ __launch_bounds__(256) void edge_trace_kernel(EdgeArgs E) {
    const ShadeArgs& A = E.a;
    const Scene& sc = A.scene;
    const uint32_t n = min(*E.q_count, E.q_cap);
    const uint32_t ne = *E.n_edges;
    const int n_total = sc.nodes[0].escape;
    const bool bil = (A.flags & MCDI_FLAG_BILINEAR) != 0;
    const int64_t N = A.g.n;
    const int64_t hw = (int64_t)A.g.height * A.g.width;
    const float scale = (float)ne * A.tau / (float)E.n_es;
    const bool lead = __lane_id() == 0;
    uint32_t c_rays = 0, c_hits = 0;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t i = wave; i < n; i += n_waves) {
        const uint32_t rec = E.queue[i];
        const int64_t pix = E.pix0 + (int64_t)(rec >> 10);
        const int j = (int)(rec & 1023u);
        if (pix >= N) continue;
        bool nonfinite;
        const Pixel P = setup_pixel(A, pix, nonfinite);
        if (!P.valid) continue;
        const uint32_t view = (uint32_t)(pix / hw);
        const uint32_t piv = (uint32_t)(pix - (int64_t)view * hw);
        EdgeGeom G;
        if (!edge_geom(E, P, piv, (uint32_t)A.g.view_base + view, j, ne, G)) continue;
        const float3 Ud = f3(A.g_cd[pix], A.g_cd[N + pix], A.g_cd[2 * N + pix]);
        const float3 Us = f3(A.g_cs[pix], A.g_cs[N + pix], A.g_cs[2 * N + pix]);
        const float3 w = G.w;
        const float NoL = dot(w, P.n);
        const float3 ex = cross(G.eab, w);
        const float J = sqrtf(dot(ex, ex)) / G.r2;
        const float3 L = probe_radiance(A.env, w, bil);
        // unshadowed integrand at w (unit density), contracted
        const float3 wl = f3(dot(w, P.t), dot(w, P.b), NoL);
        const float kdiff = (1.0f - P.m) * kInvPi * NoL;
        float g = kdiff * (Ud.x * L.x + Ud.y * L.y + Ud.z * L.z);
        if (P.nov_pos) {
            const float3 hl = normalize(P.Vl + wl);
            const float s2 = hl.x * hl.x + hl.y * hl.y;
            const float D = ggx_D(hl.z, s2, P.a2);
            const float lamL = smith_lambda(smith_t2(NoL), P.a2);
            const float Sv = D / (1.0f + P.lamV + lamL) / (4.0f * P.nov);
            const float omv = 1.0f - dot(P.Vl, hl);
            const float o2 = omv * omv;
            const float Fw = o2 * o2 * omv;
            const float3 F = f3(P.F0.x + (1.0f - P.F0.x) * Fw, P.F0.y + (1.0f - P.F0.y) * Fw,
                                P.F0.z + (1.0f - P.F0.z) * Fw);
            g += Sv * (Us.x * F.x * L.x + Us.y * F.y * L.y + Us.z * F.z * L.z);
        }
        const float wt = G.s * scale * J * g;
        if (!(wt != 0.0f && isfinite(wt))) continue;
        const float3 wo = normalize(w - (G.s * kEdgeDelta) * G.mh);
        ++c_rays;
        if (wave_anyhit(sc, make_ray(P.o, wo), n_total)) {
            ++c_hits;
            continue;
        }
        if (lead) {
            const int4 ed = E.edges[G.e];
            const float ta = 1.0f - G.t;
            float* ga = E.g_verts + 3 * (size_t)ed.x;
            float* gb = E.g_verts + 3 * (size_t)ed.y;
            atomicAdd(ga + 0, ta * wt * G.mh.x);
            atomicAdd(ga + 1, ta * wt * G.mh.y);
            atomicAdd(ga + 2, ta * wt * G.mh.z);
            atomicAdd(gb + 0, G.t * wt * G.mh.x);
            atomicAdd(gb + 1, G.t * wt * G.mh.y);
            atomicAdd(gb + 2, G.t * wt * G.mh.z);
        }
    }
    if (A.stats && lead && c_rays) {
        atomicAdd(&A.stats->rays_traced, (unsigned long long)c_rays);
        atomicAdd(&A.stats->rays_hit, (unsigned long long)c_hits);
    }
}

__global__ void edge_queue_reset(uint32_t* q_count) { *q_count = 0u; }

// corners of every edge for this call's vertex positions: (a, 0), (b, 0),
// (c, 0), (d, 1) or (0, 0, 0, 0) without a second face
__global__ void edge_pack_kernel(const int4* __restrict__ edges, const uint32_t* n_edges, const float* verts,
                                 float4* egeo, uint32_t cap) {
    const uint32_t n = min(*n_edges, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int4 ed = edges[i];
        const float3 a = load_vert(verts, ed.x), b = load_vert(verts, ed.y), c = load_vert(verts, ed.z);
        float4* q = egeo + 4 * (size_t)i;
        q[0] = make_float4(a.x, a.y, a.z, 0.0f);
        q[1] = make_float4(b.x, b.y, b.z, 0.0f);
        q[2] = make_float4(c.x, c.y, c.z, 0.0f);
        if (ed.w >= 0) {
            const float3 d = load_vert(verts, ed.w);
            q[3] = make_float4(d.x, d.y, d.z, 1.0f);
        } else {
            q[3] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    }
}

}  // namespace

static unsigned n_blocks(const ShadeArgs& a) { return (unsigned)((a.g.n + kBlock - 1) / kBlock); }
static size_t marg_lds(const ShadeArgs& a) { return sizeof(float) * (size_t)((a.env.H + 1 + 3) & ~3); }

hipError_t launch_gen_rays(const ShadeArgs& a, uint32_t* hitbits, hipStream_t s) {
    if (a.stats)
        hipLaunchKernelGGL((gen_rays_kernel<true>), dim3(n_blocks(a)), dim3(kBlock), marg_lds(a), s, a, hitbits);
    else
        hipLaunchKernelGGL((gen_rays_kernel<false>), dim3(n_blocks(a)), dim3(kBlock), marg_lds(a), s, a, hitbits);
    return hipGetLastError();
}

hipError_t launch_order_tiles(const int32_t* ray_count, int64_t n_tiles, int32_t* order, hipStream_t s) {
    hipLaunchKernelGGL(order_tiles_kernel, dim3(1), dim3(1024), 0, s, ray_count, n_tiles, order);
    return hipGetLastError();
}

hipError_t launch_trace_rays(const ShadeArgs& a, uint32_t* hitbits, hipStream_t s) {
    if (a.stats)
        hipLaunchKernelGGL((trace_rays_kernel<true>), dim3(n_blocks(a)), dim3(kBlock), 0, s, a, hitbits);
    else
        hipLaunchKernelGGL((trace_rays_kernel<false>), dim3(n_blocks(a)), dim3(kBlock), 0, s, a, hitbits);
    return hipGetLastError();
}

hipError_t launch_shade_fwd(const ShadeArgs& a, hipStream_t s) {
    const bool dump = (a.flags & MCDI_FLAG_DUMP) != 0, bil = (a.flags & MCDI_FLAG_BILINEAR) != 0;
    const dim3 g(n_blocks(a)), b(kBlock);
    if (dump && bil) hipLaunchKernelGGL((shade_kernel<false, true, true>), g, b, marg_lds(a), s, a);
    else if (dump) hipLaunchKernelGGL((shade_kernel<false, true, false>), g, b, marg_lds(a), s, a);
    else if (bil) hipLaunchKernelGGL((shade_kernel<false, false, true>), g, b, marg_lds(a), s, a);
    else hipLaunchKernelGGL((shade_kernel<false, false, false>), g, b, marg_lds(a), s, a);
    return hipGetLastError();
}

hipError_t launch_serve(const ServeItem* items_dev, int n_items, int64_t total_tiles, int* tile_counter,
                        float4* scratch, int spp_max, int n_workgroups, int max_H, hipStream_t s) {
    hipLaunchKernelGGL(serve_reset, dim3(1), dim3(1), 0, s, tile_counter);
    const size_t lds = sizeof(float) * (3 * kHotMax + (size_t)max_H + 1);
    hipLaunchKernelGGL(serve_kernel, dim3(n_workgroups), dim3(kBlock), lds, s, items_dev, n_items, total_tiles,
                       tile_counter, scratch, spp_max);
    return hipGetLastError();
}

hipError_t launch_shade_bwd(const ShadeArgs& a, hipStream_t s) {
    const size_t lds = marg_lds(a) + sizeof(float) * 3 * kHotMax;
    if (a.flags & MCDI_FLAG_BILINEAR)
        hipLaunchKernelGGL(shade_bwd_bilinear_kernel, dim3(n_blocks(a)), dim3(kBlock), lds, s, a);
    else
        hipLaunchKernelGGL((shade_kernel<true, false, false>), dim3(n_blocks(a)), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_trace(const Scene& sc, const float* o, const float* d, int64_t n, uint8_t* hit, int brute,
                        hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(trace_kernel, dim3((unsigned)blocks), dim3(256), 0, s, sc, o, d, n, hit, brute);
    return hipGetLastError();
}

hipError_t launch_edge_pack(const EdgeArgs& e, uint32_t cap, hipStream_t s) {
    const uint32_t blocks = (cap + 255) / 256 < 4096u ? (cap + 255) / 256 : 4096u;
    hipLaunchKernelGGL(edge_pack_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, e.edges, e.n_edges, e.verts,
                       const_cast<float4*>(e.egeo), cap);
    return hipGetLastError();
}

hipError_t launch_edge_grad(const EdgeArgs& e, hipStream_t s) {
    if (e.npix <= 0) return hipSuccess;
    hipLaunchKernelGGL(edge_queue_reset, dim3(1), dim3(1), 0, s, e.q_count);
    hipLaunchKernelGGL(edge_gen_kernel, dim3((unsigned)((e.npix + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, e);
    // the queue's length is on the device: a fixed grid of 8192 wavefronts
    // strides over it, one record per wavefront
    hipLaunchKernelGGL(edge_trace_kernel, dim3(2048), dim3(256), 0, s, e);
    return hipGetLastError();
}

}  // namespace mcdi
