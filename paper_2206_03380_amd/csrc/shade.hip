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

// Multiply-adds are fused only within one source expression, never across
// statements, so a sample's arithmetic rounds the same way in every loop that
// evaluates it (the staged forward's walk over live samples, the decision
// dump's full walk, the serving kernel's lockstep walk) and their results
// agree bit for bit.  (Set before the shared headers, whose inline functions
// are compiled here; the triangle test turns contraction off itself.)
#pragma clang fp contract(on)

#include "device_common.h"
#include "shade_common.h"

namespace mcdi {

namespace {

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
    float4 tx;     // the texel's (r, g, b, pdf), read once per sample
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
// How each stage draws a light sample:
//  kDrawGen  ray generation: whether the density is positive, from the
//            texels' 2-bit density classes (the density table for tiny
//            densities): the sample's density itself is not used there;
//  kDrawFwd  forward shading: the texel's radiance and density, kept for the
//            evaluation;
//  kDrawBwd  adjoint: the density from the radiance table (the evaluation
//            reads that line again) and always the binary row search, which
//            needs fewer registers than the adjoint has to spare.
// The other two read the row's candidates in one go (cdf_find_row) where the
// tables ask for it (env.win).
enum DrawMode { kDrawGen, kDrawFwd, kDrawBwd };

template <int MODE>
__device__ __forceinline__ bool draw_light(const ShadeArgs& A, const Pixel& P, const float* s_marg, uint4 r0,
                                           Sample& S) {
    const int H = A.env.H, W = A.env.W;
    const float x0 = u01(r0.x), x1 = u01(r0.y);
    const int i = cdf_find(s_marg, H, x0);
    const float* crow = A.env.cond + (size_t)i * (W + 1);
    float c0, c1;
    int j;
    if (MODE != kDrawBwd && A.env.win) {
        j = cdf_find_row(crow, A.env.guide + (size_t)i * (A.env.G + 1), A.env.G, x1, c0, c1);
    } else {
        j = cdf_find_guided(crow, A.env.guide + (size_t)i * (A.env.G + 1), A.env.G, x1);
        c0 = crow[j];
        c1 = crow[j + 1];
    }
    const float m0 = s_marg[i], m1 = s_marg[i + 1];
    S.y = (float)i + (x0 - m0) / (m1 - m0);
    S.x = (float)j + (x1 - c0) / (c1 - c0);
    const float v = S.y / (float)H;
    const float u = S.x / (float)W;
    float st, ct, sp, cp;
    sincospif(v, &st, &ct);
    sincospif(2.0f * u, &sp, &cp);
    S.w = f3(st * cp, ct, st * sp);
    S.texel = i * W + j;
    if (MODE == kDrawFwd) {
        S.tx = A.env.tex[S.texel];
    } else if (MODE == kDrawGen) {
        // generation only asks whether the density is positive: the
        // texel's class answers it except for tiny densities (class 2)
        const uint32_t cls = (A.env.dclass[S.texel >> 2] >> (2 * (S.texel & 3))) & 3u;
        S.tx.w = cls == 2u ? A.env.pdf[S.texel] : (float)cls;
    } else {
        S.tx.w = A.env.tex[S.texel].w;
    }
    S.pL = st > 0.0f ? S.tx.w / (2.0f * kPi * kPi * st) : 0.0f;
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
template <bool KEEP>
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
    if (KEEP) {
        S.tx = A.env.tex[S.texel];
        if (light_on && rho > 0.0f) S.pL = S.tx.w / (2.0f * kPi * kPi * rho);
    } else if (light_on && rho > 0.0f) {
        S.pL = A.env.tex[S.texel].w / (2.0f * kPi * kPi * rho);
    }
}

// where the adjoint puts probe-gradient records of non-hot texels: the tile's
// record region and its LDS fill counter (base NULL: direct global atomics)
struct RecSink {
    float4* base;
    uint32_t* count;
};

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

// balance-heuristic denominator of a sample: the densities of the techniques
// in use at its direction
__device__ __forceinline__ float mis_density(const Pixel& P, const Sample& S) {
    const float3 hl = normalize(P.Vl + S.wl);
    const float D = ggx_D(hl.z, hl.x * hl.x + hl.y * hl.y, P.a2);
    const float pcos = S.wl.z * kInvPi;
    const float pggx = P.nov_pos ? P.G1V * D / (4.0f * P.nov) : 0.0f;
    return S.pL + P.bsdf_w * (P.q * pcos + (1.0f - P.q) * pggx);
}

// FROZEN: the sample was drawn from another pixel state, whose density
// (Pt_frozen) weighs it; P and S.wl evaluate it
template <bool BWD, bool BIL, bool FROZEN = false>
__device__ __forceinline__ void eval_sample(const ShadeArgs& A, const Pixel& P, const Sample& S, float Hv,
                                            float invspp, FwdAcc& fa, BwdAcc& ba, float3 Ud, float3 Us,
                                            float* s_hot, const RecSink& rs, float Pt_frozen = 0.0f) {
    const float NoL = S.wl.z;
    const float3 hl = normalize(P.Vl + S.wl);
    const float NoH = hl.z;
    const float s2 = hl.x * hl.x + hl.y * hl.y;
    const float VoH = dot(P.Vl, hl);
    const float D = ggx_D(NoH, s2, P.a2);
    const float pcos = NoL * kInvPi;
    const float pggx = P.nov_pos ? P.G1V * D / (4.0f * P.nov) : 0.0f;
    // balance heuristic over the techniques in use
    const float Pt = FROZEN ? Pt_frozen : S.pL + P.bsdf_w * (P.q * pcos + (1.0f - P.q) * pggx);
    const float w = Hv / Pt;
    float3 L;
    float pdf_uv = 0.0f;   // nearest lookup: the texel's density (pdf table)
    if (BIL) {
        const Taps T = bilinear_taps(A.env, S.x, S.y);
        L = T.w[0] * texel_rgb(A.env, T.t[0]) + T.w[1] * texel_rgb(A.env, T.t[1]) +
            T.w[2] * texel_rgb(A.env, T.t[2]) + T.w[3] * texel_rgb(A.env, T.t[3]);
    } else {
        // the forward keeps the texel from the draw; the adjoint, short of
        // registers, reads it again
        const float4 tx = BWD ? A.env.tex[S.texel] : S.tx;
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

// bit k of the result = bit 2k of x (k < 16)
__device__ __forceinline__ uint32_t even_bits(uint32_t x) {
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return x;
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
    uint32_t lw = 0u;   // live bits of the current word
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
                if (tech == 0) has = light_on && draw_light<kDrawGen>(A, P, s_marg, r0, S);
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
                lw |= 1u << (slot & 31);
                ++c_rays;
            }
        }
        if (A.live && active && ((s & 15) == 15 || s == spp - 1)) {
            A.live[(s >> 4) * N + pix] = lw;
            lw = 0u;
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
// Binary walk: pre-order with skip links, one 16-byte node per step, no stack.
template <bool COUNT>
__device__ __forceinline__ void trace_tile_binary(const ShadeArgs& A, int64_t tile, const float4* R, int count,
                                                  uint32_t* hitbits, int* s_next) {
    const Scene& sc = A.scene;
    const int64_t N = A.g.n;
    const int64_t base_pix = tile * kBlock;
    const int n_total = sc.nodes[0].escape;
    const uint32_t n_tris = (uint32_t)sc.n_tris;
    const QFrame F = *sc.frame;
    const char* tri_bytes = reinterpret_cast<const char*>(sc.tris);
    const __amdgpu_buffer_rsrc_t qrs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)sc.qnodes, (short)0, (int)((uint32_t)n_total * 16u), kBufferWord3);
    const int lane = __lane_id();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    bool active = false, exhausted = false;
    Ray ray;
    QRay qray;
    int node = n_total;
    uint32_t p0 = 0u, p1 = 0u;
    uint32_t tag = 0u;     // the ray's pixel within the tile | sample slot << 8
    uint32_t c_hits = 0, c_box = 0, c_tri = 0, c_bstep = 0, c_tstep = 0;   // steps: lane 0 only
    uint32_t c_blane = 0;
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
                    tag = __float_as_uint(rr.w);
                    const float4 o = A.origins[base_pix + (tag & 255u)];
                    ray = make_ray(f3(o.x, o.y, o.z), f3(rr.x, rr.y, rr.z));
                    qray = make_qray(ray, F);
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
                if (COUNT && walking) ++c_blane;
                if (walking) {
                    // one 16-byte load per node: the quantised box and the link
                    const uint4 n = __builtin_bit_cast(
                        uint4, __builtin_amdgcn_raw_buffer_load_b128(qrs, (uint32_t)node * 16u, 0, 0));
                    const bool leaf = (n.w & kQLeaf) != 0u;
                    if (COUNT) ++c_box;
                    const bool hit = qbox_hit(qray, n);
                    // skip links point forward; max() keeps every walk finite
                    const int next = leaf ? node + 1 : max((int)n.w, node + 1);
                    node = (hit && !leaf) ? node + 1 : next;
                    const uint32_t payload = n.w & ~kQLeaf;
                    const bool take = hit && leaf;
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
                    const uint32_t slot = tag >> 8;
                    atomicOr(hitbits + (int64_t)(slot >> 5) * N + base_pix + (tag & 255u), 1u << (slot & 31));
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
        const uint32_t h = wave_sum(c_hits), bx = wave_sum(c_box), tr = wave_sum(c_tri), bl = wave_sum(c_blane);
        if (lane == 0) {
            atomicAdd(&A.stats->box_lanes, (unsigned long long)bl);
            atomicAdd(&A.stats->rays_hit, (unsigned long long)h);
            atomicAdd(&A.stats->box_tests, (unsigned long long)bx);
            atomicAdd(&A.stats->tri_tests, (unsigned long long)tr);
            atomicAdd(&A.stats->box_slots, 64ull * c_bstep);
            atomicAdd(&A.stats->tri_slots, 64ull * c_tstep);
        }
    }
}

// Pending references of the wide traversal, per lane, in LDS: entry k of
// the workgroup's lane t at [k * kBlock + t] (lanes of a wave hit distinct
// banks whatever their stack depths).  kStack entries, and four spare rows
// for the stores of a visit that begins with a full stack (18 KB per
// workgroup: eight workgroups per CU still fit).
constexpr int kStack = 14, kStackRows = kStack + 4;

template <bool COUNT>
__device__ __forceinline__ void trace_tile_wide(const ShadeArgs& A, int64_t tile, const float4* R, int count,
                                                uint32_t* hitbits, int* s_next, uint32_t* s_stack) {
    const Scene& sc = A.scene;
    const int64_t N = A.g.n;
    const int64_t base_pix = tile * kBlock;
    const int n_total = sc.nodes[0].escape;
    const uint32_t n_tris = (uint32_t)sc.n_tris;
    const QFrame F = *sc.frame;
    const char* tri_bytes = reinterpret_cast<const char*>(sc.tris);
    // nodes as buffer resources: 32-bit offsets, and a load past the end
    // returns zeros instead of reading out of bounds
    const __amdgpu_buffer_rsrc_t qrs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)sc.qnodes, (short)0, (int)((uint32_t)n_total * 16u), kBufferWord3);
    const __amdgpu_buffer_rsrc_t grs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)sc.groups, (short)0, (int)sc.group_bytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t ors = __builtin_amdgcn_make_buffer_rsrc(
        (void*)sc.gorder, (short)0, (int)(sc.group_bytes / 16u), kBufferWord3);
    uint32_t* stk = s_stack + threadIdx.x;
    const int lane = __lane_id();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    bool active = false, exhausted = false;
    Ray ray;
    QRay qray;
    uint32_t oct3 = 0u;    // 3 x the ray's octant (bit a: negative on axis a)
    // wide: node = a wide node, a leaf reference waiting for a pending slot,
    // or kWideNone (done); binary (after a stack overflow): a node index, done
    // at n_total
    bool wide = false;
    uint32_t node = (uint32_t)n_total;
    int sp = 0;
    // (every wide walk ends: the builder checked that each internal child
    // reference is larger than its parent's index and smaller than the node
    // count, and picks the binary walk for the scene otherwise)
    uint32_t p0 = 0u, p1 = 0u;
    uint32_t tag = 0u;     // the ray's pixel within the tile | sample slot << 8
    uint32_t c_hits = 0, c_box = 0, c_tri = 0, c_bstep = 0, c_tstep = 0;   // steps: lane 0 only
    uint32_t c_blane = 0;
    // scheduling knobs: refill batch, node steps per phase check, and the
    // phase hand-over ratios (in halves)
    // (measured on the lattice: refills of 16 lanes, three visits per phase
    // check and a triangle phase that yields only to twice as many idle
    // walkers as testers take the walk from 31.9 to 29.8 ms; refills of 48
    // lanes cost 13%; with the big-triangle subtree, a box phase that hands
    // over once the lanes stuck on leaves are half as many as the walkers
    // 11.9 -> 11.6 ms, and four visits per phase check 11.4 -> 11.1 ms)
    constexpr int kRefillMin = 16, kBoxSteps = 4, kBoxSwitch2 = 1, kTriSwitch2 = 4;
    auto walkable = [&]() { return (wide ? node != kWideNone : node < (uint32_t)n_total) && p1 == 0u; };
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
                    tag = __float_as_uint(rr.w);
                    const float4 o = A.origins[base_pix + (tag & 255u)];
                    ray = make_ray(f3(o.x, o.y, o.z), f3(rr.x, rr.y, rr.z));
                    qray = make_qray(ray, F);
                    oct3 = 3u * ((rr.x < 0.0f ? 1u : 0u) | (rr.y < 0.0f ? 2u : 0u) | (rr.z < 0.0f ? 4u : 0u));
                    wide = true;
                    node = 0u;
                    sp = 0;
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
        // walk is not finished (a leaf found with the first slot taken goes
        // to the second); the phase ends once the lanes that hold a leaf and
        // cannot walk are at least as many as the lanes still walking
        while (true) {
            if (!__any(active && walkable())) break;
#pragma unroll
            for (int step = 0; step < kBoxSteps; ++step) {
                const bool walking = active && walkable();
                if (COUNT && __any(walking) && lane == 0) ++c_bstep;
                if (COUNT && walking) ++c_blane;
                if (walking && wide) {
                    if (node & kQLeaf) {
                        // a leaf reference: to the free pending slot
                        const uint32_t payload = node & ~kQLeaf;
                        if (p0 == 0u) p0 = payload;
                        else p1 = payload;
                        node = sp > 0 ? (stk[--sp * kBlock] & ~kRefLive) : kWideNone;
                    } else {
                        // one wide node: four child records from one 64-byte
                        // segment, and its visit order for the ray's octant
                        const uint32_t off = node * 64u;
                        uint4 c[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            c[k] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(grs, off + 16u * k, 0, 0));
                        const uint32_t f = (__builtin_amdgcn_raw_buffer_load_b32(ors, node * 4u, 0, 0) >> oct3) & 7u;
                        // a missed child's reference becomes 0 (no kRefLive
                        // bit: the push below does not keep it)
                        uint32_t w[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            if (COUNT && (c[k].w & ~kRefLive) != kQLeaf) ++c_box;
                            w[k] = qbox_hit(qray, c[k]) ? c[k].w : 0u;
                        }
                        // farther child of each split after the nearer one
                        // (the pushed-last is popped first): within each pair,
                        // then the pairs
                        const bool s0 = (f & 1u) != 0u, s1 = (f & 2u) != 0u, sT = (f & 4u) != 0u;
                        const uint32_t a0 = s0 ? w[1] : w[0], a1 = s0 ? w[0] : w[1];
                        const uint32_t a2 = s1 ? w[3] : w[2], a3 = s1 ? w[2] : w[3];
                        const uint32_t ws[4] = {sT ? a2 : a0, sT ? a3 : a1, sT ? a0 : a2, sT ? a1 : a3};
                        // every hit child is pushed: each record is stored at
                        // the first free row and the row is kept if the child
                        // was hit (rows up to kStack + 3 exist, so a visit
                        // starting with a full stack stays in bounds; the
                        // overflow is checked once per visit); then the top is
                        // popped as the next node
                        int row = sp;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            stk[row * kBlock] = ws[k];
                            row += (int)((ws[k] & kRefLive) >> 30);
                        }
                        sp = row;
                        const bool over = sp > kStack;
                        const uint32_t top = stk[(sp > 0 ? sp - 1 : 0) * kBlock] & ~kRefLive;
                        const uint32_t next = sp > 0 ? top : kWideNone;
                        sp = sp > 0 ? sp - 1 : 0;
                        node = next;
                        if (!over && next != kWideNone && (next & kQLeaf)) {
                            // a leaf reference on top goes to a pending slot
                            // now (this visit started with the second free),
                            // and the next entry is popped
                            const uint32_t payload = next & ~kQLeaf;
                            if (p0 == 0u) p0 = payload;
                            else p1 = payload;
                            node = sp > 0 ? (stk[--sp * kBlock] & ~kRefLive) : kWideNone;
                        }
                        if (over) {
                            // the stack is full: walk the binary tree from the
                            // root instead (the same answer, more steps)
                            wide = false;
                            node = 0u;
                            sp = 0;
                        }
                    }
                } else if (walking) {
                    // binary pre-order walk with skip links: one 16-byte node
                    const uint4 n = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(qrs, node * 16u, 0, 0));
                    const bool leaf = (n.w & kQLeaf) != 0u;
                    if (COUNT) ++c_box;
                    const bool hit = qbox_hit(qray, n);
                    // skip links point forward; max() keeps every walk finite
                    const uint32_t next = leaf ? node + 1u : max(n.w, node + 1u);
                    node = (hit && !leaf) ? node + 1u : next;
                    const uint32_t payload = n.w & ~kQLeaf;
                    const bool take = hit && leaf;
                    const bool first_free = p0 == 0u;
                    p0 = (take && first_free) ? payload : p0;
                    p1 = (take && !first_free) ? payload : p1;
                }
            }
            const bool walk = active && walkable();
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
                    const uint32_t slot = tag >> 8;
                    atomicOr(hitbits + (int64_t)(slot >> 5) * N + base_pix + (tag & 255u), 1u << (slot & 31));
                    ++c_hits;
                    active = false;
                    wide = false;
                    node = (uint32_t)n_total;
                    sp = 0;
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
            const bool idle = !testing && active && walkable();
            if (2 * __popcll(__ballot(idle)) > kTriSwitch2 * __popcll(__ballot(testing))) break;
        }
        if (active && p0 == 0u && !(wide ? node != kWideNone : node < (uint32_t)n_total)) active = false;  // miss
    }
    if (COUNT) {
        const uint32_t h = wave_sum(c_hits), bx = wave_sum(c_box), tr = wave_sum(c_tri), bl = wave_sum(c_blane);
        if (lane == 0) {
            atomicAdd(&A.stats->box_lanes, (unsigned long long)bl);
            atomicAdd(&A.stats->rays_hit, (unsigned long long)h);
            atomicAdd(&A.stats->box_tests, (unsigned long long)bx);
            atomicAdd(&A.stats->tri_tests, (unsigned long long)tr);
            atomicAdd(&A.stats->box_slots, 64ull * c_bstep);
            atomicAdd(&A.stats->tri_slots, 64ull * c_tstep);
        }
    }
}

// The walk the scene's builder chose (a uniform branch: one scalar load).
template <bool COUNT>
__device__ __forceinline__ void trace_tile(const ShadeArgs& A, int64_t tile, const float4* R, int count,
                                           uint32_t* hitbits, int* s_next, uint32_t* s_stack) {
    if (A.scene.info->wide) trace_tile_wide<COUNT>(A, tile, R, count, hitbits, s_next, s_stack);
    else trace_tile_binary<COUNT>(A, tile, R, count, hitbits, s_next);
}

// 3) evaluation: forward values or the adjoint, from the hit bits.  For the
//    adjoint, s_hot must be zeroed before and flushed after (hot_flush).
//    BIL: bilinear probe lookup (MCDI_FLAG_BILINEAR) instead of the nearest
//    texel.
// words per sample of the decision dump: 3, or 9 with the sampled world
// directions (MCDI_FLAG_DUMP_DIRS)
constexpr uint32_t kNanBits = 0x7FC00000u;
__device__ __forceinline__ int dump_stride(const ShadeArgs& A) { return (A.flags & MCDI_FLAG_DUMP_DIRS) ? 9 : 3; }

// FROZEN (forward only): samples, densities, lobe choice and visibility from
// the G-buffer A.g, the samples evaluated with the planes A.e_*.
// LOCKSTEP: the lanes step through every sample pair together, skipping a pair
// blocked twice over in place (the persistent serving kernel, whose launches
// ran a quarter slower with the per-lane walk below).
template <bool BWD, bool DUMP, bool BIL, bool FROZEN = false, bool LOCKSTEP = false>
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
    Pixel Pe;
    if (FROZEN) {
        ShadeArgs Ae = A;
        Ae.g.nrm = A.e_nrm;
        Ae.g.kd = A.e_kd;
        Ae.g.korm = A.e_korm;
        bool nf;
        Pe = setup_pixel(Ae, pix, nf);
    }
    if (!P.valid || (FROZEN && !Pe.valid)) {
        if (!BWD) {
            for (int c = 0; c < 3; ++c) { A.c_d[c * N + pix] = 0.0f; A.c_s[c * N + pix] = 0.0f; }
        } else {
            for (int c = 0; c < 3; ++c) {
                A.g_kd[c * N + pix] = 0.0f; A.g_korm[c * N + pix] = 0.0f; A.g_nrm[c * N + pix] = 0.0f;
            }
        }
        if (DUMP) {
            const int st = dump_stride(A);
            uint32_t* d = A.decisions + (size_t)pix * spp * st;
            for (int s = 0; s < spp; ++s) {
                d[st * s] = kNone; d[st * s + 1] = kNone; d[st * s + 2] = 0u;
                for (int k = 3; k < st; ++k) d[st * s + k] = kNanBits;
            }
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
    // With tau = 1 a blocked sample is weighted by H = 0 and adds nothing
    // (the incident radiance is the probe's times H, appendix A): its hit
    // bit (set only for a traced, blocked ray) skips it before it is drawn.
    // A lane walks only its pixel's sample pairs that are not blocked twice
    // over (in increasing order, so the sums are those of the full loop), so
    // a wavefront runs as many pair steps as its busiest lane rather than
    // spp.  The decision dump draws every sample and skips only the
    // evaluation.
    const bool skip_blocked = !DUMP && A.tau == 1.0f;
    if (!DUMP && !FROZEN && !LOCKSTEP && A.live) {
        // the live bits name the samples the estimator evaluates: a lane
        // draws and evaluates only those (and with tau = 1 only those not
        // blocked), pair by pair in the same increasing (sample, technique)
        // order; the two samples of a pair share the first Philox block
        for (int s0 = 0; s0 < spp; s0 += 16) {
            const uint32_t bits = A.hitbits_in[(s0 >> 4) * N + pix];
            uint32_t need = A.live[(s0 >> 4) * N + pix];
            if (skip_blocked) need &= ~bits;
            uint32_t todo = even_bits(need | (need >> 1));
            while (todo) {
                const int k = __ffs(todo) - 1;
                todo &= todo - 1u;
                const int s = s0 + k;
                const uint32_t pair = need >> (2 * k), hit = bits >> (2 * k);
                const uint4 r0 = philox10(make_uint4(piv, vid, (uint32_t)s, 0u), k0, k1);
                if (pair & 1u) {
                    Sample S;
                    draw_light<BWD ? kDrawBwd : kDrawFwd>(A, P, s_marg, r0, S);
                    const float Hv = (hit & 1u) ? 1.0f - A.tau : 1.0f;
                    eval_sample<BWD, BIL>(A, P, S, Hv, invspp, fa, ba, Ud, Us, s_hot, rs);
                }
                if (pair & 2u) {
                    Sample S;
                    const uint4 r1 = philox10(make_uint4(piv, vid, (uint32_t)s, 1u), k0, k1);
                    draw_bsdf(P, r0, r1, S);
                    bsdf_texel<!BWD>(A, light_on, S);
                    const float Hv = (hit & 2u) ? 1.0f - A.tau : 1.0f;
                    eval_sample<BWD, BIL>(A, P, S, Hv, invspp, fa, ba, Ud, Us, s_hot, rs);
                }
            }
        }
    } else {
        for (int s0 = 0; s0 < spp; s0 += 16) {
            const uint32_t bits = A.hitbits_in[(s0 >> 4) * N + pix];   // pairs s0 .. s0 + 15
            uint32_t todo = (spp - s0 >= 16) ? 0xFFFFu : (1u << (spp - s0)) - 1u;
            if (skip_blocked && !LOCKSTEP) todo &= ~even_bits(bits & (bits >> 1));
            while (todo) {
                const int s = s0 + __ffs(todo) - 1;
                todo &= todo - 1u;
                if (LOCKSTEP && skip_blocked && ((bits >> ((2 * s) & 31)) & 3u) == 3u) continue;
                const uint4 r0 = philox10(make_uint4(piv, vid, (uint32_t)s, 0u), k0, k1);
                const uint4 r1 = philox10(make_uint4(piv, vid, (uint32_t)s, 1u), k0, k1);
                uint32_t rec0 = kNone, rec1 = kNone;
                uint32_t rec2 = kDecValid | (P.nov_pos ? kDecNovPos : 0u);
                float3 dir[2] = {f3(__uint_as_float(kNanBits), 0.0f, 0.0f), f3(__uint_as_float(kNanBits), 0.0f, 0.0f)};
                for (int tech = 0; tech < 2; ++tech) {
                    if (skip_blocked && ((bits >> ((2 * s + tech) & 31)) & 1u)) continue;
                    Sample S;
                    if (tech == 0) {
                        if (!light_on) continue;
                        const bool has = draw_light<BWD ? kDrawBwd : kDrawFwd>(A, P, s_marg, r0, S);
                        rec0 = (uint32_t)S.texel;
                        if (DUMP) dir[0] = S.w;
                        if (!has) { rec2 |= kDecLCull; continue; }
                    } else {
                        if (P.bsdf_w == 0.0f) continue;
                        if (draw_bsdf(P, r0, r1, S)) rec2 |= kDecLobeCos;
                        if (DUMP) dir[1] = S.w;
                    }
                    if (!(S.wl.z > 0.0f)) { rec2 |= tech ? kDecBCull : kDecLCull; continue; }
                    if (tech == 1) {
                        bsdf_texel<!BWD>(A, light_on, S);
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
                    // H = 0: no incident radiance, whatever the probe holds there
                    if (Hv == 0.0f) continue;
                    if (FROZEN) {
                        // the sample's direction in the evaluation frame (the
                        // sampled local direction itself where the frame is the same)
                        Sample Se = S;
                        if (!(Pe.n.x == P.n.x && Pe.n.y == P.n.y && Pe.n.z == P.n.z))
                            Se.wl = f3(dot(S.w, Pe.t), dot(S.w, Pe.b), dot(S.w, Pe.n));
                        eval_sample<BWD, BIL, true>(A, Pe, Se, Hv, invspp, fa, ba, Ud, Us, s_hot, rs, mis_density(P, S));
                    } else {
                        eval_sample<BWD, BIL>(A, P, S, Hv, invspp, fa, ba, Ud, Us, s_hot, rs);
                    }
                }
                if (DUMP) {
                    const int st = dump_stride(A);
                    uint32_t* d = A.decisions + ((size_t)pix * spp + s) * st;
                    d[0] = rec0; d[1] = rec1; d[2] = rec2;
                    if (st == 9) {
                        for (int t = 0; t < 2; ++t) {
                            d[3 + 3 * t] = __float_as_uint(dir[t].x);
                            d[4 + 3 * t] = __float_as_uint(dir[t].y);
                            d[5 + 3 * t] = __float_as_uint(dir[t].z);
                        }
                    }
                }
            }
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

// eight waves per SIMD (the hardware's limit): 64 registers per lane
template <bool COUNT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void trace_rays_kernel(ShadeArgs A,
                                                                                                   uint32_t* hitbits) {
    __shared__ int s_next;
    __shared__ uint32_t s_stack[kStackRows * kBlock];
    const int64_t tile = A.tile_order ? A.tile_order[blockIdx.x] : blockIdx.x;
    if (tile < 0 || tile >= (int64_t)gridDim.x) return;   // uniform: the whole workgroup reads the same entry
    if (threadIdx.x == 0) s_next = 0;
    __syncthreads();
    trace_tile<COUNT>(A, tile, tile_region(A, tile), A.ray_count[tile], hitbits, &s_next, s_stack);
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

// forward with frozen sampling (a test instantiation: finite differences of
// the estimator with its samples held fixed)
template <bool BIL>
__global__ __launch_bounds__(kBlock) void shade_frozen_kernel(ShadeArgs A) {
    extern __shared__ float smem[];
    stage_marg(A, smem);
    __syncthreads();
    shade_tile<false, false, BIL, true>(A, blockIdx.x, smem, nullptr, RecSink{nullptr, nullptr});
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void shade_bwd_bilinear_kernel(ShadeArgs A) {
    shade_body<true, false, true>(A);
}

// ---------------------------------------------------------------------------
// Serving: one persistent launch over the tiles of many requests.  Every
// workgroup takes the next tile from a global counter and runs generation,
// traversal, the forward evaluation and (for gradient requests) the adjoint
// on it; it stops when the tiles run out, so every wave exits.  Four waves
// per SIMD (128 VGPRs, 84 bytes spilled): left to itself the compiler takes
// 171 registers for the adjoint's stretch and the whole launch runs at two
// waves, the traversal's included; on the serving mix four waves served 16%
// more requests per second, five and six (more spills) fewer.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void serve_kernel(const ServeItem* items, int n_items, int64_t total_tiles,
                                                       int* tile_counter, float4* scratch, int spp_max) {
    extern __shared__ float smem[];
    __shared__ int s_tile, s_item, s_cnt, s_next;
    __shared__ uint32_t s_stack[kStackRows * kBlock];
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
        if (reg) trace_tile<false>(A, tile, reg, s_cnt, it.hitbits, &s_next, s_stack);
        __syncthreads();
        const bool bil = (A.flags & MCDI_FLAG_BILINEAR) != 0;
        if (bil) shade_tile<false, false, true, false, true>(A, tile, s_marg, s_hot, RecSink{nullptr, nullptr});
        else shade_tile<false, false, false, false, true>(A, tile, s_marg, s_hot, RecSink{nullptr, nullptr});
        if (A.g_cd) {
            hot_zero(s_hot);
            __syncthreads();
            if (bil) shade_tile<true, false, true, false, true>(A, tile, s_marg, s_hot, RecSink{nullptr, nullptr});
            else shade_tile<true, false, false, false, true>(A, tile, s_marg, s_hot, RecSink{nullptr, nullptr});
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
    bool h;
    if (brute == 1) h = brute_anyhit(sc, r);
    else if (brute == 2) h = wbvh_anyhit(sc, r, n_total, nb, nt);
    else h = qbvh_anyhit(sc, r, n_total, nb, nt);
    hit[k] = h ? 1 : 0;
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

hipError_t launch_shade_fwd_frozen(const ShadeArgs& a, hipStream_t s) {
    const dim3 g(n_blocks(a)), b(kBlock);
    if (a.flags & MCDI_FLAG_BILINEAR) hipLaunchKernelGGL(shade_frozen_kernel<true>, g, b, marg_lds(a), s, a);
    else hipLaunchKernelGGL(shade_frozen_kernel<false>, g, b, marg_lds(a), s, a);
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

}  // namespace mcdi
