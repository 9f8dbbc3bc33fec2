// Device building blocks for gfx950: counter-based RNG, probe sampling, GGX
// material model, visible-normal sampling and the any-hit BVH traversal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mcdi_internal.h"

namespace mcdi {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvPi = 0.318309886183790671538f;
constexpr float kRMin = 0.08f;  // roughness clamp (alpha >= 0.0064)
// Word 3 of a raw buffer resource on gfx9 (data format 32, no swizzle): the
// descriptor of __builtin_amdgcn_make_buffer_rsrc for plain byte-offset loads.
constexpr int kBufferWord3 = 0x00020000;
constexpr uint32_t kNone = 0xFFFFFFFFu;

// decision-record bits (debug dump)
constexpr uint32_t kDecLobeCos = 1u << 0, kDecLCull = 1u << 1, kDecBCull = 1u << 2;
constexpr uint32_t kDecLTraced = 1u << 3, kDecBTraced = 1u << 4, kDecLHit = 1u << 5;
constexpr uint32_t kDecBHit = 1u << 6, kDecNovPos = 1u << 7, kDecValid = 1u << 8;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC 2011): ten rounds of two 32x32 products.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
    // each 32 x 32 -> 64-bit product as one multiply (both halves at once)
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// top 24 bits as a float in [0, 1), exact
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

// ---------------------------------------------------------------------------
// small vector helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float dot(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator*(float s, float3 a) { return f3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float3 normalize(float3 a) { return (1.0f / sqrtf(dot(a, a))) * a; }

// ---------------------------------------------------------------------------
// binary search: largest k in [0, n-1] with cdf[k] <= x (cdf[0] = 0 <= x <
// 1 = cdf[n], non-decreasing) -- skips zero-width bins.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cdf_find(const float* cdf, int n, float x) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// The same search with the row's guide (guide[g] = cdf_find(cdf, n, g / G),
// g = 0..G, G a power of two): for x in [0, 1) with g = floor(x G), the
// answer lies in [guide[g], guide[g + 1]], since g / G <= x < (g + 1) / G and
// both bounds are exact in FP32; the binary search over that range returns
// the same column as cdf_find.
__device__ __forceinline__ int cdf_find_guided(const float* cdf, const int32_t* guide, int G, float x) {
    const int g = min(max((int)(x * (float)G), 0), G - 1);
    int lo = guide[g], hi = guide[g + 1] + 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// The guided search of one conditional row with the candidates read in one
// go, and the CDF values on both sides of the answer (c0 = cdf[j],
// c1 = cdf[j + 1]).  Four aligned 16-byte loads, issued together, cover the
// 13 to 16 entries from the cell's first candidate on.  When the cell's
// candidates fit, the answer is the first candidate plus the number of later
// candidates (below the cell's end) that are <= x, which over a
// non-decreasing CDF is the binary search's answer; otherwise the binary
// search runs, mostly over the lines just read.  One round trip for the
// candidates instead of one per probe: with many waves in flight a line read
// by one probe is often evicted before the next (cdf_find_guided's probes
// then each go to memory).  The row must be 4-byte aligned within a 16-byte
// aligned table that extends at least 16 floats past the row's last entry.
__device__ __forceinline__ int cdf_find_row(const float* cdf, const int32_t* guide, int G, float x, float& c0,
                                            float& c1) {
    constexpr int NQ = 4, NW = 4 * NQ;
    const int g = min(max((int)(x * (float)G), 0), G - 1);
    int lo = guide[g], hi = guide[g + 1] + 1;
    const float* p = cdf + lo;
    const int o = (int)(((uintptr_t)p >> 2) & 3u);
    const float4* a = (const float4*)(p - o);
    float w[NW];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const float4 v = a[q];
        w[4 * q] = v.x; w[4 * q + 1] = v.y; w[4 * q + 2] = v.z; w[4 * q + 3] = v.w;
    }
    if (hi - lo <= NW - 1 - o) {
        // window slot t holds cdf[lo - o + t]; the answer's slot is o + cnt
        const int span = hi - lo;
        int cnt = 0;
#pragma unroll
        for (int t = 1; t < NW; ++t) {
            const int k = t - o;   // offset from lo
            cnt += (k >= 1 && k < span && w[t] <= x) ? 1 : 0;
        }
        const int s0 = o + cnt;
        float v0 = w[0], v1 = w[1];
#pragma unroll
        for (int t = 1; t < NW; ++t) {
            v0 = (t == s0) ? w[t] : v0;
            v1 = (t == s0 + 1) ? w[t] : v1;
        }
        c0 = v0;
        c1 = v1;
        return lo + cnt;
    }
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] <= x) lo = mid; else hi = mid;
    }
    c0 = cdf[lo];
    c1 = cdf[lo + 1];
    return lo;
}

// ---------------------------------------------------------------------------
// GGX with Smith height-correlated masking (alpha = roughness^2)
// ---------------------------------------------------------------------------
// D written with s2 = |n x h|^2 (local: h.x^2 + h.y^2) for 1 - (n.h)^2
__device__ __forceinline__ float ggx_D(float noh, float s2, float a2) {
    const float den = a2 * noh * noh + s2;
    return a2 / (kPi * den * den);
}

__device__ __forceinline__ float smith_t2(float x) { return (1.0f - x * x) / (x * x); }

__device__ __forceinline__ float smith_lambda(float t2, float a2) {
    return 0.5f * (sqrtf(1.0f + a2 * t2) - 1.0f);
}

// ---------------------------------------------------------------------------
// Watertight ray/triangle test (Woop, Benthin, Wald; JCGT 2013), any hit with
// t in (0, inf).  The ray is pre-sheared: kz is the dominant axis of d and the
// rows M* give the sheared coordinates of (v - o).  Edge functions use no
// contraction so a shared edge gives exactly negated values in its two
// triangles; an exactly-zero edge function is re-evaluated in FP64.
// ---------------------------------------------------------------------------
struct Ray {
    float3 o;
    float3 inv;      // 1/d (zero components replaced, boxes only)
    float3 clo, chi; // slab offsets for the low and high box corners (box_hit)
    float3 mx, my;   // shear rows
    float sz;        // 1/d[kz]
    int kz;
};

// Slab offsets: t = corner * inv + c with c = -(o * inv) -/+ e on the near/far
// side of each axis.  o*inv is rounded once, so e = 2^-21 |o*inv| (eight times
// that rounding plus the rounding of c itself) keeps every near distance an
// under- and every far distance an over-estimate before the final rounding of
// the FMA.
__device__ __forceinline__ void slab_offsets(float o, float inv, float& clo, float& chi) {
    const float oi = o * inv;
    const float e = fabsf(oi) * 0x1p-21f;
    const float cn = -oi - e, cf = -oi + e;
    clo = inv >= 0.0f ? cn : cf;
    chi = inv >= 0.0f ? cf : cn;
}

__device__ __forceinline__ float comp(float3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

// Reciprocals use the hardware approximation (<= 1 ulp): the shear constants
// only need to be the same for every triangle a ray meets, and the box test
// widens t_far for the extra ulp.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ Ray make_ray(float3 o, float3 d) {
    Ray r;
    r.o = o;
    const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    const float dz = comp(d, kz);
    if (dz < 0.0f) { const int t = kx; kx = ky; ky = t; }
    const float rz = fast_rcp(dz);
    const float sx = comp(d, kx) * rz, sy = comp(d, ky) * rz;
    r.sz = rz;
    r.kz = kz;
    // rows: e_kx - sx e_kz and e_ky - sy e_kz
    r.mx = f3(kx == 0 ? 1.f : 0.f, kx == 1 ? 1.f : 0.f, kx == 2 ? 1.f : 0.f);
    r.my = f3(ky == 0 ? 1.f : 0.f, ky == 1 ? 1.f : 0.f, ky == 2 ? 1.f : 0.f);
    if (kz == 0) { r.mx.x = -sx; r.my.x = -sy; }
    if (kz == 1) { r.mx.y = -sx; r.my.y = -sy; }
    if (kz == 2) { r.mx.z = -sx; r.my.z = -sy; }
    const float tiny = 1e-30f;
    r.inv = f3(fast_rcp(d.x != 0.0f ? d.x : tiny), fast_rcp(d.y != 0.0f ? d.y : tiny),
               fast_rcp(d.z != 0.0f ? d.z : tiny));
    slab_offsets(o.x, r.inv.x, r.clo.x, r.chi.x);
    slab_offsets(o.y, r.inv.y, r.clo.y, r.chi.y);
    slab_offsets(o.z, r.inv.z, r.clo.z, r.chi.z);
    return r;
}

__device__ __forceinline__ bool tri_anyhit(const Ray& r, float4 v0, float4 v1, float4 v2) {
#pragma clang fp contract(off)
    const float3 A = f3(v0.x, v0.y, v0.z) - r.o;
    const float3 B = f3(v1.x, v1.y, v1.z) - r.o;
    const float3 C = f3(v2.x, v2.y, v2.z) - r.o;
    const float az = comp(A, r.kz), bz = comp(B, r.kz), cz = comp(C, r.kz);
    // sheared x, y: component kx (ky) minus s * component kz
    const float Ax = dot(r.mx, A), Ay = dot(r.my, A);
    const float Bx = dot(r.mx, B), By = dot(r.my, B);
    const float Cx = dot(r.mx, C), Cy = dot(r.my, C);
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    const float det = U + V + W;
    if (det == 0.0f) return false;
    const float T = U * (r.sz * az) + V * (r.sz * bz) + W * (r.sz * cz);
    return det > 0.0f ? (T > 0.0f) : (T < 0.0f);
}

// Conservative slab test (Ize 2013: widen t_far by 1 + 2 gamma(n)), t >= 0;
// n = 4 covers the subtraction, the product and the 1-ulp reciprocal, and the
// factor is rounded up.
__device__ __forceinline__ bool box_hit(const Ray& r, float4 a, float4 b) {
    const float tx0 = fmaf(a.x, r.inv.x, r.clo.x), tx1 = fmaf(b.x, r.inv.x, r.chi.x);
    const float ty0 = fmaf(a.y, r.inv.y, r.clo.y), ty1 = fmaf(b.y, r.inv.y, r.chi.y);
    const float tz0 = fmaf(a.z, r.inv.z, r.clo.z), tz1 = fmaf(b.z, r.inv.z, r.chi.z);
    const float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
    const float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
    return tn <= tf * 1.000001f;
}

// Slab constants of a ray against the scene's quantisation frame: the plane q
// of axis a lies at base + q step, so t = q (step inv) + (base - o) inv, one
// FMA per plane.  The offsets carry a margin of 2^-20 (65535 |step inv| +
// |(base - o) inv|) -- sixteen times the roundings of the two products, the
// difference and the FMA against the magnitudes involved -- on the side that
// keeps near distances under- and far distances over-estimated; they also
// cover the reciprocal's 1-ulp error, so the final comparison needs no slack.
// Which plane of an axis is near follows from the sign of the direction: per
// axis a byte selector gathers the near plane's 16-bit coordinate (low half)
// and the far plane's (high half) from the two words holding them, so that
// the test needs no min/max pairs.
struct QRay {
    float3 s, cn, cf;
    uint32_t sx, sy, sz;
};

__device__ __forceinline__ void qslab(float o, float inv, float base, float step, float& s, float& cn,
                                      float& cf) {
    s = step * inv;
    const float c = (base - o) * inv;
    const float e = 0x1p-20f * (fabsf(s) * 65535.0f + fabsf(c));
    cn = c - e;
    cf = c + e;
}

__device__ __forceinline__ QRay make_qray(const Ray& r, const QFrame& F) {
    QRay q;
    qslab(r.o.x, r.inv.x, F.base[0], F.step[0], q.s.x, q.cn.x, q.cf.x);
    qslab(r.o.y, r.inv.y, F.base[1], F.step[1], q.s.y, q.cn.y, q.cf.y);
    qslab(r.o.z, r.inv.z, F.base[2], F.step[2], q.s.z, q.cn.z, q.cf.z);
    // x: lo in word 0 of n.x, hi in word 1 of n.y; y: lo in word 1 of n.x,
    // hi in word 0 of n.z; z: lo in word 0 of n.y, hi in word 1 of n.z
    // (selector bytes 0-3 take the second operand, 4-7 the first)
    q.sx = r.inv.x >= 0.0f ? 0x07060100u : 0x01000706u;
    q.sy = r.inv.y >= 0.0f ? 0x05040302u : 0x03020504u;
    q.sz = r.inv.z >= 0.0f ? 0x07060100u : 0x01000706u;
    return q;
}

__device__ __forceinline__ bool qbox_hit(const QRay& q, uint4 n) {
    const uint32_t ax = __builtin_amdgcn_perm(n.y, n.x, q.sx);
    const uint32_t ay = __builtin_amdgcn_perm(n.z, n.x, q.sy);
    const uint32_t az = __builtin_amdgcn_perm(n.z, n.y, q.sz);
    const float tnx = fmaf((float)(ax & 0xFFFFu), q.s.x, q.cn.x), tfx = fmaf((float)(ax >> 16), q.s.x, q.cf.x);
    const float tny = fmaf((float)(ay & 0xFFFFu), q.s.y, q.cn.y), tfy = fmaf((float)(ay >> 16), q.s.y, q.cf.y);
    const float tnz = fmaf((float)(az & 0xFFFFu), q.s.z, q.cn.z), tfz = fmaf((float)(az >> 16), q.s.z, q.cf.z);
    const float tn = fmaxf(fmaxf(fmaxf(tnx, tny), tnz), 0.0f);
    const float tf = fminf(fminf(tfx, tfy), tfz);
    return tn <= tf;
}

// Stackless any-hit traversal over the quantised nodes (the order and the
// skip links of the pre-order BVH; a leaf's escape is the next node).
template <bool COUNT = false>
__device__ __forceinline__ bool qbvh_anyhit(const Scene& sc, const Ray& r, int n_total, uint32_t& n_box,
                                            uint32_t& n_tri) {
    const uint4* nodes = reinterpret_cast<const uint4*>(sc.qnodes);
    const QRay q = make_qray(r, *sc.frame);
    int i = 0;
    while (i < n_total) {
        const uint4 n = nodes[i];
        const bool leaf = (n.w & kQLeaf) != 0u;
        // skip links always point forward; anything else ends the walk
        const int next = leaf ? i + 1 : ((int)n.w > i ? (int)n.w : n_total);
        if (COUNT) ++n_box;
        if (!qbox_hit(q, n)) { i = next; continue; }
        if (!leaf) { ++i; continue; }
        const uint32_t payload = n.w & ~kQLeaf;
        const int first = (int)(payload >> 3);
        const int cnt = (first + (int)(payload & 7u) <= sc.n_tris) ? (int)(payload & 7u) : 0;
        for (int k = 0; k < cnt; ++k) {
            const float4* t = sc.tris + 3 * (first + k);
            if (COUNT) ++n_tri;
            if (tri_anyhit(r, t[0], t[1], t[2])) return true;
        }
        i = next;
    }
    return false;
}

// Any-hit traversal of the 4-wide hierarchy with a stack of pending
// references (a one-ray form; the shading kernels keep their stacks in LDS).
// Hit children are pushed in the node's visit order for the ray's octant and
// the last pushed is taken next, so each split's farther child comes first,
// as in the shading kernels' walk.  A stack that would overflow sends the ray
// to the binary traversal from the root, which gives the same answer.
template <bool COUNT = false>
__device__ __forceinline__ bool wbvh_anyhit(const Scene& sc, const Ray& r, int n_total, uint32_t& n_box,
                                            uint32_t& n_tri) {
    constexpr int kDepth = 64;
    const uint4* g = reinterpret_cast<const uint4*>(sc.groups);
    const uint32_t n_groups = sc.group_bytes / 64u;
    const QRay q = make_qray(r, *sc.frame);
    const uint32_t oct3 =
        3u * ((r.inv.x < 0.0f ? 1u : 0u) | (r.inv.y < 0.0f ? 2u : 0u) | (r.inv.z < 0.0f ? 4u : 0u));
    uint32_t stack[kDepth];
    int sp = 0;
    uint32_t node = n_total > 0 ? 0u : kWideNone;
    while (true) {
        if (node == kWideNone) {
            if (sp == 0) return false;
            node = stack[--sp];
        }
        if (node & kQLeaf) {
            const uint32_t payload = node & ~kQLeaf;
            const int first = (int)(payload >> 3);
            const int cnt = (first + (int)(payload & 7u) <= sc.n_tris) ? (int)(payload & 7u) : 0;
            for (int k = 0; k < cnt; ++k) {
                const float4* t = sc.tris + 3 * (first + k);
                if (COUNT) ++n_tri;
                if (tri_anyhit(r, t[0], t[1], t[2])) return true;
            }
            node = kWideNone;
            continue;
        }
        if (node >= n_groups) { node = kWideNone; continue; }   // never for a valid hierarchy
        const uint32_t f = (sc.gorder[node] >> oct3) & 7u;
        // slot order: swap within the first pair, within the second, the pairs
        for (int p = 0; p < 4; ++p) {
            int k = p;
            if (f & 4u) k ^= 2;
            if ((k < 2 && (f & 1u)) || (k >= 2 && (f & 2u))) k ^= 1;
            const uint4 c = g[4 * (size_t)node + k];
            if (COUNT && (c.w & ~kRefLive) != kQLeaf) ++n_box;
            if (!qbox_hit(q, c)) continue;
            if (sp >= kDepth) return qbvh_anyhit<COUNT>(sc, r, n_total, n_box, n_tri);
            stack[sp++] = c.w & ~kRefLive;
        }
        node = kWideNone;   // the last pushed is popped next
    }
}

// Stackless any-hit traversal over the pre-order BVH with skip links.
// COUNT: tally box tests and triangle tests (statistics instantiation only).
template <bool COUNT = false>
__device__ __forceinline__ bool bvh_anyhit(const Scene& sc, const Ray& r, int n_total, uint32_t& n_box,
                                           uint32_t& n_tri) {
    const float4* nodes = reinterpret_cast<const float4*>(sc.nodes);
    int i = 0;
    while (i < n_total) {
        const float4 a = nodes[2 * i];
        const float4 b = nodes[2 * i + 1];
        const int escape = __float_as_int(a.w);
        const int payload = __float_as_int(b.w);
        // skip links always point forward; anything else ends the walk
        const int next = escape > i ? escape : n_total;
        if (COUNT) ++n_box;
        if (!box_hit(r, a, b)) { i = next; continue; }
        if (payload == 0) { ++i; continue; }
        const int first = payload >> 3;
        const int cnt = (first + (payload & 7) <= sc.n_tris) ? (payload & 7) : 0;
        for (int k = 0; k < cnt; ++k) {
            const float4* t = sc.tris + 3 * (first + k);
            if (COUNT) ++n_tri;
            if (tri_anyhit(r, t[0], t[1], t[2])) return true;
        }
        i = next;
    }
    return false;
}

__device__ __forceinline__ bool brute_anyhit(const Scene& sc, const Ray& r) {
    for (int64_t k = 0; k < sc.n_tris; ++k) {
        const float4* t = sc.tris + 3 * k;
        if (tri_anyhit(r, t[0], t[1], t[2])) return true;
    }
    return false;
}

}  // namespace mcdi
