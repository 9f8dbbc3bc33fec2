// Edge-sampled visibility gradient of the shadow term on gfx950: a sample
// kernel that keeps the silhouette samples above the horizon of every pixel
// as 4-byte records, and a trace kernel that evaluates each kept sample, traces
// its out-side ray with a whole wavefront and scatters the term into the vertex
// gradient (paper: section 3.1 "Shadow gradients"; appendix "Visibility
// Gradients from Shadows").
#include <hip/hip_runtime.h>
#include <math.h>

#include "device_common.h"
#include "edge_internal.h"
#include "shade_common.h"

namespace mcdi {

namespace {

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
    bool sharp;          // its sampling class
    float t, s;          // point on the edge; +1 when the face lies on the +mh side
    float3 w, mh;        // unit direction to the point; unit arc normal
    float r2;            // squared distance to the point
    float3 eab;
};

// the sample's random numbers and its edge's corners, fetched in one go
struct EdgeFetch {
    uint32_t e;
    bool sharp;
    float t;
    float4 pa, pb, pc, pd;
};

// the sample's class (sharp edges are E.gain times as likely per edge: an
// exact integer test on the 24-bit uniform of x2), its edge (uniform in
// the class) and that edge's corners, packed in one 64-byte line (sharp
// edges first) for this call
__device__ __forceinline__ EdgeFetch edge_fetch(const EdgeArgs& E, uint32_t piv, uint32_t vid, int j, uint32_t ne,
                                                uint32_t ns) {
    const uint32_t k0 = (uint32_t)E.a.seed, k1 = (uint32_t)(E.a.seed >> 32);
    const uint4 r = philox10(make_uint4(piv, vid, (uint32_t)j, 2u), k0, k1);
    const uint64_t num = (uint64_t)E.gain * ns, den = num + (uint64_t)(ne - ns);
    EdgeFetch F;
    F.sharp = (uint64_t)(r.z >> 8) * den < (num << 24);
    const uint32_t line = (F.sharp ? 0u : ns) + __umulhi(r.x, F.sharp ? ns : ne - ns);
    F.t = u01(r.y);
    const float4* q = E.egeo + 4 * (size_t)line;
    F.pa = q[0];
    F.pb = q[1];
    F.pc = q[2];
    F.pd = q[3];
    F.e = __float_as_uint(F.pa.w);
    return F;
}

__device__ __forceinline__ bool edge_test(const Pixel& P, const EdgeFetch& F, EdgeGeom& G) {
    G.e = F.e;
    G.sharp = F.sharp;
    G.t = F.t;
    const float3 va = f3(F.pa.x, F.pa.y, F.pa.z);
    const float3 qa = va - P.o;
    G.eab = f3(F.pb.x, F.pb.y, F.pb.z) - va;
    const float3 m = cross(qa, G.eab);   // = (a - o) x (b - o)
    const float sc = dot(qa, cross(G.eab, f3(F.pc.x, F.pc.y, F.pc.z) - va));
    // the second face's side (its corner is zero without a second face)
    const float sd = dot(qa, cross(G.eab, f3(F.pd.x, F.pd.y, F.pd.z) - va));
    const float ml2 = dot(m, m);
    const float3 w = qa + G.t * G.eab;
    G.r2 = dot(w, w);
    G.w = (1.0f / sqrtf(G.r2)) * w;
    G.mh = (1.0f / sqrtf(ml2)) * m;
    G.s = sc > 0.0f ? 1.0f : -1.0f;
    // evaluated without branches, so that every load of the sample is issued
    // before any of its values is needed
    const bool covered = (F.pd.w != 0.0f) & (((sc > 0.0f) & (sd < 0.0f)) | ((sc < 0.0f) & (sd > 0.0f)));
    // a non-finite corner makes a side non-finite: no term
    return (sc != 0.0f) & isfinite(sc) & isfinite(sd) & !covered & (ml2 > 0.0f) & (dot(G.w, P.n) > 0.0f);
}

__device__ __forceinline__ bool edge_geom(const EdgeArgs& E, const Pixel& P, uint32_t piv, uint32_t vid, int j,
                                          uint32_t ne, uint32_t ns, EdgeGeom& G) {
    return edge_test(P, edge_fetch(E, piv, vid, j, ne, ns), G);
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
//    their loads overlap (eight waves per SIMD: the corner-line reads miss
//    L2 and need the waves in flight).  Each workgroup reserves the queue space of a chunk
//    with one atomic: the queue counter is a single address, and one atomic
//    per wave and sample serialises behind it when candidates are common.
__global__ __launch_bounds__(kBlock, 8) void edge_gen_kernel(EdgeArgs E) {
    constexpr int kWaves = kBlock / 64;
    __shared__ uint32_t s_wave[kWaves];
    __shared__ uint32_t s_base;
    const ShadeArgs& A = E.a;
    const int64_t local = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t pix = E.pix0 + local;
    const bool active = local < E.npix && pix < A.g.n;
    const uint32_t ne = *E.n_edges, ns = *E.n_sharp;
    bool nonfinite = false, valid = false;
    Pixel P;
    if (active) valid = pixel_origin(A, pix, P, nonfinite);
    const bool go = valid && ne > 0u && A.tau != 0.0f;
    const int64_t hw = (int64_t)A.g.height * A.g.width;
    const uint32_t view = active ? (uint32_t)(pix / hw) : 0u;
    const uint32_t piv = active ? (uint32_t)(pix - (int64_t)view * hw) : 0u;
    const uint32_t vid = (uint32_t)A.g.view_base + view;
    const int lane = __lane_id();
    const int wid = threadIdx.x >> 6;
    for (int j0 = 0; j0 < E.n_es; j0 += 32) {
        const int nj = E.n_es - j0 < 32 ? E.n_es - j0 : 32;
        uint32_t bits = 0u;
        if (go) {
            // two samples per step: both fetches are in flight before either test
            int jj = 0;
            for (; jj + 1 < nj; jj += 2) {
                const EdgeFetch F0 = edge_fetch(E, piv, vid, j0 + jj, ne, ns);
                const EdgeFetch F1 = edge_fetch(E, piv, vid, j0 + jj + 1, ne, ns);
                EdgeGeom G;
                if (edge_test(P, F0, G)) bits |= 1u << jj;
                if (edge_test(P, F1, G)) bits |= 2u << jj;
            }
            if (jj < nj) {
                EdgeGeom G;
                if (edge_geom(E, P, piv, vid, j0 + jj, ne, ns, G)) bits |= 1u << jj;
            }
        }
        // block-uniform: every wave of the workgroup reaches the barriers
        if (!__syncthreads_or(bits != 0u)) continue;
        const uint32_t c = (uint32_t)__popc(bits);
        uint32_t incl = c;  // inclusive prefix of c over the wave's lanes
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t up = (uint32_t)__shfl_up((int)incl, off);
            if (lane >= off) incl += up;
        }
        if (lane == 63) s_wave[wid] = incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int w = 0; w < kWaves; ++w) tot += s_wave[w];
            s_base = atomicAdd(E.q_count, tot);
        }
        __syncthreads();
        uint32_t at = s_base + incl - c;
        for (int w = 0; w < wid; ++w) at += s_wave[w];
        for (uint32_t m = bits; m != 0u; m &= m - 1u, ++at) {
            // the queue holds every sample of the pass; the check only
            // guards the bound
            if (at < E.q_cap) E.queue[at] = ((uint32_t)local << 10) | (uint32_t)(j0 + __ffs(m) - 1);
        }
        // s_wave and s_base are rewritten by the next chunk
        __syncthreads();
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

// a queued sample recomputed: ray origin, out-side direction, the term and
// where it goes (false: the sample carries no term)
struct EdgeTerm {
    float3 o, wo, mh;
    float wt, t;
    uint32_t e;
};

__device__ __forceinline__ bool edge_term(const EdgeArgs& E, uint32_t rec, uint32_t ne, uint32_t ns, float2 scale,
                                          bool bil, EdgeTerm& T) {
    const ShadeArgs& A = E.a;
    const int64_t N = A.g.n;
    const int64_t hw = (int64_t)A.g.height * A.g.width;
    const int64_t pix = E.pix0 + (int64_t)(rec >> 10);
    const int j = (int)(rec & 1023u);
    if (pix >= N) return false;
    bool nonfinite;
    const Pixel P = setup_pixel(A, pix, nonfinite);
    if (!P.valid) return false;
    const uint32_t view = (uint32_t)(pix / hw);
    const uint32_t piv = (uint32_t)(pix - (int64_t)view * hw);
    EdgeGeom G;
    if (!edge_geom(E, P, piv, (uint32_t)A.g.view_base + view, j, ne, ns, G)) return false;
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
    T.wt = G.s * (G.sharp ? scale.x : scale.y) * J * g;
    if (!(T.wt != 0.0f && isfinite(T.wt))) return false;
    T.o = P.o;
    T.wo = normalize(w - (G.s * kEdgeDelta) * G.mh);
    T.mh = G.mh;
    T.t = G.t;
    T.e = G.e;
    return true;
}

__device__ __forceinline__ void edge_scatter(const EdgeArgs& E, const EdgeTerm& T) {
    const int4 ed = E.edges[T.e];
    const float ta = 1.0f - T.t;
    float* ga = E.g_verts + 3 * (size_t)ed.x;
    float* gb = E.g_verts + 3 * (size_t)ed.y;
    atomicAdd(ga + 0, ta * T.wt * T.mh.x);
    atomicAdd(ga + 1, ta * T.wt * T.mh.y);
    atomicAdd(ga + 2, ta * T.wt * T.mh.z);
    atomicAdd(gb + 0, T.t * T.wt * T.mh.x);
    atomicAdd(gb + 1, T.t * T.wt * T.mh.y);
    atomicAdd(gb + 2, T.t * T.wt * T.mh.z);
}

// 2) the queued candidates: each is recomputed, its term evaluated and its
//    out-side ray traced; a ray that reaches the probe adds the term to both
//    vertices of the edge.  Few candidates (the usual case: silhouettes
//    above the horizon are rare): one per wavefront, the ray walked by all 64
//    lanes.  Many (heavy geometry): one per lane, which keeps every lane busy.
__global__ __launch_bounds__(256) void edge_trace_kernel(EdgeArgs E) {
    const ShadeArgs& A = E.a;
    const Scene& sc = A.scene;
    const uint32_t n = min(*E.q_count, E.q_cap);
    const uint32_t ne = *E.n_edges, ns = *E.n_sharp;
    const int n_total = sc.nodes[0].escape;
    const bool bil = (A.flags & MCDI_FLAG_BILINEAR) != 0;
    // per class: class size over class probability, times tau / n_es; the
    // sharp class takes ceil(2^24 num / den) of the 2^24 values of the test
    const uint64_t num = (uint64_t)E.gain * ns, den = num + (uint64_t)(ne - ns);
    const uint64_t cs = den ? ((num << 24) + den - 1) / den : 0;
    const float k = A.tau / (float)E.n_es;
    const float2 scale = make_float2(cs ? (float)ns * 16777216.0f / (float)cs * k : 0.0f,
                                     cs < 16777216u ? (float)(ne - ns) * 16777216.0f / (float)(16777216u - cs) * k
                                                    : 0.0f);
    const bool lead = __lane_id() == 0;
    uint32_t c_rays = 0, c_hits = 0;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n_threads = gridDim.x * blockDim.x;
    if (n >= kEdgeLaneMode) {
        for (uint32_t i = tid; i < n; i += n_threads) {
            EdgeTerm T;
            if (!edge_term(E, E.queue[i], ne, ns, scale, bil, T)) continue;
            ++c_rays;
            uint32_t nb = 0, nt = 0;
            // the 4-wide walk where the builder chose it (deep scenes)
            const Ray ray = make_ray(T.o, T.wo);
            const bool blocked = n_total > 0 && (sc.info->wide ? wbvh_anyhit(sc, ray, n_total, nb, nt)
                                                               : bvh_anyhit(sc, ray, n_total, nb, nt));
            if (blocked) {
                ++c_hits;
                continue;
            }
            edge_scatter(E, T);
        }
        if (A.stats) {
            const uint32_t a = wave_sum(c_rays), b = wave_sum(c_hits);
            if (lead && a) {
                atomicAdd(&A.stats->rays_traced, (unsigned long long)a);
                atomicAdd(&A.stats->rays_hit, (unsigned long long)b);
            }
        }
        return;
    }
    for (uint32_t i = tid >> 6; i < n; i += n_threads >> 6) {
        EdgeTerm T;
        if (!edge_term(E, E.queue[i], ne, ns, scale, bil, T)) continue;
        ++c_rays;
        if (wave_anyhit(sc, make_ray(T.o, T.wo), n_total)) {
            ++c_hits;
            continue;
        }
        if (lead) edge_scatter(E, T);
    }
    if (A.stats && lead && c_rays) {
        atomicAdd(&A.stats->rays_traced, (unsigned long long)c_rays);
        atomicAdd(&A.stats->rays_hit, (unsigned long long)c_hits);
    }
}

__global__ void edge_queue_reset(uint32_t* q_count) { *q_count = 0u; }

// Sampling class of an edge: sharp when it has one face, or when the normals
// of its faces, (b-a)x(c-a) and (a-b)x(d-b), are more than 20 degrees apart
// (dot < 0, or dot^2 < cos^2(20 deg) |n1|^2 |n2|^2).  FP32, no contraction,
// in this order: the CPU check takes the same decision bit for bit.
__device__ bool edge_is_sharp(const int4& ed, const float* __restrict__ verts) {
#pragma clang fp contract(off)
    if (ed.w < 0) return true;
    const float3 A = load_vert(verts, ed.x), B = load_vert(verts, ed.y);
    const float3 Cc = load_vert(verts, ed.z), D = load_vert(verts, ed.w);
    const float e1x = B.x - A.x, e1y = B.y - A.y, e1z = B.z - A.z;
    const float e2x = Cc.x - A.x, e2y = Cc.y - A.y, e2z = Cc.z - A.z;
    const float f1x = A.x - B.x, f1y = A.y - B.y, f1z = A.z - B.z;
    const float f2x = D.x - B.x, f2y = D.y - B.y, f2z = D.z - B.z;
    const float n1x = e1y * e2z - e1z * e2y, n1y = e1z * e2x - e1x * e2z, n1z = e1x * e2y - e1y * e2x;
    const float n2x = f1y * f2z - f1z * f2y, n2y = f1z * f2x - f1x * f2z, n2z = f1x * f2y - f1y * f2x;
    const float dt = n1x * n2x + n1y * n2y + n1z * n2z;
    const float q1 = n1x * n1x + n1y * n1y + n1z * n1z;
    const float q2 = n2x * n2x + n2y * n2y + n2z * n2z;
    const float lhs = dt * dt;
    const float rhs = kSharpCos2 * (q1 * q2);
    return dt < 0.0f || lhs < rhs;
}

constexpr int kPackItems = 4;
constexpr int kPackThreads = 256;
constexpr int kPackBlock = kPackItems * kPackThreads;

// exclusive scan over the workgroup; *total the sum
__device__ __forceinline__ uint32_t pack_scan(uint32_t v, uint32_t* s_buf, uint32_t* total) {
    const int t = threadIdx.x;
    s_buf[t] = v;
    __syncthreads();
    for (int off = 1; off < kPackThreads; off <<= 1) {
        const uint32_t add = t >= off ? s_buf[t - off] : 0u;
        __syncthreads();
        s_buf[t] += add;
        __syncthreads();
    }
    const uint32_t incl = s_buf[t];
    *total = s_buf[kPackThreads - 1];
    __syncthreads();
    return incl - v;
}

// sharp edges per block of kPackBlock edges
__global__ __launch_bounds__(kPackThreads) void edge_class_count(const int4* __restrict__ edges,
                                                                 const uint32_t* n_edges, const float* verts,
                                                                 uint32_t* bsum) {
    __shared__ uint32_t s_buf[kPackThreads];
    const uint32_t n = *n_edges;
    const uint32_t i0 = blockIdx.x * (uint32_t)kPackBlock + threadIdx.x * (uint32_t)kPackItems;
    uint32_t v = 0;
    for (int k = 0; k < kPackItems; ++k)
        if (i0 + k < n && edge_is_sharp(edges[i0 + k], verts)) ++v;
    uint32_t total;
    pack_scan(v, s_buf, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// exclusive scan of the block counts in place (one workgroup); the sharp count
__global__ __launch_bounds__(kPackThreads) void edge_class_scan(uint32_t nb, uint32_t* bsum, uint32_t* n_sharp) {
    __shared__ uint32_t s_buf[kPackThreads];
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kPackThreads) {
        const uint32_t i = b0 + threadIdx.x;
        const uint32_t v = i < nb ? bsum[i] : 0u;
        uint32_t total;
        const uint32_t ex = pack_scan(v, s_buf, &total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *n_sharp = carry;
}

// corners of every edge for this call's vertex positions, sharp edges first
// and each class in edge order: (a, edge id bits), (b, 0), (c, 0), (d, 1) or
// (0, 0, 0, 0) without a second face
__global__ __launch_bounds__(kPackThreads) void edge_pack_kernel(const int4* __restrict__ edges,
                                                                 const uint32_t* n_edges, const float* verts,
                                                                 const uint32_t* __restrict__ bsum,
                                                                 const uint32_t* n_sharp, float4* egeo) {
    __shared__ uint32_t s_buf[kPackThreads];
    const uint32_t n = *n_edges, ns = *n_sharp;
    const uint32_t i0 = blockIdx.x * (uint32_t)kPackBlock + threadIdx.x * (uint32_t)kPackItems;
    bool sharp[kPackItems];
    uint32_t v = 0;
    for (int k = 0; k < kPackItems; ++k) {
        sharp[k] = i0 + k < n && edge_is_sharp(edges[i0 + k], verts);
        v += sharp[k] ? 1u : 0u;
    }
    uint32_t total;
    uint32_t before = bsum[blockIdx.x] + pack_scan(v, s_buf, &total);   // sharp edges before i0
    for (int k = 0; k < kPackItems; ++k) {
        const uint32_t i = i0 + k;
        if (i >= n) break;
        const uint32_t at = sharp[k] ? before : ns + (i - before);
        if (sharp[k]) ++before;
        const int4 ed = edges[i];
        const float3 a = load_vert(verts, ed.x), b = load_vert(verts, ed.y), c = load_vert(verts, ed.z);
        float4* q = egeo + 4 * (size_t)at;
        q[0] = make_float4(a.x, a.y, a.z, __uint_as_float(i));
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

uint32_t edge_pack_blocks(uint32_t cap) { return (cap + kPackBlock - 1) / kPackBlock; }

hipError_t launch_edge_pack(const EdgeArgs& e, uint32_t cap, uint32_t* bsum, uint32_t* n_sharp, hipStream_t s) {
    const uint32_t nb = edge_pack_blocks(cap);
    float4* egeo = const_cast<float4*>(e.egeo);
    hipLaunchKernelGGL(edge_class_count, dim3(nb > 0 ? nb : 1), dim3(kPackThreads), 0, s, e.edges, e.n_edges, e.verts,
                       bsum);
    hipLaunchKernelGGL(edge_class_scan, dim3(1), dim3(kPackThreads), 0, s, nb > 0 ? nb : 1u, bsum, n_sharp);
    hipLaunchKernelGGL(edge_pack_kernel, dim3(nb > 0 ? nb : 1), dim3(kPackThreads), 0, s, e.edges, e.n_edges, e.verts,
                       bsum, n_sharp, egeo);
    return hipGetLastError();
}

hipError_t launch_edge_grad(const EdgeArgs& e, hipStream_t s, hipEvent_t gen_begin, hipEvent_t gen_end) {
    if (e.npix <= 0) return hipSuccess;
    hipLaunchKernelGGL(edge_queue_reset, dim3(1), dim3(1), 0, s, e.q_count);
    if (gen_begin) {
        const hipError_t r = hipEventRecord(gen_begin, s);
        if (r != hipSuccess) return r;
    }
    hipLaunchKernelGGL(edge_gen_kernel, dim3((unsigned)((e.npix + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, e);
    if (gen_end) {
        const hipError_t r = hipEventRecord(gen_end, s);
        if (r != hipSuccess) return r;
    }
    // the queue's length is on the device: a fixed grid of 8192 wavefronts
    // strides over it (one record per wavefront or per lane)
    hipLaunchKernelGGL(edge_trace_kernel, dim3(2048), dim3(256), 0, s, e);
    return hipGetLastError();
}

}  // namespace mcdi
