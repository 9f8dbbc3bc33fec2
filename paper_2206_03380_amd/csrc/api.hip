// Host runtime of the C ABI declared in include/mcdi.h: argument validation,
// handle ownership, stream-ordered allocation and kernel launches.
#include <hip/hip_runtime.h>
#include <algorithm>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "edge_internal.h"
#include "mcdi_internal.h"

using namespace mcdi;

namespace {

thread_local std::string g_err;

// traversal timing (MCDI_FLAG_TIME_TRACE): event pairs recorded around the
// trace kernel on the caller's stream
struct TraceTimer {
    static constexpr int kMax = 1024;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    int used = 0;
    ~TraceTimer() {
        for (auto& p : pool) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    }
    // next free pair, or nullptr when full
    std::pair<hipEvent_t, hipEvent_t>* next() {
        if (used >= kMax) return nullptr;
        if (used == (int)pool.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess) return nullptr;
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                return nullptr;
            }
            pool.emplace_back(a, b);
        }
        return &pool[used++];
    }
};
// Process-wide (a framework may run the backward pass on a thread of its
// own), guarded by g_timer_mu.
TraceTimer g_timer;       // traversal kernels (MCDI_FLAG_TIME_TRACE)
TraceTimer g_timer_adj;   // adjoint and edge-sample kernels (MCDI_FLAG_TIME_ADJOINT)
std::mutex g_timer_mu;

std::pair<hipEvent_t, hipEvent_t>* timer_next(TraceTimer& t) {
    std::lock_guard<std::mutex> lock(g_timer_mu);
    return t.next();
}

mcdi_status fail(mcdi_status st, const char* fmt, ...);

mcdi_status drain_times(TraceTimer& t, float* out, int32_t cap, int32_t* n, const char* who) {
    std::lock_guard<std::mutex> lock(g_timer_mu);
    int32_t k = 0;
    for (int i = 0; i < t.used; ++i) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(t.pool[i].second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.pool[i].first, t.pool[i].second);
        if (e != hipSuccess) {
            t.used = 0;
            return fail(MCDI_E_DEVICE, "%s: %s", who, hipGetErrorString(e));
        }
        if (k < cap) out[k] = ms;
        ++k;
    }
    t.used = 0;
    *n = k < cap ? k : cap;
    return MCDI_OK;
}

mcdi_status fail(mcdi_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

mcdi_status ok() {
    g_err.clear();
    return MCDI_OK;
}

struct Alloc {
    mcdi_allocator user{};
    bool has_user = false;
    void* get(size_t bytes, hipStream_t s) const {
        if (bytes == 0) bytes = 256;
        if (has_user) {
            // the kernels read tables with 16-byte loads
            void* p = user.alloc(user.ctx, bytes, (void*)s);
            if (p && ((uintptr_t)p & 255u)) {
                user.free(user.ctx, p, (void*)s);
                return nullptr;
            }
            return p;
        }
        void* p = nullptr;
        if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void put(void* p, hipStream_t s) const {
        if (!p) return;
        if (has_user) user.free(user.ctx, p, (void*)s);
        else (void)hipFreeAsync(p, s);
    }
};

Alloc make_alloc(const mcdi_allocator* a) {
    Alloc r;
    if (a && a->alloc && a->free) {
        r.user = *a;
        r.has_user = true;
    }
    return r;
}

void* temp_alloc(void* ctx, size_t b, hipStream_t s) { return static_cast<Alloc*>(ctx)->get(b, s); }
void temp_free(void* ctx, void* p, hipStream_t s) { static_cast<Alloc*>(ctx)->put(p, s); }

}  // namespace

struct mcdi_scene_s {
    Alloc alloc;
    hipStream_t stream = nullptr;
    int64_t n_tris = 0;
    Node* nodes = nullptr;
    float4* tris = nullptr;
    QNode* qnodes = nullptr;
    QNode* groups = nullptr;       // 4 * group_cap records, then group_cap visit orders
    size_t group_cap = 0;
    QFrame* frame = nullptr;
    DeviceSceneInfo* info = nullptr;
    hipEvent_t built = nullptr;     // recorded on the build stream after the build
    hipEvent_t last_use = nullptr;  // recorded after the last enqueued work that reads the scene
    bool used = false;
};

namespace {

Scene scene_view(mcdi_scene sc) {
    return Scene{sc->nodes, sc->tris, sc->n_tris, sc->qnodes, sc->frame, sc->groups,
                 (uint32_t)(sizeof(QNode) * 4 * sc->group_cap),
                 reinterpret_cast<const uint32_t*>(sc->groups + 4 * sc->group_cap), sc->info};
}

// work that reads the scene on stream u waits for the build (a no-op order
// on the build stream itself)
hipError_t scene_acquire(mcdi_scene sc, hipStream_t u) { return hipStreamWaitEvent(u, sc->built, 0); }

// marks the end of work that reads the scene on stream u; the scene's memory
// is released only after it
hipError_t scene_release(mcdi_scene sc, hipStream_t u) {
    sc->used = true;
    return hipEventRecord(sc->last_use, u);
}

}  // namespace

struct mcdi_env_s {
    Alloc alloc;
    hipStream_t stream = nullptr;
    int32_t H = 0, W = 0;
    const float* rgb = nullptr;
    float* cond = nullptr;
    float* marg = nullptr;
    float* pdf = nullptr;
    double* rowsum = nullptr;  // [H + 1]
    int32_t* light = nullptr;
    int32_t* hot_slot = nullptr;   // [H*W]
    int32_t* hot_texel = nullptr;  // [kHotMax]
    int32_t* n_hot = nullptr;
    int32_t* guide = nullptr;      // [H][G+1]
    int32_t G = 1;
    int32_t win = 0;
    float4* tex = nullptr;         // [H*W] (r, g, b, pdf)
    uint8_t* dclass = nullptr;     // [(H*W + 3) / 4] density classes
};

extern "C" {

const char* mcdi_last_error(void) { return g_err.c_str(); }

mcdi_status mcdi_trace_times(float* out, int32_t cap, int32_t* n) {
    if (!n || (cap > 0 && !out)) return fail(MCDI_E_INVALID, "mcdi_trace_times: NULL argument");
    mcdi_status st = drain_times(g_timer, out, cap, n, "mcdi_trace_times");
    return st == MCDI_OK ? ok() : st;
}

mcdi_status mcdi_adjoint_times(float* out, int32_t cap, int32_t* n) {
    if (!n || (cap > 0 && !out)) return fail(MCDI_E_INVALID, "mcdi_adjoint_times: NULL argument");
    mcdi_status st = drain_times(g_timer_adj, out, cap, n, "mcdi_adjoint_times");
    return st == MCDI_OK ? ok() : st;
}

const char* mcdi_version(void) { return "mcdi 0.1 gfx950"; }

mcdi_status mcdi_build_scene(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                             const mcdi_allocator* alloc, void* stream, mcdi_scene* out) {
    if (!out) return fail(MCDI_E_INVALID, "mcdi_build_scene: out is NULL");
    if (n_verts < 0 || n_tris < 0) return fail(MCDI_E_INVALID, "mcdi_build_scene: negative count");
    if (n_verts >= (int64_t)1 << 31) return fail(MCDI_E_UNSUPPORTED, "mcdi_build_scene: n_verts >= 2^31");
    if (n_tris >= (int64_t)1 << 26) return fail(MCDI_E_UNSUPPORTED, "mcdi_build_scene: n_tris >= 2^26");
    if (n_tris > 0 && (!verts || !tris)) return fail(MCDI_E_INVALID, "mcdi_build_scene: NULL verts/tris");
    if (n_tris > 0 && n_verts == 0) return fail(MCDI_E_INVALID, "mcdi_build_scene: triangles without vertices");
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(MCDI_E_INVALID, "mcdi_build_scene: allocator incomplete");
    hipStream_t s = (hipStream_t)stream;
    mcdi_scene sc = new (std::nothrow) mcdi_scene_s;
    if (!sc) return fail(MCDI_E_OOM, "mcdi_build_scene: host allocation failed");
    sc->alloc = make_alloc(alloc);
    sc->stream = s;
    sc->n_tris = n_tris;
    const size_t n_nodes = n_tris > 0 ? (size_t)(2 * n_tris - 1) : 1;
    sc->nodes = (Node*)sc->alloc.get(sizeof(Node) * n_nodes, s);
    sc->tris = (float4*)sc->alloc.get(sizeof(float4) * 3 * (size_t)(n_tris > 0 ? n_tris : 1), s);
    sc->qnodes = (QNode*)sc->alloc.get(sizeof(QNode) * n_nodes, s);
    sc->frame = (QFrame*)sc->alloc.get(sizeof(QFrame), s);
    sc->group_cap = n_tris > 1 ? (size_t)n_tris : 1;
    sc->groups = (QNode*)sc->alloc.get((sizeof(QNode) * 4 + sizeof(uint32_t)) * sc->group_cap, s);
    sc->info = (DeviceSceneInfo*)sc->alloc.get(sizeof(DeviceSceneInfo), s);
    if (!sc->nodes || !sc->tris || !sc->qnodes || !sc->frame || !sc->groups || !sc->info) {
        mcdi_destroy_scene(sc);
        return fail(MCDI_E_OOM, "mcdi_build_scene: device allocation failed (%lld triangles)", (long long)n_tris);
    }
    if (hipEventCreateWithFlags(&sc->built, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&sc->last_use, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        mcdi_destroy_scene(sc);
        return fail(MCDI_E_DEVICE, "mcdi_build_scene: event creation failed");
    }
    TempAlloc ta{temp_alloc, temp_free, &sc->alloc};
    int oom = 0;
    hipError_t e = build_bvh(verts, n_verts, tris, n_tris, sc->nodes, sc->tris, sc->qnodes, sc->frame, sc->groups, sc->info, ta,
                             s, &oom);
    if (e == hipSuccess) e = hipEventRecord(sc->built, s);
    if (e != hipSuccess) {
        mcdi_destroy_scene(sc);
        if (oom) return fail(MCDI_E_OOM, "mcdi_build_scene: temporary allocation failed");
        return fail(MCDI_E_DEVICE, "mcdi_build_scene: %s", hipGetErrorString(e));
    }
    *out = sc;
    return ok();
}

void mcdi_destroy_scene(mcdi_scene sc) {
    if (!sc) return;
    // the memory goes back in the build stream's order, after the last
    // enqueued work that reads it
    if (sc->used) (void)hipStreamWaitEvent(sc->stream, sc->last_use, 0);
    sc->alloc.put(sc->nodes, sc->stream);
    sc->alloc.put(sc->tris, sc->stream);
    sc->alloc.put(sc->qnodes, sc->stream);
    sc->alloc.put(sc->frame, sc->stream);
    sc->alloc.put(sc->groups, sc->stream);
    sc->alloc.put(sc->info, sc->stream);
    if (sc->built) (void)hipEventDestroy(sc->built);
    if (sc->last_use) (void)hipEventDestroy(sc->last_use);
    delete sc;
}

mcdi_status mcdi_scene_info(mcdi_scene sc, mcdi_scene_info_t* info) {
    if (!sc || !info) return fail(MCDI_E_INVALID, "mcdi_scene_info: NULL argument");
    DeviceSceneInfo h{};
    hipError_t e = hipStreamSynchronize(sc->stream);
    if (e == hipSuccess) e = hipMemcpy(&h, sc->info, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_scene_info: %s", hipGetErrorString(e));
    info->n_tris = sc->n_tris;
    info->n_nodes = h.n_nodes;
    info->max_depth = h.max_depth;
    info->bad_tris = h.bad_tris;
    info->n_groups = h.n_groups;
    info->wide = h.wide;
    info->depth_complexity = h.depth_complexity;
    info->n_big = h.n_big;
    return ok();
}

mcdi_status mcdi_scene_nodes(mcdi_scene sc, void* nodes, float* tris, void* stream) {
    if (!sc) return fail(MCDI_E_INVALID, "mcdi_scene_nodes: NULL scene");
    hipStream_t s = (hipStream_t)stream;
    DeviceSceneInfo h{};
    hipError_t e = hipStreamSynchronize(sc->stream);
    if (e == hipSuccess) e = hipMemcpy(&h, sc->info, sizeof(h), hipMemcpyDeviceToHost);
    if (e == hipSuccess && nodes && h.n_nodes > 0)
        e = hipMemcpyAsync(nodes, sc->nodes, sizeof(Node) * (size_t)h.n_nodes, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && tris && sc->n_tris > 0)
        e = hipMemcpyAsync(tris, sc->tris, sizeof(float4) * 3 * (size_t)sc->n_tris, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = scene_release(sc, s);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_scene_nodes: %s", hipGetErrorString(e));
    return ok();
}

mcdi_status mcdi_build_env_cdf(const float* env_rgb, int32_t H, int32_t W, const mcdi_allocator* alloc,
                               void* stream, mcdi_env* out) {
    if (!out) return fail(MCDI_E_INVALID, "mcdi_build_env_cdf: out is NULL");
    if (!env_rgb) return fail(MCDI_E_INVALID, "mcdi_build_env_cdf: env_rgb is NULL");
    if (H < 1 || W < 1) return fail(MCDI_E_INVALID, "mcdi_build_env_cdf: H and W must be >= 1");
    if (H > 4096 || W > 4096) return fail(MCDI_E_UNSUPPORTED, "mcdi_build_env_cdf: H and W must be <= 4096");
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(MCDI_E_INVALID, "mcdi_build_env_cdf: allocator incomplete");
    hipStream_t s = (hipStream_t)stream;
    mcdi_env ev = new (std::nothrow) mcdi_env_s;
    if (!ev) return fail(MCDI_E_OOM, "mcdi_build_env_cdf: host allocation failed");
    ev->alloc = make_alloc(alloc);
    ev->stream = s;
    ev->H = H;
    ev->W = W;
    ev->rgb = env_rgb;
    // 16 floats past the last row: the row search reads aligned windows
    ev->cond = (float*)ev->alloc.get(sizeof(float) * ((size_t)H * (W + 1) + 16), s);
    ev->marg = (float*)ev->alloc.get(sizeof(float) * (size_t)(H + 1), s);
    ev->pdf = (float*)ev->alloc.get(sizeof(float) * (size_t)H * W, s);
    ev->rowsum = (double*)ev->alloc.get(sizeof(double) * (size_t)(H + 1), s);
    ev->light = (int32_t*)ev->alloc.get(sizeof(int32_t), s);
    ev->hot_slot = (int32_t*)ev->alloc.get(sizeof(int32_t) * (size_t)H * W, s);
    ev->hot_texel = (int32_t*)ev->alloc.get(sizeof(int32_t) * kHotMax, s);
    ev->n_hot = (int32_t*)ev->alloc.get(sizeof(int32_t), s);
    ev->win = env_row_window(H, W);
    ev->G = env_guide_cells(W, ev->win);
    ev->guide = (int32_t*)ev->alloc.get(sizeof(int32_t) * (size_t)H * (ev->G + 1), s);
    ev->tex = (float4*)ev->alloc.get(sizeof(float4) * (size_t)H * W, s);
    ev->dclass = (uint8_t*)ev->alloc.get(((size_t)H * W + 3) / 4, s);
    if (!ev->cond || !ev->marg || !ev->pdf || !ev->rowsum || !ev->light || !ev->hot_slot || !ev->hot_texel ||
        !ev->n_hot || !ev->guide || !ev->tex || !ev->dclass) {
        mcdi_destroy_env(ev);
        return fail(MCDI_E_OOM, "mcdi_build_env_cdf: device allocation failed");
    }
    hipError_t e = launch_env_cdf(env_rgb, H, W, ev->cond, ev->marg, ev->pdf, ev->rowsum, ev->light, s);
    if (e == hipSuccess) e = launch_env_guide(ev->cond, H, W, ev->G, ev->guide, s);
    if (e == hipSuccess) e = launch_env_pack(env_rgb, ev->pdf, (int64_t)H * W, ev->tex, s);
    if (e == hipSuccess) e = launch_env_dclass(ev->pdf, (int64_t)H * W, ev->dclass, s);
    if (e == hipSuccess) e = launch_env_hot(ev->pdf, H, W, ev->hot_slot, ev->hot_texel, ev->n_hot, s);
    if (e != hipSuccess) {
        mcdi_destroy_env(ev);
        return fail(MCDI_E_DEVICE, "mcdi_build_env_cdf: %s", hipGetErrorString(e));
    }
    *out = ev;
    return ok();
}

void mcdi_destroy_env(mcdi_env ev) {
    if (!ev) return;
    ev->alloc.put(ev->cond, ev->stream);
    ev->alloc.put(ev->marg, ev->stream);
    ev->alloc.put(ev->pdf, ev->stream);
    ev->alloc.put(ev->rowsum, ev->stream);
    ev->alloc.put(ev->light, ev->stream);
    ev->alloc.put(ev->hot_slot, ev->stream);
    ev->alloc.put(ev->hot_texel, ev->stream);
    ev->alloc.put(ev->n_hot, ev->stream);
    ev->alloc.put(ev->guide, ev->stream);
    ev->alloc.put(ev->dclass, ev->stream);
    ev->alloc.put(ev->tex, ev->stream);
    delete ev;
}

mcdi_status mcdi_env_tables(mcdi_env ev, float* cond, float* marg, float* pdf, void* stream) {
    if (!ev) return fail(MCDI_E_INVALID, "mcdi_env_tables: NULL env");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    const size_t H = (size_t)ev->H, W = (size_t)ev->W;
    if (cond && e == hipSuccess) e = hipMemcpyAsync(cond, ev->cond, sizeof(float) * H * (W + 1), hipMemcpyDeviceToDevice, s);
    if (marg && e == hipSuccess) e = hipMemcpyAsync(marg, ev->marg, sizeof(float) * (H + 1), hipMemcpyDeviceToDevice, s);
    if (pdf && e == hipSuccess) e = hipMemcpyAsync(pdf, ev->pdf, sizeof(float) * H * W, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_env_tables: %s", hipGetErrorString(e));
    return ok();
}

static mcdi_status fill_common(const char* who, mcdi_scene sc, mcdi_env ev, const mcdi_gbuffer* g,
                               const mcdi_params* p, ShadeArgs& a) {
    if (!sc || !ev || !g || !p) return fail(MCDI_E_INVALID, "%s: NULL scene/env/gbuffer/params", who);
    if (g->n_views < 1 || g->height < 1 || g->width < 1)
        return fail(MCDI_E_INVALID, "%s: n_views, height, width must be >= 1", who);
    const int64_t n = (int64_t)g->n_views * g->height * g->width;
    if (n >= (int64_t)1 << 31) return fail(MCDI_E_UNSUPPORTED, "%s: more than 2^31 - 1 pixels", who);
    if (!g->pos || !g->nrm || !g->kd || !g->korm || !g->mask || !g->eye)
        return fail(MCDI_E_INVALID, "%s: NULL G-buffer plane", who);
    if (p->spp < 1 || p->spp > 1024) return fail(MCDI_E_INVALID, "%s: spp must be in [1, 1024]", who);
    if (!std::isfinite(p->tau) || !std::isfinite(p->ray_eps) || p->ray_eps < 0.0f)
        return fail(MCDI_E_INVALID, "%s: tau must be finite and ray_eps finite and >= 0", who);
    if ((p->flags & MCDI_FLAG_DUMP) && !p->decisions)
        return fail(MCDI_E_INVALID, "%s: MCDI_FLAG_DUMP without a decisions buffer", who);
    if ((p->flags & MCDI_FLAG_LIGHT_OFF) && (p->flags & MCDI_FLAG_BSDF_OFF))
        return fail(MCDI_E_INVALID, "%s: LIGHT_OFF and BSDF_OFF leave no sampling technique", who);
    if ((p->flags & MCDI_FLAG_FORCE_COS) && (p->flags & MCDI_FLAG_FORCE_GGX))
        return fail(MCDI_E_INVALID, "%s: FORCE_COS and FORCE_GGX together", who);
    std::memset(&a, 0, sizeof(a));
    a.scene = scene_view(sc);
    a.env = EnvView{ev->H, ev->W, ev->cond, ev->marg, ev->light, ev->hot_slot, ev->hot_texel, ev->n_hot, ev->guide,
                    ev->G, ev->tex, ev->pdf, ev->win, ev->dclass};
    a.g = GBufView{g->n_views, g->height, g->width, g->view_base, g->pos, g->nrm, g->kd, g->korm, g->mask, g->eye, n};
    a.spp = p->spp;
    a.flags = p->flags;
    a.seed = p->seed;
    a.tau = p->tau;
    a.ray_eps = p->ray_eps;
    a.decisions = (p->flags & MCDI_FLAG_DUMP) ? p->decisions : nullptr;
    return MCDI_OK;
}

// Ray queue workspace of the forward pipeline, from the scene's allocator.
struct Workspace {
    const Alloc* alloc = nullptr;
    hipStream_t s = nullptr;
    void* base = nullptr;
    ~Workspace() {
        if (base) alloc->put(base, s);
    }
};

static mcdi_status trace_pipeline(const char* who, mcdi_scene sc, ShadeArgs& a, uint32_t* hitbits, hipStream_t s,
                                  Workspace& ws, uint32_t** bits_out) {
    const int64_t n = a.g.n;
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    const size_t words = (size_t)((2 * a.spp + 31) / 32);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t sz_rays = a.tau != 0.0f ? al(sizeof(float4) * (size_t)blocks * 2 * a.spp * kBlock) : 0;
    const size_t sz_cnt = al(sizeof(int32_t) * (size_t)blocks);
    const size_t sz_org = al(sizeof(float4) * (size_t)n);
    const size_t sz_bits = hitbits ? 0 : al(sizeof(uint32_t) * words * (size_t)n);
    // live samples (with tracing): the shading then walks only those
    const size_t sz_live = (a.tau != 0.0f && !a.live) ? al(sizeof(uint32_t) * words * (size_t)n) : 0;
    ws.alloc = &sc->alloc;
    ws.s = s;
    ws.base = sc->alloc.get(sz_rays + 2 * sz_cnt + sz_org + sz_bits + sz_live, s);
    if (!ws.base) return fail(MCDI_E_OOM, "%s: workspace allocation failed", who);
    char* p = (char*)ws.base;
    a.rays = sz_rays ? (float4*)p : nullptr;
    p += sz_rays;
    a.ray_count = (int32_t*)p;
    p += sz_cnt;
    a.tile_order = (int32_t*)p;
    p += sz_cnt;
    a.origins = (float4*)p;
    p += sz_org;
    uint32_t* bits = hitbits ? hitbits : (uint32_t*)p;
    p += sz_bits;
    if (sz_live) a.live = (uint32_t*)p;
    // the generator needs a ray region even when nothing is traced
    ShadeArgs g = a;
    if (!g.rays) g.tau = 0.0f;
    hipError_t e = launch_gen_rays(g, bits, s);
    // tiles with the most rays are traversed first
    if (e == hipSuccess && a.tau != 0.0f) e = launch_order_tiles(a.ray_count, blocks, a.tile_order, s);
    // the BVH may still be building on another stream: wait for it before
    // the traversal (and before its timing starts)
    if (e == hipSuccess && a.tau != 0.0f) e = scene_acquire(sc, s);
    std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
    if ((a.flags & MCDI_FLAG_TIME_TRACE) && e == hipSuccess && a.tau != 0.0f) {
        ev = timer_next(g_timer);
        if (ev) e = hipEventRecord(ev->first, s);
    }
    if (e == hipSuccess && a.tau != 0.0f) e = launch_trace_rays(a, bits, s);
    if (ev && e == hipSuccess) e = hipEventRecord(ev->second, s);
    if (e == hipSuccess && a.tau != 0.0f) e = scene_release(sc, s);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "%s: %s", who, hipGetErrorString(e));
    *bits_out = bits;
    return MCDI_OK;
}

mcdi_status mcdi_shade_fwd(mcdi_scene sc, mcdi_env ev, const mcdi_gbuffer* g, const mcdi_params* p, float* c_d,
                           float* c_s, uint32_t* hitbits, mcdi_stats* stats, void* stream) {
    ShadeArgs a;
    mcdi_status st = fill_common("mcdi_shade_fwd", sc, ev, g, p, a);
    if (st != MCDI_OK) return st;
    if (!c_d || !c_s) return fail(MCDI_E_INVALID, "mcdi_shade_fwd: NULL c_d/c_s");
    if (p->tau != 0.0f) a.live = p->live;   // NULL: the workspace keeps them
    hipStream_t s = (hipStream_t)stream;
    a.c_d = c_d;
    a.c_s = c_s;
    a.stats = stats;
    Workspace ws;
    uint32_t* bits = nullptr;
    st = trace_pipeline("mcdi_shade_fwd", sc, a, hitbits, s, ws, &bits);
    if (st != MCDI_OK) return st;
    a.hitbits_in = bits;
    hipError_t e = launch_shade_fwd(a, s);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_shade_fwd: %s", hipGetErrorString(e));
    return ok();
}

mcdi_status mcdi_shade_fwd_frozen(mcdi_scene sc, mcdi_env ev_s, const mcdi_gbuffer* g_s, mcdi_env ev_e,
                                  const mcdi_gbuffer* g_e, const mcdi_params* p, float* c_d, float* c_s,
                                  void* stream) {
    ShadeArgs a;
    mcdi_status st = fill_common("mcdi_shade_fwd_frozen", sc, ev_s, g_s, p, a);
    if (st != MCDI_OK) return st;
    if (!ev_e || !g_e || !c_d || !c_s) return fail(MCDI_E_INVALID, "mcdi_shade_fwd_frozen: NULL argument");
    if (p->flags & (MCDI_FLAG_DUMP | MCDI_FLAG_DUMP_DIRS | MCDI_FLAG_TIME_TRACE | MCDI_FLAG_TIME_ADJOINT))
        return fail(MCDI_E_INVALID, "mcdi_shade_fwd_frozen: dump and timing flags are not supported");
    if (ev_e->H != ev_s->H || ev_e->W != ev_s->W)
        return fail(MCDI_E_INVALID, "mcdi_shade_fwd_frozen: the probes differ in size");
    if (g_e->n_views != g_s->n_views || g_e->height != g_s->height || g_e->width != g_s->width ||
        g_e->view_base != g_s->view_base || g_e->pos != g_s->pos || g_e->mask != g_s->mask || g_e->eye != g_s->eye)
        return fail(MCDI_E_INVALID,
                    "mcdi_shade_fwd_frozen: the G-buffers must share size, view_base, pos, mask and eye");
    if (!g_e->nrm || !g_e->kd || !g_e->korm) return fail(MCDI_E_INVALID, "mcdi_shade_fwd_frozen: NULL G-buffer plane");
    hipStream_t s = (hipStream_t)stream;
    a.c_d = c_d;
    a.c_s = c_s;
    a.e_nrm = g_e->nrm;
    a.e_kd = g_e->kd;
    a.e_korm = g_e->korm;
    // probe texels: the evaluation probe's radiance with the sampling probe's density
    const int64_t n_tex = (int64_t)ev_s->H * ev_s->W;
    Workspace wt;
    wt.alloc = &sc->alloc;
    wt.s = s;
    wt.base = sc->alloc.get(sizeof(float4) * (size_t)n_tex, s);
    if (!wt.base) return fail(MCDI_E_OOM, "mcdi_shade_fwd_frozen: workspace allocation failed");
    Workspace ws;
    uint32_t* bits = nullptr;
    st = trace_pipeline("mcdi_shade_fwd_frozen", sc, a, nullptr, s, ws, &bits);
    if (st != MCDI_OK) return st;
    a.hitbits_in = bits;
    a.env.tex = (float4*)wt.base;
    hipError_t e = launch_env_mix(ev_e->tex, ev_s->tex, n_tex, (float4*)wt.base, s);
    if (e == hipSuccess) e = launch_shade_fwd_frozen(a, s);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_shade_fwd_frozen: %s", hipGetErrorString(e));
    return ok();
}

mcdi_status mcdi_shade_bwd(mcdi_scene sc, mcdi_env ev, const mcdi_gbuffer* g, const mcdi_params* p,
                           const float* g_cd, const float* g_cs, const uint32_t* hitbits, float* g_kd,
                           float* g_korm, float* g_nrm, float* g_env, mcdi_stats* stats, void* stream) {
    ShadeArgs a;
    mcdi_status st = fill_common("mcdi_shade_bwd", sc, ev, g, p, a);
    if (st != MCDI_OK) return st;
    if (p->flags & MCDI_FLAG_DUMP) return fail(MCDI_E_INVALID, "mcdi_shade_bwd: MCDI_FLAG_DUMP is forward-only");
    if (!g_cd || !g_cs || !g_kd || !g_korm || !g_nrm)
        return fail(MCDI_E_INVALID, "mcdi_shade_bwd: NULL gradient buffer");
    hipStream_t s = (hipStream_t)stream;
    a.g_cd = g_cd;
    a.g_cs = g_cs;
    a.g_kd = g_kd;
    a.g_korm = g_korm;
    a.g_nrm = g_nrm;
    a.g_env = g_env;
    a.stats = stats;
    Workspace ws;
    if (p->tau != 0.0f && hitbits) a.live = p->live;   // a re-trace keeps its own
    if (hitbits) {
        a.hitbits_in = hitbits;
    } else {
        // re-trace: same rays as the forward pass
        uint32_t* bits = nullptr;
        st = trace_pipeline("mcdi_shade_bwd", sc, a, nullptr, s, ws, &bits);
        if (st != MCDI_OK) return st;
        a.hitbits_in = bits;
    }
    // probe gradient: per-tile records binned after the adjoint (see
    // env_scatter.hip); positions in the sorted records are 32-bit
    Workspace wr;
    EnvScatter es{};
    const int64_t tiles = (a.g.n + kBlock - 1) / kBlock;
    // records per tile: one per sample (the bilinear record is two float4s)
    const int64_t region = 2 * (int64_t)a.spp * kBlock;
    const bool bil = (a.flags & MCDI_FLAG_BILINEAR) != 0;
    if (g_env && tiles * region <= ((int64_t)1 << 30) && env_scatter_plan(ev->H, ev->W, tiles, (uint32_t)region, bil, es)) {
        wr.alloc = &sc->alloc;
        wr.s = s;
        wr.base = sc->alloc.get(env_scatter_bytes(es), s);
        if (wr.base) {   // without the workspace the adjoint scatters directly
            env_scatter_carve(wr.base, es);
            es.g_env = g_env;
            a.rec = es.rec;
            a.rec_count = es.tile_count;
            a.rec_region = es.region;
        }
    }
    hipError_t e = a.rec ? launch_env_scatter_init(es, s) : hipSuccess;
    std::pair<hipEvent_t, hipEvent_t>* tev = nullptr;
    if ((a.flags & MCDI_FLAG_TIME_ADJOINT) && e == hipSuccess) {
        tev = timer_next(g_timer_adj);
        if (tev) e = hipEventRecord(tev->first, s);
    }
    if (e == hipSuccess) e = launch_shade_bwd(a, s);
    if (tev && e == hipSuccess) e = hipEventRecord(tev->second, s);
    if (e == hipSuccess && a.rec) e = launch_env_scatter(es, s);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_shade_bwd: %s", hipGetErrorString(e));
    return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: requests are admitted while the server's memory budget and slot
// count allow, and their tiles packed, oldest request first, into persistent
// launches of bounded work.  A launch ends in a tail of a few long tiles, so
// launches alternate between two lanes (streams of the server's own): the
// next launch fills the compute units while the previous one drains.  The
// caller's stream (home) carries only the server's allocations and frees;
// a lane waits for home before its first use of memory allocated there.
// ---------------------------------------------------------------------------
namespace {

constexpr int kLanes = 2;

struct SrvReq {
    int64_t ticket = 0;
    ShadeArgs args{};
    int64_t tiles = 0, next_tile = 0;
    int outstanding = 0;       // launches in flight holding tiles of the request
    size_t bytes = 0;          // scratch the request holds while admitted
    hipEvent_t ready = nullptr;  // recorded on the caller's input stream, or null
    unsigned ready_seen = 0;   // lanes already made to wait for `ready`
    void* scratch = nullptr;
    uint32_t* hitbits = nullptr;
    float4* origins = nullptr;
    bool grad = false;
    mcdi_scene scene_handle = nullptr;
};

struct SrvLane {
    hipStream_t stream = nullptr;
    float4* rays = nullptr;        // per-workgroup ray regions of the persistent grid
    int* counter = nullptr;
    ServeItem* items_dev = nullptr;
    ServeItem* staging = nullptr;  // pinned host
    bool busy = false;             // a launch in flight
    int64_t home_seen = 0;         // home epoch this lane has waited for
};

struct SrvLaunch {
    int lane = 0;
    hipEvent_t done = nullptr;
    std::vector<SrvReq*> reqs;
};

}  // namespace

struct mcdi_server_s {
    Alloc alloc;
    hipStream_t home = nullptr;
    mcdi_server_config cfg{};
    SrvLane lane[kLanes];
    hipEvent_t home_ev = nullptr;  // recorded on home after allocations
    int64_t home_epoch = 0;        // allocations made on home so far (a counter)
    int64_t home_recorded = 0;     // epoch home_ev was last recorded at
    std::deque<SrvReq*> queue;     // submitted, not admitted
    std::vector<SrvReq*> admitted;
    std::vector<SrvLaunch> in_flight;
    std::vector<hipEvent_t> spare_events;
    std::deque<int64_t> completed; // tickets done, not yet reported
    size_t used = 0;
    int64_t next_ticket = 1, launches = 0;
};

namespace {

size_t srv_align(size_t b) { return (b + 255) & ~(size_t)255; }

size_t srv_hitbit_bytes(int64_t n, int32_t spp) {
    return srv_align(sizeof(uint32_t) * (size_t)((2 * spp + 31) / 32) * (size_t)n);
}

size_t srv_request_bytes(int64_t n, int32_t spp) {
    return srv_hitbit_bytes(n, spp) + srv_align(sizeof(float4) * (size_t)n);
}

hipEvent_t srv_event(mcdi_server sv) {
    if (!sv->spare_events.empty()) {
        hipEvent_t e = sv->spare_events.back();
        sv->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void* srv_get(mcdi_server sv, size_t bytes) {
    void* p = sv->alloc.get(bytes, sv->home);
    if (p) ++sv->home_epoch;
    return p;
}

void srv_release(mcdi_server sv, SrvReq* r) {
    // only after every launch that used it has been seen to finish
    if (r->scratch) sv->alloc.put(r->scratch, sv->home);
    r->scratch = nullptr;
    if (r->ready) sv->spare_events.push_back(r->ready);
    r->ready = nullptr;
}

void srv_finish(mcdi_server sv, SrvLaunch& L) {
    for (SrvReq* r : L.reqs) {
        if (--r->outstanding > 0 || r->next_tile < r->tiles) continue;
        sv->used -= r->bytes;
        sv->admitted.erase(std::find(sv->admitted.begin(), sv->admitted.end(), r));
        sv->completed.push_back(r->ticket);
        srv_release(sv, r);
        delete r;
    }
    sv->lane[L.lane].busy = false;
    sv->spare_events.push_back(L.done);
}

// finished launches (block: wait for the oldest first)
mcdi_status srv_retire(mcdi_server sv, bool block) {
    for (size_t i = 0; i < sv->in_flight.size();) {
        SrvLaunch& L = sv->in_flight[i];
        const hipError_t q = (block && i == 0) ? hipEventSynchronize(L.done) : hipEventQuery(L.done);
        if (q == hipErrorNotReady) {
            (void)hipGetLastError();
            ++i;
            continue;
        }
        if (q != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_server_poll: %s", hipGetErrorString(q));
        srv_finish(sv, L);
        sv->in_flight.erase(sv->in_flight.begin() + (ptrdiff_t)i);
    }
    return MCDI_OK;
}

void srv_admit(mcdi_server sv) {
    while (!sv->queue.empty() && (int)sv->admitted.size() < sv->cfg.slots &&
           sv->used + sv->queue.front()->bytes <= (size_t)sv->cfg.budget_bytes) {
        SrvReq* r = sv->queue.front();
        r->scratch = srv_get(sv, r->bytes);
        if (!r->scratch) return;   // the device is short of memory: retry after completions
        r->hitbits = (uint32_t*)r->scratch;
        r->origins = (float4*)((char*)r->scratch + srv_hitbit_bytes(r->args.g.n, r->args.spp));
        sv->queue.pop_front();
        sv->used += r->bytes;
        sv->admitted.push_back(r);
    }
}

// order a lane after home's allocations so far
hipError_t srv_sync_home(mcdi_server sv, SrvLane& ln) {
    if (ln.home_seen == sv->home_epoch) return hipSuccess;
    hipError_t e = hipSuccess;
    if (sv->home_recorded != sv->home_epoch) {
        e = hipEventRecord(sv->home_ev, sv->home);
        if (e != hipSuccess) return e;
        sv->home_recorded = sv->home_epoch;
    }
    e = hipStreamWaitEvent(ln.stream, sv->home_ev, 0);
    if (e == hipSuccess) ln.home_seen = sv->home_epoch;
    return e;
}

// one launch of pending tiles on an idle lane, oldest admitted request first,
// up to the launch's work
mcdi_status srv_launch(mcdi_server sv, bool* launched) {
    *launched = false;
    int li = -1;
    for (int i = 0; i < kLanes && li < 0; ++i)
        if (!sv->lane[i].busy) li = i;
    if (li < 0) return MCDI_OK;
    SrvLane& ln = sv->lane[li];
    struct Pick { SrvReq* r; int64_t first, count; };
    std::vector<Pick> picks;
    int64_t budget = sv->cfg.launch_samples;
    for (SrvReq* r : sv->admitted) {
        if (r->next_tile >= r->tiles || budget <= 0) continue;
        const int64_t per_tile = (int64_t)kBlock * r->args.spp * (r->grad ? 2 : 1);
        int64_t take = budget / per_tile;
        take = take < 1 ? 1 : take;
        take = take < r->tiles - r->next_tile ? take : r->tiles - r->next_tile;
        picks.push_back({r, r->next_tile, take});
        budget -= take * per_tile;
    }
    if (picks.empty()) return MCDI_OK;
    if ((int)picks.size() > sv->cfg.slots) return fail(MCDI_E_DEVICE, "mcdi_server_poll: item buffer too small");
    ServeItem* h = ln.staging;   // the lane's previous copy has completed (its launch finished)
    int64_t total = 0;
    int max_H = 1;
    for (size_t i = 0; i < picks.size(); ++i) {
        SrvReq* r = picks[i].r;
        ShadeArgs a = r->args;
        a.hitbits_in = r->hitbits;
        a.origins = r->origins;
        a.rays = ln.rays;   // marks tracing available; regions are per workgroup
        h[i].args = a;
        h[i].hitbits = r->hitbits;
        h[i].first_tile = picks[i].first;
        h[i].first_global = total;
        total += picks[i].count;
        if (a.env.H > max_H) max_H = a.env.H;
    }
    if (total >= ((int64_t)1 << 31)) return fail(MCDI_E_UNSUPPORTED, "mcdi_server_poll: too many tiles");
    SrvLaunch L;
    L.lane = li;
    L.done = srv_event(sv);
    if (!L.done) return fail(MCDI_E_DEVICE, "mcdi_server_poll: event creation failed");
    hipError_t e = srv_sync_home(sv, ln);
    // inputs: after the caller's writes on its stream
    for (const Pick& p : picks)
        if (e == hipSuccess && p.r->ready && !(p.r->ready_seen & (1u << li))) {
            e = hipStreamWaitEvent(ln.stream, p.r->ready, 0);
            p.r->ready_seen |= 1u << li;
        }
    if (e == hipSuccess)
        e = hipMemcpyAsync(ln.items_dev, h, sizeof(ServeItem) * picks.size(), hipMemcpyHostToDevice, ln.stream);
    std::vector<mcdi_scene> scenes;
    for (const Pick& p : picks)
        if (std::find(scenes.begin(), scenes.end(), p.r->scene_handle) == scenes.end())
            scenes.push_back(p.r->scene_handle);
    for (mcdi_scene sc : scenes)
        if (e == hipSuccess) e = scene_acquire(sc, ln.stream);
    if (e == hipSuccess)
        e = launch_serve(ln.items_dev, (int)picks.size(), total, ln.counter, ln.rays, sv->cfg.spp_max,
                         sv->cfg.n_workgroups, max_H, ln.stream);
    for (mcdi_scene sc : scenes)
        if (e == hipSuccess) e = scene_release(sc, ln.stream);
    if (e == hipSuccess) e = hipEventRecord(L.done, ln.stream);
    if (e != hipSuccess) {
        sv->spare_events.push_back(L.done);
        return fail(MCDI_E_DEVICE, "mcdi_server_poll: %s", hipGetErrorString(e));
    }
    for (const Pick& p : picks) {
        p.r->next_tile += p.count;
        ++p.r->outstanding;
        L.reqs.push_back(p.r);
    }
    ln.busy = true;
    sv->in_flight.push_back(L);
    ++sv->launches;
    *launched = true;
    return MCDI_OK;
}

// retire, admit, and keep both lanes busy
mcdi_status srv_pump(mcdi_server sv, bool block) {
    mcdi_status st = srv_retire(sv, block);
    if (st != MCDI_OK) return st;
    srv_admit(sv);
    for (;;) {
        bool launched = false;
        st = srv_launch(sv, &launched);
        if (st != MCDI_OK || !launched) return st;
    }
}

}  // namespace

extern "C" {

int64_t mcdi_server_request_bytes(int64_t n_pixels, int32_t spp) {
    if (n_pixels < 0 || spp < 1) return 0;
    return (int64_t)srv_request_bytes(n_pixels, spp);
}

mcdi_status mcdi_server_create(const mcdi_server_config* cfg, const mcdi_allocator* alloc, void* stream,
                               mcdi_server* out) {
    if (!out || !cfg) return fail(MCDI_E_INVALID, "mcdi_server_create: NULL argument");
    if (cfg->spp_max < 1 || cfg->spp_max > 1024)
        return fail(MCDI_E_INVALID, "mcdi_server_create: spp_max must be in [1, 1024]");
    if (cfg->n_workgroups < 0 || cfg->n_workgroups > 65536)
        return fail(MCDI_E_INVALID, "mcdi_server_create: bad n_workgroups");
    if (cfg->slots < 1 || cfg->slots > 65536 || cfg->budget_bytes < 1 || cfg->launch_samples < 1)
        return fail(MCDI_E_INVALID,
                    "mcdi_server_create: slots must be in [1, 65536], budget_bytes and launch_samples >= 1");
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(MCDI_E_INVALID, "mcdi_server_create: allocator incomplete");
    mcdi_server sv = new (std::nothrow) mcdi_server_s;
    if (!sv) return fail(MCDI_E_OOM, "mcdi_server_create: host allocation failed");
    sv->alloc = make_alloc(alloc);
    sv->home = (hipStream_t)stream;
    sv->cfg = *cfg;
    if (sv->cfg.n_workgroups == 0) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        sv->cfg.n_workgroups = 4 * cus;
    }
    bool dev_ok = hipEventCreateWithFlags(&sv->home_ev, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < kLanes && dev_ok; ++i)
        dev_ok = hipStreamCreateWithFlags(&sv->lane[i].stream, hipStreamNonBlocking) == hipSuccess;
    if (!dev_ok) {
        (void)hipGetLastError();
        mcdi_server_destroy(sv);
        return fail(MCDI_E_DEVICE, "mcdi_server_create: stream or event creation failed");
    }
    bool mem_ok = true;
    for (int i = 0; i < kLanes && mem_ok; ++i) {
        SrvLane& ln = sv->lane[i];
        ln.rays = (float4*)srv_get(sv, sizeof(float4) * (size_t)sv->cfg.n_workgroups * 2 * sv->cfg.spp_max * kBlock);
        ln.counter = (int*)srv_get(sv, sizeof(int));
        // one item per admitted request at most: the item buffers never grow
        ln.items_dev = (ServeItem*)srv_get(sv, sizeof(ServeItem) * (size_t)sv->cfg.slots);
        if (hipHostMalloc((void**)&ln.staging, sizeof(ServeItem) * (size_t)sv->cfg.slots, hipHostMallocDefault) !=
            hipSuccess) {
            (void)hipGetLastError();
            ln.staging = nullptr;
        }
        mem_ok = ln.rays && ln.counter && ln.items_dev && ln.staging;
    }
    if (!mem_ok) {
        mcdi_server_destroy(sv);
        return fail(MCDI_E_OOM, "mcdi_server_create: allocation failed");
    }
    *out = sv;
    return ok();
}

mcdi_status mcdi_server_submit(mcdi_server sv, const mcdi_request* req, void* input_stream, int64_t* ticket) {
    if (!sv || !req || !ticket) return fail(MCDI_E_INVALID, "mcdi_server_submit: NULL argument");
    ShadeArgs a;
    mcdi_status st = fill_common("mcdi_server_submit", req->scene, req->env, &req->gbuf, &req->params, a);
    if (st != MCDI_OK) return st;
    if (req->params.spp > sv->cfg.spp_max) return fail(MCDI_E_INVALID, "mcdi_server_submit: spp > spp_max");
    if (req->params.flags & (MCDI_FLAG_DUMP | MCDI_FLAG_DUMP_DIRS | MCDI_FLAG_TIME_TRACE | MCDI_FLAG_TIME_ADJOINT))
        return fail(MCDI_E_INVALID, "mcdi_server_submit: dump and timing flags are not served");
    if (!req->c_d || !req->c_s) return fail(MCDI_E_INVALID, "mcdi_server_submit: NULL c_d/c_s");
    if (req->g_cd && (!req->g_cs || !req->g_kd || !req->g_korm || !req->g_nrm))
        return fail(MCDI_E_INVALID, "mcdi_server_submit: incomplete gradient buffers");
    const size_t bytes = srv_request_bytes(a.g.n, a.spp);
    if (bytes > (size_t)sv->cfg.budget_bytes)
        return fail(MCDI_E_UNSUPPORTED, "mcdi_server_submit: request needs %zu bytes, above the budget %lld", bytes,
                    (long long)sv->cfg.budget_bytes);
    SrvReq* r = new (std::nothrow) SrvReq;
    if (!r) return fail(MCDI_E_OOM, "mcdi_server_submit: host allocation failed");
    a.c_d = req->c_d;
    a.c_s = req->c_s;
    a.g_cd = req->g_cd;
    a.g_cs = req->g_cs;
    a.g_kd = req->g_kd;
    a.g_korm = req->g_korm;
    a.g_nrm = req->g_nrm;
    a.g_env = req->g_cd ? req->g_env : nullptr;
    r->args = a;
    r->scene_handle = req->scene;
    r->grad = req->g_cd != nullptr;
    r->tiles = (a.g.n + kBlock - 1) / kBlock;
    r->bytes = bytes;
    r->ready = srv_event(sv);
    if (!r->ready || hipEventRecord(r->ready, (hipStream_t)input_stream) != hipSuccess) {
        (void)hipGetLastError();
        if (r->ready) sv->spare_events.push_back(r->ready);
        delete r;
        return fail(MCDI_E_DEVICE, "mcdi_server_submit: event record on the input stream failed");
    }
    r->ticket = sv->next_ticket++;
    sv->queue.push_back(r);
    *ticket = r->ticket;
    st = srv_pump(sv, false);
    return st == MCDI_OK ? ok() : st;
}

static int32_t srv_report(mcdi_server sv, int64_t* done, int32_t cap) {
    int32_t k = 0;
    while (k < cap && !sv->completed.empty()) {
        done[k++] = sv->completed.front();
        sv->completed.pop_front();
    }
    return k;
}

mcdi_status mcdi_server_poll(mcdi_server sv, int64_t* done, int32_t cap, int32_t* n_done) {
    if (!sv || !n_done || (cap > 0 && !done)) return fail(MCDI_E_INVALID, "mcdi_server_poll: NULL argument");
    const mcdi_status st = srv_pump(sv, false);
    *n_done = srv_report(sv, done, cap);
    return st == MCDI_OK ? ok() : st;
}

mcdi_status mcdi_server_wait(mcdi_server sv, int64_t* done, int32_t cap, int32_t* n_done) {
    if (!sv || !n_done || (cap > 0 && !done)) return fail(MCDI_E_INVALID, "mcdi_server_wait: NULL argument");
    mcdi_status st = MCDI_OK;
    while (sv->completed.empty() && (!sv->in_flight.empty() || !sv->queue.empty() || !sv->admitted.empty())) {
        st = srv_pump(sv, true);
        if (st != MCDI_OK) break;
        if (sv->in_flight.empty() && sv->completed.empty()) {
            // nothing could be launched: the allocator refused the admission
            st = fail(MCDI_E_OOM, "mcdi_server_wait: requests cannot be admitted (device allocation failed)");
            break;
        }
    }
    *n_done = srv_report(sv, done, cap);
    return st == MCDI_OK ? ok() : st;
}

mcdi_status mcdi_server_info(mcdi_server sv, mcdi_server_info_t* info) {
    if (!sv || !info) return fail(MCDI_E_INVALID, "mcdi_server_info: NULL argument");
    info->used_bytes = (int64_t)sv->used;
    info->launches = sv->launches;
    info->queued = (int32_t)sv->queue.size();
    info->admitted = (int32_t)sv->admitted.size();
    info->in_flight = (int32_t)sv->in_flight.size();
    info->reserved = 0;
    return ok();
}

void mcdi_server_destroy(mcdi_server sv) {
    if (!sv) return;
    for (int i = 0; i < kLanes; ++i)
        if (sv->lane[i].stream) (void)hipStreamSynchronize(sv->lane[i].stream);
    for (SrvLaunch& L : sv->in_flight) sv->spare_events.push_back(L.done);
    for (SrvReq* r : sv->admitted) {
        srv_release(sv, r);
        delete r;
    }
    for (SrvReq* r : sv->queue) {
        srv_release(sv, r);
        delete r;
    }
    for (int i = 0; i < kLanes; ++i) {
        SrvLane& ln = sv->lane[i];
        sv->alloc.put(ln.rays, sv->home);
        sv->alloc.put(ln.counter, sv->home);
        sv->alloc.put(ln.items_dev, sv->home);
        if (ln.staging) (void)hipHostFree(ln.staging);
        if (ln.stream) (void)hipStreamDestroy(ln.stream);
    }
    for (hipEvent_t e : sv->spare_events) (void)hipEventDestroy(e);
    if (sv->home_ev) (void)hipEventDestroy(sv->home_ev);
    delete sv;
}

mcdi_status mcdi_image_loss(const float* kd, const float* c_d, const float* c_s, const float* ref,
                            const uint8_t* mask, int64_t n, float w_light, float* loss, float* g_kd, float* g_cd,
                            float* g_cs, const mcdi_allocator* alloc, void* stream) {
    if (!kd || !c_d || !c_s || !ref || !mask || !loss) return fail(MCDI_E_INVALID, "mcdi_image_loss: NULL input");
    if (n < 1) return fail(MCDI_E_INVALID, "mcdi_image_loss: n must be >= 1");
    if (n >= ((int64_t)1 << 31)) return fail(MCDI_E_UNSUPPORTED, "mcdi_image_loss: n >= 2^31");
    if (!std::isfinite(w_light)) return fail(MCDI_E_INVALID, "mcdi_image_loss: w_light must be finite");
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(MCDI_E_INVALID, "mcdi_image_loss: allocator incomplete");
    hipStream_t s = (hipStream_t)stream;
    Alloc al = make_alloc(alloc);
    void* scratch = al.get(image_loss_scratch_bytes(n), s);
    if (!scratch) return fail(MCDI_E_OOM, "mcdi_image_loss: scratch allocation failed");
    hipError_t e = launch_image_loss(kd, c_d, c_s, ref, mask, n, w_light, loss, g_kd, g_cd, g_cs, scratch, s);
    al.put(scratch, s);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_image_loss: %s", hipGetErrorString(e));
    return ok();
}

mcdi_status mcdi_image_loss_noalloc(const float* kd, const float* c_d, const float* c_s, const float* ref,
                                    const uint8_t* mask, int64_t n, float w_light, float* loss, float* g_kd,
                                    float* g_cd, float* g_cs, void* stream) {
    if (!kd || !c_d || !c_s || !ref || !mask || !loss)
        return fail(MCDI_E_INVALID, "mcdi_image_loss_noalloc: NULL input");
    if (n < 1) return fail(MCDI_E_INVALID, "mcdi_image_loss_noalloc: n must be >= 1");
    if (n >= ((int64_t)1 << 31)) return fail(MCDI_E_UNSUPPORTED, "mcdi_image_loss_noalloc: n >= 2^31");
    if (!std::isfinite(w_light)) return fail(MCDI_E_INVALID, "mcdi_image_loss_noalloc: w_light must be finite");
    if (image_loss_scratch_bytes(n) > kLossStaticScratch)
        return fail(MCDI_E_UNSUPPORTED, "mcdi_image_loss_noalloc: n = %lld needs %zu bytes of scratch, above the "
                    "static %zu", (long long)n, image_loss_scratch_bytes(n), kLossStaticScratch);
    // the current device's static scratch: no allocation; every entry the
    // kernels read is written earlier in the same call, so nothing is cleared
    void* scratch = nullptr;
    hipError_t e = image_loss_static_scratch(&scratch);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_image_loss_noalloc: %s", hipGetErrorString(e));
    e = launch_image_loss(kd, c_d, c_s, ref, mask, n, w_light, loss, g_kd, g_cd, g_cs, scratch, (hipStream_t)stream);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_image_loss_noalloc: %s", hipGetErrorString(e));
    return ok();
}

static mcdi_status bilat_args(const char* who, const mcdi_bilateral_guide* g, int32_t nc, BilatArgs& a) {
    if (!g) return fail(MCDI_E_INVALID, "%s: NULL guide", who);
    if (g->n_views < 0 || g->height < 0 || g->width < 0)
        return fail(MCDI_E_INVALID, "%s: negative size", who);
    const int64_t n = (int64_t)g->n_views * g->height * g->width;
    if (n >= ((int64_t)1 << 31)) return fail(MCDI_E_UNSUPPORTED, "%s: n_views*height*width >= 2^31", who);
    if (nc != 1 && nc != 3 && nc != 6) return fail(MCDI_E_UNSUPPORTED, "%s: n_chan must be 1, 3 or 6", who);
    if (!(std::isfinite(g->sigma) && g->sigma > 0.0f)) return fail(MCDI_E_INVALID, "%s: sigma must be > 0", who);
    if (!(std::isfinite(g->sigma_z) && g->sigma_z >= 0.0f))
        return fail(MCDI_E_INVALID, "%s: sigma_z must be >= 0", who);
    if (!(std::isfinite(g->sigma_n) && g->sigma_n > 0.0f))
        return fail(MCDI_E_INVALID, "%s: sigma_n must be > 0", who);
    if (n > 0 && (!g->depth || !g->nrm || !g->mask)) return fail(MCDI_E_INVALID, "%s: NULL guide buffer", who);
    a = BilatArgs{g->n_views, g->height, g->width, n, g->depth, g->nrm, g->mask,
                  g->sigma, g->sigma_z, g->sigma_n, bilateral_radius(g->sigma), 0, 0};
    bilateral_tiles(a);
    if ((int64_t)a.tiles_x * a.tiles_y * a.V >= ((int64_t)1 << 31))
        return fail(MCDI_E_UNSUPPORTED, "%s: too many tiles", who);
    return MCDI_OK;
}

int32_t mcdi_bilateral_radius(float sigma) { return bilateral_radius(sigma); }

mcdi_status mcdi_bilateral_fwd(const mcdi_bilateral_guide* g, int32_t nc, const float* in, float* out,
                               float* wsum, void* stream) {
    BilatArgs a;
    mcdi_status st = bilat_args("mcdi_bilateral_fwd", g, nc, a);
    if (st != MCDI_OK) return st;
    if (a.n > 0 && (!in || !out)) return fail(MCDI_E_INVALID, "mcdi_bilateral_fwd: NULL colour buffer");
    if (a.n > 0 && (const float*)out == in) return fail(MCDI_E_INVALID, "mcdi_bilateral_fwd: out aliases in");
    hipError_t e = launch_bilateral_fwd(a, nc, in, out, wsum, (hipStream_t)stream);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_bilateral_fwd: %s", hipGetErrorString(e));
    return ok();
}

mcdi_status mcdi_bilateral_bwd(const mcdi_bilateral_guide* g, int32_t nc, const float* g_out, const float* wsum,
                               float* g_in, void* stream) {
    BilatArgs a;
    mcdi_status st = bilat_args("mcdi_bilateral_bwd", g, nc, a);
    if (st != MCDI_OK) return st;
    if (a.n > 0 && (!g_out || !wsum || !g_in)) return fail(MCDI_E_INVALID, "mcdi_bilateral_bwd: NULL buffer");
    if (a.n > 0 && (const float*)g_in == g_out) return fail(MCDI_E_INVALID, "mcdi_bilateral_bwd: g_in aliases g_out");
    hipError_t e = launch_bilateral_bwd(a, nc, g_out, wsum, g_in, (hipStream_t)stream);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_bilateral_bwd: %s", hipGetErrorString(e));
    return ok();
}

mcdi_status mcdi_view_depth(const mcdi_gbuffer* g, float* depth, void* stream) {
    if (!g) return fail(MCDI_E_INVALID, "mcdi_view_depth: NULL gbuffer");
    if (g->n_views < 0 || g->height < 0 || g->width < 0) return fail(MCDI_E_INVALID, "mcdi_view_depth: negative size");
    const int64_t n = (int64_t)g->n_views * g->height * g->width;
    if (n >= ((int64_t)1 << 31)) return fail(MCDI_E_UNSUPPORTED, "mcdi_view_depth: n >= 2^31");
    if (n > 0 && (!g->pos || !g->mask || !g->eye || !depth)) return fail(MCDI_E_INVALID, "mcdi_view_depth: NULL buffer");
    GBufView v{g->n_views, g->height, g->width, g->view_base, g->pos, g->nrm, g->kd, g->korm, g->mask, g->eye, n};
    hipError_t e = launch_view_depth(v, depth, (hipStream_t)stream);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_view_depth: %s", hipGetErrorString(e));
    return ok();
}

mcdi_status mcdi_trace_anyhit(mcdi_scene sc, const float* orig, const float* dir, int64_t n, uint8_t* hit,
                              int32_t brute, void* stream) {
    if (!sc) return fail(MCDI_E_INVALID, "mcdi_trace_anyhit: NULL scene");
    if (n < 0) return fail(MCDI_E_INVALID, "mcdi_trace_anyhit: negative n");
    if (n >= (int64_t)1 << 31) return fail(MCDI_E_UNSUPPORTED, "mcdi_trace_anyhit: n >= 2^31");
    if (n > 0 && (!orig || !dir || !hit)) return fail(MCDI_E_INVALID, "mcdi_trace_anyhit: NULL buffer");
    if (brute < 0 || brute > 2) return fail(MCDI_E_INVALID, "mcdi_trace_anyhit: mode must be 0, 1 or 2");
    hipError_t e = scene_acquire(sc, (hipStream_t)stream);
    if (e == hipSuccess)
        e = launch_trace(scene_view(sc), orig, dir, n, hit, brute, (hipStream_t)stream);
    if (e == hipSuccess) e = scene_release(sc, (hipStream_t)stream);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_trace_anyhit: %s", hipGetErrorString(e));
    return ok();
}

struct mcdi_edges_s {
    Alloc alloc;
    hipStream_t stream = nullptr;
    int64_t n_verts = 0, n_tris = 0;
    int4* rows = nullptr;        // [max(3 n_tris, 1)]
    uint32_t* count = nullptr;   // E
};

mcdi_status mcdi_build_edges(const int32_t* tris, int64_t n_tris, int64_t n_verts, const mcdi_allocator* alloc,
                             void* stream, mcdi_edges* out) {
    if (!out) return fail(MCDI_E_INVALID, "mcdi_build_edges: out is NULL");
    if (n_verts < 0 || n_tris < 0) return fail(MCDI_E_INVALID, "mcdi_build_edges: negative count");
    if (n_verts >= (int64_t)1 << 31) return fail(MCDI_E_UNSUPPORTED, "mcdi_build_edges: n_verts >= 2^31");
    if (n_tris >= (int64_t)1 << 26) return fail(MCDI_E_UNSUPPORTED, "mcdi_build_edges: n_tris >= 2^26");
    if (n_tris > 0 && !tris) return fail(MCDI_E_INVALID, "mcdi_build_edges: NULL tris");
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(MCDI_E_INVALID, "mcdi_build_edges: allocator incomplete");
    hipStream_t s = (hipStream_t)stream;
    mcdi_edges ed = new (std::nothrow) mcdi_edges_s;
    if (!ed) return fail(MCDI_E_OOM, "mcdi_build_edges: host allocation failed");
    ed->alloc = make_alloc(alloc);
    ed->stream = s;
    ed->n_verts = n_verts;
    ed->n_tris = n_tris;
    const int64_t sides = 3 * n_tris;
    ed->rows = (int4*)ed->alloc.get(sizeof(int4) * (size_t)(sides > 0 ? sides : 1), s);
    ed->count = (uint32_t*)ed->alloc.get(sizeof(uint32_t), s);
    const int bits = edge_table_bits(sides);
    const size_t slots = (size_t)1 << bits;
    const uint32_t nb = edge_scan_blocks(sides);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t sz_keys = al(sizeof(unsigned long long) * slots), sz_slot = al(sizeof(uint32_t) * slots);
    const size_t sz_of = al(sizeof(uint32_t) * (size_t)(sides > 0 ? sides : 1));
    const size_t sz_b = al(sizeof(uint32_t) * ((size_t)nb + 1));
    void* tmp = ed->rows && ed->count ? ed->alloc.get(sz_keys + 2 * sz_slot + sz_of + sz_b, s) : nullptr;
    if (!tmp) {
        mcdi_destroy_edges(ed);
        return fail(MCDI_E_OOM, "mcdi_build_edges: device allocation failed (%lld triangles)", (long long)n_tris);
    }
    char* p = (char*)tmp;
    unsigned long long* keys = (unsigned long long*)p;
    uint32_t* first = (uint32_t*)(p + sz_keys);
    uint32_t* second = (uint32_t*)(p + sz_keys + sz_slot);
    uint32_t* slot_of = (uint32_t*)(p + sz_keys + 2 * sz_slot);
    uint32_t* bsum = (uint32_t*)(p + sz_keys + 2 * sz_slot + sz_of);
    hipError_t e = launch_edges_build(tris, n_tris, n_verts, bits, keys, first, second, slot_of, bsum, ed->rows,
                                      ed->count, s);
    ed->alloc.put(tmp, s);
    if (e != hipSuccess) {
        mcdi_destroy_edges(ed);
        return fail(MCDI_E_DEVICE, "mcdi_build_edges: %s", hipGetErrorString(e));
    }
    *out = ed;
    return ok();
}

void mcdi_destroy_edges(mcdi_edges ed) {
    if (!ed) return;
    ed->alloc.put(ed->rows, ed->stream);
    ed->alloc.put(ed->count, ed->stream);
    delete ed;
}

mcdi_status mcdi_edges_count(mcdi_edges ed, int64_t* n_edges) {
    if (!ed || !n_edges) return fail(MCDI_E_INVALID, "mcdi_edges_count: NULL argument");
    uint32_t h = 0;
    hipError_t e = hipStreamSynchronize(ed->stream);
    if (e == hipSuccess) e = hipMemcpy(&h, ed->count, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_edges_count: %s", hipGetErrorString(e));
    *n_edges = (int64_t)h;
    return ok();
}

mcdi_status mcdi_edges_copy(mcdi_edges ed, int32_t* rows, void* stream) {
    if (!ed || !rows) return fail(MCDI_E_INVALID, "mcdi_edges_copy: NULL argument");
    int64_t n = 0;
    mcdi_status st = mcdi_edges_count(ed, &n);
    if (st != MCDI_OK) return st;
    if (n == 0) return ok();
    hipError_t e = hipMemcpyAsync(rows, ed->rows, sizeof(int4) * (size_t)n, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_edges_copy: %s", hipGetErrorString(e));
    return ok();
}

mcdi_status mcdi_shade_bwd_edges(mcdi_scene sc, mcdi_env ev, mcdi_edges ed, const float* verts, int64_t n_verts,
                                 const mcdi_gbuffer* g, const mcdi_params* p, int32_t edge_spp, uint32_t sharp_gain,
                                 const float* g_cd, const float* g_cs, float* g_verts, mcdi_stats* stats,
                                 void* stream) {
    ShadeArgs a;
    mcdi_status st = fill_common("mcdi_shade_bwd_edges", sc, ev, g, p, a);
    if (st != MCDI_OK) return st;
    if (p->flags & MCDI_FLAG_DUMP) return fail(MCDI_E_INVALID, "mcdi_shade_bwd_edges: MCDI_FLAG_DUMP is forward-only");
    if (!ed) return fail(MCDI_E_INVALID, "mcdi_shade_bwd_edges: NULL edges");
    if (n_verts != ed->n_verts)
        return fail(MCDI_E_INVALID, "mcdi_shade_bwd_edges: n_verts %lld differs from the edges' %lld",
                    (long long)n_verts, (long long)ed->n_verts);
    if (edge_spp < 1 || edge_spp > 1024)
        return fail(MCDI_E_INVALID, "mcdi_shade_bwd_edges: edge_spp must be in [1, 1024]");
    if (sharp_gain < 1 || sharp_gain > kSharpGainMax)
        return fail(MCDI_E_INVALID, "mcdi_shade_bwd_edges: sharp_gain must be in [1, %u]", kSharpGainMax);
    if (!g_cd || !g_cs || (n_verts > 0 && (!verts || !g_verts)))
        return fail(MCDI_E_INVALID, "mcdi_shade_bwd_edges: NULL buffer");
    if (a.tau == 0.0f || ed->n_tris == 0) return ok();
    hipStream_t s = (hipStream_t)stream;
    a.g_cd = g_cd;
    a.g_cs = g_cs;
    a.stats = stats;
    EdgeArgs E;
    std::memset(&E, 0, sizeof(E));
    E.a = a;
    E.edges = ed->rows;
    E.n_edges = ed->count;
    E.verts = verts;
    E.g_verts = g_verts;
    E.n_es = edge_spp;
    E.gain = sharp_gain;
    // pixels per pass: every sample of a pass fits the queue, and the pixel
    // in pass fits its 22 bits of the record
    int64_t per = ((int64_t)(kEdgeQueueMax / (uint32_t)edge_spp) / kBlock) * kBlock;
    if (per > kEdgePassMax) per = kEdgePassMax;
    const int64_t n = a.g.n;
    const int64_t chunk = per < n ? per : ((n + kBlock - 1) / kBlock) * kBlock;
    E.q_cap = (uint32_t)(chunk * edge_spp);
    Workspace ws;
    ws.alloc = &sc->alloc;
    ws.s = s;
    const size_t sz_q = ((sizeof(uint32_t) * (size_t)E.q_cap) + 255) & ~(size_t)255;
    const uint32_t cap_edges = (uint32_t)(3 * ed->n_tris);   // at most one edge per triangle side
    const size_t sz_geo = sizeof(float4) * 4 * (size_t)cap_edges;
    const size_t sz_bsum = ((sizeof(uint32_t) * ((size_t)edge_pack_blocks(cap_edges) + 1)) + 255) & ~(size_t)255;
    ws.base = sc->alloc.get(sz_q + 256 + sz_geo + sz_bsum, s);
    if (!ws.base) return fail(MCDI_E_OOM, "mcdi_shade_bwd_edges: workspace allocation failed");
    E.queue = (uint32_t*)ws.base;
    E.q_count = (uint32_t*)((char*)ws.base + sz_q);
    uint32_t* n_sharp = E.q_count + 1;
    E.n_sharp = n_sharp;
    E.egeo = (const float4*)((char*)ws.base + sz_q + 256);
    uint32_t* bsum = (uint32_t*)((char*)ws.base + sz_q + 256 + sz_geo);
    hipError_t pe = launch_edge_pack(E, cap_edges, bsum, n_sharp, s);
    if (pe == hipSuccess) pe = scene_acquire(sc, s);
    if (pe != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_shade_bwd_edges: %s", hipGetErrorString(pe));
    for (int64_t p0 = 0; p0 < n; p0 += chunk) {
        E.pix0 = p0;
        E.npix = n - p0 < chunk ? n - p0 : chunk;
        std::pair<hipEvent_t, hipEvent_t>* tev = (a.flags & MCDI_FLAG_TIME_ADJOINT) ? timer_next(g_timer_adj) : nullptr;
        hipError_t e = tev ? launch_edge_grad(E, s, tev->first, tev->second) : launch_edge_grad(E, s);
        if (e != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_shade_bwd_edges: %s", hipGetErrorString(e));
    }
    hipError_t re = scene_release(sc, s);
    if (re != hipSuccess) return fail(MCDI_E_DEVICE, "mcdi_shade_bwd_edges: %s", hipGetErrorString(re));
    return ok();
}

}  // extern "C"
