/*
 * mcdi.h -- C ABI of the differentiable Monte Carlo direct-illumination
 * library for AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, per G-buffer pixel, the direct-illumination
 * rendering equation against an HDR environment probe with shadow rays
 * (Hasselgren, Hofmann & Munkberg, NeurIPS 2022, section 3.1 "Direct
 * Illumination"), estimated by Monte Carlo with multiple importance sampling
 * over three techniques -- a piecewise-constant 2D distribution over the
 * probe, cosine sampling of the diffuse lobe and GGX visible-normal sampling
 * (section 4.1 "Multiple Importance Sampling"; appendix D "Sampling") -- and
 * returns diffuse lighting demodulated from the albedo and specular lighting
 * separately (section 4.2 "Denoising").  The backward pass replays the same
 * random numbers (section 4.1; appendix D) and differentiates only the
 * material evaluation: sampling and visibility are detached (section 3.1
 * "Shadow gradients"; section 4.1).  Shadowed samples are weighted by
 * H = 1 - tau (appendix A "Optimization and Regularization").
 *
 * Conventions shared by every call:
 *   - Pointers named as device buffers are device memory owned by the caller;
 *     the library never frees them.  Handles own the device memory they
 *     allocate, through the optional allocator hook (NULL: stream-ordered
 *     hipMallocAsync / hipFreeAsync).
 *   - `stream` is a hipStream_t passed as void*.  Every call only enqueues
 *     work on it and returns; nothing synchronises the device unless stated.
 *   - Per-pixel arrays are planar float32 [C][N], N = n_views*height*width,
 *     pixel id (view*height + y)*width + x.
 *   - Status codes only; no C++ exception crosses the ABI.  Arguments are
 *     validated before anything is enqueued; a non-OK status leaves every
 *     output untouched.  mcdi_last_error() returns a thread-local message for
 *     the last non-OK status of the calling thread.
 *   - Data-dependent anomalies are not errors: a pixel with a non-finite
 *     input, a zero normal or a zero view vector shades to 0 and gets zero
 *     gradients (counted in mcdi_stats); a probe whose total luminance is 0
 *     disables the light technique.
 */
#ifndef MCDI_H
#define MCDI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MCDI_OK = 0,
    MCDI_E_INVALID = -1,     /* bad argument (null pointer, size, range) */
    MCDI_E_OOM = -2,         /* device allocation failed */
    MCDI_E_DEVICE = -3,      /* HIP runtime error while enqueuing */
    MCDI_E_UNSUPPORTED = -4  /* size beyond a documented limit */
} mcdi_status;

typedef struct mcdi_scene_s* mcdi_scene; /* opaque BVH over a triangle mesh */
typedef struct mcdi_env_s* mcdi_env;     /* opaque probe sampling tables */

/* Optional device allocator (e.g. a framework's caching allocator).
 * alloc returns device memory usable in stream order on `stream`, aligned to
 * 256 bytes, or NULL; free releases it in stream order.  A misaligned block
 * is handed back to free and the call fails with MCDI_E_OOM. */
typedef struct {
    void* ctx;
    void* (*alloc)(void* ctx, size_t bytes, void* stream);
    void (*free)(void* ctx, void* ptr, void* stream);
} mcdi_allocator;

/* ---------------------------------------------------------------------------
 * Scene: the triangle mesh the shadow rays are traced against (the mesh the
 * paper extracts every iteration, section 3 and figure "system").
 *
 * verts   device float32 [n_verts][3]
 * tris    device int32   [n_tris][3], vertex indices
 * Builds a bounding-volume hierarchy on the device (Morton-ordered linear BVH,
 * leaves of <= 4 triangles, depth-first node order with skip links), and a
 * copy of its nodes whose boxes are quantised outward to 16 bits per
 * coordinate against the scene's bounding box (16 bytes per node; a box grows
 * by at most 1/65535 of the scene's extent per side, which costs box tests,
 * never a wrong answer), and a 4-wide hierarchy: the binary tree collapsed
 * every other level, each wide node holding the quantised boxes and
 * references of up to four children in one 64-byte segment (one memory round
 * trip tests four boxes).  The build also measures the scene's depth
 * complexity (the leaf boxes' surface areas summed, over the root box's):
 * shadow rays walk the 4-wide hierarchy when it is at least 4 (volume-
 * filling geometry: long walks bound by memory latency), else the binary
 * one (surfaces: short cache-resident walks bound by instruction issue).
 * Either walk gives the same answers.
 * Big triangles (a box whose longest side is at least 1/8 of the longest side
 * of the triangle centroids' bounds: the walls around a scene, say) form the
 * root's first subtree, one triangle per leaf, when the mesh also has smaller
 * ones; both walks take that subtree first, so the shadow rays those big
 * occluders stop end early.
 * A triangle with an index outside [0, n_verts) or a non-finite vertex is
 * replaced by a degenerate triangle that no ray hits (counted in
 * mcdi_scene_info).  n_tris = 0 gives a scene every ray misses.
 * verts/tris are read during the call's stream work only; the handle keeps no
 * reference to them.  Limits: n_verts < 2^31, n_tris < 2^26 (node and triangle
 * byte offsets stay 32-bit).
 * Streams: every call that reads the scene makes its stream wait for the build
 * (an event), right before its first kernel that reads the BVH, so a scene may
 * be built on one stream and used on others, and the work of such a call that
 * does not need the BVH (ray generation) overlaps the build.
 * ------------------------------------------------------------------------- */
mcdi_status mcdi_build_scene(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                             const mcdi_allocator* alloc, void* stream, mcdi_scene* out);

/* Frees the scene's memory in stream order on the stream it was built on,
 * after the work of the last call that read the scene (also on another
 * stream).  With calls enqueued on several streams at once, only the last one
 * enqueued is waited for: the caller orders the others. */
void mcdi_destroy_scene(mcdi_scene scene);

typedef struct {
    int64_t n_tris;
    int32_t n_nodes;      /* BVH nodes after leaf collapsing */
    int32_t max_depth;    /* longest root-to-leaf path */
    int32_t bad_tris;     /* triangles replaced by degenerate ones */
    int32_t n_groups;     /* 4-wide nodes */
    int32_t wide;         /* 1: shadow rays walk the 4-wide hierarchy, 0: the binary one */
    float depth_complexity; /* sum of the leaf boxes' surface areas over the root box's */
    int32_t n_big;        /* big triangles (see mcdi_build_scene) */
} mcdi_scene_info_t;

/* Synchronises the scene's stream and reports build statistics. */
mcdi_status mcdi_scene_info(mcdi_scene scene, mcdi_scene_info_t* info);

/* Copies the scene's BVH, for inspection and tests, into caller device
 * buffers (either may be NULL), in stream order:
 *   nodes  n_nodes x 8 words (mcdi_scene_info), depth-first pre-order:
 *          float lo[3], int32 escape, float hi[3], int32 payload.  escape is
 *          the index just past the node's subtree (node 0: the node count);
 *          payload 0 = internal node (first child at index + 1), else
 *          (first_triangle << 3) | count (1..4) of a leaf;
 *   tris   n_tris x 12 floats: the triangles in leaf order, three vertices
 *          of (x, y, z, 0).
 * Byte counts: 32 n_nodes and 48 n_tris. */
mcdi_status mcdi_scene_nodes(mcdi_scene scene, void* nodes, float* tris, void* stream);

/* ---------------------------------------------------------------------------
 * Environment probe sampling tables (section 4.1: light importance sampling
 * with a piecewise-constant 2D distribution; rebuilt every optimisation
 * iteration because the probe is an optimisation variable).
 *
 * env_rgb  device float32 [H][W][3] linear radiance, lat-long: row i covers
 *          polar angle [i, i+1)*pi/H from +Y, column j covers azimuth
 *          [j, j+1)*2pi/W with azimuth = atan2(z, x).
 * Texel weight = max(0, (r+g+b)/3) * sin(pi (i+1/2)/H), summed left to right
 * in FP64; each table entry is rounded once to FP32:
 *   cond [H][W+1]  per-row CDF, cond[i][0] = 0, cond[i][W] = 1
 *   marg [H+1]     marginal CDF over rows
 *   pdf  [H][W]    (w_ij / sum w) * W * H, the texel's density in (u, v)
 * The handle also keeps a copy of the radiance, packed with the density as
 * one float4 (r, g, b, pdf) per texel so that a sample reads both from one
 * cache line.  env_rgb is read only by the build's stream work; shading uses
 * the copy, so a changed probe needs a new handle.
 * Limits: 1 <= H <= 4096, 1 <= W <= 4096.
 * ------------------------------------------------------------------------- */
mcdi_status mcdi_build_env_cdf(const float* env_rgb, int32_t H, int32_t W, const mcdi_allocator* alloc,
                               void* stream, mcdi_env* out);
/* Frees the tables in stream order on the stream they were built on.  Unlike
 * a scene, the tables carry no events: work on other streams that uses them
 * must be ordered after the build and before the destroy by the caller. */
void mcdi_destroy_env(mcdi_env env);

/* Copies the tables into caller device buffers (any may be NULL), in stream
 * order: cond [H][W+1], marg [H+1], pdf [H][W] float32. */
mcdi_status mcdi_env_tables(mcdi_env env, float* cond, float* marg, float* pdf, void* stream);

/* ---------------------------------------------------------------------------
 * Shading
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t n_views, height, width;
    int32_t view_base;      /* global id of view 0; keys the random numbers */
    const float* pos;       /* device [3][N] world position */
    const float* nrm;       /* device [3][N] shading normal (need not be unit) */
    const float* kd;        /* device [3][N] diffuse albedo */
    const float* korm;      /* device [3][N] (occlusion, roughness, metallic); occlusion unused */
    const uint8_t* mask;    /* device [N] nonzero = covered pixel */
    const float* eye;       /* device [n_views][3] camera position */
} mcdi_gbuffer;

/* Flags */
/* Technique subsets (the sampling ablation of appendix D: cosine, BSDF and
 * light-probe sampling alone against MIS; every subset is unbiased):
 *   LIGHT_OFF              BSDF sampling only (cosine/GGX mixture)
 *   BSDF_OFF               light-probe sampling only
 *   LIGHT_OFF | FORCE_COS  cosine sampling only
 *   LIGHT_OFF | FORCE_GGX  GGX visible-normal sampling only (cosine where n.v <= 0)
 * LIGHT_OFF with BSDF_OFF, and FORCE_COS with FORCE_GGX, are rejected. */
#define MCDI_FLAG_LIGHT_OFF   (1u << 0) /* no light-technique sample; p_light = 0 */
#define MCDI_FLAG_FORCE_COS   (1u << 1) /* lobe probability q = 1 (cosine only) */
#define MCDI_FLAG_BSDF_OFF    (1u << 2) /* no BSDF-technique sample; BSDF density not in the MIS sum */
#define MCDI_FLAG_FORCE_GGX   (1u << 3) /* lobe probability q = 0 where n.v > 0 (GGX only) */
/* Probe lookup filter (section 3.1 keeps the probe as a float texture and
 * names no filter).  Default: the nearest texel.  BILINEAR: tent weights
 * around texel centres (texel (i, j) centred at (j + 1/2, i + 1/2) in texel
 * units x = phi W / 2 pi, y = theta H / pi), columns wrapping across phi = 0,
 * rows clamped at the poles; a light sample is looked up at its own sampled
 * coordinates.  The light technique keeps the per-texel density, and the
 * probe gradient of a sample goes to its four taps.  Light-only sampling
 * (BSDF_OFF) never reaches the radiance that filtering spreads into texels of
 * zero sampling weight. */
#define MCDI_FLAG_BILINEAR    (1u << 4)
#define MCDI_FLAG_DUMP        (1u << 8) /* write per-sample decision records */
/* With MCDI_FLAG_DUMP: each record also holds the two sampled world
 * directions (FP32 bits; NaN where the technique drew none), 9 words instead
 * of 3 -- the parity protocol compares them with the oracle's. */
#define MCDI_FLAG_DUMP_DIRS   (1u << 10)
#define MCDI_FLAG_TIME_TRACE  (1u << 9) /* bracket the traversal kernel with HIP events */
#define MCDI_FLAG_TIME_ADJOINT (1u << 11) /* bracket the adjoint kernel of mcdi_shade_bwd, and the
                                             edge-sample kernel of each pass of mcdi_shade_bwd_edges,
                                             with HIP events */

typedef struct {
    int32_t spp;            /* samples per pixel, 1..1024; each = 1 light + 1 BSDF sample */
    uint32_t flags;
    uint64_t seed;          /* Philox4x32-10 key */
    float tau;              /* shadow weight: H = 1 - tau on hit (appendix A) */
    float ray_eps;          /* shadow-ray origin offset along the normal (world units) */
    uint32_t* decisions;    /* device [N][spp][3] when MCDI_FLAG_DUMP ([N][spp][9] with
                               MCDI_FLAG_DUMP_DIRS: words 3-5 and 6-8 the light and BSDF
                               samples' world directions), else NULL */
    uint32_t* live;         /* optional device [ceil(2 spp / 32)][N] u32 in the hit bits' layout
                               (bit 2s + t of word (2s + t) / 32: technique t of sample s; t = 0
                               light, 1 BSDF): the samples drawn with a density above the horizon,
                               which the estimator evaluates.  mcdi_shade_fwd writes it (when
                               tau != 0); mcdi_shade_bwd, given it with the same forward's hit
                               bits, draws and differentiates only those samples instead of
                               drawing every sample pair to find them -- the same gradients bit
                               for bit, less work where most samples are blocked or below the
                               horizon.  NULL: the forward keeps its own, the adjoint draws.
                               Ignored when tau is 0 and by the other calls. */
} mcdi_params;

/* Device-side counters, accumulated (+=) by every call that receives them.
 * Passing stats selects an instrumented instantiation of the same kernel. */
typedef struct {
    unsigned long long valid_pixels;
    unsigned long long invalid_pixels;   /* masked-in pixels with bad inputs */
    unsigned long long rays_traced;
    unsigned long long rays_hit;
    unsigned long long samples_culled;   /* below the horizon */
    unsigned long long box_tests;        /* child boxes tested (empty slots of wide nodes not counted) */
    unsigned long long tri_tests;        /* ray/triangle tests */
    unsigned long long box_slots;        /* lane slots of the box phase: 64 per wavefront step */
    unsigned long long tri_slots;        /* lane slots of the triangle phase */
    unsigned long long box_lanes;        /* lanes that stepped in the box phase, summed over its steps */
} mcdi_stats;

/* Forward pass.
 *   c_d, c_s  device [3][N] float32, overwritten: demodulated diffuse and
 *             specular lighting, so that the shaded colour is kd*c_d + c_s.
 *   hitbits   device uint32 [ceil(2*spp/32)][N] or NULL; bit 2s (2s+1) of a
 *             pixel = the light (BSDF) sample s was occluded.  Overwritten.
 *   stats     device mcdi_stats or NULL (accumulated).
 * Random numbers: Philox4x32-10 with key = seed and counter = (pixel in view,
 * view_base + view, s, block), blocks 0 and 1 per sample. */
mcdi_status mcdi_shade_fwd(mcdi_scene scene, mcdi_env env, const mcdi_gbuffer* gbuf,
                           const mcdi_params* params, float* c_d, float* c_s, uint32_t* hitbits,
                           mcdi_stats* stats, void* stream);

/* Test hook: the forward pass with frozen sampling.  The sampling G-buffer
 * g_s and probe env_s draw every sample, its technique densities (the
 * balance-heuristic denominator), the lobe choice q and the shadow ray; the
 * evaluation G-buffer g_e (its nrm, kd and korm planes) and probe env_e (its
 * radiance) evaluate the BSDF, the cosine and the incident radiance of each
 * sample (the sample's world direction re-expressed in g_e's shading frame).
 * With g_e = g_s and env_e = env_s it equals mcdi_shade_fwd.  Central
 * differences of it in the evaluation inputs are the derivatives that
 * mcdi_shade_bwd computes, since the backward pass detaches sampling
 * (section 4.1; section 3.1 "Shadow gradients").
 * g_e must share size, view_base, pos, mask and eye with g_s; the probes
 * must have the same size.  A pixel invalid in either G-buffer shades to 0.
 * Allocates the ray workspace and a copy of the probe texels from the
 * scene's allocator.  DUMP and TIME flags are rejected. */
mcdi_status mcdi_shade_fwd_frozen(mcdi_scene scene, mcdi_env env_s, const mcdi_gbuffer* g_s, mcdi_env env_e,
                                  const mcdi_gbuffer* g_e, const mcdi_params* params, float* c_d, float* c_s,
                                  void* stream);

/* Backward pass of the detached estimator, same samples as the forward.
 *   g_cd, g_cs   device [3][N] upstream gradients dL/dc_d, dL/dc_s
 *   hitbits      the forward pass's hit bits, or NULL to re-trace the rays
 *   g_kd, g_korm, g_nrm  device [3][N], overwritten (g_korm[0] = 0)
 *   g_env        device [H][W][3], ACCUMULATED (+=); the caller zeroes it.
 * Summation order of g_env is not deterministic (float atomics). */
mcdi_status mcdi_shade_bwd(mcdi_scene scene, mcdi_env env, const mcdi_gbuffer* gbuf,
                           const mcdi_params* params, const float* g_cd, const float* g_cs,
                           const uint32_t* hitbits, float* g_kd, float* g_korm, float* g_nrm,
                           float* g_env, mcdi_stats* stats, void* stream);

/* Any-hit queries for explicit rays (tests and tools).
 *   orig, dir  device float32 [3][n]; hit device uint8 [n] (1 = occluded),
 *   t in (0, inf), no culling.  mode (the `brute` argument): 0 traverses the
 *   binary hierarchy, 1 tests every triangle, 2 traverses the 4-wide
 *   hierarchy (the one the shading calls use). */
mcdi_status mcdi_trace_anyhit(mcdi_scene scene, const float* orig, const float* dir, int64_t n,
                              uint8_t* hit, int32_t brute, void* stream);

/* ---------------------------------------------------------------------------
 * Visibility gradients of the shadow term (section 3.1 "Shadow gradients";
 * the appendix "Visibility Gradients from Shadows"): the derivative of the
 * shadowed direct-illumination integral with respect to the vertex positions
 * of the occluding mesh, which mcdi_shade_bwd leaves out (detached
 * visibility).  Estimated by edge sampling: seen from the shadow-ray origin,
 * the directions a triangle blocks are bounded by the arcs of its edges, and
 * the derivative of the integral is an integral along the silhouette arcs of
 * the jump of the integrand times the arcs' normal velocity.
 *
 * mcdi_edges: the mesh's unique edges, built on the device.
 *   tris     device int32 [n_tris][3], the index buffer of mcdi_build_scene
 * Rows (a, b, c, d) int32, one per undirected edge, in order of first
 * appearance: triangle f's side k runs from corner k to corner k+1 (sides
 * in f-major, k-minor order); a-b is the edge as its first side has it, c
 * the opposite corner of that face, d the opposite corner of the second face
 * with the edge, or -1 (boundary edge; faces after the second are ignored).
 * A triangle with a corner outside [0, n_verts) adds no edge, nor does a side
 * whose corners coincide.  tris is read only by the build's stream work.
 * Limits: n_verts < 2^31, n_tris < 2^26.
 * ------------------------------------------------------------------------- */
typedef struct mcdi_edges_s* mcdi_edges;

mcdi_status mcdi_build_edges(const int32_t* tris, int64_t n_tris, int64_t n_verts, const mcdi_allocator* alloc,
                             void* stream, mcdi_edges* out);

/* Frees the handle's memory in stream order on the stream it was built on. */
void mcdi_destroy_edges(mcdi_edges edges);

/* Synchronises the handle's stream; *n_edges = number of rows E. */
mcdi_status mcdi_edges_count(mcdi_edges edges, int64_t* n_edges);

/* Synchronises the handle's stream, then copies the E x 4 rows into a caller
 * device int32 buffer in stream order on `stream`. */
mcdi_status mcdi_edges_copy(mcdi_edges edges, int32_t* rows, void* stream);

/* Edge-sampled visibility gradient of sum over pixels of g_cd . c_d +
 * g_cs . c_s with respect to the vertex positions.
 *   scene, edges  built from the same mesh; verts device float32
 *                 [n_verts][3] are its vertex positions (n_verts must equal
 *                 the count the edges were built with)
 *   params        seed, tau, ray_eps and MCDI_FLAG_BILINEAR as in the forward
 *                 pass (the other technique flags do not apply; spp is
 *                 validated but unused)
 *   edge_spp      edge samples per pixel, 1..1024
 *   sharp_gain    1..1024: sharp edges are this many times as likely per edge
 *                 as the others (1: a uniform choice over the edges).  The
 *                 expectation does not depend on it; the variance and the
 *                 number of traced rays do
 *   g_cd, g_cs    device [3][N] upstream gradients
 *   g_verts       device float32 [n_verts][3], ACCUMULATED (+=); the caller
 *                 zeroes it
 *   stats         valid_pixels, invalid_pixels, rays_traced (out-side rays)
 *                 and rays_hit are accumulated, or NULL
 * Edge classes: an edge is sharp when it has one face (d = -1) or when its
 * face normals (b-a)x(c-a) and (a-b)x(d-b) are more than 20 degrees apart
 * (dot < 0 or dot^2 < cos^2(20 deg) |n1|^2 |n2|^2, evaluated in FP32 in this
 * order without contraction); nS sharp edges, nR = E - nS others.
 * Per pixel and edge sample j: Philox4x32-10 with key = seed and counter =
 * (pixel in view, view_base + view, j, 2) gives x0..x3.  With K = sharp_gain,
 * the sample is in the sharp class when (x2 >> 8) (K nS + nR) < K nS 2^24
 * (probability P_S = ceil(2^24 K nS / (K nS + nR)) / 2^24), and its edge is the
 * ((x0 n_class) >> 32)-th of the class, in row order; the point on it is
 * x(t) = a + t (b - a) with t = the 24-bit uniform of x1.  From the
 * shadow-ray origin o = p + ray_eps n, with r = |x - o|, w = (x - o)/r and
 * m = (a - o) x (b - o): a sample counts when the edge is a silhouette (d =
 * -1, or c and d not strictly on opposite sides of the plane through o with
 * normal m), n.w > 0, and the out-side ray from o along w turned by 2^-13
 * radians away from the face misses the mesh.  It adds (n_class / P_class) s
 * tau g(w) |(b - a) x w| / (r^2 edge_spp) times (1 - t) m/|m| to vertex a and
 * t m/|m| to vertex b, where s = the sign of m . (c - o) and g is the
 * unshadowed integrand of c_d and c_s at w contracted with g_cd and g_cs.
 * G-buffer positions are held fixed (the receivers do not move).
 * Summation order of g_verts is not deterministic (float atomics). */
mcdi_status mcdi_shade_bwd_edges(mcdi_scene scene, mcdi_env env, mcdi_edges edges, const float* verts,
                                 int64_t n_verts, const mcdi_gbuffer* gbuf, const mcdi_params* params,
                                 int32_t edge_spp, uint32_t sharp_gain, const float* g_cd, const float* g_cs,
                                 float* g_verts, mcdi_stats* stats, void* stream);

/* ---------------------------------------------------------------------------
 * Image loss on the estimator's outputs (appendix A): composition
 * c = kd*c_d + c_s (section 4.2), L1 on tonemapped colours with
 * T(x) = sRGB(log(max(x,0) + 1)), and the light regulariser
 * |Y(T(c_d + c_s)) - V(T(ref))| with Y = (r+g+b)/3 and V = max(r,g,b).
 *   L_image = mean over valid pixels and channels, L_light = mean over valid
 *   pixels, L = L_image + w_light * L_light.
 *   kd, c_d, c_s, ref  device [3][N]; mask device [N]
 *   loss               device float [3]: L_image, L_light, L (overwritten)
 *   g_kd, g_cd, g_cs   device [3][N], dL/d*, overwritten (each may be NULL)
 * Deterministic (fixed-order FP64 reduction of per-workgroup partial sums).
 * ------------------------------------------------------------------------- */
mcdi_status mcdi_image_loss(const float* kd, const float* c_d, const float* c_s, const float* ref,
                            const uint8_t* mask, int64_t n, float w_light, float* loss, float* g_kd, float* g_cd,
                            float* g_cs, const mcdi_allocator* alloc, void* stream);

/* The same image loss without any allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid hipMalloc.  Arguments, outputs and
 * results are those of mcdi_image_loss (bit for bit: the same kernels).  The
 * per-block partial sums live in a static device array of 1 MiB per device
 * instead of allocated scratch, so n is limited to what it holds (about
 * 5.2e8 pixels); a larger n returns MCDI_E_UNSUPPORTED before anything is
 * enqueued.  Every call on one device shares that device's array: calls that
 * overlap in time on one device (different streams or threads) race and give
 * wrong results; calls ordered on one stream do not.  The first call on a
 * device looks up the array's address (no allocation). */
mcdi_status mcdi_image_loss_noalloc(const float* kd, const float* c_d, const float* c_s, const float* ref,
                                    const uint8_t* mask, int64_t n, float w_light, float* loss, float* g_kd,
                                    float* g_cd, float* g_cs, void* stream);

/* ---------------------------------------------------------------------------
 * Differentiable cross-bilateral denoiser (appendix B "Bilateral Denoiser"):
 * the spatial filter of SVGF evaluated densely, applied to the demodulated
 * diffuse and the specular lighting (section 4.2 "Denoising").
 *   out(p) = sum_q in(q) w(p,q) / W(p),  W(p) = sum_q w(p,q),
 *   w(p,q) = exp(-|p-q|^2 / (2 sigma^2))
 *          * exp(-|z(p) - z(q)| / (sigma_z |grad z(p) . (p-q)| + 1e-5))
 *          * max(0, n(p) . n(q))^sigma_n
 * over q in the (2R+1)^2 square around p inside the same view, with
 * R = mcdi_bilateral_radius(sigma) = clamp(ceil(3 sigma), 1, 8).  grad z is
 * the central difference of the depth guide over the valid 4-neighbours
 * (one-sided where one is missing, 0 where both are).  Pixels with mask 0
 * neither contribute nor receive (their outputs are 0).  The backward pass
 * propagates to the colours only: g_in(q) = sum_p g_out(p) w(p,q) / W(p).
 *   depth   device [N] depth guide (mcdi_view_depth gives |pos - eye|)
 *   nrm     device [3][N] normal guide, normalised by the filter
 *   in/out  device [n_chan][N], n_chan in {1, 3, 6} (6: c_d and c_s stacked,
 *           filtered with the same weights); out must not alias in
 *   wsum    device [N]: W(p), written by the forward (may be NULL there) and
 *           required by the backward
 * sigma > 0, sigma_z >= 0, sigma_n > 0, all finite.  Deterministic.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t n_views, height, width;
    const float* depth;
    const float* nrm;
    const uint8_t* mask;
    float sigma, sigma_z, sigma_n;
} mcdi_bilateral_guide;

int32_t mcdi_bilateral_radius(float sigma);
mcdi_status mcdi_bilateral_fwd(const mcdi_bilateral_guide* guide, int32_t n_chan, const float* in, float* out,
                               float* wsum, void* stream);
mcdi_status mcdi_bilateral_bwd(const mcdi_bilateral_guide* guide, int32_t n_chan, const float* g_out,
                               const float* wsum, float* g_in, void* stream);

/* Depth guide of a G-buffer: depth[p] = |pos(p) - eye(view of p)| for valid
 * pixels, 0 elsewhere.  depth device float32 [N]. */
mcdi_status mcdi_view_depth(const mcdi_gbuffer* gbuf, float* depth, void* stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of shading requests over resident scenes and
 * probe tables (the per-iteration shading of section 3 issued by many
 * independent callers).
 *
 * A request is one G-buffer (scene, probe tables, parameters) with its output
 * buffers; with g_cd non-NULL the adjoint runs too.  Requests are admitted in
 * submission order while the server's memory budget and slot count allow: an
 * admitted request holds device scratch of
 *     mcdi_server_request_bytes(N, spp) = align256(4 * ceil(2 spp / 32) * N)
 *                                       + align256(16 * N)
 * (its hit bits and ray origins) from the server's allocator until it
 * completes.  Their tiles (256 consecutive pixels) are packed, oldest admitted
 * request first, into persistent launches of at most launch_samples samples
 * (a forward+backward sample counts twice; a launch takes at least one tile
 * of each request it serves).  Launches run on two streams the server
 * creates (lanes), one launch in flight per lane, so that the tail of one
 * launch overlaps the next; requests submitted meanwhile join the next
 * launch.  A request completes when every launch holding its tiles has
 * finished.  `stream` (home) carries the server's allocations and frees
 * only; a lane waits for home before it first uses memory allocated there.
 * Every pixel is computed exactly as by mcdi_shade_fwd / mcdi_shade_bwd (the
 * random numbers depend on the pixel and view_base only), so a request's
 * per-pixel results do not depend on what it was served with (the probe
 * gradient up to FP32 summation order).
 *
 * Ownership: inputs and outputs are caller device buffers that must stay
 * valid, and unread and unwritten by the caller, until the request's ticket
 * is reported by mcdi_server_poll or mcdi_server_wait; the same holds for
 * its scene and probe handles (a scene destroyed earlier would only wait for
 * the last lane that read it).  The server owns its
 * ray queues (n_workgroups regions of 2 * spp_max * 256 rays of 16 bytes),
 * two item buffers and two pinned host staging areas of `slots` items each
 * (allocated at create), and the requests' scratch; destroy frees them.
 * Threads: calls on one server come from one thread.
 * ------------------------------------------------------------------------- */
typedef struct mcdi_server_s* mcdi_server;

typedef struct {
    int64_t budget_bytes;   /* device scratch the admitted requests may hold, >= 1 */
    int64_t launch_samples; /* work of one launch, in samples, >= 1 */
    int32_t slots;          /* most requests admitted at once, 1..65536 */
    int32_t spp_max;        /* largest spp of a request, 1..1024 */
    int32_t n_workgroups;   /* persistent grid size, 0..65536 (0: 4 per compute unit) */
    int32_t reserved;
} mcdi_server_config;

typedef struct {
    mcdi_scene scene;
    mcdi_env env;
    mcdi_gbuffer gbuf;
    mcdi_params params;     /* flags: the technique and lookup flags only (no DUMP, no TIME_*) */
    float* c_d;             /* device [3][N], written */
    float* c_s;             /* device [3][N], written */
    const float* g_cd;      /* device [3][N] upstream gradients, or NULL: forward only */
    const float* g_cs;
    float* g_kd;            /* device [3][N], written (with g_cd) */
    float* g_korm;
    float* g_nrm;
    float* g_env;           /* device [H][W][3], accumulated (with g_cd; may be NULL) */
} mcdi_request;

typedef struct {
    int64_t used_bytes;     /* scratch held by admitted requests */
    int64_t launches;       /* launches enqueued since create */
    int32_t queued;         /* submitted, not admitted */
    int32_t admitted;       /* admitted, not completed */
    int32_t in_flight;      /* launches not known to have finished */
    int32_t reserved;
} mcdi_server_info_t;

/* Errors: MCDI_E_INVALID for a bad config; MCDI_E_OOM if the ray queues or
 * item buffers cannot be allocated (*out untouched, nothing leaked). */
mcdi_status mcdi_server_create(const mcdi_server_config* config, const mcdi_allocator* alloc, void* stream,
                               mcdi_server* out);

/* Scratch bytes a request of n pixels at spp holds while admitted. */
int64_t mcdi_server_request_bytes(int64_t n_pixels, int32_t spp);

/* Queues a request and stores its ticket (> 0, increasing) in *ticket.  The
 * server's first read of the request's inputs waits for the work enqueued on
 * input_stream so far (an event; pass the server's own stream when no wait is
 * needed -- NULL is the null stream).  Then admits and launches what it can
 * without blocking.  Errors (nothing queued, *ticket untouched):
 * MCDI_E_INVALID for a bad request (as mcdi_shade_fwd, plus spp > spp_max,
 * DUMP/TIME flags, incomplete gradient buffers); MCDI_E_UNSUPPORTED if the
 * request's scratch alone exceeds budget_bytes.  A device error while
 * launching earlier requests is returned too (this request is queued). */
mcdi_status mcdi_server_submit(mcdi_server server, const mcdi_request* req, void* input_stream, int64_t* ticket);

/* Retires finished launches, admits and launches without blocking, and
 * copies at most cap tickets of completed requests (oldest first; each is
 * reported once) to done, their count to *n_done.  If the allocator returns
 * NULL at admission, the request stays queued and admission is retried at
 * the next call. */
mcdi_status mcdi_server_poll(mcdi_server server, int64_t* done, int32_t cap, int32_t* n_done);

/* As poll, but blocks on the oldest launch in flight until at least one
 * request has completed (returns at once with *n_done = 0 when nothing is
 * pending).  MCDI_E_OOM when queued requests cannot be admitted because the
 * allocator fails with nothing in flight. */
mcdi_status mcdi_server_wait(mcdi_server server, int64_t* done, int32_t cap, int32_t* n_done);

mcdi_status mcdi_server_info(mcdi_server server, mcdi_server_info_t* info);

/* Synchronises the server's stream, then frees its memory; requests not yet
 * completed are abandoned (their outputs undefined). */
void mcdi_server_destroy(mcdi_server server);

/* Durations (ms) of the traversal kernels of the calls made with
 * MCDI_FLAG_TIME_TRACE in this process (from any thread) since the previous
 * mcdi_trace_times call, oldest first (at most 1024 are kept).  Synchronises on their end
 * events, copies at most cap values to out, stores the count in *n and
 * forgets them. */
mcdi_status mcdi_trace_times(float* out, int32_t cap, int32_t* n);

/* The same for the kernels bracketed by MCDI_FLAG_TIME_ADJOINT: the adjoint
 * kernel of mcdi_shade_bwd (the evaluation kernel only, not the
 * probe-gradient scatter that follows it) and the edge-sample kernel of each
 * pass of mcdi_shade_bwd_edges, in call order. */
mcdi_status mcdi_adjoint_times(float* out, int32_t cap, int32_t* n);

/* Thread-local text of the last non-OK status ("" if none). */
const char* mcdi_last_error(void);

/* Library version string. */
const char* mcdi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MCDI_H */
