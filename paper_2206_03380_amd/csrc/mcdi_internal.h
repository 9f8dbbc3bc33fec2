// Internal declarations shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcdi.h"

namespace mcdi {

// BVH node, 32 bytes: box, skip link and payload.  Nodes are stored in
// depth-first pre-order, so the first child of an internal node is the next
// node and `escape` is the index just past the node's subtree.  payload = 0
// for an internal node; (first_triangle << 3) | count for a leaf (1..7).
struct alignas(16) Node {
    float lo[3];
    int32_t escape;
    float hi[3];
    int32_t payload;
};

constexpr int kLeafMax = 4;
// Big triangles: a triangle whose box's longest side is at least 1/kBigTriDiv
// of the longest side of the triangle centroids' bounds.  When a mesh has both
// big and small ones, the big ones form the root's first subtree, in leaves of
// at most kBigLeafMax.
constexpr float kBigTriDiv = 8.0f;
constexpr int kBigLeafMax = 1;
constexpr int kHotMax = 1024;   // probe texels privatised in LDS by the adjoint
constexpr int kBlock = 256;     // pixels per workgroup in the shading kernels

struct DeviceSceneInfo {
    int32_t n_nodes;
    int32_t max_depth;
    int32_t bad_tris;
    int32_t n_groups;          // wide nodes
    int32_t wide;              // 1: shadow rays walk the wide hierarchy
    float depth_complexity;    // sum of leaf box areas / root box area
    int32_t wide_bad;          // a wide reference failed the builder's check
    int32_t n_big;             // big triangles (the root's first subtree when 0 < n_big < n_tris)
    double leaf_area;          // the sum (accumulated by the builder)
};

// The scene's quantisation frame: node box coordinates as 16-bit integers q,
// the plane q standing for base + q * step (per axis).
struct QFrame {
    float base[3];
    float step[3];
};

// Compact node of the shadow-ray traversal (16 bytes, one load): the box of
// the Node with the same index quantised against the frame outward (lo
// rounded down, hi rounded up: it contains the exact box) and one link word.
//   x = qlo.x | qlo.y << 16, y = qlo.z | qhi.x << 16, z = qhi.y | qhi.z << 16
//   w = leaf: 0x80000000 | payload (first_triangle << 3 | count), its
//       escape being the next index; internal: the escape index
struct QNode {
    uint32_t x, y, z, w;
};
constexpr uint32_t kQLeaf = 0x80000000u;
// Set in every child reference of a wide node (references stay below 2^29):
// a walk replaces the reference of a child whose box it missed by 0 and
// pushes the rest, advancing its stack past each reference that has the bit.
constexpr uint32_t kRefLive = 1u << 30;

// Wide node of the shadow-ray traversal: four child records in QNode form
// (64 bytes, one aligned segment), w = the child's wide-node index (internal)
// or kQLeaf | payload (leaf); unused slots have an empty box.  Node 0 is the
// root.
constexpr uint32_t kWideNone = 0xFFFFFFFFu;   // no node (a traversal state)

struct Scene {
    const Node* nodes;    // [>= 1]
    const float4* tris;   // [3 * n_tris] vertex positions, w unused
    int64_t n_tris;
    const QNode* qnodes;  // [>= 1] the same nodes, quantised
    const QFrame* frame;
    const QNode* groups;  // [4 * capacity] wide nodes
    uint32_t group_bytes; // 64 * capacity (the bound of a buffer resource)
    const uint32_t* gorder;   // [capacity] each wide node's visit orders (per ray octant)
    const DeviceSceneInfo* info;   // info->wide selects the traversal (read by the kernels)
};

// Traversal choice, made by the builder on the device.  The depth
// complexity -- the surface areas of the leaf boxes summed, over the root
// box's -- estimates how many leaves a ray through the scene crosses.  Surface
// scenes (about 1.5 for the displaced spheres) are walked on the binary
// hierarchy, whose cache-resident walk is bound by instruction issue;
// volume-filling ones (16 for the beam lattice in its room, 95 for the beams
// alone), whose rays cross many boxes and whose walk is bound by memory round
// trips, on the 4-wide hierarchy (about a quarter of the round trips).
constexpr float kWideDepthComplexity = 4.0f;

struct EnvView {
    int32_t H, W;
    const float* cond;    // [H][W+1]
    const float* marg;    // [H+1]
    const int32_t* light_enabled;  // device flag: total weight > 0
    const int32_t* hot_slot;       // [H*W] LDS slot of a hot texel or -1
    const int32_t* hot_texel;      // [kHotMax] texel of each slot
    const int32_t* n_hot;          // number of hot texels (<= kHotMax)
    const int32_t* guide;          // [H][G+1] search guide of the conditional rows
    int32_t G;                     // guide cells per row (power of two)
    const float4* tex;             // [H*W] (r, g, b, pdf): radiance and density in one line
    const float* pdf;              // [H*W] the density alone (tex.w), a quarter of tex's lines
    int32_t win;                   // 1: row searches read the cell's candidates in one go
    const uint8_t* dclass;         // [(H*W + 3) / 4] density classes, 2 bits per texel
};

struct GBufView {
    int32_t n_views, height, width, view_base;
    const float *pos, *nrm, *kd, *korm;
    const uint8_t* mask;
    const float* eye;
    int64_t n;  // pixels
};

struct ShadeArgs {
    Scene scene;
    EnvView env;
    GBufView g;
    int32_t spp;
    uint32_t flags;
    uint64_t seed;
    float tau;
    float ray_eps;
    uint32_t* decisions;
    // forward
    float* c_d;
    float* c_s;
    uint32_t* hitbits_out;
    // backward
    const float* g_cd;
    const float* g_cs;
    const uint32_t* hitbits_in;
    // live samples, [words][N] in the hit bits' layout: bit 2s + t set where
    // technique t's sample s was drawn with a density and above the horizon
    // (the samples the estimator evaluates).  Ray generation writes it when
    // tracing; the shading passes, given it, walk only those samples.  NULL:
    // not kept.
    uint32_t* live;
    float* g_kd;
    float* g_korm;
    float* g_nrm;
    float* g_env;
    mcdi_stats* stats;
    // forward ray queue (one region of 2*spp*kBlock rays per workgroup)
    float4* rays;          // (direction, local pixel | slot << 8)
    int32_t* ray_count;    // [blocks]
    int32_t* tile_order;   // [blocks] traversal order of the tiles (most rays first), or NULL
    float4* origins;       // [N]
    // adjoint: probe-gradient records of non-hot texels, one region of
    // rec_region records per tile and a record count per tile, binned and
    // summed by the env-scatter pass; NULL: direct atomics.  Nearest lookup:
    // one float4 (texel bits, 3 values).  Bilinear lookup: two float4s
    // (base bits, fx, fy, 0) (3 values, 0), the base being the sample's
    // upper-left tap in the extended grid of H + 1 rows (row i0 + 1, i0 in
    // [-1, H-1]) by W columns.
    float4* rec;
    uint32_t* rec_count;
    uint32_t rec_region;
    // frozen sampling (forward only): the planes that evaluate the samples
    // drawn from g (normal, albedo, occlusion/roughness/metallic); NULL
    // otherwise
    const float* e_nrm;
    const float* e_kd;
    const float* e_korm;
};

// one serving work item: a contiguous range of tiles of one request
struct ServeItem {
    ShadeArgs args;        // outputs, upstream gradients (g_cd != null: adjoint too)
    uint32_t* hitbits;     // [words][N] of the request
    int64_t first_tile;    // first tile of the range within the request
    int64_t first_global;  // index of that tile in the launch's tile queue
};

// kernel launchers (return hipError_t of the launch)
hipError_t launch_serve(const ServeItem* items_dev, int n_items, int64_t total_tiles, int* tile_counter,
                        float4* scratch, int spp_max, int n_workgroups, int max_H, hipStream_t s);
hipError_t launch_env_cdf(const float* env, int H, int W, float* cond, float* marg, float* pdf,
                          double* rowsum, int32_t* light_enabled, hipStream_t s);
// Search guide of the conditional CDF rows: guide[i][g] = the largest column
// k <= W-1 with cond[i][k] <= g / G, for g = 0..G.
int env_row_window(int H, int W);
int env_guide_cells(int W, int win);
// (r, g, b, pdf) per texel, after the tables
hipError_t launch_env_pack(const float* env, const float* pdf, int64_t n, float4* tex, hipStream_t s);
// out[k] = (rgb[k].xyz, dens[k].w)
hipError_t launch_env_mix(const float4* rgb, const float4* dens, int64_t n, float4* out, hipStream_t s);
hipError_t launch_env_guide(const float* cond, int H, int W, int G, int32_t* guide, hipStream_t s);
// density classes of the texels, 2 bits each, 4 to a byte (dclass_kernel)
hipError_t launch_env_dclass(const float* pdf, int64_t n, uint8_t* dclass, hipStream_t s);
hipError_t launch_env_hot(const float* pdf, int H, int W, int32_t* hot_slot, int32_t* hot_texel, int32_t* n_hot,
                          hipStream_t s);
// forward = gen_rays -> trace_rays -> shade; hit bits are produced by the
// first two and read by the third
hipError_t launch_gen_rays(const ShadeArgs& a, uint32_t* hitbits, hipStream_t s);
hipError_t launch_order_tiles(const int32_t* ray_count, int64_t n_tiles, int32_t* order, hipStream_t s);
hipError_t launch_trace_rays(const ShadeArgs& a, uint32_t* hitbits, hipStream_t s);
hipError_t launch_shade_fwd(const ShadeArgs& a, hipStream_t s);
hipError_t launch_shade_bwd(const ShadeArgs& a, hipStream_t s);
// forward with frozen sampling: samples, densities, lobe choice and
// visibility from a.g, the material and the probe radiance evaluated from
// a.e_* and a.env.tex (whose w, the density, is the sampling probe's)
hipError_t launch_shade_fwd_frozen(const ShadeArgs& a, hipStream_t s);
hipError_t launch_trace(const Scene& sc, const float* o, const float* d, int64_t n, uint8_t* hit,
                        int brute, hipStream_t s);

// Probe-gradient scatter of the adjoint over the records the adjoint kernel
// leaves in per-tile regions: bucket histogram, counting-sort scatter by
// bucket, and per-bucket LDS accumulation flushed into g_env.
struct EnvScatter {
    int32_t bil;          // records of the bilinear lookup (two float4s, keyed by base)
    int32_t H, W;         // probe size
    float* acc4;          // bilinear: [4][(H+1) W][3] per-tap sums at each base, gathered into g_env
    float4* rec;          // [n_tiles][region] records as appended
    uint32_t* tile_count; // [n_tiles] records in each region
    uint32_t region;
    int64_t n_tiles;
    float4* sorted;       // [cap] records ordered by bucket
    uint32_t* cursor;     // [K] bucket sizes, then fill cursors
    uint32_t* start;      // [K + 1] bucket starts
    uint32_t* bmax;       // [K] bits of the largest |value| in each bucket
    uint32_t* wg_hist;    // [n_wg][K] records per bucket of each histogram workgroup
    uint32_t cap;         // n_tiles * region
    int32_t K, shift;     // K buckets of 2^shift texels
    int32_t n_texels;
    int32_t n_wg;         // workgroups of the histogram and scatter steps
    float* g_env;
};
// bil: records of the bilinear lookup; false when the extended grid is too
// large for the bucket size the accumulation needs (use direct atomics)
bool env_scatter_plan(int H, int W, int64_t n_tiles, uint32_t region, bool bil, EnvScatter& p);
size_t env_scatter_bytes(const EnvScatter& p);     // after env_scatter_plan
void env_scatter_carve(void* base, EnvScatter& p); // lay the buffers out in base
hipError_t launch_env_scatter_init(const EnvScatter& p, hipStream_t s);
hipError_t launch_env_scatter(const EnvScatter& p, hipStream_t s);

size_t image_loss_scratch_bytes(int64_t n);
// Static scratch of the allocation-free image loss: 1 MiB per device, enough
// for image_loss_scratch_bytes(n) up to n of about 5.2e8 pixels.
constexpr size_t kLossStaticScratch = (size_t)1 << 20;
constexpr int kLossStaticDevices = 64;
// Device address of the current device's static scratch (looked up once per
// device, kept for the process).
hipError_t image_loss_static_scratch(void** out);
hipError_t launch_image_loss(const float* kd, const float* cd, const float* cs, const float* ref,
                             const uint8_t* mask, int64_t n, float w_light, float* loss, float* g_kd, float* g_cd,
                             float* g_cs, void* scratch, hipStream_t s);

// Cross-bilateral filter over V views of H x W pixels (N = V*H*W).
constexpr int kBilatMaxR = 8;
struct BilatArgs {
    int32_t V, H, W;
    int64_t n;
    const float* depth;    // [N]
    const float* nrm;      // [3][N]
    const uint8_t* mask;   // [N]
    float sigma, sigma_z, sigma_n;
    int32_t R;             // footprint radius
    int32_t tiles_x, tiles_y;
};
int bilateral_radius(float sigma);
void bilateral_tiles(BilatArgs& a);
hipError_t launch_bilateral_fwd(const BilatArgs& a, int nc, const float* in, float* out, float* wsum,
                                hipStream_t s);
hipError_t launch_bilateral_bwd(const BilatArgs& a, int nc, const float* g_out, const float* wsum, float* g_in,
                                hipStream_t s);
hipError_t launch_view_depth(const GBufView& g, float* depth, hipStream_t s);

struct TempAlloc {
    void* (*alloc)(void* ctx, size_t bytes, hipStream_t s);
    void (*free)(void* ctx, void* p, hipStream_t s);
    void* ctx;
};
// groups_out: capacity for max(1, n_tris) wide nodes (>= internal nodes + 1),
// followed by as many 32-bit visit orders
hipError_t build_bvh(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                     Node* nodes_out, float4* tris_out, QNode* qnodes_out, QFrame* frame_out, QNode* groups_out,
                     DeviceSceneInfo* info, const TempAlloc& ta, hipStream_t s, int* oom);

}  // namespace mcdi
