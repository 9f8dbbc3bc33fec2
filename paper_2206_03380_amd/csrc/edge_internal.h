// Internal declarations of the edge-sampled visibility gradient: the mesh
// edge list and the sample / trace passes.
#pragma once

#include "mcdi_internal.h"

namespace mcdi {

// edge-sampled visibility gradient of the shadow term: one kernel over a
// range of pixels queues the edge samples that are silhouettes above the
// horizon, a second recomputes them, traces their out-side rays and scatters
// the terms of the rays that miss into g_verts
constexpr float kEdgeDelta = 1.0f / 8192.0f;   // angle of the out-side ray off the edge (radians)
constexpr uint32_t kEdgeQueueMax = 1u << 25;   // queue records per pass (4 bytes each)
constexpr int64_t kEdgePassMax = 1 << 22;      // pixels per pass (22 bits of the record)
// from this many queued rays on, one lane traces each ray instead of one wavefront
constexpr uint32_t kEdgeLaneMode = 1u << 16;
// edge classes of the sampling distribution: sharp edges have one face, or
// face normals more than 20 degrees apart; the call's gain weights them
constexpr float kSharpCos2 = 0.883022221559489f;   // cos^2(20 degrees)
constexpr uint32_t kSharpGainMax = 1024;
struct EdgeArgs {
    ShadeArgs a;             // scene, env, G-buffer, seed, tau, ray_eps, flags, g_cd, g_cs, stats
    const int4* edges;       // [E] (a, b, c, d) rows
    const uint32_t* n_edges; // E (device)
    const float* verts;      // [Nv][3]
    const float4* egeo;      // [E][4] corners (a, edge id), b, c, (d, 1 when present); sharp edges first
    const uint32_t* n_sharp; // edges of the sharp class (device)
    float* g_verts;          // [Nv][3], accumulated
    int32_t n_es;            // edge samples per pixel
    uint32_t gain;           // per-edge weight of the sharp class (1: uniform over edges)
    int64_t pix0, npix;      // pixel range of this pass
    uint32_t* queue;         // [q_cap]: pixel in pass << 10 | edge sample
    uint32_t* q_count;
    uint32_t q_cap;
};

// one pass of the edge-sampled visibility gradient over [pix0, pix0 + npix)
// gen_begin / gen_end (or null): events recorded right before and after the
// edge-sample kernel
hipError_t launch_edge_grad(const EdgeArgs& e, hipStream_t s, hipEvent_t gen_begin = nullptr,
                            hipEvent_t gen_end = nullptr);
// classifies the edges and packs their corners into e.egeo, sharp edges
// first (cap >= E); bsum: [edge_pack_blocks(cap)] block sums
uint32_t edge_pack_blocks(uint32_t cap);
hipError_t launch_edge_pack(const EdgeArgs& e, uint32_t cap, uint32_t* bsum, uint32_t* n_sharp, hipStream_t s);

// unique mesh edges: hash table of 2^bits slots (keys, first and second
// side), side -> slot map [3 n_tris], block sums [edge_scan_blocks]
int edge_table_bits(int64_t n_sides);
uint32_t edge_scan_blocks(int64_t n_sides);
hipError_t launch_edges_build(const int32_t* tris, int64_t n_tris, int64_t n_verts, int bits,
                              unsigned long long* keys, uint32_t* first, uint32_t* second, uint32_t* slot_of,
                              uint32_t* bsum, int4* rows, uint32_t* n_edges, hipStream_t s);

}  // namespace mcdi
