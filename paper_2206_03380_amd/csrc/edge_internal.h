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
struct EdgeArgs {
    ShadeArgs a;             // scene, env, G-buffer, seed, tau, ray_eps, flags, g_cd, g_cs, stats
    const int4* edges;       // [E] (a, b, c, d) rows
    const uint32_t* n_edges; // E (device)
    const float* verts;      // [Nv][3]
    const float4* egeo;      // [E][4] corners a, b, c, d of each edge (d.w = 1 when present)
    float* g_verts;          // [Nv][3], accumulated
    int32_t n_es;            // edge samples per pixel
    int64_t pix0, npix;      // pixel range of this pass
    uint32_t* queue;         // [q_cap]: pixel in pass << 10 | edge sample
    uint32_t* q_count;
    uint32_t q_cap;
};

// one pass of the edge-sampled visibility gradient over [pix0, pix0 + npix)
hipError_t launch_edge_grad(const EdgeArgs& e, hipStream_t s);
// packs the corners of the first min(E, cap) edges into e.egeo
hipError_t launch_edge_pack(const EdgeArgs& e, uint32_t cap, hipStream_t s);

// unique mesh edges: hash table of 2^bits slots (keys, first and second
// side), side -> slot map [3 n_tris], block sums [edge_scan_blocks]
int edge_table_bits(int64_t n_sides);
uint32_t edge_scan_blocks(int64_t n_sides);
hipError_t launch_edges_build(const int32_t* tris, int64_t n_tris, int64_t n_verts, int bits,
                              unsigned long long* keys, uint32_t* first, uint32_t* second, uint32_t* slot_of,
                              uint32_t* bsum, int4* rows, uint32_t* n_edges, hipStream_t s);

}  // namespace mcdi
