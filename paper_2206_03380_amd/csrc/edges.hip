// Unique edges of an indexed triangle mesh, for the edge-sampled visibility
// gradient of the shadow term.  Each triangle side (f, k) runs from corner k
// to corner k+1; its opposite corner is k+2.  The undirected edges go into an
// open-addressing hash table keyed by (min, max) vertex index, which keeps the
// first side (lowest side id 3f + k) and the second side of each edge.  An
// order-preserving compaction of the first sides then writes one row
// (a, b, c, d) per edge: a-b and c from the first side, d the opposite corner
// of the second side or -1.  Rows come out in order of first appearance, so
// the list is deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "edge_internal.h"
#include "mcdi_internal.h"

namespace mcdi {

namespace {

constexpr unsigned long long kEmpty = ~0ull;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kScanItems = 4;                     // sides per thread in the compaction
constexpr int kScanThreads = 256;
constexpr int kScanBlock = kScanItems * kScanThreads;

__device__ __forceinline__ uint32_t hash_slot(unsigned long long key, int bits) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - bits));
}

// side u = 3 f + k: corners a -> b and the opposite corner c; false when the
// triangle has a corner outside [0, nv) or the side's corners coincide
__device__ __forceinline__ bool side_of(const int32_t* __restrict__ tris, int64_t nv, uint32_t u, int32_t& a,
                                        int32_t& b, int32_t& c) {
    const uint32_t f = u / 3u, k = u - 3u * f;
    const int32_t t0 = tris[3 * (size_t)f], t1 = tris[3 * (size_t)f + 1], t2 = tris[3 * (size_t)f + 2];
    if (t0 < 0 || t1 < 0 || t2 < 0 || t0 >= nv || t1 >= nv || t2 >= nv) return false;
    a = k == 0 ? t0 : (k == 1 ? t1 : t2);
    b = k == 0 ? t1 : (k == 1 ? t2 : t0);
    c = k == 0 ? t2 : (k == 1 ? t0 : t1);
    return a != b;
}

__global__ void edge_table_init(unsigned long long* keys, uint32_t* first, uint32_t* second, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        keys[i] = kEmpty;
        first[i] = kNone;
        second[i] = kNone;
    }
}

// insert every side's edge; the lowest side id of an edge becomes its first
__global__ void edge_insert(const int32_t* __restrict__ tris, int64_t nv, uint32_t n_sides,
                            unsigned long long* keys, uint32_t* first, uint32_t* slot_of, int bits) {
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_sides) return;
    int32_t a, b, c;
    uint32_t slot = kNone;
    if (side_of(tris, nv, u, a, b, c)) {
        const unsigned long long key =
            ((unsigned long long)(uint32_t)min(a, b) << 32) | (unsigned long long)(uint32_t)max(a, b);
        const uint32_t mask = (bits >= 32) ? kNone : ((1u << bits) - 1u);
        uint32_t h = hash_slot(key, bits);
        // the table holds at least twice as many slots as sides: a free slot
        // is always found; the bound only keeps the loop finite
        for (uint32_t probe = 0; probe <= mask; ++probe) {
            const unsigned long long prev = atomicCAS(keys + h, kEmpty, key);
            if (prev == kEmpty || prev == key) {
                slot = h;
                break;
            }
            h = (h + 1u) & mask;
        }
        if (slot != kNone) atomicMin(first + slot, u);
    }
    slot_of[u] = slot;
}

// the lowest side id after the first is the edge's second side
__global__ void edge_second(uint32_t n_sides, const uint32_t* __restrict__ slot_of, const uint32_t* first,
                            uint32_t* second) {
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_sides) return;
    const uint32_t s = slot_of[u];
    if (s != kNone && first[s] != u) atomicMin(second + s, u);
}

__device__ __forceinline__ bool is_first(uint32_t u, uint32_t n_sides, const uint32_t* __restrict__ slot_of,
                                         const uint32_t* __restrict__ first) {
    if (u >= n_sides) return false;
    const uint32_t s = slot_of[u];
    return s != kNone && first[s] == u;
}

// exclusive scan of v over the workgroup (kScanThreads lanes); returns the
// prefix, *total the sum
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* s_buf, uint32_t* total) {
    const int t = threadIdx.x;
    s_buf[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const uint32_t add = t >= off ? s_buf[t - off] : 0u;
        __syncthreads();
        s_buf[t] += add;
        __syncthreads();
    }
    const uint32_t incl = s_buf[t];
    *total = s_buf[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

// first sides per block of kScanBlock sides
__global__ __launch_bounds__(kScanThreads) void edge_count(uint32_t n_sides, const uint32_t* __restrict__ slot_of,
                                                           const uint32_t* __restrict__ first, uint32_t* bsum) {
    __shared__ uint32_t s_buf[kScanThreads];
    const uint32_t u0 = blockIdx.x * (uint32_t)kScanBlock + threadIdx.x * (uint32_t)kScanItems;
    uint32_t v = 0;
    for (int i = 0; i < kScanItems; ++i) v += is_first(u0 + i, n_sides, slot_of, first) ? 1u : 0u;
    uint32_t total;
    block_scan(v, s_buf, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// exclusive scan of the block counts in place (one workgroup); the edge count
__global__ __launch_bounds__(kScanThreads) void edge_scan(uint32_t nb, uint32_t* bsum, uint32_t* n_edges) {
    __shared__ uint32_t s_buf[kScanThreads];
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const uint32_t i = b0 + threadIdx.x;
        const uint32_t v = i < nb ? bsum[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_scan(v, s_buf, &total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *n_edges = carry;
}

__global__ __launch_bounds__(kScanThreads) void edge_write(const int32_t* __restrict__ tris, int64_t nv,
                                                           uint32_t n_sides, const uint32_t* __restrict__ slot_of,
                                                           const uint32_t* __restrict__ first,
                                                           const uint32_t* __restrict__ second,
                                                           const uint32_t* __restrict__ bsum, int4* rows) {
    __shared__ uint32_t s_buf[kScanThreads];
    const uint32_t u0 = blockIdx.x * (uint32_t)kScanBlock + threadIdx.x * (uint32_t)kScanItems;
    bool own[kScanItems];
    uint32_t v = 0;
    for (int i = 0; i < kScanItems; ++i) {
        own[i] = is_first(u0 + i, n_sides, slot_of, first);
        v += own[i] ? 1u : 0u;
    }
    uint32_t total;
    uint32_t at = bsum[blockIdx.x] + block_scan(v, s_buf, &total);
    for (int i = 0; i < kScanItems; ++i) {
        if (!own[i]) continue;
        const uint32_t u = u0 + i;
        int32_t a = 0, b = 0, c = 0, d = -1;
        side_of(tris, nv, u, a, b, c);
        const uint32_t sec = second[slot_of[u]];
        if (sec != kNone) {
            int32_t a2, b2, c2;
            if (side_of(tris, nv, sec, a2, b2, c2)) d = c2;
        }
        rows[at++] = make_int4(a, b, c, d);
    }
}

}  // namespace

int edge_table_bits(int64_t n_sides) {
    int bits = 8;
    while (((int64_t)1 << bits) < 2 * n_sides) ++bits;
    return bits;
}

uint32_t edge_scan_blocks(int64_t n_sides) { return (uint32_t)((n_sides + kScanBlock - 1) / kScanBlock); }

hipError_t launch_edges_build(const int32_t* tris, int64_t n_tris, int64_t n_verts, int bits,
                              unsigned long long* keys, uint32_t* first, uint32_t* second, uint32_t* slot_of,
                              uint32_t* bsum, int4* rows, uint32_t* n_edges, hipStream_t s) {
    const uint32_t n_sides = (uint32_t)(3 * n_tris);
    const uint32_t slots = 1u << bits;
    hipLaunchKernelGGL(edge_table_init, dim3((slots + 255) / 256 < 8192u ? (slots + 255) / 256 : 8192u), dim3(256), 0, s, keys,
                       first, second, slots);
    if (n_sides == 0) {
        hipLaunchKernelGGL(edge_scan, dim3(1), dim3(kScanThreads), 0, s, 0u, bsum, n_edges);
        return hipGetLastError();
    }
    const dim3 g((n_sides + 255) / 256), b(256);
    hipLaunchKernelGGL(edge_insert, g, b, 0, s, tris, n_verts, n_sides, keys, first, slot_of, bits);
    hipLaunchKernelGGL(edge_second, g, b, 0, s, n_sides, slot_of, first, second);
    const uint32_t nb = edge_scan_blocks(n_sides);
    hipLaunchKernelGGL(edge_count, dim3(nb), dim3(kScanThreads), 0, s, n_sides, slot_of, first, bsum);
    hipLaunchKernelGGL(edge_scan, dim3(1), dim3(kScanThreads), 0, s, nb, bsum, n_edges);
    hipLaunchKernelGGL(edge_write, dim3(nb), dim3(kScanThreads), 0, s, tris, n_verts, n_sides, slot_of, first,
                       second, bsum, rows);
    return hipGetLastError();
}

}  // namespace mcdi
