// Device BVH construction for the shadow-ray mesh (rebuilt whenever the mesh
// changes: the paper re-extracts its mesh every optimisation iteration).
//
// Linear BVH: 63-bit Morton codes of triangle centroids, a radix sort, the
// binary radix tree of the sorted codes built in parallel (one lane per
// internal node, Karras 2012), a bottom-up pass that fits boxes and counts
// the nodes that survive collapsing subtrees of <= 4 triangles into leaves,
// and a final pass that writes every surviving node at its depth-first
// pre-order index with a skip link, so traversal needs no stack.
#include <hip/hip_runtime.h>
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>

#include "mcdi_internal.h"

namespace mcdi {
namespace {

__device__ __forceinline__ int ord_key(float f) {
    const int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float ord_val(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7FFFFFFF); }

__global__ void init_bounds(int* b) {
    if (threadIdx.x < 3) b[threadIdx.x] = 0x7FFFFFFF;        // min keys
    else if (threadIdx.x < 6) b[threadIdx.x] = (int)0x80000000;  // max keys
}

__device__ __forceinline__ float wave_min(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// fetch vertices, replace bad triangles by a degenerate one, centroid bounds
__global__ __launch_bounds__(256) void tri_prep(const float* verts, int64_t nv, const int32_t* tris, int64_t nt,
                                                float4* tmp, int* cb, DeviceSceneInfo* info) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float cx = INFINITY, cy = INFINITY, cz = INFINITY, Cx = -INFINITY, Cy = -INFINITY, Cz = -INFINITY;
    if (f < nt) {
        float4 v[3];
        bool ok = true;
        for (int c = 0; c < 3; ++c) {
            const int32_t id = tris[3 * f + c];
            if (id < 0 || id >= nv) { ok = false; v[c] = make_float4(0, 0, 0, 0); continue; }
            v[c] = make_float4(verts[3 * (size_t)id], verts[3 * (size_t)id + 1], verts[3 * (size_t)id + 2], 0.0f);
            ok = ok && isfinite(v[c].x) && isfinite(v[c].y) && isfinite(v[c].z);
        }
        if (!ok) {
            atomicAdd(&info->bad_tris, 1);
            v[0] = v[1] = v[2] = make_float4(0, 0, 0, 0);
        }
        tmp[3 * f] = v[0];
        tmp[3 * f + 1] = v[1];
        tmp[3 * f + 2] = v[2];
        const float x = (v[0].x + v[1].x + v[2].x) * (1.0f / 3.0f);
        const float y = (v[0].y + v[1].y + v[2].y) * (1.0f / 3.0f);
        const float z = (v[0].z + v[1].z + v[2].z) * (1.0f / 3.0f);
        cx = Cx = x; cy = Cy = y; cz = Cz = z;
    }
    cx = wave_min(cx); cy = wave_min(cy); cz = wave_min(cz);
    Cx = wave_max(Cx); Cy = wave_max(Cy); Cz = wave_max(Cz);
    if ((threadIdx.x & 63) == 0 && cx <= Cx) {
        atomicMin(cb + 0, ord_key(cx)); atomicMin(cb + 1, ord_key(cy)); atomicMin(cb + 2, ord_key(cz));
        atomicMax(cb + 3, ord_key(Cx)); atomicMax(cb + 4, ord_key(Cy)); atomicMax(cb + 5, ord_key(Cz));
    }
}

__device__ __forceinline__ uint64_t spread3(uint64_t x) {
    x &= 0x1FFFFFull;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ __launch_bounds__(256) void morton(const float4* tmp, int64_t nt, const int* cb, uint64_t* keys,
                                              uint32_t* vals) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nt) return;
    const float4 a = tmp[3 * f], b = tmp[3 * f + 1], c = tmp[3 * f + 2];
    const float p[3] = {(a.x + b.x + c.x) * (1.0f / 3.0f), (a.y + b.y + c.y) * (1.0f / 3.0f),
                        (a.z + b.z + c.z) * (1.0f / 3.0f)};
    uint64_t code = 0;
    for (int k = 0; k < 3; ++k) {
        const float lo = ord_val(cb[k]), hi = ord_val(cb[3 + k]);
        const float ext = hi - lo;
        float u = ext > 0.0f ? (p[k] - lo) / ext : 0.5f;
        u = fminf(fmaxf(u, 0.0f), 1.0f);
        const uint64_t q = (uint64_t)fminf(u * 2097152.0f, 2097151.0f);
        code |= spread3(q) << (2 - k);
    }
    keys[f] = code;
    vals[f] = (uint32_t)f;
}

struct Tree {
    int32_t* parent;   // [2nt-1]
    int32_t* left;     // [nt-1] node ids (leaf k = nt-1+k)
    int32_t* right;
    int32_t* first;    // [nt-1] sorted-primitive range
    int32_t* last;
    int32_t* flag;     // [nt-1]
    int32_t* cnt;      // [2nt-1] surviving nodes in the subtree
    float4* box;       // [2*(2nt-1)]
};

__device__ __forceinline__ int prefix_len(const uint64_t* keys, int nt, int a, int b) {
    if (b < 0 || b >= nt) return -1;
    const uint64_t ka = keys[a], kb = keys[b];
    if (ka == kb) return 64 + __clz((uint32_t)(a ^ b));
    return __clzll((long long)(ka ^ kb));
}

__global__ void fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

__global__ __launch_bounds__(256) void radix_tree(const uint64_t* keys, int nt, Tree T) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt - 1) return;
    const int d = prefix_len(keys, nt, i, i + 1) > prefix_len(keys, nt, i, i - 1) ? 1 : -1;
    const int dmin = prefix_len(keys, nt, i, i - d);
    int lmax = 2;
    while (prefix_len(keys, nt, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(keys, nt, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = prefix_len(keys, nt, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(keys, nt, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int g = i + s * d + (d < 0 ? -1 : 0);
    const int lo = min(i, j), hi = max(i, j);
    const int L = (lo == g) ? (nt - 1 + g) : g;
    const int R = (hi == g + 1) ? (nt - 1 + g + 1) : g + 1;
    T.left[i] = L;
    T.right[i] = R;
    T.first[i] = lo;
    T.last[i] = hi;
    T.parent[L] = i;
    T.parent[R] = i;
    T.flag[i] = 0;
    if (i == 0) T.parent[0] = -1;
}

__device__ __forceinline__ void tri_box(const float4* t, float4& lo, float4& hi) {
    lo = make_float4(fminf(t[0].x, fminf(t[1].x, t[2].x)), fminf(t[0].y, fminf(t[1].y, t[2].y)),
                     fminf(t[0].z, fminf(t[1].z, t[2].z)), 0.0f);
    hi = make_float4(fmaxf(t[0].x, fmaxf(t[1].x, t[2].x)), fmaxf(t[0].y, fmaxf(t[1].y, t[2].y)),
                     fmaxf(t[0].z, fmaxf(t[1].z, t[2].z)), 0.0f);
}

// fit node p from its two finished children
__device__ __forceinline__ void fit_node(int p, int nt, const Tree& T) {
    const int l = T.left[p], r = T.right[p];
    const float4 al = T.box[2 * l], ah = T.box[2 * l + 1], bl = T.box[2 * r], bh = T.box[2 * r + 1];
    T.box[2 * p] = make_float4(fminf(al.x, bl.x), fminf(al.y, bl.y), fminf(al.z, bl.z), 0.0f);
    T.box[2 * p + 1] = make_float4(fmaxf(ah.x, bh.x), fmaxf(ah.y, bh.y), fmaxf(ah.z, bh.z), 0.0f);
    const int size = T.last[p] - T.first[p] + 1;
    T.cnt[p] = size <= kLeafMax ? 1 : 1 + T.cnt[l] + T.cnt[r];
}

// Bottom-up refit, first phase: workgroup b fits the leaves of sorted
// positions [256 b, 256 b + 256) and every internal node whose range lies
// inside them, the second of the two children to arrive fitting the parent.
// All of that happens inside one workgroup, so workgroup-scope atomics order
// it (an agent-scope release would write the L2 back on every step).  A climb
// that reaches a node spanning workgroups stops there and records the child
// it finished.
__global__ __launch_bounds__(256) void refit_local(const float4* tmp, const uint32_t* vals, int nt, Tree T,
                                                   int* top_list, int* top_count) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    const int lo = blockIdx.x * blockDim.x, hi = min(nt, lo + (int)blockDim.x) - 1;
    const int leaf = nt - 1 + k;
    float4 blo, bhi;
    tri_box(tmp + 3 * (size_t)vals[k], blo, bhi);
    T.box[2 * leaf] = blo;
    T.box[2 * leaf + 1] = bhi;
    T.cnt[leaf] = 1;
    int c = leaf;
    int p = T.parent[leaf];
    for (int guard = 0; p >= 0 && p < nt - 1 && guard < 4096; ++guard) {
        if (T.first[p] < lo || T.last[p] > hi) {
            top_list[atomicAdd(top_count, 1)] = c;
            return;
        }
        const int old = __hip_atomic_fetch_add(&T.flag[p], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == 0) return;
        fit_node(p, nt, T);
        c = p;
        p = T.parent[p];
    }
}

// Second phase, one workgroup: the nodes spanning workgroups (ancestors of
// the recorded children), with the first phase's results visible across the
// launch boundary.
__global__ __launch_bounds__(1024) void refit_top(const int* top_list, const int* top_count, int nt, Tree T) {
    const int m = *top_count;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        int p = T.parent[top_list[i]];
        for (int guard = 0; p >= 0 && p < nt - 1 && guard < 4096; ++guard) {
            const int old = __hip_atomic_fetch_add(&T.flag[p], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0) break;
            fit_node(p, nt, T);
            p = T.parent[p];
        }
    }
}

__global__ __launch_bounds__(256) void emit(int nt, Tree T, Node* out, DeviceSceneInfo* info) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= 2 * nt - 1) return;
    const bool is_prim = x >= nt - 1;
    if (x != 0) {
        const int p = T.parent[x];
        if (p < 0 || p >= nt - 1) return;                       // not linked (never for a valid tree)
        if (T.last[p] - T.first[p] + 1 <= kLeafMax) return;  // inside a collapsed leaf
    }
    int idx = 0, depth = 0, cur = x;
    while (cur != 0 && depth < 4096) {
        const int p = T.parent[cur];
        if (p < 0 || p >= nt - 1) return;
        const int l = T.left[p];
        idx += (cur == l) ? 1 : 1 + T.cnt[l];
        cur = p;
        ++depth;
    }
    if (idx < 0 || idx >= 2 * nt - 1) return;
    int payload = 0;
    if (is_prim) {
        payload = ((x - (nt - 1)) << 3) | 1;
    } else {
        const int size = T.last[x] - T.first[x] + 1;
        if (size <= kLeafMax) payload = (T.first[x] << 3) | size;
    }
    const float4 lo = T.box[2 * x], hi = T.box[2 * x + 1];
    Node nd;
    nd.lo[0] = lo.x; nd.lo[1] = lo.y; nd.lo[2] = lo.z;
    nd.hi[0] = hi.x; nd.hi[1] = hi.y; nd.hi[2] = hi.z;
    nd.escape = idx + T.cnt[x];
    nd.payload = payload;
    out[idx] = nd;
    atomicMax(&info->max_depth, depth);
    if (x == 0) info->n_nodes = T.cnt[0];
}

__global__ void reorder(const float4* tmp, const uint32_t* vals, int64_t nt, float4* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    const float4* t = tmp + 3 * (size_t)vals[k];
    out[3 * k] = t[0];
    out[3 * k + 1] = t[1];
    out[3 * k + 2] = t[2];
}

// scene of 0 or 1 triangles
__global__ void tiny_scene(const float4* tmp, int nt, Node* out, float4* tris_out, DeviceSceneInfo* info) {
    Node nd;
    if (nt == 0) {
        for (int k = 0; k < 3; ++k) { nd.lo[k] = 0.0f; nd.hi[k] = 0.0f; }
        nd.escape = 0;  // loop bound read by traversal: no nodes
        nd.payload = 0;
        info->n_nodes = 0;
    } else {
        float4 lo, hi;
        tri_box(tmp, lo, hi);
        nd.lo[0] = lo.x; nd.lo[1] = lo.y; nd.lo[2] = lo.z;
        nd.hi[0] = hi.x; nd.hi[1] = hi.y; nd.hi[2] = hi.z;
        nd.escape = 1;
        nd.payload = (0 << 3) | 1;
        tris_out[0] = tmp[0]; tris_out[1] = tmp[1]; tris_out[2] = tmp[2];
        info->n_nodes = 1;
    }
    out[0] = nd;
    info->max_depth = 0;
}

__global__ void init_info(DeviceSceneInfo* info) {
    info->n_nodes = 0;
    info->max_depth = 0;
    info->bad_tris = 0;
    info->pad = 0;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t build_bvh(const float* verts, int64_t nv, const int32_t* tris, int64_t nt64, Node* nodes_out,
                     float4* tris_out, DeviceSceneInfo* info, const TempAlloc& ta, hipStream_t s, int* oom) {
    *oom = 0;
    const int nt = (int)nt64;
    hipLaunchKernelGGL(init_info, dim3(1), dim3(1), 0, s, info);
    const size_t n_nodes = nt > 0 ? (size_t)(2 * nt - 1) : 1;
    // temporary storage (one block, carved)
    size_t sort_bytes = 0;
    if (nt > 1) {
        hipError_t e = rocprim::radix_sort_pairs(nullptr, sort_bytes, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                                 (uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)nt, 0, 63, s);
        if (e != hipSuccess) return e;
    }
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t ntm = nt > 0 ? (size_t)nt : 1;
    const size_t sz_tmp = al(sizeof(float4) * 3 * ntm), sz_keys = al(sizeof(uint64_t) * ntm),
                 sz_vals = al(sizeof(uint32_t) * ntm), sz_i = al(sizeof(int32_t) * n_nodes),
                 sz_box = al(sizeof(float4) * 2 * n_nodes), sz_cb = al(sizeof(int) * 8), sz_sort = al(sort_bytes);
    const size_t total = sz_tmp + 2 * sz_keys + 2 * sz_vals + 8 * sz_i + sz_box + sz_cb + sz_sort;
    char* base = (char*)ta.alloc(ta.ctx, total, s);
    if (!base) { *oom = 1; return hipErrorOutOfMemory; }
    char* p = base;
    auto take = [&](size_t b) { char* r = p; p += b; return r; };
    float4* tmp = (float4*)take(sz_tmp);
    uint64_t* keys = (uint64_t*)take(sz_keys);
    uint64_t* keys2 = (uint64_t*)take(sz_keys);
    uint32_t* vals = (uint32_t*)take(sz_vals);
    uint32_t* vals2 = (uint32_t*)take(sz_vals);
    Tree T;
    T.parent = (int32_t*)take(sz_i);
    T.left = (int32_t*)take(sz_i);
    T.right = (int32_t*)take(sz_i);
    T.first = (int32_t*)take(sz_i);
    T.last = (int32_t*)take(sz_i);
    T.flag = (int32_t*)take(sz_i);
    T.cnt = (int32_t*)take(sz_i);
    int32_t* top_list = (int32_t*)take(sz_i);
    T.box = (float4*)take(sz_box);
    int* cb = (int*)take(sz_cb);
    void* sort_tmp = take(sz_sort);
    hipError_t err = hipSuccess;
    if (nt > 0) {
        hipLaunchKernelGGL(init_bounds, dim3(1), dim3(64), 0, s, cb);
        hipLaunchKernelGGL(tri_prep, dim3(nblk(nt)), dim3(256), 0, s, verts, nv, tris, (int64_t)nt, tmp, cb, info);
    }
    if (nt <= 1) {
        hipLaunchKernelGGL(tiny_scene, dim3(1), dim3(1), 0, s, tmp, nt, nodes_out, tris_out, info);
    } else {
        hipLaunchKernelGGL(morton, dim3(nblk(nt)), dim3(256), 0, s, tmp, (int64_t)nt, cb, keys, vals);
        err = rocprim::radix_sort_pairs(sort_tmp, sort_bytes, keys, keys2, vals, vals2, (size_t)nt, 0, 63, s);
        if (err == hipSuccess) {
            hipLaunchKernelGGL(fill_i32, dim3(nblk(2 * nt - 1)), dim3(256), 0, s, T.parent, (int64_t)(2 * nt - 1), -1);
            hipLaunchKernelGGL(fill_i32, dim3(nblk(2 * nt - 1)), dim3(256), 0, s, T.cnt, (int64_t)(2 * nt - 1), 0);
            hipLaunchKernelGGL(radix_tree, dim3(nblk(nt - 1)), dim3(256), 0, s, keys2, nt, T);
            hipLaunchKernelGGL(fill_i32, dim3(1), dim3(256), 0, s, cb + 6, (int64_t)1, 0);   // top-node count
            hipLaunchKernelGGL(refit_local, dim3(nblk(nt)), dim3(256), 0, s, tmp, vals2, nt, T, top_list, cb + 6);
            hipLaunchKernelGGL(refit_top, dim3(1), dim3(1024), 0, s, top_list, cb + 6, nt, T);
            hipLaunchKernelGGL(emit, dim3(nblk(2 * nt - 1)), dim3(256), 0, s, nt, T, nodes_out, info);
            hipLaunchKernelGGL(reorder, dim3(nblk(nt)), dim3(256), 0, s, tmp, vals2, (int64_t)nt, tris_out);
        }
    }
    if (err == hipSuccess) err = hipGetLastError();
    ta.free(ta.ctx, base, s);
    return err;
}

}  // namespace mcdi
