// Device BVH construction for the shadow-ray mesh (rebuilt whenever the mesh
// changes: the paper re-extracts its mesh every optimisation iteration).
//
// Linear BVH: 63-bit Morton codes of triangle centroids (under a top bit that
// puts the mesh's big triangles first, see morton()), a radix sort, the
// binary radix tree of the sorted codes built in parallel (one lane per
// internal node, Karras 2012), box fitting and the counts of the nodes that
// survive collapsing subtrees of <= 4 triangles (1 among the big ones) into
// leaves, and a final pass that writes every surviving node at its depth-first
// pre-order index with a skip link, so traversal needs no stack.
//
// Fitting runs in two parts over blocks of 256 sorted triangles.  Nodes whose
// triangles lie in one block are fitted bottom-up inside that block's
// workgroup (workgroup-scope atomics pick the second child to arrive).  A
// node spanning blocks is fitted directly: its box is the union of a suffix
// box of its first block, a prefix box of its last block and a sparse-table
// query over the whole blocks between (min and max are idempotent, so two
// overlapping power-of-two ranges cover the span), and its surviving-node
// count is 2 L - 1 for the L leaves in its range, read from a prefix sum of
// leaf marks (every surviving internal node has two surviving children).  No
// dependency chain crosses workgroups.
#include <hip/hip_runtime.h>
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "mcdi_internal.h"

namespace mcdi {
namespace {

__device__ __forceinline__ int ord_key(float f) {
    const int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float ord_val(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7FFFFFFF); }

__device__ __forceinline__ float wave_min(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

constexpr int kFitBlock = 256;   // triangles per fitting block (= workgroup size of the block passes)

// fetch vertices, replace bad triangles by a degenerate one; centroid bounds
// of the workgroup's triangles to part[6 * blockIdx.x] (min xyz, max xyz)
__global__ __launch_bounds__(256) void tri_prep(const float* verts, int64_t nv, const int32_t* tris, int64_t nt,
                                                float4* tmp, float* part, DeviceSceneInfo* info) {
    __shared__ float sb[4][6];
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
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sb[w][0] = cx; sb[w][1] = cy; sb[w][2] = cz;
        sb[w][3] = Cx; sb[w][4] = Cy; sb[w][5] = Cz;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        float v = sb[0][k];
        for (int j = 1; j < 4; ++j) v = k < 3 ? fminf(v, sb[j][k]) : fmaxf(v, sb[j][k]);
        part[6 * (size_t)blockIdx.x + k] = v;
    }
}

// scene centroid bounds from the per-workgroup parts, as order-preserving
// integer keys (one workgroup)
__global__ __launch_bounds__(256) void bounds_reduce(const float* part, int nb, int* cb) {
    __shared__ float sb[4][6];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int k = 0; k < 6; ++k) v[k] = k < 3 ? fminf(v[k], part[6 * (size_t)b + k]) : fmaxf(v[k], part[6 * (size_t)b + k]);
    for (int k = 0; k < 3; ++k) { v[k] = wave_min(v[k]); v[3 + k] = wave_max(v[3 + k]); }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 6; ++k) sb[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        float r = sb[0][k];
        for (int j = 1; j < 4; ++j) r = k < 3 ? fminf(r, sb[j][k]) : fmaxf(r, sb[j][k]);
        cb[k] = ord_key(r);
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

// Key of a triangle: bit 63 clear for a big triangle (its box's longest side
// at least 1/kBigTriDiv of the centroid bounds' longest side), set for the
// others, above the 63-bit Morton code of its centroid.  A mesh with both
// kinds splits at the root into the big triangles (first) and the rest: a
// room's walls, say, stop most shadow rays leaving the geometry inside it,
// and under the Morton order alone each wall triangle widens the box of every
// node it shares with the small triangles around its centroid.  The big ones
// are counted into info->n_big.
__global__ __launch_bounds__(256) void morton(const float4* tmp, int64_t nt, const int* cb, uint64_t* keys,
                                              uint32_t* vals, DeviceSceneInfo* info) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool big = false;
    if (f < nt) {
        const float4 a = tmp[3 * f], b = tmp[3 * f + 1], c = tmp[3 * f + 2];
        const float p[3] = {(a.x + b.x + c.x) * (1.0f / 3.0f), (a.y + b.y + c.y) * (1.0f / 3.0f),
                            (a.z + b.z + c.z) * (1.0f / 3.0f)};
        const float sx = fmaxf(a.x, fmaxf(b.x, c.x)) - fminf(a.x, fminf(b.x, c.x));
        const float sy = fmaxf(a.y, fmaxf(b.y, c.y)) - fminf(a.y, fminf(b.y, c.y));
        const float sz = fmaxf(a.z, fmaxf(b.z, c.z)) - fminf(a.z, fminf(b.z, c.z));
        uint64_t code = 0;
        float cext = 0.0f;
        for (int k = 0; k < 3; ++k) {
            const float lo = ord_val(cb[k]), hi = ord_val(cb[3 + k]);
            const float ext = hi - lo;
            cext = fmaxf(cext, ext);
            float u = ext > 0.0f ? (p[k] - lo) / ext : 0.5f;
            u = fminf(fmaxf(u, 0.0f), 1.0f);
            const uint64_t q = (uint64_t)fminf(u * 2097152.0f, 2097151.0f);
            code |= spread3(q) << (2 - k);
        }
        big = fmaxf(sx, fmaxf(sy, sz)) * kBigTriDiv >= cext;
        keys[f] = big ? code : (code | (1ull << 63));
        vals[f] = (uint32_t)f;
    }
    const uint64_t m = __ballot(big);
    if ((threadIdx.x & 63) == 0 && m != 0) atomicAdd(&info->n_big, (int)__popcll(m));
}

struct Tree {
    int32_t* parent;   // [2nt-1]
    int32_t* left;     // [nt-1] node ids (leaf k = nt-1+k)
    int32_t* right;
    int32_t* first;    // [nt-1] sorted-primitive range
    int32_t* last;
    int32_t* flag;     // [nt-1]
    int32_t* axis;     // [nt-1] the axis the node's Morton split separates its children on
    int32_t* cnt;      // [2nt-1] surviving nodes in the subtree
    float4* box;       // [2*(2nt-1)]
    // block fitting (blocks of kFitBlock sorted triangles)
    int32_t* mark;     // [nt] 1 at the first triangle of every leaf
    int32_t* mark_pre; // [nt] exclusive prefix of mark within the block
    int32_t* blk_base; // [nb+1] leaf marks before each block
    float4* pre;       // [2nt] box of the block's triangles up to k (inclusive)
    float4* suf;       // [2nt] box of the block's triangles from k to the block end
    float4* st;        // [levels][nb][2] sparse table of block boxes
    const int32_t* nbig;   // the big triangles' count (sorted first)
    int nb, levels;
};

// Most triangles a leaf holds: kLeafMax, and kBigLeafMax inside the big
// triangles' subtree (sorted range [0, n_big)) of a mesh that has both kinds.
// Every node but the root lies entirely on one side of n_big.
__device__ __forceinline__ int leaf_cap(const Tree& T, int nt, int last) {
    const int nb = *T.nbig;
    return (nb < nt && last < nb) ? kBigLeafMax : kLeafMax;
}

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
    // the split is at the first bit the range's codes differ in, bit 63 - dnode
    // (x, y, z interleaved from bit 62 down: bit b is x, y or z as b % 3 is 2,
    // 1 or 0); the left child holds the codes with a 0 there, the lower side;
    // equal codes (split by index) take x.  A split at bit 63 (the root of a
    // mesh with big and small triangles) is 3: no axis, the left child (the
    // big triangles) first for every ray
    T.axis[i] = dnode == 0 ? 3 : dnode < 64 ? 2 - (63 - dnode) % 3 : 0;
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
    T.cnt[p] = size <= leaf_cap(T, nt, T.last[p]) ? 1 : 1 + T.cnt[l] + T.cnt[r];
}

// leaf marks: a node of <= leaf_cap triangles whose parent has more is a
// leaf of the collapsed tree (the root, when the whole mesh fits in one)
__global__ __launch_bounds__(256) void mark_leaves(int nt, Tree T) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= 2 * nt - 1) return;
    const bool prim = x >= nt - 1;
    const int first = prim ? x - (nt - 1) : T.first[x];
    const int last = prim ? first : T.last[x];
    const int size = last - first + 1;
    if (size > leaf_cap(T, nt, last)) return;
    if (x != 0) {
        const int p = T.parent[x];
        if (p < 0 || p >= nt - 1 || T.last[p] - T.first[p] + 1 <= leaf_cap(T, nt, T.last[p])) return;
    }
    if (first >= 0 && first < nt) T.mark[first] = 1;
}

// Block pass (workgroup b = sorted triangles [256 b, 256 b + 256)): leaf
// boxes, the block's prefix and suffix boxes and leaf-mark prefix, its box
// (sparse-table level 0) and mark count; then the bottom-up fit of every node
// inside the block, the second of the two children to arrive fitting the
// parent.  That climb stays inside one workgroup, so workgroup-scope atomics
// order it (an agent-scope release would write the L2 back on every step); it
// stops at the first node spanning blocks.
__global__ __launch_bounds__(kFitBlock) void fit_block(const float4* tmp, const uint32_t* vals, int nt, Tree T) {
    __shared__ float4 slo[kFitBlock], shi[kFitBlock];
    __shared__ int sm[kFitBlock];
    const int t = threadIdx.x;
    const int lo = blockIdx.x * kFitBlock;
    const int hi = min(nt, lo + kFitBlock) - 1;
    const int k = lo + t;
    const bool valid = k <= hi;
    float4 blo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f), bhi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
    int m = 0;
    if (valid) {
        tri_box(tmp + 3 * (size_t)vals[k], blo, bhi);
        const int leaf = nt - 1 + k;
        T.box[2 * leaf] = blo;
        T.box[2 * leaf + 1] = bhi;
        T.cnt[leaf] = 1;
        m = T.mark[k];
    }
    // inclusive prefix (Hillis-Steele) of boxes and marks
    slo[t] = blo; shi[t] = bhi; sm[t] = m;
    __syncthreads();
    for (int o = 1; o < kFitBlock; o <<= 1) {
        float4 al = slo[t], ah = shi[t];
        int am = sm[t];
        if (t >= o) {
            const float4 bl = slo[t - o], bh = shi[t - o];
            al = make_float4(fminf(al.x, bl.x), fminf(al.y, bl.y), fminf(al.z, bl.z), 0.0f);
            ah = make_float4(fmaxf(ah.x, bh.x), fmaxf(ah.y, bh.y), fmaxf(ah.z, bh.z), 0.0f);
            am += sm[t - o];
        }
        __syncthreads();
        slo[t] = al; shi[t] = ah; sm[t] = am;
        __syncthreads();
    }
    if (valid) {
        T.pre[2 * k] = slo[t];
        T.pre[2 * k + 1] = shi[t];
        T.mark_pre[k] = sm[t] - m;
    }
    if (k == hi) {
        T.st[2 * blockIdx.x] = slo[t];
        T.st[2 * blockIdx.x + 1] = shi[t];
        T.blk_base[blockIdx.x] = sm[t];   // the block's mark count (scanned by block_table)
    }
    __syncthreads();
    // suffix: the same scan from the block end
    slo[t] = blo; shi[t] = bhi;
    __syncthreads();
    for (int o = 1; o < kFitBlock; o <<= 1) {
        float4 al = slo[t], ah = shi[t];
        if (t + o < kFitBlock) {
            const float4 bl = slo[t + o], bh = shi[t + o];
            al = make_float4(fminf(al.x, bl.x), fminf(al.y, bl.y), fminf(al.z, bl.z), 0.0f);
            ah = make_float4(fmaxf(ah.x, bh.x), fmaxf(ah.y, bh.y), fmaxf(ah.z, bh.z), 0.0f);
        }
        __syncthreads();
        slo[t] = al; shi[t] = ah;
        __syncthreads();
    }
    if (valid) {
        T.suf[2 * k] = slo[t];
        T.suf[2 * k + 1] = shi[t];
    }
    if (!valid) return;
    int p = T.parent[nt - 1 + k];
    for (int guard = 0; p >= 0 && p < nt - 1 && guard < 4096; ++guard) {
        if (T.first[p] < lo || T.last[p] > hi) return;   // spans blocks: fit_top
        const int old = __hip_atomic_fetch_add(&T.flag[p], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == 0) return;
        fit_node(p, nt, T);
        p = T.parent[p];
    }
}

// One workgroup: exclusive scan of the block mark counts (blk_base, with the
// total at nb) and the sparse table over block boxes, level j holding the box
// of blocks [b, b + 2^j) (clamped at the last block).
__global__ __launch_bounds__(1024) void block_table(Tree T) {
    __shared__ int s[1024];
    const int t = threadIdx.x, nb = T.nb;
    int carry = 0;
    for (int c0 = 0; c0 < nb; c0 += 1024) {
        const int b = c0 + t;
        const int v = b < nb ? T.blk_base[b] : 0;
        s[t] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int a = t >= o ? s[t - o] : 0;
            __syncthreads();
            s[t] += a;
            __syncthreads();
        }
        if (b < nb) T.blk_base[b] = carry + s[t] - v;
        const int tot = s[1023];
        __syncthreads();
        carry += tot;
    }
    if (t == 0) T.blk_base[nb] = carry;
    for (int j = 1; j < T.levels; ++j) {
        const float4* prev = T.st + 2 * (size_t)(j - 1) * nb;
        float4* cur = T.st + 2 * (size_t)j * nb;
        const int h = 1 << (j - 1);
        for (int b = t; b < nb; b += 1024) {
            const int b2 = min(b + h, nb - 1);
            const float4 al = prev[2 * b], ah = prev[2 * b + 1], bl = prev[2 * b2], bh = prev[2 * b2 + 1];
            cur[2 * b] = make_float4(fminf(al.x, bl.x), fminf(al.y, bl.y), fminf(al.z, bl.z), 0.0f);
            cur[2 * b + 1] = make_float4(fmaxf(ah.x, bh.x), fmaxf(ah.y, bh.y), fmaxf(ah.z, bh.z), 0.0f);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void grow(float4& lo, float4& hi, const float4* b) {
    lo = make_float4(fminf(lo.x, b[0].x), fminf(lo.y, b[0].y), fminf(lo.z, b[0].z), 0.0f);
    hi = make_float4(fmaxf(hi.x, b[1].x), fmaxf(hi.y, b[1].y), fmaxf(hi.z, b[1].z), 0.0f);
}

// leaves before sorted position i (i in [0, nt])
__device__ __forceinline__ int leaves_before(const Tree& T, int nt, int i) {
    return i >= nt ? T.blk_base[T.nb] : T.blk_base[i / kFitBlock] + T.mark_pre[i];
}

// every internal node spanning blocks: box and surviving-node count directly
__global__ __launch_bounds__(256) void fit_top(int nt, Tree T) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nt - 1) return;
    const int f = T.first[p], l = T.last[p];
    if (f < 0 || l >= nt || f > l) return;
    const int bf = f / kFitBlock, bl = l / kFitBlock;
    if (bf == bl) return;   // fitted by its block
    float4 lo = T.suf[2 * f], hi = T.suf[2 * f + 1];
    grow(lo, hi, T.pre + 2 * (size_t)l);
    const int n = bl - bf - 1;   // whole blocks strictly between
    if (n > 0) {
        int j = 31 - __clz(n);
        j = min(j, T.levels - 1);
        grow(lo, hi, T.st + 2 * ((size_t)j * T.nb + bf + 1));
        grow(lo, hi, T.st + 2 * ((size_t)j * T.nb + (bl - (1 << j))));
    }
    T.box[2 * p] = lo;
    T.box[2 * p + 1] = hi;
    T.cnt[p] = 2 * (leaves_before(T, nt, l + 1) - leaves_before(T, nt, f)) - 1;
}

// Quantisation frame of the scene from its root box: base below the box and
// a step such that base + 65535 step lies above it, both with a pad of
// 2^-20 of the largest extent, base rounded down and step up to FP32.
__device__ void qframe_of(float4 rlo, float4 rhi, QFrame& F) {
    const double ext = fmax(fmax((double)rhi.x - rlo.x, (double)rhi.y - rlo.y), (double)rhi.z - rlo.z);
    const double pad = fmax(ext * 0x1p-20, 1e-30);
    const double lo[3] = {rlo.x, rlo.y, rlo.z}, hi[3] = {rhi.x, rhi.y, rhi.z};
    for (int a = 0; a < 3; ++a) {
        F.base[a] = __double2float_rd(lo[a] - pad);
        F.step[a] = __double2float_ru((hi[a] + pad - (double)F.base[a]) / 65535.0);
    }
}

// Outward 16-bit quantisation: the plane of q_lo is at or below lo, that of
// q_hi at or above hi (exact in FP64: q * step needs at most 41 bits).  A
// non-finite coordinate gives the whole range.
__device__ uint32_t quant_lo(float v, float base, float step) {
    if (!isfinite(v)) return 0u;
    double q = floor(((double)v - base) / step);
    q = fmin(fmax(q, 0.0), 65535.0);
    while (q > 0.0 && (double)base + q * (double)step > (double)v) q -= 1.0;
    return (uint32_t)q;
}
__device__ uint32_t quant_hi(float v, float base, float step) {
    if (!isfinite(v)) return 65535u;
    double q = ceil(((double)v - base) / step);
    q = fmin(fmax(q, 0.0), 65535.0);
    while (q < 65535.0 && (double)base + q * (double)step < (double)v) q += 1.0;
    return (uint32_t)q;
}

__device__ QNode quantise(const QFrame& F, const Node& nd) {
    uint32_t l[3], h[3];
    for (int a = 0; a < 3; ++a) {
        l[a] = quant_lo(nd.lo[a], F.base[a], F.step[a]);
        h[a] = quant_hi(nd.hi[a], F.base[a], F.step[a]);
    }
    QNode q;
    q.x = l[0] | (l[1] << 16);
    q.y = l[2] | (h[0] << 16);
    q.z = h[1] | (h[2] << 16);
    q.w = nd.payload != 0 ? (kQLeaf | (uint32_t)nd.payload) : (uint32_t)nd.escape;
    return q;
}

__global__ __launch_bounds__(256) void emit(int nt, Tree T, Node* out, QNode* qout, QFrame* frame,
                                            DeviceSceneInfo* info, int32_t* gflag, int32_t* naxis) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= 2 * nt - 1) return;
    const bool is_prim = x >= nt - 1;
    if (x != 0) {
        const int p = T.parent[x];
        if (p < 0 || p >= nt - 1) return;                       // not linked (never for a valid tree)
        if (T.last[p] - T.first[p] + 1 <= leaf_cap(T, nt, T.last[p])) return;  // inside a collapsed leaf
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
        if (size <= leaf_cap(T, nt, T.last[x])) payload = (T.first[x] << 3) | size;
    }
    const float4 lo = T.box[2 * x], hi = T.box[2 * x + 1];
    Node nd;
    nd.lo[0] = lo.x; nd.lo[1] = lo.y; nd.lo[2] = lo.z;
    nd.hi[0] = hi.x; nd.hi[1] = hi.y; nd.hi[2] = hi.z;
    nd.escape = idx + T.cnt[x];
    nd.payload = payload;
    out[idx] = nd;
    naxis[idx] = is_prim ? 0 : T.axis[x];
    // the root's box (internal node 0) sets the frame, the same for every thread
    QFrame F;
    qframe_of(T.box[0], T.box[1], F);
    qout[idx] = quantise(F, nd);
    if (idx == 0) *frame = F;
    // a wide node for the root and for every internal node at even depth
    gflag[idx] = (idx == 0 || (payload == 0 && (depth & 1) == 0)) ? 1 : 0;
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

// The 4-wide hierarchy of the shadow-ray traversal, collapsed from the binary
// one: a wide node for the root and for every internal node N at even depth,
// whose up to four children are N's children, a child that is internal being
// replaced by its own two children.  Slots 0-1 hold what N's first child
// contributes (itself when it is a leaf, else its two children), slots 2-3
// what the second contributes; a child record is the quantised box of that
// binary node with w = its wide node's index (internal) or kQLeaf | payload
// (leaf), and an unused slot holds an empty record (lo > hi: no ray hits it);
// every record's w also carries kRefLive.
// Wide nodes are numbered in the binary pre-order of their nodes (an
// exclusive scan of the flags), so the wide hierarchy is in pre-order too.
//
// Beside each wide node, its visit order: for each of the eight octants of a
// ray direction (bit a set where the component on axis a is negative), three
// bits -- swap slots 0 and 1, swap slots 2 and 3, swap the two pairs -- that
// put each binary split's child farther along the ray after the nearer one in
// slot order (the big triangles' child after the other at the split that
// separates them).  The walk pushes hit children in slot order and pops the
// last pushed, so it descends into the farther child first.
__device__ __forceinline__ QNode empty_record() {
    QNode q;
    q.x = 0xFFFFFFFFu;   // lo.x = lo.y = 65535
    q.y = 0x0000FFFFu;   // lo.z = 65535, hi.x = 0
    q.z = 0u;            // hi.y = hi.z = 0
    q.w = kQLeaf;        // an empty leaf, should it ever be taken
    return q;
}

// 1 when a ray of octant o should take the split's left child first: the
// left child lies farther along the ray on the split's axis, or holds the big
// triangles (axis 3)
__device__ __forceinline__ uint32_t left_first(int axis, int o) {
    return axis == 3 ? 1u : (uint32_t)((o >> axis) & 1);
}

__device__ __forceinline__ QNode child_record(const Node* out, const QNode* qout, const int32_t* gidx, int x) {
    QNode q = qout[x];
    if (out[x].payload == 0) q.w = (uint32_t)gidx[x];
    return q;
}

__global__ __launch_bounds__(256) void wide_groups(const Node* out, const QNode* qout, const int32_t* gflag,
                                                   const int32_t* gidx, const int32_t* naxis, int n_max,
                                                   QNode* groups, uint32_t* gorder, DeviceSceneInfo* info) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n_max) return;
    const int n_nodes = out[0].escape;            // surviving binary nodes
    if (x >= n_nodes || !gflag[x]) return;
    const int self = gidx[x];
    QNode* g = groups + 4 * (size_t)self;
    for (int k = 0; k < 4; ++k) g[k] = empty_record();
    uint32_t order = 0u;
    if (out[x].payload != 0) {                    // a root that is a leaf
        g[0] = child_record(out, qout, gidx, x);
    } else {
        const int c[2] = {x + 1, out[x + 1].escape};
        int sub_axis[2] = {-1, -1};
        for (int i = 0; i < 2; ++i) {
            const int y = c[i];
            if (y <= x || y >= n_nodes) continue;    // never for a valid tree
            if (out[y].payload != 0) {
                g[2 * i] = child_record(out, qout, gidx, y);
            } else {
                sub_axis[i] = naxis[y];
                const int d[2] = {y + 1, out[y + 1].escape};
                for (int j = 0; j < 2; ++j)
                    if (d[j] > y && d[j] < n_nodes) g[2 * i + j] = child_record(out, qout, gidx, d[j]);
            }
        }
        const int top = naxis[x];
        for (int o = 0; o < 8; ++o) {
            uint32_t f = left_first(top, o) << 2;
            if (sub_axis[0] >= 0) f |= left_first(sub_axis[0], o);
            if (sub_axis[1] >= 0) f |= left_first(sub_axis[1], o) << 1;
            order |= f << (3 * o);
        }
    }
    gorder[self] = order;
    // the walk's termination rests on this: every internal child reference
    // lies past its parent and inside the node array (pre-order numbering);
    // a violation (never for a valid tree) sends the scene to the binary walk
    const int n_groups = gidx[n_max - 1] + gflag[n_max - 1];
    for (int i = 0; i < 4; ++i) {
        const uint32_t w = g[i].w;
        if (!(w & kQLeaf) && ((int)w <= self || (int)w >= n_groups)) atomicOr(&info->wide_bad, 1);
        g[i].w = w | kRefLive;
    }
}

__global__ void tiny_scene(const float4* tmp, int nt, Node* out, float4* tris_out, QNode* qout, QFrame* frame,
                           DeviceSceneInfo* info, QNode* groups, uint32_t* gorder) {
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
    QFrame F;
    qframe_of(make_float4(nd.lo[0], nd.lo[1], nd.lo[2], 0.0f), make_float4(nd.hi[0], nd.hi[1], nd.hi[2], 0.0f), F);
    qout[0] = quantise(F, nd);
    *frame = F;
    info->max_depth = 0;
    groups[0] = nt == 0 ? empty_record() : qout[0];
    for (int k = 1; k < 4; ++k) groups[k] = empty_record();
    for (int k = 0; k < 4; ++k) groups[k].w |= kRefLive;
    gorder[0] = 0u;
    info->n_groups = 1;
}

__global__ void count_groups(const int32_t* gflag, const int32_t* gidx, int n, DeviceSceneInfo* info) {
    info->n_groups = gidx[n - 1] + gflag[n - 1];
}

__global__ void init_info(DeviceSceneInfo* info) {
    info->n_nodes = 0;
    info->max_depth = 0;
    info->bad_tris = 0;
    info->n_groups = 0;
    info->wide = 0;
    info->wide_bad = 0;
    info->n_big = 0;
    info->depth_complexity = 0.0f;
    info->leaf_area = 0.0;
}

__device__ __forceinline__ double box_area(const Node& nd) {
    const double dx = fmax((double)nd.hi[0] - nd.lo[0], 0.0), dy = fmax((double)nd.hi[1] - nd.lo[1], 0.0),
                 dz = fmax((double)nd.hi[2] - nd.lo[2], 0.0);
    return 2.0 * (dx * dy + dy * dz + dz * dx);
}

// the leaf boxes' surface areas, summed into info->leaf_area
__global__ __launch_bounds__(256) void leaf_area_sum(const Node* out, int n_max, DeviceSceneInfo* info) {
    __shared__ double part[4];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0;
    if (x < n_max && x < out[0].escape && out[x].payload != 0) a = box_area(out[x]);
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&info->leaf_area, part[0] + part[1] + part[2] + part[3]);
}

// depth complexity and the traversal it selects
__global__ void choose_walk(const Node* out, DeviceSceneInfo* info) {
    const double root = box_area(out[0]);
    const double d = root > 0.0 ? info->leaf_area / root : 0.0;
    info->depth_complexity = (float)d;
    info->wide = (d >= (double)kWideDepthComplexity && info->wide_bad == 0) ? 1 : 0;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t build_bvh(const float* verts, int64_t nv, const int32_t* tris, int64_t nt64, Node* nodes_out,
                     float4* tris_out, QNode* qnodes_out, QFrame* frame_out, QNode* groups_out,
                     DeviceSceneInfo* info, const TempAlloc& ta, hipStream_t s, int* oom) {
    *oom = 0;
    const int nt = (int)nt64;
    hipLaunchKernelGGL(init_info, dim3(1), dim3(1), 0, s, info);
    const size_t n_nodes = nt > 0 ? (size_t)(2 * nt - 1) : 1;
    // temporary storage (one block, carved)
    size_t sort_bytes = 0;
    if (nt > 1) {
        hipError_t e = rocprim::radix_sort_pairs(nullptr, sort_bytes, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                                 (uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)nt, 0, 64, s);
        if (e != hipSuccess) return e;
    }
    size_t scan_bytes = 0;
    if (nt > 1) {
        hipError_t e = rocprim::exclusive_scan(nullptr, scan_bytes, (const int32_t*)nullptr, (int32_t*)nullptr, 0,
                                               n_nodes, rocprim::plus<int32_t>(), s);
        if (e != hipSuccess) return e;
    }
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t ntm = nt > 0 ? (size_t)nt : 1;
    const int nb = (int)((ntm + kFitBlock - 1) / kFitBlock);
    int levels = 1;
    while ((1 << levels) <= nb) ++levels;   // 2^(levels-1) <= nb < 2^levels
    const size_t sz_tmp = al(sizeof(float4) * 3 * ntm), sz_keys = al(sizeof(uint64_t) * ntm),
                 sz_vals = al(sizeof(uint32_t) * ntm), sz_i = al(sizeof(int32_t) * n_nodes),
                 sz_box = al(sizeof(float4) * 2 * n_nodes), sz_cb = al(sizeof(int) * 8), sz_sort = al(sort_bytes),
                 sz_part = al(sizeof(float) * 6 * (size_t)nblk(ntm)), sz_nt = al(sizeof(int32_t) * ntm),
                 sz_base = al(sizeof(int32_t) * (size_t)(nb + 1)), sz_pre = al(sizeof(float4) * 2 * ntm),
                 sz_st = al(sizeof(float4) * 2 * (size_t)nb * (size_t)levels);
    const size_t sz_scan = al(scan_bytes);
    const size_t total = sz_tmp + 2 * sz_keys + 2 * sz_vals + 11 * sz_i + sz_box + sz_cb + sz_sort + sz_part +
                         2 * sz_nt + sz_base + 2 * sz_pre + sz_st + sz_scan;
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
    T.axis = (int32_t*)take(sz_i);
    T.cnt = (int32_t*)take(sz_i);
    T.box = (float4*)take(sz_box);
    int* cb = (int*)take(sz_cb);
    void* sort_tmp = take(sz_sort);
    float* part = (float*)take(sz_part);
    T.mark = (int32_t*)take(sz_nt);
    T.mark_pre = (int32_t*)take(sz_nt);
    T.blk_base = (int32_t*)take(sz_base);
    T.pre = (float4*)take(sz_pre);
    T.suf = (float4*)take(sz_pre);
    T.st = (float4*)take(sz_st);
    int32_t* gflag = (int32_t*)take(sz_i);
    int32_t* gidx = (int32_t*)take(sz_i);
    int32_t* naxis = (int32_t*)take(sz_i);
    void* scan_tmp = take(sz_scan);
    // the visit orders follow the wide nodes in the same allocation
    uint32_t* gorder = reinterpret_cast<uint32_t*>(groups_out + 4 * ntm);
    T.nb = nb;
    T.levels = levels;
    T.nbig = &info->n_big;
    hipError_t err = hipSuccess;
    if (nt > 0) {
        hipLaunchKernelGGL(tri_prep, dim3(nblk(nt)), dim3(256), 0, s, verts, nv, tris, (int64_t)nt, tmp, part, info);
        hipLaunchKernelGGL(bounds_reduce, dim3(1), dim3(256), 0, s, part, (int)nblk(nt), cb);
    }
    if (nt <= 1) {
        hipLaunchKernelGGL(tiny_scene, dim3(1), dim3(1), 0, s, tmp, nt, nodes_out, tris_out, qnodes_out, frame_out,
                           info, groups_out, gorder);
    } else {
        hipLaunchKernelGGL(morton, dim3(nblk(nt)), dim3(256), 0, s, tmp, (int64_t)nt, cb, keys, vals, info);
        err = rocprim::radix_sort_pairs(sort_tmp, sort_bytes, keys, keys2, vals, vals2, (size_t)nt, 0, 64, s);
        if (err == hipSuccess) {
            hipLaunchKernelGGL(fill_i32, dim3(nblk(2 * nt - 1)), dim3(256), 0, s, T.parent, (int64_t)(2 * nt - 1), -1);
            hipLaunchKernelGGL(fill_i32, dim3(nblk(2 * nt - 1)), dim3(256), 0, s, T.cnt, (int64_t)(2 * nt - 1), 0);
            hipLaunchKernelGGL(fill_i32, dim3(nblk(nt)), dim3(256), 0, s, T.mark, (int64_t)nt, 0);
            hipLaunchKernelGGL(radix_tree, dim3(nblk(nt - 1)), dim3(256), 0, s, keys2, nt, T);
            hipLaunchKernelGGL(mark_leaves, dim3(nblk(2 * nt - 1)), dim3(256), 0, s, nt, T);
            hipLaunchKernelGGL(fit_block, dim3((unsigned)nb), dim3(kFitBlock), 0, s, tmp, vals2, nt, T);
            hipLaunchKernelGGL(block_table, dim3(1), dim3(1024), 0, s, T);
            hipLaunchKernelGGL(fit_top, dim3(nblk(nt - 1)), dim3(256), 0, s, nt, T);
            hipLaunchKernelGGL(fill_i32, dim3(nblk(2 * nt - 1)), dim3(256), 0, s, gflag, (int64_t)(2 * nt - 1), 0);
            hipLaunchKernelGGL(emit, dim3(nblk(2 * nt - 1)), dim3(256), 0, s, nt, T, nodes_out, qnodes_out,
                               frame_out, info, gflag, naxis);
            hipLaunchKernelGGL(reorder, dim3(nblk(nt)), dim3(256), 0, s, tmp, vals2, (int64_t)nt, tris_out);
            err = rocprim::exclusive_scan(scan_tmp, scan_bytes, gflag, gidx, 0, (size_t)(2 * nt - 1),
                                          rocprim::plus<int32_t>(), s);
        }
        if (err == hipSuccess) {
            hipLaunchKernelGGL(wide_groups, dim3(nblk(2 * nt - 1)), dim3(256), 0, s, nodes_out, qnodes_out, gflag,
                               gidx, naxis, 2 * nt - 1, groups_out, gorder, info);
            hipLaunchKernelGGL(count_groups, dim3(1), dim3(1), 0, s, gflag, gidx, 2 * nt - 1, info);
            hipLaunchKernelGGL(leaf_area_sum, dim3(nblk(2 * nt - 1)), dim3(256), 0, s, nodes_out, 2 * nt - 1, info);
            hipLaunchKernelGGL(choose_walk, dim3(1), dim3(1), 0, s, nodes_out, info);
        }
    }
    if (err == hipSuccess) err = hipGetLastError();
    ta.free(ta.ctx, base, s);
    return err;
}

}  // namespace mcdi
