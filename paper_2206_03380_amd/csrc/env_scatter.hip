// Probe-gradient scatter of the adjoint (section 3.1: the probe texels are
// optimisation variables; each light or BSDF sample adds its coefficient times
// the upstream gradient to the texel its direction falls in).
//
// Global float atomics on this chip retire about one 128-byte line per clock
// per XCD whatever their scope, so an atomic per sample and channel to random
// texels is bound by line requests, not bandwidth.  Texels outside the
// per-workgroup LDS hot set therefore go through records instead: the adjoint
// appends one 16-byte record (texel, three values) per sample to its tile's
// region (LDS fill counter, one atomic per wave), and this pass sums them:
//   1. histogram: records per bucket of 1024 (large probes: up to 4096)
//      consecutive texels, per
//      workgroup in LDS, kept per workgroup and added to the bucket totals;
//   2. scan: bucket starts and fill cursors;
//   3. scatter: counting sort by bucket; each batch of records is sorted in
//      LDS first so the global writes come out as contiguous runs;
//   4. accumulate: fixed chunks of the sorted records, each bucket segment
//      summed exactly in 64-bit fixed point in an LDS copy of its texels
//      (integer LDS atomics run about six times faster than float ones
//      here), then one float global add per touched texel channel,
//      consecutive lanes on consecutive channels (16 per cache line).
// Fixed point: a chunk adds at most 2^c records of magnitude below 2^e (e from
// the bucket's largest |value|, found by the histogram step), so with scale
// 2^(62-c-e) the int64 sum cannot overflow, and each record is rounded by at
// most 2^-(63-c-e), i.e. < 2^-(63-c) of the bucket maximum.  The chunks split
// the records actually written (R, read on the device) over the launch's
// workgroups: a chunk holds max(2^10, ceil(R / workgroups)) records and c is
// the ceiling of its log2.  There are min(2048, ceil(capacity / 2^10))
// workgroups and R <= capacity <= 2^30, so 10 <= c <= 19: the rounding of one
// record is below 2^-44 of the bucket maximum.  (Sizing the chunks by the
// capacity instead left most workgroups idle when most samples add nothing:
// on the 1.0M-triangle room 95% of the shadow rays are blocked, and 8.7M
// records filled 67 chunks of a 268M-record capacity.)  A bucket with a non-finite value takes
// the float-atomic path instead, so NaN and infinity propagate as with direct
// atomics.
// Each record crosses HBM five times (written, read by the histogram and the
// scatter, written sorted, read by the accumulation).
//
// The bilinear lookup spreads a sample's coefficient over four taps.  Its
// record (32 bytes) carries the upper-left tap as a base index in an extended
// grid of H + 1 rows (row i0 + 1 for i0 in [-1, H-1], so the row above the
// first row centre is representable) and the fractions fx, fy.  Buckets and
// the sort run on the base; the accumulation sums the four tap weights into
// four accumulators at the base, and a gather adds, for every texel, the
// accumulators of the bases whose taps land on it (columns wrapping, rows
// clamped at the poles).  One record per sample instead of four.
#include <hip/hip_runtime.h>

#include "mcdi_internal.h"

namespace mcdi {
namespace {

constexpr int kMinShift = 10;          // at least 1024 texels per bucket
constexpr int kMaxShift = 12;          // 4096 texels: 96 KB of LDS per fixed-point bucket copy
constexpr int kMaxBuckets = 4096;      // 4096 x 4096 texels at most
constexpr int kGridMax = 2048;
constexpr int kBatch = 1024;           // records per LDS sort batch
constexpr uint32_t kChunkMin = 1024;   // sorted records per accumulate workgroup, at least

__device__ __forceinline__ uint32_t rec_texel(const float4& r) { return __float_as_uint(r.x); }

// records: S float4s each (1 nearest, 2 bilinear); the key is the first word,
// the three values are words 1..3 (nearest) or the second float4's x, y, z
template <bool BIL> struct RecT;
template <> struct RecT<false> {
    float4 a;
    __device__ __forceinline__ static RecT load(const float4* base, uint32_t i) { return RecT{base[i]}; }
    __device__ __forceinline__ void store(float4* base, uint32_t i) const { base[i] = a; }
    __device__ __forceinline__ uint32_t key() const { return rec_texel(a); }
    __device__ __forceinline__ float v(int c) const { return c == 0 ? a.y : (c == 1 ? a.z : a.w); }
};
template <> struct RecT<true> {
    float4 a, b;
    __device__ __forceinline__ static RecT load(const float4* base, uint32_t i) {
        return RecT{base[2 * (size_t)i], base[2 * (size_t)i + 1]};
    }
    __device__ __forceinline__ void store(float4* base, uint32_t i) const {
        base[2 * (size_t)i] = a;
        base[2 * (size_t)i + 1] = b;
    }
    __device__ __forceinline__ uint32_t key() const { return rec_texel(a); }
    __device__ __forceinline__ float v(int c) const { return c == 0 ? b.x : (c == 1 ? b.y : b.z); }
};

int tile_grid(int64_t n_tiles) { return (int)(n_tiles < kGridMax ? n_tiles : kGridMax); }

__global__ __launch_bounds__(1024) void init_kernel(EnvScatter p) {
    for (int b = threadIdx.x; b < p.K; b += blockDim.x) {
        p.cursor[b] = 0u;
        p.bmax[b] = 0u;
    }
}

// bilinear accumulators to zero (grid-stride)
__global__ __launch_bounds__(256) void zero_acc4(float* acc, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) acc[k] = 0.0f;
}

// bits of the largest |value| of a record: for non-negative floats the bit
// patterns order like the values, and NaN sorts above infinity (bilinear tap
// weights are at most 1, so this also bounds every tap's value)
template <bool BIL>
__device__ __forceinline__ uint32_t abs_max_bits(const RecT<BIL>& r) {
    const uint32_t a = __float_as_uint(r.v(0)) & 0x7FFFFFFFu, b = __float_as_uint(r.v(1)) & 0x7FFFFFFFu,
                   c = __float_as_uint(r.v(2)) & 0x7FFFFFFFu;
    return max(a, max(b, c));
}

// Records per bucket and the largest |value| per bucket over the tiles
// blockIdx.x, + gridDim.x, ...: counts kept per workgroup (for the scatter)
// and added to the bucket totals.
template <bool BIL>
__global__ __launch_bounds__(256) void hist_kernel(EnvScatter p) {
    __shared__ uint32_t h[kMaxBuckets];
    __shared__ uint32_t hm[kMaxBuckets];
    for (int b = threadIdx.x; b < p.K; b += 256) {
        h[b] = 0u;
        hm[b] = 0u;
    }
    __syncthreads();
    constexpr int S = BIL ? 2 : 1;
    for (int64_t t = blockIdx.x; t < p.n_tiles; t += gridDim.x) {
        const float4* r = p.rec + (size_t)t * p.region * S;
        const uint32_t c = p.tile_count[t];
        for (uint32_t i = threadIdx.x; i < c; i += 1024) {
            RecT<BIL> v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (i + 256 * j < c) v[j] = RecT<BIL>::load(r, i + 256 * j);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (i + 256 * j < c) {
                    const uint32_t b = v[j].key() >> p.shift;
                    atomicAdd(&h[b], 1u);
                    atomicMax(&hm[b], abs_max_bits<BIL>(v[j]));
                }
        }
    }
    __syncthreads();
    uint32_t* mine = p.wg_hist + (size_t)blockIdx.x * p.K;
    for (int b = threadIdx.x; b < p.K; b += 256) {
        mine[b] = h[b];
        if (h[b]) {
            atomicAdd(&p.cursor[b], h[b]);
            atomicMax(&p.bmax[b], hm[b]);
        }
    }
}

// exclusive scan of the bucket sizes: one block of 1024 threads, four
// consecutive buckets per thread
__global__ __launch_bounds__(1024) void scan_kernel(EnvScatter p) {
    __shared__ uint32_t s[1024];
    const int t = threadIdx.x;
    uint32_t v[4], sum = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int b = 4 * t + j;
        v[j] = b < p.K ? p.cursor[b] : 0u;
        sum += v[j];
    }
    s[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t a = t >= o ? s[t - o] : 0u;
        __syncthreads();
        s[t] += a;
        __syncthreads();
    }
    uint32_t run = s[t] - sum;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int b = 4 * t + j;
        if (b < p.K) {
            p.start[b] = run;
            p.cursor[b] = run;
        }
        run += v[j];
    }
    if (t == 1023) p.start[p.K] = s[t];
}

// exclusive scan of a[0..K) in place by 256 threads (ends with a barrier)
__device__ void block_scan_k(uint32_t* a, int K, uint32_t* s256) {
    const int per = (K + 255) / 256;
    const int b0 = threadIdx.x * per;
    uint32_t sum = 0u;
    for (int j = 0; j < per; ++j)
        if (b0 + j < K) sum += a[b0 + j];
    s256[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)o ? s256[threadIdx.x - o] : 0u;
        __syncthreads();
        s256[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = s256[threadIdx.x] - sum;
    for (int j = 0; j < per; ++j)
        if (b0 + j < K) {
            const uint32_t v = a[b0 + j];
            a[b0 + j] = run;
            run += v;
        }
    __syncthreads();
}

// Counting-sort scatter over the same tiles as the histogram workgroup.
// LDS: lh, lofs, dst [K] each, then the batch [kBatch] of sorted records.
template <bool BIL>
__global__ __launch_bounds__(256) void scatter_kernel(EnvScatter p) {
    extern __shared__ uint32_t sm[];
    __shared__ uint32_t s256[256];
    constexpr int S = BIL ? 2 : 1;
    const int K = p.K;
    uint32_t* lh = sm;
    uint32_t* lofs = sm + K;
    uint32_t* dst = sm + 2 * K;   // next global position of each bucket
    float4* srt = (float4*)(sm + ((3 * K + 3) & ~3));
    const uint32_t* mine = p.wg_hist + (size_t)blockIdx.x * K;
    for (int b = threadIdx.x; b < K; b += 256) dst[b] = mine[b] ? atomicAdd(&p.cursor[b], mine[b]) : 0u;
    __syncthreads();
    for (int64_t t = blockIdx.x; t < p.n_tiles; t += gridDim.x) {
        const float4* rr = p.rec + (size_t)t * p.region * S;
        const uint32_t c = p.tile_count[t];
        for (uint32_t b0 = 0; b0 < c; b0 += kBatch) {
            const int n = (int)min((uint32_t)kBatch, c - b0);
            RecT<BIL> r[kBatch / 256];
            uint32_t rank[kBatch / 256];
            for (int b = threadIdx.x; b < K; b += 256) lh[b] = 0u;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kBatch / 256; ++j) {
                const int i = threadIdx.x + 256 * j;
                if (i < n) r[j] = RecT<BIL>::load(rr, b0 + i);
            }
#pragma unroll
            for (int j = 0; j < kBatch / 256; ++j) {
                const int i = threadIdx.x + 256 * j;
                if (i < n) rank[j] = atomicAdd(&lh[r[j].key() >> p.shift], 1u);
            }
            __syncthreads();
            for (int b = threadIdx.x; b < K; b += 256) lofs[b] = lh[b];
            __syncthreads();
            block_scan_k(lofs, K, s256);
#pragma unroll
            for (int j = 0; j < kBatch / 256; ++j) {
                const int i = threadIdx.x + 256 * j;
                if (i < n) r[j].store(srt, lofs[r[j].key() >> p.shift] + rank[j]);
            }
            __syncthreads();
            for (int i = threadIdx.x; i < n; i += 256) {
                const RecT<BIL> v = RecT<BIL>::load(srt, (uint32_t)i);
                const uint32_t b = v.key() >> p.shift;
                v.store(p.sorted, dst[b] + ((uint32_t)i - lofs[b]));
            }
            __syncthreads();
            for (int b = threadIdx.x; b < K; b += 256) dst[b] += lh[b];
            __syncthreads();
        }
    }
}

// acc holds A accumulators of 3 channels per texel of the bucket, [a][texel][3]:
// A = 1 (nearest) or the four taps (bilinear), flushed into g_env or acc4
template <bool BIL>
__global__ __launch_bounds__(256) void accumulate_kernel(EnvScatter p) {
    extern __shared__ long long acc[];   // [A][3 << shift] fixed point (or float in the same space)
    constexpr int A = BIL ? 4 : 1;
    const uint32_t R = p.start[p.K];
    const uint32_t chunk = max(kChunkMin, (uint32_t)(((uint64_t)R + gridDim.x - 1) / gridDim.x));
    int chunk_log2 = 0;
    while ((1u << chunk_log2) < chunk) ++chunk_log2;
    const uint64_t lo64 = (uint64_t)blockIdx.x * chunk;
    if (lo64 >= R) return;
    const uint32_t lo = (uint32_t)lo64;
    const uint32_t hi = (uint32_t)(lo64 + chunk < R ? lo64 + chunk : R);
    const int b0 = (int)(RecT<BIL>::load(p.sorted, lo).key() >> p.shift);
    const int b1 = (int)(RecT<BIL>::load(p.sorted, hi - 1).key() >> p.shift);
    float* accf = (float*)acc;
    const int slab = 3 << p.shift;       // one accumulator's span in acc
    for (int b = b0; b <= b1; ++b) {
        const uint32_t s = max(lo, p.start[b]), e = min(hi, p.start[b + 1]);
        if (s >= e) continue;
        const int first = b << p.shift;
        const int n_tex = min(1 << p.shift, p.n_texels - first);
        const uint32_t mb = p.bmax[b];
        const bool fixed = mb < 0x7F800000u;   // finite
        int ex = 0;
        frexpf(__uint_as_float(mb), &ex);      // every |value| in the bucket < 2^ex
        const int S = 62 - chunk_log2 - ex;
        const double scale = ldexp(1.0, S), unscale = ldexp(1.0, -S);
        for (int a = 0; a < A; ++a)
            for (int k = threadIdx.x; k < 3 * n_tex; k += 256) {
                if (fixed) acc[a * slab + k] = 0;
                else accf[2 * (a * slab + k)] = 0.0f;
            }
        __syncthreads();
        for (uint32_t i = s + threadIdx.x; i < e; i += 1024) {
            RecT<BIL> r[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (i + 256 * j < e) r[j] = RecT<BIL>::load(p.sorted, i + 256 * j);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (i + 256 * j < e) {
                    const int k = 3 * (int)(r[j].key() - (uint32_t)first);
                    float w[A];
                    if (BIL) {
                        const float fx = r[j].a.y, fy = r[j].a.z;
                        w[0] = (1.0f - fx) * (1.0f - fy);
                        w[A > 1 ? 1 : 0] = fx * (1.0f - fy);
                        w[A > 2 ? 2 : 0] = (1.0f - fx) * fy;
                        w[A > 3 ? 3 : 0] = fx * fy;
                    } else {
                        w[0] = 1.0f;
                    }
#pragma unroll
                    for (int a = 0; a < A; ++a) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const float v = BIL ? w[a] * r[j].v(c) : r[j].v(c);
                            if (fixed) {
                                unsigned long long* ai = (unsigned long long*)acc;
                                atomicAdd(&ai[a * slab + k + c], (unsigned long long)__double2ll_rn((double)v * scale));
                            } else {
                                atomicAdd(&accf[2 * (a * slab + k + c)], v);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
        for (int a = 0; a < A; ++a) {
            float* g = BIL ? p.acc4 + ((size_t)a * p.n_texels + first) * 3 : p.g_env + 3 * (size_t)first;
            for (int k = threadIdx.x; k < 3 * n_tex; k += 256) {
                const float v = fixed ? (float)((double)acc[a * slab + k] * unscale) : accf[2 * (a * slab + k)];
                if (v != 0.0f) atomicAdd(g + k, v);
            }
        }
        __syncthreads();
    }
}

// Bilinear: g_env[i][j] += the four per-tap accumulators of the bases whose
// taps land on texel (i, j).  A base at extended row r (= i0 + 1) and column
// c puts tap 00 on (clamp(r - 1), c), tap 01 on (clamp(r - 1), c + 1 mod W),
// tap 10 on (clamp(r), c) and tap 11 on (clamp(r), c + 1 mod W).
__global__ __launch_bounds__(256) void gather_kernel(EnvScatter p) {
    const int64_t n = (int64_t)p.H * p.W;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= 3 * n) return;
    const int c3 = (int)(k % 3);
    const int64_t t = k / 3;
    const int i = (int)(t / p.W), j = (int)(t % p.W);
    const int jm = j == 0 ? p.W - 1 : j - 1;
    const int64_t X = (int64_t)(p.H + 1) * p.W;   // extended texels per accumulator
    auto at = [&](int a, int r, int c) { return p.acc4[((size_t)a * X + (size_t)r * p.W + c) * 3 + c3]; };
    float v = at(0, i + 1, j) + at(1, i + 1, jm) + at(2, i, j) + at(3, i, jm);
    if (i == 0) v += at(0, 0, j) + at(1, 0, jm);
    if (i == p.H - 1) v += at(2, p.H, j) + at(3, p.H, jm);
    // an atomic add: g_env is accumulated, and another call may add into it
    // concurrently (several views' backward passes on several streams)
    if (v != 0.0f) atomicAdd(p.g_env + k, v);
}

// workgroups of the accumulation: one per kChunkMin records of capacity, at
// most kGridMax; each takes an equal share of the records actually written
unsigned accumulate_grid(uint32_t cap) {
    const uint32_t g = (cap + kChunkMin - 1) / kChunkMin;
    return g < (uint32_t)kGridMax ? g : (unsigned)kGridMax;
}

}  // namespace

bool env_scatter_plan(int H, int W, int64_t n_tiles, uint32_t region, bool bil, EnvScatter& p) {
    // bilinear keys run over the extended grid of H + 1 rows; its four
    // fixed-point accumulators per texel need buckets of 1024 texels (96 KB)
    const int n_tex = bil ? (H + 1) * W : H * W;
    int shift = kMinShift;
    while (((int64_t)kMaxBuckets << shift) < n_tex) ++shift;   // <= kMaxShift for 4096 x 4096
    if (bil && shift > kMinShift) return false;
    p.bil = bil ? 1 : 0;
    p.H = H;
    p.W = W;
    p.shift = shift;
    p.K = (n_tex + (1 << shift) - 1) >> shift;
    p.n_texels = n_tex;
    p.n_tiles = n_tiles;
    p.region = region;
    p.cap = (uint32_t)(n_tiles * (int64_t)region);
    p.n_wg = tile_grid(n_tiles);
    return true;
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t env_scatter_bytes(const EnvScatter& p) {
    const size_t S = p.bil ? 2 : 1;
    return 2 * al256(sizeof(float4) * S * (size_t)p.cap) + al256(sizeof(uint32_t) * (size_t)p.n_tiles) +
           (p.bil ? al256(sizeof(float) * 12 * (size_t)p.n_texels) : 0) +
           2 * al256(sizeof(uint32_t) * (size_t)p.K) + al256(sizeof(uint32_t) * (size_t)(p.K + 1)) +
           al256(sizeof(uint32_t) * (size_t)p.K * (size_t)p.n_wg);
}

void env_scatter_carve(void* base, EnvScatter& p) {
    const size_t S = p.bil ? 2 : 1;
    char* c = (char*)base;
    p.rec = (float4*)c;
    c += al256(sizeof(float4) * S * (size_t)p.cap);
    p.sorted = (float4*)c;
    c += al256(sizeof(float4) * S * (size_t)p.cap);
    if (p.bil) {
        p.acc4 = (float*)c;
        c += al256(sizeof(float) * 12 * (size_t)p.n_texels);
    } else {
        p.acc4 = nullptr;
    }
    p.tile_count = (uint32_t*)c;
    c += al256(sizeof(uint32_t) * (size_t)p.n_tiles);
    p.cursor = (uint32_t*)c;
    c += al256(sizeof(uint32_t) * (size_t)p.K);
    p.start = (uint32_t*)c;
    c += al256(sizeof(uint32_t) * (size_t)(p.K + 1));
    p.bmax = (uint32_t*)c;
    c += al256(sizeof(uint32_t) * (size_t)p.K);
    p.wg_hist = (uint32_t*)c;
}

hipError_t launch_env_scatter_init(const EnvScatter& p, hipStream_t s) {
    hipLaunchKernelGGL(init_kernel, dim3(1), dim3(1024), 0, s, p);
    if (p.bil) {
        const int64_t n = 12 * (int64_t)p.n_texels;
        const int64_t g = (n + 255) / 256;
        hipLaunchKernelGGL(zero_acc4, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, s, p.acc4, n);
    }
    return hipGetLastError();
}

template <bool BIL>
static hipError_t launch_env_scatter_t(const EnvScatter& p, hipStream_t s) {
    constexpr int S = BIL ? 2 : 1;
    hipLaunchKernelGGL(hist_kernel<BIL>, dim3(p.n_wg), dim3(256), 0, s, p);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, p);
    const size_t lds_sc = sizeof(uint32_t) * (size_t)((3 * p.K + 3) & ~3) + sizeof(float4) * S * kBatch;
    if (lds_sc > 65536) {   // above the default dynamic LDS limit (large probes only)
        const hipError_t e = hipFuncSetAttribute((const void*)scatter_kernel<BIL>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_sc);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(scatter_kernel<BIL>, dim3(p.n_wg), dim3(256), lds_sc, s, p);
    const unsigned grid = accumulate_grid(p.cap);
    const size_t lds_acc = sizeof(long long) * (3u << p.shift) * (BIL ? 4 : 1);
    if (lds_acc > 65536) {   // above the default dynamic LDS limit
        const hipError_t e = hipFuncSetAttribute((const void*)accumulate_kernel<BIL>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_acc);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(accumulate_kernel<BIL>, dim3(grid), dim3(256), lds_acc, s, p);
    if (BIL) {
        const int64_t n = 3 * (int64_t)p.H * p.W;
        hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_env_scatter(const EnvScatter& p, hipStream_t s) {
    if (p.cap == 0) return hipSuccess;
    return p.bil ? launch_env_scatter_t<true>(p, s) : launch_env_scatter_t<false>(p, s);
}

}  // namespace mcdi
