// vr_prims.hip -- device-wide primitives: exclusive scan, stable LSD radix
// sort of (key, index) pairs, fills.  Written for wave64: ranks inside a
// wavefront come from 64-bit ballots, tiles are staged through LDS so that the
// scatter writes contiguous runs per digit.
#include "vr_internal.h"

namespace vr {
namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread (blockDim = 256).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* smem /*>= 4*/, uint32_t* total) {
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) smem[w] = inc;
    __syncthreads();
    uint32_t wpre = 0, tot = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        if (i < w) wpre += smem[i];
        tot += smem[i];
    }
    __syncthreads();
    if (total) *total = tot;
    return wpre + inc - v;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const uint32_t* in, int64_t n, uint32_t* part) {
    __shared__ uint32_t sm[8];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + j * SCAN_BLOCK + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_excl_scan(s, sm, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const uint32_t* in, uint32_t* out, int64_t n,
                                                           const uint32_t* part_scanned,
                                                           uint32_t* total_dev, int64_t nblocks,
                                                           const uint32_t* part_raw) {
    static_assert(SCAN_ITEMS == 8, "the vector path moves a lane's items as two 16-byte words");
    __shared__ uint32_t sm[8];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    // a full tile of 16-byte aligned arrays moves as two 16-byte words per
    // lane; a lane's eight 4-byte accesses 32 bytes apart ran at half the rate
    const bool vec = ((((uintptr_t)in) | ((uintptr_t)out)) & 15) == 0 && (int64_t)(blockIdx.x + 1) * SCAN_TILE <= n;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
    if (vec) {
        const uint4 a = reinterpret_cast<const uint4*>(in + base)[0];
        const uint4 b = reinterpret_cast<const uint4*>(in + base)[1];
        v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w, v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
    } else {
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            int64_t i = base + j;
            v[j] = (i < n) ? in[i] : 0u;
        }
    }
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) s += v[j];
    uint32_t off = block_excl_scan(s, sm, nullptr) + (part_scanned ? part_scanned[blockIdx.x] : 0u);
    if (vec) {
        uint32_t o[SCAN_ITEMS];
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            o[j] = off;
            off += v[j];
        }
        reinterpret_cast<uint4*>(out + base)[0] = make_uint4(o[0], o[1], o[2], o[3]);
        reinterpret_cast<uint4*>(out + base)[1] = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            int64_t i = base + j;
            if (i < n) out[i] = off;
            off += v[j];
        }
    }
    if (total_dev && blockIdx.x == nblocks - 1 && threadIdx.x == SCAN_BLOCK - 1)
        *total_dev = off;
    (void)part_raw;
}

// Byte-input scan (0/1 flags): a lane's eight bytes are one 8-byte word, so
// the flags cost a quarter of the traffic of a uint32 scan's input.
__device__ __forceinline__ uint32_t byte_sum(uint32_t x) {
    return (x & 255u) + ((x >> 8) & 255u) + ((x >> 16) & 255u) + (x >> 24);
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce_u8(const uint8_t* in, int64_t n, uint32_t* part) {
    __shared__ uint32_t sm[8];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
    if ((((uintptr_t)in) & 7) == 0 && base + SCAN_ITEMS <= n) {
        const uint2 w = *reinterpret_cast<const uint2*>(in + base);
        s = byte_sum(w.x) + byte_sum(w.y);
    } else {
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j)
            if (base + j < n) s += in[base + j];
    }
    uint32_t tot;
    block_excl_scan(s, sm, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply_u8(const uint8_t* in, uint32_t* out, int64_t n,
                                                              const uint32_t* part_scanned) {
    __shared__ uint32_t sm[8];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    const bool full = (int64_t)(blockIdx.x + 1) * SCAN_TILE <= n;
    uint32_t v[SCAN_ITEMS];
    if (full && (((uintptr_t)in) & 7) == 0) {
        const uint2 w = *reinterpret_cast<const uint2*>(in + base);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = (w.x >> (8 * j)) & 255u;
            v[4 + j] = (w.y >> (8 * j)) & 255u;
        }
    } else {
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) v[j] = base + j < n ? (uint32_t)in[base + j] : 0u;
    }
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) s += v[j];
    uint32_t off = block_excl_scan(s, sm, nullptr) + (part_scanned ? part_scanned[blockIdx.x] : 0u);
    uint32_t o[SCAN_ITEMS];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        o[j] = off;
        off += v[j];
    }
    if (full && (((uintptr_t)out) & 15) == 0) {
        reinterpret_cast<uint4*>(out + base)[0] = make_uint4(o[0], o[1], o[2], o[3]);
        reinterpret_cast<uint4*>(out + base)[1] = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j)
            if (base + j < n) out[base + j] = o[j];
    }
}

template <class T>
__global__ void k_fill(T* p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_iota(uint32_t* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (uint32_t)i;
}

// ---- radix sort ------------------------------------------------------------
constexpr int RS_BLOCK = 256;
constexpr int RS_WAVES = RS_BLOCK / 64;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_BLOCK * RS_ITEMS;   // 4096 keys per tile
constexpr int RS_RADIX = 256;

template <class K>
__global__ __launch_bounds__(RS_BLOCK) void k_radix_count(const K* keys, int64_t n, int shift,
                                                           uint32_t* hist, int num_tiles) {
    __shared__ uint32_t h[RS_RADIX];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
    for (int j = 0; j < RS_ITEMS; ++j) {
        int64_t i = base + j * RS_BLOCK + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * num_tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one 8-bit digit: every wavefront ranks its 16 x 64 keys
// by ballots, the block turns the per-wave digit counts into tile offsets,
// and the tile moves out through LDS in digit order -- the keys first, then
// the values through the same buffer, so the block needs LDS for one array
// of keys only (four blocks of 64-bit keys per CU).
template <class K>
__global__ __launch_bounds__(RS_BLOCK) void k_radix_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                             K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                             int64_t n, int shift,
                                                             const uint32_t* __restrict__ offs, int num_tiles) {
    __shared__ uint32_t wcnt[RS_WAVES][RS_RADIX];
    __shared__ uint32_t toff[RS_RADIX];
    __shared__ uint32_t goff[RS_RADIX];
    __shared__ uint32_t sm[8];
    __shared__ K lk[RS_TILE];
    uint32_t* lv = reinterpret_cast<uint32_t*>(lk);
    const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
    for (int i = tid; i < RS_WAVES * RS_RADIX; i += RS_BLOCK) (&wcnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t tbase = (int64_t)blockIdx.x * RS_TILE;
    const int64_t base = tbase + (int64_t)w * (RS_ITEMS * 64);
    K key[RS_ITEMS];
    uint32_t rank[RS_ITEMS];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int64_t i = base + j * 64 + lane;
        const bool valid = i < n;
        key[j] = valid ? kin[i] : K(0);
        const uint32_t d = (uint32_t)(key[j] >> shift) & 255u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        uint32_t before = 0;
        if (valid) before = wcnt[w][d];
        rank[j] = before + (uint32_t)__popcll(m & lt);
        // the highest peer lane publishes the new running count of the digit
        if (valid && lane == 63 - __clzll(m)) wcnt[w][d] = before + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // digit totals, per-wave prefixes and the tile-level exclusive offsets
    {
        const int d = tid;
        uint32_t run = 0;
#pragma unroll
        for (int ww = 0; ww < RS_WAVES; ++ww) {
            uint32_t c = wcnt[ww][d];
            wcnt[ww][d] = run;
            run += c;
        }
        uint32_t ex = block_excl_scan(run, sm, nullptr);
        toff[d] = ex;
        goff[d] = offs[(int64_t)d * num_tiles + blockIdx.x];
    }
    __syncthreads();
    // a key's place in the tile, in digit order
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int64_t i = base + j * 64 + lane;
        if (i < n) {
            const uint32_t d = (uint32_t)(key[j] >> shift) & 255u;
            rank[j] += toff[d] + wcnt[w][d];
            lk[rank[j]] = key[j];
        }
    }
    __syncthreads();
    const int cnt = (int)((n - tbase) < RS_TILE ? (n - tbase) : RS_TILE);
    uint32_t dst[RS_ITEMS];
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int i = tid + j * RS_BLOCK;
        if (i < cnt) {
            const K k = lk[i];
            const uint32_t d = (uint32_t)(k >> shift) & 255u;
            dst[j] = goff[d] + (uint32_t)i - toff[d];
            kout[dst[j]] = k;
        }
    }
    __syncthreads();
    // the values through the same buffer, to the places their keys went
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int64_t i = base + j * 64 + lane;
        if (i < n) lv[rank[j]] = vin[i];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int i = tid + j * RS_BLOCK;
        if (i < cnt) vout[dst[j]] = lv[i];
    }
}

template <class K>
int sort_input_impl(vr_ctx* ctx, K* keys, uint32_t* vals, int64_t n, int bits, K** kin, uint32_t** vin,
                    int first_bit = 0) {
    *kin = keys;
    *vin = vals;
    if (n <= 1 || bits <= first_bit || ((bits - first_bit + 7) / 8) % 2 == 0) return VR_OK;
    VR_WS(kalt, ctx, K, WS_SORT_KEYS_B, n);
    VR_WS(valt, ctx, uint32_t, WS_SORT_VALS_B, n);
    *kin = kalt;
    *vin = valt;
    return VR_OK;
}

// Input pairs in (kin, vin), which is either (keys, vals) or the alternate
// buffers; passes ping-pong between the two pairs, and the result is copied
// into (keys, vals) only where it ends in the other one.
template <class K>
int sort_pairs_impl(vr_ctx* ctx, K* kin, uint32_t* vin, K* keys, uint32_t* vals, int64_t n, int bits,
                    hipStream_t s, int first_bit = 0) {
    if (n <= 1 || bits <= first_bit) {
        if (n == 1 && kin != keys) {
            VR_HIP(ctx, hipMemcpyAsync(keys, kin, sizeof(K), hipMemcpyDeviceToDevice, s));
            VR_HIP(ctx, hipMemcpyAsync(vals, vin, sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        }
        return VR_OK;
    }
    const int num_tiles = (int)((n + RS_TILE - 1) / RS_TILE);
    VR_WS(kalt, ctx, K, WS_SORT_KEYS_B, n);
    VR_WS(valt, ctx, uint32_t, WS_SORT_VALS_B, n);
    VR_WS(hist, ctx, uint32_t, WS_SORT_HIST, (int64_t)RS_RADIX * num_tiles);
    if (kin != keys && (kin != kalt || vin != valt))
        return set_err(ctx, VR_ERR_INVALID_ARG, "sort input is neither the output nor the alternate buffers");
    K* k0 = kin; K* k1 = kin == keys ? kalt : keys;
    uint32_t* v0 = vin; uint32_t* v1 = vin == vals ? valt : vals;
    const int passes = (bits - first_bit + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = first_bit + p * 8;
        hipLaunchKernelGGL(k_radix_count<K>, dim3(num_tiles), dim3(RS_BLOCK), 0, s, k0, n, shift, hist,
                           num_tiles);
        VR_LAUNCH_CHECK(ctx);
        int rc = scan_u32(ctx, hist, hist, (int64_t)RS_RADIX * num_tiles, nullptr, s);
        if (rc) return rc;
        VR_TIMED(ctx, "radix_scatter", s, n,
                 hipLaunchKernelGGL(k_radix_scatter<K>, dim3(num_tiles), dim3(RS_BLOCK), 0, s, k0, v0, k1, v1, n,
                                    shift, hist, num_tiles));
        VR_LAUNCH_CHECK(ctx);
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    if (k0 != keys) {
        VR_HIP(ctx, hipMemcpyAsync(keys, k0, n * sizeof(K), hipMemcpyDeviceToDevice, s));
        VR_HIP(ctx, hipMemcpyAsync(vals, v0, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
    return VR_OK;
}

}  // namespace

int scan_u32(vr_ctx* ctx, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev, hipStream_t s) {
    if (n <= 0) {
        if (total_dev) return fill_u32(ctx, total_dev, 0u, 1, s);
        return VR_OK;
    }
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(SCAN_BLOCK), 0, s, in, out, n, nullptr, total_dev,
                           (int64_t)1, nullptr);
        VR_LAUNCH_CHECK(ctx);
        return VR_OK;
    }
    // partial sums live in a fresh region per recursion level
    static const int slots[2] = {WS_SCAN_TMP, WS_SCAN_TMP2};
    static thread_local int depth = 0;
    if (depth >= 2) return set_err(ctx, VR_ERR_UNSUPPORTED, "scan of %lld elements too deep", (long long)n);
    uint32_t* part = wsT<uint32_t>(ctx, slots[depth], nb);
    if (!part) return VR_ERR_OUT_OF_MEMORY;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, part);
    VR_LAUNCH_CHECK(ctx);
    ++depth;
    int rc = scan_u32(ctx, part, part, nb, nullptr, s);
    --depth;
    if (rc) return rc;
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, out, n, part, total_dev,
                       nb, nullptr);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

int scan_u8(vr_ctx* ctx, const uint8_t* in, uint32_t* out, int64_t n, hipStream_t s) {
    if (n <= 0) return VR_OK;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_apply_u8, dim3(1), dim3(SCAN_BLOCK), 0, s, in, out, n, nullptr);
        VR_LAUNCH_CHECK(ctx);
        return VR_OK;
    }
    // the tile sums take the second scratch slot: scan_u32 below keeps its
    // own partials in the first, and needs the second only beyond
    // SCAN_TILE^2 tile sums
    if (nb > (int64_t)SCAN_TILE * SCAN_TILE)
        return set_err(ctx, VR_ERR_UNSUPPORTED, "byte scan of %lld elements too deep", (long long)n);
    uint32_t* part = wsT<uint32_t>(ctx, WS_SCAN_TMP2, nb);
    if (!part) return VR_ERR_OUT_OF_MEMORY;
    hipLaunchKernelGGL(k_scan_reduce_u8, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, part);
    VR_LAUNCH_CHECK(ctx);
    int rc = scan_u32(ctx, part, part, nb, nullptr, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_scan_apply_u8, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, out, n, part);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

int sort_pairs_u32(vr_ctx* ctx, uint32_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s) {
    return sort_pairs_impl<uint32_t>(ctx, keys, vals, keys, vals, n, bits, s);
}

int sort_pairs_u64(vr_ctx* ctx, uint64_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s) {
    return sort_pairs_impl<uint64_t>(ctx, keys, vals, keys, vals, n, bits, s);
}

int sort_input_u64(vr_ctx* ctx, uint64_t* keys, uint32_t* vals, int64_t n, int bits, uint64_t** kin,
                   uint32_t** vin, int first_bit) {
    return sort_input_impl<uint64_t>(ctx, keys, vals, n, bits, kin, vin, first_bit);
}

int sort_pairs_u64_from(vr_ctx* ctx, uint64_t* kin, uint32_t* vin, uint64_t* keys, uint32_t* vals, int64_t n,
                        int bits, hipStream_t s, int first_bit) {
    return sort_pairs_impl<uint64_t>(ctx, kin, vin, keys, vals, n, bits, s, first_bit);
}

int sort_input_u32(vr_ctx* ctx, uint32_t* keys, uint32_t* vals, int64_t n, int bits, uint32_t** kin,
                   uint32_t** vin) {
    return sort_input_impl<uint32_t>(ctx, keys, vals, n, bits, kin, vin);
}

int sort_pairs_u32_from(vr_ctx* ctx, uint32_t* kin, uint32_t* vin, uint32_t* keys, uint32_t* vals, int64_t n,
                        int bits, hipStream_t s) {
    return sort_pairs_impl<uint32_t>(ctx, kin, vin, keys, vals, n, bits, s);
}

int fill_i32(vr_ctx* ctx, int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return VR_OK;
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

int fill_u32(vr_ctx* ctx, uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return VR_OK;
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

int iota_u32(vr_ctx* ctx, uint32_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return VR_OK;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

}  // namespace vr
