// vr_grid.h -- integer-grid cell lists and lock-free union-find shared by
// the 3D and 6D friends-of-friends kernels.
#pragma once
#include "vr_internal.h"

namespace vr {

// Cell keys hold z, y, x cell coordinates of b bits each (b up to 21).
using ckey_t = uint64_t;
constexpr ckey_t EMPTY = ~ckey_t(0);

__device__ __forceinline__ ckey_t cell_key(uint32_t x, uint32_t y, uint32_t z, int b) {
    return ((ckey_t)z << (2 * b)) | ((ckey_t)y << b) | (ckey_t)x;
}

__device__ __forceinline__ uint32_t hash_key(ckey_t k, uint32_t mask) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return (uint32_t)k & mask;
}

// Appends val for each taking lane: one atomic per wavefront.  Every lane of
// the wavefront must call it.
__device__ __forceinline__ void wave_append(int* counter, int32_t* list, bool take, int32_t val) {
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int lane = (int)lane_id();
    const int first = __builtin_ctzll(m);
    int base = 0;
    if (lane == first) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, first, 64);
    if (take) list[base + __popcll(m & ((1ull << lane) - 1ull))] = val;
}

__device__ __forceinline__ int hash_find(const ckey_t* __restrict__ hkeys, const uint32_t* __restrict__ hvals,
                                         uint32_t hmask, ckey_t k) {
    uint32_t h = hash_key(k, hmask);
    for (;;) {
        const ckey_t kk = hkeys[h];
        if (kk == k) return (int)hvals[h];
        if (kk == EMPTY) return -1;
        h = (h + 1) & hmask;
    }
}

__device__ __forceinline__ int uf_find(int* parent, int a) {
    int p = parent[a];
    while (p != a) {
        int g = parent[p];
        if (g != p) parent[a] = g;  // path halving; every write points closer to the root
        a = p;
        p = g;
    }
    return a;
}

__device__ __forceinline__ void uf_union(int* parent, int a, int b) {
    for (;;) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a > b) { int t = a; a = b; b = t; }
        int old = atomicCAS(&parent[b], b, a);
        if (old == b) return;
        b = old;
    }
}


// atomicMin(&base[key], val) for every valid lane.  When all valid lanes of
// the wavefront share one key (a dense component), the wave reduces first and
// issues a single atomic, which removes the contention on big components.
__device__ __forceinline__ void wave_atomic_min(int* base, int key, int val, bool valid) {
    const uint64_t act = __ballot(valid);
    if (act == 0) return;
    const int first = __ffsll((unsigned long long)act) - 1;
    const int k0 = __shfl(key, first, 64);
    if (__ballot(valid && key == k0) == act) {
        int v = valid ? val : 0x7FFFFFFF;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
        // values only decrease: a plain read that is already no larger
        // makes the atomic unnecessary (a stale read only costs the atomic)
        if ((int)__lane_id() == first && v < base[k0]) atomicMin(&base[k0], v);
    } else if (valid && val < base[key]) {
        atomicMin(&base[key], val);
    }
}

// Cell list of a point set on the periodic grid: sorted keys, sorted
// original indices, sorted coordinates, cell starts and an open-addressing
// hash from occupied cell keys to cell numbers.
struct CellList {
    ckey_t* key;
    uint32_t *idx, *sx, *sy, *sz, *cell_start;
    ckey_t* hkeys;
    uint32_t* hvals;
    uint32_t hmask;
    int64_t n_cells;
};

// 3D FOF on the two-level grid (coarse cells of side 2^s, fine cells whose
// members are all linked); applicable for 4 .. 4096 coarse cells a side.
bool fof3d_fine_applicable(int gb, int s);
int fof3d_fine(vr_ctx* ctx, const vr_particles* p, double ell2, int s, int32_t* label, hipStream_t st);

// Cell list of n points with cells of side 2^s grid units.  Uses workspace
// slots A0..A8, FLAG and the sort slots.
int build_cell_list(vr_ctx* ctx, int64_t n, const uint32_t* qx, const uint32_t* qy, const uint32_t* qz, int gb,
                    int s, CellList& cl, hipStream_t st);

}  // namespace vr
