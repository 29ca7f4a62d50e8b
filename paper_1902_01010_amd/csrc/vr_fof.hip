// vr_fof.hip -- quantisation, integer-grid cell lists and 3D friends-of-
// friends (Sec. 2.1, Eq. fof3d), and group tables.
//
// Cell list: particles are keyed by the cell of side 2^s >= ellx (so every
// link lies in the same or an adjacent cell), sorted by a device radix sort,
// and cell -> [start, end) ranges are found through an open-addressing hash
// of the occupied cells.  Links are decided by the exact integer squared
// distance tested in FP64 against the squared linking length.  Components
// come from a lock-free union-find on sorted positions (hooking the larger
// root under the smaller), compressed by pointer jumping; the label is the
// smallest ORIGINAL index of each component.
#include "vr_grid.h"

namespace vr {
namespace {


__global__ void k_quantize(int64_t n, const float* __restrict__ x, const float* __restrict__ y,
                           const float* __restrict__ z, double scale, uint32_t mask,
                           uint32_t* __restrict__ qx, uint32_t* __restrict__ qy, uint32_t* __restrict__ qz) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    qx[i] = (uint32_t)((int64_t)floor((double)x[i] * scale)) & mask;
    qy[i] = (uint32_t)((int64_t)floor((double)y[i] * scale)) & mask;
    qz[i] = (uint32_t)((int64_t)floor((double)z[i] * scale)) & mask;
}

__global__ void k_cellkey(int64_t n, const uint32_t* __restrict__ qx, const uint32_t* __restrict__ qy,
                          const uint32_t* __restrict__ qz, int s, int b, ckey_t* __restrict__ key,
                          uint32_t* __restrict__ idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = cell_key(qx[i] >> s, qy[i] >> s, qz[i] >> s, b);
    idx[i] = (uint32_t)i;
}

__global__ void k_gather3(int64_t n, const uint32_t* __restrict__ idx, const uint32_t* __restrict__ qx,
                          const uint32_t* __restrict__ qy, const uint32_t* __restrict__ qz,
                          uint32_t* __restrict__ sx, uint32_t* __restrict__ sy, uint32_t* __restrict__ sz) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t i = idx[p];
    sx[p] = qx[i];
    sy[p] = qy[i];
    sz[p] = qz[i];
}

__global__ void k_cell_flags(int64_t n, const ckey_t* __restrict__ key, uint32_t* __restrict__ flag) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    flag[p] = (p == 0 || key[p] != key[p - 1]) ? 1u : 0u;
}

__global__ void k_cell_starts(int64_t n, const ckey_t* __restrict__ key, const uint32_t* __restrict__ scan,
                              uint32_t* __restrict__ cell_start, ckey_t* __restrict__ hkeys,
                              uint32_t* __restrict__ hvals, uint32_t hmask) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const bool start = (p == 0 || key[p] != key[p - 1]);
    // the exclusive scan counts starts before p: the last cell ends at n
    if (p == n - 1) cell_start[start ? scan[p] + 1 : scan[p]] = (uint32_t)n;
    if (start) {
        const uint32_t c = scan[p];
        cell_start[c] = (uint32_t)p;
        const ckey_t k = key[p];
        uint32_t h = hash_key(k, hmask);
        for (;;) {
            const ckey_t old = atomicCAS((unsigned long long*)&hkeys[h], (unsigned long long)EMPTY,
                                         (unsigned long long)k);
            if (old == EMPTY) { hvals[h] = c; break; }
            h = (h + 1) & hmask;
        }
    }
}

// One thread per sorted position.  Pairs are visited once: the own cell
// from p+1 on, plus the 13 neighbour cells that follow in (dz, dy, dx) order
// (when the grid has at least 3 cells per side), otherwise all 26 distinct
// neighbours with the partner restricted to later positions.
template <bool HALF>
__global__ __launch_bounds__(256) void k_link3d(int64_t n, const ckey_t* __restrict__ key,
                                                const uint32_t* __restrict__ sx, const uint32_t* __restrict__ sy,
                                                const uint32_t* __restrict__ sz, const uint32_t* __restrict__ cell_start,
                                                const ckey_t* __restrict__ hkeys, const uint32_t* __restrict__ hvals,
                                                uint32_t hmask, int b, int gb, double ell2, int* parent) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const ckey_t k = key[p];
    const int nc = 1 << b;
    const int cx = (int)(k & (nc - 1)), cy = (int)((k >> b) & (nc - 1)), cz = (int)(k >> (2 * b));
    const int px = (int)sx[p], py = (int)sy[p], pz = (int)sz[p];
    constexpr bool half = HALF;
    ckey_t seen[HALF ? 1 : 27];
    int nseen = 0;
    for (int o = 0; o < 27; ++o) {
        const int dz = o / 9 - 1, dy = (o / 3) % 3 - 1, dx = o % 3 - 1;
        const int lin = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
        if (half && lin < 13) continue;  // only the own cell (13) and the later half
        const uint32_t nx = (uint32_t)((cx + dx + nc) & (nc - 1));
        const uint32_t ny = (uint32_t)((cy + dy + nc) & (nc - 1));
        const uint32_t nz = (uint32_t)((cz + dz + nc) & (nc - 1));
        const ckey_t nk = cell_key(nx, ny, nz, b);
        if constexpr (!HALF) {
            bool dup = false;
            for (int t = 0; t < nseen; ++t) dup |= seen[t] == nk;
            if (dup) continue;
            seen[nseen++] = nk;
        }
        const int c = hash_find(hkeys, hvals, hmask, nk);
        if (c < 0) continue;
        uint32_t s = cell_start[c], e = cell_start[c + 1];
        const bool later_only = (nk == k) || !half;
        if (later_only && s <= (uint32_t)p) s = (uint32_t)p + 1;
        for (uint32_t q = s; q < e; ++q) {
            const int ddx = min_image((int)sx[q] - px, gb);
            const int ddy = min_image((int)sy[q] - py, gb);
            const int ddz = min_image((int)sz[q] - pz, gb);
            const double d2 = (double)ddx * ddx + (double)ddy * ddy + (double)ddz * ddz;
            if (d2 < ell2) uf_union(parent, (int)p, (int)q);
        }
    }
}

__global__ void k_iota_i32(int64_t n, int* p) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int)i;
}

__global__ void k_compress(int64_t n, int* parent) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int r = (int)p;
    while (parent[r] != r) r = parent[r];
    parent[p] = r;
}

__global__ void k_min_orig(int64_t n, const int* __restrict__ parent, const uint32_t* __restrict__ idx,
                           int* __restrict__ mn) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < n;
    wave_atomic_min(mn, valid ? parent[p] : 0, valid ? (int)idx[p] : 0x7FFFFFFF, valid);
}

__global__ void k_write_label(int64_t n, const int* __restrict__ parent, const uint32_t* __restrict__ idx,
                              const int* __restrict__ mn, int32_t* __restrict__ label) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    label[idx[p]] = mn[parent[p]];
}

// ---- groups -----------------------------------------------------------------
// The labelled particles (0 <= label < n) are compacted in index order and
// sorted with their particle indices by label (stable, so members of one
// label stay in index order); label runs become segments, kept segments are
// ordered by (size desc, label asc) and scattered into the member table.
// Unlabelled particles never enter the sort: their group_of is -1 at once.
__global__ void k_label_flags(int64_t n, const int32_t* __restrict__ label, uint8_t* __restrict__ flag,
                              int32_t* __restrict__ group_of) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int l = label[i];
    const bool has = l >= 0 && l < n;
    flag[i] = has ? 1 : 0;
    if (!has) group_of[i] = -1;
}

__global__ void k_label_total(int64_t n, const uint8_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                              uint32_t* __restrict__ total) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *total = pos[n - 1] + flag[n - 1];
}

__global__ void k_label_keys(int64_t n, const int32_t* __restrict__ label, const uint8_t* __restrict__ flag,
                             const uint32_t* __restrict__ pos, uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const uint32_t k = pos[i];
    key[k] = (uint32_t)label[i];
    val[k] = (uint32_t)i;
}

__global__ void k_run_flags(int64_t n, const uint32_t* __restrict__ key, uint32_t* __restrict__ flag) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) flag[p] = (p == 0 || key[p] != key[p - 1]) ? 1u : 0u;
}

__global__ void k_run_starts(int64_t n, const uint32_t* __restrict__ key, const uint32_t* __restrict__ scan,
                             uint32_t* __restrict__ run_start) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const bool start = (p == 0 || key[p] != key[p - 1]);
    if (start) run_start[scan[p]] = (uint32_t)p;
    if (p == n - 1) run_start[start ? scan[p] + 1 : scan[p]] = (uint32_t)n;
}

__global__ void k_run_keep(int64_t nrun, const uint32_t* __restrict__ run_start, int32_t n_min,
                           uint32_t* __restrict__ keep) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nrun) return;
    const uint32_t a = run_start[s], b = run_start[s + 1];
    keep[s] = b - a >= (uint32_t)n_min ? 1u : 0u;
}

__global__ void k_run_compact(int64_t nrun, int64_t n, const uint32_t* __restrict__ keep,
                              const uint32_t* __restrict__ pos, const uint32_t* __restrict__ run_start,
                              uint32_t* __restrict__ gkey, uint32_t* __restrict__ grun, int32_t* __restrict__ run_group) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nrun) return;
    run_group[s] = -1;
    if (!keep[s]) return;
    const uint32_t g = pos[s];
    gkey[g] = (uint32_t)n - (run_start[s + 1] - run_start[s]);  // ascending key = descending size
    grun[g] = (uint32_t)s;
}

__global__ void k_group_sizes(int64_t ng, const uint32_t* __restrict__ grun, const uint32_t* __restrict__ run_start,
                              uint32_t* __restrict__ gsize, int32_t* __restrict__ run_group) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g > ng) return;
    if (g == ng) { gsize[g] = 0; return; }
    const uint32_t s = grun[g];
    gsize[g] = run_start[s + 1] - run_start[s];
    run_group[s] = (int32_t)g;
}

__global__ void k_group_scatter(int64_t n, const uint32_t* __restrict__ runid, const uint32_t* __restrict__ run_start,
                                const int32_t* __restrict__ run_group, const uint32_t* __restrict__ goff,
                                const uint32_t* __restrict__ val, int32_t* __restrict__ group_of,
                                int32_t* __restrict__ members) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    // runid holds the exclusive scan of run starts: the run of p is the
    // number of starts up to and including p, minus one
    const uint32_t s0 = runid[p];
    const uint32_t s = (run_start[s0] == (uint32_t)p) ? s0 : s0 - 1;
    const int g = run_group[s];
    const uint32_t i = val[p];
    group_of[i] = g;
    if (g >= 0) members[goff[g] + ((uint32_t)p - run_start[s])] = (int32_t)i;
}

__global__ void k_u32_to_i32(int64_t n, const uint32_t* __restrict__ a, int32_t* __restrict__ b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (int32_t)a[i];
}

inline int bits_for(uint64_t v) {
    int b = 0;
    while ((uint64_t(1) << b) <= v && b < 63) ++b;
    return b;
}

}  // namespace

}  // namespace vr

using namespace vr;

extern "C" int vr_quantize(vr_ctx* ctx, int64_t n, const float* x, const float* y, const float* z,
                           double box, int32_t grid_bits, uint32_t* qx, uint32_t* qy, uint32_t* qz,
                           void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, VR_ERR_INVALID_ARG, "n out of range");
    if (grid_bits < 1 || grid_bits > 21) return set_err(ctx, VR_ERR_INVALID_ARG, "grid_bits not in 1..21");
    if (!(box > 0)) return set_err(ctx, VR_ERR_INVALID_ARG, "box must be positive");
    if (n == 0) return VR_OK;
    if (!x || !y || !z || !qx || !qy || !qz) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    const double scale = ldexp(1.0, grid_bits) / box;
    hipLaunchKernelGGL(k_quantize, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, n, x, y, z, scale,
                       (uint32_t)((1u << grid_bits) - 1u), qx, qy, qz);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

namespace vr {

// Build the cell list of n points (coordinates qx/qy/qz, grid bits gb) with
// cells of side 2^s.  Output arrays live in workspace slots A0..A7.
int build_cell_list(vr_ctx* ctx, int64_t n, const uint32_t* qx, const uint32_t* qy, const uint32_t* qz, int gb,
                    int s, CellList& cl, hipStream_t st) {
    const int b = gb - s;
    VR_WS(key, ctx, ckey_t, WS_A0, n);
    VR_WS(idx, ctx, uint32_t, WS_A1, n);
    VR_WS(sx, ctx, uint32_t, WS_A2, n);
    VR_WS(sy, ctx, uint32_t, WS_A3, n);
    VR_WS(sz, ctx, uint32_t, WS_A4, n);
    VR_WS(flag, ctx, uint32_t, WS_A5, n);
    VR_WS(cstart, ctx, uint32_t, WS_A6, n + 1);
    ckey_t* kin;
    uint32_t* iin;
    int rc = sort_input_u64(ctx, key, idx, n, 3 * b, &kin, &iin);
    if (rc) return rc;
    hipLaunchKernelGGL(k_cellkey, dim3(grid_for(n, 256)), dim3(256), 0, st, n, qx, qy, qz, s, b, kin, iin);
    VR_LAUNCH_CHECK(ctx);
    if ((rc = sort_pairs_u64_from(ctx, kin, iin, key, idx, n, 3 * b, st))) return rc;
    hipLaunchKernelGGL(k_gather3, dim3(grid_for(n, 256)), dim3(256), 0, st, n, idx, qx, qy, qz, sx, sy, sz);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_cell_flags, dim3(grid_for(n, 256)), dim3(256), 0, st, n, key, flag);
    VR_LAUNCH_CHECK(ctx);
    uint32_t* ncell_dev = (uint32_t*)ws(ctx, WS_FLAG, 64);
    if (!ncell_dev) return VR_ERR_OUT_OF_MEMORY;
    rc = scan_u32(ctx, flag, flag, n, ncell_dev, st);
    if (rc) return rc;
    uint32_t ncell = 0;
    rc = read_back(ctx, ncell_dev, &ncell, sizeof ncell, st);
    if (rc) return rc;
    uint32_t hsize = 1024;
    while (hsize < 2u * ncell) hsize <<= 1;
    VR_WS(hkeys, ctx, ckey_t, WS_A7, hsize);
    VR_WS(hvals, ctx, uint32_t, WS_A8, hsize);
    rc = fill_u32(ctx, reinterpret_cast<uint32_t*>(hkeys), 0xFFFFFFFFu, 2 * (int64_t)hsize, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_cell_starts, dim3(grid_for(n, 256)), dim3(256), 0, st, n, key, flag, cstart, hkeys, hvals,
                       hsize - 1);
    VR_LAUNCH_CHECK(ctx);
    cl = CellList{key, idx, sx, sy, sz, cstart, hkeys, hvals, hsize - 1, (int64_t)ncell};
    return VR_OK;
}

}  // namespace vr

extern "C" int vr_fof3d(vr_ctx* ctx, const vr_particles* p, double ellx, int32_t* label, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_particles(ctx, p, false);
    if (rc) return rc;
    const int gb = p->grid_bits;
    const double u = ellx * ldexp(1.0, gb) / p->box;
    if (!(u > 0) || !(u < ldexp(1.0, gb - 1)))
        return set_err(ctx, VR_ERR_INVALID_ARG, "ellx must satisfy 0 < ellx < box/2");
    const double ell2 = u * u;
    const int64_t n = p->n;
    if (n == 0) return VR_OK;
    if (!label) return set_err(ctx, VR_ERR_INVALID_ARG, "label is NULL");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    int s = 0;
    while ((double)(1 << s) < u && s < gb) ++s;
    if (fof3d_fine_applicable(gb, s)) return fof3d_fine(ctx, p, ell2, s, label, st);
    // very coarse grids (fewer than 4 cells a side): one level, all 27 neighbours
    CellList cl;
    rc = build_cell_list(ctx, n, p->qx, p->qy, p->qz, gb, s, cl, st);
    if (rc) return rc;
    VR_WS(parent, ctx, int, WS_B0, n);
    VR_WS(mn, ctx, int, WS_B1, n);
    hipLaunchKernelGGL(k_iota_i32, dim3(grid_for(n, 256)), dim3(256), 0, st, n, parent);
    VR_LAUNCH_CHECK(ctx);
    if ((1 << (gb - s)) >= 3)
        VR_TIMED(ctx, "fof_link3d", st, n,
                 hipLaunchKernelGGL(k_link3d<true>, dim3(grid_for(n, 256)), dim3(256), 0, st, n, cl.key, cl.sx,
                                    cl.sy, cl.sz, cl.cell_start, cl.hkeys, cl.hvals, cl.hmask, gb - s, gb, ell2,
                                    parent));
    else
        VR_TIMED(ctx, "fof_link3d", st, n,
                 hipLaunchKernelGGL(k_link3d<false>, dim3(grid_for(n, 256)), dim3(256), 0, st, n, cl.key, cl.sx,
                                    cl.sy, cl.sz, cl.cell_start, cl.hkeys, cl.hvals, cl.hmask, gb - s, gb, ell2,
                                    parent));
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_compress, dim3(grid_for(n, 256)), dim3(256), 0, st, n, parent);
    VR_LAUNCH_CHECK(ctx);
    rc = fill_i32(ctx, mn, 0x7FFFFFFF, n, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_min_orig, dim3(grid_for(n, 256)), dim3(256), 0, st, n, parent, cl.idx, mn);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_write_label, dim3(grid_for(n, 256)), dim3(256), 0, st, n, parent, cl.idx, mn, label);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

extern "C" int vr_groups(vr_ctx* ctx, int64_t n, const int32_t* label, int32_t n_min, int32_t* n_groups,
                         int32_t* group_of, int32_t* offsets, int32_t* members, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, VR_ERR_INVALID_ARG, "n out of range");
    if (n_min < 1) return set_err(ctx, VR_ERR_INVALID_ARG, "n_min must be >= 1");
    if (!n_groups) return set_err(ctx, VR_ERR_INVALID_ARG, "n_groups is NULL");
    *n_groups = 0;
    if (n > 0 && (!label || !group_of || !offsets || !members))
        return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) return VR_OK;
    VR_WS(key, ctx, uint32_t, WS_B2, n);
    VR_WS(val, ctx, uint32_t, WS_B3, n);
    VR_WS(runid, ctx, uint32_t, WS_B4, n);
    VR_WS(run_start, ctx, uint32_t, WS_B5, n + 1);
    VR_WS(keep, ctx, uint32_t, WS_B6, n);
    VR_WS(kpos, ctx, uint32_t, WS_B7, n);
    VR_WS(run_group, ctx, int32_t, WS_B8, n);
    VR_WS(tot, ctx, uint32_t, WS_FLAG, 4);
    // the labelled particles, compacted in index order: the byte flags live
    // in keep and their positions in runid until the runs need them
    uint8_t* flag = reinterpret_cast<uint8_t*>(keep);
    hipLaunchKernelGGL(k_label_flags, dim3(grid_for(n, 256)), dim3(256), 0, st, n, label, flag, group_of);
    VR_LAUNCH_CHECK(ctx);
    int rc = scan_u8(ctx, flag, runid, n, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_label_total, dim3(1), dim3(64), 0, st, n, flag, runid, tot);
    VR_LAUNCH_CHECK(ctx);
    // labels are below n; the compacted pairs go where the sort ends in place
    const int kbits = bits_for((uint64_t)(n - 1));
    uint32_t *kin = key, *vin = val;
    if ((rc = sort_input_u32(ctx, key, val, n, kbits, &kin, &vin))) return rc;
    hipLaunchKernelGGL(k_label_keys, dim3(grid_for(n, 256)), dim3(256), 0, st, n, label, flag, runid, kin, vin);
    VR_LAUNCH_CHECK(ctx);
    uint32_t m32 = 0;
    rc = read_back(ctx, tot, &m32, sizeof m32, st);
    if (rc) return rc;
    const int64_t m = m32;  // labelled particles
    uint32_t nrun = 0;
    if (m > 0) {
        rc = sort_pairs_u32_from(ctx, kin, vin, key, val, m, kbits, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_run_flags, dim3(grid_for(m, 256)), dim3(256), 0, st, m, key, runid);
        VR_LAUNCH_CHECK(ctx);
        rc = scan_u32(ctx, runid, runid, m, tot, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_run_starts, dim3(grid_for(m, 256)), dim3(256), 0, st, m, key, runid, run_start);
        VR_LAUNCH_CHECK(ctx);
        rc = read_back(ctx, tot, &nrun, sizeof nrun, st);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_run_keep, dim3(grid_for(nrun, 256)), dim3(256), 0, st, (int64_t)nrun, run_start, n_min,
                       keep);
    VR_LAUNCH_CHECK(ctx);
    uint32_t ng = 0;
    if (nrun > 0) {
        rc = scan_u32(ctx, keep, kpos, nrun, tot, st);
        if (rc) return rc;
        rc = read_back(ctx, tot, &ng, sizeof ng, st);
        if (rc) return rc;
    }
    *n_groups = (int32_t)ng;
    VR_WS(gkey, ctx, uint32_t, WS_B9, ng + 1);
    VR_WS(grun, ctx, uint32_t, WS_C0, ng + 1);
    VR_WS(gsize, ctx, uint32_t, WS_C1, ng + 1);
    hipLaunchKernelGGL(k_run_compact, dim3(grid_for(nrun, 256)), dim3(256), 0, st, (int64_t)nrun, n, keep, kpos,
                       run_start, gkey, grun, run_group);
    VR_LAUNCH_CHECK(ctx);
    if (ng > 0) {
        rc = sort_pairs_u32(ctx, gkey, grun, ng, bits_for((uint64_t)n), st);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_group_sizes, dim3(grid_for((int64_t)ng + 1, 256)), dim3(256), 0, st, (int64_t)ng, grun,
                       run_start, gsize, run_group);
    VR_LAUNCH_CHECK(ctx);
    rc = scan_u32(ctx, gsize, gsize, (int64_t)ng + 1, nullptr, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_u32_to_i32, dim3(grid_for((int64_t)ng + 1, 256)), dim3(256), 0, st, (int64_t)ng + 1, gsize,
                       offsets);
    VR_LAUNCH_CHECK(ctx);
    if (m > 0)
        hipLaunchKernelGGL(k_group_scatter, dim3(grid_for(m, 256)), dim3(256), 0, st, m, runid, run_start,
                           run_group, gsize, val, group_of, members);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}
