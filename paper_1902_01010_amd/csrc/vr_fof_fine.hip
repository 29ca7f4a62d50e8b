// vr_fof_fine.hip -- 3D friends-of-friends with a two-level grid (Sec. 2.1,
// Eq. fof3d).
//
// Coarse cells have side S = 2^s >= ellx, so every link joins a cell to
// itself or to one of its 26 neighbours; each coarse cell is cut into fine
// cells of side f = 2^k with 3 (f-1)^2 < ellx^2, so all members of a fine cell
// are linked to each other and start out as one union-find tree.  Particles
// are sorted by (coarse cell in row-major order, fine cell), a dense table
// gives the start of every (y, z) row of coarse cells, and each fine cell is
// one thread that walks the fine cells of its own and the 13 following
// coarse cells.  Exact integer bounds on the squared distance between two
// fine-cell boxes skip far pairs and link pairs that are entirely within
// ellx without testing particles; only the remaining pairs test particle
// pairs, stopping at the first link.  Every decision compares an exact
// integer squared distance d2 with l2c = ceil(ell2): for an integer d2,
// d2 < ell2 exactly when d2 < l2c, so the integer test decides as the plain
// definition's FP64 test does.
#include "vr_grid.h"

namespace vr {
namespace {

struct FineGrid {
    int gb, s, k, b, lr, r;
    int nc;   // coarse cells per side
};

// Sort key of particle i: its fine-cell key (coarse cell in row-major order,
// then the fine cell inside it) above the particle's offsets inside its fine
// cell (3 k bits), which the sort carries along without ordering by them.
// With grid_bits <= 21 the whole key takes at most 63 bits.
__global__ void k_finekey(int64_t n, const uint32_t* __restrict__ qx, const uint32_t* __restrict__ qy,
                          const uint32_t* __restrict__ qz, FineGrid G, uint64_t* __restrict__ key,
                          uint32_t* __restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t x = qx[i], y = qy[i], z = qz[i];
    const uint64_t ck = ((uint64_t)(z >> G.s) << (2 * G.b)) | ((uint64_t)(y >> G.s) << G.b) | (uint64_t)(x >> G.s);
    const uint32_t m = (uint32_t)G.r - 1;
    const uint64_t sub = ((uint64_t)((z >> G.k) & m) << (2 * G.lr)) | ((uint64_t)((y >> G.k) & m) << G.lr) |
                         (uint64_t)((x >> G.k) & m);
    const uint32_t om = (1u << G.k) - 1u;
    const uint64_t off = ((uint64_t)(z & om) << (2 * G.k)) | ((uint64_t)(y & om) << G.k) | (uint64_t)(x & om);
    key[i] = (((ck << (3 * G.lr)) | sub) << (3 * G.k)) | off;
    idx[i] = (uint32_t)i;
}

// In place after the sort: the fine-cell key, and the coordinates rebuilt
// from it and the carried offsets (sequential, where a gather through the
// sorted order would fetch a cache line per coordinate).
__global__ void k_decode_q(int64_t n, FineGrid G, uint64_t* __restrict__ key, uint32_t* __restrict__ sx,
                           uint32_t* __restrict__ sy, uint32_t* __restrict__ sz) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint64_t e = key[p];
    const uint64_t kf = e >> (3 * G.k);
    const uint32_t om = (1u << G.k) - 1u;
    const uint32_t ox = (uint32_t)e & om, oy = (uint32_t)(e >> G.k) & om, oz = (uint32_t)(e >> (2 * G.k)) & om;
    const int lr3 = 3 * G.lr;
    const uint64_t ck = kf >> lr3;
    const uint32_t sub = (uint32_t)(kf & ((1ull << lr3) - 1));
    const uint32_t ncm = (uint32_t)G.nc - 1u, rm = (uint32_t)G.r - 1u;
    const uint32_t fx = (uint32_t)(ck & ncm) * (uint32_t)G.r + (sub & rm);
    const uint32_t fy = (uint32_t)((ck >> G.b) & ncm) * (uint32_t)G.r + ((sub >> G.lr) & rm);
    const uint32_t fz = (uint32_t)(ck >> (2 * G.b)) * (uint32_t)G.r + (sub >> (2 * G.lr));
    key[p] = kf;
    sx[p] = (fx << G.k) | ox;
    sy[p] = (fy << G.k) | oy;
    sz[p] = (fz << G.k) | oz;
}

__global__ void k_key_flags(int64_t n, const uint64_t* __restrict__ key, uint32_t* __restrict__ flag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) flag[p] = (p == 0 || key[p] != key[p - 1]) ? 1u : 0u;
}

__global__ void k_fine_starts(int64_t n, const uint64_t* __restrict__ key, const uint32_t* __restrict__ scan,
                              uint32_t* __restrict__ fine_start, uint32_t* __restrict__ fid, int* __restrict__ parent) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const bool start = (p == 0 || key[p] != key[p - 1]);
    const uint32_t f = start ? scan[p] : scan[p] - 1;
    fid[p] = f;
    if (start) fine_start[f] = (uint32_t)p;
    if (p == n - 1) fine_start[f + 1] = (uint32_t)n;
}

// every member of a fine cell starts in the tree of the cell's first member
__global__ void k_parent_init(int64_t n, const uint32_t* __restrict__ fid, const uint32_t* __restrict__ fine_start,
                              int* __restrict__ parent) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) parent[p] = (int)fine_start[fid[p]];
}

__device__ __forceinline__ uint32_t lower_bound_u64(const uint64_t* __restrict__ key, uint32_t lo, uint32_t hi,
                                                    uint64_t v) {
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (key[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// row_start[r] = first sorted position of coarse row r = z * nc + y
__global__ void k_rows(int64_t nrows, int64_t n, const uint64_t* __restrict__ key, int shift,
                       uint32_t* __restrict__ row_start) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > nrows) return;
    row_start[r] = r == nrows ? (uint32_t)n : lower_bound_u64(key, 0, (uint32_t)n, (uint64_t)r << shift);
}

// Coarse cells with at least DENSE_CC occupied fine cells (halo cores, where
// one thread would walk up to 14 x 64 candidate cells one memory round trip
// at a time) are linked by k_link_tile3 instead, a wavefront each.
constexpr uint32_t DENSE_CC = 48;
constexpr int TILE_R = 4;  // fine cells per coarse side where the tiles apply (r^3 <= 64 lanes)

// Number of occupied coarse cells before coarse cell `cell` (row-major
// index): the prefix count of its 64-cell word plus the occupancy bits
// below `cell` in that word (two independent loads).  Occupied cells are
// numbered in sorted order, so this is also the coarse index of `cell`
// when it is occupied.
__device__ __forceinline__ uint32_t coarse_rank(const uint64_t* __restrict__ occ, const uint32_t* __restrict__ pre,
                                                uint64_t cell) {
    const uint64_t w = cell >> 6;
    return pre[w] + (uint32_t)__popcll(occ[w] & ((1ull << (cell & 63)) - 1ull));
}

// One thread per fine cell A of the sparse coarse cells.  frec[F] holds
// fine cell F's key (two words), its first member and its end (bit 31 of
// the end: F lies in a dense coarse cell).  The fine cells of a run of
// coarse cells x0 .. x1 in one row are cfs[rank(x0)] .. cfs[rank(x1 + 1)] - 1.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_link_fine(int64_t nfine, const uint4* __restrict__ frec,
                                                   const uint32_t* __restrict__ sx, const uint32_t* __restrict__ sy,
                                                   const uint32_t* __restrict__ sz, FineGrid G, int64_t l2c,
                                                   int* parent, unsigned xchunk, const uint32_t* __restrict__ cfs,
                                                   const uint64_t* __restrict__ occ, const uint32_t* __restrict__ pre) {
    const int64_t A = (int64_t)xcd_swizzle(blockIdx.x, gridDim.x, xchunk) * blockDim.x + threadIdx.x;
    if (A >= nfine) return;
    const uint4 fa = frec[A];
    if (fa.w >> 31) return;  // dense coarse cell: linked by k_link_tile3
    const uint32_t a0 = fa.z, a1 = fa.w;
    const uint64_t ka = ((uint64_t)fa.y << 32) | fa.x;
    const int lr3 = 3 * G.lr;
    const int rm = G.r - 1, ncm = G.nc - 1;
    const uint64_t cka = ka >> lr3;
    const int cx = (int)(cka & ncm), cy = (int)((cka >> G.b) & ncm), cz = (int)(cka >> (2 * G.b));
    const uint32_t suba = (uint32_t)(ka & ((1ull << lr3) - 1));
    const int gax = cx * G.r + (int)(suba & rm);
    const int gay = cy * G.r + (int)((suba >> G.lr) & rm);
    const int gaz = cz * G.r + (int)(suba >> (2 * G.lr));
    const int fbits = G.gb - G.k;  // fine cells per side = 2^fbits
    const int64_t f = int64_t(1) << G.k;
    // candidate runs of coarse cells [r_lo, r_hi): the own row (x .. x+1,
    // from the fine cell after A) and the four following rows (x-1 .. x+1),
    // two runs a row (the second empty unless the run wraps round the box).
    // Every index is fixed at compile time, so the runs stay in registers,
    // and all rank loads are issued before any is used.
    constexpr int NRUN = 10;
    uint64_t r_lo[NRUN], r_hi[NRUN];
#pragma unroll
    for (int rr = 0; rr < 5; ++rr) {
        const int dz = rr >= 2 ? 1 : 0, dy = rr == 0 ? 0 : (rr == 1 ? 1 : rr - 3);
        const uint64_t row = (uint64_t)((cz + dz) & ncm) * (uint64_t)G.nc + (uint64_t)((cy + dy) & ncm);
        const uint64_t base = row * (uint64_t)G.nc;
        const int xa = rr == 0 ? cx : cx - 1, xb = cx + 1;
        if (xa < 0) {
            r_lo[2 * rr] = base + ncm; r_hi[2 * rr] = base + ncm + 1;
            r_lo[2 * rr + 1] = base; r_hi[2 * rr + 1] = base + xb + 1;
        } else if (xb > ncm) {
            r_lo[2 * rr] = base + xa; r_hi[2 * rr] = base + ncm + 1;
            r_lo[2 * rr + 1] = base; r_hi[2 * rr + 1] = base + 1;
        } else {
            r_lo[2 * rr] = base + xa; r_hi[2 * rr] = base + xb + 1;
            r_lo[2 * rr + 1] = 0; r_hi[2 * rr + 1] = 0;
        }
    }
    uint32_t c_lo[NRUN], c_hi[NRUN];
#pragma unroll
    for (int u = 0; u < NRUN; ++u) {
        c_lo[u] = c_hi[u] = 0;
        if (r_lo[u] < r_hi[u]) {
            c_lo[u] = coarse_rank(occ, pre, r_lo[u]);
            c_hi[u] = coarse_rank(occ, pre, r_hi[u]);
        }
    }
    uint32_t f_lo[NRUN], f_hi[NRUN];
#pragma unroll
    for (int u = 0; u < NRUN; ++u) {
        f_lo[u] = f_hi[u] = 0;
        if (c_lo[u] < c_hi[u]) {
            f_lo[u] = cfs[c_lo[u]];
            f_hi[u] = cfs[c_hi[u]];
        }
    }
    // A's root, refreshed only when B's differs: components only merge, so
    // roots once equal stay equal, and a stale root still lies on the path
    // to the current one
    int ra = uf_find(parent, (int)a0);
    for (int u = 0; u < NRUN; ++u) {
        // run u's fine cells, picked by value so the arrays stay in registers
        uint32_t B0 = 0, Bend = 0;
#pragma unroll
        for (int j = 0; j < NRUN; ++j)
            if (u == j) { B0 = f_lo[j]; Bend = f_hi[j]; }
        // the own coarse cell (in the own row's runs): only cells after A
        if (B0 <= (uint32_t)A && (uint32_t)A < Bend) B0 = (uint32_t)A + 1;
        for (; B0 < Bend; B0 += 2) {
            // two candidate records per round trip; the exact box bound
            // settles most of them without touching their members
            uint4 fr[2];
#pragma unroll
            for (int j = 0; j < 2; ++j)
                if (B0 + j < Bend) fr[j] = frec[B0 + j];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (B0 + j >= Bend) break;
                const uint64_t kb = ((uint64_t)fr[j].y << 32) | fr[j].x;
                const uint64_t ckb = kb >> lr3;
                const uint32_t subb = (uint32_t)(kb & ((1ull << lr3) - 1));
                const int gbx = (int)(ckb & ncm) * G.r + (int)(subb & rm);
                const int gby = (int)((ckb >> G.b) & ncm) * G.r + (int)((subb >> G.lr) & rm);
                const int gbz = (int)(ckb >> (2 * G.b)) * G.r + (int)(subb >> (2 * G.lr));
                const int64_t gx = abs(min_image(gbx - gax, fbits));
                const int64_t gy = abs(min_image(gby - gay, fbits));
                const int64_t gz = abs(min_image(gbz - gaz, fbits));
                // exact bounds of the squared distance between the two boxes
                const int64_t lx = gx ? (gx - 1) * f + 1 : 0, ly = gy ? (gy - 1) * f + 1 : 0,
                              lz = gz ? (gz - 1) * f + 1 : 0;
                if (lx * lx + ly * ly + lz * lz >= l2c) continue;
                const uint32_t b0 = fr[j].z, b1 = fr[j].w & 0x7fffffffu;
                const int pb = parent[b0];
                // b0's parent is A's (possibly stale) root: one component
                if (pb == ra) continue;
                const int rb = uf_find(parent, pb);
                if (rb == ra) continue;
                ra = uf_find(parent, ra);
                if (ra == rb) continue;
                const int64_t ux = (gx + 1) * f - 1, uy = (gy + 1) * f - 1, uz = (gz + 1) * f - 1;
                bool hit = ux * ux + uy * uy + uz * uz < l2c;
                for (uint32_t pp = a0; pp < a1 && !hit; ++pp) {
                    const int px = (int)sx[pp], py = (int)sy[pp], pz = (int)sz[pp];
                    for (uint32_t q = b0; q < b1; ++q) {
                        const int dx = min_image((int)sx[q] - px, G.gb);
                        const int dy = min_image((int)sy[q] - py, G.gb);
                        const int dz = min_image((int)sz[q] - pz, G.gb);
                        if ((int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz < l2c) {
                            hit = true;
                            break;
                        }
                    }
                }
                if (hit) uf_union(parent, ra, rb);
            }
        }
    }
}

// occupancy bits per 64-cell word (the scan turns them into the prefix
// counts of coarse_rank); the extra last word counts nothing
__global__ void k_occ_count(int64_t words, const uint64_t* __restrict__ occ, uint32_t* __restrict__ cnt) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w <= words) cnt[w] = w < words ? (uint32_t)__popcll(occ[w]) : 0u;
}

// fine-cell records for the sweep: key, first member, end | dense << 31
__global__ void k_frec(int64_t nfine, const uint32_t* __restrict__ fine_start, const uint64_t* __restrict__ key,
                       const uint32_t* __restrict__ cid, const uint32_t* __restrict__ cfs, int mark_dense,
                       uint4* __restrict__ frec) {
    const int64_t F = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (F >= nfine) return;
    const uint32_t b0 = fine_start[F], b1 = fine_start[F + 1];
    const uint64_t k = key[b0];
    uint32_t dense = 0;
    if (mark_dense) {
        const uint32_t c = cid[F];
        dense = cfs[c + 1] - cfs[c] >= DENSE_CC ? 1u : 0u;
    }
    frec[F] = make_uint4((uint32_t)k, (uint32_t)(k >> 32), b0, b1 | (dense << 31));
}

// coarse-cell starts among the fine cells: flag[F] = 1 where F opens a coarse cell
__global__ void k_coarse_flags(int64_t nfine, const uint32_t* __restrict__ fine_start,
                               const uint64_t* __restrict__ key, int lr3, uint32_t* __restrict__ flag) {
    const int64_t F = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (F >= nfine) return;
    flag[F] = (F == 0 || (key[fine_start[F]] >> lr3) != (key[fine_start[F - 1]] >> lr3)) ? 1u : 0u;
}

// after an exclusive scan of the flags in place: cid[F] = coarse index of F,
// cfs[c] = first fine cell of coarse cell c, cfs[ncoarse] = nfine
__global__ void k_coarse_starts(int64_t nfine, const uint32_t* __restrict__ fine_start,
                                const uint64_t* __restrict__ key, int lr3, uint32_t* __restrict__ cid,
                                uint32_t* __restrict__ cfs, unsigned long long* __restrict__ occ) {
    const int64_t F = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (F >= nfine) return;
    const uint64_t ck = key[fine_start[F]] >> lr3;
    const bool start = F == 0 || ck != (key[fine_start[F - 1]] >> lr3);
    const uint32_t c = start ? cid[F] : cid[F] - 1;
    cid[F] = c;
    if (start) {
        cfs[c] = (uint32_t)F;
        atomicOr(&occ[ck >> 6], 1ull << (ck & 63));
    }
    if (F == nfine - 1) cfs[c + 1] = (uint32_t)nfine;
}

__global__ void k_dense_cc(int64_t ncoarse, const uint32_t* __restrict__ cfs, int* __restrict__ count,
                           int32_t* __restrict__ list) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool take = c < ncoarse && cfs[c + 1] - cfs[c] >= DENSE_CC;
    wave_append(count, list, take, (int32_t)c);
}

// The root of a without path-halving stores: the staging of a tile walks the
// roots of all its candidates, which many tiles share, and stores there
// would make every tile write the same lines.
__device__ __forceinline__ int uf_root(const int* parent, int a) {
    int p = parent[a];
    while (p != a) {
        a = p;
        p = parent[a];
    }
    return a;
}

// One wavefront per dense coarse cell, a lane per fine cell A of it.  The
// candidate fine cells -- the coarse cell's own (numbered first; only those
// after A count), then those of its 13 forward neighbours -- are staged in
// LDS 64 at a time with their fine-grid coordinates, first member and
// union-find root as of staging.  A pass with no divergence marks, per lane,
// the candidates whose box lower bound may lie within ellx (the bound without
// its +1 terms, in small integers) and whose root is not the lane's; only the
// marked ones take the exact bound, the root refresh, the particle tests and
// the union.  Once a core has merged, its pairs are left out by the mask.
// It runs twice: first (certain = 1) only for pairs whose boxes lie wholly
// within ellx, which merges the cores without a particle test; then, after
// every such link of every tile, for the other pairs, whose particle tests
// are then needed only where the cores did not already join them.
__global__ __launch_bounds__(64) void k_link_tile3(const int32_t* __restrict__ dense, const uint32_t* __restrict__ cfs,
                                                   const uint32_t* __restrict__ fine_start,
                                                   const uint32_t* __restrict__ fid, const uint64_t* __restrict__ key,
                                                   const uint32_t* __restrict__ sx, const uint32_t* __restrict__ sy,
                                                   const uint32_t* __restrict__ sz,
                                                   const uint32_t* __restrict__ row_start, FineGrid G, int64_t l2c,
                                                   float tq, int* parent, unsigned xchunk, int certain) {
    __shared__ __align__(16) int cgx[64];
    __shared__ __align__(16) int cgy[64];
    __shared__ __align__(16) int cgz[64];
    __shared__ __align__(16) int crt[64];
    __shared__ uint32_t cb0[64], cb1[64], cF[64];
    const int lane = (int)threadIdx.x;
    const uint32_t c = (uint32_t)dense[xcd_swizzle(blockIdx.x, gridDim.x, xchunk)];
    const uint32_t fA0 = cfs[c], nA = cfs[c + 1] - fA0;  // DENSE_CC .. 64
    const bool valid = (uint32_t)lane < nA;
    const uint32_t A = fA0 + (valid ? (uint32_t)lane : 0u);
    const int lr3 = 3 * G.lr;
    const int rm = G.r - 1, ncm = G.nc - 1;
    const int fbits = G.gb - G.k;  // fine cells per side = 2^fbits
    const int64_t f = int64_t(1) << G.k;
    const uint32_t a0 = fine_start[A], a1 = fine_start[A + 1];
    const uint64_t ka = key[a0];
    const uint64_t cka = ka >> lr3;
    const int cx = (int)(cka & ncm), cy = (int)((cka >> G.b) & ncm), cz = (int)(cka >> (2 * G.b));
    const uint32_t suba = (uint32_t)(ka & ((1ull << lr3) - 1));
    const int gax = cx * G.r + (int)(suba & rm);
    const int gay = cy * G.r + (int)((suba >> G.lr) & rm);
    const int gaz = cz * G.r + (int)(suba >> (2 * G.lr));
    // lane q < 14: segment q's fine cells -- the own coarse cell, then the
    // forward neighbours (+1, 0, 0), (-1..1, +1, 0), (-1..1, -1..1, +1)
    uint32_t seg_s = 0, seg_n = 0;
    if (lane == 0) {
        seg_s = fA0;
        seg_n = nA;
    } else if (lane < 14) {
        int dx, dy, dz;
        if (lane == 1) { dx = 1; dy = 0; dz = 0; }
        else if (lane < 5) { dx = lane - 3; dy = 1; dz = 0; }
        else { dx = (lane - 5) % 3 - 1; dy = (lane - 5) / 3 - 1; dz = 1; }
        const uint32_t row = (uint32_t)((cz + dz) & ncm) * (uint32_t)G.nc + (uint32_t)((cy + dy) & ncm);
        const uint64_t cell = (uint64_t)row * (uint64_t)G.nc + (uint64_t)((cx + dx) & ncm);
        const uint32_t rs = row_start[row], re = row_start[row + 1];
        const uint32_t lo = lower_bound_u64(key, rs, re, cell << lr3);
        const uint32_t hi = lower_bound_u64(key, lo, re, (cell + 1) << lr3);
        if (lo < hi) {
            seg_s = fid[lo];
            seg_n = fid[hi - 1] - seg_s + 1;
        }
    }
    uint32_t incl = seg_n;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    const uint32_t total = __shfl(incl, 13, 64);
    const uint32_t seg_b = incl - seg_n;
    // near the box faces a forward neighbour can lie across the periodic
    // boundary; elsewhere plain fine-cell differences are the minimum images
    const bool wrap = cx == 0 || cx == ncm || cy == 0 || cy == ncm || cz == ncm;
    int ra = valid ? uf_find(parent, (int)a0) : -1;
    for (uint32_t c0 = 0; c0 < total; c0 += 64) {
        const uint32_t cc = c0 + (uint32_t)lane;
        int sg = 0;
#pragma unroll
        for (int o = 1; o < 14; ++o) {
            const uint32_t bo = __shfl(seg_b, o, 64);
            if (bo <= cc) sg = o;
        }
        const uint32_t F = __shfl(seg_s, sg, 64) + (cc - __shfl(seg_b, sg, 64));
        __builtin_amdgcn_wave_barrier();
        if (cc < total) {
            const uint32_t b0 = fine_start[F], b1 = fine_start[F + 1];
            const uint64_t kb = key[b0];
            const uint64_t ckb = kb >> lr3;
            const uint32_t subb = (uint32_t)(kb & ((1ull << lr3) - 1));
            cgx[lane] = (int)(ckb & ncm) * G.r + (int)(subb & rm);
            cgy[lane] = (int)((ckb >> G.b) & ncm) * G.r + (int)((subb >> G.lr) & rm);
            cgz[lane] = (int)(ckb >> (2 * G.b)) * G.r + (int)(subb >> (2 * G.lr));
            cb0[lane] = b0;
            cb1[lane] = b1;
            cF[lane] = F;
            crt[lane] = uf_root(parent, (int)b0);
        }
        __builtin_amdgcn_wave_barrier();
        const int m = (int)min(64u, total - c0);
        if (!valid) continue;
        ra = uf_root(parent, ra);
        uint32_t tk[2] = {0u, 0u};
#pragma unroll
        for (int b4 = 0; b4 < 16; ++b4) {
            if (4 * b4 < m) {
                const int4 X = *reinterpret_cast<const int4*>(&cgx[4 * b4]);
                const int4 Y = *reinterpret_cast<const int4*>(&cgy[4 * b4]);
                const int4 Z = *reinterpret_cast<const int4*>(&cgz[4 * b4]);
                const int4 RT = *reinterpret_cast<const int4*>(&crt[4 * b4]);
                const int xs[4] = {X.x, X.y, X.z, X.w}, ys[4] = {Y.x, Y.y, Y.z, Y.w}, zs[4] = {Z.x, Z.y, Z.z, Z.w};
                const int rts[4] = {RT.x, RT.y, RT.z, RT.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    int dx = xs[u] - gax, dy = ys[u] - gay, dz = zs[u] - gaz;
                    if (wrap) {
                        dx = min_image(dx, fbits);
                        dy = min_image(dy, fbits);
                        dz = min_image(dz, fbits);
                    }
                    // candidates sit in adjacent coarse cells: |d| < 2 r
                    const int ex = max(abs(dx) - 1, 0), ey = max(abs(dy) - 1, 0), ez = max(abs(dz) - 1, 0);
                    const int bit = 4 * b4 + u;
                    if ((float)(ex * ex + ey * ey + ez * ez) < tq && rts[u] != ra) tk[bit >> 5] |= 1u << (bit & 31);
                }
            }
        }
        uint64_t take = ((uint64_t)tk[1] << 32) | tk[0];
        if (m < 64) take &= (uint64_t(1) << m) - 1;
        while (take) {
            const int j = __builtin_ctzll(take);
            take &= take - 1;
            if (c0 + (uint32_t)j < nA && cF[j] <= A) continue;  // own coarse cell: later cells only
            const int64_t gx = abs(min_image(cgx[j] - gax, fbits));
            const int64_t gy = abs(min_image(cgy[j] - gay, fbits));
            const int64_t gz = abs(min_image(cgz[j] - gaz, fbits));
            const int64_t lx = gx ? (gx - 1) * f + 1 : 0, ly = gy ? (gy - 1) * f + 1 : 0,
                          lz = gz ? (gz - 1) * f + 1 : 0;
            if (lx * lx + ly * ly + lz * lz >= l2c) continue;
            const int64_t ux = (gx + 1) * f - 1, uy = (gy + 1) * f - 1, uz = (gz + 1) * f - 1;
            const bool inside = ux * ux + uy * uy + uz * uz < l2c;
            if (inside != (certain != 0)) continue;
            int rb = crt[j];
            if (rb == ra) continue;
            rb = uf_find(parent, rb);
            if (rb == ra) continue;
            ra = uf_find(parent, ra);
            if (ra == rb) continue;
            bool hit = inside;
            const uint32_t q0 = cb0[j], q1 = cb1[j];
            for (uint32_t pp = a0; pp < a1 && !hit; ++pp) {
                const int px = (int)sx[pp], py = (int)sy[pp], pz = (int)sz[pp];
                for (uint32_t q = q0; q < q1; ++q) {
                    const int dx = min_image((int)sx[q] - px, G.gb);
                    const int dy = min_image((int)sy[q] - py, G.gb);
                    const int dz = min_image((int)sz[q] - pz, G.gb);
                    if ((int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz < l2c) {
                        hit = true;
                        break;
                    }
                }
            }
            if (hit) uf_union(parent, ra, rb);
        }
    }
}

__global__ void k_compress_f(int64_t n, int* parent) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int r = (int)p;
    while (parent[r] != r) r = parent[r];
    parent[p] = r;
}

// Smallest original index per component: every root first stores its own
// index (no atomics for the many singletons), then the other members lower
// it atomically.
__global__ void k_root_idx_f(int64_t n, const int* __restrict__ parent, const uint32_t* __restrict__ idx,
                             int* __restrict__ mn) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n && parent[p] == (int)p) mn[p] = (int)idx[p];
}

__global__ void k_min_orig_f(int64_t n, const int* __restrict__ parent, const uint32_t* __restrict__ idx,
                             int* __restrict__ mn) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < n && parent[p] != (int)p;
    wave_atomic_min(mn, valid ? parent[p] : 0, valid ? (int)idx[p] : 0x7FFFFFFF, valid);
}

__global__ void k_label_f(int64_t n, const int* __restrict__ parent, const uint32_t* __restrict__ idx,
                          const int* __restrict__ mn, int32_t* __restrict__ label) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) label[idx[p]] = mn[parent[p]];
}

}  // namespace

bool fof3d_fine_applicable(int gb, int s) {
    const int b = gb - s;
    return b >= 2 && b <= 12;  // 4 .. 4096 coarse cells a side
}

int fof3d_fine(vr_ctx* ctx, const vr_particles* p, double ell2, int s, int32_t* label, hipStream_t st) {
    const int64_t n = p->n;
    FineGrid G;
    G.gb = p->grid_bits;
    G.s = s;
    int k = 0;
    while (k + 1 <= s && 3.0 * (double)((int64_t(2) << k) - 1) * (double)((int64_t(2) << k) - 1) < ell2) ++k;
    G.k = k;
    G.b = G.gb - s;
    G.lr = s - k;
    G.r = 1 << G.lr;
    G.nc = 1 << G.b;
    const int key_bits = 3 * (G.gb - k);
    const int64_t nrows = (int64_t)G.nc * G.nc;
    VR_WS(key, ctx, uint64_t, WS_A0, n);
    VR_WS(idx, ctx, uint32_t, WS_A1, n);
    VR_WS(sx, ctx, uint32_t, WS_A2, n);
    VR_WS(sy, ctx, uint32_t, WS_A3, n);
    VR_WS(sz, ctx, uint32_t, WS_A4, n);
    VR_WS(scan, ctx, uint32_t, WS_A5, n);
    VR_WS(fine_start, ctx, uint32_t, WS_A6, n + 1);
    VR_WS(fid, ctx, uint32_t, WS_A7, n);
    VR_WS(row_start, ctx, uint32_t, WS_A8, nrows + 1);
    VR_WS(parent, ctx, int, WS_B0, n);
    VR_WS(mn, ctx, int, WS_B1, n);
    VR_WS(tot, ctx, uint32_t, WS_FLAG, 4);
    const unsigned gn = grid_for(n, 256);
    uint64_t* kin;
    uint32_t* iin;
    const int off_bits = 3 * k;
    int rc = sort_input_u64(ctx, key, idx, n, off_bits + key_bits, &kin, &iin, off_bits);
    if (rc) return rc;
    hipLaunchKernelGGL(k_finekey, dim3(gn), dim3(256), 0, st, n, p->qx, p->qy, p->qz, G, kin, iin);
    VR_LAUNCH_CHECK(ctx);
    if ((rc = sort_pairs_u64_from(ctx, kin, iin, key, idx, n, off_bits + key_bits, st, off_bits))) return rc;
    hipLaunchKernelGGL(k_decode_q, dim3(gn), dim3(256), 0, st, n, G, key, sx, sy, sz);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_key_flags, dim3(gn), dim3(256), 0, st, n, key, scan);
    VR_LAUNCH_CHECK(ctx);
    if ((rc = scan_u32(ctx, scan, scan, n, tot, st))) return rc;
    hipLaunchKernelGGL(k_fine_starts, dim3(gn), dim3(256), 0, st, n, key, scan, fine_start, fid, parent);
    VR_LAUNCH_CHECK(ctx);
    uint32_t nfine = 0;
    if ((rc = read_back(ctx, tot, &nfine, sizeof nfine, st))) return rc;
    hipLaunchKernelGGL(k_parent_init, dim3(gn), dim3(256), 0, st, n, fid, fine_start, parent);
    VR_LAUNCH_CHECK(ctx);
    // coarse index per fine cell, first fine cell per coarse cell, the
    // occupancy bit of every coarse cell with prefix counts per 64 cells
    // (nc^3 / 8 + nc^3 / 16 bytes), the dense coarse cells (fine grids of 4
    // a side), and one record per fine cell for the sweep
    const uint64_t ncell3 = (uint64_t)G.nc * (uint64_t)G.nc * (uint64_t)G.nc;
    const int64_t owords = (int64_t)(ncell3 >> 6) + 1;  // nc >= 4: ncell3 is a multiple of 64
    uint32_t* cid = scan;  // the fine-start flags are no longer needed
    VR_WS(cfs, ctx, uint32_t, WS_B2, (int64_t)nfine + 1);
    VR_WS(occ, ctx, unsigned long long, WS_B4, owords);
    VR_WS(pre, ctx, uint32_t, WS_B5, owords + 1);
    VR_WS(frec, ctx, uint4, WS_B6, (int64_t)nfine);
    if ((rc = fill_u32(ctx, reinterpret_cast<uint32_t*>(occ), 0u, 2 * owords, st))) return rc;
    const unsigned gf = grid_for(nfine, 256);
    hipLaunchKernelGGL(k_coarse_flags, dim3(gf), dim3(256), 0, st, (int64_t)nfine, fine_start, key, 3 * G.lr, cid);
    VR_LAUNCH_CHECK(ctx);
    if ((rc = scan_u32(ctx, cid, cid, nfine, tot, st))) return rc;
    uint32_t ncoarse = 0;
    if ((rc = read_back(ctx, tot, &ncoarse, sizeof ncoarse, st))) return rc;
    hipLaunchKernelGGL(k_coarse_starts, dim3(gf), dim3(256), 0, st, (int64_t)nfine, fine_start, key, 3 * G.lr, cid,
                       cfs, occ);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_occ_count, dim3(grid_for(owords, 256)), dim3(256), 0, st, owords - 1,
                       reinterpret_cast<const uint64_t*>(occ), pre);
    VR_LAUNCH_CHECK(ctx);
    if ((rc = scan_u32(ctx, pre, pre, owords, nullptr, st))) return rc;
    int32_t* dense = nullptr;
    int ndense = 0;
    if (G.r == TILE_R) {
        VR_WS(dense_w, ctx, int32_t, WS_B3, (int64_t)nfine + 1);
        VR_WS(cnt, ctx, int, WS_FLAG2, 4);
        if ((rc = fill_i32(ctx, cnt, 0, 1, st))) return rc;
        hipLaunchKernelGGL(k_dense_cc, dim3(grid_for(ncoarse, 256)), dim3(256), 0, st, (int64_t)ncoarse, cfs, cnt,
                           dense_w);
        VR_LAUNCH_CHECK(ctx);
        if ((rc = read_back(ctx, cnt, &ndense, sizeof ndense, st))) return rc;
        if (ndense > 0) {
            dense = dense_w;
            // the tiles find their neighbour cells by row
            hipLaunchKernelGGL(k_rows, dim3(grid_for(nrows + 1, 256)), dim3(256), 0, st, nrows, n, key,
                               G.b + 3 * G.lr, row_start);
            VR_LAUNCH_CHECK(ctx);
        }
    }
    hipLaunchKernelGGL(k_frec, dim3(gf), dim3(256), 0, st, (int64_t)nfine, fine_start, key, cid, cfs,
                       ndense > 0 ? 1 : 0, frec);
    VR_LAUNCH_CHECK(ctx);
    // the tile mask keeps B where (f e)^2 summed < ell2 with e = |g| - 1:
    // e2 < ell2 / f^2, compared in FP32 against a threshold rounded up
    const double fk = std::ldexp(1.0, k);
    const float tq = (float)(ell2 / (fk * fk) * (1.0 + 1e-6)) + 1e-6f;
    const int64_t l2c = (int64_t)std::ceil(ell2);  // ell2 < 2^40: exact
#define VR_TILE3(CERTAIN)                                                                                        \
    VR_TIMED(ctx, "fof_link3d", st, 0,                                                                           \
             hipLaunchKernelGGL(k_link_tile3, dim3((unsigned)ndense), dim3(64), 0, st, dense, cfs, fine_start, fid, \
                                key, sx, sy, sz, row_start, G, l2c, tq, parent, (unsigned)ctx->xcd_chunk, CERTAIN)); \
    VR_LAUNCH_CHECK(ctx)
    if (ndense > 0) { VR_TILE3(1); }
    VR_TIMED(ctx, "fof_link3d", st, n,
             hipLaunchKernelGGL(k_link_fine, dim3(grid_for(nfine, 256)), dim3(256), 0, st, (int64_t)nfine, frec, sx,
                                sy, sz, G, l2c, parent, (unsigned)ctx->xcd_chunk, cfs,
                                reinterpret_cast<const uint64_t*>(occ), pre));
    VR_LAUNCH_CHECK(ctx);
    if (ndense > 0) { VR_TILE3(0); }
#undef VR_TILE3
    hipLaunchKernelGGL(k_compress_f, dim3(gn), dim3(256), 0, st, n, parent);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_root_idx_f, dim3(gn), dim3(256), 0, st, n, parent, idx, mn);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_min_orig_f, dim3(gn), dim3(256), 0, st, n, parent, idx, mn);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_label_f, dim3(gn), dim3(256), 0, st, n, parent, idx, mn, label);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

}  // namespace vr
