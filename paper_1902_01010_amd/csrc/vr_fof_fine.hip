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
// pairs, stopping at the first link.  Every decision uses the exact integer
// squared distance in FP64 against ell2, as the plain definition does.
#include "vr_grid.h"

namespace vr {
namespace {

struct FineGrid {
    int gb, s, k, b, lr, r;
    int nc;   // coarse cells per side
};

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
    key[i] = (ck << (3 * G.lr)) | sub;
    idx[i] = (uint32_t)i;
}

__global__ void k_gather_q(int64_t n, const uint32_t* __restrict__ idx, const uint32_t* __restrict__ qx,
                           const uint32_t* __restrict__ qy, const uint32_t* __restrict__ qz, uint32_t* __restrict__ sx,
                           uint32_t* __restrict__ sy, uint32_t* __restrict__ sz) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t i = idx[p];
    sx[p] = qx[i];
    sy[p] = qy[i];
    sz[p] = qz[i];
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

__global__ __launch_bounds__(256) void k_link_fine(int64_t nfine, const uint32_t* __restrict__ fine_start,
                                                   const uint32_t* __restrict__ fid, const uint64_t* __restrict__ key,
                                                   const uint32_t* __restrict__ sx, const uint32_t* __restrict__ sy,
                                                   const uint32_t* __restrict__ sz,
                                                   const uint32_t* __restrict__ row_start, FineGrid G, double ell2,
                                                   int* parent, unsigned xchunk) {
    const int64_t A = (int64_t)xcd_swizzle(blockIdx.x, gridDim.x, xchunk) * blockDim.x + threadIdx.x;
    if (A >= nfine) return;
    const uint32_t a0 = fine_start[A], a1 = fine_start[A + 1];
    const uint64_t ka = key[a0];
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
    // the own row (x and x+1) and the four following rows (x-1 .. x+1)
    const int rdz[5] = {0, 0, 1, 1, 1}, rdy[5] = {0, 1, -1, 0, 1};
    // A's root, refreshed only when B's differs: components only merge, so
    // roots once equal stay equal, and a stale root still lies on the path
    // to the current one
    int ra = uf_find(parent, (int)a0);
    for (int rr = 0; rr < 5; ++rr) {
        const int nz = (cz + rdz[rr]) & ncm, ny = (cy + rdy[rr]) & ncm;
        const uint32_t row = (uint32_t)nz * (uint32_t)G.nc + (uint32_t)ny;
        const uint32_t rs = row_start[row], re = row_start[row + 1];
        if (rs == re) continue;
        const int xa = rr == 0 ? cx : cx - 1, xb = cx + 1;
        int px0[2], px1[2], np = 0;
        if (xa < 0) { px0[np] = G.nc - 1; px1[np++] = G.nc - 1; px0[np] = 0; px1[np++] = xb; }
        else if (xb > ncm) { px0[np] = xa; px1[np++] = ncm; px0[np] = 0; px1[np++] = 0; }
        else { px0[np] = xa; px1[np++] = xb; }
        for (int pc = 0; pc < np; ++pc) {
            const uint64_t base = (uint64_t)row * (uint64_t)G.nc;
            const uint32_t lo = lower_bound_u64(key, rs, re, (base + (uint64_t)px0[pc]) << lr3);
            const uint32_t hi = lower_bound_u64(key, lo, re, (base + (uint64_t)px1[pc] + 1) << lr3);
            if (lo >= hi) continue;
            uint32_t fb0 = fid[lo];
            const uint32_t fb1 = fid[hi - 1];
            if (rr == 0 && px0[pc] == cx && fb0 <= (uint32_t)A) fb0 = (uint32_t)A + 1;  // own coarse cell: later cells
            if (fb0 > fb1) continue;
            // B's first member, key and parent, and the next cell's start are
            // all loaded at the top of an iteration, with no load waiting for
            // another: one memory round trip per candidate cell that the
            // exact box bound or the parent test settles
            uint32_t next_b0 = fine_start[fb0];
            for (uint32_t B = fb0; B <= fb1; ++B) {
                const uint32_t b0 = next_b0, b1 = fine_start[B + 1];
                next_b0 = b1;
                const uint64_t kb = key[b0];
                const int pb = parent[b0];
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
                const double dmin = (double)(lx * lx + ly * ly + lz * lz);
                if (dmin >= ell2) continue;
                // b0's parent is A's (possibly stale) root: one component
                if (pb == ra) continue;
                const int rb = uf_find(parent, pb);
                if (rb == ra) continue;
                ra = uf_find(parent, ra);
                if (ra == rb) continue;
                const int64_t ux = (gx + 1) * f - 1, uy = (gy + 1) * f - 1, uz = (gz + 1) * f - 1;
                const double dmax = (double)(ux * ux + uy * uy + uz * uz);
                bool hit = dmax < ell2;
                for (uint32_t pp = a0; pp < a1 && !hit; ++pp) {
                    const int px = (int)sx[pp], py = (int)sy[pp], pz = (int)sz[pp];
                    for (uint32_t q = b0; q < b1; ++q) {
                        const int dx = min_image((int)sx[q] - px, G.gb);
                        const int dy = min_image((int)sy[q] - py, G.gb);
                        const int dz = min_image((int)sz[q] - pz, G.gb);
                        const double d2 = (double)dx * dx + (double)dy * dy + (double)dz * dz;
                        if (d2 < ell2) { hit = true; break; }
                    }
                }
                if (hit) uf_union(parent, ra, rb);
            }
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
    hipLaunchKernelGGL(k_finekey, dim3(gn), dim3(256), 0, st, n, p->qx, p->qy, p->qz, G, key, idx);
    VR_LAUNCH_CHECK(ctx);
    int rc = sort_pairs_u64(ctx, key, idx, n, key_bits, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_gather_q, dim3(gn), dim3(256), 0, st, n, idx, p->qx, p->qy, p->qz, sx, sy, sz);
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
    hipLaunchKernelGGL(k_rows, dim3(grid_for(nrows + 1, 256)), dim3(256), 0, st, nrows, n, key, G.b + 3 * G.lr,
                       row_start);
    VR_LAUNCH_CHECK(ctx);
    VR_TIMED(ctx, "fof_link3d", st, n,
             hipLaunchKernelGGL(k_link_fine, dim3(grid_for(nfine, 256)), dim3(256), 0, st, (int64_t)nfine, fine_start,
                                fid, key, sx, sy, sz, row_start, G, ell2, parent, (unsigned)ctx->xcd_chunk));
    VR_LAUNCH_CHECK(ctx);
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
