// vr_species.hip -- two particle species, the DM+Baryons mode (Sec. 2.1 and
// Sec. 2.4, Eq. baryondist).
//
// 3D FOF with dark-matter-seeded links: the dark matter is compacted and
// linked by the ordinary 3D FOF; then every baryon scans the 27 cells (of
// side >= ellx) of a cell list of the dark matter around it and is united,
// in one lock-free union-find over all particles seeded with the dark-matter
// components, with every dark-matter particle closer than ellx.  Baryons
// never test each other.  Union by smaller root keeps the smallest index of
// a component at its root.
//
// Baryon assignment: each baryon of a host looks for the host's dark matter
// nearest in phase space, D2 = d2 / ell2 + dv2 / sigma_v^2, on a cell list
// of the hosts' dark matter, ring by ring of cells around its own; once the
// nearest possible spatial term of the next ring exceeds the best D2 found,
// nothing further can tie or beat it.  A first pass on cells 8 times finer
// than ellx settles most baryons within two rings; the others search the
// ellx grid for up to 8 rings, then all the dark matter of their host.
#include "vr_grid.h"
#include "vr_kd.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace vr {
namespace {

__global__ void k_dm_flag(int64_t n, const uint8_t* __restrict__ isb, uint32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = isb[i] ? 0u : 1u;
}

__global__ void k_dm_compact(int64_t n, const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                             const uint32_t* __restrict__ qx, const uint32_t* __restrict__ qy,
                             const uint32_t* __restrict__ qz, uint32_t* __restrict__ cx, uint32_t* __restrict__ cy,
                             uint32_t* __restrict__ cz, int32_t* __restrict__ orig) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const uint32_t k = pos[i];
    cx[k] = qx[i];
    cy[k] = qy[i];
    cz[k] = qz[i];
    orig[k] = (int32_t)i;
}

// parent: every particle its own root, then each dark-matter particle under
// the smallest index of its dark-matter component
__global__ void k_iota_par(int64_t n, int* __restrict__ parent) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) parent[i] = (int)i;
}

__global__ void k_seed_dm(int64_t ndm, const int32_t* __restrict__ orig, const int32_t* __restrict__ labc,
                          int* __restrict__ parent) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < ndm) parent[orig[k]] = orig[labc[k]];
}

// The cells around a point: all 27 when the grid has 3 or more a side, else
// the distinct ones among them.
template <class F>
__device__ __forceinline__ void cells27(int px, int py, int pz, int s, int b, const uint32_t* __restrict__ hkeys,
                                        const uint32_t* __restrict__ hvals, uint32_t hmask, F&& visit) {
    const int nc = 1 << b;
    const int cx = px >> s, cy = py >> s, cz = pz >> s;
    uint32_t seen = 0;
    for (int o = 0; o < 27; ++o) {
        const int dz = o / 9 - 1, dy = (o / 3) % 3 - 1, dx = o % 3 - 1;
        const uint32_t nx = (uint32_t)((cx + dx + nc) & (nc - 1));
        const uint32_t ny = (uint32_t)((cy + dy + nc) & (nc - 1));
        const uint32_t nz = (uint32_t)((cz + dz + nc) & (nc - 1));
        if (nc < 3) {
            const uint32_t bit = 1u << (nx + 2 * ny + 4 * nz);
            if (seen & bit) continue;
            seen |= bit;
        }
        const int c = hash_find(hkeys, hvals, hmask, (nz << (2 * b)) | (ny << b) | nx);
        if (c >= 0) visit(c);
    }
}

// The dark-matter component (its smallest index) of every cell-list
// position, and per cell that component when all its members share it.
__global__ void k_cell_roots(int64_t ncell, const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ idx,
                             const int32_t* __restrict__ orig, const int32_t* __restrict__ labc,
                             int32_t* __restrict__ proot, int32_t* __restrict__ uroot) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int u = -2;
    for (uint32_t q = cstart[c]; q < cstart[c + 1]; ++q) {
        const int r = orig[labc[idx[q]]];
        proot[q] = r;
        u = u == -2 ? r : (u == r ? u : -1);
    }
    uroot[c] = u < 0 ? -1 : u;
}

// A baryon joins every dark-matter component with a member closer than
// ellx.  Components already joined (the last four) are not tested again,
// so in a dense core one member found near settles whole cells at once.
__global__ __launch_bounds__(256) void k_attach(int64_t n, const uint8_t* __restrict__ isb,
                                                const uint32_t* __restrict__ qx, const uint32_t* __restrict__ qy,
                                                const uint32_t* __restrict__ qz, CellList cl,
                                                const int32_t* __restrict__ proot, const int32_t* __restrict__ uroot,
                                                int s, int b, int gb, double ell2, int* parent) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !isb[i]) return;
    const int px = (int)qx[i], py = (int)qy[i], pz = (int)qz[i];
    int k0 = -1, k1 = -1, k2 = -1, k3 = -1;
    cells27(px, py, pz, s, b, cl.hkeys, cl.hvals, cl.hmask, [&](int c) {
        const int ur = uroot[c];
        if (ur >= 0 && (ur == k0 || ur == k1 || ur == k2 || ur == k3)) return;
        for (uint32_t q = cl.cell_start[c]; q < cl.cell_start[c + 1]; ++q) {
            const int r = proot[q];
            if (r == k0 || r == k1 || r == k2 || r == k3) continue;
            const int ddx = min_image((int)cl.sx[q] - px, gb);
            const int ddy = min_image((int)cl.sy[q] - py, gb);
            const int ddz = min_image((int)cl.sz[q] - pz, gb);
            const double d2 = (double)ddx * ddx + (double)ddy * ddy + (double)ddz * ddz;
            if (d2 < ell2) {
                uf_union(parent, (int)i, r);
                k3 = k2;
                k2 = k1;
                k1 = k0;
                k0 = r;
                if (ur >= 0) return;  // the cell holds this component only
            }
        }
    });
}

__global__ void k_roots(int64_t n, int* parent, int32_t* __restrict__ label) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) label[i] = uf_find(parent, (int)i);
}

// ---- baryon assignment -----------------------------------------------------
__global__ void k_member_host(const int32_t* __restrict__ off, int32_t* __restrict__ owner) {
    const int h = blockIdx.x;
    for (int k = off[h] + (int)threadIdx.x; k < off[h + 1]; k += blockDim.x) owner[k] = h;
}

__global__ void k_dm_members(int64_t M, const int32_t* __restrict__ mem, const uint8_t* __restrict__ isb,
                             uint32_t* __restrict__ flag) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < M) flag[k] = isb[mem[k]] ? 0u : 1u;
}

// compacted dark matter of the hosts, in host order: coordinates, particle
// index and host
__global__ void k_dm_member_compact(int64_t M, const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                                    const int32_t* __restrict__ mem, const int32_t* __restrict__ owner,
                                    const uint32_t* __restrict__ qx, const uint32_t* __restrict__ qy,
                                    const uint32_t* __restrict__ qz, uint32_t* __restrict__ cx,
                                    uint32_t* __restrict__ cy, uint32_t* __restrict__ cz, int32_t* __restrict__ dmi,
                                    int32_t* __restrict__ dmh) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M || !flag[k]) return;
    const uint32_t j = pos[k];
    const int i = mem[k];
    cx[j] = qx[i];
    cy[j] = qy[i];
    cz[j] = qz[i];
    dmi[j] = i;
    dmh[j] = owner[k];
}


// ---- a cell list with 64-bit cell keys (up to 2^21 cells a side) ----------
constexpr uint64_t EMPTY64 = ~0ull;

__device__ __forceinline__ uint64_t hash64(uint64_t k, uint64_t mask) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k & mask;
}

struct Grid64 {
    const uint64_t* hkeys;
    const uint32_t* hvals;
    uint64_t hmask;
    const uint32_t *cell_start, *idx, *sx, *sy, *sz;
    __device__ __forceinline__ int find(uint64_t k) const {
        uint64_t h = hash64(k, hmask);
        for (;;) {
            const uint64_t kk = hkeys[h];
            if (kk == k) return (int)hvals[h];
            if (kk == EMPTY64) return -1;
            h = (h + 1) & hmask;
        }
    }
};

__global__ void k_key64(int64_t n, const uint32_t* __restrict__ x, const uint32_t* __restrict__ y,
                        const uint32_t* __restrict__ z, int s, int b, uint64_t* __restrict__ key,
                        uint32_t* __restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = ((uint64_t)(z[i] >> s) << (2 * b)) | ((uint64_t)(y[i] >> s) << b) | (uint64_t)(x[i] >> s);
    idx[i] = (uint32_t)i;
}

__global__ void k_gather64(int64_t n, const uint32_t* __restrict__ idx, const uint32_t* __restrict__ x,
                           const uint32_t* __restrict__ y, const uint32_t* __restrict__ z, const uint64_t* __restrict__ key,
                           uint32_t* __restrict__ sx, uint32_t* __restrict__ sy, uint32_t* __restrict__ sz,
                           uint32_t* __restrict__ start) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t i = idx[p];
    sx[p] = x[i];
    sy[p] = y[i];
    sz[p] = z[i];
    start[p] = (p == 0 || key[p] != key[p - 1]) ? 1u : 0u;
}

__global__ void k_starts64(int64_t n, const uint64_t* __restrict__ key, const uint32_t* __restrict__ flag,
                           const uint32_t* __restrict__ scan, uint32_t* __restrict__ cell_start,
                           uint64_t* __restrict__ hkeys, uint32_t* __restrict__ hvals, uint64_t hmask) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const bool st = flag[p] != 0;
    if (p == n - 1) cell_start[st ? scan[p] + 1 : scan[p]] = (uint32_t)n;
    if (!st) return;
    const uint32_t c = scan[p];
    cell_start[c] = (uint32_t)p;
    const uint64_t k = key[p];
    uint64_t h = hash64(k, hmask);
    for (;;) {
        const unsigned long long old = atomicCAS((unsigned long long*)&hkeys[h], (unsigned long long)EMPTY64,
                                                 (unsigned long long)k);
        if (old == EMPTY64) {
            hvals[h] = c;
            return;
        }
        h = (h + 1) & hmask;
    }
}

struct Best {
    double d;
    int j;  // particle index of the dark matter, INT_MAX for none
};

__device__ __forceinline__ void consider(Best& bst, double D2, int j) {
    if (D2 < bst.d || (D2 == bst.d && j < bst.j)) {
        bst.d = D2;
        bst.j = j;
    }
}

__global__ __launch_bounds__(256) void k_assign(int64_t M, const int32_t* __restrict__ mem,
                                                const int32_t* __restrict__ owner, const uint8_t* __restrict__ isb,
                                                const int32_t* __restrict__ sub, const uint32_t* __restrict__ qx,
                                                const uint32_t* __restrict__ qy, const uint32_t* __restrict__ qz,
                                                const float* __restrict__ vx, const float* __restrict__ vy,
                                                const float* __restrict__ vz, Grid64 cl,
                                                const uint32_t* __restrict__ cx, const uint32_t* __restrict__ cy,
                                                const uint32_t* __restrict__ cz, const int32_t* __restrict__ dmi,
                                                const int32_t* __restrict__ dmh, const uint32_t* __restrict__ dm_off,
                                                int s, int b, int gb, double ell2, double sv2, int rmax,
                                                const uint8_t* __restrict__ todo_in, uint8_t* __restrict__ todo_out,
                                                int32_t* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    if (todo_in && !todo_in[k]) return;
    const int i = mem[k];
    if (!isb[i]) {
        out[i] = sub[i];
        if (todo_out) todo_out[k] = 0;
        return;
    }
    const int h = owner[k];
    const int px = (int)qx[i], py = (int)qy[i], pz = (int)qz[i];
    const double bx = (double)vx[i], by = (double)vy[i], bz = (double)vz[i];
    Best bst{INFINITY, 0x7FFFFFFF};
    // D2 = d2 / ell2 + dv2 / sigma_v^2 of the dark matter j at (x, y, z)
    auto test = [&](uint32_t x, uint32_t y, uint32_t z, int j) {
        const int ddx = min_image((int)x - px, gb);
        const int ddy = min_image((int)y - py, gb);
        const int ddz = min_image((int)z - pz, gb);
        const double d2 = (double)ddx * ddx + (double)ddy * ddy + (double)ddz * ddz;
        const double ax = bx - (double)vx[j], ay = by - (double)vy[j], az = bz - (double)vz[j];
        consider(bst, d2 / ell2 + (ax * ax + ay * ay + az * az) / sv2, j);
    };
    const int nc = 1 << b;
    const int ox = px >> s, oy = py >> s, oz = pz >> s;
    const double side = (double)(1 << s);
    // rings up to nc/2 - 1 never meet a cell twice; past rmax rings the
    // next pass (a coarser grid, or the host's whole list) takes over
    const int rlim = min(nc / 2 - 1, rmax);
    bool done = false;
    for (int r = 0; r <= rlim && !done; ++r) {
        for (int dz = -r; dz <= r; ++dz)
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    if (max(max(abs(dx), abs(dy)), abs(dz)) != r) continue;
                    const uint64_t nx = (uint64_t)((ox + dx + nc) & (nc - 1));
                    const uint64_t ny = (uint64_t)((oy + dy + nc) & (nc - 1));
                    const uint64_t nz = (uint64_t)((oz + dz + nc) & (nc - 1));
                    const int c = cl.find((nz << (2 * b)) | (ny << b) | nx);
                    if (c < 0) continue;
                    for (uint32_t q = cl.cell_start[c]; q < cl.cell_start[c + 1]; ++q) {
                        const uint32_t jc = cl.idx[q];
                        if (dmh[jc] == h) test(cl.sx[q], cl.sy[q], cl.sz[q], dmi[jc]);
                    }
                }
        // every point beyond ring r lies at least r cells away along an axis
        const double lim = (double)r * side;
        done = lim * lim / ell2 > bst.d;
    }
    if (!done && todo_out) {
        todo_out[k] = 1;  // left to the coarse pass
        return;
    }
    if (!done) {
        // a sparse host: all of its dark matter
        bst = Best{INFINITY, 0x7FFFFFFF};
        for (uint32_t jc = dm_off[h]; jc < dm_off[h + 1]; ++jc) test(cx[jc], cy[jc], cz[jc], dmi[jc]);
    }
    if (todo_out) todo_out[k] = 0;
    out[i] = bst.j == 0x7FFFFFFF ? -1 : sub[bst.j];
}

__global__ void k_dm_offsets(int n_hosts, int64_t M, const int32_t* __restrict__ off, const uint32_t* __restrict__ pos,
                             const uint32_t* __restrict__ total, uint32_t* __restrict__ dm_off) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h > n_hosts) return;
    dm_off[h] = (h == n_hosts || off[h] >= M) ? total[0] : pos[off[h]];
}


// ---- label utilities --------------------------------------------------------
__global__ void k_label_stats(int64_t n, const int32_t* __restrict__ label, int* __restrict__ cnt,
                              int* __restrict__ low, int* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int l = label[i];
    if (l < 0) return;
    if (l >= n) {
        atomicOr(bad, 1);
        return;
    }
    atomicAdd(&cnt[l], 1);
    atomicMin(&low[l], (int)i);
}

__global__ void k_label_min(int64_t n, const int32_t* __restrict__ label, const int* __restrict__ cnt,
                            const int* __restrict__ low, int min_size, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int l = label[i];
    out[i] = (l >= 0 && l < n && cnt[l] >= min_size) ? low[l] : -1;
}

__global__ void k_keep_flags(int64_t M, const int32_t* __restrict__ mem, const uint8_t* __restrict__ drop,
                             uint32_t* __restrict__ flag) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < M) flag[k] = drop[mem[k]] ? 0u : 1u;
}

__global__ void k_keep_scatter(int64_t M, const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                               const int32_t* __restrict__ mem, int32_t* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < M && flag[k]) out[pos[k]] = mem[k];
}

}  // namespace
}  // namespace vr

using namespace vr;

extern "C" int vr_fof3d_dm(vr_ctx* ctx, const vr_particles* p, double ellx, const uint8_t* is_baryon, int32_t* label,
                           void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_particles(ctx, p, false);
    if (rc) return rc;
    const int gb = p->grid_bits;
    const double u = ellx * ldexp(1.0, gb) / p->box;
    if (!(u > 0) || !(u < ldexp(1.0, gb - 1)))
        return set_err(ctx, VR_ERR_INVALID_ARG, "ellx must satisfy 0 < ellx < box/2");
    const int64_t n = p->n;
    if (n == 0) return VR_OK;
    if (!label || !is_baryon) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    VR_WS(flag, ctx, uint32_t, WS_C0, n);
    VR_WS(pos, ctx, uint32_t, WS_C1, n);
    VR_WS(tot, ctx, uint32_t, WS_C9, 4);
    hipLaunchKernelGGL(k_dm_flag, dim3(grid_for(n, 256)), dim3(256), 0, st, n, is_baryon, flag);
    VR_LAUNCH_CHECK(ctx);
    if ((rc = scan_u32(ctx, flag, pos, n, tot, st))) return rc;
    uint32_t ndm32 = 0;
    if ((rc = read_back(ctx, tot, &ndm32, sizeof ndm32, st))) return rc;
    const int64_t ndm = ndm32;
    VR_WS(parent, ctx, int, WS_D2, n);
    hipLaunchKernelGGL(k_iota_par, dim3(grid_for(n, 256)), dim3(256), 0, st, n, parent);
    VR_LAUNCH_CHECK(ctx);
    if (ndm > 0) {
        VR_WS(cx, ctx, uint32_t, WS_C2, ndm);
        VR_WS(cy, ctx, uint32_t, WS_C3, ndm);
        VR_WS(cz, ctx, uint32_t, WS_C4, ndm);
        VR_WS(orig, ctx, int32_t, WS_C5, ndm);
        VR_WS(labc, ctx, int32_t, WS_C6, ndm);
        hipLaunchKernelGGL(k_dm_compact, dim3(grid_for(n, 256)), dim3(256), 0, st, n, flag, pos, p->qx, p->qy, p->qz,
                           cx, cy, cz, orig);
        VR_LAUNCH_CHECK(ctx);
        // the dark matter alone, by the ordinary 3D FOF
        vr_particles pdm = *p;
        pdm.n = ndm;
        pdm.qx = cx;
        pdm.qy = cy;
        pdm.qz = cz;
        pdm.vx = pdm.vy = pdm.vz = nullptr;
        pdm.mass = nullptr;
        pdm.mass_value = 1.0;
        if ((rc = vr_fof3d(ctx, &pdm, ellx, labc, stream))) return rc;
        hipLaunchKernelGGL(k_seed_dm, dim3(grid_for(ndm, 256)), dim3(256), 0, st, ndm, orig, labc, parent);
        VR_LAUNCH_CHECK(ctx);
        if (ndm < n) {
            // baryons join every dark-matter particle within ellx
            int s = 0;
            while ((double)(1 << s) < u && s < gb) ++s;
            CellList cl;
            if ((rc = build_cell_list(ctx, ndm, cx, cy, cz, gb, s, cl, st))) return rc;
            VR_WS(proot, ctx, int32_t, WS_C7, ndm);
            VR_WS(uroot, ctx, int32_t, WS_C8, cl.n_cells + 1);
            hipLaunchKernelGGL(k_cell_roots, dim3(grid_for(cl.n_cells, 256)), dim3(256), 0, st, cl.n_cells,
                               cl.cell_start, cl.idx, orig, labc, proot, uroot);
            VR_LAUNCH_CHECK(ctx);
            VR_TIMED(ctx, "fof_attach", st, n - ndm,
                     hipLaunchKernelGGL(k_attach, dim3(grid_for(n, 256)), dim3(256), 0, st, n, is_baryon, p->qx,
                                        p->qy, p->qz, cl, proot, uroot, s, gb - s, gb, u * u, parent));
            VR_LAUNCH_CHECK(ctx);
        }
    }
    hipLaunchKernelGGL(k_roots, dim3(grid_for(n, 256)), dim3(256), 0, st, n, parent, label);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

namespace vr {
namespace {

// Cell list of n points (cells of side 2^s) with 64-bit keys, in workspace
// slots D2..D9 and the sort slots.
int build_grid64(vr_ctx* ctx, int64_t n, const uint32_t* x, const uint32_t* y, const uint32_t* z, int gb, int s,
                 Grid64& g, hipStream_t st) {
    const int b = gb - s;
    VR_WS(key, ctx, uint64_t, WS_D2, n);
    VR_WS(idx, ctx, uint32_t, WS_D3, n);
    VR_WS(sx, ctx, uint32_t, WS_D4, n);
    VR_WS(sy, ctx, uint32_t, WS_D5, n);
    VR_WS(sz, ctx, uint32_t, WS_D6, n);
    VR_WS(flag, ctx, uint32_t, WS_D7, n);
    VR_WS(cstart, ctx, uint32_t, WS_D8, n + 1);
    VR_WS(tot, ctx, uint32_t, WS_FLAG2, 4);
    hipLaunchKernelGGL(k_key64, dim3(grid_for(n, 256)), dim3(256), 0, st, n, x, y, z, s, b, key, idx);
    VR_LAUNCH_CHECK(ctx);
    int rc = sort_pairs_u64(ctx, key, idx, n, 3 * b, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_gather64, dim3(grid_for(n, 256)), dim3(256), 0, st, n, idx, x, y, z, key, sx, sy, sz, flag);
    VR_LAUNCH_CHECK(ctx);
    VR_WS(scan, ctx, uint32_t, WS_A0, n);
    if ((rc = scan_u32(ctx, flag, scan, n, tot, st))) return rc;
    uint32_t ncell = 0;
    if ((rc = read_back(ctx, tot, &ncell, sizeof ncell, st))) return rc;
    uint64_t hsize = 1024;
    while (hsize < 2ull * ncell) hsize <<= 1;
    VR_WS(hkeys, ctx, uint64_t, WS_D9, hsize);
    VR_WS(hvals, ctx, uint32_t, WS_A1, hsize);
    if ((rc = fill_u32(ctx, reinterpret_cast<uint32_t*>(hkeys), 0xFFFFFFFFu, 2 * (int64_t)hsize, st))) return rc;
    hipLaunchKernelGGL(k_starts64, dim3(grid_for(n, 256)), dim3(256), 0, st, n, key, flag, scan, cstart, hkeys, hvals,
                       hsize - 1);
    VR_LAUNCH_CHECK(ctx);
    g = Grid64{hkeys, hvals, hsize - 1, cstart, idx, sx, sy, sz};
    return VR_OK;
}

}  // namespace
}  // namespace vr

extern "C" int vr_assign_baryons(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts, const int32_t* host_offsets,
                                 const int32_t* host_members, const uint8_t* is_baryon, const int32_t* sub,
                                 double ellx, double sigma_v, int32_t* out, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_particles(ctx, p, true);
    if (rc) return rc;
    if ((rc = check_hosts(ctx, n_hosts, host_offsets, host_members))) return rc;
    const int gb = p->grid_bits;
    const double u = ellx * ldexp(1.0, gb) / p->box;
    if (!(u > 0) || !(u < ldexp(1.0, gb - 1)) || !(sigma_v > 0) || !std::isfinite(sigma_v))
        return set_err(ctx, VR_ERR_INVALID_ARG, "need 0 < ellx < box/2 and sigma_v > 0");
    if (n_hosts == 0) return VR_OK;
    if (!is_baryon || !sub || !out) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> off;
    if ((rc = read_host_offsets(ctx, n_hosts, host_offsets, p->n, 0, off, st))) return rc;
    const int64_t M = off[n_hosts];
    if (M == 0) return VR_OK;
    VR_WS(owner, ctx, int32_t, WS_C0, M);
    VR_WS(flag, ctx, uint32_t, WS_C1, M);
    VR_WS(pos, ctx, uint32_t, WS_C2, M);
    VR_WS(tot, ctx, uint32_t, WS_C9, 4);
    hipLaunchKernelGGL(k_member_host, dim3(n_hosts), dim3(256), 0, st, host_offsets, owner);
    hipLaunchKernelGGL(k_dm_members, dim3(grid_for(M, 256)), dim3(256), 0, st, M, host_members, is_baryon, flag);
    VR_LAUNCH_CHECK(ctx);
    if ((rc = scan_u32(ctx, flag, pos, M, tot, st))) return rc;
    uint32_t ndm32 = 0;
    if ((rc = read_back(ctx, tot, &ndm32, sizeof ndm32, st))) return rc;
    const int64_t ndm = ndm32;
    VR_WS(cx, ctx, uint32_t, WS_C3, ndm + 1);
    VR_WS(cy, ctx, uint32_t, WS_C4, ndm + 1);
    VR_WS(cz, ctx, uint32_t, WS_C5, ndm + 1);
    VR_WS(dmi, ctx, int32_t, WS_C6, ndm + 1);
    VR_WS(dmh, ctx, int32_t, WS_C7, ndm + 1);
    VR_WS(dm_off, ctx, uint32_t, WS_C8, n_hosts + 1);
    hipLaunchKernelGGL(k_dm_member_compact, dim3(grid_for(M, 256)), dim3(256), 0, st, M, flag, pos, host_members,
                       owner, p->qx, p->qy, p->qz, cx, cy, cz, dmi, dmh);
    hipLaunchKernelGGL(k_dm_offsets, dim3(grid_for(n_hosts + 1, 256)), dim3(256), 0, st, n_hosts, M, host_offsets,
                       pos, tot, dm_off);
    VR_LAUNCH_CHECK(ctx);
    int s = 0;
    while ((double)(1 << s) < u && s < gb) ++s;
    Grid64 cl{};
    if (ndm > 0) {
        // first pass on cells 8 times finer than ellx, two rings: enough where
        // the dark matter is dense; the rest go to the ellx grid
        const int sf = std::max(s - 3, 0);
        if ((rc = build_grid64(ctx, ndm, cx, cy, cz, gb, sf, cl, st))) return rc;
        VR_WS(todo, ctx, uint8_t, WS_D1, M);
        VR_TIMED(ctx, "assign_baryons", st, M - ndm,
                 hipLaunchKernelGGL(k_assign, dim3(grid_for(M, 256)), dim3(256), 0, st, M, host_members, owner,
                                    is_baryon, sub, p->qx, p->qy, p->qz, p->vx, p->vy, p->vz, cl, cx, cy, cz, dmi, dmh,
                                    dm_off, sf, gb - sf, gb, u * u, sigma_v * sigma_v, 2, nullptr, todo, out));
        VR_LAUNCH_CHECK(ctx);
        if ((rc = build_grid64(ctx, ndm, cx, cy, cz, gb, s, cl, st))) return rc;
        VR_TIMED(ctx, "assign_baryons", st, 0,
                 hipLaunchKernelGGL(k_assign, dim3(grid_for(M, 256)), dim3(256), 0, st, M, host_members, owner,
                                    is_baryon, sub, p->qx, p->qy, p->qz, p->vx, p->vy, p->vz, cl, cx, cy, cz, dmi, dmh,
                                    dm_off, s, gb - s, gb, u * u, sigma_v * sigma_v, 8, todo, nullptr, out));
        VR_LAUNCH_CHECK(ctx);
        return VR_OK;
    }
    if (ndm == 0) {
        // no dark matter anywhere: every baryon gets -1 (the kernel's scan
        // would find nothing); a one-entry empty table keeps it in bounds
        VR_WS(h0, ctx, uint32_t, WS_D0, 8);
        if ((rc = fill_u32(ctx, h0, 0xFFFFFFFFu, 2, st)) || (rc = fill_u32(ctx, h0 + 2, 0u, 6, st))) return rc;
        cl.hkeys = reinterpret_cast<const uint64_t*>(h0);
        cl.hvals = h0 + 2;
        cl.hmask = 0;
        cl.cell_start = h0 + 2;
    }
    // no dark matter at all: every baryon gets -1
    VR_TIMED(ctx, "assign_baryons", st, M - ndm,
             hipLaunchKernelGGL(k_assign, dim3(grid_for(M, 256)), dim3(256), 0, st, M, host_members, owner, is_baryon,
                                sub, p->qx, p->qy, p->qz, p->vx, p->vy, p->vz, cl, cx, cy, cz, dmi, dmh, dm_off, s,
                                gb - s, gb, u * u, sigma_v * sigma_v, 0, nullptr, nullptr, out));
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

extern "C" int vr_relabel_min(vr_ctx* ctx, int64_t n, const int32_t* label, int32_t min_size, int32_t* out,
                              void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    if (n < 0 || n >= (int64_t(1) << 31) || min_size < 1)
        return set_err(ctx, VR_ERR_INVALID_ARG, "need 0 <= n < 2^31 and min_size >= 1");
    if (n == 0) return VR_OK;
    if (!label || !out) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    VR_WS(cnt, ctx, int, WS_D5, n);
    VR_WS(low, ctx, int, WS_D6, n);
    VR_WS(bad, ctx, int, WS_FLAG2, 4);
    int rc;
    if ((rc = fill_i32(ctx, cnt, 0, n, st)) || (rc = fill_i32(ctx, low, 0x7FFFFFFF, n, st)) ||
        (rc = fill_i32(ctx, bad, 0, 1, st)))
        return rc;
    hipLaunchKernelGGL(k_label_stats, dim3(grid_for(n, 256)), dim3(256), 0, st, n, label, cnt, low, bad);
    hipLaunchKernelGGL(k_label_min, dim3(grid_for(n, 256)), dim3(256), 0, st, n, label, cnt, low, min_size, out);
    VR_LAUNCH_CHECK(ctx);
    int badh = 0;
    if ((rc = read_back(ctx, bad, &badh, sizeof badh, st))) return rc;
    if (badh) return set_err(ctx, VR_ERR_INVALID_ARG, "a label is >= n");
    return VR_OK;
}

extern "C" int vr_select_members(vr_ctx* ctx, int64_t n, int32_t n_groups, const int32_t* offsets,
                                 const int32_t* members, const uint8_t* drop, int32_t* out_offsets,
                                 int32_t* out_members, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_hosts(ctx, n_groups, offsets, members);
    if (rc) return rc;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, VR_ERR_INVALID_ARG, "n out of range");
    if (n_groups == 0) return VR_OK;
    if (!drop || !out_offsets || !out_members) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> off;
    if ((rc = read_host_offsets(ctx, n_groups, offsets, n, 0, off, st))) return rc;
    const int64_t M = off[n_groups];
    VR_WS(flag, ctx, uint32_t, WS_D7, M + 1);
    VR_WS(pos, ctx, uint32_t, WS_D8, M + 1);
    VR_WS(tot, ctx, uint32_t, WS_D9, 4);
    if (M > 0) {
        hipLaunchKernelGGL(k_keep_flags, dim3(grid_for(M, 256)), dim3(256), 0, st, M, members, drop, flag);
        VR_LAUNCH_CHECK(ctx);
    }
    if ((rc = scan_u32(ctx, flag, pos, M, tot, st))) return rc;
    if (M > 0) {
        hipLaunchKernelGGL(k_keep_scatter, dim3(grid_for(M, 256)), dim3(256), 0, st, M, flag, pos, members,
                           out_members);
        VR_LAUNCH_CHECK(ctx);
    }
    // a group starts where the kept members before its first one end
    hipLaunchKernelGGL(k_dm_offsets, dim3(grid_for(n_groups + 1, 256)), dim3(256), 0, st, n_groups, M, offsets,
                       pos, tot, reinterpret_cast<uint32_t*>(out_offsets));
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}
