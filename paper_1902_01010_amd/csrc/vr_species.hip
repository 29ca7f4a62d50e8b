// vr_species.hip -- two particle species, the DM+Baryons mode (Sec. 2.1 and
// Sec. 2.4, Eq. baryondist).
//
// 3D FOF with dark-matter-seeded links: the dark matter is compacted and
// linked by the ordinary 3D FOF; then every baryon scans the cells (of side
// >= ellx) of a cell list of the dark matter around it, its own first, and
// joins every dark-matter component with a member closer than ellx.  A
// baryon hangs below the root of the first component it meets; one that
// meets a second bridges the two roots by the lock-free union-find.
// Baryons never test each other.  Labels are the smallest index over each
// component (a baryon may be smaller than its dark-matter root).
//
// Baryon assignment: each baryon of a host takes the label of the host's
// dark matter nearest in phase space, D2 = d2 / ell2 + dv2 / sigma_v^2.  A
// host's dark matter is ordered along a six-dimensional Morton curve of the
// scaled coordinates and boxed in a fanout-64 tree; 64 baryons adjacent on
// the same curve walk it together in one wavefront, each lane starting from
// the dark matter next to it on the curve.  Members are scored with the
// exact D2, so the answer is that of a brute-force scan.
#include "vr_grid.h"
#include "vr_kd.h"

#include <mutex>

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

// The cells around a point that may hold a point closer than ellx (own cell
// first): of the 27 when the grid has 3 or more a side, those whose nearest
// grid point lies within ellx; else the distinct ones among them.
template <class F>
__device__ __forceinline__ void cells27(int px, int py, int pz, int s, int b, double ell2,
                                        const ckey_t* __restrict__ hkeys, const uint32_t* __restrict__ hvals,
                                        uint32_t hmask, F&& visit) {
    const int nc = 1 << b;
    const int side = 1 << s;
    const int cx = px >> s, cy = py >> s, cz = pz >> s;
    const int fx = px & (side - 1), fy = py & (side - 1), fz = pz & (side - 1);
    // squared distance along one axis to the nearest grid point of the
    // neighbouring cell at offset d (distinct cells when nc >= 3)
    auto gap2 = [side](int f, int d) -> double {
        const double g = d < 0 ? (double)f + 1.0 : (d > 0 ? (double)(side - f) : 0.0);
        return g * g;
    };
    uint32_t seen = 0;
    for (int t = 0; t < 27; ++t) {
        const int o = (t + 13) % 27;  // the own cell first
        const int dz = o / 9 - 1, dy = (o / 3) % 3 - 1, dx = o % 3 - 1;
        const uint32_t nx = (uint32_t)((cx + dx + nc) & (nc - 1));
        const uint32_t ny = (uint32_t)((cy + dy + nc) & (nc - 1));
        const uint32_t nz = (uint32_t)((cz + dz + nc) & (nc - 1));
        if (nc < 3) {
            const uint32_t bit = 1u << (nx + 2 * ny + 4 * nz);
            if (seen & bit) continue;
            seen |= bit;
        } else if (gap2(fx, dx) + gap2(fy, dy) + gap2(fz, dz) >= ell2) {
            continue;  // no member of that cell is closer than ellx
        }
        const int c = hash_find(hkeys, hvals, hmask, cell_key(nx, ny, nz, b));
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
    cells27(px, py, pz, s, b, ell2, cl.hkeys, cl.hvals, cl.hmask, [&](int c) {
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
                if (k0 < 0) {
                    // the first component: the baryon hangs below its root.
                    // Nothing ever links below a baryon, so only this
                    // thread writes parent[i], and no root is contended.
                    parent[i] = uf_find(parent, r);
                } else {
                    uf_union(parent, (int)i, r);  // a bridge: dark-matter roots meet
                }
                k3 = k2;
                k2 = k1;
                k1 = k0;
                k0 = r;
                if (ur >= 0) return;  // the cell holds this component only
            }
        }
    });
}

// Roots are dark matter (the smallest dark-matter index of the component);
// a baryon hung below one may have a smaller index, so the label is the
// smallest index over the component, found in three passes.
__global__ void k_roots(int64_t n, int* parent, int32_t* __restrict__ label, int* __restrict__ low) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    label[i] = uf_find(parent, (int)i);
    low[i] = (int)i;
}

__global__ void k_low(int64_t n, const uint8_t* __restrict__ isb, const int32_t* __restrict__ label,
                      int* __restrict__ low) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !isb[i]) return;
    const int r = label[i];
    if (r != (int)i && (int)i < low[r]) atomicMin(&low[r], (int)i);
}

__global__ void k_low_label(int64_t n, const int* __restrict__ low, int32_t* __restrict__ label) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) label[i] = low[label[i]];
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


// ---- phase-space tree over the dark matter of each host --------------------
// Scaled so that D^2 of Eq. (baryondist) is a plain squared distance in six
// dimensions: position (unwrapped against a reference member of the host)
// over ellx, velocity over sigma_v.  A host's dark matter is sorted along a
// six-dimensional Morton curve; runs of 64 members make the leaves, runs of
// 64 nodes the next level up, to one root per host.  One wavefront searches
// for one baryon: a lane per child box (or per leaf member), the nearest box
// first, boxes whose lower bound exceeds the best D^2 so far dropped.  Leaf
// members are scored with the exact D^2 of a brute-force scan (ties to the
// smaller particle index), so the answer does not depend on the tree.
constexpr int T6_FAN = 64;
constexpr int T6_MAX_DEPTH = 8;
constexpr int T6_LEV_SHIFT = 28;

// per host: reference position, extents of the unwrapped position over all
// members, order-preserving integer images of the dark matter's velocity
// extents, and whether every unwrapped difference is the periodic one
struct HostBox {
    int ref[3];
    int umin[3], umax[3];
    unsigned vmin[3], vmax[3];
    int ok;
};

__device__ __forceinline__ unsigned f2o(float f) {
    const unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float o2f(unsigned u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

struct Tree6 {
    const int32_t* lvl;  // (depth + 1) x (n_hosts + 1): first node of each host per level; level 0 = members
    int H1;              // n_hosts + 1
    int depth;           // levels above the members; the top one has one node per host
    int base[T6_MAX_DEPTH + 1];  // first box of each level (level >= 1)
    const float* box;    // 12 floats a node: lower corner, then upper corner
    const HostBox* hbox;
    const uint32_t *sx, *sy, *sz;  // members in tree order
    const float *svx, *svy, *svz;
    const int32_t* sj;  // particle index
    const uint64_t* dkey;  // Morton keys of the members in tree order (ascending)
};

__global__ void k_host_init(int n_hosts, const int32_t* __restrict__ off, const int32_t* __restrict__ mem,
                            const uint32_t* __restrict__ qx, const uint32_t* __restrict__ qy,
                            const uint32_t* __restrict__ qz, HostBox* __restrict__ hb) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n_hosts) return;
    HostBox b;
    b.ref[0] = b.ref[1] = b.ref[2] = 0;
    if (off[h] < off[h + 1]) {
        const int i = mem[off[h]];
        b.ref[0] = (int)qx[i];
        b.ref[1] = (int)qy[i];
        b.ref[2] = (int)qz[i];
    }
    for (int d = 0; d < 3; ++d) {
        b.umin[d] = INT_MAX;
        b.umax[d] = INT_MIN;
        b.vmin[d] = 0xFFFFFFFFu;
        b.vmax[d] = 0u;
    }
    b.ok = 0;
    hb[h] = b;
}

// extents per host: a thread folds 16 members of its block's chunk of 4096
// (a partial result per host it meets), and a wavefront whose last partial
// results share one host reduces them before the atomics
constexpr int EXT_PER_THREAD = 16;

__global__ __launch_bounds__(256) void k_host_extent(int64_t M, const int32_t* __restrict__ mem,
                                                     const int32_t* __restrict__ owner, const uint8_t* __restrict__ isb,
                                                     const uint32_t* __restrict__ qx, const uint32_t* __restrict__ qy,
                                                     const uint32_t* __restrict__ qz, const float* __restrict__ vx,
                                                     const float* __restrict__ vy, const float* __restrict__ vz,
                                                     int gb, HostBox* __restrict__ hb) {
    const int64_t base = (int64_t)blockIdx.x * (256 * EXT_PER_THREAD) + threadIdx.x;
    int h = -1;
    int lo[3], hi[3];
    unsigned vlo[3], vhi[3];
    auto reset = [&]() __attribute__((always_inline)) {
        for (int d = 0; d < 3; ++d) {
            lo[d] = INT_MAX;
            hi[d] = INT_MIN;
            vlo[d] = 0xFFFFFFFFu;
            vhi[d] = 0u;
        }
    };
    auto flush = [&](int hh) __attribute__((always_inline)) {
        HostBox* b = hb + hh;
        for (int d = 0; d < 3; ++d) {
            atomicMin(&b->umin[d], lo[d]);
            atomicMax(&b->umax[d], hi[d]);
            atomicMin(&b->vmin[d], vlo[d]);
            atomicMax(&b->vmax[d], vhi[d]);
        }
    };
    reset();
    for (int r = 0; r < EXT_PER_THREAD; ++r) {
        const int64_t k = base + (int64_t)r * 256;
        if (k >= M) break;
        const int hk = owner[k];
        if (hk != h) {
            if (h >= 0) flush(h);
            reset();
            h = hk;
        }
        const int i = mem[k];
        const int q[3] = {(int)qx[i], (int)qy[i], (int)qz[i]};
        for (int d = 0; d < 3; ++d) {
            const int u = min_image(q[d] - hb[h].ref[d], gb);
            lo[d] = min(lo[d], u);
            hi[d] = max(hi[d], u);
        }
        if (!isb[i]) {
            const unsigned o[3] = {f2o(vx[i]), f2o(vy[i]), f2o(vz[i])};
            for (int d = 0; d < 3; ++d) {
                vlo[d] = min(vlo[d], o[d]);
                vhi[d] = max(vhi[d], o[d]);
            }
        }
    }
    const int h0 = __shfl(h, 0, 64);
    if (h0 >= 0 && __ballot(h != h0) == 0) {
        for (int o = 32; o; o >>= 1)
            for (int d = 0; d < 3; ++d) {
                lo[d] = min(lo[d], __shfl_xor(lo[d], o, 64));
                hi[d] = max(hi[d], __shfl_xor(hi[d], o, 64));
                vlo[d] = min(vlo[d], (unsigned)__shfl_xor((int)vlo[d], o, 64));
                vhi[d] = max(vhi[d], (unsigned)__shfl_xor((int)vhi[d], o, 64));
            }
        if (lane_id() == 0) flush(h);
    } else if (h >= 0) {
        flush(h);
    }
}

__global__ void k_host_ok(int n_hosts, int gb, HostBox* __restrict__ hb) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n_hosts) return;
    const int64_t half = int64_t(1) << (gb - 1);
    bool ok = true;
    for (int d = 0; d < 3; ++d) ok = ok && ((int64_t)hb[h].umax[d] - hb[h].umin[d] < half);
    hb[h].ok = ok ? 1 : 0;
}

__device__ __forceinline__ void scaled6(const HostBox& b, uint32_t x, uint32_t y, uint32_t z, float vx, float vy,
                                        float vz, int gb, float ix, float iv, float* o) {
    o[0] = (float)min_image((int)x - b.ref[0], gb) * ix;
    o[1] = (float)min_image((int)y - b.ref[1], gb) * ix;
    o[2] = (float)min_image((int)z - b.ref[2], gb) * ix;
    o[3] = vx * iv;
    o[4] = vy * iv;
    o[5] = vz * iv;
}

// Morton key: host in the high bits, then mbits interleaved bits of each
// scaled coordinate over the host's box (clamped: baryons may lie outside
// the dark matter's velocity range)
__device__ __forceinline__ uint64_t key6(const HostBox& b, int h, const float* y, float ix, float iv, int mbits) {
    float lo[6], ext = 0.f;
    for (int d = 0; d < 3; ++d) {
        lo[d] = (float)b.umin[d] * ix;
        ext = fmaxf(ext, (float)b.umax[d] * ix - lo[d]);
        lo[d + 3] = o2f(b.vmin[d]) * iv;
        ext = fmaxf(ext, o2f(b.vmax[d]) * iv - lo[d + 3]);
    }
    const uint32_t top = (1u << mbits) - 1u;
    const float sc = ext > 0.f ? (float)(1u << mbits) / ext : 0.f;
    uint32_t c[6];
    for (int d = 0; d < 6; ++d) c[d] = min(top, (uint32_t)fmaxf((y[d] - lo[d]) * sc, 0.f));
    uint64_t m = 0;
    for (int bit = mbits - 1; bit >= 0; --bit)
        for (int d = 0; d < 6; ++d) m = (m << 1) | ((c[d] >> bit) & 1u);
    return ((uint64_t)h << (6 * mbits)) | m;
}

// keys of the compacted dark matter
__global__ void k_key6(int64_t ndm, const uint32_t* __restrict__ cx, const uint32_t* __restrict__ cy,
                       const uint32_t* __restrict__ cz, const int32_t* __restrict__ dmi,
                       const int32_t* __restrict__ dmh, const float* __restrict__ vx, const float* __restrict__ vy,
                       const float* __restrict__ vz, const HostBox* __restrict__ hb, int gb, float ix, float iv,
                       int mbits, uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ndm) return;
    const int h = dmh[j], i = dmi[j];
    const HostBox b = hb[h];
    float y[6];
    scaled6(b, cx[j], cy[j], cz[j], vx[i], vy[i], vz[i], gb, ix, iv, y);
    key[j] = key6(b, h, y, ix, iv, mbits);
    val[j] = (uint32_t)j;
}

// keys of the baryons (member positions in blist), so that neighbouring
// wavefronts search neighbouring parts of the tree
__global__ void k_bkey6(int64_t nb, const int32_t* __restrict__ blist, const int32_t* __restrict__ mem,
                        const int32_t* __restrict__ owner, const uint32_t* __restrict__ qx,
                        const uint32_t* __restrict__ qy, const uint32_t* __restrict__ qz, const float* __restrict__ vx,
                        const float* __restrict__ vy, const float* __restrict__ vz, const HostBox* __restrict__ hb,
                        int gb, float ix, float iv, int mbits, uint64_t* __restrict__ key) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb) return;
    const int k = blist[t];
    const int h = owner[k], i = mem[k];
    const HostBox b = hb[h];
    float y[6];
    scaled6(b, qx[i], qy[i], qz[i], vx[i], vy[i], vz[i], gb, ix, iv, y);
    key[t] = key6(b, h, y, ix, iv, mbits);
}

__global__ void k_gather6(int64_t ndm, const uint32_t* __restrict__ val, const uint32_t* __restrict__ cx,
                          const uint32_t* __restrict__ cy, const uint32_t* __restrict__ cz,
                          const int32_t* __restrict__ dmi, const float* __restrict__ vx, const float* __restrict__ vy,
                          const float* __restrict__ vz, uint32_t* __restrict__ sx, uint32_t* __restrict__ sy,
                          uint32_t* __restrict__ sz, float* __restrict__ svx, float* __restrict__ svy,
                          float* __restrict__ svz, int32_t* __restrict__ sj) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ndm) return;
    const uint32_t j = val[p];
    const int i = dmi[j];
    sx[p] = cx[j];
    sy[p] = cy[j];
    sz[p] = cz[j];
    svx[p] = vx[i];
    svy[p] = vy[i];
    svz[p] = vz[i];
    sj[p] = i;
}

__device__ __forceinline__ int host_of_node(const int32_t* lvl, int H1, int g) {
    int lo = 0, hi = H1 - 1;  // last h with lvl[h] <= g
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (lvl[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// boxes of level lev: one wavefront per node, a lane per child
__global__ __launch_bounds__(256) void k_boxes6(int64_t n_nodes, int lev, Tree6 t, int gb, float ix, float iv,
                                                float* __restrict__ box) {
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= n_nodes) return;
    const int lane = (int)lane_id();
    const int32_t* L = t.lvl + (int64_t)lev * t.H1;
    const int32_t* C = t.lvl + (int64_t)(lev - 1) * t.H1;
    const int h = host_of_node(L, t.H1, (int)g);
    const int c = C[h] + T6_FAN * ((int)g - L[h]) + lane;
    float lo[6], hi[6];
    for (int d = 0; d < 6; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
    if (c < C[h + 1]) {
        if (lev == 1) {
            scaled6(t.hbox[h], t.sx[c], t.sy[c], t.sz[c], t.svx[c], t.svy[c], t.svz[c], gb, ix, iv, lo);
            for (int d = 0; d < 6; ++d) hi[d] = lo[d];
        } else {
            const float* cb = t.box + (int64_t)(t.base[lev - 1] + c) * 12;
            for (int d = 0; d < 6; ++d) {
                lo[d] = cb[d];
                hi[d] = cb[6 + d];
            }
        }
    }
    for (int o = 32; o; o >>= 1)
        for (int d = 0; d < 6; ++d) {
            lo[d] = fminf(lo[d], __shfl_xor(lo[d], o, 64));
            hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], o, 64));
        }
    float* ob = box + (int64_t)(t.base[lev] + g) * 12;
    if (lane < 6) ob[lane] = lo[lane];
    else if (lane < 12) ob[lane] = hi[lane - 6];
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

// dark-matter members keep their own label
__global__ void k_assign_dm(int64_t M, const int32_t* __restrict__ mem, const uint8_t* __restrict__ isb,
                            const int32_t* __restrict__ sub, int no_dm, int32_t* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const int i = mem[k];
    if (!isb[i]) out[i] = sub[i];
    else if (no_dm) out[i] = -1;
}

__global__ void k_baryon_list(int64_t M, const uint32_t* __restrict__ dmflag, const uint32_t* __restrict__ pos,
                              int32_t* __restrict__ blist) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < M && !dmflag[k]) blist[k - pos[k]] = (int32_t)k;
}

// One wavefront per 64 consecutive baryons of the tree-ordered list.  The
// lanes of one host walk its tree together: a node is opened when its box
// may hold a closer member for any of them, and each lane keeps its own
// best.  Leaves are staged in LDS; a lane scores a member exactly only when
// a float distance, with a margin for the rounding of the scaled
// coordinates, does not already rule it out.
constexpr int T6_WAVES = 4;

__global__ __launch_bounds__(256) void k_assign6(int64_t nb, const int32_t* __restrict__ blist,
                                                 const int32_t* __restrict__ mem, const int32_t* __restrict__ owner,
                                                 const int32_t* __restrict__ sub, const uint32_t* __restrict__ qx,
                                                 const uint32_t* __restrict__ qy, const uint32_t* __restrict__ qz,
                                                 const float* __restrict__ vx, const float* __restrict__ vy,
                                                 const float* __restrict__ vz, const uint64_t* __restrict__ bkey,
                                                 Tree6 t, int gb, double ell2, double sv2, float ix, float iv,
                                                 int32_t* __restrict__ out) {
    __shared__ int stack[T6_WAVES][T6_MAX_DEPTH * T6_FAN];
    __shared__ float4 sya[T6_WAVES][T6_FAN], syb[T6_WAVES][T6_FAN], svl[T6_WAVES][T6_FAN];
    __shared__ uint4 sqp[T6_WAVES][T6_FAN];
    const int w = (int)(threadIdx.x >> 6);
    const int lane = (int)lane_id();
    const int64_t wave = (int64_t)blockIdx.x * T6_WAVES + w;
    if (wave * 64 >= nb) return;
    const int64_t bi = wave * 64 + lane;
    const bool valid = bi < nb;
    int i = 0, h = -1, px = 0, py = 0, pz = 0;
    float fvx = 0.f, fvy = 0.f, fvz = 0.f;
    if (valid) {
        const int k = blist[bi];
        i = mem[k];
        h = owner[k];
        px = (int)qx[i];
        py = (int)qy[i];
        pz = (int)qz[i];
        fvx = vx[i];
        fvy = vy[i];
        fvz = vz[i];
    }
    const double bx = (double)fvx, by = (double)fvy, bz = (double)fvz;
    Best bst{INFINITY, 0x7FFFFFFF};
    int* stk = stack[w];
    // members [p0, p1) of the tree order into LDS, a lane each
    auto stage = [&](int p0, int p1, const HostBox& hb) __attribute__((always_inline)) {
        const int p = p0 + lane;
        if (p < p1) {
            const uint32_t x = t.sx[p], yy = t.sy[p], z = t.sz[p];
            const float a = t.svx[p], b = t.svy[p], c = t.svz[p];
            float y6[6];
            scaled6(hb, x, yy, z, a, b, c, gb, ix, iv, y6);
            sya[w][lane] = make_float4(y6[0], y6[1], y6[2], y6[3]);
            syb[w][lane] = make_float4(y6[4], y6[5], 0.f, 0.f);
            sqp[w][lane] = make_uint4(x, yy, z, (uint32_t)t.sj[p]);
            svl[w][lane] = make_float4(a, b, c, 0.f);
        }
        __builtin_amdgcn_wave_barrier();
    };
    // exact D^2 of staged member q, as a brute-force scan computes it
    auto exact = [&](int q) __attribute__((always_inline)) {
        const uint4 e = sqp[w][q];
        const float4 v = svl[w][q];
        const int ddx = min_image((int)e.x - px, gb);
        const int ddy = min_image((int)e.y - py, gb);
        const int ddz = min_image((int)e.z - pz, gb);
        const double d2 = (double)ddx * ddx + (double)ddy * ddy + (double)ddz * ddz;
        const double ax = bx - (double)v.x, ay = by - (double)v.y, az = bz - (double)v.z;
        consider(bst, d2 / ell2 + (ax * ax + ay * ay + az * az) / sv2, (int)e.w);
    };
    uint64_t pending = __ballot(valid);
    while (pending) {
        const int hh = __builtin_amdgcn_readfirstlane(__shfl(h, __builtin_ctzll(pending), 64));
        const bool mine = valid && h == hh;
        pending &= ~__ballot(mine);
        const int d0 = t.lvl[hh], d1 = t.lvl[hh + 1];
        if (d0 == d1) continue;  // no dark matter in this host
        const HostBox hb = t.hbox[hh];
        if (!hb.ok) {
            // a host wider than half the box: all of its dark matter
            for (int p0 = d0; p0 < d1; p0 += T6_FAN) {
                const int p1 = min(p0 + T6_FAN, d1);
                stage(p0, p1, hb);
                if (mine)
                    for (int q = 0; q < p1 - p0; ++q) exact(q);
                __builtin_amdgcn_wave_barrier();
            }
            continue;
        }
        float y[6];
        scaled6(hb, (uint32_t)px, (uint32_t)py, (uint32_t)pz, fvx, fvy, fvz, gb, ix, iv, y);
        if (mine) {
            // a first best: the eight dark-matter members next to this
            // baryon along the curve (baryons and dark matter share the key)
            const uint64_t kb = bkey[bi];
            int lo = d0, hi = d1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (t.dkey[mid] < kb) lo = mid + 1;
                else hi = mid;
            }
            const int q0 = max(d0, min(lo - 4, d1 - 8)), q1 = min(d1, q0 + 8);
            for (int q = q0; q < q1; ++q) {
                const int ddx = min_image((int)t.sx[q] - px, gb);
                const int ddy = min_image((int)t.sy[q] - py, gb);
                const int ddz = min_image((int)t.sz[q] - pz, gb);
                const double d2 = (double)ddx * ddx + (double)ddy * ddy + (double)ddz * ddz;
                const double ax = bx - (double)t.svx[q], ay = by - (double)t.svy[q], az = bz - (double)t.svz[q];
                consider(bst, d2 / ell2 + (ax * ax + ay * ay + az * az) / sv2, t.sj[q]);
            }
        }
        // the packet's box, and the margins for the rounding of the scaled
        // coordinates (a few ulps of the largest of them)
        float qlo[6], qhi[6], amax = 0.f;
        for (int d = 0; d < 6; ++d) {
            qlo[d] = mine ? y[d] : INFINITY;
            qhi[d] = mine ? y[d] : -INFINITY;
            if (mine) amax = fmaxf(amax, fabsf(y[d]));
        }
        for (int o = 32; o; o >>= 1) {
            for (int d = 0; d < 6; ++d) {
                qlo[d] = fminf(qlo[d], __shfl_xor(qlo[d], o, 64));
                qhi[d] = fmaxf(qhi[d], __shfl_xor(qhi[d], o, 64));
            }
            amax = fmaxf(amax, __shfl_xor(amax, o, 64));
        }
        const int top = t.depth;
        const int root = t.lvl[(int64_t)top * t.H1 + hh];
        {
            const float* rb = t.box + (int64_t)(t.base[top] + root) * 12;
            for (int d = 0; d < 12; ++d) amax = fmaxf(amax, fabsf(rb[d]));
        }
        const float E = amax * 0x1p-19f;
        const double dlt = 5.0 * (double)amax * 0x1p-22;
        // a float squared distance above thr rules a member out
        auto thr_of = [&]() __attribute__((always_inline)) -> float {
            if (!(bst.d < INFINITY)) return INFINITY;
            const double r = sqrt(bst.d) * (1.0 + 0x1p-40) + dlt;
            return (float)(r * r * (1.0 + 0x1p-19));
        };
        float thr = thr_of();
        if (lane == 0) stk[0] = (top << T6_LEV_SHIFT) | root;
        __builtin_amdgcn_wave_barrier();
        int sp = 1;
        while (sp > 0) {
            --sp;
            const int e = __builtin_amdgcn_readfirstlane(stk[sp]);
            const int lev = e >> T6_LEV_SHIFT;
            const int node = e & ((1 << T6_LEV_SHIFT) - 1);
            const float* nbx = t.box + (int64_t)(t.base[lev] + node) * 12;
            float lb = 0.f;
            for (int d = 0; d < 6; ++d) {
                const float g = fmaxf(fmaxf(nbx[d] - y[d], y[d] - nbx[6 + d]) - E, 0.f);
                lb += g * g;
            }
            lb *= 1.f - 0x1p-20f;
            const bool need = mine && (double)lb <= bst.d;
            if (!__ballot(need)) continue;
            const int32_t* L = t.lvl + (int64_t)lev * t.H1;
            const int32_t* C = t.lvl + (int64_t)(lev - 1) * t.H1;
            const int c0 = C[hh] + T6_FAN * (node - L[hh]);
            const int c1 = min(c0 + T6_FAN, C[hh + 1]);
            if (lev == 1) {
                stage(c0, c1, hb);
                if (need) {
                    for (int q = 0; q < c1 - c0; ++q) {
                        const float4 A = sya[w][q], B = syb[w][q];
                        const float e0 = y[0] - A.x, e1 = y[1] - A.y, e2 = y[2] - A.z;
                        const float e3 = y[3] - A.w, e4 = y[4] - B.x, e5 = y[5] - B.y;
                        const float dF = e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3 + e4 * e4 + e5 * e5;
                        if (dF <= thr) {
                            exact(q);
                            thr = thr_of();
                        }
                    }
                }
                __builtin_amdgcn_wave_barrier();
                continue;
            }
            // children within reach of a lane that opened this node
            double mb = need ? bst.d : 0.0;
            for (int o = 32; o; o >>= 1) mb = fmax(mb, __shfl_xor(mb, o, 64));
            const int c = c0 + lane;
            bool keep = false;
            float key = INFINITY;
            if (c < c1) {
                const float* cb = t.box + (int64_t)(t.base[lev - 1] + c) * 12;
                float bb = 0.f, cd = 0.f;
                for (int d = 0; d < 6; ++d) {
                    const float lo = cb[d], hi = cb[6 + d];
                    const float g = fmaxf(fmaxf(lo - qhi[d], qlo[d] - hi) - E, 0.f);
                    bb += g * g;
                    const float m = 0.5f * (qlo[d] + qhi[d]);
                    const float gc = fmaxf(fmaxf(lo - m, m - hi), 0.f);
                    cd += gc * gc;
                }
                keep = (double)(bb * (1.f - 0x1p-20f)) <= mb;
                key = cd;
            }
            const uint64_t km = __ballot(keep);
            if (!km) continue;
            float mn = keep ? key : INFINITY;
            for (int o = 32; o; o >>= 1) mn = fminf(mn, __shfl_xor(mn, o, 64));
            const int first = __builtin_ctzll(__ballot(keep && key == mn));
            const uint64_t others = km & ~(1ull << first);
            const int no = __popcll(others);
            const int ent = ((lev - 1) << T6_LEV_SHIFT) | c;
            // the child nearest the packet's centre goes on top, opened next
            if (keep && lane != first) stk[sp + __popcll(others & ((1ull << lane) - 1ull))] = ent;
            if (lane == first) stk[sp + no] = ent;
            sp += no + 1;
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (valid) out[i] = bst.j == 0x7FFFFFFF ? -1 : sub[bst.j];
}

// The dark-matter-weighted mean over hosts of ellv_host[h] * inv_alpha (the
// hosts' sigma_v), one workgroup: FP64 partial sums per thread in host
// order, then a tree over the 256 threads.
__global__ __launch_bounds__(256) void k_dm_weighted_sigma(int n_hosts, const uint32_t* __restrict__ dm_off,
                                                           const double* __restrict__ ellv, double inv_alpha,
                                                           double* __restrict__ out) {
    __shared__ double sw[256], sn[256];
    double a = 0.0, c = 0.0;
    for (int h = threadIdx.x; h < n_hosts; h += 256) {
        const double k = (double)(dm_off[h + 1] - dm_off[h]);
        a += k * ellv[h];
        c += k;
    }
    sw[threadIdx.x] = a;
    sn[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sw[threadIdx.x] += sw[threadIdx.x + o];
            sn[threadIdx.x] += sn[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sn[0] > 0 ? sw[0] / sn[0] * inv_alpha : 0.0;
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
    VR_WS(low, ctx, int, WS_D3, n);
    hipLaunchKernelGGL(k_roots, dim3(grid_for(n, 256)), dim3(256), 0, st, n, parent, label, low);
    hipLaunchKernelGGL(k_low, dim3(grid_for(n, 256)), dim3(256), 0, st, n, is_baryon, label, low);
    hipLaunchKernelGGL(k_low_label, dim3(grid_for(n, 256)), dim3(256), 0, st, n, low, label);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

extern "C" int vr_assign_baryons(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts, const int32_t* host_offsets,
                                 const int32_t* host_members, const uint8_t* is_baryon, const int32_t* sub,
                                 double ellx, double sigma_v, const double* ellv_host, double alpha_v,
                                 double* sigma_v_used, int32_t* out, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_particles(ctx, p, true);
    if (rc) return rc;
    if ((rc = check_hosts(ctx, n_hosts, host_offsets, host_members))) return rc;
    const int gb = p->grid_bits;
    const double u = ellx * ldexp(1.0, gb) / p->box;
    if (!(u > 0) || !(u < ldexp(1.0, gb - 1)) || !std::isfinite(sigma_v))
        return set_err(ctx, VR_ERR_INVALID_ARG, "need 0 < ellx < box/2 and a finite sigma_v");
    const bool from_hosts = !(sigma_v > 0);
    if (from_hosts && (!ellv_host || !(alpha_v > 0)))
        return set_err(ctx, VR_ERR_INVALID_ARG, "sigma_v <= 0 needs ellv_host and alpha_v > 0");
    if (sigma_v_used) *sigma_v_used = from_hosts ? 0.0 : sigma_v;
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
    if (ndm == 0) {
        hipLaunchKernelGGL(k_assign_dm, dim3(grid_for(M, 256)), dim3(256), 0, st, M, host_members, is_baryon, sub, 1,
                           out);
        VR_LAUNCH_CHECK(ctx);
        return VR_OK;
    }
    if (from_hosts) {
        VR_WS(sv_dev, ctx, double, WS_D1, 2);
        hipLaunchKernelGGL(k_dm_weighted_sigma, dim3(1), dim3(256), 0, st, n_hosts, dm_off, ellv_host,
                           1.0 / alpha_v, sv_dev);
        VR_LAUNCH_CHECK(ctx);
        if ((rc = read_back(ctx, sv_dev, &sigma_v, sizeof sigma_v, st))) return rc;
        if (!(sigma_v > 0) || !std::isfinite(sigma_v))
            return set_err(ctx, VR_ERR_INVALID_ARG, "sigma_v from the hosts is %g, not positive", sigma_v);
        if (sigma_v_used) *sigma_v_used = sigma_v;
    }
    const int64_t nb = M - ndm;
    const float ix = (float)(1.0 / u), iv = (float)(1.0 / sigma_v);
    // per-host boxes and the wrap check
    VR_WS(hbox, ctx, HostBox, WS_D0, n_hosts);
    hipLaunchKernelGGL(k_host_init, dim3(grid_for(n_hosts, 256)), dim3(256), 0, st, n_hosts, host_offsets,
                       host_members, p->qx, p->qy, p->qz, hbox);
    hipLaunchKernelGGL(k_host_extent, dim3(grid_for(M, 256 * EXT_PER_THREAD)), dim3(256), 0, st, M, host_members,
                       owner, is_baryon, p->qx, p->qy, p->qz, p->vx, p->vy, p->vz, gb, hbox);
    hipLaunchKernelGGL(k_host_ok, dim3(grid_for(n_hosts, 256)), dim3(256), 0, st, n_hosts, gb, hbox);
    VR_LAUNCH_CHECK(ctx);
    // tree order: by host, then along the Morton curve
    int hbits = 1;
    while (hbits < 62 && (int64_t(1) << hbits) < n_hosts) ++hbits;
    const int mbits = std::min(8, (64 - hbits) / 6);
    VR_WS(key, ctx, uint64_t, WS_D2, ndm);
    VR_WS(val, ctx, uint32_t, WS_D3, ndm);
    hipLaunchKernelGGL(k_key6, dim3(grid_for(ndm, 256)), dim3(256), 0, st, ndm, cx, cy, cz, dmi, dmh, p->vx, p->vy,
                       p->vz, hbox, gb, ix, iv, mbits, key, val);
    VR_LAUNCH_CHECK(ctx);
    if ((rc = sort_pairs_u64(ctx, key, val, ndm, hbits + 6 * mbits, st))) return rc;
    Tree6 t{};
    {
        VR_WS(sx, ctx, uint32_t, WS_D4, ndm);
        VR_WS(sy, ctx, uint32_t, WS_D5, ndm);
        VR_WS(sz, ctx, uint32_t, WS_D6, ndm);
        VR_WS(svx, ctx, float, WS_D7, ndm);
        VR_WS(svy, ctx, float, WS_D8, ndm);
        VR_WS(svz, ctx, float, WS_D9, ndm);
        VR_WS(sj, ctx, int32_t, WS_A0, ndm);
        hipLaunchKernelGGL(k_gather6, dim3(grid_for(ndm, 256)), dim3(256), 0, st, ndm, val, cx, cy, cz, dmi, p->vx,
                           p->vy, p->vz, sx, sy, sz, svx, svy, svz, sj);
        VR_LAUNCH_CHECK(ctx);
        t.sx = sx;
        t.sy = sy;
        t.sz = sz;
        t.svx = svx;
        t.svy = svy;
        t.svz = svz;
        t.sj = sj;
        t.dkey = key;
    }
    // level sizes: runs of 64 per host, up to one node per host
    std::vector<uint32_t> doff(n_hosts + 1);
    if ((rc = read_back(ctx, dm_off, doff.data(), doff.size() * sizeof(uint32_t), st))) return rc;
    const int H1 = n_hosts + 1;
    std::vector<int32_t> lvl(doff.begin(), doff.end());
    std::vector<int64_t> cnt(n_hosts);
    for (int h = 0; h < n_hosts; ++h) cnt[h] = (int64_t)doff[h + 1] - doff[h];
    int depth = 0;
    int64_t total = 0;
    for (bool more = true; more;) {
        if (depth == T6_MAX_DEPTH) return set_err(ctx, VR_ERR_UNSUPPORTED, "phase-space tree too deep");
        more = false;
        int64_t run = 0;
        const size_t at = lvl.size();
        lvl.resize(at + H1);
        for (int h = 0; h < n_hosts; ++h) {
            lvl[at + h] = (int32_t)run;
            cnt[h] = (cnt[h] + T6_FAN - 1) / T6_FAN;
            more = more || cnt[h] > 1;
            run += cnt[h];
        }
        lvl[at + n_hosts] = (int32_t)run;
        ++depth;
        t.base[depth] = (int)total;
        total += run;
        if (run >= (int64_t(1) << T6_LEV_SHIFT) || total >= (int64_t(1) << 31) / 12)
            return set_err(ctx, VR_ERR_UNSUPPORTED, "phase-space tree too large");
    }
    VR_WS(lvl_d, ctx, int32_t, WS_A2, (int64_t)lvl.size());
    VR_HIP(ctx, hipMemcpyAsync(lvl_d, lvl.data(), lvl.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    VR_HIP(ctx, hipStreamSynchronize(st));  // lvl leaves scope
    VR_WS(box, ctx, float, WS_A1, 12 * total);
    t.lvl = lvl_d;
    t.H1 = H1;
    t.depth = depth;
    t.box = box;
    t.hbox = hbox;
    for (int l = 1; l <= depth; ++l) {
        const int64_t nl = lvl[(size_t)l * H1 + n_hosts];
        hipLaunchKernelGGL(k_boxes6, dim3((unsigned)((nl + 3) / 4)), dim3(256), 0, st, nl, l, t, gb, ix, iv, box);
        VR_LAUNCH_CHECK(ctx);
    }
    VR_WS(blist, ctx, int32_t, WS_A3, nb + 1);
    VR_WS(bkey, ctx, uint64_t, WS_A5, nb + 1);
    hipLaunchKernelGGL(k_baryon_list, dim3(grid_for(M, 256)), dim3(256), 0, st, M, flag, pos, blist);
    VR_LAUNCH_CHECK(ctx);
    if (nb > 0) {
        hipLaunchKernelGGL(k_bkey6, dim3(grid_for(nb, 256)), dim3(256), 0, st, nb, blist, host_members, owner, p->qx,
                           p->qy, p->qz, p->vx, p->vy, p->vz, hbox, gb, ix, iv, mbits, bkey);
        VR_LAUNCH_CHECK(ctx);
    }
    if (nb > 1 && (rc = sort_pairs_u64(ctx, bkey, reinterpret_cast<uint32_t*>(blist), nb, hbits + 6 * mbits, st)))
        return rc;
    hipLaunchKernelGGL(k_assign_dm, dim3(grid_for(M, 256)), dim3(256), 0, st, M, host_members, is_baryon, sub, 0, out);
    VR_LAUNCH_CHECK(ctx);
    if (nb > 0) {
        VR_TIMED(ctx, "assign_baryons", st, nb,
                 hipLaunchKernelGGL(k_assign6, dim3((unsigned)((nb + 64 * T6_WAVES - 1) / (64 * T6_WAVES))),
                                    dim3(64 * T6_WAVES), 0, st, nb, blist,
                                    host_members, owner, sub, p->qx, p->qy, p->qz, p->vx, p->vy, p->vz, bkey, t, gb,
                                    u * u, sigma_v * sigma_v, ix, iv, out));
        VR_LAUNCH_CHECK(ctx);
    }
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

// ---- vr_relabel_min without allocation ---------------------------------------
// The counts, minima and error flag of vr_relabel_min_noalloc live in this
// fixed device array: VR_NOALLOC_MAX_LABELS ints of counts, as many of minima,
// then the flag.  Each GPU holds its own copy until the process ends; in host
// code `scratch` names no device address, so kernels only ever get the
// per-device address that noalloc_scratch_init() takes once per device.
namespace {
constexpr int64_t NOALLOC_INTS = 2 * (int64_t)VR_NOALLOC_MAX_LABELS + 64;
static __device__ __align__(256) int32_t scratch[NOALLOC_INTS];
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};
}  // namespace

namespace vr {
// Called by vr_create with `device` current: records that device's address of
// `scratch` (once per device; later calls find it recorded).
int noalloc_scratch_init(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES)
        return set_err(nullptr, VR_ERR_UNSUPPORTED, "device %d beyond the %d the fixed scratch supports", device,
                       NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return VR_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return set_err(nullptr, VR_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                       hipGetErrorString(e));
    g_scratch_dev[device] = static_cast<int32_t*>(ptr);
    return VR_OK;
}
}  // namespace vr

extern "C" int vr_relabel_min_noalloc(vr_ctx* ctx, int64_t n, const int32_t* label, int32_t min_size, int32_t* out,
                                      void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    if (n < 0 || min_size < 1) return set_err(ctx, VR_ERR_INVALID_ARG, "need n >= 0 and min_size >= 1");
    if (n > (int64_t)VR_NOALLOC_MAX_LABELS)
        return set_err(ctx, VR_ERR_INVALID_ARG, "n = %lld exceeds the %d labels of the fixed scratch", (long long)n,
                       VR_NOALLOC_MAX_LABELS);
    if (n == 0) return VR_OK;
    if (!label || !out) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    int32_t* base = (ctx->device >= 0 && ctx->device < NOALLOC_MAX_DEVICES) ? g_scratch_dev[ctx->device] : nullptr;
    if (!base) return set_err(ctx, VR_ERR_HIP, "no scratch address recorded for device %d", ctx->device);
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    int32_t* cnt = base;
    int32_t* low = base + VR_NOALLOC_MAX_LABELS;
    int32_t* bad = base + 2 * (int64_t)VR_NOALLOC_MAX_LABELS;
    // what a previous call left behind is cleared by fill kernels
    int rc;
    if ((rc = fill_i32(ctx, cnt, 0, n, st)) || (rc = fill_i32(ctx, low, 0x7FFFFFFF, n, st)) ||
        (rc = fill_i32(ctx, bad, 0, 1, st)))
        return rc;
    hipLaunchKernelGGL(k_label_stats, dim3(grid_for(n, 256)), dim3(256), 0, st, n, label, cnt, low, bad);
    hipLaunchKernelGGL(k_label_min, dim3(grid_for(n, 256)), dim3(256), 0, st, n, label, cnt, low, min_size, out);
    VR_LAUNCH_CHECK(ctx);
    // the flag comes back through the context's pinned host words
    int32_t* flag_h = reinterpret_cast<int32_t*>(ctx->pinned);
    VR_HIP(ctx, hipMemcpyAsync(flag_h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    VR_HIP(ctx, hipStreamSynchronize(st));
    if (*flag_h) return set_err(ctx, VR_ERR_INVALID_ARG, "a label is >= n");
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
