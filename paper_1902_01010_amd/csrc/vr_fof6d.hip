// vr_fof6d.hip -- velocity linking length of a host and 6D friends-of-
// friends over the outliers (Sec. 2.1, Eq. fof6d, with the substructure
// linking length of Sec. 2.2), and the paper's own substructure linker
// (Sec. 2.2, Eq. linkingcriteria).
//
// Participants (hosted particles with R, or L, at or above the threshold)
// are compacted, put on their own integer-grid cell list with cells of side
// 2^s >= ellx_s, and every candidate pair is tested in FP64, d2 being the
// exact integer squared distance: for Eq. fof6d d2 / ells2 + dv2 / ellv^2 < 1
// in exactly that order; for Eq. linkingcriteria d2 < ells2, speeds about
// the local mean velocity within a factor Vr and directions within the
// opening angle.  Components come from the same lock-free union-find as the
// 3D search; labels are the smallest participant index.
#include "vr_grid.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

namespace vr {
namespace {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int N>
__device__ __forceinline__ void bsum(double (&v)[N], double* sm) {
    const int lane = __lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int i = 0; i < N; ++i) {
        double s = wsum(v[i]);
        if (lane == 0) sm[w * N + i] = s;
    }
    __syncthreads();
    for (int i = 0; i < N; ++i) {
        double s = 0;
        for (int ww = 0; ww < nw; ++ww) s += sm[ww * N + i];
        v[i] = s;
    }
    __syncthreads();
}

// sigma_v of a host from the mass-weighted dispersion tensor of all members
// about their mass-weighted mean velocity.  Members are cut into chunks of
// ELLV_CHUNK; one workgroup sums a chunk and one thread per host adds its
// chunks in order, so the result does not depend on scheduling.  One pass:
// velocities are summed relative to the host's first member v0, and the
// tensor is E[(v - v0)(v - v0)^T] - (vbar - v0)(vbar - v0)^T, equal to the
// tensor about vbar up to rounding (v0 is a member, so both terms are of
// the size of the dispersion).
constexpr int ELLV_CHUNK = 8192;
constexpr int ELLV_PART = 10;  // M, sum m (v - v0), sum m (v - v0)(v - v0)^T

__global__ __launch_bounds__(256) void k_ellv_sums(const int4* __restrict__ chunks, const int32_t* __restrict__ mem,
                                                   const int32_t* __restrict__ off, const float* __restrict__ vx,
                                                   const float* __restrict__ vy, const float* __restrict__ vz,
                                                   const float* __restrict__ mass, double mass_value,
                                                   double* __restrict__ part) {
    __shared__ double sm[4 * ELLV_PART];
    const int4 c = chunks[blockIdx.x];
    const int i0 = mem[off[c.x]];
    const double v0x = (double)vx[i0], v0y = (double)vy[i0], v0z = (double)vz[i0];
    double a[ELLV_PART] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = c.y + threadIdx.x; k < c.z; k += blockDim.x) {
        const int i = mem[k];
        const double m = mass ? (double)mass[i] : mass_value;
        const double d0 = (double)vx[i] - v0x, d1 = (double)vy[i] - v0y, d2 = (double)vz[i] - v0z;
        a[0] += m;
        a[1] += m * d0;
        a[2] += m * d1;
        a[3] += m * d2;
        a[4] += m * d0 * d0;
        a[5] += m * d1 * d1;
        a[6] += m * d2 * d2;
        a[7] += m * d0 * d1;
        a[8] += m * d0 * d2;
        a[9] += m * d1 * d2;
    }
    bsum<ELLV_PART>(a, sm);
    if (threadIdx.x == 0)
        for (int q = 0; q < ELLV_PART; ++q) part[(int64_t)blockIdx.x * ELLV_PART + q] = a[q];
}

__global__ void k_ellv_final(int n_hosts, const int* __restrict__ chunk_off, const double* __restrict__ part,
                             double alpha_v, double* __restrict__ ellv) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n_hosts) return;
    double c[ELLV_PART] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = chunk_off[h]; k < chunk_off[h + 1]; ++k)
        for (int q = 0; q < ELLV_PART; ++q) c[q] += part[(int64_t)k * ELLV_PART + q];
    const double M = c[0];
    const double e0 = c[1] / M, e1 = c[2] / M, e2 = c[3] / M;  // vbar - v0
    const double s00 = c[4] / M - e0 * e0, s11 = c[5] / M - e1 * e1, s22 = c[6] / M - e2 * e2;
    const double s01 = c[7] / M - e0 * e1, s02 = c[8] / M - e0 * e2, s12 = c[9] / M - e1 * e2;
    const double det = s00 * (s11 * s22 - s12 * s12) - s01 * (s01 * s22 - s12 * s02) + s02 * (s01 * s12 - s11 * s02);
    ellv[h] = alpha_v * pow(det, 1.0 / 6.0);
}

__global__ void k_participants(int64_t n, const int32_t* __restrict__ host_of, const float* __restrict__ R,
                               float thr, int32_t n_hosts, uint32_t* __restrict__ flag, int* __restrict__ bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int h = host_of[i];
    flag[i] = (h >= 0 && h < n_hosts && (R == nullptr || R[i] >= thr)) ? 1u : 0u;
}

__global__ void k_compact_part(int64_t n, const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                               const uint32_t* __restrict__ qx, const uint32_t* __restrict__ qy,
                               const uint32_t* __restrict__ qz, uint32_t* __restrict__ cx, uint32_t* __restrict__ cy,
                               uint32_t* __restrict__ cz, int32_t* __restrict__ orig) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const uint32_t k = pos[i];
    cx[k] = qx[i];
    cy[k] = qy[i];
    cz[k] = qz[i];
    orig[k] = (int32_t)i;
}

// per sorted position: original particle index, velocity and host
__global__ void k_sorted_attrs(int64_t np, const uint32_t* __restrict__ cidx, const int32_t* __restrict__ orig,
                               const float* __restrict__ vx, const float* __restrict__ vy, const float* __restrict__ vz,
                               const int32_t* __restrict__ host_of, int32_t* __restrict__ sorig,
                               float* __restrict__ svx, float* __restrict__ svy, float* __restrict__ svz,
                               int32_t* __restrict__ shost) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int32_t i = orig[cidx[p]];
    sorig[p] = i;
    svx[p] = vx[i];
    svy[p] = vy[i];
    svz[p] = vz[i];
    shost[p] = host_of[i];
}

// Velocity relative to the local mean velocity and its norm, per sorted
// position (the paper's linker).
__global__ void k_sorted_u(int64_t np, int64_t n, const int32_t* __restrict__ sorig, const float* __restrict__ vx,
                           const float* __restrict__ vy, const float* __restrict__ vz, const float* __restrict__ vbar,
                           double* __restrict__ su0, double* __restrict__ su1, double* __restrict__ su2,
                           double* __restrict__ ss) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int32_t i = sorig[p];
    const double u0 = (double)vx[i] - (double)vbar[3 * (int64_t)i];  // particle-major
    const double u1 = (double)vy[i] - (double)vbar[3 * (int64_t)i + 1];
    const double u2 = (double)vz[i] - (double)vbar[3 * (int64_t)i + 2];
    su0[p] = u0;
    su1[p] = u1;
    su2[p] = u2;
    ss[p] = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
}

struct SubLink {
    const double *u0, *u1, *u2, *s;  // per sorted position
    double Vr, cos_op;
};

// PAPER = false: Eq. fof6d; true: Eq. linkingcriteria (sub.* used, ellv not).
template <bool HALF, bool PAPER>
__global__ __launch_bounds__(256) void k_link6d(int64_t np, const ckey_t* __restrict__ key,
                                                const uint32_t* __restrict__ sx, const uint32_t* __restrict__ sy,
                                                const uint32_t* __restrict__ sz, const float* __restrict__ svx,
                                                const float* __restrict__ svy, const float* __restrict__ svz,
                                                const int32_t* __restrict__ shost, const double* __restrict__ ellv,
                                                const uint32_t* __restrict__ cell_start,
                                                const ckey_t* __restrict__ hkeys, const uint32_t* __restrict__ hvals,
                                                uint32_t hmask, int b, int gb, double ell2, int* parent,
                                                unsigned xchunk, SubLink sub) {
    const int64_t p = (int64_t)xcd_swizzle(blockIdx.x, gridDim.x, xchunk) * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const ckey_t k = key[p];
    const int nc = 1 << b;
    const int cx = (int)(k & (nc - 1)), cy = (int)((k >> b) & (nc - 1)), cz = (int)(k >> (2 * b));
    const int px = (int)sx[p], py = (int)sy[p], pz = (int)sz[p];
    const double vpx = (double)svx[p], vpy = (double)svy[p], vpz = (double)svz[p];
    const int hp = shost[p];
    const double ev = PAPER ? 1.0 : ellv[hp];
    const double ev2 = ev * ev;
    double up0 = 0, up1 = 0, up2 = 0, sp = 0;
    if constexpr (PAPER) {
        up0 = sub.u0[p];
        up1 = sub.u1[p];
        up2 = sub.u2[p];
        sp = sub.s[p];
        if (!(sp > 0)) return;  // no direction: links nothing
    }
    // t = d2/ell2 + dv2/ev2 is formed with reciprocals first; that differs
    // from the divided form by a few ulps, so only t within 1e-9 of 1 needs
    // the divided form itself
    const double rl2 = 1.0 / ell2, rv2 = 1.0 / ev2;
    // p's root, refreshed only when a partner's differs (components only
    // merge), so a link inside one component costs a single find
    int rp = uf_find(parent, (int)p);
    auto join = [&](int q) __attribute__((always_inline)) {
        const int rq = uf_find(parent, q);
        if (rq == rp) return;
        rp = uf_find(parent, rp);
        if (rp != rq) uf_union(parent, rp, rq);
    };
    ckey_t seen[HALF ? 1 : 27];
    int nseen = 0;
    for (int o = 0; o < 27; ++o) {
        const int dz = o / 9 - 1, dy = (o / 3) % 3 - 1, dx = o % 3 - 1;
        const int lin = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
        if (HALF && lin < 13) continue;
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
        if (((nk == k) || !HALF) && s <= (uint32_t)p) s = (uint32_t)p + 1;
        for (uint32_t q = s; q < e; ++q) {
            const int ddx = min_image((int)sx[q] - px, gb);
            const int ddy = min_image((int)sy[q] - py, gb);
            const int ddz = min_image((int)sz[q] - pz, gb);
            const double d2 = (double)ddx * ddx + (double)ddy * ddy + (double)ddz * ddz;
            // d2 >= ell2 makes the rounded d2/ell2 >= 1 and so t >= 1: no link
            if (d2 >= ell2 || shost[q] != hp) continue;
            if constexpr (PAPER) {
                const double sq = sub.s[q];
                if (!(sq > 0) || !(sp <= sub.Vr * sq && sq <= sub.Vr * sp)) continue;
                const double dot = up0 * sub.u0[q] + up1 * sub.u1[q] + up2 * sub.u2[q];
                if (dot >= sub.cos_op * (sp * sq)) join((int)q);
                continue;
            }
            const double ax = vpx - (double)svx[q], ay = vpy - (double)svy[q], az = vpz - (double)svz[q];
            const double dv2 = ax * ax + ay * ay + az * az;
            const double ta = d2 * rl2 + dv2 * rv2;
            bool link = ta < 1.0 - 1e-9;
            if (!link && ta <= 1.0 + 1e-9) link = d2 / ell2 + dv2 / ev2 < 1.0;
            if (link) join((int)q);
        }
    }
}


// ---- the linking sweep by tiles ---------------------------------------------
// One wavefront per tile of (at most) 64 participants of one cell, lane =
// participant p.  The own cell (candidates after p) and its 13 forward
// neighbour cells are staged through LDS 64 candidates at a time --
// coordinates, velocity, host, the paper linker's relative velocity, and the
// candidate's union-find root as read at staging -- so each candidate is
// fetched once per wavefront and read by all lanes from LDS.  An FP32
// distance prefilter (coordinate differences are exact integers below 2^21,
// the rounded square sum lies within 2e-7 of the exact one) passes every
// candidate that may lie inside the linking length; those get the exact
// integer d2 and the FP64 predicate of k_link6d.  A candidate's parent, read
// at staging, is one of its ancestors: equal to p's root, the pair is already
// joined and no further global access is needed.

// tiles of 64 participants per cell
// Tiles of cells with at least HEAVY_CELL participants (subhalo cores, whose
// tiles carry thousands of candidates each) come first in the list, so they
// start with the launch instead of finishing after it: cnt[c] counts a heavy
// cell's tiles, cnt[ncell + c] a light one's, and one scan over both halves
// gives every cell its first tile.
constexpr uint32_t HEAVY_CELL = 64;

__global__ void k_tile_count(int64_t ncell, const uint32_t* __restrict__ cell_start, uint32_t* __restrict__ cnt) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const uint32_t m = cell_start[c + 1] - cell_start[c];
    const uint32_t nt = (m + 63) >> 6;
    cnt[c] = m >= HEAVY_CELL ? nt : 0;
    cnt[ncell + c] = m >= HEAVY_CELL ? 0 : nt;
}

__global__ void k_tile_write(int64_t ncell, const uint32_t* __restrict__ cell_start, const uint32_t* __restrict__ toff,
                             int2* __restrict__ tiles) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const uint32_t s = cell_start[c], e = cell_start[c + 1];
    uint32_t t = e - s >= HEAVY_CELL ? toff[c] : toff[ncell + c];
    for (uint32_t q = s; q < e; q += 64) tiles[t++] = make_int2((int)c, (int)q);
}

template <bool PAPER>
__global__ __launch_bounds__(64) void k_link6d_tile(const int2* __restrict__ tiles, const uint32_t* __restrict__ ntiles,
                                                    const ckey_t* __restrict__ key, const uint32_t* __restrict__ sx,
                                                    const uint32_t* __restrict__ sy, const uint32_t* __restrict__ sz,
                                                    const float* __restrict__ svx, const float* __restrict__ svy,
                                                    const float* __restrict__ svz, const int32_t* __restrict__ shost,
                                                    const double* __restrict__ ellv,
                                                    const uint32_t* __restrict__ cell_start,
                                                    const ckey_t* __restrict__ hkeys, const uint32_t* __restrict__ hvals,
                                                    uint32_t hmask, int b, int gb, double ell2, int* parent,
                                                    unsigned xchunk, SubLink sub) {
    __shared__ __align__(16) int cxs[64];
    __shared__ __align__(16) int cys[64];
    __shared__ __align__(16) int czs[64];
    __shared__ __align__(16) int crt[64];
    __shared__ int chs[64], cq[64];
    __shared__ float cvx[64], cvy[64], cvz[64];
    __shared__ double cu0[PAPER ? 64 : 1], cu1[PAPER ? 64 : 1], cu2[PAPER ? 64 : 1], cs_[PAPER ? 64 : 1];
    const uint32_t t = xcd_swizzle(blockIdx.x, gridDim.x, xchunk);
    if (t >= ntiles[0]) return;
    const int lane = (int)threadIdx.x;
    const int2 tl = tiles[t];
    const uint32_t q0 = (uint32_t)tl.y, cend = cell_start[tl.x + 1];
    const uint32_t p = q0 + (uint32_t)lane;
    bool valid = p < cend;
    const ckey_t k = key[q0];
    const int nc = 1 << b;
    const int cx = (int)(k & (nc - 1)), cy = (int)((k >> b) & (nc - 1)), cz = (int)(k >> (2 * b));
    // lane o < 14: the candidate range of segment o -- the 13 forward
    // neighbour cells, then the own cell from the tile's first participant --
    // all looked up at once
    uint32_t seg_s = 0, seg_n = 0;
    if (lane < 14) {
        if (lane == 13) {
            seg_s = q0;
            seg_n = cend - q0;
        } else {
            const int o = 14 + lane;  // forward offsets 14..26
            const int dz = o / 9 - 1, dy = (o / 3) % 3 - 1, dx = o % 3 - 1;
            const uint32_t nx = (uint32_t)((cx + dx + nc) & (nc - 1));
            const uint32_t ny = (uint32_t)((cy + dy + nc) & (nc - 1));
            const uint32_t nz = (uint32_t)((cz + dz + nc) & (nc - 1));
            const int c2 = hash_find(hkeys, hvals, hmask, cell_key(nx, ny, nz, b));
            if (c2 >= 0) {
                seg_s = cell_start[c2];
                seg_n = cell_start[c2 + 1] - seg_s;
            }
        }
    }
    // exclusive prefix of the segment lengths over lanes 0..13
    uint32_t incl = seg_n;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    const uint32_t total = __shfl(incl, 13, 64);
    const uint32_t seg_b = incl - seg_n;  // first candidate number of this lane's segment
    const uint32_t own_b = __shfl(seg_b, 13, 64);

    const int px = valid ? (int)sx[p] : 0, py = valid ? (int)sy[p] : 0, pz = valid ? (int)sz[p] : 0;
    const double vpx = valid ? (double)svx[p] : 0.0, vpy = valid ? (double)svy[p] : 0.0,
                 vpz = valid ? (double)svz[p] : 0.0;
    const int hp = valid ? shost[p] : -1;
    const double ev = (PAPER || !valid) ? 1.0 : ellv[hp];
    const double ev2 = ev * ev;
    double up0 = 0, up1 = 0, up2 = 0, sp = 0;
    if constexpr (PAPER) {
        if (valid) {
            up0 = sub.u0[p];
            up1 = sub.u1[p];
            up2 = sub.u2[p];
            sp = sub.s[p];
        }
        if (!(sp > 0)) valid = false;  // no direction: links nothing
    }
    const double rl2 = 1.0 / ell2, rv2 = 1.0 / ev2;
    // no candidate with an FP32 square sum above this lies within ell
    const float ellf = (float)(ell2 * (1.0 + 1e-6)) + 1.0f;
    int rp = valid ? uf_find(parent, (int)p) : -1;
    // Near the box faces a forward neighbour can sit across the periodic
    // boundary; elsewhere the plain coordinate differences are the minimum
    // images (cells span far less than half the box).
    const int ncm = nc - 1;
    const bool wrap = cx == 0 || cx == ncm || cy == 0 || cy == ncm || cz == ncm;
    for (uint32_t c0 = 0; c0 < total; c0 += 64) {
        const uint32_t c = c0 + (uint32_t)lane;
        // the segment holding candidate c: the last lane o < 14 whose first
        // candidate number is <= c (empty segments share numbers); every lane
        // takes part in the shuffles, lanes past the end load nothing
        int sg = 0;
#pragma unroll
        for (int o = 1; o < 14; ++o) {
            const uint32_t bo = __shfl(seg_b, o, 64);
            if (bo <= c) sg = o;
        }
        const uint32_t q = __shfl(seg_s, sg, 64) + (c - __shfl(seg_b, sg, 64));
        __builtin_amdgcn_wave_barrier();
        if (c < total) {
            cq[lane] = (int)q;
            cxs[lane] = (int)sx[q];
            cys[lane] = (int)sy[q];
            czs[lane] = (int)sz[q];
            chs[lane] = shost[q];
            cvx[lane] = svx[q];
            cvy[lane] = svy[q];
            cvz[lane] = svz[q];
            // q's root as of staging (one find per candidate and chunk, all
            // lanes at once): once a core has merged, a linked pair then
            // matches the participant's root without a find of its own
            crt[lane] = uf_find(parent, (int)q);
            if constexpr (PAPER) {
                cu0[lane] = sub.u0[q];
                cu1[lane] = sub.u1[q];
                cu2[lane] = sub.u2[q];
                cs_[lane] = sub.s[q];
            }
        }
        __builtin_amdgcn_wave_barrier();
        const int m = (int)min(64u, total - c0);
        if (!valid) continue;
        rp = uf_find(parent, rp);  // as fresh as the staged roots
        // pass 1, no divergence: a bit per staged candidate whose FP32
        // squared distance may lie within ell (differences are exact
        // integers below 2^22; the rounded sum is within 2e-7 of the exact
        // one, which ellf covers) and whose staged root is not the lane's
        // (a link inside one component changes nothing); pass 2 takes the
        // marked ones exactly
        uint32_t tk[2] = {0u, 0u};
#pragma unroll
        for (int b4 = 0; b4 < 16; ++b4) {
            if (4 * b4 < m) {
                const int4 X = *reinterpret_cast<const int4*>(&cxs[4 * b4]);
                const int4 Y = *reinterpret_cast<const int4*>(&cys[4 * b4]);
                const int4 Z = *reinterpret_cast<const int4*>(&czs[4 * b4]);
                const int4 RT = *reinterpret_cast<const int4*>(&crt[4 * b4]);
                const int xs[4] = {X.x, X.y, X.z, X.w}, ys[4] = {Y.x, Y.y, Y.z, Y.w}, zs[4] = {Z.x, Z.y, Z.z, Z.w};
                const int rts[4] = {RT.x, RT.y, RT.z, RT.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    int dx = xs[u] - px, dy = ys[u] - py, dz = zs[u] - pz;
                    if (wrap) {
                        dx = min_image(dx, gb);
                        dy = min_image(dy, gb);
                        dz = min_image(dz, gb);
                    }
                    const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
                    const int bit = 4 * b4 + u;
                    if (fmaf(fx, fx, fmaf(fy, fy, fz * fz)) <= ellf && rts[u] != rp) tk[bit >> 5] |= 1u << (bit & 31);
                }
            }
        }
        uint64_t take = ((uint64_t)tk[1] << 32) | tk[0];
        if (m < 64) take &= (uint64_t(1) << m) - 1;
        while (take) {
            const int j = __builtin_ctzll(take);
            take &= take - 1;
            const int qq = cq[j];
            // own cell: only the candidates after p
            if (c0 + (uint32_t)j >= own_b && (uint32_t)qq <= p) continue;
            if (chs[j] != hp) continue;
            const int ddx = min_image(cxs[j] - px, gb);
            const int ddy = min_image(cys[j] - py, gb);
            const int ddz = min_image(czs[j] - pz, gb);
            const double d2 = (double)ddx * ddx + (double)ddy * ddy + (double)ddz * ddz;
            if (d2 >= ell2) continue;
            bool link;
            if constexpr (PAPER) {
                const double sq = cs_[j];
                if (!(sq > 0) || !(sp <= sub.Vr * sq && sq <= sub.Vr * sp)) continue;
                const double dot = up0 * cu0[j] + up1 * cu1[j] + up2 * cu2[j];
                link = dot >= sub.cos_op * (sp * sq);
            } else {
                const double ax = vpx - (double)cvx[j], ay = vpy - (double)cvy[j], az = vpz - (double)cvz[j];
                const double dv2 = ax * ax + ay * ay + az * az;
                const double ta = d2 * rl2 + dv2 * rv2;
                link = ta < 1.0 - 1e-9;
                if (!link && ta <= 1.0 + 1e-9) link = d2 / ell2 + dv2 / ev2 < 1.0;
            }
            if (!link || crt[j] == rp) continue;
            const int rq = uf_find(parent, qq);
            if (rq == rp) continue;
            rp = uf_find(parent, rp);
            if (rp != rq) uf_union(parent, rp, rq);
            rp = uf_find(parent, rp);
        }
    }
}

// ---- second, relaxed stage of the paper's linker --------------------------
// Sizes of the first-stage components (labels are particle indices).
__global__ void k_label_sizes(int64_t n, const int32_t* __restrict__ label1, int* __restrict__ size) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && label1[i] >= 0) atomicAdd(&size[label1[i]], 1);
}

// A member of a candidate group must be a relaxed participant.
__global__ void k_check_tagged(int64_t n, const int32_t* __restrict__ label1, const int* __restrict__ size,
                               int n_min, const uint32_t* __restrict__ flag, int* __restrict__ bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int l = label1[i];
    if (l >= 0 && size[l] >= n_min && !flag[i]) atomicOr(bad, 1);
}

__global__ void k_first_tags(int64_t np, const int32_t* __restrict__ sorig, const int32_t* __restrict__ label1,
                             const int* __restrict__ size, int n_min, int32_t* __restrict__ tag) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int l = label1[sorig[p]];
    tag[p] = (l >= 0 && size[l] >= n_min) ? l : -1;
}

// The relaxed criteria of the paper's linker between sorted positions p, q
// (same host and d2 < ell2 already known).
__device__ __forceinline__ bool relaxed_link(const SubLink& sub, double up0, double up1, double up2, double sp, int q) {
    const double sq = sub.s[q];
    if (!(sp > 0) || !(sq > 0) || !(sp <= sub.Vr * sq && sq <= sub.Vr * sp)) return false;
    const double dot = up0 * sub.u0[q] + up1 * sub.u1[q] + up2 * sub.u2[q];
    return dot >= sub.cos_op * (sp * sq);
}

// Visits every participant q != p in the 27 cells around p's cell (each once)
// that shares p's host, lies within ell2 and meets the relaxed criteria.
template <class F>
__device__ __forceinline__ void for_relaxed(int64_t p, const ckey_t* __restrict__ key, const uint32_t* __restrict__ sx,
                                            const uint32_t* __restrict__ sy, const uint32_t* __restrict__ sz,
                                            const int32_t* __restrict__ shost, const uint32_t* __restrict__ cell_start,
                                            const ckey_t* __restrict__ hkeys, const uint32_t* __restrict__ hvals,
                                            uint32_t hmask, int b, int gb, double ell2, const SubLink& sub, F&& visit) {
    const ckey_t k = key[p];
    const int nc = 1 << b;
    const int cx = (int)(k & (nc - 1)), cy = (int)((k >> b) & (nc - 1)), cz = (int)(k >> (2 * b));
    const int px = (int)sx[p], py = (int)sy[p], pz = (int)sz[p];
    const int hp = shost[p];
    const double up0 = sub.u0[p], up1 = sub.u1[p], up2 = sub.u2[p], sp = sub.s[p];
    if (!(sp > 0)) return;
    // with fewer than 3 cells a side the 27 offsets repeat cells (at most 8
    // distinct ones): a bit per cell keeps each visit single
    uint32_t seen = 0;
    for (int o = 0; o < 27; ++o) {
        const int dz = o / 9 - 1, dy = (o / 3) % 3 - 1, dx = o % 3 - 1;
        const uint32_t nx = (uint32_t)((cx + dx + nc) & (nc - 1));
        const uint32_t ny = (uint32_t)((cy + dy + nc) & (nc - 1));
        const uint32_t nz = (uint32_t)((cz + dz + nc) & (nc - 1));
        const ckey_t nk = cell_key(nx, ny, nz, b);
        if (nc < 3) {
            const uint32_t bit = 1u << (nx + 2 * ny + 4 * nz);
            if (seen & bit) continue;
            seen |= bit;
        }
        const int c = hash_find(hkeys, hvals, hmask, nk);
        if (c < 0) continue;
        for (uint32_t q = cell_start[c]; q < cell_start[c + 1]; ++q) {
            if ((int64_t)q == p) continue;
            const int ddx = min_image((int)sx[q] - px, gb);
            const int ddy = min_image((int)sy[q] - py, gb);
            const int ddz = min_image((int)sz[q] - pz, gb);
            const double d2 = (double)ddx * ddx + (double)ddy * ddy + (double)ddz * ddz;
            if (d2 >= ell2 || shost[q] != hp) continue;
            if (relaxed_link(sub, up0, up1, up2, sp, (int)q)) visit((int)q);
        }
    }
}

// Synchronous growth rounds: an untagged participant takes the smallest tag
// among its relaxed neighbours tagged in the previous round.

// The rounds are pushed from the frontier (the particles tagged in the
// previous round).  An untagged participant can only border particles
// tagged in the previous round (a tagged neighbour of an earlier round would
// have tagged it already), and the relaxed link is symmetric, so the
// smallest tag pushed to it is the one it would pull.
__global__ void k_frontier_init(int64_t np, const int32_t* __restrict__ tag, int32_t* __restrict__ prop,
                                int32_t* __restrict__ front, int* __restrict__ nfront) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < np;
    if (valid) prop[p] = INT_MAX;
    wave_append(nfront, front, valid && tag[p] >= 0, (int32_t)p);
}

__global__ __launch_bounds__(256) void k_grow_push(int nf, const int32_t* __restrict__ front, const ckey_t* __restrict__ key,
                                                   const uint32_t* __restrict__ sx, const uint32_t* __restrict__ sy,
                                                   const uint32_t* __restrict__ sz, const int32_t* __restrict__ shost,
                                                   const uint32_t* __restrict__ cell_start,
                                                   const ckey_t* __restrict__ hkeys, const uint32_t* __restrict__ hvals,
                                                   uint32_t hmask, int b, int gb, double ell2, SubLink sub,
                                                   const int32_t* __restrict__ tag, int32_t* __restrict__ prop) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int p = front[i];
    const int t = tag[p];
    for_relaxed(p, key, sx, sy, sz, shost, cell_start, hkeys, hvals, hmask, b, gb, ell2, sub, [&](int q) {
        if (tag[q] < 0) atomicMin(&prop[q], t);
    });
}

__global__ void k_grow_apply(int64_t np, int32_t* __restrict__ tag, int32_t* __restrict__ prop,
                             int32_t* __restrict__ front, int* __restrict__ nfront) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = q < np;
    const int v = valid ? prop[q] : INT_MAX;
    const bool got = v != INT_MAX;
    if (got) {
        tag[q] = v;
        prop[q] = INT_MAX;
    }
    wave_append(nfront, front, got, (int32_t)q);
}

// Relaxed links between different groups (each unordered link once, from its
// lower position): counted, or written as (lower tag, upper tag) keys with the
// first-stage sizes of both groups.
template <bool EMIT>
__global__ __launch_bounds__(256) void k_cross(int64_t np, const ckey_t* __restrict__ key,
                                               const uint32_t* __restrict__ sx, const uint32_t* __restrict__ sy,
                                               const uint32_t* __restrict__ sz, const int32_t* __restrict__ shost,
                                               const uint32_t* __restrict__ cell_start,
                                               const ckey_t* __restrict__ hkeys, const uint32_t* __restrict__ hvals,
                                               uint32_t hmask, int b, int gb, double ell2, SubLink sub,
                                               const int32_t* __restrict__ tag, const int* __restrict__ size,
                                               unsigned long long* __restrict__ count, int64_t cap,
                                               uint64_t* __restrict__ pairs, int2* __restrict__ sizes) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int a = tag[p];
    if (a < 0) return;
    for_relaxed(p, key, sx, sy, sz, shost, cell_start, hkeys, hvals, hmask, b, gb, ell2, sub, [&](int q) {
        const int c = tag[q];
        if ((int64_t)q <= p || c < 0 || c == a) return;
        const unsigned long long at = atomicAdd(count, 1ull);
        if (EMIT && (int64_t)at < cap) {
            const int lo = min(a, c), hi = max(a, c);
            pairs[at] = ((uint64_t)(uint32_t)lo << 32) | (uint32_t)hi;
            sizes[at] = make_int2(size[lo], size[hi]);
        }
    });
}

__global__ void k_remap_tags(int64_t np, const int* __restrict__ remap, int32_t* __restrict__ tag,
                             const int32_t* __restrict__ sorig, int* __restrict__ low) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int t = tag[p];
    if (t < 0) return;
    const int r = remap[t];
    tag[p] = r;
    atomicMin(&low[r], sorig[p]);
}

__global__ void k_grow_labels(int64_t np, const int32_t* __restrict__ tag, const int32_t* __restrict__ sorig,
                              const int* __restrict__ low, int32_t* __restrict__ label) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int t = tag[p];
    if (t >= 0) label[sorig[p]] = low[t];
}

__global__ void k_iota_i(int64_t n, int* p) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int)i;
}

__global__ void k_compress_min(int64_t np, int* parent, const int32_t* __restrict__ sorig, int* __restrict__ mn) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < np;
    int r = valid ? (int)p : 0;
    if (valid) {
        while (parent[r] != r) r = parent[r];
        parent[p] = r;
    }
    // every lane takes part: neighbours in cell order mostly share a root
    wave_atomic_min(mn, r, valid ? sorig[p] : 0x7FFFFFFF, valid);
}

__global__ void k_label6(int64_t np, const int* __restrict__ parent, const int32_t* __restrict__ sorig,
                         const int* __restrict__ mn, int32_t* __restrict__ label6) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    label6[sorig[p]] = mn[parent[p]];
}

}  // namespace
}  // namespace vr

using namespace vr;

extern "C" int vr_host_ellv(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts, const int32_t* host_offsets,
                            const int32_t* host_members, double alpha_v, double* ellv_host, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_particles(ctx, p, true);
    if (rc) return rc;
    if ((rc = check_hosts(ctx, n_hosts, host_offsets, host_members))) return rc;
    if (!(alpha_v > 0)) return set_err(ctx, VR_ERR_INVALID_ARG, "alpha_v must be positive");
    if (n_hosts == 0) return VR_OK;
    if (!ellv_host) return set_err(ctx, VR_ERR_INVALID_ARG, "ellv_host is NULL");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> off(n_hosts + 1);
    int rc0 = copy_to_host(ctx, off.data(), host_offsets, (n_hosts + 1) * sizeof(int32_t), st);
    if (rc0) return rc0;
    if (off[0] != 0) return set_err(ctx, VR_ERR_INVALID_ARG, "host_offsets[0] must be 0");
    std::vector<int4> chunks;
    std::vector<int> coff(n_hosts + 1, 0);
    for (int h = 0; h < n_hosts; ++h) {
        if (off[h + 1] <= off[h] || off[h + 1] > p->n)
            return set_err(ctx, VR_ERR_INVALID_ARG, "host %d is empty or out of range", h);
        for (int s = off[h]; s < off[h + 1]; s += ELLV_CHUNK)
            chunks.push_back(make_int4(h, s, std::min(off[h + 1], s + ELLV_CHUNK), 0));
        coff[h + 1] = (int)chunks.size();
    }
    const int nch = (int)chunks.size();
    VR_WS(chunks_d, ctx, int4, WS_D4, nch);
    VR_WS(coff_d, ctx, int, WS_D5, n_hosts + 1);
    VR_WS(part, ctx, double, WS_D6, (int64_t)nch * ELLV_PART);
    {
        // both tables through the pinned upload buffer: no wait here
        const size_t bc = (size_t)nch * sizeof(int4), bo = (size_t)(n_hosts + 1) * sizeof(int);
        char* up = static_cast<char*>(upload_begin(ctx, bc + bo));
        if (!up) return VR_ERR_HIP;
        std::memcpy(up, chunks.data(), bc);
        std::memcpy(up + bc, coff.data(), bo);
        VR_HIP(ctx, hipMemcpyAsync(chunks_d, up, bc, hipMemcpyHostToDevice, st));
        VR_HIP(ctx, hipMemcpyAsync(coff_d, up + bc, bo, hipMemcpyHostToDevice, st));
        if (int rc1 = upload_end(ctx, st)) return rc1;
    }
    hipLaunchKernelGGL(k_ellv_sums, dim3(nch), dim3(256), 0, st, chunks_d, host_members, host_offsets, p->vx, p->vy,
                       p->vz, p->mass, p->mass_value, part);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_ellv_final, dim3(grid_for(n_hosts, 256)), dim3(256), 0, st, n_hosts, coff_d, part, alpha_v,
                       ellv_host);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

namespace {

// Both linkers: sub == nullptr gives Eq. fof6d with ellv_host, otherwise
// Eq. linkingcriteria with sub->vbar, Vr, cos_op.
struct SubArgs {
    const float* vbar;
    double Vr, cos_op;
};

int link_outliers(vr_ctx* ctx, const vr_particles* p, const int32_t* host_of, const double* ellv_host,
                  int32_t n_hosts, double ellx_s, const float* R, float R_threshold, int32_t* label6,
                  const SubArgs* sub, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_particles(ctx, p, true);
    if (rc) return rc;
    const int gb = p->grid_bits;
    const double u = ellx_s * ldexp(1.0, gb) / p->box;
    if (!(u > 0) || !(u < ldexp(1.0, gb - 1)))
        return set_err(ctx, VR_ERR_INVALID_ARG, "ellx_s must satisfy 0 < ellx_s < box/2");
    if (n_hosts < 0) return set_err(ctx, VR_ERR_INVALID_ARG, "n_hosts < 0");
    const int64_t n = p->n;
    if (n == 0) return VR_OK;
    if (!host_of || !label6 || (!sub && n_hosts > 0 && !ellv_host) || (sub && (!sub->vbar || !R)))
        return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    if (!sub && n_hosts > 0) {
        std::vector<double> ev(n_hosts);
        if ((rc = copy_to_host(ctx, ev.data(), ellv_host, n_hosts * sizeof(double), st))) return rc;
        for (int h = 0; h < n_hosts; ++h)
            if (!(ev[h] > 0) || !std::isfinite(ev[h]))
                return set_err(ctx, VR_ERR_INVALID_ARG, "ellv_host[%d] = %g is not a positive number", h, ev[h]);
    }
    const double ell2 = u * u;
    VR_WS(flag, ctx, uint32_t, WS_C0, n);
    VR_WS(pos, ctx, uint32_t, WS_C1, n);
    VR_WS(bad, ctx, int, WS_FLAG2, 4);
    VR_WS(tot, ctx, uint32_t, WS_C9, 4);
    rc = fill_i32(ctx, bad, 0, 1, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_participants, dim3(grid_for(n, 256)), dim3(256), 0, st, n, host_of, R, R_threshold, n_hosts,
                       flag, bad);
    VR_LAUNCH_CHECK(ctx);
    rc = scan_u32(ctx, flag, pos, n, tot, st);
    if (rc) return rc;
    int32_t* hostpin = reinterpret_cast<int32_t*>(ctx->pinned);
    VR_HIP(ctx, hipMemcpyAsync(hostpin, tot, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    VR_HIP(ctx, hipMemcpyAsync(hostpin + 1, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    VR_HIP(ctx, hipStreamSynchronize(st));
    const int64_t np = (uint32_t)hostpin[0];
    if (hostpin[1]) return set_err(ctx, VR_ERR_INVALID_ARG, "host_of holds a host id >= n_hosts");
    rc = fill_i32(ctx, label6, -1, n, st);
    if (rc) return rc;
    if (np == 0) return VR_OK;
    VR_WS(cx, ctx, uint32_t, WS_C2, np);
    VR_WS(cy, ctx, uint32_t, WS_C3, np);
    VR_WS(cz, ctx, uint32_t, WS_C4, np);
    VR_WS(orig, ctx, int32_t, WS_C5, np);
    hipLaunchKernelGGL(k_compact_part, dim3(grid_for(n, 256)), dim3(256), 0, st, n, flag, pos, p->qx, p->qy, p->qz, cx,
                       cy, cz, orig);
    VR_LAUNCH_CHECK(ctx);
    int s = 0;
    while ((double)(1 << s) < u && s < gb) ++s;
    CellList cl;
    rc = build_cell_list(ctx, np, cx, cy, cz, gb, s, cl, st);
    if (rc) return rc;
    VR_WS(sorig, ctx, int32_t, WS_C6, np);
    VR_WS(svx, ctx, float, WS_C7, np);
    VR_WS(svy, ctx, float, WS_C8, np);
    VR_WS(svz, ctx, float, WS_D0, np);
    VR_WS(shost, ctx, int32_t, WS_D1, np);
    VR_WS(parent, ctx, int, WS_D2, np);
    VR_WS(mn, ctx, int, WS_D3, np);
    hipLaunchKernelGGL(k_sorted_attrs, dim3(grid_for(np, 256)), dim3(256), 0, st, np, cl.idx, orig, p->vx, p->vy,
                       p->vz, host_of, sorig, svx, svy, svz, shost);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_iota_i, dim3(grid_for(np, 256)), dim3(256), 0, st, np, parent);
    VR_LAUNCH_CHECK(ctx);
    SubLink sl{nullptr, nullptr, nullptr, nullptr, 1.0, 1.0};
    if (sub) {
        VR_WS(su0, ctx, double, WS_D4, np);
        VR_WS(su1, ctx, double, WS_D5, np);
        VR_WS(su2, ctx, double, WS_D6, np);
        VR_WS(ss, ctx, double, WS_D7, np);
        hipLaunchKernelGGL(k_sorted_u, dim3(grid_for(np, 256)), dim3(256), 0, st, np, n, sorig, p->vx, p->vy, p->vz,
                           sub->vbar, su0, su1, su2, ss);
        VR_LAUNCH_CHECK(ctx);
        sl = SubLink{su0, su1, su2, ss, sub->Vr, sub->cos_op};
    }
    const int b = gb - s;
    const unsigned xc = (unsigned)ctx->xcd_chunk;
    const dim3 g(grid_for(np, 256));
#define VR_LINK6D(HALF, PAPER)                                                                                    \
    VR_TIMED(ctx, sub ? "fof_link_sub" : "fof_link6d", st, np,                                                  \
             hipLaunchKernelGGL((k_link6d<HALF, PAPER>), g, dim3(256), 0, st, np, cl.key, cl.sx, cl.sy, cl.sz, svx, \
                                svy, svz, shost, ellv_host, cl.cell_start, cl.hkeys, cl.hvals, cl.hmask, b, gb, ell2, \
                                parent, xc, sl))
    if ((1 << b) >= 4) {
        // tiles of 64 participants per cell: at most ncell + np / 64 of them
        const int64_t ncell = cl.n_cells;
        const int64_t tmax = ncell + (np + 63) / 64;
        VR_WS(tcnt, ctx, uint32_t, WS_D8, 2 * ncell + 1);
        VR_WS(ttot, ctx, uint32_t, WS_D9, 4);
        VR_WS(tiles, ctx, int2, WS_B7, tmax);
        hipLaunchKernelGGL(k_tile_count, dim3(grid_for(ncell, 256)), dim3(256), 0, st, ncell, cl.cell_start, tcnt);
        VR_LAUNCH_CHECK(ctx);
        if ((rc = scan_u32(ctx, tcnt, tcnt, 2 * ncell, ttot, st))) return rc;
        hipLaunchKernelGGL(k_tile_write, dim3(grid_for(ncell, 256)), dim3(256), 0, st, ncell, cl.cell_start, tcnt, tiles);
        VR_LAUNCH_CHECK(ctx);
#define VR_LINK6T(PAPER)                                                                                           \
        VR_TIMED(ctx, sub ? "fof_link_sub" : "fof_link6d", st, np,                                               \
                 hipLaunchKernelGGL((k_link6d_tile<PAPER>), dim3((unsigned)tmax), dim3(64), 0, st, tiles, ttot, cl.key, \
                                    cl.sx, cl.sy, cl.sz, svx, svy, svz, shost, ellv_host, cl.cell_start, cl.hkeys,   \
                                    cl.hvals, cl.hmask, b, gb, ell2, parent, xc, sl))
        if (sub) VR_LINK6T(true); else VR_LINK6T(false);
#undef VR_LINK6T
    } else {
        if (sub) VR_LINK6D(false, true); else VR_LINK6D(false, false);
    }
#undef VR_LINK6D
    VR_LAUNCH_CHECK(ctx);
    rc = fill_i32(ctx, mn, 0x7FFFFFFF, np, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_compress_min, dim3(grid_for(np, 256)), dim3(256), 0, st, np, parent, sorig, mn);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_label6, dim3(grid_for(np, 256)), dim3(256), 0, st, np, parent, sorig, mn, label6);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

}  // namespace

extern "C" int vr_fof6d(vr_ctx* ctx, const vr_particles* p, const int32_t* host_of, const double* ellv_host,
                        int32_t n_hosts, double ellx_s, const float* R, float R_threshold, int32_t* label6,
                        void* stream) {
    return link_outliers(ctx, p, host_of, ellv_host, n_hosts, ellx_s, R, R_threshold, label6, nullptr, stream);
}

extern "C" int vr_fof_sub(vr_ctx* ctx, const vr_particles* p, const int32_t* host_of, int32_t n_hosts,
                          const float* vbar, double ellx_s, const float* L, float L_threshold, double Vr,
                          double cos_theta_op, int32_t* label, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    if (!(Vr >= 1.0) || !(cos_theta_op >= -1.0 && cos_theta_op <= 1.0))
        return set_err(ctx, VR_ERR_INVALID_ARG, "need Vr >= 1 and -1 <= cos_theta_op <= 1");
    const SubArgs sa{vbar, Vr, cos_theta_op};
    return link_outliers(ctx, p, host_of, nullptr, n_hosts, ellx_s, L, L_threshold, label, &sa, stream);
}

namespace {
__global__ void k_scatter_i(int k, const int* __restrict__ at, const int* __restrict__ val, int* __restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) dst[at[i]] = val[i];
}
}  // namespace

extern "C" int vr_sub_grow(vr_ctx* ctx, const vr_particles* p, const int32_t* host_of, int32_t n_hosts,
                           const float* vbar, const float* L, float L_threshold, double gamma_L, double ellx_s,
                           double gamma_x, double Vr, double gamma_V, double cos_op_relaxed, double f_merge,
                           int32_t n_min, const int32_t* label1, int32_t* label_out, int32_t* rounds, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_particles(ctx, p, true);
    if (rc) return rc;
    if (!(gamma_L >= 1.0) || !(gamma_x >= 1.0) || !(gamma_V >= 1.0) || !(Vr >= 1.0) || n_min < 1 ||
        !(cos_op_relaxed >= -1.0 && cos_op_relaxed <= 1.0) || !(f_merge >= 0) || n_hosts < 0)
        return set_err(ctx, VR_ERR_INVALID_ARG, "need gammas >= 1, Vr >= 1, n_min >= 1, |cos| <= 1, f_merge >= 0");
    const int gb = p->grid_bits;
    const double u = gamma_x * ellx_s * ldexp(1.0, gb) / p->box;
    if (!(u > 0) || !(u < ldexp(1.0, gb - 1)))
        return set_err(ctx, VR_ERR_INVALID_ARG, "the relaxed linking length must lie in (0, box/2)");
    const int64_t n = p->n;
    if (rounds) *rounds = 0;
    if (n == 0) return VR_OK;
    if (!host_of || !vbar || !L || !label1 || !label_out) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const double ell2 = u * u;
    const float Lth2 = (float)((double)L_threshold / gamma_L);
    VR_WS(flag, ctx, uint32_t, WS_C0, n);
    VR_WS(pos, ctx, uint32_t, WS_C1, n);
    VR_WS(bad, ctx, int, WS_FLAG2, 4);
    VR_WS(tot, ctx, uint32_t, WS_C9, 4);
    VR_WS(size, ctx, int, WS_B0, n);
    if ((rc = fill_i32(ctx, bad, 0, 2, st)) || (rc = fill_i32(ctx, size, 0, n, st))) return rc;
    hipLaunchKernelGGL(k_participants, dim3(grid_for(n, 256)), dim3(256), 0, st, n, host_of, L, Lth2, n_hosts, flag,
                       bad);
    hipLaunchKernelGGL(k_label_sizes, dim3(grid_for(n, 256)), dim3(256), 0, st, n, label1, size);
    hipLaunchKernelGGL(k_check_tagged, dim3(grid_for(n, 256)), dim3(256), 0, st, n, label1, size, n_min, flag, bad);
    VR_LAUNCH_CHECK(ctx);
    rc = scan_u32(ctx, flag, pos, n, tot, st);
    if (rc) return rc;
    int32_t* pin = reinterpret_cast<int32_t*>(ctx->pinned);
    VR_HIP(ctx, hipMemcpyAsync(pin, tot, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    VR_HIP(ctx, hipMemcpyAsync(pin + 1, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    VR_HIP(ctx, hipStreamSynchronize(st));
    const int64_t np = (uint32_t)pin[0];
    if (pin[1]) return set_err(ctx, VR_ERR_INVALID_ARG, "a member of a candidate group is not a relaxed participant");
    if ((rc = fill_i32(ctx, label_out, -1, n, st))) return rc;
    if (np == 0) return VR_OK;
    VR_WS(cx, ctx, uint32_t, WS_C2, np);
    VR_WS(cy, ctx, uint32_t, WS_C3, np);
    VR_WS(cz, ctx, uint32_t, WS_C4, np);
    VR_WS(orig, ctx, int32_t, WS_C5, np);
    hipLaunchKernelGGL(k_compact_part, dim3(grid_for(n, 256)), dim3(256), 0, st, n, flag, pos, p->qx, p->qy, p->qz, cx,
                       cy, cz, orig);
    VR_LAUNCH_CHECK(ctx);
    int sb = 0;
    while ((double)(1 << sb) < u && sb < gb) ++sb;
    CellList cl;
    if ((rc = build_cell_list(ctx, np, cx, cy, cz, gb, sb, cl, st))) return rc;
    VR_WS(sorig, ctx, int32_t, WS_C6, np);
    VR_WS(svx, ctx, float, WS_C7, np);
    VR_WS(svy, ctx, float, WS_C8, np);
    VR_WS(svz, ctx, float, WS_D0, np);
    VR_WS(shost, ctx, int32_t, WS_D1, np);
    VR_WS(tagA, ctx, int32_t, WS_D2, np);
    VR_WS(tagB, ctx, int32_t, WS_D3, np);
    VR_WS(su0, ctx, double, WS_D4, np);
    VR_WS(su1, ctx, double, WS_D5, np);
    VR_WS(su2, ctx, double, WS_D6, np);
    VR_WS(ss, ctx, double, WS_D7, np);
    hipLaunchKernelGGL(k_sorted_attrs, dim3(grid_for(np, 256)), dim3(256), 0, st, np, cl.idx, orig, p->vx, p->vy,
                       p->vz, host_of, sorig, svx, svy, svz, shost);
    hipLaunchKernelGGL(k_sorted_u, dim3(grid_for(np, 256)), dim3(256), 0, st, np, n, sorig, p->vx, p->vy, p->vz, vbar,
                       su0, su1, su2, ss);
    hipLaunchKernelGGL(k_first_tags, dim3(grid_for(np, 256)), dim3(256), 0, st, np, sorig, label1, size, n_min, tagA);
    VR_LAUNCH_CHECK(ctx);
    const SubLink sl{su0, su1, su2, ss, gamma_V * Vr, cos_op_relaxed};
    const int b = gb - sb;
    const dim3 g(grid_for(np, 256));
    // growth rounds until nothing changes, pushed from each round's frontier
    VR_WS(front, ctx, int32_t, WS_D8, np);
    int* nfront = bad + 1;
    int32_t* prop = tagB;
    if ((rc = fill_i32(ctx, nfront, 0, 1, st))) return rc;
    hipLaunchKernelGGL(k_frontier_init, g, dim3(256), 0, st, np, tagA, prop, front, nfront);
    VR_LAUNCH_CHECK(ctx);
    VR_HIP(ctx, hipMemcpyAsync(pin, nfront, sizeof(int), hipMemcpyDeviceToHost, st));
    VR_HIP(ctx, hipStreamSynchronize(st));
    int nr = 0;
    for (int nf = pin[0]; nf > 0;) {
        VR_TIMED(ctx, "sub_grow", st, nf,
                 hipLaunchKernelGGL(k_grow_push, dim3(grid_for(nf, 256)), dim3(256), 0, st, nf, front, cl.key, cl.sx,
                                    cl.sy, cl.sz, shost, cl.cell_start, cl.hkeys, cl.hvals, cl.hmask, b, gb, ell2, sl,
                                    tagA, prop));
        if ((rc = fill_i32(ctx, nfront, 0, 1, st))) return rc;
        hipLaunchKernelGGL(k_grow_apply, g, dim3(256), 0, st, np, tagA, prop, front, nfront);
        VR_LAUNCH_CHECK(ctx);
        VR_HIP(ctx, hipMemcpyAsync(pin, nfront, sizeof(int), hipMemcpyDeviceToHost, st));
        VR_HIP(ctx, hipStreamSynchronize(st));
        nf = pin[0];
        if (nf > 0) ++nr;
    }
    if (rounds) *rounds = nr;
    // relaxed links between different groups: count, then collect
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(tot);
    if ((rc = fill_u32(ctx, tot, 0u, 2, st))) return rc;
    hipLaunchKernelGGL(k_cross<false>, g, dim3(256), 0, st, np, cl.key, cl.sx, cl.sy, cl.sz, shost, cl.cell_start,
                       cl.hkeys, cl.hvals, cl.hmask, b, gb, ell2, sl, tagA, size, cnt, (int64_t)0, nullptr, nullptr);
    VR_LAUNCH_CHECK(ctx);
    unsigned long long ncross = 0;
    if ((rc = read_back(ctx, cnt, &ncross, sizeof ncross, st))) return rc;
    std::vector<uint64_t> hp(ncross);
    std::vector<int2> hs(ncross);
    if (ncross > 0) {
        VR_WS(pairs, ctx, uint64_t, WS_B3, ncross);
        VR_WS(psz, ctx, int2, WS_B4, ncross);
        if ((rc = fill_u32(ctx, tot, 0u, 2, st))) return rc;
        hipLaunchKernelGGL(k_cross<true>, g, dim3(256), 0, st, np, cl.key, cl.sx, cl.sy, cl.sz, shost, cl.cell_start,
                           cl.hkeys, cl.hvals, cl.hmask, b, gb, ell2, sl, tagA, size, cnt, (int64_t)ncross, pairs, psz);
        VR_LAUNCH_CHECK(ctx);
        if ((rc = copy_to_host(ctx, hp.data(), pairs, ncross * sizeof(uint64_t), st))) return rc;
        if ((rc = copy_to_host(ctx, hs.data(), psz, ncross * sizeof(int2), st))) return rc;
    }
    // joins: the relaxed links of a pair of groups against f_merge times the
    // first-stage size of either; union by smaller label, transitive
    std::unordered_map<uint64_t, std::pair<int64_t, int2>> per;
    for (unsigned long long i = 0; i < ncross; ++i) {
        auto& e = per[hp[i]];
        ++e.first;
        e.second = hs[i];
    }
    std::unordered_map<int, int> parent;
    auto find = [&](int x) {
        for (;;) {
            auto it = parent.find(x);
            if (it == parent.end() || it->second == x) return x;
            x = it->second;
        }
    };
    for (auto& kv : per) {
        const int a = (int)(kv.first >> 32), c = (int)(kv.first & 0xFFFFFFFFu);
        const double k = (double)kv.second.first;
        if (k > f_merge * (double)kv.second.second.x || k > f_merge * (double)kv.second.second.y) {
            const int ra = find(a), rc2 = find(c);
            if (ra != rc2) parent[std::max(ra, rc2)] = std::min(ra, rc2);
        }
    }
    std::vector<int> at, val;
    for (auto& kv : parent) {
        const int r = find(kv.first);
        if (r != kv.first) {
            at.push_back(kv.first);
            val.push_back(r);
        }
    }
    VR_WS(remap, ctx, int, WS_B1, n);
    VR_WS(low, ctx, int, WS_B2, n);
    hipLaunchKernelGGL(k_iota_i, dim3(grid_for(n, 256)), dim3(256), 0, st, n, remap);
    VR_LAUNCH_CHECK(ctx);
    if (!at.empty()) {
        const int k = (int)at.size();
        VR_WS(dat, ctx, int, WS_B5, k);
        VR_WS(dval, ctx, int, WS_B6, k);
        VR_HIP(ctx, hipMemcpyAsync(dat, at.data(), k * sizeof(int), hipMemcpyHostToDevice, st));
        VR_HIP(ctx, hipMemcpyAsync(dval, val.data(), k * sizeof(int), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_scatter_i, dim3(grid_for(k, 256)), dim3(256), 0, st, k, dat, dval, remap);
        VR_LAUNCH_CHECK(ctx);
    }
    if ((rc = fill_i32(ctx, low, 0x7FFFFFFF, n, st))) return rc;
    hipLaunchKernelGGL(k_remap_tags, g, dim3(256), 0, st, np, remap, tagA, sorig, low);
    hipLaunchKernelGGL(k_grow_labels, g, dim3(256), 0, st, np, tagA, sorig, low, label_out);
    VR_LAUNCH_CHECK(ctx);
    // the host vectors above are copied asynchronously: wait before they go away
    VR_HIP(ctx, hipStreamSynchronize(st));
    return VR_OK;
}
