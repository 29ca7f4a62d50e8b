// vr_unbind.hip -- unbinding by directly summed Plummer-softened potentials
// (Sec. 2.2, Eq. binding), all groups batched per pass.
//
// Every pass has two launches.  The potential launch runs over work items
// (group, i-tile, j-range): the j members are staged through LDS as float
// grid-unit coordinates (exact small integers) and mass; each lane owns one i
// and sums 1/sqrt(r^2 + eps^2) terms in FP32 over runs of at most 64 j
// before adding the run into an FP64 accumulator, which is then added
// atomically to the member's FP64 potential.  The per-group launch (one
// workgroup per active group) then finds the potential minimum (candidates
// within the FP32 error band are re-evaluated exactly in FP64, so the chosen
// centre is the FP64 argmin), selects the members nearest to it with an
// 11-bit radix select over (d2, index) keys, takes their mass-weighted mean
// velocity as the frame, evaluates beta_E T + W, and compacts the survivors
// in place (stable, so index order is kept).
//
// The persistent schedule updates the potential incrementally: the group
// kernel keeps each survivor's FP64 sum with it and writes the members it
// removed to a side list; the next pass subtracts those members' terms from
// the survivors' sums (|S| |D| pairs instead of |S|^2).  A group returns to
// a full recompute once the members removed since its last one exceed a
// quarter of its current size, which bounds the error the subtractions add
// to that of a full FP32-tiled sum (a quarter of it).
#include "vr_internal.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>

namespace vr {
namespace {

constexpr int UB = 256;                 // threads per workgroup
constexpr int ST_ACTIVE = 0, ST_BOUND = 1, ST_DISSOLVED = 2;
constexpr int MAX_CAND = 64;
constexpr double REFINE_TOL = 4e-5;     // > twice the FP32 error bound of the tiled sums

struct Members {
    int32_t* gidx;
    float *x, *y, *z;    // grid units relative to the group's first member (exact integers)
    float *vx, *vy, *vz;
    float* m;            // null for uniform mass
};

// Members removed by a group's last pass, at the group's base (stable
// order), and the per-group bookkeeping of the incremental potential:
// nrm = members removed by the last pass; since = removed since the last
// full recompute; mode = 1 when the next pass may subtract them instead of
// recomputing.
struct Removed {
    float *x, *y, *z, *m;
    int *nrm, *since, *mode;
};

// Member-parallel set-up: member k of group g (found by bisection of the
// offsets) gets its grid offsets from the group's first member, its
// velocity and mass; its particle's bound flag and potential are reset.
__global__ void k_ub_init(int ng, int64_t M, const int32_t* __restrict__ off, const int32_t* __restrict__ mem,
                          const uint32_t* __restrict__ qx, const uint32_t* __restrict__ qy,
                          const uint32_t* __restrict__ qz, const float* __restrict__ vx, const float* __restrict__ vy,
                          const float* __restrict__ vz, const float* __restrict__ mass, int gb, Members W,
                          uint8_t* __restrict__ bound, double* __restrict__ phi) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    int lo = 0, hi = ng - 1;  // last group with off[g] <= k
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid - 1;
    }
    const int r = mem[off[lo]];
    const int i = mem[k];
    const int rx = (int)qx[r], ry = (int)qy[r], rz = (int)qz[r];
    W.gidx[k] = i;
    W.x[k] = (float)min_image((int)qx[i] - rx, gb);
    W.y[k] = (float)min_image((int)qy[i] - ry, gb);
    W.z[k] = (float)min_image((int)qz[i] - rz, gb);
    W.vx[k] = vx[i];
    W.vy[k] = vy[i];
    W.vz[k] = vz[i];
    if (mass) W.m[k] = mass[i];
    bound[i] = 0;
    phi[i] = NAN;
}

// Per-group state, and nbig = the first group with fewer than wide_min
// members (*nbig holds ng beforehand): the leading groups up to there take
// the wide group kernel.
__global__ void k_ub_state(int ng, const int32_t* __restrict__ off, int n_min, int wide_min, Removed Rm,
                           int* __restrict__ cnt, int* __restrict__ state, int32_t* __restrict__ iters,
                           int* __restrict__ nbig) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const int n = off[g + 1] - off[g];
    cnt[g] = n;
    state[g] = n < n_min ? ST_DISSOLVED : ST_ACTIVE;
    iters[g] = 0;
    Rm.nrm[g] = 0;
    Rm.since[g] = 0;
    Rm.mode[g] = 0;
    if (n < wide_min) atomicMin(nbig, g);
}

__global__ void k_ub_zero(int na, const int* __restrict__ active, const int32_t* __restrict__ off,
                          const int* __restrict__ cnt, double* __restrict__ acc) {
    const int g = active[blockIdx.x];
    const int s = off[g], e = s + cnt[g];
    for (int k = s + threadIdx.x; k < e; k += blockDim.x) acc[k] = 0.0;
}

// Sum over staged j of m_j / sqrt(r^2 + eps^2) for one i, in FP32 over at
// most 64 terms (the caller adds it to an FP64 accumulator; 64 same-sign
// FP32 terms stay within 64 * 2^-24 relative).  CHECK = the chunk may hold
// j == i or, with eps = 0, a coincident pair; otherwise every term is
// finite and taken.  r^2 + eps^2 is at least min(eps^2, 1) in grid units
// squared (coordinates are integers), a normal FP32 number (the host refuses
// a smaller nonzero eps^2), so the hardware reciprocal square root needs no
// rescaling for subnormal inputs and gives rsqrtf's result.
template <bool UNIFORM, bool CHECK>
__device__ __forceinline__ float tile_sum(const float4* __restrict__ sj, int t0, int t1, float xi, float yi, float zi,
                                          float eps2, int jbase, int i) {
    float accf = 0.f;
#pragma unroll 4
    for (int t = t0; t < t1; ++t) {
        const float4 q = sj[t];
        const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
        const float s2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
        float rinv;
        if (CHECK) rinv = (jbase + t != i && s2 > 0.f) ? __builtin_amdgcn_rsqf(s2) : 0.f;
        else rinv = __builtin_amdgcn_rsqf(s2);
        accf = UNIFORM ? accf + rinv : fmaf(q.w, rinv, accf);
    }
    return accf;
}

// Potential tiles: item = (group, i0, j0, j1).
template <bool UNIFORM>
__global__ __launch_bounds__(UB) void k_ub_potential(const int4* __restrict__ items, const int32_t* __restrict__ off,
                                                     const int* __restrict__ cnt, Members W, float eps2,
                                                     double* __restrict__ acc, int tile) {
    extern __shared__ float4 sj[];
    const int4 it = items[blockIdx.x];
    const int g = it.x, base = off[g], n = cnt[g];
    const int i = it.y + (int)threadIdx.x;
    const bool valid = i < n;
    const float xi = valid ? W.x[base + i] : 0.f, yi = valid ? W.y[base + i] : 0.f, zi = valid ? W.z[base + i] : 0.f;
    double accd = 0.0;
    for (int j0 = it.z; j0 < it.w; j0 += tile) {
        const int jn = min(tile, it.w - j0);
        __syncthreads();
        for (int t = threadIdx.x; t < jn; t += blockDim.x) {
            const int k = base + j0 + t;
            sj[t] = make_float4(W.x[k], W.y[k], W.z[k], UNIFORM ? 1.f : W.m[k]);
        }
        __syncthreads();
        // rows of this wavefront: [iw, iw + 64)
        const int iw = it.y + ((int)threadIdx.x & ~63);
        for (int t0 = 0; t0 < jn; t0 += 64) {
            const int t1 = min(t0 + 64, jn);
            const bool check = eps2 == 0.f || (j0 + t0 < iw + 64 && j0 + t1 > iw);
            accd += (double)(check ? tile_sum<UNIFORM, true>(sj, t0, t1, xi, yi, zi, eps2, j0, i)
                                   : tile_sum<UNIFORM, false>(sj, t0, t1, xi, yi, zi, eps2, j0, i));
        }
    }
    if (valid) atomicAdd(&acc[base + i], accd);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int N>
__device__ __forceinline__ void bsum(double (&v)[N], double* sm) {
    const int lane = __lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int k = 0; k < N; ++k) {
        double s = wsum(v[k]);
        if (lane == 0) sm[w * N + k] = s;
    }
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        double s = 0;
        for (int ww = 0; ww < nw; ++ww) s += sm[ww * N + k];
        v[k] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ uint32_t wscan(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t bscan(uint32_t v, uint32_t* sm, uint32_t* total) {
    const int lane = __lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t inc = wscan(v);
    if (lane == 63) sm[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int k = 0; k < nw; ++k) {
        if (k < w) pre += sm[k];
        tot += sm[k];
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

__device__ __forceinline__ uint64_t ref_key(const Members& W, int base, int pos, int px, int py, int pz, int gb) {
    const int64_t dx = min_image((int)W.x[base + pos] - px, gb);
    const int64_t dy = min_image((int)W.y[base + pos] - py, gb);
    const int64_t dz = min_image((int)W.z[base + pos] - pz, gb);
    return ((uint64_t)(dx * dx + dy * dy + dz * dz) << 22) | (uint64_t)pos;
}

// One group per workgroup of BS threads.  With split != 0 (no active list)
// BS = UB_WIDE takes the groups before *nbig and BS = UB the others, so the
// largest groups get four times the threads.
constexpr int UB_WIDE = 1024;
template <int BS>
__global__ __launch_bounds__(BS) void k_ub_group(const int* __restrict__ active, const int32_t* __restrict__ off,
                                                 int* __restrict__ cnt, int* __restrict__ state,
                                                 int32_t* __restrict__ iters, Members W, Removed Rm,
                                                 double* __restrict__ acc, double eps2g, double scale,
                                                 double mass_value, double beta_E, double frac_ref, int n_min,
                                                 int n_ref_min, int frame_type, int gb, uint8_t* __restrict__ bound,
                                                 double* __restrict__ phi, int max_iter,
                                                 const int* __restrict__ nbig) {
    constexpr int NW = BS / 64;
    constexpr int BPT = 2048 / BS;  // histogram bins per thread
    static_assert(BS >= 256 && BS <= 2048 && 2048 % BS == 0, "block size");
    __shared__ double smd[4 * NW];
    __shared__ uint32_t smu[NW];
    __shared__ uint32_t hist[2048];
    __shared__ int cand[MAX_CAND];
    __shared__ int s_p, s_bucket;
    __shared__ uint32_t s_below;
    __shared__ double s_min;
    __shared__ int s_minpos;
    // with no active list every group has a block and finished ones leave
    const int g = active ? active[blockIdx.x] : (int)blockIdx.x;
    if (nbig && (BS == UB_WIDE ? g >= *nbig : g < *nbig)) return;
    if (!active && (state[g] != ST_ACTIVE || iters[g] >= max_iter)) return;
    const int base = off[g];
    const int n = cnt[g];
    const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6, nw = blockDim.x >> 6;
    const bool uniform = W.m == nullptr;

    // 1. largest accumulated 1/r sum = deepest potential (ties: lowest position)
    double best = -1.0;
    int bpos = 0x7FFFFFFF;
    for (int k = tid; k < n; k += blockDim.x) {
        const double a = acc[base + k];
        if (a > best || (a == best && k < bpos)) { best = a; bpos = k; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int op = __shfl_xor(bpos, o, 64);
        if (ob > best || (ob == best && op < bpos)) { best = ob; bpos = op; }
    }
    if (lane == 0) { smd[w] = best; smu[w] = (uint32_t)bpos; }
    __syncthreads();
    if (tid == 0) {
        double b = smd[0];
        int bp = (int)smu[0];
        for (int ww = 1; ww < nw; ++ww)
            if (smd[ww] > b || (smd[ww] == b && (int)smu[ww] < bp)) { b = smd[ww]; bp = (int)smu[ww]; }
        s_min = b;
        s_minpos = bp;
    }
    __syncthreads();
    // 2-3. every member within the FP32 error band of the extreme gets an
    // exact FP64 sum; candidates are enumerated in position order, MAX_CAND
    // at a time, so the result does not depend on how many there are.
    const double thr = s_min * (1.0 - REFINE_TOL);
    double cbest = -1.0;
    int cpos = s_minpos;
    for (uint32_t first = 0;; first += MAX_CAND) {
        uint32_t seen = 0;
        for (int c0 = 0; c0 < n; c0 += blockDim.x) {
            const int k = c0 + tid;
            const bool in = k < n && acc[base + k] >= thr;
            uint32_t tot;
            const uint32_t r = seen + bscan(in ? 1u : 0u, smu, &tot);
            if (in && r >= first && r < first + MAX_CAND) cand[r - first] = k;
            seen += tot;
        }
        __syncthreads();
        const int ncand = (int)min(seen - first, (uint32_t)MAX_CAND);
        for (int c = 0; c < ncand; ++c) {
            const int pc = cand[c];
            const double cx = (double)W.x[base + pc], cy = (double)W.y[base + pc], cz = (double)W.z[base + pc];
            double s1[1] = {0.0};
            for (int k = tid; k < n; k += blockDim.x) {
                if (k == pc) continue;
                const double dx = cx - (double)W.x[base + k], dy = cy - (double)W.y[base + k],
                             dz = cz - (double)W.z[base + k];
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (eps2g == 0.0 && r2 == 0.0) continue;
                const double m = uniform ? 1.0 : (double)W.m[base + k];
                s1[0] += m / sqrt(r2 + eps2g);
            }
            bsum<1>(s1, smd);
            if (s1[0] > cbest || (s1[0] == cbest && pc < cpos)) { cbest = s1[0]; cpos = pc; }
        }
        if (first + MAX_CAND >= seen) break;
    }
    if (tid == 0) s_p = cpos;
    __syncthreads();
    const int p = s_p;
    // 4. velocity frame
    double fr[4] = {0, 0, 0, 0};
    if (frame_type == 1) {
        int64_t nref = (int64_t)ceil(frac_ref * (double)n);
        if (nref < n_ref_min) nref = n_ref_min;
        if (nref > n) nref = n;
        const int px = (int)W.x[base + p], py = (int)W.y[base + p], pz = (int)W.z[base + p];
        // radix select of the key of rank nref-1, 11 bits at a time from the top
        uint64_t prefix = 0;
        uint32_t rank = (uint32_t)(nref - 1);
        for (int shift = 55; shift >= 0; shift -= 11) {
            for (int k = tid; k < 2048; k += blockDim.x) hist[k] = 0;
            __syncthreads();
            const uint64_t hmask = (shift + 11 >= 64) ? 0ull : ~((1ull << (shift + 11)) - 1);
            for (int k = tid; k < n; k += blockDim.x) {
                const uint64_t key = ref_key(W, base, k, px, py, pz, gb);
                if (((key ^ prefix) & hmask) == 0) atomicAdd(&hist[(key >> shift) & 2047u], 1u);
            }
            __syncthreads();
            uint32_t loc = 0;
            for (int k = 0; k < BPT; ++k) loc += hist[tid * BPT + k];
            uint32_t tot;
            const uint32_t ex = bscan(loc, smu, &tot);
            if (rank >= ex && rank < ex + loc) {
                uint32_t c = ex;
                for (int k = 0; k < BPT; ++k) {
                    const uint32_t hh = hist[tid * BPT + k];
                    if (rank < c + hh) { s_bucket = tid * BPT + k; s_below = c; break; }
                    c += hh;
                }
            }
            __syncthreads();
            prefix |= (uint64_t)s_bucket << shift;
            rank -= s_below;
            __syncthreads();
        }
        for (int k = tid; k < n; k += blockDim.x) {
            if (ref_key(W, base, k, px, py, pz, gb) > prefix) continue;
            const double m = uniform ? mass_value : (double)W.m[base + k];
            fr[0] += m;
            fr[1] += m * (double)W.vx[base + k];
            fr[2] += m * (double)W.vy[base + k];
            fr[3] += m * (double)W.vz[base + k];
        }
    } else {
        for (int k = tid; k < n; k += blockDim.x) {
            const double m = uniform ? mass_value : (double)W.m[base + k];
            fr[0] += m;
            fr[1] += m * (double)W.vx[base + k];
            fr[2] += m * (double)W.vy[base + k];
            fr[3] += m * (double)W.vz[base + k];
        }
    }
    bsum<4>(fr, smd);
    const double vr0 = fr[1] / fr[0], vr1 = fr[2] / fr[0], vr2 = fr[3] / fr[0];
    // 5. energies, removal and stable in-place compaction; survivors keep
    // their sums, removed members go to the side list
    uint32_t kept = 0, gone = 0;
    for (int c0 = 0; c0 < n; c0 += blockDim.x) {
        const int k = c0 + tid;
        const bool valid = k < n;
        int32_t gi = 0;
        float x = 0, y = 0, z = 0, ux = 0, uy = 0, uz = 0, mm = 0;
        double a = 0.0;
        bool keep = false;
        if (valid) {
            gi = W.gidx[base + k];
            x = W.x[base + k]; y = W.y[base + k]; z = W.z[base + k];
            ux = W.vx[base + k]; uy = W.vy[base + k]; uz = W.vz[base + k];
            mm = uniform ? 0.f : W.m[base + k];
            a = acc[base + k];
            const double m = uniform ? mass_value : (double)mm;
            const double ph = scale * (uniform ? mass_value : 1.0) * a;
            const double dx = (double)ux - vr0, dy = (double)uy - vr1, dz = (double)uz - vr2;
            const double T = 0.5 * m * (dx * dx + dy * dy + dz * dz);
            const double Wp = m * ph;
            const double E = beta_E * T + Wp;
            keep = !(E >= 0.0);
            phi[gi] = ph;
        }
        uint32_t tot, totr;
        const uint32_t r = bscan(keep ? 1u : 0u, smu, &tot);
        const uint32_t rr = bscan((valid && !keep) ? 1u : 0u, smu, &totr);
        if (keep) {
            const int dst = base + (int)(kept + r);
            W.gidx[dst] = gi;
            W.x[dst] = x; W.y[dst] = y; W.z[dst] = z;
            W.vx[dst] = ux; W.vy[dst] = uy; W.vz[dst] = uz;
            if (!uniform) W.m[dst] = mm;
            acc[dst] = a;
        } else if (valid) {
            const int dst = base + (int)(gone + rr);
            Rm.x[dst] = x; Rm.y[dst] = y; Rm.z[dst] = z;
            Rm.m[dst] = uniform ? 1.f : mm;
        }
        kept += tot;
        gone += totr;
        __syncthreads();
    }
    if (kept == (uint32_t)n) {
        for (int k = tid; k < n; k += blockDim.x) bound[W.gidx[base + k]] = 1;
        if (tid == 0) state[g] = ST_BOUND;
    } else if ((int)kept < n_min) {
        if (tid == 0) state[g] = ST_DISSOLVED;
    }
    if (tid == 0) {
        cnt[g] = (int)kept;
        iters[g] += 1;
        // the next pass subtracts the removed terms while those removed since
        // the last full recompute stay within a quarter of the survivors
        const int since = Rm.since[g] + (int)gone;
        const bool incr = 4 * (int64_t)since <= (int64_t)kept;
        Rm.nrm[g] = (int)gone;
        Rm.since[g] = incr ? since : 0;
        Rm.mode[g] = incr ? 1 : 0;
    }
}

// ---- persistent, graph-replayed passes -------------------------------------
// Device-side plan of one pass: the active groups in the given order (the
// group tables come in decreasing size, so the largest work is queued first)
// and the prefix of their work-item counts; item = (i-tile of 64, j-range).
struct UbPlan {
    int n_active;     // groups scheduled in this pass
    int total_items;
    int head;         // work-queue head
    int remaining;    // groups still active after the pass (read by the host)
    int stuck;        // active groups that reached max_iter
    int pad[3];
    double pairs;     // ordered pairs scheduled since the last reset
};

__global__ void k_ub_plan_reset(UbPlan* plan) {
    if (threadIdx.x == 0) plan->pairs = 0.0;
}

constexpr int PLAN_T = 1024;

__global__ __launch_bounds__(PLAN_T) void k_ub_plan(int ng, const int* __restrict__ cnt, const int* __restrict__ state,
                                                    const int32_t* __restrict__ iters, int max_iter, int jchunk,
                                                    const int* __restrict__ nrm, const int* __restrict__ mode,
                                                    int* __restrict__ act, int* __restrict__ item_off, UbPlan* plan) {
    __shared__ uint32_t sm[32];
    __shared__ double smd[PLAN_T / 64];
    uint32_t carry_g = 0, carry_i = 0;
    double pairs = 0.0;
    for (int base = 0; base < ng; base += PLAN_T) {
        const int g = base + (int)threadIdx.x;
        const bool on = g < ng && state[g] == ST_ACTIVE && iters[g] < max_iter;
        const int n = on ? cnt[g] : 0;
        // j over all members (full) or over the members removed last pass
        const int nj = (on && mode[g]) ? nrm[g] : n;
        pairs += (double)n * (double)(on && mode[g] ? nj : (n > 0 ? n - 1 : 0));
        const uint32_t items = on ? (uint32_t)(((n + 63) / 64) * ((nj + jchunk - 1) / jchunk)) : 0u;
        uint32_t tg, ti;
        const uint32_t pg = bscan(on ? 1u : 0u, sm, &tg);
        const uint32_t pi = bscan(items, sm, &ti);
        if (on) {
            act[carry_g + pg] = g;
            item_off[carry_g + pg] = (int)(carry_i + pi);
        }
        carry_g += tg;
        carry_i += ti;
    }
    pairs = wsum(pairs);
    if (__lane_id() == 0) smd[threadIdx.x >> 6] = pairs;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tp = 0.0;
        for (int k = 0; k < PLAN_T / 64; ++k) tp += smd[k];
        item_off[carry_g] = (int)carry_i;
        plan->n_active = (int)carry_g;
        plan->total_items = (int)carry_i;
        plan->head = 0;
        plan->pairs += tp;
    }
}

__global__ void k_ub_zero_p(const UbPlan* __restrict__ plan, const int* __restrict__ act,
                            const int32_t* __restrict__ off, const int* __restrict__ cnt, const int* __restrict__ mode,
                            double* __restrict__ acc) {
    if ((int)blockIdx.x >= plan->n_active) return;
    const int g = act[blockIdx.x];
    if (mode[g]) return;  // sums kept: the pass subtracts
    const int s = off[g], e = s + cnt[g];
    for (int k = s + threadIdx.x; k < e; k += blockDim.x) acc[k] = 0.0;
}

// Persistent potential kernel: wavefront w takes item w first, then pops
// items nwaves, nwaves + 1, ... from the queue until it is empty (so a light
// pass costs no burst of atomics on the queue head, and wavefronts beyond the
// item count leave at once); lane = one i of a 64-row tile, j staged through
// the wave's LDS slice.
template <bool UNIFORM>
__global__ __launch_bounds__(UB) void k_ub_potential_p(UbPlan* plan, const int* __restrict__ act,
                                                       const int* __restrict__ item_off, const int32_t* __restrict__ off,
                                                       const int* __restrict__ cnt, Members W, Removed Rm, float eps2,
                                                       double* __restrict__ acc, int jchunk, int tile) {
    extern __shared__ float4 sjall[];
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    float4* sj = sjall + wv * tile;
    const int na = plan->n_active, total = plan->total_items;
    const int nwaves = (int)(gridDim.x * (blockDim.x >> 6));
    int it = (int)(blockIdx.x * (blockDim.x >> 6)) + wv;
    for (;; ) {
        if (it >= total) break;
        // the group holding item `it`
        int lo = 0, hi = na - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_off[mid] <= it) lo = mid; else hi = mid - 1;
        }
        const int g = act[lo];
        const int base = off[g], n = cnt[g];
        // full: j over the members; incremental: j over last pass's removed
        const bool incr = Rm.mode[g] != 0;
        const int nj = incr ? Rm.nrm[g] : n;
        const float* __restrict__ jx = incr ? Rm.x : W.x;
        const float* __restrict__ jy = incr ? Rm.y : W.y;
        const float* __restrict__ jz = incr ? Rm.z : W.z;
        const float* __restrict__ jm = incr ? Rm.m : W.m;
        const int njc = (nj + jchunk - 1) / jchunk;
        const int local = it - item_off[lo];
        const int i0 = (local / njc) * 64, j0 = (local % njc) * jchunk;
        const int j1 = min(nj, j0 + jchunk);
        const int i = i0 + lane;
        const bool valid = i < n;
        const float xi = valid ? W.x[base + i] : 0.f, yi = valid ? W.y[base + i] : 0.f, zi = valid ? W.z[base + i] : 0.f;
        // a removed member is never i itself; only coincident pairs need care
        const int iself = incr ? -1 : i;
        double accd = 0.0;
        for (int jb = j0; jb < j1; jb += tile) {
            const int jn = min(tile, j1 - jb);
            __builtin_amdgcn_wave_barrier();
            for (int t = lane; t < jn; t += 64) {
                const int k = base + jb + t;
                sj[t] = make_float4(jx[k], jy[k], jz[k], UNIFORM ? 1.f : jm[k]);
            }
            __builtin_amdgcn_wave_barrier();
            for (int t0 = 0; t0 < jn; t0 += 64) {
                const int t1 = min(t0 + 64, jn);
                const bool check = eps2 == 0.f || (!incr && jb + t0 < i0 + 64 && jb + t1 > i0);
                accd += (double)(check ? tile_sum<UNIFORM, true>(sj, t0, t1, xi, yi, zi, eps2, jb, iself)
                                       : tile_sum<UNIFORM, false>(sj, t0, t1, xi, yi, zi, eps2, jb, iself));
            }
        }
        if (valid) atomicAdd(&acc[base + i], incr ? -accd : accd);
        int nx = 0;
        if (lane == 0) nx = atomicAdd(&plan->head, 1);
        it = nwaves + __shfl(nx, 0, 64);
    }
}

__global__ __launch_bounds__(PLAN_T) void k_ub_count(int ng, const int* __restrict__ state,
                                                     const int32_t* __restrict__ iters, int max_iter, UbPlan* plan) {
    __shared__ uint32_t sm[32];
    uint32_t rem = 0, stuck = 0;
    for (int g = threadIdx.x; g < ng; g += PLAN_T) {
        if (state[g] != ST_ACTIVE) continue;
        if (iters[g] < max_iter) ++rem; else ++stuck;
    }
    uint32_t tr, ts;
    bscan(rem, sm, &tr);
    bscan(stuck, sm, &ts);
    if (threadIdx.x == 0) {
        plan->remaining = (int)tr;
        plan->stuck = (int)ts;
    }
}

}  // namespace
}  // namespace vr

using namespace vr;

namespace {

constexpr int PERSIST_MAX_TILE = 1024;  // 4 waves x tile x 16 B of LDS per workgroup
constexpr int PASSES_PER_GRAPH = 4;

// Everything a captured pass depends on; a cached graph is reused only when
// all of it is unchanged.
struct UbGraphKey {
    const void* ptrs[24];
    int ints[12];
    double dbls[6];
};

void ub_graph_release(vr_ctx* ctx) {
    if (ctx->ub_exec) (void)hipGraphExecDestroy((hipGraphExec_t)ctx->ub_exec);
    if (ctx->ub_graph) (void)hipGraphDestroy((hipGraph_t)ctx->ub_graph);
    ctx->ub_exec = nullptr;
    ctx->ub_graph = nullptr;
    ctx->ub_key.clear();
}

// One pass = plan (active list and work items) -> zero the accumulators of
// the active groups -> persistent potential over the item queue -> one
// workgroup per active group for frame, energies and compaction.  Passes are
// captured PASSES_PER_GRAPH at a time in a graph that is replayed until no
// group is active; the host reads two counters per replay.
int unbind_persistent(vr_ctx* ctx, const vr_particles* p, int32_t ng, const int32_t* offsets,
                      const vr_unbind_params* up, const Members& W, const Removed& Rm, double* acc, int* cnt, int* state,
                      int32_t* iters, uint8_t* bound, double* phi, int* act, const int* nbig, float eps2f,
                      double eps2g, double scale, int tile, hipStream_t st) {
    VR_WS(plan, ctx, UbPlan, WS_D4, 1);
    VR_WS(item_off, ctx, int, WS_D5, (int64_t)ng + 1);
    const bool uniform = W.m == nullptr;
    const int jchunk = ctx->unbind_jchunk;
    const size_t lds = (size_t)(UB / 64) * tile * sizeof(float4);
    int bpc = 0;
    if (uniform)
        VR_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k_ub_potential_p<true>, UB, lds));
    else
        VR_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k_ub_potential_p<false>, UB, lds));
    if (ctx->unbind_bpc > 0 && ctx->unbind_bpc < bpc) bpc = ctx->unbind_bpc;
    if (bpc < 1) bpc = 1;
    const unsigned pgrid = (unsigned)(ctx->num_cus * bpc);

    UbGraphKey key;
    std::memset(&key, 0, sizeof key);
    const void* kp[24] = {offsets, W.gidx, W.x, W.y, W.z, W.vx, W.vy, W.vz, W.m, acc, cnt, state, iters, bound, phi,
                          act, Rm.x, Rm.y, Rm.z, Rm.m, Rm.nrm, Rm.since, Rm.mode, nbig};
    std::memcpy(key.ptrs, kp, sizeof kp);
    const int ki[12] = {ng, up->max_iter, jchunk, tile, (int)pgrid, up->n_min, up->n_ref_min, up->frame_type,
                        p->grid_bits, uniform ? 1 : 0, 0, 0};
    std::memcpy(key.ints, ki, sizeof ki);
    const double kd[6] = {(double)eps2f, eps2g, scale, p->mass_value, up->beta_E, up->frac_ref};
    std::memcpy(key.dbls, kd, sizeof kd);
    // plan and item_off are workspace too: their addresses are part of the key
    std::string kbytes((const char*)&key, sizeof key);
    kbytes.append((const char*)&plan, sizeof plan);
    kbytes.append((const char*)&item_off, sizeof item_off);

    if (!ctx->ub_exec || ctx->ub_key != kbytes) {
        ub_graph_release(ctx);
        if (!ctx->cap_stream) VR_HIP(ctx, hipStreamCreateWithFlags((hipStream_t*)&ctx->cap_stream, hipStreamNonBlocking));
        hipStream_t cs = (hipStream_t)ctx->cap_stream;
        VR_HIP(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < PASSES_PER_GRAPH; ++k) {
            hipLaunchKernelGGL(k_ub_plan, dim3(1), dim3(PLAN_T), 0, cs, ng, cnt, state, iters, up->max_iter, jchunk,
                               Rm.nrm, Rm.mode, act, item_off, plan);
            hipLaunchKernelGGL(k_ub_zero_p, dim3(ng), dim3(256), 0, cs, plan, act, offsets, cnt, Rm.mode, acc);
            if (uniform)
                hipLaunchKernelGGL(k_ub_potential_p<true>, dim3(pgrid), dim3(UB), lds, cs, plan, act, item_off,
                                   offsets, cnt, W, Rm, eps2f, acc, jchunk, tile);
            else
                hipLaunchKernelGGL(k_ub_potential_p<false>, dim3(pgrid), dim3(UB), lds, cs, plan, act, item_off,
                                   offsets, cnt, W, Rm, eps2f, acc, jchunk, tile);
            hipLaunchKernelGGL(k_ub_group<UB_WIDE>, dim3(ng), dim3(UB_WIDE), 0, cs, (const int*)nullptr, offsets, cnt,
                               state, iters, W, Rm, acc, eps2g, scale, p->mass_value, up->beta_E, up->frac_ref,
                               up->n_min, up->n_ref_min, up->frame_type, p->grid_bits, bound, phi, up->max_iter, nbig);
            hipLaunchKernelGGL(k_ub_group<UB>, dim3(ng), dim3(UB), 0, cs, (const int*)nullptr, offsets, cnt, state,
                               iters, W, Rm, acc, eps2g, scale, p->mass_value, up->beta_E, up->frac_ref, up->n_min,
                               up->n_ref_min, up->frame_type, p->grid_bits, bound, phi, up->max_iter, nbig);
        }
        hipLaunchKernelGGL(k_ub_count, dim3(1), dim3(PLAN_T), 0, cs, ng, state, iters, up->max_iter, plan);
        hipGraph_t graph = nullptr;
        const hipError_t le = hipGetLastError();
        const hipError_t ce = hipStreamEndCapture(cs, &graph);
        if (le != hipSuccess || ce != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return set_err(ctx, VR_ERR_HIP, "capturing the unbinding passes failed: %s",
                           hipGetErrorString(le != hipSuccess ? le : ce));
        }
        ctx->ub_graph = graph;
        hipGraphExec_t exec = nullptr;
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            ub_graph_release(ctx);
            return set_err(ctx, VR_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
        }
        ctx->ub_exec = exec;
        ctx->ub_key = kbytes;
    }

    hipLaunchKernelGGL(k_ub_plan_reset, dim3(1), dim3(64), 0, st, plan);
    VR_LAUNCH_CHECK(ctx);
    hipEvent_t e0 = nullptr;
    if (ctx->timing) {
        e0 = timer_event(ctx);
        (void)hipEventRecord(e0, st);
    }
    int* counters = reinterpret_cast<int*>(ctx->pinned);
    for (int launch = 0;; ++launch) {
        VR_HIP(ctx, hipGraphLaunch((hipGraphExec_t)ctx->ub_exec, st));
        VR_HIP(ctx, hipMemcpyAsync(counters, &plan->remaining, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        VR_HIP(ctx, hipStreamSynchronize(st));
        if (counters[0] == 0) break;
        // every replay advances each remaining group by PASSES_PER_GRAPH
        // passes, so the loop ends after max_iter / PASSES_PER_GRAPH replays
        if ((int64_t)launch * PASSES_PER_GRAPH > (int64_t)up->max_iter + PASSES_PER_GRAPH)
            return set_err(ctx, VR_ERR_HIP, "unbinding replays did not advance");
    }
    const int stuck = counters[1];
    double pairs = 0.0;
    if (ctx->timing) {
        hipEvent_t e1 = timer_event(ctx);
        (void)hipEventRecord(e1, st);
        VR_HIP(ctx, hipMemcpyAsync(ctx->pinned, &plan->pairs, sizeof(double), hipMemcpyDeviceToHost, st));
        VR_HIP(ctx, hipStreamSynchronize(st));
        std::memcpy(&pairs, ctx->pinned, sizeof(double));
        timer_push(ctx, "unbind_persistent", e0, e1, pairs);
    }
    if (stuck > 0)
        return set_err(ctx, VR_ERR_NOT_CONVERGED, "%d groups still lose members after %d passes", stuck, up->max_iter);
    return VR_OK;
}

}  // namespace

namespace vr {
void unbind_release(vr_ctx* ctx) { ub_graph_release(ctx); }
}  // namespace vr

extern "C" int vr_unbind(vr_ctx* ctx, const vr_particles* p, int32_t n_groups, const int32_t* offsets,
                         const int32_t* members, const vr_unbind_params* up, uint8_t* bound, double* phi,
                         int32_t* iters, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_particles(ctx, p, true);
    if (rc) return rc;
    if ((rc = check_hosts(ctx, n_groups, offsets, members))) return rc;
    if (!up) return set_err(ctx, VR_ERR_INVALID_ARG, "params is NULL");
    if (!(up->eps >= 0) || !(up->G > 0) || up->n_min < 1 || up->max_iter < 1 || up->n_ref_min < 1 ||
        !(up->frac_ref >= 0) || (up->frame_type != 0 && up->frame_type != 1))
        return set_err(ctx, VR_ERR_INVALID_ARG, "bad unbinding parameters");
    if (up->tile != 0 && (up->tile < 64 || up->tile > 4096 || (up->tile & 63)))
        return set_err(ctx, VR_ERR_INVALID_ARG, "tile must be 0 or a multiple of 64 in [64, 4096]");
    if (n_groups == 0) return VR_OK;
    if (!bound || !phi || !iters) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL output");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> off(n_groups + 1);
    int rc0 = copy_to_host(ctx, off.data(), offsets, (n_groups + 1) * sizeof(int32_t), st);
    if (rc0) return rc0;
    if (off[0] != 0) return set_err(ctx, VR_ERR_INVALID_ARG, "offsets[0] must be 0");
    for (int g = 0; g < n_groups; ++g) {
        if (off[g + 1] < off[g]) return set_err(ctx, VR_ERR_INVALID_ARG, "offsets must be non-decreasing");
        if (off[g + 1] - off[g] > (1 << 22)) return set_err(ctx, VR_ERR_UNSUPPORTED, "group %d exceeds 2^22 members", g);
    }
    const int64_t M = off[n_groups];
    if (M > p->n) return set_err(ctx, VR_ERR_INVALID_ARG, "more members than particles");
    const bool uniform = p->mass == nullptr;
    Members W;
    VR_WS(wg, ctx, int32_t, WS_C0, M);
    VR_WS(wx, ctx, float, WS_C1, M); VR_WS(wy, ctx, float, WS_C2, M); VR_WS(wz, ctx, float, WS_C3, M);
    VR_WS(wvx, ctx, float, WS_C4, M); VR_WS(wvy, ctx, float, WS_C5, M); VR_WS(wvz, ctx, float, WS_C6, M);
    VR_WS(wm, ctx, float, WS_C7, uniform ? 1 : M);
    W.gidx = wg; W.x = wx; W.y = wy; W.z = wz; W.vx = wvx; W.vy = wvy; W.vz = wvz; W.m = uniform ? nullptr : wm;
    VR_WS(acc, ctx, double, WS_C8, M);
    VR_WS(cnt, ctx, int, WS_D0, n_groups);
    VR_WS(state, ctx, int, WS_D1, n_groups);
    VR_WS(act, ctx, int, WS_D2, n_groups);
    Removed Rm;
    VR_WS(rx, ctx, float, WS_B0, M); VR_WS(ry, ctx, float, WS_B1, M); VR_WS(rz, ctx, float, WS_B2, M);
    VR_WS(rmass, ctx, float, WS_B3, M);
    VR_WS(nrm, ctx, int, WS_B4, n_groups); VR_WS(since, ctx, int, WS_B5, n_groups); VR_WS(mode, ctx, int, WS_B6, n_groups);
    Rm.x = rx; Rm.y = ry; Rm.z = rz; Rm.m = rmass; Rm.nrm = nrm; Rm.since = since; Rm.mode = mode;
    VR_WS(nbig, ctx, int, WS_D6, 1);
    {
        int rc = fill_i32(ctx, nbig, n_groups, 1, st);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_ub_state, dim3(grid_for(n_groups, 256)), dim3(256), 0, st, n_groups, offsets, up->n_min,
                       ctx->unbind_wide, Rm, cnt, state, iters, nbig);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_ub_init, dim3(grid_for(M, 256)), dim3(256), 0, st, n_groups, (int64_t)M, offsets, members,
                       p->qx, p->qy, p->qz, p->vx, p->vy, p->vz, p->mass, p->grid_bits, W, bound, phi);
    VR_LAUNCH_CHECK(ctx);
    const double unit = p->box / ldexp(1.0, p->grid_bits);
    const double epsg = up->eps / unit;
    const double eps2g = epsg * epsg;
    const float eps2f = (float)eps2g;
    if (eps2f > 0.f && eps2f < FLT_MIN)
        return set_err(ctx, VR_ERR_UNSUPPORTED, "softening eps = %g is below the FP32 normal range in grid units",
                       up->eps);
    const double scale = -up->G / unit;  // potential = scale * mass * sum(1/r) in grid units
    int tile = up->tile ? up->tile : (ctx->tuned_tile ? ctx->tuned_tile : 256);
    if (up->persistent)
        return unbind_persistent(ctx, p, n_groups, offsets, up, W, Rm, acc, cnt, state, iters, bound, phi, act, nbig,
                                 eps2f, eps2g, scale, std::min(tile, PERSIST_MAX_TILE), st);
    std::vector<int> hcnt(n_groups), hstate(n_groups), hact;
    std::vector<int4> items;
    for (int pass = 0;; ++pass) {
        if (int rc1 = copy_to_host(ctx, hcnt.data(), cnt, n_groups * sizeof(int), st)) return rc1;
        if (int rc1 = copy_to_host(ctx, hstate.data(), state, n_groups * sizeof(int), st)) return rc1;
        hact.clear();
        items.clear();
        double pairs = 0.0, nmem = 0.0;
        for (int g = 0; g < n_groups; ++g) {
            if (hstate[g] != ST_ACTIVE) continue;
            hact.push_back(g);
            const int n = hcnt[g];
            pairs += (double)n * (double)(n - 1);
            nmem += n;
            const int jchunk = ctx->unbind_jchunk;
            for (int i0 = 0; i0 < n; i0 += UB)
                for (int j0 = 0; j0 < n; j0 += jchunk) items.push_back(make_int4(g, i0, j0, std::min(n, j0 + jchunk)));
        }
        if (hact.empty()) break;
        if (pass >= up->max_iter)
            return set_err(ctx, VR_ERR_NOT_CONVERGED, "%zu groups still lose members after %d passes", hact.size(),
                           up->max_iter);
        const int na = (int)hact.size();
        const int64_t ni = (int64_t)items.size();
        VR_WS(items_d, ctx, int4, WS_D3, ni);
        VR_HIP(ctx, hipMemcpyAsync(act, hact.data(), na * sizeof(int), hipMemcpyHostToDevice, st));
        VR_HIP(ctx, hipMemcpyAsync(items_d, items.data(), ni * sizeof(int4), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_ub_zero, dim3(na), dim3(256), 0, st, na, act, offsets, cnt, acc);
        VR_LAUNCH_CHECK(ctx);
        const size_t lds = (size_t)tile * sizeof(float4);
        if (uniform)
            VR_TIMED(ctx, "unbind_potential", st, pairs,
                     hipLaunchKernelGGL(k_ub_potential<true>, dim3((unsigned)ni), dim3(UB), lds, st, items_d, offsets,
                                        cnt, W, eps2f, acc, tile));
        else
            VR_TIMED(ctx, "unbind_potential", st, pairs,
                     hipLaunchKernelGGL(k_ub_potential<false>, dim3((unsigned)ni), dim3(UB), lds, st, items_d, offsets,
                                        cnt, W, eps2f, acc, tile));
        VR_LAUNCH_CHECK(ctx);
        VR_TIMED(ctx, "unbind_group", st, nmem,
                 hipLaunchKernelGGL(k_ub_group<UB>, dim3(na), dim3(UB), 0, st, act, offsets, cnt, state, iters, W, Rm,
                                    acc, eps2g, scale, p->mass_value, up->beta_E, up->frac_ref, up->n_min,
                                    up->n_ref_min, up->frame_type, p->grid_bits, bound, phi, up->max_iter,
                                    (const int*)nullptr));
        VR_LAUNCH_CHECK(ctx);
    }
    return VR_OK;
}
