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
#include "vr_internal.h"

#include <cmath>

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

__global__ void k_ub_init(int ng, const int32_t* __restrict__ off, const int32_t* __restrict__ mem,
                          const uint32_t* __restrict__ qx, const uint32_t* __restrict__ qy,
                          const uint32_t* __restrict__ qz, const float* __restrict__ vx, const float* __restrict__ vy,
                          const float* __restrict__ vz, const float* __restrict__ mass, int gb, int n_min, Members W,
                          int* __restrict__ cnt, int* __restrict__ state, int32_t* __restrict__ iters,
                          uint8_t* __restrict__ bound, double* __restrict__ phi) {
    const int g = blockIdx.x;
    const int s = off[g], e = off[g + 1];
    const int r = mem[s];
    const int rx = (int)qx[r], ry = (int)qy[r], rz = (int)qz[r];
    for (int k = s + threadIdx.x; k < e; k += blockDim.x) {
        const int i = mem[k];
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
    if (threadIdx.x == 0) {
        cnt[g] = e - s;
        state[g] = (e - s < n_min) ? ST_DISSOLVED : ST_ACTIVE;
        iters[g] = 0;
    }
}

__global__ void k_ub_zero(int na, const int* __restrict__ active, const int32_t* __restrict__ off,
                          const int* __restrict__ cnt, double* __restrict__ acc) {
    const int g = active[blockIdx.x];
    const int s = off[g], e = s + cnt[g];
    for (int k = s + threadIdx.x; k < e; k += blockDim.x) acc[k] = 0.0;
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
        for (int t0 = 0; t0 < jn; t0 += 64) {
            const int t1 = min(t0 + 64, jn);
            float accf = 0.f;
            for (int t = t0; t < t1; ++t) {
                const float4 q = sj[t];
                const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
                const float s2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
                const float rinv = (j0 + t != i && s2 > 0.f) ? rsqrtf(s2) : 0.f;
                accf = UNIFORM ? accf + rinv : fmaf(q.w, rinv, accf);
            }
            accd += (double)accf;
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

__global__ __launch_bounds__(UB) void k_ub_group(const int* __restrict__ active, const int32_t* __restrict__ off,
                                                 int* __restrict__ cnt, int* __restrict__ state,
                                                 int32_t* __restrict__ iters, Members W,
                                                 const double* __restrict__ acc, double eps2g, double scale,
                                                 double mass_value, double beta_E, double frac_ref, int n_min,
                                                 int n_ref_min, int frame_type, int gb, uint8_t* __restrict__ bound,
                                                 double* __restrict__ phi, int* __restrict__ overflow) {
    __shared__ double smd[4 * 8];
    __shared__ uint32_t smu[8];
    __shared__ uint32_t hist[2048];
    __shared__ int cand[MAX_CAND];
    __shared__ double cacc[MAX_CAND];
    __shared__ int s_ncand, s_p, s_bucket;
    __shared__ uint32_t s_below;
    __shared__ double s_min;
    __shared__ int s_minpos;
    const int g = active[blockIdx.x];
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
    if (tid == 0) s_ncand = 0;
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
    // 2. candidates within the FP32 error band of the extreme
    const double thr = s_min * (1.0 - REFINE_TOL);
    for (int k = tid; k < n; k += blockDim.x)
        if (acc[base + k] >= thr) {
            const int c = atomicAdd(&s_ncand, 1);
            if (c < MAX_CAND) cand[c] = k;
        }
    __syncthreads();
    const int ncand = min(s_ncand, MAX_CAND);
    if (tid == 0 && s_ncand > MAX_CAND) atomicAdd(overflow, 1);
    // 3. exact FP64 sums for the candidates
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
        if (tid == 0) cacc[c] = s1[0];
    }
    __syncthreads();
    if (tid == 0) {
        int bp = s_minpos;
        double b = -1.0;
        for (int c = 0; c < ncand; ++c)
            if (cacc[c] > b || (cacc[c] == b && cand[c] < bp)) { b = cacc[c]; bp = cand[c]; }
        s_p = bp;
    }
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
            for (int k = 0; k < 8; ++k) loc += hist[tid * 8 + k];
            uint32_t tot;
            const uint32_t ex = bscan(loc, smu, &tot);
            if (rank >= ex && rank < ex + loc) {
                uint32_t c = ex;
                for (int k = 0; k < 8; ++k) {
                    const uint32_t hh = hist[tid * 8 + k];
                    if (rank < c + hh) { s_bucket = tid * 8 + k; s_below = c; break; }
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
    // 5. energies, removal and stable in-place compaction
    uint32_t kept = 0;
    for (int c0 = 0; c0 < n; c0 += blockDim.x) {
        const int k = c0 + tid;
        const bool valid = k < n;
        int32_t gi = 0;
        float x = 0, y = 0, z = 0, ux = 0, uy = 0, uz = 0, mm = 0;
        bool keep = false;
        if (valid) {
            gi = W.gidx[base + k];
            x = W.x[base + k]; y = W.y[base + k]; z = W.z[base + k];
            ux = W.vx[base + k]; uy = W.vy[base + k]; uz = W.vz[base + k];
            mm = uniform ? 0.f : W.m[base + k];
            const double m = uniform ? mass_value : (double)mm;
            const double ph = scale * (uniform ? mass_value : 1.0) * acc[base + k];
            const double dx = (double)ux - vr0, dy = (double)uy - vr1, dz = (double)uz - vr2;
            const double T = 0.5 * m * (dx * dx + dy * dy + dz * dz);
            const double Wp = m * ph;
            const double E = beta_E * T + Wp;
            keep = !(E >= 0.0);
            phi[gi] = ph;
        }
        uint32_t tot;
        const uint32_t r = bscan(keep ? 1u : 0u, smu, &tot);
        if (keep) {
            const int dst = base + (int)(kept + r);
            W.gidx[dst] = gi;
            W.x[dst] = x; W.y[dst] = y; W.z[dst] = z;
            W.vx[dst] = ux; W.vy[dst] = uy; W.vz[dst] = uz;
            if (!uniform) W.m[dst] = mm;
        }
        kept += tot;
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
    }
}

}  // namespace
}  // namespace vr

using namespace vr;

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
    VR_HIP(ctx, hipMemcpyAsync(off.data(), offsets, (n_groups + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    VR_HIP(ctx, hipStreamSynchronize(st));
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
    VR_WS(ovf, ctx, int, WS_FLAG2, 4);
    rc = fill_i32(ctx, ovf, 0, 1, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_ub_init, dim3(n_groups), dim3(256), 0, st, n_groups, offsets, members, p->qx, p->qy, p->qz,
                       p->vx, p->vy, p->vz, p->mass, p->grid_bits, up->n_min, W, cnt, state, iters, bound, phi);
    VR_LAUNCH_CHECK(ctx);
    const double unit = p->box / ldexp(1.0, p->grid_bits);
    const double epsg = up->eps / unit;
    const double eps2g = epsg * epsg;
    const float eps2f = (float)eps2g;
    const double scale = -up->G / unit;  // potential = scale * mass * sum(1/r) in grid units
    int tile = up->tile ? up->tile : (ctx->tuned_tile ? ctx->tuned_tile : 256);
    std::vector<int> hcnt(n_groups), hstate(n_groups), hact;
    std::vector<int4> items;
    for (int pass = 0;; ++pass) {
        VR_HIP(ctx, hipMemcpyAsync(hcnt.data(), cnt, n_groups * sizeof(int), hipMemcpyDeviceToHost, st));
        VR_HIP(ctx, hipMemcpyAsync(hstate.data(), state, n_groups * sizeof(int), hipMemcpyDeviceToHost, st));
        VR_HIP(ctx, hipStreamSynchronize(st));
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
                 hipLaunchKernelGGL(k_ub_group, dim3(na), dim3(UB), 0, st, act, offsets, cnt, state, iters, W, acc,
                                    eps2g, scale, p->mass_value, up->beta_E, up->frac_ref, up->n_min, up->n_ref_min,
                                    up->frame_type, p->grid_bits, bound, phi, ovf));
        VR_LAUNCH_CHECK(ctx);
    }
    return VR_OK;
}
