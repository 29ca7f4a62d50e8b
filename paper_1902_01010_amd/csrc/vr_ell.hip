// vr_ell.hip -- the normalised ratio L (Sec. 2.2, Eqs. skewgaus and ell) and
// significance cleaning of candidate groups (Eq. ellsig).
//
// Fit.  Members are mapped to their host, then counted on the fine R grid:
// a workgroup takes 4096 consecutive members; when they all belong to one
// host (every member of a large host does) the counts gather in LDS and are
// flushed once, otherwise each member adds to the host's row in HBM.  One
// workgroup per host then merges bin pairs, compacts the non-empty merged
// bins in order, and fits the skew-Gaussian: the weighted least-squares cost
// of the log model at a peak position c is a pair of wave-wide FP64
// reductions over the bins; the four waves share the scan over the
// merged-bin centres, wave 0 runs the golden-section refinement.  A last
// pass writes L for every member.
//
// Cleaning.  A stable radix sort orders every group's members by L (keys:
// group id above the order-preserving bits of the float L; the members are
// ascending within a group, so equal L keep index order).  One workgroup per
// group forms the suffix sums of the sorted L from the top in FP64 and finds
// the smallest number of removed members whose remainder meets the bound.
#include "vr_kd.h"

#include <cmath>

namespace vr {
namespace {

constexpr int EB = 256;         // threads of the per-host and per-group workgroups
constexpr int MAXBINS = 2048;   // fine bins held in LDS by the fit
constexpr int HCHUNK = 4096;    // members per histogram workgroup

__global__ void k_elem_owner(const int32_t* __restrict__ off, int32_t* __restrict__ owner) {
    const int h = blockIdx.x;
    for (int k = off[h] + (int)threadIdx.x; k < off[h + 1]; k += blockDim.x) owner[k] = h;
}

__global__ __launch_bounds__(EB) void k_ell_hist(int64_t M, const int32_t* __restrict__ mem,
                                                 const int32_t* __restrict__ owner, const float* __restrict__ R,
                                                 double lo, double inv_w, int nbins, uint32_t* __restrict__ hist) {
    __shared__ uint32_t sh[MAXBINS];
    const int64_t k0 = (int64_t)blockIdx.x * HCHUNK;
    const int64_t k1 = k0 + HCHUNK < M ? k0 + HCHUNK : M;
    const int h0 = owner[k0];
    const bool one = h0 == owner[k1 - 1];  // uniform: hosts are contiguous runs
    if (one) {
        for (int b = threadIdx.x; b < nbins; b += EB) sh[b] = 0;
        __syncthreads();
    }
    for (int64_t k = k0 + threadIdx.x; k < k1; k += EB) {
        const double r = (double)R[mem[k]];
        if (!isfinite(r)) continue;
        const double t = floor((r - lo) * inv_w);
        if (!(t >= 0.0 && t < (double)nbins)) continue;
        const int b = (int)t;
        if (one)
            atomicAdd(&sh[b], 1u);
        else
            atomicAdd(&hist[(int64_t)owner[k] * nbins + b], 1u);
    }
    if (one) {
        __syncthreads();
        for (int b = threadIdx.x; b < nbins; b += EB)
            if (sh[b]) atomicAdd(&hist[(int64_t)h0 * nbins + b], sh[b]);
    }
}

// Sum over the wave, identical in every lane (tree to lane 0, broadcast).
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return __shfl(v, 0, 64);
}

// Weighted least-squares cost of the log model at peak c over the nb bins
// (centres xs, counts ws, ys = ln ws); wave-wide, every lane returns it.
// The model ln n = a - p (x-c)^2 [x<c] - q (x-c)^2 [x>=c] is linear in
// beta = (a, p, q) with the design row g = (1, -lo, -hi), lo and hi the two
// one-sided squared offsets.  The normal matrix N = sum w g g^T and the
// right-hand side r = sum w g y are accumulated entry by entry and N beta = r
// is solved with the adjugate of N; the cost is then summed from the
// residuals.  +inf when a side of c holds no bin (N singular).
__device__ double wave_cost(const double* xs, const double* ws, const double* ys, int nb, double c, double* apq) {
    const int lane = __lane_id();
    // N (symmetric): n00, n11, n22, n01, n02, n12; r: r0, r1, r2
    double n00 = 0, n11 = 0, n22 = 0, n01 = 0, n02 = 0, n12 = 0, r0 = 0, r1 = 0, r2 = 0;
    for (int j = lane; j < nb; j += 64) {
        const double off = xs[j] - c;
        const double g1 = xs[j] < c ? -(off * off) : 0.0;
        const double g2 = xs[j] < c ? 0.0 : -(off * off);
        const double w = ws[j], wy = w * ys[j];
        n00 += w;
        n11 += w * g1 * g1;
        n22 += w * g2 * g2;
        n01 += w * g1;
        n02 += w * g2;
        n12 += w * g1 * g2;
        r0 += wy;
        r1 += wy * g1;
        r2 += wy * g2;
    }
    n00 = wave_sum(n00);
    n11 = wave_sum(n11);
    n22 = wave_sum(n22);
    n01 = wave_sum(n01);
    n02 = wave_sum(n02);
    n12 = wave_sum(n12);
    r0 = wave_sum(r0);
    r1 = wave_sum(r1);
    r2 = wave_sum(r2);
    if (!(n11 > 0) || !(n22 > 0)) return INFINITY;
    const Sym3Adj A = sym3_adjugate(n00, n11, n22, n01, n02, n12);
    if (!(A.det > 0)) return INFINITY;
    const double a = (A.xx * r0 + A.xy * r1 + A.xz * r2) / A.det;
    const double pp = (A.xy * r0 + A.yy * r1 + A.yz * r2) / A.det;
    const double qq = (A.xz * r0 + A.yz * r1 + A.zz * r2) / A.det;
    double J = 0;
    for (int j = lane; j < nb; j += 64) {
        const double off = xs[j] - c;
        const double sq = off * off;
        const double fit = xs[j] < c ? a - pp * sq : a - qq * sq;
        const double res = ys[j] - fit;
        J += ws[j] * res * res;
    }
    if (apq) {
        apq[0] = a;
        apq[1] = pp;
        apq[2] = qq;
    }
    return wave_sum(J);
}

__global__ __launch_bounds__(EB) void k_ell_fit(const uint32_t* __restrict__ hist, int nbins, double lo, double width,
                                                int peak_min, int max_merge, int giters, double* __restrict__ fit,
                                                int32_t* __restrict__ status, int32_t* __restrict__ merge) {
    __shared__ uint32_t cnt[MAXBINS], cnt2[MAXBINS / 2];
    __shared__ double xs[MAXBINS], ws[MAXBINS], ys[MAXBINS];
    __shared__ uint32_t red[EB / 64];
    __shared__ double bestJ[EB / 64];
    __shared__ int bestB[EB / 64];
    __shared__ int s_nb, s_bf, s_bl;
    const int h = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int b = t; b < nbins; b += EB) cnt[b] = hist[(int64_t)h * nbins + b];
    __syncthreads();
    // merge bin pairs until the fullest merged bin holds peak_min
    int g = 1, L = nbins;
    for (;;) {
        uint32_t m = 0;
        for (int b = t; b < L; b += EB) m = max(m, cnt[b]);
        for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
        if (lane == 0) red[wv] = m;
        __syncthreads();
        uint32_t full = red[0];
        for (int w = 1; w < EB / 64; ++w) full = max(full, red[w]);
        __syncthreads();
        if (!(g < max_merge && full < (uint32_t)peak_min)) break;
        for (int b = t; b < L / 2; b += EB) cnt2[b] = cnt[2 * b] + cnt[2 * b + 1];
        __syncthreads();
        for (int b = t; b < L / 2; b += EB) cnt[b] = cnt2[b];
        __syncthreads();
        L /= 2;
        g *= 2;
    }
    const double step = width * g;
    // non-empty merged bins, in order (wave 0 compacts with ballots)
    if (wv == 0) {
        int nb = 0, bf = -1, bl = -1;
        for (int b0 = 0; b0 < L; b0 += 64) {
            const int b = b0 + lane;
            const bool nz = b < L && cnt[b] > 0;
            const uint64_t mask = __ballot(nz);
            if (nz) {
                const int j = nb + __popcll(mask & lanemask_lt());
                xs[j] = lo + ((double)b + 0.5) * step;
                ws[j] = (double)cnt[b];
                ys[j] = log((double)cnt[b]);
            }
            if (mask) {
                if (bf < 0) bf = b0 + __ffsll((unsigned long long)mask) - 1;
                bl = b0 + 63 - __clzll(mask);
            }
            nb += __popcll(mask);
        }
        if (lane == 0) {
            s_nb = nb;
            s_bf = bf;
            s_bl = bl;
        }
    }
    __syncthreads();
    const int nb = s_nb, bf = s_bf, bl = s_bl;
    double* f = fit + 4 * (int64_t)h;
    if (nb == 0) {
        if (t == 0) {
            f[0] = f[1] = f[2] = f[3] = NAN;
            status[h] = -1;
            if (merge) merge[h] = g;
        }
        return;
    }
    // least cost over the merged-bin centres; ties go to the lowest bin
    double bj = INFINITY;
    int bb = -1;
    if (nb >= 4)
        for (int b = bf + wv; b <= bl; b += EB / 64) {
            const double J = wave_cost(xs, ws, ys, nb, lo + ((double)b + 0.5) * step, nullptr);
            if (J < bj) {
                bj = J;
                bb = b;
            }
        }
    if (lane == 0) {
        bestJ[wv] = bj;
        bestB[wv] = bb;
    }
    __syncthreads();
    if (wv != 0) return;
    double best = bestJ[0];
    int bbest = bestB[0];
    for (int w = 1; w < EB / 64; ++w)
        if (bestJ[w] < best || (bestJ[w] == best && bestB[w] >= 0 && bestB[w] < bbest)) {
            best = bestJ[w];
            bbest = bestB[w];
        }
    bool ok = false;
    double res[4];
    if (isfinite(best)) {
        const double cbest = lo + ((double)bbest + 0.5) * step;
        const double phi = 0.6180339887498949;
        double a = cbest - step, b = cbest + step;
        double x1 = b - phi * (b - a), x2 = a + phi * (b - a);
        double f1 = wave_cost(xs, ws, ys, nb, x1, nullptr);
        double f2 = wave_cost(xs, ws, ys, nb, x2, nullptr);
        for (int it = 0; it < giters; ++it) {
            if (f1 < f2) {
                b = x2;
                x2 = x1;
                f2 = f1;
                x1 = b - phi * (b - a);
                f1 = wave_cost(xs, ws, ys, nb, x1, nullptr);
            } else {
                a = x1;
                x1 = x2;
                f1 = f2;
                x2 = a + phi * (b - a);
                f2 = wave_cost(xs, ws, ys, nb, x2, nullptr);
            }
        }
        double c = 0.5 * (a + b);
        if (!(wave_cost(xs, ws, ys, nb, c, nullptr) <= best)) c = cbest;
        double apq[3];
        wave_cost(xs, ws, ys, nb, c, apq);
        if (apq[1] > 0 && apq[2] > 0) {
            res[0] = c;
            res[1] = 1.0 / sqrt(2.0 * apq[2]);
            res[2] = sqrt(apq[2] / apq[1]);
            res[3] = exp(apq[0]);
            ok = true;
        }
    }
    if (!ok) {
        // mean and dispersion of the merged histogram
        double sw = 0, swx = 0, m = 0;
        for (int j = lane; j < nb; j += 64) {
            sw += ws[j];
            swx += ws[j] * xs[j];
            m = fmax(m, ws[j]);
        }
        sw = wave_sum(sw);
        swx = wave_sum(swx);
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
        const double mean = swx / sw;
        double sxx = 0;
        for (int j = lane; j < nb; j += 64) sxx += ws[j] * (xs[j] - mean) * (xs[j] - mean);
        const double sd = sqrt(wave_sum(sxx) / sw);
        res[0] = mean;
        res[1] = sd > 0 ? sd : step;
        res[2] = 1.0;
        res[3] = m;
    }
    if (lane == 0) {
        f[0] = res[0];
        f[1] = res[1];
        f[2] = res[2];
        f[3] = res[3];
        status[h] = ok ? 1 : 0;
        if (merge) merge[h] = g;
    }
}

__global__ void k_ell_apply(int64_t M, const int32_t* __restrict__ mem, const int32_t* __restrict__ owner,
                            const float* __restrict__ R, const double* __restrict__ fit, float* __restrict__ ell) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const int i = mem[k];
    const int h = owner[k];
    ell[i] = (float)(((double)R[i] - fit[4 * (int64_t)h]) / fit[4 * (int64_t)h + 1]);
}

// (group, order-preserving bits of L) keys with the member as value
__global__ void k_clean_keys(int64_t M, const int32_t* __restrict__ mem, const int32_t* __restrict__ owner,
                             const float* __restrict__ ell, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const int i = mem[k];
    const uint32_t u = __float_as_uint(ell[i]);
    const uint32_t ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    keys[k] = ((uint64_t)(uint32_t)owner[k] << 32) | ord;
    vals[k] = (uint32_t)i;
}

// Per group: kstar = the smallest k such that the N - k members of largest L
// have mean >= Lbar (1 + beta / sqrt(N - k)) with N - k >= n_min; N if none.
__global__ __launch_bounds__(EB) void k_clean_eval(const int32_t* __restrict__ off, const uint32_t* __restrict__ sorted,
                                                   const float* __restrict__ ell, double Lbar, double beta, int n_min,
                                                   int32_t* __restrict__ kstar) {
    __shared__ double wsum[EB / 64];
    __shared__ int wmin[EB / 64];
    const int g = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int s = off[g], N = off[g + 1] - off[g];
    double carry = 0;  // sum of the positions above the current chunk
    int kbest = N;
    // chunks of EB positions from the top; thread t of a chunk holds
    // position top - t, so an inclusive prefix over t is a suffix sum
    for (int top = N - 1; top >= 0; top -= EB) {
        const int k = top - t;
        double v = k >= 0 ? (double)ell[sorted[s + k]] : 0.0;
        // inclusive scan over the wave, then over the waves
        for (int o = 1; o < 64; o <<= 1) {
            const double u = __shfl_up(v, o, 64);
            if (lane >= o) v += u;
        }
        if (lane == 63) wsum[wv] = v;
        __syncthreads();
        double before = carry;
        for (int w = 0; w < wv; ++w) before += wsum[w];
        double chunk = 0;
        for (int w = 0; w < EB / 64; ++w) chunk += wsum[w];
        const double S = before + v;  // sum of positions k .. N-1
        if (k >= 0) {
            const int m = N - k;
            if (m >= n_min && S / (double)m >= Lbar * (1.0 + beta / sqrt((double)m))) kbest = min(kbest, k);
        }
        carry += chunk;
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) kbest = min(kbest, __shfl_xor(kbest, o, 64));
    if (lane == 0) wmin[wv] = kbest;
    __syncthreads();
    if (t == 0) {
        int kb = wmin[0];
        for (int w = 1; w < EB / 64; ++w) kb = min(kb, wmin[w]);
        kstar[g] = kb;
    }
}

__global__ void k_clean_mark(const int32_t* __restrict__ off, const int32_t* __restrict__ owner,
                             const uint32_t* __restrict__ sorted, const int32_t* __restrict__ kstar, int64_t M,
                             uint8_t* __restrict__ gone) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const int g = owner[k];
    gone[sorted[k]] = (k - off[g]) < kstar[g] ? 1 : 0;
}

// One wave per group: kept members take the smallest kept index.
__global__ void k_clean_relabel(const int32_t* __restrict__ off, const int32_t* __restrict__ mem,
                                const uint8_t* __restrict__ gone, int32_t* __restrict__ label) {
    const int g = blockIdx.x;
    const int lane = threadIdx.x;
    const int s = off[g], e = off[g + 1];
    int root = -1;
    for (int k0 = s; k0 < e && root < 0; k0 += 64) {
        const int k = k0 + lane;
        const uint64_t kept = __ballot(k < e && !gone[mem[k]]);
        if (kept) root = __shfl(k < e ? mem[k] : 0, __ffsll((unsigned long long)kept) - 1, 64);
    }
    for (int k = s + lane; k < e; k += 64) {
        const int i = mem[k];
        label[i] = gone[i] ? -1 : root;
    }
}

}  // namespace
}  // namespace vr

using namespace vr;

extern "C" int vr_ell_fit(vr_ctx* ctx, int64_t n, int32_t n_hosts, const int32_t* host_offsets,
                          const int32_t* host_members, const float* R, const vr_ell_params* ep, double* fit,
                          int32_t* status, int32_t* merge, float* ell, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_hosts(ctx, n_hosts, host_offsets, host_members);
    if (rc) return rc;
    if (!ep) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL vr_ell_params");
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, VR_ERR_INVALID_ARG, "n out of range");
    if (!(ep->width > 0) || !std::isfinite(ep->lo) || ep->nbins < 1 || ep->nbins > MAXBINS || ep->max_merge < 1 ||
        (ep->max_merge & (ep->max_merge - 1)) || ep->nbins % ep->max_merge || ep->peak_min < 1 ||
        ep->golden_iters < 0 || ep->golden_iters > 200)
        return set_err(ctx, VR_ERR_INVALID_ARG, "invalid vr_ell_params");
    if (n_hosts == 0) return VR_OK;
    if (!R || !fit || !status || !ell) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> off;
    rc = read_host_offsets(ctx, n_hosts, host_offsets, n, 0, off, st);
    if (rc) return rc;
    const int64_t M = off[n_hosts];
    VR_WS(owner, ctx, int32_t, WS_A0, M);
    VR_WS(hist, ctx, uint32_t, WS_A1, (int64_t)n_hosts * ep->nbins);
    VR_TIMED(ctx, "ell_fit", st, M, {
        hipLaunchKernelGGL(k_elem_owner, dim3(n_hosts), dim3(256), 0, st, host_offsets, owner);
        rc = fill_u32(ctx, hist, 0u, (int64_t)n_hosts * ep->nbins, st);
        if (rc == VR_OK && M > 0)
            hipLaunchKernelGGL(k_ell_hist, dim3(grid_for(M, HCHUNK)), dim3(EB), 0, st, M, host_members, owner, R,
                               ep->lo, 1.0 / ep->width, ep->nbins, hist);
        if (rc == VR_OK)
            hipLaunchKernelGGL(k_ell_fit, dim3(n_hosts), dim3(EB), 0, st, hist, ep->nbins, ep->lo, ep->width,
                               ep->peak_min, ep->max_merge, ep->golden_iters, fit, status, merge);
        if (rc == VR_OK && M > 0)
            hipLaunchKernelGGL(k_ell_apply, dim3(grid_for(M, 256)), dim3(256), 0, st, M, host_members, owner, R, fit,
                               ell);
    });
    if (rc) return rc;
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

extern "C" int vr_ell_clean(vr_ctx* ctx, int64_t n, int32_t n_groups, const int32_t* offsets,
                            const int32_t* members, const float* ell, double ell_th, double beta, int32_t n_min,
                            int32_t* label, int32_t* removed, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_hosts(ctx, n_groups, offsets, members);
    if (rc) return rc;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, VR_ERR_INVALID_ARG, "n out of range");
    if (n_min < 1 || !std::isfinite(ell_th) || !std::isfinite(beta))
        return set_err(ctx, VR_ERR_INVALID_ARG, "need n_min >= 1 and finite ell_th, beta");
    if (n_groups == 0) return VR_OK;
    if (!ell || !label) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> off;
    rc = read_host_offsets(ctx, n_groups, offsets, n, 0, off, st);
    if (rc) return rc;
    const int64_t M = off[n_groups];
    if (M == 0) return VR_OK;
    const double Lbar = std::sqrt(2.0 / M_PI) * std::exp(-0.5 * ell_th * ell_th) / std::erfc(ell_th / std::sqrt(2.0));
    VR_WS(owner, ctx, int32_t, WS_A0, M);
    VR_WS(keys, ctx, uint64_t, WS_A1, M);
    VR_WS(vals, ctx, uint32_t, WS_A2, M);
    VR_WS(gone, ctx, uint8_t, WS_A3, n);
    VR_WS(kst, ctx, int32_t, WS_A4, n_groups);
    int gbits = 1;
    while ((int64_t(1) << gbits) < n_groups) ++gbits;
    VR_TIMED(ctx, "ell_clean", st, M, {
        hipLaunchKernelGGL(k_elem_owner, dim3(n_groups), dim3(256), 0, st, offsets, owner);
        hipLaunchKernelGGL(k_clean_keys, dim3(grid_for(M, 256)), dim3(256), 0, st, M, members, owner, ell, keys,
                           vals);
        rc = sort_pairs_u64(ctx, keys, vals, M, 32 + gbits, st);
        if (rc == VR_OK) {
            hipLaunchKernelGGL(k_clean_eval, dim3(n_groups), dim3(EB), 0, st, offsets, vals, ell, Lbar, beta, n_min,
                               kst);
            hipLaunchKernelGGL(k_clean_mark, dim3(grid_for(M, 256)), dim3(256), 0, st, offsets, owner, vals, kst, M,
                               gone);
            hipLaunchKernelGGL(k_clean_relabel, dim3(n_groups), dim3(64), 0, st, offsets, members, gone, label);
        }
    });
    if (rc) return rc;
    VR_LAUNCH_CHECK(ctx);
    if (removed) VR_HIP(ctx, hipMemcpyAsync(removed, kst, n_groups * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    return VR_OK;
}
