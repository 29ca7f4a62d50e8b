// vr_kd.hip -- level-synchronous KD trees over the members of many hosts.
//
// Each active node is one workgroup: it reduces the members' bounding box,
// chooses the split dimension (normalised Shannon entropy of the binned
// member masses, Sec. 2.2, or the widest extent for the neighbour-search
// tree), finds the member of rank floor(n/2) in (coordinate, index) order with
// a two-pass 11-bit radix select, and writes a stable partition into the other
// element buffer.  Node segments therefore stay in ascending particle-index
// order, which makes every split exactly reproducible.
#include "vr_kd.h"

#include <climits>
#include <cmath>

namespace vr {
namespace {

constexpr int KB = 256;

__device__ __forceinline__ uint32_t wave_incl_scan_u(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t block_excl_scan_u(uint32_t v, uint32_t* sm, uint32_t* total) {
    const int lane = __lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t inc = wave_incl_scan_u(v);
    if (lane == 63) sm[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) pre += sm[i];
        tot += sm[i];
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

// Bounding box of positions [s, e) reduced over the block into smn/smx.
__device__ void block_bbox(const Elems& src, int s, int e, int* s_mn, int* s_mx, int (*smn)[4], int (*smx)[4]) {
    int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
    for (int k = s + (int)threadIdx.x; k < e; k += blockDim.x)
        for (int d = 0; d < 3; ++d) {
            int u = src.u[d][k];
            mn[d] = min(mn[d], u);
            mx[d] = max(mx[d], u);
        }
    const int lane = __lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int d = 0; d < 3; ++d) {
        for (int o = 32; o > 0; o >>= 1) {
            mn[d] = min(mn[d], __shfl_xor(mn[d], o, 64));
            mx[d] = max(mx[d], __shfl_xor(mx[d], o, 64));
        }
        if (lane == 0) { smn[d][w] = mn[d]; smx[d][w] = mx[d]; }
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int a = INT_MAX, b = INT_MIN;
        for (int ww = 0; ww < nw; ++ww) { a = min(a, smn[threadIdx.x][ww]); b = max(b, smx[threadIdx.x][ww]); }
        s_mn[threadIdx.x] = a;
        s_mx[threadIdx.x] = b;
    }
    __syncthreads();
}

__global__ void k_kd_init(int n_hosts, const int32_t* __restrict__ off, const int32_t* __restrict__ mem,
                          const uint32_t* __restrict__ qx, const uint32_t* __restrict__ qy,
                          const uint32_t* __restrict__ qz, const float* __restrict__ mass, int gb, Elems A) {
    const int h = blockIdx.x;
    const int s = off[h], e = off[h + 1];
    const int r = mem[s];
    const int rx = (int)qx[r], ry = (int)qy[r], rz = (int)qz[r];
    for (int k = s + threadIdx.x; k < e; k += blockDim.x) {
        const int i = mem[k];
        A.u[0][k] = rx + min_image((int)qx[i] - rx, gb);
        A.u[1][k] = ry + min_image((int)qy[i] - ry, gb);
        A.u[2][k] = rz + min_image((int)qz[i] - rz, gb);
        A.gidx[k] = i;
        if (mass) A.mass[k] = mass[i];
    }
}

__global__ __launch_bounds__(KB) void k_kd_roots(const int32_t* __restrict__ off, const int* __restrict__ ncell,
                                                 Elems A, KdNode* nodes, int* active, int* n_active, int* leaves,
                                                 int* n_leaves, int* active_members) {
    __shared__ int smn[3][4], smx[3][4];
    __shared__ int s_mn[3], s_mx[3];
    const int h = blockIdx.x;
    const int s = off[h], e = off[h + 1];
    block_bbox(A, s, e, s_mn, s_mx, smn, smx);
    if (threadIdx.x == 0) {
        KdNode nd;
        nd.host = h; nd.start = s; nd.end = e; nd.buf = 0;
        for (int d = 0; d < 3; ++d) {
            nd.lo[d] = nd.bmin[d] = s_mn[d];
            nd.hi[d] = nd.bmax[d] = s_mx[d];
        }
        nd.dim = -1; nd.t = 0; nd.left = nd.right = -1;
        nodes[h] = nd;
        if (e - s > ncell[h]) {
            active[atomicAdd(n_active, 1)] = h;
            atomicAdd(active_members, e - s);
        } else {
            leaves[atomicAdd(n_leaves, 1)] = h;
        }
    }
}

__global__ __launch_bounds__(KB) void k_kd_level(KdNode* __restrict__ nodes, const int* __restrict__ active,
                                                 int* __restrict__ next_active, int* __restrict__ n_next,
                                                 int* __restrict__ leaves, int* __restrict__ n_leaves,
                                                 int* __restrict__ n_nodes, int* __restrict__ next_members, Elems A,
                                                 Elems B, const int* __restrict__ ncell, int nb, int mode,
                                                 int use_mass) {
    __shared__ int smn[3][4], smx[3][4];
    __shared__ double hist[3][64];
    __shared__ uint32_t sel[2048];
    __shared__ uint32_t scan_sm[8];
    __shared__ int s_best, s_b1, s_below1, s_b2, s_below2;
    __shared__ int s_mn[3], s_mx[3];

    const int id = active[blockIdx.x];
    const KdNode nd = nodes[id];
    const Elems src = nd.buf ? B : A;
    const Elems dst = nd.buf ? A : B;
    const int start = nd.start, end = nd.end, n = end - start;
    const int tid = threadIdx.x;

    if (mode != KD_WIDEST)
        for (int i = tid; i < 3 * 64; i += blockDim.x) (&hist[0][0])[i] = 0.0;
    block_bbox(src, start, end, s_mn, s_mx, smn, smx);
    if (mode != KD_WIDEST) {
        // mass histograms of the non-degenerate dimensions
        for (int k = start + tid; k < end; k += blockDim.x) {
            const double wgt = use_mass ? (double)src.mass[k] : 1.0;
            for (int d = 0; d < 3; ++d) {
                if (s_mx[d] == s_mn[d]) continue;
                const int64_t bin = ((int64_t)(src.u[d][k] - s_mn[d]) * nb) / ((int64_t)s_mx[d] - s_mn[d] + 1);
                atomicAdd(&hist[d][bin], wgt);
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        int best = -1;
        if (mode == KD_WIDEST) {
            for (int d = 0; d < 3; ++d)
                if (s_mx[d] > s_mn[d] && (best < 0 || s_mx[d] - s_mn[d] > s_mx[best] - s_mn[best])) best = d;
        } else {
            double S[3];
            for (int d = 0; d < 3; ++d) {
                S[d] = 0.0;
                if (s_mx[d] == s_mn[d]) continue;
                double tot = 0.0;
                for (int k = 0; k < nb; ++k) tot += hist[d][k];
                double sacc = 0.0;
                for (int k = 0; k < nb; ++k)
                    if (hist[d][k] > 0) {
                        double pk = hist[d][k] / tot;
                        sacc -= pk * log(pk);
                    }
                S[d] = sacc / log((double)nb);
            }
            for (int d = 0; d < 3; ++d) {
                if (s_mx[d] == s_mn[d]) continue;
                if (best < 0) { best = d; continue; }
                bool better = mode == KD_MIN_ENTROPY ? (S[d] < S[best] - 1e-12) : (S[d] > S[best] + 1e-12);
                if (better) best = d;
            }
        }
        s_best = best;
        for (int d = 0; d < 3; ++d) {
            nodes[id].bmin[d] = s_mn[d];
            nodes[id].bmax[d] = s_mx[d];
        }
    }
    __syncthreads();
    const int best = s_best;
    if (best < 0) {  // all members coincide: the node stays a leaf
        if (tid == 0) leaves[atomicAdd(n_leaves, 1)] = id;
        return;
    }
    const int dmin = s_mn[best];
    const int nl = n / 2;
    const int* ub = src.u[best];
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = tid; i < 2048; i += blockDim.x) sel[i] = 0;
        __syncthreads();
        const int b1 = pass ? s_b1 : 0;
        for (int k = start + tid; k < end; k += blockDim.x) {
            const uint32_t v = (uint32_t)(ub[k] - dmin);
            if (pass == 0) atomicAdd(&sel[v >> 11], 1u);
            else if ((int)(v >> 11) == b1) atomicAdd(&sel[v & 2047u], 1u);
        }
        __syncthreads();
        const int want = pass ? nl - s_below1 : nl;
        uint32_t loc = 0;
        for (int i = 0; i < 8; ++i) loc += sel[tid * 8 + i];
        uint32_t tot;
        const uint32_t ex = block_excl_scan_u(loc, scan_sm, &tot);
        if ((uint32_t)want >= ex && (uint32_t)want < ex + loc) {
            uint32_t c = ex;
            for (int i = 0; i < 8; ++i) {
                const uint32_t h = sel[tid * 8 + i];
                if ((uint32_t)want < c + h) {
                    if (pass == 0) { s_b1 = tid * 8 + i; s_below1 = (int)c; }
                    else { s_b2 = tid * 8 + i; s_below2 = (int)c; }
                    break;
                }
                c += h;
            }
        }
        __syncthreads();
    }
    const int t = dmin + ((s_b1 << 11) | s_b2);
    const int need = nl - (s_below1 + s_below2);  // members equal to t that go left
    uint32_t carry_l = 0, carry_e = 0, carry_r = 0;
    for (int base = start; base < end; base += blockDim.x) {
        const int k = base + tid;
        const bool valid = k < end;
        const int v = valid ? ub[k] : 0;
        const bool is_less = valid && v < t;
        const bool is_eq = valid && v == t;
        uint32_t tot_e;
        const uint32_t eq_before = block_excl_scan_u(is_eq ? 1u : 0u, scan_sm, &tot_e) + carry_e;
        const bool left = is_less || (is_eq && (int)eq_before < need);
        const bool right = valid && !left;
        uint32_t tot_lr;
        const uint32_t pk = block_excl_scan_u((left ? 1u : 0u) | (right ? (1u << 10) : 0u), scan_sm, &tot_lr);
        if (valid) {
            const int pos = left ? start + (int)(carry_l + (pk & 1023u)) : start + nl + (int)(carry_r + (pk >> 10));
            dst.u[0][pos] = src.u[0][k];
            dst.u[1][pos] = src.u[1][k];
            dst.u[2][pos] = src.u[2][k];
            dst.gidx[pos] = src.gidx[k];
            if (use_mass) dst.mass[pos] = src.mass[k];
        }
        carry_e += tot_e;
        carry_l += tot_lr & 1023u;
        carry_r += tot_lr >> 10;
    }
    if (tid == 0) {
        const int c0 = atomicAdd(n_nodes, 2);
        KdNode L = nd, R = nd;
        L.buf = R.buf = nd.buf ^ 1;
        L.end = start + nl;
        R.start = start + nl;
        L.hi[best] = t - 1;
        R.lo[best] = t;
        L.dim = R.dim = -1;
        L.left = L.right = R.left = R.right = -1;
        nodes[c0] = L;
        nodes[c0 + 1] = R;
        nodes[id].dim = best;
        nodes[id].t = t;
        nodes[id].left = c0;
        nodes[id].right = c0 + 1;
        const int nc = ncell[nd.host];
        int grow = 0;
        if (nl > nc) { next_active[atomicAdd(n_next, 1)] = c0; grow += nl; }
        else leaves[atomicAdd(n_leaves, 1)] = c0;
        if (n - nl > nc) { next_active[atomicAdd(n_next, 1)] = c0 + 1; grow += n - nl; }
        else leaves[atomicAdd(n_leaves, 1)] = c0 + 1;
        if (grow) atomicAdd(next_members, grow);  // members the next level will visit
    }
}

// Leaves: bounding box of the members, and their segment moved into buffer A.
__global__ __launch_bounds__(KB) void k_kd_leaves(const int* __restrict__ leaves, KdNode* __restrict__ nodes, Elems A,
                                                  Elems B, int use_mass) {
    __shared__ int smn[3][4], smx[3][4];
    __shared__ int s_mn[3], s_mx[3];
    const int id = leaves[blockIdx.x];
    const KdNode nd = nodes[id];
    if (nd.buf)
        for (int k = nd.start + threadIdx.x; k < nd.end; k += blockDim.x) {
            A.u[0][k] = B.u[0][k];
            A.u[1][k] = B.u[1][k];
            A.u[2][k] = B.u[2][k];
            A.gidx[k] = B.gidx[k];
            if (use_mass) A.mass[k] = B.mass[k];
        }
    __syncthreads();
    block_bbox(A, nd.start, nd.end, s_mn, s_mx, smn, smx);
    if (threadIdx.x == 0) {
        for (int d = 0; d < 3; ++d) {
            nodes[id].bmin[d] = s_mn[d];
            nodes[id].bmax[d] = s_mx[d];
        }
        nodes[id].buf = 0;
    }
}

}  // namespace

int read_host_offsets(vr_ctx* ctx, int32_t n_hosts, const int32_t* host_offsets, int64_t n, int64_t min_size,
                      std::vector<int32_t>& off, hipStream_t st) {
    off.assign(n_hosts + 1, 0);
    if (n_hosts == 0) return VR_OK;
    VR_HIP(ctx, hipMemcpyAsync(off.data(), host_offsets, (n_hosts + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    VR_HIP(ctx, hipStreamSynchronize(st));
    if (off[0] != 0) return set_err(ctx, VR_ERR_INVALID_ARG, "host_offsets[0] must be 0");
    for (int h = 0; h < n_hosts; ++h) {
        const int64_t NH = (int64_t)off[h + 1] - off[h];
        if (NH < min_size)
            return set_err(ctx, VR_ERR_INVALID_ARG, "host %d has %lld members (need >= %lld)", h, (long long)NH,
                           (long long)min_size);
    }
    if (off[n_hosts] > n) return set_err(ctx, VR_ERR_INVALID_ARG, "more host members than particles");
    return VR_OK;
}

int kd_build(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts, const int32_t* host_offsets,
             const int32_t* host_members, const std::vector<int32_t>& off, const std::vector<int>& ncell, int mode,
             int nbins, KdTree& tree, hipStream_t st) {
    int64_t node_cap = 0;
    for (int h = 0; h < n_hosts; ++h) {
        const int64_t NH = (int64_t)off[h + 1] - off[h];
        const int64_t minleaf = std::max<int64_t>(1, (ncell[h] + 1) / 2);
        node_cap += 2 * ((NH + minleaf - 1) / minleaf) + 1;
    }
    const int64_t M = off[n_hosts];
    const int use_mass = p->mass ? 1 : 0;
    Elems A, B;
    VR_WS(a0, ctx, int, WS_A0, M); VR_WS(a1, ctx, int, WS_A1, M); VR_WS(a2, ctx, int, WS_A2, M);
    VR_WS(ag, ctx, int, WS_A3, M); VR_WS(am, ctx, float, WS_A4, use_mass ? M : 1);
    VR_WS(b0, ctx, int, WS_B0, M); VR_WS(b1, ctx, int, WS_B1, M); VR_WS(b2, ctx, int, WS_B2, M);
    VR_WS(bg, ctx, int, WS_B3, M); VR_WS(bm, ctx, float, WS_B4, use_mass ? M : 1);
    A.u[0] = a0; A.u[1] = a1; A.u[2] = a2; A.gidx = ag; A.mass = am;
    B.u[0] = b0; B.u[1] = b1; B.u[2] = b2; B.gidx = bg; B.mass = bm;
    VR_WS(nodes, ctx, KdNode, WS_A5, node_cap);
    VR_WS(act0, ctx, int, WS_A6, node_cap);
    VR_WS(act1, ctx, int, WS_A7, node_cap);
    VR_WS(leaves, ctx, int, WS_A8, node_cap);
    VR_WS(ncell_d, ctx, int, WS_B5, n_hosts);
    // counters: 0 active nodes now, 1 active next, 2 leaves, 3 nodes, 4 members now, 5 members next
    VR_WS(counters, ctx, int, WS_FLAG, 8);
    VR_HIP(ctx, hipMemcpyAsync(ncell_d, ncell.data(), n_hosts * sizeof(int), hipMemcpyHostToDevice, st));
    int* init_counts = reinterpret_cast<int*>(ctx->pinned);
    for (int k = 0; k < 8; ++k) init_counts[k] = 0;
    init_counts[3] = n_hosts;
    VR_HIP(ctx, hipMemcpyAsync(counters, init_counts, 8 * sizeof(int), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_kd_init, dim3(n_hosts), dim3(256), 0, st, n_hosts, host_offsets, host_members, p->qx, p->qy,
                       p->qz, p->mass, p->grid_bits, A);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_kd_roots, dim3(n_hosts), dim3(KB), 0, st, host_offsets, ncell_d, A, nodes, act0, counters + 0,
                       leaves, counters + 2, counters + 4);
    VR_LAUNCH_CHECK(ctx);
    int* cur = act0;
    int* nxt = act1;
    for (int level = 0;; ++level) {
        int cnt[8];
        int rc = read_back(ctx, counters, cnt, sizeof cnt, st);
        if (rc) return rc;
        const int na = cnt[0];
        if (na == 0) break;
        if (level >= 64) return set_err(ctx, VR_ERR_NOT_CONVERGED, "KD build exceeded 64 levels");
        rc = fill_i32(ctx, counters + 1, 0, 1, st);
        if (rc) return rc;
        rc = fill_i32(ctx, counters + 5, 0, 1, st);
        if (rc) return rc;
        VR_TIMED(ctx, "kd_level", st, cnt[4],
                 hipLaunchKernelGGL(k_kd_level, dim3(na), dim3(KB), 0, st, nodes, cur, nxt, counters + 1, leaves,
                                    counters + 2, counters + 3, counters + 5, A, B, ncell_d, nbins, mode, use_mass));
        VR_LAUNCH_CHECK(ctx);
        VR_HIP(ctx, hipMemcpyAsync(counters + 0, counters + 1, sizeof(int), hipMemcpyDeviceToDevice, st));
        VR_HIP(ctx, hipMemcpyAsync(counters + 4, counters + 5, sizeof(int), hipMemcpyDeviceToDevice, st));
        std::swap(cur, nxt);
    }
    int nleaf = 0;
    int rc = read_back(ctx, counters + 2, &nleaf, sizeof nleaf, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_kd_leaves, dim3(nleaf), dim3(KB), 0, st, leaves, nodes, A, B, use_mass);
    VR_LAUNCH_CHECK(ctx);
    tree.nodes = nodes;
    tree.leaves = leaves;
    tree.n_leaves = nleaf;
    tree.F = A;
    tree.use_mass = use_mass;
    return VR_OK;
}

}  // namespace vr
