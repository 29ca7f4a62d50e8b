// vr_kd.hip -- level-synchronous KD trees over the members of many hosts,
// built from presorted lists.
//
// For each dimension d the members are sorted once by (host, u_d, index)
// with the device radix sort.  Every node then owns the same position range
// in the three lists, and the list of dimension d holds its members in
// (u_d, index) order, so the member of rank floor(n/2) -- the split point --
// and the bounding box are read off directly.  One level costs a handful of
// element-parallel passes for all nodes of all hosts at once: entropy
// histograms (cells tree), the split decision per node, a left/right flag
// per member, and a stable partition of each list by a global prefix sum
// (subtracting the prefix at the segment start makes it segmented).  No
// node is ever handled by a single workgroup, so the few huge top-level
// nodes cost no more per member than the many small ones.  The levels and
// the active-node counts that size their launches follow from the host
// sizes alone, so the whole build is queued without waiting on the device;
// the kernels read the true counts, which only nodes of coincident members
// (kept as leaves) make smaller.
#include "vr_kd.h"

#include <climits>
#include <cmath>

namespace vr {
namespace {

constexpr int KB = 256;
constexpr int HCH = 2048;  // positions per histogram block
constexpr int HASH_SLOTS = 256;  // partial sums of the content hash

// One element's share of the content hash of a build's inputs: a 64-bit
// mix of its position, member, unwrapped coordinates and host.  The shares
// are summed, so the hash covers every element whatever the order of the
// additions.
__device__ __forceinline__ unsigned long long elem_hash(int64_t e, int i, int a, int b, int c, int h) {
    uint64_t x = (uint64_t)e * 0x9E3779B97F4A7C15ull;
    x ^= (uint64_t)(uint32_t)i * 0xC2B2AE3D27D4EB4Full;
    x ^= (((uint64_t)(uint32_t)a << 32) | (uint32_t)b) * 0x165667B19E3779F9ull;
    x ^= (((uint64_t)(uint32_t)c << 32) | (uint32_t)h) * 0x27D4EB2F165667C5ull;
    x ^= x >> 31;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 29;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 32;
    return (unsigned long long)x;
}

// Element arrays by element id, and the sort keys of the presort; the
// HASH_SLOTS words of hash (zeroed beforehand) receive partial sums of the
// content hash of (member, coordinates, host) over all elements, one slot
// per wavefront in turn, so no single address takes every wavefront's add.
__global__ void k_elems(int64_t M, int n_hosts, const int32_t* __restrict__ off, const int32_t* __restrict__ mem,
                        const uint32_t* __restrict__ qx, const uint32_t* __restrict__ qy,
                        const uint32_t* __restrict__ qz, const float* __restrict__ mass, int gb, int* __restrict__ u0,
                        int* __restrict__ u1, int* __restrict__ u2, int* __restrict__ g, float* __restrict__ m,
                        int* __restrict__ host, unsigned long long* __restrict__ hash) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long hv = 0;
    if (e < M) {
        int lo = 0, hi = n_hosts - 1;  // host with off[h] <= e < off[h+1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const int h = lo;
        const int r = mem[off[h]];
        const int i = mem[e];
        const int rx = (int)qx[r], ry = (int)qy[r], rz = (int)qz[r];
        const int a = rx + min_image((int)qx[i] - rx, gb), b = ry + min_image((int)qy[i] - ry, gb),
                  c = rz + min_image((int)qz[i] - rz, gb);
        u0[e] = a;
        u1[e] = b;
        u2[e] = c;
        g[e] = i;
        host[e] = h;
        if (mass) m[e] = mass[i];
        hv = elem_hash(e, i, a, b, c, h);
    }
    // every lane of the wavefront reaches the sum
    for (int o = 32; o > 0; o >>= 1) hv += (unsigned long long)__shfl_xor((long long)hv, o, 64);
    if ((threadIdx.x & 63) == 0 && hv)
        atomicAdd(&hash[((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % HASH_SLOTS], hv);
}

__global__ void k_presort_keys(int64_t M, const int* __restrict__ u, const int* __restrict__ host,
                               uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M) return;
    // unwrapped coordinates lie in [-2^20, 3 * 2^20): 22 bits after the shift
    key[e] = ((uint64_t)host[e] << 22) | (uint64_t)(uint32_t)(u[e] + (1 << 20));
    val[e] = (uint32_t)e;
}

__global__ void k_roots(int n_hosts, const int32_t* __restrict__ off, const int* __restrict__ ncell, KdNode* nodes,
                        int* active, int* counters, int* leaves, int* __restrict__ seg_node_unused) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n_hosts) return;
    KdNode nd;
    nd.host = h;
    nd.start = off[h];
    nd.end = off[h + 1];
    nd.slot = -1;
    nd.dim = -1;
    nd.t = 0;
    nd.left = nd.right = -1;
    for (int d = 0; d < 3; ++d) nd.lo[d] = nd.hi[d] = nd.bmin[d] = nd.bmax[d] = 0;
    nodes[h] = nd;
    if (nd.end - nd.start > ncell[h]) {
        active[atomicAdd(&counters[0], 1)] = h;
        atomicAdd(&counters[4], nd.end - nd.start);
    } else {
        leaves[atomicAdd(&counters[2], 1)] = h;
    }
    (void)seg_node_unused;
}

// Between two levels: the next level's active-node and member counts become
// the current ones, and the next ones restart from zero (counters[0] and
// [4] are this level's, [1] and [5] the next level's).  One thread.
__global__ void k_level_counters(int* counters, int roll, int clear) {
    if (threadIdx.x != 0) return;
    if (roll) {
        counters[0] = counters[1];
        counters[4] = counters[5];
    }
    if (clear) {
        counters[1] = 0;
        counters[5] = 0;
    }
}

__global__ void k_seg_init(int64_t M, const int* __restrict__ host, int* __restrict__ seg_node) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < M) seg_node[p] = host[p];  // hosts keep their ranges in every list
}

// Bounding box of every active node from the sorted lists; the root region is
// its bounding box.
__global__ void k_bbox(const int* __restrict__ nact, const int* __restrict__ active, KdNode* nodes,
                       const int* __restrict__ l0, const int* __restrict__ l1, const int* __restrict__ l2,
                       const int* __restrict__ u0, const int* __restrict__ u1, const int* __restrict__ u2,
                       int n_hosts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *nact) return;
    const int id = active[i];
    KdNode& nd = nodes[id];
    const int s = nd.start, e = nd.end - 1;
    nd.bmin[0] = u0[l0[s]]; nd.bmax[0] = u0[l0[e]];
    nd.bmin[1] = u1[l1[s]]; nd.bmax[1] = u1[l1[e]];
    nd.bmin[2] = u2[l2[s]]; nd.bmax[2] = u2[l2[e]];
    nd.slot = i;
    if (id < n_hosts)
        for (int d = 0; d < 3; ++d) { nd.lo[d] = nd.bmin[d]; nd.hi[d] = nd.bmax[d]; }
}

// Mass histograms (counts for uniform mass) of the active nodes, nb bins per
// dimension spanning the members' extent.  A block whose positions all
// belong to one node accumulates in LDS first.
// The three coordinates carried in list-0 order (null when no histogram
// needs them), permuted with list 0 at every level.
struct CoordsL0 {
    const int* in[3];
    int* out[3];
};

// Nodes of one chunk that get LDS histograms: slots [base, base + HK), base
// the slot of the chunk's first active end. Deep levels put several small
// nodes in a chunk; a node outside the window adds to global memory.
constexpr int HK = 8;

template <bool COUNTS>
__global__ __launch_bounds__(KB) void k_hist(int64_t M, const int* __restrict__ seg_node, const KdNode* __restrict__ nodes,
                                             const int* __restrict__ l0, const int* __restrict__ c0,
                                             const int* __restrict__ c1, const int* __restrict__ c2,
                                             const float* __restrict__ mass, int nb, uint32_t* __restrict__ hc,
                                             double* __restrict__ hm) {
    __shared__ uint32_t lc[COUNTS ? HK * 3 * 64 : 1];
    __shared__ double lm[COUNTS ? 1 : HK * 3 * 64];
    const int64_t p0 = (int64_t)blockIdx.x * HCH;
    const int64_t p1 = min(p0 + HCH, M);
    const KdNode& nf = nodes[seg_node[p0]];
    const KdNode& nl = nodes[seg_node[p1 - 1]];
    const bool af = nf.slot >= 0 && nf.dim < 0, al = nl.slot >= 0 && nl.dim < 0;
    if (&nf == &nl && !af) return;  // one node, not active this level
    const int base = af ? nf.slot : (al ? max(0, nl.slot - (HK - 1)) : -1);
    const int nb3 = 3 * nb;
    for (int k = threadIdx.x; k < HK * nb3; k += blockDim.x) {
        if (COUNTS) lc[k] = 0;
        else lm[k] = 0.0;
    }
    __syncthreads();
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const KdNode& nd = nodes[seg_node[p]];
        if (nd.slot < 0 || nd.dim >= 0) continue;
        const int li = base >= 0 ? nd.slot - base : -1;
        const bool local = li >= 0 && li < HK;
        const int u[3] = {c0[p], c1[p], c2[p]};  // coordinates in list-0 order
        const double w = COUNTS ? 1.0 : (double)mass[l0[p]];
        for (int d = 0; d < 3; ++d) {
            if (nd.bmax[d] == nd.bmin[d]) continue;
            const int bin = (int)(((int64_t)(u[d] - nd.bmin[d]) * nb) / ((int64_t)nd.bmax[d] - nd.bmin[d] + 1));
            if (local) {
                if (COUNTS) atomicAdd(&lc[li * nb3 + d * nb + bin], 1u);
                else atomicAdd(&lm[li * nb3 + d * nb + bin], w);
            } else {
                const int64_t at = ((int64_t)nd.slot * 3 + d) * nb + bin;
                if (COUNTS) atomicAdd(&hc[at], 1u);
                else atomicAdd(&hm[at], w);
            }
        }
    }
    if (base < 0) return;
    __syncthreads();
    // a nonzero entry belongs to an active node seen above, so its slot
    // base + k / nb3 is in range
    for (int k = threadIdx.x; k < HK * nb3; k += blockDim.x) {
        const int64_t at = (int64_t)base * nb3 + k;
        if (COUNTS) {
            if (lc[k]) atomicAdd(&hc[at], lc[k]);
        } else if (lm[k] != 0.0) {
            atomicAdd(&hm[at], lm[k]);
        }
    }
}

// Normalised Shannon entropy of each dimension's histogram (the entropy
// equation of Sec. 2.2) for every active node: one wavefront per node, one
// lane per bin, so the logarithms of a node are taken in parallel.
__global__ __launch_bounds__(256) void k_entropy(const int* __restrict__ nact, const int* __restrict__ active,
                                                 const KdNode* __restrict__ nodes, int nb, int counts,
                                                 const uint32_t* __restrict__ hc, const double* __restrict__ hm,
                                                 double* __restrict__ S) {
    const int i = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = __lane_id();
    if (i >= *nact) return;
    const KdNode& nd = nodes[active[i]];
    __shared__ double sh[4][64];
    __shared__ double stot[4];
    const int w = threadIdx.x >> 6;
    for (int d = 0; d < 3; ++d) {
        const int64_t b0 = ((int64_t)i * 3 + d) * nb;
        const double h = lane < nb ? (counts ? (double)hc[b0 + lane] : hm[b0 + lane]) : 0.0;
        // totals and entropy sums run over the bins in order, as a serial
        // loop would; only the logarithms are spread over the lanes
        sh[w][lane] = h;
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            double tot = 0.0;
            for (int k = 0; k < nb; ++k) tot += sh[w][k];
            stot[w] = tot;
        }
        __builtin_amdgcn_wave_barrier();
        const double tot = stot[w];
        double term = 0.0;
        if (h > 0) {
            const double pk = h / tot;
            term = -pk * log(pk);
        }
        __builtin_amdgcn_wave_barrier();
        sh[w][lane] = term;
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            double sacc = 0.0;
            for (int k = 0; k < nb; ++k) sacc += sh[w][k];
            S[3 * (int64_t)i + d] = nd.bmax[d] == nd.bmin[d] ? 0.0 : sacc / log((double)nb);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Reserves n slots of a global counter for each lane; one atomic per
// wavefront.  Every lane of the wavefront must call it.
__device__ __forceinline__ int wave_reserve(int* counter, int n) {
    const int lane = __lane_id();
    int x = n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
    }
    const int total = __shfl(x, 63, 64);
    int base = 0;
    if (lane == 63 && total > 0) base = atomicAdd(counter, total);
    base = __shfl(base, 63, 64);
    return base + x - n;
}

// Split decision of every active node and creation of its children.  All
// lanes run to the end (the counters are reserved per wavefront).
__global__ __launch_bounds__(256) void k_split(const int* nact, const int* __restrict__ active, KdNode* nodes,
                                               const int* __restrict__ l0, const int* __restrict__ l1,
                                               const int* __restrict__ l2, const int* __restrict__ u0,
                                               const int* __restrict__ u1, const int* __restrict__ u2, int mode,
                                               const double* __restrict__ Sdim, const int* __restrict__ ncell,
                                               int* next_active, int* leaves, int* counters) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < *nact;
    const int id = valid ? active[i] : 0;
    KdNode nd;
    int best = -1;
    if (valid) {
        nd = nodes[id];
        if (mode == KD_WIDEST) {
            for (int d = 0; d < 3; ++d)
                if (nd.bmax[d] > nd.bmin[d] && (best < 0 || nd.bmax[d] - nd.bmin[d] > nd.bmax[best] - nd.bmin[best]))
                    best = d;
        } else {
            const double S[3] = {Sdim[3 * (int64_t)i], Sdim[3 * (int64_t)i + 1], Sdim[3 * (int64_t)i + 2]};
            for (int d = 0; d < 3; ++d) {
                if (nd.bmax[d] == nd.bmin[d]) continue;
                if (best < 0) { best = d; continue; }
                const bool better = mode == KD_MIN_ENTROPY ? (S[d] < S[best] - 1e-12) : (S[d] > S[best] + 1e-12);
                if (better) best = d;
            }
        }
    }
    const bool split = valid && best >= 0;
    // every member coincides: the node stays a leaf
    const bool stays = valid && best < 0;
    const int n = split ? nd.end - nd.start : 0, nl = n / 2;
    const int nc = split ? ncell[nd.host] : 0;
    const bool lact = split && nl > nc, ract = split && n - nl > nc;
    const int c0 = wave_reserve(&counters[3], split ? 2 : 0);
    const int na0 = wave_reserve(&counters[1], (int)lact + (int)ract);
    const int nl0 = wave_reserve(&counters[2], (int)stays + (split ? (int)!lact + (int)!ract : 0));
    int grow = (lact ? nl : 0) + (ract ? n - nl : 0);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) grow += __shfl_xor(grow, o, 64);
    if (__lane_id() == 0 && grow) atomicAdd(&counters[5], grow);
    if (stays) {
        nodes[id].slot = -1;
        leaves[nl0] = id;
    }
    if (!split) return;
    const int* lb = best == 0 ? l0 : (best == 1 ? l1 : l2);
    const int* ub = best == 0 ? u0 : (best == 1 ? u1 : u2);
    const int t = ub[lb[nd.start + nl]];
    KdNode L = nd, R = nd;
    L.end = nd.start + nl;
    R.start = nd.start + nl;
    L.hi[best] = t - 1;
    R.lo[best] = t;
    L.slot = R.slot = -1;
    L.dim = R.dim = -1;
    L.left = L.right = R.left = R.right = -1;
    nodes[c0] = L;
    nodes[c0 + 1] = R;
    nodes[id].dim = best;
    nodes[id].t = t;
    nodes[id].left = c0;
    nodes[id].right = c0 + 1;
    int ka = na0, kl = nl0;
    if (lact) next_active[ka++] = c0; else leaves[kl++] = c0;
    if (ract) next_active[ka] = c0 + 1; else leaves[kl] = c0 + 1;
}

// The left flags of the three lists at once (list j at lf[j * M + p]).  A
// node splits at rank nl = n / 2 of its list along the split dimension d,
// which is ordered by (u_d, element): the list along d takes its flag from
// the position, and an element of the other two lists goes left when its
// (u_d, element) is below the median's (t, em), em = that list's entry at
// rank nl.
__global__ void k_lflag3(int64_t M, const int* __restrict__ seg_node, const KdNode* __restrict__ nodes,
                         const int* __restrict__ l0, const int* __restrict__ l1, const int* __restrict__ l2,
                         const int* __restrict__ u0, const int* __restrict__ u1, const int* __restrict__ u2,
                         uint8_t* __restrict__ lf) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    const KdNode& nd = nodes[seg_node[p]];
    const int dim = nd.dim;
    if (dim < 0) {
        lf[p] = 0;
        lf[M + p] = 0;
        lf[2 * M + p] = 0;
        return;
    }
    const int nl = (nd.end - nd.start) / 2;
    const uint8_t own = (p - nd.start) < nl ? 1 : 0;
    const int* ld = dim == 0 ? l0 : (dim == 1 ? l1 : l2);
    const int* ud = dim == 0 ? u0 : (dim == 1 ? u1 : u2);
    const int em = ld[nd.start + nl], t = nd.t;
    auto left = [&](int e) -> uint8_t {
        const int ue = ud[e];
        return (ue < t || (ue == t && e < em)) ? 1 : 0;
    };
    lf[p] = dim == 0 ? own : left(l0[p]);
    lf[M + p] = dim == 1 ? own : left(l1[p]);
    lf[2 * M + p] = dim == 2 ? own : left(l2[p]);
}

// Stable partition of the three lists inside every split node (the scan
// runs over the three flag arrays back to back; differences are taken
// inside one list), then the position's node moves to its child.  The left
// flags are read by list position (lf, list j at lf[j * M + p]), coalesced.
__global__ void k_part3(int64_t M, int* __restrict__ seg_node, const KdNode* __restrict__ nodes,
                        const int* __restrict__ l0, const int* __restrict__ l1, const int* __restrict__ l2,
                        const uint8_t* __restrict__ lf, const uint32_t* __restrict__ scan, int* __restrict__ o0,
                        int* __restrict__ o1, int* __restrict__ o2, CoordsL0 c) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    const KdNode& nd = nodes[seg_node[p]];
    const int e0 = l0[p], e1 = l1[p], e2 = l2[p];
    if (nd.dim < 0) {
        o0[p] = e0;
        o1[p] = e1;
        o2[p] = e2;
        if (c.in[0]) {
            for (int d = 0; d < 3; ++d) c.out[d][p] = c.in[d][p];
        }
        return;
    }
    const int s = nd.start, nl = (nd.end - nd.start) / 2;
    const int e[3] = {e0, e1, e2};
    int* out[3] = {o0, o1, o2};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int rl = (int)(scan[j * M + p] - scan[j * M + s]);  // left members before p in the node
        const int np = lf[j * M + p] ? s + rl : s + nl + ((int)p - s - rl);
        out[j][np] = e[j];
        if (j == 0 && c.in[0]) {
            for (int d = 0; d < 3; ++d) c.out[d][np] = c.in[d][p];
        }
    }
    seg_node[p] = p < s + nl ? nd.left : nd.right;
}

// coordinates in list-0 order, for the histograms
__global__ void k_coords_l0(int64_t M, const int* __restrict__ l0, const int* __restrict__ u0,
                            const int* __restrict__ u1, const int* __restrict__ u2, int* __restrict__ c0,
                            int* __restrict__ c1, int* __restrict__ c2) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    const int e = l0[p];
    c0[p] = u0[e];
    c1[p] = u1[e];
    c2[p] = u2[e];
}

__global__ void k_leaf_bbox(int nl, const int* __restrict__ leaves, KdNode* nodes, const int* __restrict__ l0,
                            const int* __restrict__ l1, const int* __restrict__ l2, const int* __restrict__ u0,
                            const int* __restrict__ u1, const int* __restrict__ u2, int* __restrict__ leaf_min,
                            int n_hosts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl) return;
    const int id = leaves[i];
    KdNode& nd = nodes[id];
    const int s = nd.start, e = nd.end - 1;
    nd.bmin[0] = u0[l0[s]]; nd.bmax[0] = u0[l0[e]];
    nd.bmin[1] = u1[l1[s]]; nd.bmax[1] = u1[l1[e]];
    nd.bmin[2] = u2[l2[s]]; nd.bmax[2] = u2[l2[e]];
    if (id < n_hosts)  // a root that was never split: its region is its bounding box
        for (int d = 0; d < 3; ++d) { nd.lo[d] = nd.bmin[d]; nd.hi[d] = nd.bmax[d]; }
    leaf_min[id] = 0x7FFFFFFF;
}

// Members by position in list-0 order, and the smallest index of each leaf.
// c0..c2: the coordinates already in list-0 order, or null (then gathered).
__global__ void k_final(int64_t M, const int* __restrict__ l0, const int* __restrict__ seg_node,
                        const int* __restrict__ u0, const int* __restrict__ u1, const int* __restrict__ u2,
                        const int* __restrict__ c0, const int* __restrict__ c1, const int* __restrict__ c2,
                        const int* __restrict__ g, const float* __restrict__ m, Elems F, int* __restrict__ leaf_min) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < M;
    const int e = valid ? l0[p] : 0;
    const int gi = valid ? g[e] : 0x7FFFFFFF;
    if (valid) {
        F.u[0][p] = c0 ? c0[p] : u0[e];
        F.u[1][p] = c0 ? c1[p] : u1[e];
        F.u[2][p] = c0 ? c2[p] : u2[e];
        F.gidx[p] = gi;
        F.eid[p] = e;
        if (m) F.mass[p] = m[e];
    }
    // smallest particle index per leaf (wave-reduced when the wave is in one leaf)
    const int key = valid ? seg_node[p] : 0;
    const uint64_t act = __ballot(valid);
    if (act == 0) return;
    const int first = __ffsll((unsigned long long)act) - 1;
    const int k0 = __shfl(key, first, 64);
    if (__ballot(valid && key == k0) == act) {
        int v = gi;
        for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
        if ((int)__lane_id() == first) atomicMin(&leaf_min[k0], v);
    } else if (valid) {
        atomicMin(&leaf_min[key], gi);
    }
}

}  // namespace

int read_host_offsets(vr_ctx* ctx, int32_t n_hosts, const int32_t* host_offsets, int64_t n, int64_t min_size,
                      std::vector<int32_t>& off, hipStream_t st) {
    off.assign(n_hosts + 1, 0);
    if (n_hosts == 0) return VR_OK;
    int rc0 = copy_to_host(ctx, off.data(), host_offsets, (n_hosts + 1) * sizeof(int32_t), st);
    if (rc0) return rc0;
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
    const int counts = use_mass ? 0 : 1;
    int hb = 1;
    while ((1 << hb) <= n_hosts) ++hb;
    // one workspace region holds every array of the build
    Carve cv;
    int *U[3], *G, *H, *L[3], *Lalt[3], *seg, *leaf_min, *act0, *act1, *leaves, *ncell_d, *counters;
    int *C0[3], *C0alt[3];
    const int64_t MC = mode != KD_WIDEST ? M : 1;
    float* Ms;
    uint8_t* lf8;
    uint32_t* lf;
    uint64_t* pkey;
    unsigned long long* hsh;
    KdNode* nodes;
    Elems F;
    auto layout = [&]() {
        for (int d = 0; d < 3; ++d) U[d] = cv.add<int>(M);
        G = cv.add<int>(M);
        H = cv.add<int>(M);
        Ms = cv.add<float>(use_mass ? M : 1);
        for (int d = 0; d < 3; ++d) L[d] = cv.add<int>(M);
        for (int d = 0; d < 3; ++d) Lalt[d] = cv.add<int>(M);
        for (int d = 0; d < 3; ++d) C0[d] = cv.add<int>(MC);
        for (int d = 0; d < 3; ++d) C0alt[d] = cv.add<int>(MC);
        seg = cv.add<int>(M);
        lf8 = cv.add<uint8_t>(3 * M);
        lf = cv.add<uint32_t>(3 * M + 1);
        pkey = cv.add<uint64_t>(M);
        nodes = cv.add<KdNode>(node_cap);
        act0 = cv.add<int>(node_cap);
        act1 = cv.add<int>(node_cap);
        leaves = cv.add<int>(node_cap);
        leaf_min = cv.add<int>(node_cap);
        for (int d = 0; d < 3; ++d) F.u[d] = cv.add<int>(M);
        F.gidx = cv.add<int>(M);
        F.eid = cv.add<int>(M);
        F.mass = cv.add<float>(use_mass ? M : 1);
        ncell_d = cv.add<int>(n_hosts);
        counters = cv.add<int>(8);
        hsh = cv.add<unsigned long long>(HASH_SLOTS);
    };
    layout();
    const size_t total = cv.bytes;
    cv.bytes = 0;
    cv.base = static_cast<char*>(ws(ctx, WS_KD, total));
    if (!cv.base) return VR_ERR_OUT_OF_MEMORY;
    layout();
    if (!use_mass) F.mass = nullptr;
    // counters: 0 active nodes, 1 active next level, 2 leaves, 3 nodes, 4 members now, 5 members next
    VR_HIP(ctx, hipMemcpyAsync(ncell_d, ncell.data(), n_hosts * sizeof(int), hipMemcpyHostToDevice, st));
    int* init = reinterpret_cast<int*>(ctx->pinned);
    for (int k = 0; k < 8; ++k) init[k] = 0;
    init[3] = n_hosts;
    VR_HIP(ctx, hipMemcpyAsync(counters, init, 8 * sizeof(int), hipMemcpyHostToDevice, st));
    {
        int rc = fill_u32(ctx, reinterpret_cast<uint32_t*>(hsh), 0u, 2 * HASH_SLOTS, st);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_elems, dim3(grid_for(M, 256)), dim3(256), 0, st, M, n_hosts, host_offsets, host_members,
                       p->qx, p->qy, p->qz, p->mass, p->grid_bits, U[0], U[1], U[2], G, Ms, H, hsh);
    VR_LAUNCH_CHECK(ctx);
    // The three lists sorted by (host, u_d, element) depend only on the
    // elements' members, unwrapped coordinates and hosts.  The context keeps
    // the last build's lists and reuses them when this build's content hash,
    // size and key width match (the entropy cells and the neighbour tree of
    // one search are built over the same members); without room for them
    // under the workspace cap it simply sorts.
    {
        unsigned long long parts[HASH_SLOTS];
        int rc = read_back(ctx, hsh, parts, sizeof parts, st);
        if (rc) return rc;
        unsigned long long h64 = 0;
        for (int k = 0; k < HASH_SLOTS; ++k) h64 += parts[k];
        const int bits = 22 + hb;
        const std::string err_before = ctx->err;
        int* pre = static_cast<int*>(ws(ctx, WS_KD_PRE, 3 * (size_t)M * sizeof(int)));
        if (!pre) ctx->err = err_before;  // no room for the kept lists: not an error
        const bool hit = pre && ctx->kd_pre_ptr == pre && ctx->kd_pre_m == M && ctx->kd_pre_bits == bits &&
                         ctx->kd_pre_hash == h64;
        if (hit) {
            for (int d = 0; d < 3; ++d)
                VR_HIP(ctx, hipMemcpyAsync(L[d], pre + d * M, (size_t)M * sizeof(int), hipMemcpyDeviceToDevice, st));
        } else {
            for (int d = 0; d < 3; ++d) {
                uint32_t* ld = reinterpret_cast<uint32_t*>(L[d]);
                uint64_t* kin;
                uint32_t* vin;
                if ((rc = sort_input_u64(ctx, pkey, ld, M, bits, &kin, &vin))) return rc;
                hipLaunchKernelGGL(k_presort_keys, dim3(grid_for(M, 256)), dim3(256), 0, st, M, U[d], H, kin, vin);
                VR_LAUNCH_CHECK(ctx);
                if ((rc = sort_pairs_u64_from(ctx, kin, vin, pkey, ld, M, bits, st))) return rc;
            }
            ctx->kd_pre_m = -1;
            if (pre) {
                for (int d = 0; d < 3; ++d)
                    VR_HIP(ctx, hipMemcpyAsync(pre + d * M, L[d], (size_t)M * sizeof(int), hipMemcpyDeviceToDevice,
                                               st));
                ctx->kd_pre_ptr = pre;
                ctx->kd_pre_m = M;
                ctx->kd_pre_bits = bits;
                ctx->kd_pre_hash = h64;
            }
        }
    }
    if (mode != KD_WIDEST) {
        hipLaunchKernelGGL(k_coords_l0, dim3(grid_for(M, 256)), dim3(256), 0, st, M, L[0], U[0], U[1], U[2], C0[0],
                           C0[1], C0[2]);
        VR_LAUNCH_CHECK(ctx);
    }
    hipLaunchKernelGGL(k_roots, dim3(grid_for(n_hosts, 256)), dim3(256), 0, st, n_hosts, host_offsets, ncell_d, nodes,
                       act0, counters, leaves, seg);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_seg_init, dim3(grid_for(M, 256)), dim3(256), 0, st, M, H, seg);
    VR_LAUNCH_CHECK(ctx);
    int* cur = act0;
    int* nxt = act1;
    const unsigned gM = grid_for(M, 256);
    // Active nodes and their members per level as the sizes alone give them
    // (a node splits at rank floor(n/2) while it holds more than ncell; the
    // sizes of one host's nodes on a level are two consecutive integers).
    // A node of coincident members that stays a leaf only lowers the true
    // counts, which the kernels read from the device; these bound the grids
    // and the number of levels, so no level waits for the host.
    std::vector<int64_t> plan_na, plan_members;
    {
        struct Sz { int64_t s0, c0, c1; };  // c0 nodes of size s0, c1 of size s0 + 1
        std::vector<Sz> sz(n_hosts);
        for (int h = 0; h < n_hosts; ++h) sz[h] = Sz{(int64_t)off[h + 1] - off[h], 1, 0};
        for (;;) {
            int64_t na = 0, mem = 0;
            for (int h = 0; h < n_hosts; ++h) {
                Sz& z = sz[h];
                const int64_t nc = ncell[h];
                int64_t a0 = z.s0 > nc ? z.c0 : 0, a1 = z.s0 + 1 > nc ? z.c1 : 0;
                na += a0 + a1;
                mem += a0 * z.s0 + a1 * (z.s0 + 1);
                // children of the active ones: floor and ceil halves
                int64_t lo = INT64_MAX, cnt[3] = {0, 0, 0};
                const int64_t sizes[2] = {z.s0, z.s0 + 1}, counts[2] = {a0, a1};
                for (int k = 0; k < 2; ++k)
                    if (counts[k] > 0) lo = std::min(lo, sizes[k] / 2);
                if (lo == INT64_MAX) {
                    z = Sz{0, 0, 0};
                    continue;
                }
                for (int k = 0; k < 2; ++k) {
                    if (counts[k] == 0) continue;
                    const int64_t f = sizes[k] / 2, c = sizes[k] - f;
                    cnt[f - lo] += counts[k];
                    cnt[c - lo] += counts[k];
                }
                // the halves of two consecutive sizes span at most lo .. lo + 1
                z = Sz{lo, cnt[0], cnt[1] + cnt[2]};
            }
            if (na == 0) break;
            plan_na.push_back(na);
            plan_members.push_back(mem);
            if (plan_na.size() > 64) return set_err(ctx, VR_ERR_NOT_CONVERGED, "KD build exceeded 64 levels");
        }
    }
    for (int level = 0; level < (int)plan_na.size(); ++level) {
        int rc = VR_OK;
        const int na = (int)plan_na[level];
        hipEvent_t e0 = nullptr;
        if (ctx->timing) {
            e0 = timer_event(ctx);
            (void)hipEventRecord(e0, st);
        }
        hipLaunchKernelGGL(k_level_counters, dim3(1), dim3(64), 0, st, counters, level > 0 ? 1 : 0, 1);
        VR_LAUNCH_CHECK(ctx);
        hipLaunchKernelGGL(k_bbox, dim3(grid_for(na, 256)), dim3(256), 0, st, counters, cur, nodes, L[0], L[1], L[2],
                           U[0], U[1], U[2], n_hosts);
        VR_LAUNCH_CHECK(ctx);
        uint32_t* hc = nullptr;
        double* hm = nullptr;
        if (mode != KD_WIDEST) {
            const int64_t hn = (int64_t)na * 3 * nbins;
            if (counts) {
                hc = static_cast<uint32_t*>(ws(ctx, WS_KD_HIST, hn * sizeof(uint32_t)));
                if (!hc) return VR_ERR_OUT_OF_MEMORY;
                if ((rc = fill_u32(ctx, hc, 0u, hn, st))) return rc;
                hipLaunchKernelGGL(k_hist<true>, dim3(grid_for(M, HCH)), dim3(KB), 0, st, M, seg, nodes, L[0], C0[0],
                                   C0[1], C0[2], Ms, nbins, hc, hm);
            } else {
                hm = static_cast<double*>(ws(ctx, WS_KD_HIST, hn * sizeof(double)));
                if (!hm) return VR_ERR_OUT_OF_MEMORY;
                if ((rc = fill_u32(ctx, reinterpret_cast<uint32_t*>(hm), 0u, 2 * hn, st))) return rc;
                hipLaunchKernelGGL(k_hist<false>, dim3(grid_for(M, HCH)), dim3(KB), 0, st, M, seg, nodes, L[0], C0[0],
                                   C0[1], C0[2], Ms, nbins, hc, hm);
            }
            VR_LAUNCH_CHECK(ctx);
        }
        double* Sdim = nullptr;
        if (mode != KD_WIDEST) {
            Sdim = static_cast<double*>(ws(ctx, WS_KD_S, (size_t)na * 3 * sizeof(double)));
            if (!Sdim) return VR_ERR_OUT_OF_MEMORY;
            hipLaunchKernelGGL(k_entropy, dim3(grid_for((int64_t)na * 64, 256)), dim3(256), 0, st, counters, cur,
                               nodes, nbins, counts, hc, hm, Sdim);
            VR_LAUNCH_CHECK(ctx);
        }
        hipLaunchKernelGGL(k_split, dim3(grid_for(na, 256)), dim3(256), 0, st, counters, cur, nodes, L[0], L[1], L[2],
                           U[0], U[1], U[2], mode, Sdim, ncell_d, nxt, leaves, counters);
        VR_LAUNCH_CHECK(ctx);
        hipLaunchKernelGGL(k_lflag3, dim3(gM), dim3(256), 0, st, M, seg, nodes, L[0], L[1], L[2], U[0], U[1], U[2],
                           lf8);
        VR_LAUNCH_CHECK(ctx);
        if ((rc = scan_u8(ctx, lf8, lf, 3 * M, st))) return rc;
        CoordsL0 cl0{};
        if (mode != KD_WIDEST) cl0 = CoordsL0{{C0[0], C0[1], C0[2]}, {C0alt[0], C0alt[1], C0alt[2]}};
        hipLaunchKernelGGL(k_part3, dim3(gM), dim3(256), 0, st, M, seg, nodes, L[0], L[1], L[2], lf8, lf, Lalt[0],
                           Lalt[1], Lalt[2], cl0);
        VR_LAUNCH_CHECK(ctx);
        for (int j = 0; j < 3; ++j) {
            std::swap(L[j], Lalt[j]);
            std::swap(C0[j], C0alt[j]);
        }
        if (ctx->timing) {
            hipEvent_t e1 = timer_event(ctx);
            (void)hipEventRecord(e1, st);
            timer_push(ctx, "kd_level", e0, e1, (double)plan_members[level]);
        }
        std::swap(cur, nxt);
    }
    if (!plan_na.empty()) {
        hipLaunchKernelGGL(k_level_counters, dim3(1), dim3(64), 0, st, counters, 1, 0);
        VR_LAUNCH_CHECK(ctx);
    }
    int c[8];
    int rc = read_back(ctx, counters, c, sizeof c, st);
    if (rc) return rc;
    const int nleaf = c[2];
    hipLaunchKernelGGL(k_leaf_bbox, dim3(grid_for(nleaf, 256)), dim3(256), 0, st, nleaf, leaves, nodes, L[0], L[1],
                       L[2], U[0], U[1], U[2], leaf_min, n_hosts);
    VR_LAUNCH_CHECK(ctx);
    const bool have_c0 = mode != KD_WIDEST;
    hipLaunchKernelGGL(k_final, dim3(gM), dim3(256), 0, st, M, L[0], seg, U[0], U[1], U[2], have_c0 ? C0[0] : nullptr,
                       have_c0 ? C0[1] : nullptr, have_c0 ? C0[2] : nullptr, G, use_mass ? Ms : nullptr, F, leaf_min);
    VR_LAUNCH_CHECK(ctx);
    tree.nodes = nodes;
    tree.leaves = leaves;
    tree.n_leaves = nleaf;
    tree.seg_node = seg;
    tree.leaf_min = leaf_min;
    tree.F = F;
    for (int d = 0; d < 3; ++d) tree.elem_u[d] = U[d];
    tree.elem_host = H;
    tree.use_mass = use_mass;
    return VR_OK;
}

}  // namespace vr
