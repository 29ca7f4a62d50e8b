// vr_knn.hip -- local velocity density ratio R = ln(f_l / f_bg) (Sec. 2.2).
//
// Each host gets a median-split KD tree (widest dimension, leaves of at most
// 64 members, built by the presorted level-synchronous builder); members sit
// in leaf order, so 64 consecutive queries share leaves.  One wavefront
// serves 64 queries, one per lane: the wave first scans the leaves that hold
// its own queries (which fills every heap with near neighbours), then walks
// the tree of the host with a shared depth-first stack (near child first,
// for the centre of the wave's queries), visiting a node when any lane's
// ball -- radius = its current n_se-th neighbour -- reaches the node's
// bounding box.  A visited leaf is
// staged in LDS 64 members at a time.  A first pass over the chunk (the same
// LDS address for every lane, no divergence) marks in a per-lane bit mask
// the members whose FP32 squared distance may beat the lane's current worst;
// a second pass inserts the marked ones with their exact keys, each lane
// walking its own mask.  Every lane keeps its n_se best keys, unordered, in
// LDS slots grouped by eight; the largest key of each group and its slot
// sit in registers, so replacing the lane's worst key rewrites one slot and
// rereads that group's eight keys at once, with no chain of dependent LDS
// reads.  A key packs the exact integer squared distance above the member's
// rank in its host's ascending index order, so ties break by particle index
// exactly as the definition says.  The n_v velocity neighbours are then
// chosen among the n_se by (FP64 dv2, index) and the Epanechnikov estimate
// and the Gaussian background follow in FP64.
#include "vr_kd.h"

#include <cmath>

namespace vr {
namespace {

constexpr int POS_BITS = 22;
constexpr uint64_t POS_MASK = (uint64_t(1) << POS_BITS) - 1;
constexpr int STACK = 128;

__global__ void k_pos_of(int64_t M, const int* __restrict__ gidx, int* __restrict__ pos_of) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < M) pos_of[gidx[k]] = (int)k;
}

__global__ void k_subset_pos(int64_t ns, int64_t n, const int32_t* __restrict__ subset, const int* __restrict__ pos_of,
                             uint32_t* __restrict__ qpos, uint32_t* __restrict__ qval, int* __restrict__ bad) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    const int i = subset[s];
    int p = (i >= 0 && i < n) ? pos_of[i] : -1;
    if (p < 0) { atomicOr(bad, 1); p = 0; }
    qpos[s] = (uint32_t)p;
    qval[s] = (uint32_t)s;
}

// ln f_bg (Eq. fvbg): the log density of the trivariate Gaussian of mean
// vbar(x) and covariance sigma(x), particle g, at velocity vq.  The
// quadratic form is u^T adj(S) u / det S with u = vq - vbar; S is positive
// definite iff its leading principal minors S_xx, S_xx S_yy - S_xy^2 and
// det S are positive (Sylvester's criterion), else NaN.
__device__ __forceinline__ double log_fbg(const float* __restrict__ sigma, const float* __restrict__ vbar,
                                          int g, double vqx, double vqy, double vqz) {
    const float* s = sigma + (int64_t)g * 6;  // particle-major
    const double sxx = s[0], syy = s[1], szz = s[2];
    const Sym3Adj A = sym3_adjugate(sxx, syy, szz, s[3], s[4], s[5]);
    if (!(sxx > 0) || !(A.zz > 0) || !(A.det > 0)) return NAN;
    const float* vb = vbar + (int64_t)g * 3;
    const double ux = vqx - (double)vb[0];
    const double uy = vqy - (double)vb[1];
    const double uz = vqz - (double)vb[2];
    const double diag = A.xx * ux * ux + A.yy * uy * uy + A.zz * uz * uz;
    const double offd = A.xy * ux * uy + A.xz * ux * uz + A.yz * uy * uz;
    // 3 ln(2 pi) / 2
    constexpr double HALF3_LN_2PI = 2.7568155996140178;
    return -0.5 * ((diag + 2.0 * offd) / A.det + log(A.det)) - HALF3_LN_2PI;
}

// rank_of[g] = the position of particle g in host_members (-1 beforehand);
// a member outside [0, n) or listed twice raises *bad
__global__ void k_rank_of(int64_t M, int64_t n, const int* __restrict__ mem, int* __restrict__ rank_of,
                          int* __restrict__ bad) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const int g = mem[k];
    if (g < 0 || g >= n || atomicExch(&rank_of[g], (int)k) != -1) atomicOr(bad, 1);
}

// Per host member, at its host rank: (vx, vy, vz, mass) as one 16-byte
// record, so a neighbour's velocity and mass are one cache line, and the
// member's ln f_bg, so a query reads 8 bytes instead of nine floats spread
// over nine arrays.  The pass runs in particle order, where its 12 input
// arrays are read in full lines; a host's members are scattered over the
// whole particle range, so a pass in rank order would fetch a line per value.
__global__ void k_member_records(int64_t n, const int* __restrict__ rank_of, const float* __restrict__ vx,
                                 const float* __restrict__ vy, const float* __restrict__ vz,
                                 const float* __restrict__ mass, const float* __restrict__ vbar,
                                 const float* __restrict__ sigma, float4* __restrict__ V, double* __restrict__ FB) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int k = rank_of[g];
    if (k < 0) return;
    const float ux = vx[g], uy = vy[g], uz = vz[g];
    V[k] = make_float4(ux, uy, uz, mass ? mass[g] : 0.f);
    FB[k] = log_fbg(sigma, vbar, (int)g, (double)ux, (double)uy, (double)uz);
}

__device__ __forceinline__ bool vless(double a, int pa, double b, int pb) { return a < b || (a == b && pa < pb); }

// NSE: heap capacity (n_se <= NSE).  NVR > 0: exactly NVR velocity
// neighbours kept in registers (sorted by an unrolled insertion network);
// NVR == 0: any n_v <= NVLMAX, kept in LDS.
template <int NSE, int NVR, int NVLMAX>
__global__ __launch_bounds__(64) void k_knn(const uint32_t* __restrict__ qpos, int64_t nq,
                                            const KdNode* __restrict__ nodes, Elems F, const int* __restrict__ leaf_of,
                                            const float4* __restrict__ V, const double* __restrict__ FB,
                                            const int* __restrict__ elem_host, const int32_t* __restrict__ host_off,
                                            int n_se, int n_v, int use_mass, double mass_value, int gb,
                                            float* __restrict__ R, unsigned xchunk,
                                            unsigned long long* __restrict__ ncand) {
    constexpr int NVL = NVR > 0 ? 1 : NVLMAX;
    __shared__ uint64_t heap[NSE][64];
    __shared__ double vd[NVL][64];
    __shared__ int vp[NVL][64];
    __shared__ int stack[STACK];
    // the leaf chunk being scanned, SoA: x, y, z (exact integers as float)
    // and rank; four consecutive candidates are one 16-byte broadcast read
    __shared__ __align__(16) float cxs[64];
    __shared__ __align__(16) float cys[64];
    __shared__ __align__(16) float czs[64];
    __shared__ int crk[64];
    const int lane = threadIdx.x;
    const int64_t qi = (int64_t)xcd_swizzle(blockIdx.x, gridDim.x, xchunk) * 64 + lane;
    const bool active = qi < nq;
    const int e = active ? (qpos ? (int)qpos[qi] : (int)qi) : 0;
    const int h = active ? elem_host[e] : -1;
    const int base = active ? host_off[h] : 0;
    const int own = active ? leaf_of[e] : -1;
    const int px = F.u[0][e], py = F.u[1][e], pz = F.u[2][e];
    const float pxf = (float)px, pyf = (float)py, pzf = (float)pz;
    int count = 0;
    uint64_t worst = ~0ull;
    unsigned long long wcand = 0;  // wave-uniform
    // the kept keys: slot s of group s / 8; per group its largest key and
    // that key's slot; wg = the group holding the lane's largest key
    constexpr int LGS = 3;  // groups of 2^LGS slots
    constexpr int GS = 1 << LGS;
    constexpr int NG = NSE >> LGS;
    static_assert(NG * 6 <= 64, "slot indices of the group maxima are packed 6 bits each");
    uint64_t gmx[NG];
    uint64_t gix = 0;  // slot of group g's largest key in bits [6g, 6g + 6)
#pragma unroll
    for (int g = 0; g < NG; ++g) gmx[g] = 0;
    int wg = 0;
    // Slots from n_se up hold key 0, which never exceeds a kept key, so the
    // group maxima need no bound checks (a group whose largest key is 0
    // takes no replacement: no key is below 0).
    for (int sl = n_se; sl < NG * GS; ++sl) heap[sl][lane] = 0;
    // every selection below is a value select, not a branch on the lane's
    // group index
    auto top_update = [&]() __attribute__((always_inline)) {
        uint64_t m = gmx[0];
        int mg = 0;
#pragma unroll
        for (int g = 1; g < NG; ++g) {
            const bool gt = gmx[g] > m;
            m = gt ? gmx[g] : m;
            mg = gt ? g : mg;
        }
        worst = m;
        wg = mg;
    };
    // keeps key: appended while fewer than n_se are kept, else it takes the
    // slot of the largest (the caller has checked key < worst)
    auto insert = [&](uint64_t key) __attribute__((always_inline)) {
        if (count < n_se) {
            const int sl = count++;
            heap[sl][lane] = key;
            const int g = sl >> LGS;
            const bool first = (sl & (GS - 1)) == 0;
            bool up = false;
#pragma unroll
            for (int k = 0; k < NG; ++k) {
                const bool u = k == g && (first || key > gmx[k]);
                gmx[k] = u ? key : gmx[k];
                up = up || u;
            }
            const uint64_t fld = uint64_t(63) << (6 * g);
            gix = up ? ((gix & ~fld) | ((uint64_t)sl << (6 * g))) : gix;
            if (count == n_se) top_update();
            return;
        }
        const int sl = (int)((gix >> (6 * wg)) & 63);
        heap[sl][lane] = key;
        const int s0 = wg << LGS;
        uint64_t v[GS];
#pragma unroll
        for (int u = 0; u < GS; ++u) v[u] = heap[s0 + u][lane];
        uint64_t m = v[0];
        int ms = s0;
#pragma unroll
        for (int u = 1; u < GS; ++u) {
            const bool gt = v[u] > m;
            m = gt ? v[u] : m;
            ms = gt ? s0 + u : ms;
        }
#pragma unroll
        for (int k = 0; k < NG; ++k) gmx[k] = k == wg ? m : gmx[k];
        const uint64_t fld = uint64_t(63) << (6 * wg);
        gix = (gix & ~fld) | ((uint64_t)ms << (6 * wg));
        top_update();
    };
    // While a heap is not full it accepts only squared distances <= tau, a
    // bound that at least n_se members of the host are known to meet (so the
    // n_se nearest all meet it); NO_BOUND until such a bound is found.
    constexpr uint64_t NO_BOUND = ~0ull >> POS_BITS;
    uint64_t tau = NO_BOUND;
    // the same bound on keys: d2 <= tau exactly when key < (tau + 1) << POS_BITS
    uint64_t tau_key = ~0ull;

    // Stages the members [c0, min(c0 + 64, t_end)) of a leaf in LDS for the
    // unwrapped (no minimum image) scan; padding slots sit far away.
    auto stage_chunk = [&](int c0, int t_end, int hbase) __attribute__((always_inline)) {
        const int j = c0 + lane;
        const bool vj = j < t_end;
        cxs[lane] = vj ? (float)F.u[0][j] : 1e30f;
        cys[lane] = vj ? (float)F.u[1][j] : 1e30f;
        czs[lane] = vj ? (float)F.u[2][j] : 1e30f;
        crk[lane] = vj ? F.eid[j] - hbase : 0;
        __builtin_amdgcn_wave_barrier();
    };

    // Inserts the members of leaf `node` for the lanes in `mine`.
    auto scan_leaf = [&](int node, bool mine, bool nowrap, int hbase) __attribute__((always_inline)) {
        const KdNode& nd = nodes[node];
        const int s = nd.start, t_end = nd.end;
        for (int c0 = s; c0 < t_end; c0 += 64) {
            const int m = min(64, t_end - c0);
            // candidate distances this chunk gives the wave's queries
            wcand += (unsigned long long)m * (unsigned long long)__popcll(__ballot(mine));
            if (nowrap) {
                // FP32 prefilter: coordinates are integers below 2^24, so the
                // differences are exact and the rounded sum of squares is within
                // 2e-7 of the exact one; only candidates that may beat the
                // current worst key (or meet tau) get the exact integer key.
                stage_chunk(c0, t_end, hbase);
                // pass 1 (no divergence): which candidates may beat this lane's
                // current worst key; pass 2: insert them, each lane walking its
                // own mask, so the wave spends max-over-lanes insertions per
                // chunk instead of one per candidate that any lane takes.
                // Pass 1 is unrolled in blocks of 16 candidates.  The bound
                // wf enters the FMA chain, dx^2 + dy^2 + (dz^2 - wf), whose
                // rounding (three roundings of values below max(d2, wf)) stays
                // inside wf's relative slack, so a negative result marks every
                // candidate that may be taken; its sign bit is shifted into the
                // mask from the bottom, candidates from the highest index down,
                // so candidate t ends at bit t % 32 of word t / 32.  Bits past
                // the chunk's end are cleared.
                const float wf = count < n_se ? (tau == NO_BOUND ? INFINITY : (float)tau * 1.000001f + 1.0f)
                                              : (float)(worst >> POS_BITS) * 1.000001f + 1.0f;
                const float nwf = -wf;
                uint32_t tk[2] = {0u, 0u};
#pragma unroll
                for (int b = 3; b >= 0; --b) {
                    if (16 * b < m) {
#pragma unroll
                        for (int t4 = 12; t4 >= 0; t4 -= 4) {
                            const int t = 16 * b + t4;
                            const float4 X = *reinterpret_cast<const float4*>(&cxs[t]);
                            const float4 Y = *reinterpret_cast<const float4*>(&cys[t]);
                            const float4 Z = *reinterpret_cast<const float4*>(&czs[t]);
                            const float xs[4] = {X.x, X.y, X.z, X.w}, ys[4] = {Y.x, Y.y, Y.z, Y.w},
                                        zs[4] = {Z.x, Z.y, Z.z, Z.w};
#pragma unroll
                            for (int u = 3; u >= 0; --u) {
                                const float dxf = xs[u] - pxf, dyf = ys[u] - pyf, dzf = zs[u] - pzf;
                                const float sd = fmaf(dxf, dxf, fmaf(dyf, dyf, fmaf(dzf, dzf, nwf)));
                                tk[b >> 1] = __builtin_amdgcn_alignbit(tk[b >> 1], __float_as_uint(sd), 31);
                            }
                        }
                    }
                }
                uint64_t take = ((uint64_t)tk[1] << 32) | tk[0];
                if (m < 64) take &= (uint64_t(1) << m) - 1;
                if (!mine) take = 0;
                while (take) {
                    const int t = __builtin_ctzll(take);
                    take &= take - 1;
                    // |d| < 2^21: signed 64-bit squares, exact sum
                    const int dx = (int)(cxs[t] - pxf), dy = (int)(cys[t] - pyf), dz = (int)(czs[t] - pzf);
                    const uint64_t d2 = (uint64_t)((int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz);
                    const uint64_t key = (d2 << POS_BITS) | (uint64_t)(uint32_t)crk[t];
                    if (key < (count < n_se ? tau_key : worst)) insert(key);
                }
                __builtin_amdgcn_wave_barrier();
                continue;
            }
            // one member per lane, shared by lane reads
            const int j = c0 + lane;
            const bool vj = j < t_end;
            const int lx = vj ? F.u[0][j] : 0, ly = vj ? F.u[1][j] : 0, lz = vj ? F.u[2][j] : 0;
            const int le = vj ? F.eid[j] - hbase : 0;
            for (int t = 0; t < m; ++t) {
                const int cx = __builtin_amdgcn_readlane(lx, t);
                const int cy = __builtin_amdgcn_readlane(ly, t);
                const int cz = __builtin_amdgcn_readlane(lz, t);
                const int ce = __builtin_amdgcn_readlane(le, t);
                const int ddx = min_image(cx - px, gb);
                const int ddy = min_image(cy - py, gb);
                const int ddz = min_image(cz - pz, gb);
                uint64_t d2;
                if (max(max(abs(ddx), abs(ddy)), abs(ddz)) < 32768)
                    d2 = (uint64_t)((uint32_t)(ddx * ddx) + (uint32_t)(ddy * ddy) + (uint32_t)(ddz * ddz));
                else
                    d2 = (uint64_t)((int64_t)ddx * ddx + (int64_t)ddy * ddy + (int64_t)ddz * ddz);
                const uint64_t key = (d2 << POS_BITS) | (uint64_t)(uint32_t)ce;
                if (mine && (count < n_se || key < worst)) insert(key);
            }
        }
    };
    // Box distances in FP32: the per-axis gaps are exact integers below
    // 2^23 and the rounded sum is within 2^-22 of the exact one, so a bound
    // raised by 2^-20 visits every node the exact test would.
    auto needed = [&](const KdNode& nd, bool mine) __attribute__((always_inline)) {
        const float dx = (float)max(max(nd.bmin[0] - px, px - nd.bmax[0]), 0);
        const float dy = (float)max(max(nd.bmin[1] - py, py - nd.bmax[1]), 0);
        const float dz = (float)max(max(nd.bmin[2] - pz, pz - nd.bmax[2]), 0);
        const float md2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const float bnd = count < n_se ? (tau == NO_BOUND ? INFINITY : (float)tau * (1.0f + 0x1p-20f) + 1.0f)
                                       : (float)(worst >> POS_BITS) * (1.0f + 0x1p-20f) + 1.0f;
        return __ballot(mine && md2 <= bnd) != 0;
    };

    bool pending = active;
    while (__ballot(pending)) {
        const uint64_t pm = __ballot(pending);
        const int fl = __ffsll((unsigned long long)pm) - 1;
        const int hh = __shfl(h, fl, 64);
        const int hbase = host_off[hh];
        const bool mine = pending && h == hh;
        // a host narrower than half the box needs no minimum image: its
        // unwrapped coordinate differences are the periodic ones
        const KdNode& root = nodes[hh];
        const int half = 1 << (gb - 1);
        const bool nowrap = root.bmax[0] - root.bmin[0] < half && root.bmax[1] - root.bmin[1] < half &&
                            root.bmax[2] - root.bmin[2] < half;
        // the centre of this host's queries: near children and visiting order follow it
        int64_t sx = mine ? px : 0, sy = mine ? py : 0, sz = mine ? pz : 0;
        int cnt = mine ? 1 : 0;
        for (int o = 32; o > 0; o >>= 1) {
            sx += __shfl_xor(sx, o, 64);
            sy += __shfl_xor(sy, o, 64);
            sz += __shfl_xor(sz, o, 64);
            cnt += __shfl_xor(cnt, o, 64);
        }
        // wave-uniform; the near child is picked arithmetically on the split
        // dimension (a select over the three would go through memory)
        const int ccx = __builtin_amdgcn_readfirstlane((int)(sx / cnt));
        const int ccy = __builtin_amdgcn_readfirstlane((int)(sy / cnt));
        const int ccz = __builtin_amdgcn_readfirstlane((int)(sz / cnt));
        // Depth-first walk of the host's tree, near child first; skip_own:
        // the leaves holding a query of this pass were scanned already.
        auto walk = [&](bool skip_own) __attribute__((always_inline)) {
            if (lane == 0) stack[0] = hh;
            int sp = 1;
            __builtin_amdgcn_wave_barrier();
            while (sp > 0) {
                const int node = stack[--sp];
                __builtin_amdgcn_wave_barrier();
                const KdNode& nd = nodes[node];
                if (!needed(nd, mine)) continue;
                if (nd.dim < 0) {
                    if (!(skip_own && __ballot(mine && own == node))) scan_leaf(node, mine, nowrap, hbase);
                    continue;
                }
                if (sp + 2 > STACK) break;  // cannot happen for trees of depth < 64
                const int dm = nd.dim;
                const int cf = ccx + (dm >= 1) * (ccy - ccx) + (dm == 2) * (ccz - ccy);
                const int nearc = cf < nd.t ? nd.left : nd.right;
                const int farc = cf < nd.t ? nd.right : nd.left;
                if (lane == 0) {
                    stack[sp] = farc;
                    stack[sp + 1] = nearc;
                }
                sp += 2;
                __builtin_amdgcn_wave_barrier();
            }
        };
        if (!nowrap) {
            walk(false);
        } else {
            // The bound tau: a lane's own leaf suggests a squared radius T0
            // holding about n_se members (its density, n_se / (4/3 pi r^3)).
            // Members of the wave's own leaves (all in this host) are counted
            // under eight thresholds T0 * 2^((k-2)/2); the smallest threshold
            // met by n_se of them, rounded up past the FP32 error of the
            // counted distances, is a bound that n_se members meet.
            float thr[8];
            uint32_t cnt[8];
            {
                float T0 = 0.f;
                if (mine) {
                    const KdNode& on = nodes[own];
                    const float vol = (float)(on.bmax[0] - on.bmin[0] + 1) * (float)(on.bmax[1] - on.bmin[1] + 1) *
                                      (float)(on.bmax[2] - on.bmin[2] + 1);
                    const float r = cbrtf(3.0f * (float)n_se * vol / (4.0f * (float)M_PI * (float)(on.end - on.start)));
                    T0 = r * r;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    thr[k] = T0 * exp2f(0.5f * (float)(k - 2));
                    cnt[k] = 0;
                }
            }
            for (uint64_t todo = __ballot(mine); todo;) {
                const int L = __builtin_amdgcn_readlane(own, __ffsll((unsigned long long)todo) - 1);
                const KdNode& nl = nodes[L];
                for (int c0 = nl.start; c0 < nl.end; c0 += 64) {
                    stage_chunk(c0, nl.end, hbase);
                    const int m = min(64, nl.end - c0);
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        if (16 * b < m) {
#pragma unroll
                            for (int t4 = 0; t4 < 16; t4 += 4) {
                                const int t = 16 * b + t4;
                                const float4 X = *reinterpret_cast<const float4*>(&cxs[t]);
                                const float4 Y = *reinterpret_cast<const float4*>(&cys[t]);
                                const float4 Z = *reinterpret_cast<const float4*>(&czs[t]);
                                const float xs[4] = {X.x, X.y, X.z, X.w}, ys[4] = {Y.x, Y.y, Y.z, Y.w},
                                            zs[4] = {Z.x, Z.y, Z.z, Z.w};
#pragma unroll
                                for (int u = 0; u < 4; ++u) {
                                    const float dxf = xs[u] - pxf, dyf = ys[u] - pyf, dzf = zs[u] - pzf;
                                    const float d2f = fmaf(dxf, dxf, fmaf(dyf, dyf, dzf * dzf));
#pragma unroll
                                    for (int k = 0; k < 8; ++k) cnt[k] += d2f <= thr[k] ? 1u : 0u;
                                }
                            }
                        }
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                todo &= ~__ballot(mine && own == L);
            }
            if (mine) {
#pragma unroll
                for (int k = 7; k >= 0; --k)
                    if (cnt[k] >= (uint32_t)n_se) tau = (uint64_t)((double)thr[k] * (1.0 + 1e-6)) + 1;
                tau_key = tau >= NO_BOUND ? ~0ull : (tau + 1) << POS_BITS;
            }
            // the leaves of the queries themselves first: they fill every
            // heap with near neighbours, so the walk prunes from its start
            uint64_t todo = __ballot(mine);
            while (todo) {
                const int L = __builtin_amdgcn_readlane(own, __ffsll((unsigned long long)todo) - 1);
                scan_leaf(L, mine, true, hbase);
                todo &= ~__ballot(mine && own == L);
            }
            walk(true);
        }
        pending = pending && !mine;
    }
    if (ncand && lane == 0) atomicAdd(ncand, wcand);
    if (!active) return;
    // velocity neighbours among the spatial ones, by (dv2, index); velocities
    // and masses are indexed by element id = host base + rank
    const int qe = F.eid[e];
    const float4 vq = V[qe];
    const double vqx = (double)vq.x, vqy = (double)vq.y, vqz = (double)vq.z;
    double msum = 0.0;
    double h2, sw = 0.0;
    const double kW = 15.0 / (8.0 * M_PI);
    // the neighbours' velocities and masses, eight at a time: the loads of a
    // batch are issued together and waited for once
    constexpr int VB = 8;
    int bpos[VB];
    float bvx[VB], bvy[VB], bvz[VB], bms[VB];
    auto fetch = [&](int a0) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < VB; ++u) {
            const int a = a0 + u;
            bpos[u] = a < n_se ? (int)(heap[a][lane] & POS_MASK) : 0;
        }
#pragma unroll
        for (int u = 0; u < VB; ++u) {
            const float4 w = V[base + bpos[u]];
            bvx[u] = w.x;
            bvy[u] = w.y;
            bvz[u] = w.z;
            bms[u] = w.w;
        }
    };
    if constexpr (NVR > 0) {
        double vdr[NVR];
        int vpr[NVR];
#pragma unroll
        for (int i = 0; i < NVR; ++i) { vdr[i] = INFINITY; vpr[i] = 0x7FFFFFFF; }
        for (int a0 = 0; a0 < n_se; a0 += VB) {
            fetch(a0);
#pragma unroll
            for (int u = 0; u < VB; ++u) {
                if (a0 + u >= n_se) break;
                const int pos = bpos[u];
                msum += use_mass ? (double)bms[u] : mass_value;
                const double ax = vqx - (double)bvx[u], ay = vqy - (double)bvy[u], az = vqz - (double)bvz[u];
                const double dv2 = ax * ax + ay * ay + az * az;
#pragma unroll
                for (int i = NVR - 1; i > 0; --i) {
                    const bool lp = vless(dv2, pos, vdr[i - 1], vpr[i - 1]);
                    const bool lc = vless(dv2, pos, vdr[i], vpr[i]);
                    vdr[i] = lp ? vdr[i - 1] : (lc ? dv2 : vdr[i]);
                    vpr[i] = lp ? vpr[i - 1] : (lc ? pos : vpr[i]);
                }
                if (vless(dv2, pos, vdr[0], vpr[0])) { vdr[0] = dv2; vpr[0] = pos; }
            }
        }
        h2 = vdr[NVR - 1];
        if (h2 != 0.0) {
#pragma unroll
            for (int a = 0; a < NVR; ++a) {
                const double m = use_mass ? (double)V[base + vpr[a]].w : mass_value;
                sw += m * kW * (1.0 - vdr[a] / h2);
            }
        }
    } else {
        int nv = 0;
        for (int a0 = 0; a0 < n_se; a0 += VB) {
            fetch(a0);
            for (int u = 0; u < VB && a0 + u < n_se; ++u) {
                const int pos = bpos[u];
                msum += use_mass ? (double)bms[u] : mass_value;
                const double ax = vqx - (double)bvx[u], ay = vqy - (double)bvy[u], az = vqz - (double)bvz[u];
                const double dv2 = ax * ax + ay * ay + az * az;
                if (nv == n_v) {
                    if (!vless(dv2, pos, vd[n_v - 1][lane], vp[n_v - 1][lane])) continue;
                    --nv;
                }
                int i = nv++;
                while (i > 0 && vless(dv2, pos, vd[i - 1][lane], vp[i - 1][lane])) {
                    vd[i][lane] = vd[i - 1][lane];
                    vp[i][lane] = vp[i - 1][lane];
                    --i;
                }
                vd[i][lane] = dv2;
                vp[i][lane] = pos;
            }
        }
        h2 = vd[n_v - 1][lane];
        if (h2 != 0.0)
            for (int a = 0; a < n_v; ++a) {
                const double m = use_mass ? (double)V[base + vp[a][lane]].w : mass_value;
                sw += m * kW * (1.0 - vd[a][lane] / h2);
            }
    }
    const double lfl = h2 == 0.0 ? INFINITY : log(sw) - 1.5 * log(h2) - log(msum);
    R[F.gidx[e]] = (float)(lfl - FB[qe]);
}

template <int NSE, int NVR, int NVLMAX>
int launch_knn(vr_ctx* ctx, const uint32_t* qpos, int64_t nq, const KdTree& tree, const float4* V,
               const double* FB, const int32_t* host_off, const vr_particles* p, int n_se, int n_v, float* R,
               hipStream_t st) {
    VR_TIMED(ctx, "knn", st, nq,
             hipLaunchKernelGGL((k_knn<NSE, NVR, NVLMAX>), dim3(grid_for(nq, 64)), dim3(64), 0, st, qpos, nq, tree.nodes,
                                tree.F, tree.seg_node, V, FB, tree.elem_host, host_off, n_se, n_v, tree.use_mass, p->mass_value, p->grid_bits, R, (unsigned)ctx->xcd_chunk,
                                ctx->timing ? ctx->knn_cand : nullptr));
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}


// ---- large neighbour sets (n_se > 64, up to the paper's 256) --------------
// One wavefront per query.  Candidates of a visited leaf are keyed by the
// lanes (exact d2 << 22 | rank, minimum image), and those below the current
// bound W are appended to an LDS buffer.  When the buffer holds n_se + 64
// keys or more, a bitwise radix select over the wave finds the n_se-th
// smallest key T; the keys up to T are kept and W = T.  The tree walk (one
// shared stack, near child first) prunes nodes whose box is no nearer than
// W allows.  The n_v velocity neighbours are then taken from the n_se by
// repeated wave-wide minima of (FP64 dv2, rank).
constexpr int BIG_CAP = 256;              // largest n_se
constexpr int BIG_EXTRA = 192;            // keys appended past n_se before the buffer is cut back
constexpr int BIG_BUF = BIG_CAP + BIG_EXTRA + 64;  // room for one more leaf chunk
constexpr int BIG_J = BIG_BUF / 64;       // buffer slots per lane

// The r-th smallest (0-based) of the valid keys k[j] of all lanes.
// The key of rank r (0-based) among the valid keys of the wavefront, by a
// radix select over byte digits: per digit, a histogram of the keys that
// share the digits chosen so far, and a wave-wide prefix over its 256
// buckets to find the one holding rank r.  Keys are distinct.  hist: 256
// words of LDS.
__device__ __forceinline__ uint64_t wave_select(const uint64_t (&k)[BIG_J], const bool (&v)[BIG_J], int r,
                                                uint32_t* hist) {
    uint64_t lo = ~0ull, hi = 0;
#pragma unroll
    for (int j = 0; j < BIG_J; ++j)
        if (v[j]) {
            lo = min(lo, k[j]);
            hi = max(hi, k[j]);
        }
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, (uint64_t)__shfl_xor((unsigned long long)lo, o, 64));
        hi = max(hi, (uint64_t)__shfl_xor((unsigned long long)hi, o, 64));
    }
    if (lo == hi) return lo;
    const int lane = (int)lane_id();
    // digits above the highest differing byte are those of every key
    int shift = ((63 - __clzll(lo ^ hi)) >> 3) << 3;
    uint64_t above = shift + 8 >= 64 ? 0 : ~0ull << (shift + 8);
    uint64_t prefix = lo & above;
    for (;;) {
#pragma unroll
        for (int t = 0; t < 4; ++t) hist[4 * lane + t] = 0;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j = 0; j < BIG_J; ++j)
            if (v[j] && (k[j] & above) == prefix) atomicAdd(&hist[(k[j] >> shift) & 255], 1u);
        __builtin_amdgcn_wave_barrier();
        uint32_t c[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) c[t] = hist[4 * lane + t];
        const uint32_t sum = c[0] + c[1] + c[2] + c[3];
        uint32_t incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        const uint32_t excl = incl - sum;
        // the lane whose buckets span rank r names the digit
        int digit = -1;
        uint32_t below = excl;
        if ((uint32_t)r >= excl && (uint32_t)r < incl) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (digit < 0 && (uint32_t)r < below + c[t]) digit = 4 * lane + t;
                else if (digit < 0) below += c[t];
            }
        }
        const uint64_t owner = __ballot(digit >= 0);
        const int src = __builtin_ctzll(owner);
        digit = __shfl(digit, src, 64);
        below = __shfl(below, src, 64);
        r -= (int)below;
        prefix |= (uint64_t)digit << shift;
        __builtin_amdgcn_wave_barrier();
        if (shift == 0) break;
        above = ~0ull << shift;
        shift -= 8;
    }
    return prefix;
}

__global__ __launch_bounds__(64) void k_knn_big(const uint32_t* __restrict__ qpos, int64_t nq,
                                                const KdNode* __restrict__ nodes, Elems F,
                                                const float4* __restrict__ V, const double* __restrict__ FB,
                                                const int* __restrict__ elem_host, const int32_t* __restrict__ host_off,
                                                int n_se, int n_v, int use_mass, double mass_value, int gb,
                                                float* __restrict__ R, unsigned xchunk) {
    __shared__ uint64_t buf[BIG_BUF];
    __shared__ uint32_t sel_hist[256];
    __shared__ int stack[STACK];
    __shared__ double sel_d[32];
    __shared__ int sel_p[32];
    const int lane = threadIdx.x;
    const int64_t qi = (int64_t)xcd_swizzle(blockIdx.x, gridDim.x, xchunk);
    if (qi >= nq) return;  // uniform
    const int e = qpos ? (int)qpos[qi] : (int)qi;
    const int h = elem_host[e];
    const int base = host_off[h];
    const int px = F.u[0][e], py = F.u[1][e], pz = F.u[2][e];
    int nb = 0;            // keys in buf (uniform)
    uint64_t W = ~0ull;    // keys below W are taken (uniform)

    auto compact = [&]() __attribute__((always_inline)) {
        uint64_t k[BIG_J];
        bool v[BIG_J];
#pragma unroll
        for (int j = 0; j < BIG_J; ++j) {
            v[j] = lane + 64 * j < nb;
            k[j] = v[j] ? buf[lane + 64 * j] : 0;
        }
        const uint64_t T = wave_select(k, v, n_se - 1, sel_hist);
        __builtin_amdgcn_wave_barrier();
        int at = 0;
#pragma unroll
        for (int j = 0; j < BIG_J; ++j) {
            const bool keep = v[j] && k[j] <= T;
            const uint64_t m = __ballot(keep);
            if (keep) buf[at + __popcll(m & lanemask_lt())] = k[j];
            at += __popcll(m);
        }
        __builtin_amdgcn_wave_barrier();
        nb = n_se;
        W = T;
    };
    auto scan = [&](int node) __attribute__((always_inline)) {
        const KdNode& nd = nodes[node];
        for (int c0 = nd.start; c0 < nd.end; c0 += 64) {
            const int j = c0 + lane;
            bool take = false;
            uint64_t key = 0;
            if (j < nd.end) {
                const int64_t dx = min_image(F.u[0][j] - px, gb), dy = min_image(F.u[1][j] - py, gb),
                              dz = min_image(F.u[2][j] - pz, gb);
                const uint64_t d2 = (uint64_t)(dx * dx + dy * dy + dz * dz);
                key = (d2 << POS_BITS) | (uint64_t)(uint32_t)(F.eid[j] - base);
                take = key < W;
            }
            const uint64_t m = __ballot(take);
            if (take) buf[nb + __popcll(m & lanemask_lt())] = key;
            nb += __popcll(m);
            __builtin_amdgcn_wave_barrier();
            if (nb >= n_se + BIG_EXTRA) compact();
        }
    };
    if (lane == 0) stack[0] = h;
    int sp = 1;
    __builtin_amdgcn_wave_barrier();
    while (sp > 0) {
        const int node = stack[--sp];
        __builtin_amdgcn_wave_barrier();
        const KdNode& nd = nodes[node];
        const int64_t bx = max(max(nd.bmin[0] - px, px - nd.bmax[0]), 0);
        const int64_t by = max(max(nd.bmin[1] - py, py - nd.bmax[1]), 0);
        const int64_t bz = max(max(nd.bmin[2] - pz, pz - nd.bmax[2]), 0);
        int64_t md2 = bx * bx + by * by + bz * bz;
        if (md2 > (int64_t(1) << 41)) md2 = int64_t(1) << 41;
        if (nb >= n_se && ((uint64_t)md2 << POS_BITS) >= W) continue;
        if (nd.dim < 0) {
            scan(node);
            continue;
        }
        if (sp + 2 > STACK) break;  // cannot happen for trees of depth < 64
        const int dm = nd.dim;
        const int cf = px + (dm >= 1) * (py - px) + (dm == 2) * (pz - py);
        const int nearc = cf < nd.t ? nd.left : nd.right;
        const int farc = cf < nd.t ? nd.right : nd.left;
        if (lane == 0) {
            stack[sp] = farc;
            stack[sp + 1] = nearc;
        }
        sp += 2;
        __builtin_amdgcn_wave_barrier();
    }
    if (nb > n_se) compact();
    // the n_se spatial neighbours: velocity distances and the mass of the set
    const int qe = F.eid[e];
    const float4 vq = V[qe];
    const double vqx = (double)vq.x, vqy = (double)vq.y, vqz = (double)vq.z;
    double dv[BIG_CAP / 64];
    int ps[BIG_CAP / 64];
    double msum = 0.0;
#pragma unroll
    for (int j = 0; j < BIG_CAP / 64; ++j) {
        const int a = lane + 64 * j;
        dv[j] = INFINITY;
        ps[j] = 0x7FFFFFFF;
        if (a < n_se) {
            const int pos = (int)(buf[a] & POS_MASK);
            const float4 w = V[base + pos];
            msum += use_mass ? (double)w.w : mass_value;
            const double ax = vqx - (double)w.x, ay = vqy - (double)w.y, az = vqz - (double)w.z;
            dv[j] = ax * ax + ay * ay + az * az;
            ps[j] = pos;
        }
    }
    for (int o = 32; o > 0; o >>= 1) msum += __shfl_xor(msum, o, 64);
    // the n_v nearest in velocity, smallest first, by (dv2, rank)
    for (int i = 0; i < n_v; ++i) {
        double bd = INFINITY;
        int bp = 0x7FFFFFFF;
#pragma unroll
        for (int j = 0; j < BIG_CAP / 64; ++j)
            if (vless(dv[j], ps[j], bd, bp)) {
                bd = dv[j];
                bp = ps[j];
            }
        for (int o = 32; o > 0; o >>= 1) {
            const double od = __shfl_xor(bd, o, 64);
            const int op = __shfl_xor(bp, o, 64);
            if (vless(od, op, bd, bp)) {
                bd = od;
                bp = op;
            }
        }
#pragma unroll
        for (int j = 0; j < BIG_CAP / 64; ++j)
            if (ps[j] == bp) {
                dv[j] = INFINITY;
                ps[j] = 0x7FFFFFFF;
            }
        if (lane == 0) {
            sel_d[i] = bd;
            sel_p[i] = bp;
        }
    }
    __builtin_amdgcn_wave_barrier();
    if (lane != 0) return;
    const double kW = 15.0 / (8.0 * M_PI);
    const double h2 = sel_d[n_v - 1];
    double sw = 0.0;
    if (h2 != 0.0)
        for (int a = 0; a < n_v; ++a) {
            const double m = use_mass ? (double)V[base + sel_p[a]].w : mass_value;
            sw += m * kW * (1.0 - sel_d[a] / h2);
        }
    const double lfl = h2 == 0.0 ? INFINITY : log(sw) - 1.5 * log(h2) - log(msum);
    R[F.gidx[e]] = (float)(lfl - FB[qe]);
}

int launch_knn_big(vr_ctx* ctx, const uint32_t* qpos, int64_t nq, const KdTree& tree, const float4* V,
                   const double* FB, const int32_t* host_off, const vr_particles* p, int n_se, int n_v, float* R,
                   hipStream_t st) {
    if (nq > INT32_MAX) return set_err(ctx, VR_ERR_UNSUPPORTED, "too many queries for one launch");
    VR_TIMED(ctx, "knn", st, nq,
             hipLaunchKernelGGL(k_knn_big, dim3((unsigned)std::max<int64_t>(nq, 1)), dim3(64), 0, st, qpos, nq,
                                tree.nodes, tree.F, V, FB, tree.elem_host, host_off, n_se,
                                n_v, tree.use_mass, p->mass_value, p->grid_bits, R, (unsigned)ctx->xcd_chunk));
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

}  // namespace
}  // namespace vr

using namespace vr;

extern "C" int vr_local_vdensity(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts, const int32_t* host_offsets,
                                 const int32_t* host_members, const float* vbar, const float* sigma, int32_t n_se,
                                 int32_t n_v, const int32_t* subset, int64_t n_subset, float* R, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_particles(ctx, p, true);
    if (rc) return rc;
    if ((rc = check_hosts(ctx, n_hosts, host_offsets, host_members))) return rc;
    if (n_v < 2 || n_v > n_se || n_se > 256 || (n_se > 64 && n_v > 32))
        return set_err(ctx, VR_ERR_INVALID_ARG,
                       "need 2 <= n_v <= n_se <= 256, and n_v <= 32 when n_se > 64 (got n_se=%d, n_v=%d)", n_se, n_v);
    if (subset && n_subset < 0) return set_err(ctx, VR_ERR_INVALID_ARG, "n_subset < 0");
    if (n_hosts == 0 || (subset && n_subset == 0)) return VR_OK;
    if (!vbar || !sigma || !R) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> off;
    rc = read_host_offsets(ctx, n_hosts, host_offsets, p->n, n_se, off, st);
    if (rc) return rc;
    for (int h = 0; h < n_hosts; ++h)
        if ((int64_t)off[h + 1] - off[h] > (int64_t(1) << POS_BITS))
            return set_err(ctx, VR_ERR_UNSUPPORTED, "host %d has more than 2^%d members", h, POS_BITS);
    const int64_t M = off[n_hosts];
    VR_WS(rank_of, ctx, int32_t, WS_C2, p->n);
    VR_WS(dup, ctx, int, WS_FLAG, 4);
    rc = fill_i32(ctx, rank_of, -1, p->n, st);
    if (rc) return rc;
    rc = fill_i32(ctx, dup, 0, 1, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_rank_of, dim3(grid_for(M, 256)), dim3(256), 0, st, M, p->n, host_members, rank_of, dup);
    VR_LAUNCH_CHECK(ctx);
    int duph = 0;
    rc = read_back(ctx, dup, &duph, sizeof duph, st);
    if (rc) return rc;
    if (duph) return set_err(ctx, VR_ERR_INVALID_ARG, "host_members lists a particle twice or outside [0, n)");
    std::vector<int> nc(n_hosts, ctx->knn_leaf);
    KdTree tree;
    rc = kd_build(ctx, p, n_hosts, host_offsets, host_members, off, nc, KD_WIDEST, 2, tree, st);
    if (rc) return rc;
    VR_WS(V, ctx, float4, WS_C0, M);
    VR_WS(FB, ctx, double, WS_C1, M);
    hipLaunchKernelGGL(k_member_records, dim3(grid_for(p->n, 256)), dim3(256), 0, st, p->n, rank_of, p->vx, p->vy,
                       p->vz, p->mass, vbar, sigma, V, FB);
    VR_LAUNCH_CHECK(ctx);
    const uint32_t* qpos = nullptr;
    int64_t nq = M;
    if (subset) {
        VR_WS(pos_of, ctx, int, WS_C4, p->n);
        VR_WS(qp, ctx, uint32_t, WS_C5, n_subset);
        VR_WS(qv, ctx, uint32_t, WS_C6, n_subset);
        VR_WS(bad, ctx, int, WS_FLAG2, 4);
        rc = fill_i32(ctx, pos_of, -1, p->n, st);
        if (rc) return rc;
        rc = fill_i32(ctx, bad, 0, 1, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_pos_of, dim3(grid_for(M, 256)), dim3(256), 0, st, M, tree.F.gidx, pos_of);
        VR_LAUNCH_CHECK(ctx);
        hipLaunchKernelGGL(k_subset_pos, dim3(grid_for(n_subset, 256)), dim3(256), 0, st, n_subset, p->n, subset, pos_of,
                           qp, qv, bad);
        VR_LAUNCH_CHECK(ctx);
        int badh = 0;
        rc = read_back(ctx, bad, &badh, sizeof badh, st);
        if (rc) return rc;
        if (badh) return set_err(ctx, VR_ERR_INVALID_ARG, "subset lists a particle that is in no host");
        int bits = 1;
        while ((int64_t(1) << bits) < M) ++bits;
        rc = sort_pairs_u32(ctx, qp, qv, n_subset, bits, st);
        if (rc) return rc;
        qpos = qp;
        nq = n_subset;
    }
    if (n_se <= 32 && n_v == 8)
        return launch_knn<32, 8, 1>(ctx, qpos, nq, tree, V, FB, host_offsets, p, n_se, n_v, R, st);
    if (n_se <= 32)
        return launch_knn<32, 0, 32>(ctx, qpos, nq, tree, V, FB, host_offsets, p, n_se, n_v, R, st);
    if (n_se <= 64)
        return launch_knn<64, 0, 64>(ctx, qpos, nq, tree, V, FB, host_offsets, p, n_se, n_v, R, st);
    // larger sets, up to the paper's defaults (n_se 256, n_v 32): a wavefront per query
    return launch_knn_big(ctx, qpos, nq, tree, V, FB, host_offsets, p, n_se, n_v, R, st);
}
