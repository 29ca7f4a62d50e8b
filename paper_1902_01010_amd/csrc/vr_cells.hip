// vr_cells.hip -- entropy KD cells, per-cell velocity moments and their
// inverse-distance interpolation (Sec. 2.2: the entropy equation and Eqs.
// meanpos, meanvel, meandispvel, cellinterp).
//
// The tree is built level-synchronously for all hosts at once.  Each active
// node is one workgroup: it reduces the members' bounding box, histograms
// their masses per dimension into nbins bins, picks the split dimension by
// the normalised Shannon entropy, finds the median (rank floor(n/2) in
// (coordinate, index) order) with a two-pass 11-bit radix select, and writes
// a stable partition into the other element buffer, so every node's members
// stay in ascending particle-index order.  Leaves become cells numbered per
// host by their smallest member.
#include "vr_kd.h"

#include <cmath>

namespace vr {
namespace {

constexpr int KB = 256;

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int N>
__device__ __forceinline__ void block_sum_d(double (&v)[N], double* sm /* >= 4*N */) {
    const int lane = __lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double s = wave_sum_d(v[i]);
        if (lane == 0) sm[w * N + i] = s;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double s = 0;
        for (int ww = 0; ww < nw; ++ww) s += sm[ww * N + i];
        v[i] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ int floor_half(int a) { return a >= 0 ? a / 2 : -((-a + 1) / 2); }

__global__ void k_leaf_keys(int nleaf, const int* __restrict__ leaves, const KdNode* __restrict__ nodes,
                            const int* __restrict__ leaf_min, uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    const int id = leaves[i];
    key[i] = ((uint64_t)nodes[id].host << 32) | (uint32_t)leaf_min[id];
    val[i] = (uint32_t)id;
}

__global__ void k_leaf_cell(int nleaf, const uint32_t* __restrict__ sorted_node, int* __restrict__ leaf_cell) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nleaf) leaf_cell[sorted_node[c]] = c;
}

// Cell moments (Eqs. meanpos, meanvel, meandispvel), one workgroup per cell.
// Row layout: host, n, M, xbar[3], vbar[3], sigma[6], lo[3], hi[3], nbr[6], volume.
__global__ __launch_bounds__(KB) void k_cell_moments(int ncells, const uint32_t* __restrict__ cell_node,
                                                     const KdNode* __restrict__ nodes, Elems src,
                                                     const float* __restrict__ vx, const float* __restrict__ vy,
                                                     const float* __restrict__ vz, int use_mass, double mass_value,
                                                     double unit, double* __restrict__ table) {
    __shared__ double sm[4 * 13];
    const int c = blockIdx.x;
    const KdNode nd = nodes[cell_node[c]];
    // one pass: velocities are summed relative to the cell's first member,
    // v0, and the dispersion is E[(v - v0)(v - v0)^T] - (vbar - v0)(vbar - v0)^T,
    // the same FP64 moments as two passes about vbar up to rounding (both
    // terms are of the size of the dispersion, since v0 is a member)
    const int g0 = src.gidx[nd.start];
    const double v0[3] = {(double)vx[g0], (double)vy[g0], (double)vz[g0]};
    double acc[13] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = nd.start + threadIdx.x; k < nd.end; k += blockDim.x) {
        const double m = use_mass ? (double)src.mass[k] : mass_value;
        const int g = src.gidx[k];
        const double d0 = (double)vx[g] - v0[0], d1 = (double)vy[g] - v0[1], d2 = (double)vz[g] - v0[2];
        acc[0] += m;
        acc[1] += m * ((double)src.u[0][k] * unit);
        acc[2] += m * ((double)src.u[1][k] * unit);
        acc[3] += m * ((double)src.u[2][k] * unit);
        acc[4] += m * d0;
        acc[5] += m * d1;
        acc[6] += m * d2;
        acc[7] += m * d0 * d0;
        acc[8] += m * d1 * d1;
        acc[9] += m * d2 * d2;
        acc[10] += m * d0 * d1;
        acc[11] += m * d0 * d2;
        acc[12] += m * d1 * d2;
    }
    block_sum_d<13>(acc, sm);
    const double M = acc[0];
    const double dm[3] = {acc[4] / M, acc[5] / M, acc[6] / M};  // vbar - v0
    const double vb[3] = {v0[0] + dm[0], v0[1] + dm[1], v0[2] + dm[2]};
    const double s6[6] = {acc[7] - M * dm[0] * dm[0], acc[8] - M * dm[1] * dm[1], acc[9] - M * dm[2] * dm[2],
                          acc[10] - M * dm[0] * dm[1], acc[11] - M * dm[0] * dm[2], acc[12] - M * dm[1] * dm[2]};
    if (threadIdx.x == 0) {
        double* row = table + (int64_t)c * VR_CELL_COLS;
        row[0] = (double)nd.host;
        row[1] = (double)(nd.end - nd.start);
        row[2] = M;
        for (int d = 0; d < 3; ++d) { row[3 + d] = acc[1 + d] / M; row[6 + d] = vb[d]; }
        for (int e = 0; e < 6; ++e) row[9 + e] = s6[e] / M;
        double vol = 1.0;
        for (int d = 0; d < 3; ++d) {
            row[15 + d] = (double)nd.lo[d];
            row[18 + d] = (double)nd.hi[d];
            vol *= (double)((int64_t)nd.hi[d] - nd.lo[d] + 1) * unit;
        }
        row[27] = vol;
    }
}

// Face neighbours: probe one grid unit outside each face at the face centre
// and descend the host's tree to the leaf holding the probe.
__global__ void k_cell_faces(int ncells, const uint32_t* __restrict__ cell_node, const KdNode* __restrict__ nodes,
                             const int* __restrict__ leaf_cell, double* __restrict__ table) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncells * 6) return;
    const int c = i / 6, f = i % 6, d = f / 2;
    const KdNode nd = nodes[cell_node[c]];
    const KdNode root = nodes[nd.host];
    int pt[3];
    for (int e = 0; e < 3; ++e) pt[e] = floor_half(nd.lo[e] + nd.hi[e]);
    pt[d] = (f % 2 == 0) ? nd.lo[d] - 1 : nd.hi[d] + 1;
    bool inside = true;
    for (int e = 0; e < 3; ++e) inside &= pt[e] >= root.lo[e] && pt[e] <= root.hi[e];
    double out = -1.0;
    if (inside) {
        int cur = nd.host;
        for (int guard = 0; guard < 64 && nodes[cur].dim >= 0; ++guard) {
            const KdNode& x = nodes[cur];
            cur = pt[x.dim] < x.t ? x.left : x.right;
        }
        out = (double)leaf_cell[cur];
    }
    table[(int64_t)c * VR_CELL_COLS + 21 + f] = out;
}

// Inverse-distance interpolation (Eq. cellinterp) over the own cell and its
// face neighbours, in the order own, -x, +x, -y, +y, -z, +z.
__global__ __launch_bounds__(KB) void k_cell_interp(int ncells, int64_t n, const uint32_t* __restrict__ cell_node,
                                                    const KdNode* __restrict__ nodes, Elems src,
                                                    const double* __restrict__ table, int64_t cell_base,
                                                    double unit, float* __restrict__ vbar, float* __restrict__ sigma,
                                                    float* __restrict__ rho, int32_t* __restrict__ cell_of) {
    __shared__ double cv[7][9];
    __shared__ double cx[7][3];
    __shared__ int s_ns;
    const int c = blockIdx.x;
    const KdNode nd = nodes[cell_node[c]];
    const double* row = table + (int64_t)c * VR_CELL_COLS;
    // the cell and its face neighbours (-x, +x, -y, +y, -z, +z), in that
    // order: thread a < 7 loads entry a, so the rows arrive in one round trip
    if (threadIdx.x < 7) {
        const int a = (int)threadIdx.x;
        const int id = a == 0 ? c : (int)row[21 + a - 1];  // -1: no neighbour on that face
        const uint64_t have = __ballot(id >= 0) & 127u;
        if (id >= 0) {
            const int slot = __popcll(have & ((1ull << a) - 1ull));
            const double* r = table + (int64_t)id * VR_CELL_COLS;
            for (int d = 0; d < 3; ++d) { cx[slot][d] = r[3 + d]; cv[slot][d] = r[6 + d]; }
            for (int e = 0; e < 6; ++e) cv[slot][3 + e] = r[9 + e];
        }
        if (a == 0) s_ns = __popcll(have);
    }
    __syncthreads();
    const int ns = s_ns;
    const float rho_c = (float)(row[2] / row[27]);
    for (int k = nd.start + threadIdx.x; k < nd.end; k += blockDim.x) {
        const double xk0 = (double)src.u[0][k] * unit, xk1 = (double)src.u[1][k] * unit,
                     xk2 = (double)src.u[2][k] * unit;
        double wv[7];
        int exact = -1;
        for (int a = 0; a < ns; ++a) {
            const double dx = xk0 - cx[a][0], dy = xk1 - cx[a][1], dz = xk2 - cx[a][2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r == 0.0) { exact = a; break; }
            wv[a] = 1.0 / r;
        }
        double o[9];
        if (exact >= 0) {
            for (int e = 0; e < 9; ++e) o[e] = cv[exact][e];
        } else {
            double ws = 0.0, sv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int a = 0; a < ns; ++a) {
                ws += wv[a];
                for (int e = 0; e < 9; ++e) sv[e] += wv[a] * cv[a][e];
            }
            for (int e = 0; e < 9; ++e) o[e] = sv[e] / ws;
        }
        const int g = src.gidx[k];
        // particle-major: a member's 3 + 6 values are two contiguous records
        for (int d = 0; d < 3; ++d) vbar[(int64_t)g * 3 + d] = (float)o[d];
        for (int e = 0; e < 6; ++e) sigma[(int64_t)g * 6 + e] = (float)o[3 + e];
        if (rho) rho[g] = rho_c;
        if (cell_of) cell_of[g] = (int32_t)(cell_base + c);
    }
}

}  // namespace
}  // namespace vr

using namespace vr;

extern "C" int vr_cell_moments(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts, const int32_t* host_offsets,
                               const int32_t* host_members, const vr_cell_params* cp, float* vbar, float* sigma,
                               float* rho_cell, int32_t* cell_of, int64_t cell_capacity, double* cell_table,
                               int64_t* n_cells, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_particles(ctx, p, true);
    if (rc) return rc;
    if ((rc = check_hosts(ctx, n_hosts, host_offsets, host_members))) return rc;
    if (!cp || !n_cells) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL params or n_cells");
    if (cp->nbins < 2 || cp->nbins > 64) return set_err(ctx, VR_ERR_INVALID_ARG, "nbins must be in 2..64");
    if (cp->ncell_floor < 1 || cp->ncell_div < 1 || !(cp->f_cell > 0))
        return set_err(ctx, VR_ERR_INVALID_ARG, "bad cell parameters");
    if (cp->split_rule != 0 && cp->split_rule != 1) return set_err(ctx, VR_ERR_INVALID_ARG, "split_rule is 0 or 1");
    *n_cells = 0;
    if (n_hosts == 0) return VR_OK;
    if (!vbar || !sigma) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL output");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> off;
    rc = read_host_offsets(ctx, n_hosts, host_offsets, p->n, cp->ncell_div, off, st);
    if (rc) return rc;
    std::vector<int> nc(n_hosts);
    for (int h = 0; h < n_hosts; ++h) {
        const int64_t NH = (int64_t)off[h + 1] - off[h];
        int64_t c = (int64_t)std::ceil(cp->f_cell * (double)NH);
        if (c < cp->ncell_floor) c = cp->ncell_floor;
        if (c > NH / cp->ncell_div) c = NH / cp->ncell_div;
        nc[h] = (int)c;
    }
    KdTree tree;
    rc = kd_build(ctx, p, n_hosts, host_offsets, host_members, off, nc,
                  cp->split_rule == 0 ? KD_MIN_ENTROPY : KD_MAX_ENTROPY, cp->nbins, tree, st);
    if (rc) return rc;
    const int nleaf = tree.n_leaves;
    const int use_mass = tree.use_mass;
    *n_cells = nleaf;
    if (cell_table && cell_capacity < nleaf)
        return set_err(ctx, VR_ERR_INVALID_ARG, "cell_capacity %lld < %d cells", (long long)cell_capacity, nleaf);
    // node ids are below 2 * leaves: every split adds two nodes
    VR_WS(leaf_cell, ctx, int, WS_A9, (int64_t)tree.n_leaves * 2 + 2 * n_hosts + 8);
    VR_WS(lkey, ctx, uint64_t, WS_B6, nleaf);
    VR_WS(lval, ctx, uint32_t, WS_B7, nleaf);
    VR_WS(table, ctx, double, WS_B8, (int64_t)nleaf * VR_CELL_COLS);
    KdNode* nodes = tree.nodes;
    hipLaunchKernelGGL(k_leaf_keys, dim3(grid_for(nleaf, 256)), dim3(256), 0, st, nleaf, tree.leaves, nodes,
                       tree.leaf_min, lkey, lval);
    VR_LAUNCH_CHECK(ctx);
    int hb = 1;
    while ((1 << hb) <= n_hosts) ++hb;
    rc = sort_pairs_u64(ctx, lkey, lval, nleaf, 32 + hb, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_leaf_cell, dim3(grid_for(nleaf, 256)), dim3(256), 0, st, nleaf, lval, leaf_cell);
    VR_LAUNCH_CHECK(ctx);
    const double unit = p->box / ldexp(1.0, p->grid_bits);
    hipLaunchKernelGGL(k_cell_moments, dim3(nleaf), dim3(KB), 0, st, nleaf, lval, nodes, tree.F, p->vx, p->vy, p->vz,
                       use_mass, p->mass_value, unit, table);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_cell_faces, dim3(grid_for((int64_t)nleaf * 6, 256)), dim3(256), 0, st, nleaf, lval, nodes,
                       leaf_cell, table);
    VR_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_cell_interp, dim3(nleaf), dim3(KB), 0, st, nleaf, p->n, lval, nodes, tree.F, table, (int64_t)0,
                       unit, vbar, sigma, rho_cell, cell_of);
    VR_LAUNCH_CHECK(ctx);
    if (cell_table)
        VR_HIP(ctx, hipMemcpyAsync(cell_table, table, (size_t)nleaf * VR_CELL_COLS * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
    return VR_OK;
}
