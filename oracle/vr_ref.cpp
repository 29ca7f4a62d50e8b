// vr_ref.cpp -- plain FP64 CPU oracle of the phase-space halo-finder hot path.
//
// TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
// CPU-baseline leg of the benchmark, never by the product path.  Written from
// the paper (Elahi et al., VELOCIraptor): every function cites the passage it
// follows.  Nothing here is blocked, fused or reordered beyond what the
// definitions state; the uniform grids below only enumerate candidate pairs
// that the brute-force predicate then decides.
//
// Build: g++ -O2 -std=c++17 -fno-fast-math -ffp-contract=off -shared -fPIC
//
// Parity unpinned (by the paper): the face-neighbour probe rule and the
// minimum-entropy choice of the split dimension of the cell tree; both are
// readings of an under-specified passage and only structural invariants pin
// them.

#include "vr_ref.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

int g_threads = 1;

// Dynamic parallel-for over [0, n): each worker takes the next index.
void parallel_for(int64_t n, const std::function<void(int64_t)>& body) {
    int nt = g_threads;
    if (nt <= 1 || n <= 1) {
        for (int64_t i = 0; i < n; ++i) body(i);
        return;
    }
    if (nt > n) nt = (int)n;
    std::atomic<int64_t> next(0);
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&]() {
            for (;;) {
                int64_t i = next.fetch_add(1);
                if (i >= n) break;
                body(i);
            }
        });
    for (auto& th : pool) th.join();
}

inline double mass_of(const vr_ref_particles* p, int64_t i) {
    return p->mass ? (double)p->mass[i] : p->mass_value;
}

// Periodic minimum image of a grid-coordinate difference:
// ((a - b + half) mod size) - half, a value in [-half, half).
inline int64_t min_image(int64_t a, int64_t b, int32_t gb) {
    const int64_t size = int64_t(1) << gb, half = size >> 1;
    int64_t d = (a - b + half) % size;
    if (d < 0) d += size;
    return d - half;
}

inline int64_t dist2_grid(const vr_ref_particles* p, int64_t i, int64_t j) {
    const int32_t gb = p->grid_bits;
    int64_t dx = min_image(p->qx[i], p->qx[j], gb);
    int64_t dy = min_image(p->qy[i], p->qy[j], gb);
    int64_t dz = min_image(p->qz[i], p->qz[j], gb);
    return dx * dx + dy * dy + dz * dz;
}

inline double dv2_of(const vr_ref_particles* p, int64_t i, int64_t j) {
    double a = (double)p->vx[i] - (double)p->vx[j];
    double b = (double)p->vy[i] - (double)p->vy[j];
    double c = (double)p->vz[i] - (double)p->vz[j];
    return a * a + b * b + c * c;
}

bool valid_particles(const vr_ref_particles* p) {
    if (!p || p->n < 0 || p->n >= (int64_t(1) << 31)) return false;
    if (p->grid_bits < 1 || p->grid_bits > 21) return false;
    if (!(p->box > 0)) return false;
    if (p->n > 0 && (!p->qx || !p->qy || !p->qz)) return false;
    const uint32_t lim = uint32_t(1) << p->grid_bits;
    for (int64_t i = 0; i < p->n; ++i)
        if (p->qx[i] >= lim || p->qy[i] >= lim || p->qz[i] >= lim) return false;
    return true;
}

bool has_vel(const vr_ref_particles* p) { return p->n == 0 || (p->vx && p->vy && p->vz); }

// Union-find with union by smallest root: every root is the smallest index
// of its tree, so the final root of a component is its smallest member.
struct MinUnionFind {
    std::vector<int32_t> parent;
    explicit MinUnionFind(int64_t n) : parent(n) { std::iota(parent.begin(), parent.end(), 0); }
    int32_t find(int32_t a) {
        while (parent[a] != a) {
            parent[a] = parent[parent[a]];
            a = parent[a];
        }
        return a;
    }
    void unite(int32_t a, int32_t b) {
        int32_t ra = find(a), rb = find(b);
        if (ra == rb) return;
        if (ra < rb) parent[rb] = ra; else parent[ra] = rb;
    }
};

// Candidate-pair enumeration on a periodic uniform grid whose cell side
// (2^s grid units) is at least the linking length, so every pair closer than
// the linking length lies in the same or an adjacent cell.  Calls
// visit(i, j) once for every unordered pair (i != j) of listed points in
// neighbouring cells; the caller applies the exact predicate.
void for_grid_pairs(const vr_ref_particles* p, const std::vector<int32_t>& pts,
                    double ell_grid, const std::function<void(int32_t, int32_t)>& visit) {
    const int32_t gb = p->grid_bits;
    int s = 0;
    while ((double)(int64_t(1) << s) < ell_grid && s < gb) ++s;
    const int64_t nc = int64_t(1) << (gb - s);
    auto key_of = [&](int64_t cx, int64_t cy, int64_t cz) {
        return (uint64_t)((cz * nc + cy) * nc + cx);
    };
    std::unordered_map<uint64_t, std::vector<int32_t>> cells;
    cells.reserve(pts.size() * 2 + 1);
    for (int32_t i : pts)
        cells[key_of(p->qx[i] >> s, p->qy[i] >> s, p->qz[i] >> s)].push_back(i);
    for (auto& kv : cells) {
        const uint64_t ka = kv.first;
        const std::vector<int32_t>& A = kv.second;
        const int64_t ax = ka % nc, ay = (ka / nc) % nc, az = ka / (nc * nc);
        std::vector<uint64_t> nb;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int64_t bx = ((ax + dx) % nc + nc) % nc;
                    int64_t by = ((ay + dy) % nc + nc) % nc;
                    int64_t bz = ((az + dz) % nc + nc) % nc;
                    nb.push_back(key_of(bx, by, bz));
                }
        std::sort(nb.begin(), nb.end());
        nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
        for (uint64_t kb : nb) {
            if (kb < ka) continue;  // each unordered cell pair once
            auto it = cells.find(kb);
            if (it == cells.end()) continue;
            const std::vector<int32_t>& B = it->second;
            if (kb == ka) {
                for (size_t x = 0; x < A.size(); ++x)
                    for (size_t y = x + 1; y < A.size(); ++y) visit(A[x], A[y]);
            } else {
                for (int32_t a : A)
                    for (int32_t b : B) visit(a, b);
            }
        }
    }
}

bool members_ok(int64_t n, int32_t n_hosts, const int32_t* off, const int32_t* mem) {
    if (n_hosts < 0) return false;
    if (n_hosts == 0) return true;
    if (!off || !mem || off[0] != 0) return false;
    for (int32_t h = 0; h < n_hosts; ++h) {
        if (off[h + 1] < off[h]) return false;
        for (int32_t k = off[h]; k < off[h + 1]; ++k) {
            if (mem[k] < 0 || mem[k] >= n) return false;
            if (k > off[h] && mem[k] <= mem[k - 1]) return false;
        }
    }
    return true;
}

}  // namespace

extern "C" {

int vr_ref_set_threads(int n_threads) {
    g_threads = n_threads < 1 ? 1 : n_threads;
    return g_threads;
}

// Quantisation onto the 2^grid_bits integer grid of the box (the configs fix
// 21-bit grid coordinates in a periodic box).
int vr_ref_quantize(int64_t n, const float* x, const float* y, const float* z,
                    double box, int32_t grid_bits, uint32_t* qx, uint32_t* qy, uint32_t* qz) {
    if (n < 0 || grid_bits < 1 || grid_bits > 21 || !(box > 0)) return -1;
    if (n > 0 && (!x || !y || !z || !qx || !qy || !qz)) return -1;
    const double scale = std::ldexp(1.0, grid_bits) / box;
    const int64_t mask = (int64_t(1) << grid_bits) - 1;
    for (int64_t i = 0; i < n; ++i) {
        qx[i] = (uint32_t)((int64_t)std::floor((double)x[i] * scale) & mask);
        qy[i] = (uint32_t)((int64_t)std::floor((double)y[i] * scale) & mask);
        qz[i] = (uint32_t)((int64_t)std::floor((double)z[i] * scale) & mask);
    }
    return 0;
}

double vr_ref_ell2_grid(double ell, double box, int32_t grid_bits) {
    double u = ell * std::ldexp(1.0, grid_bits) / box;
    return u * u;
}

// 3D FOF, Eq. fof3d (Sec. 2.1): |x_i - x_j|^2 / ellx^2 < 1, strict.
int vr_ref_fof3d(const vr_ref_particles* p, double ellx, int32_t* label) {
    if (!valid_particles(p) || (p->n > 0 && !label)) return -1;
    const double ell2 = vr_ref_ell2_grid(ellx, p->box, p->grid_bits);
    const double half = std::ldexp(1.0, p->grid_bits - 1);
    if (!(ell2 > 0) || !(std::sqrt(ell2) < half)) return -1;
    MinUnionFind uf(p->n);
    std::vector<int32_t> all(p->n);
    std::iota(all.begin(), all.end(), 0);
    for_grid_pairs(p, all, std::sqrt(ell2), [&](int32_t i, int32_t j) {
        if ((double)dist2_grid(p, i, j) < ell2) uf.unite(i, j);
    });
    for (int64_t i = 0; i < p->n; ++i) label[i] = uf.find((int32_t)i);
    return 0;
}

// Groups of at least N_min members (Sec. 2.2, last paragraph of the
// unbinding passage), in a deterministic order.
int vr_ref_groups(int64_t n, const int32_t* label, int32_t n_min, int32_t* n_groups,
                  int32_t* group_of, int32_t* offsets, int32_t* members) {
    if (n < 0 || n_min < 1 || !n_groups || (n > 0 && (!label || !group_of || !offsets || !members)))
        return -1;
    std::unordered_map<int32_t, std::vector<int32_t>> comp;
    for (int64_t i = 0; i < n; ++i) {
        if (label[i] < 0) continue;
        if (label[i] >= n) return -1;
        comp[label[i]].push_back((int32_t)i);
    }
    std::vector<std::vector<int32_t>*> keep;
    for (auto& kv : comp)
        if ((int64_t)kv.second.size() >= n_min) keep.push_back(&kv.second);
    std::sort(keep.begin(), keep.end(), [](const std::vector<int32_t>* a, const std::vector<int32_t>* b) {
        if (a->size() != b->size()) return a->size() > b->size();
        return a->front() < b->front();
    });
    for (int64_t i = 0; i < n; ++i) group_of[i] = -1;
    int32_t pos = 0;
    if (offsets) offsets[0] = 0;
    for (size_t g = 0; g < keep.size(); ++g) {
        for (int32_t i : *keep[g]) {  // members were appended in ascending order
            members[pos++] = i;
            group_of[i] = (int32_t)g;
        }
        offsets[g + 1] = pos;
    }
    *n_groups = (int32_t)keep.size();
    return 0;
}

// Normalised Shannon entropy of the mass histogram (Sec. 2.2).
double vr_ref_entropy(int32_t nb, const double* hist) {
    double tot = 0.0;
    for (int32_t k = 0; k < nb; ++k) tot += hist[k];
    if (!(tot > 0) || nb < 2) return 0.0;
    double s = 0.0;
    for (int32_t k = 0; k < nb; ++k) {
        if (hist[k] > 0) {
            double pk = hist[k] / tot;
            s -= pk * std::log(pk);
        }
    }
    return s / std::log((double)nb);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Entropy KD cells (Sec. 2.2: cells of N_cell particles split along the
// dimension chosen by the entropy of a binned mass histogram; moments from
// Eqs. meanpos, meanvel, meandispvel; interpolation from Eq. cellinterp).
namespace {

struct KdNode {
    int64_t lo[3], hi[3];
    int dim = -1;        // split dimension, -1 for a leaf
    int64_t t = 0;       // split value: left iff coordinate < t
    int left = -1, right = -1;
    std::vector<int32_t> mem;  // positions into the host arrays (leaves only)
};

struct HostCells {
    std::vector<KdNode> nodes;
    std::vector<int> leaves;  // node ids, ordered by smallest member index
};

void kd_split(HostCells& hc, int node, const std::vector<int64_t> (&u)[3],
              const std::vector<double>& m, const std::vector<int32_t>& gidx,
              int64_t ncell, const vr_ref_cell_params* cp) {
    std::vector<int32_t> mem = std::move(hc.nodes[node].mem);
    const int64_t n = (int64_t)mem.size();
    if (n <= ncell) { hc.nodes[node].mem = std::move(mem); return; }
    int64_t mn[3], mx[3];
    for (int d = 0; d < 3; ++d) {
        mn[d] = mx[d] = u[d][mem[0]];
        for (int32_t k : mem) { mn[d] = std::min(mn[d], u[d][k]); mx[d] = std::max(mx[d], u[d][k]); }
    }
    const int nb = cp->nbins;
    double S[3];
    for (int d = 0; d < 3; ++d) {
        S[d] = 0;
        if (mx[d] == mn[d]) continue;
        std::vector<double> h(nb, 0.0);
        for (int32_t k : mem) h[((u[d][k] - mn[d]) * nb) / (mx[d] - mn[d] + 1)] += m[k];
        S[d] = vr_ref_entropy(nb, h.data());
    }
    int best = -1;
    for (int d = 0; d < 3; ++d) {
        if (mx[d] == mn[d]) continue;
        if (best < 0) { best = d; continue; }
        bool better = cp->split_rule == 0 ? (S[d] < S[best] - 1e-12) : (S[d] > S[best] + 1e-12);
        if (better) best = d;
    }
    if (best < 0) { hc.nodes[node].mem = std::move(mem); return; }  // all coincident
    const int d = best;
    std::sort(mem.begin(), mem.end(), [&](int32_t a, int32_t b) {
        if (u[d][a] != u[d][b]) return u[d][a] < u[d][b];
        return gidx[a] < gidx[b];
    });
    const int64_t nl = n / 2;
    KdNode L, R;
    for (int e = 0; e < 3; ++e) { L.lo[e] = R.lo[e] = hc.nodes[node].lo[e]; L.hi[e] = R.hi[e] = hc.nodes[node].hi[e]; }
    const int64_t t = u[d][mem[nl]];
    L.hi[d] = t - 1;
    R.lo[d] = t;
    L.mem.assign(mem.begin(), mem.begin() + nl);
    R.mem.assign(mem.begin() + nl, mem.end());
    hc.nodes[node].dim = d;
    hc.nodes[node].t = t;
    int li = (int)hc.nodes.size();
    hc.nodes.push_back(std::move(L));
    int ri = (int)hc.nodes.size();
    hc.nodes.push_back(std::move(R));
    hc.nodes[node].left = li;
    hc.nodes[node].right = ri;
    kd_split(hc, li, u, m, gidx, ncell, cp);
    kd_split(hc, ri, u, m, gidx, ncell, cp);
}

}  // namespace

extern "C" int vr_ref_cell_moments(const vr_ref_particles* p, int32_t n_hosts,
                                   const int32_t* host_offsets, const int32_t* host_members,
                                   const vr_ref_cell_params* cp, float* vbar, float* sigma,
                                   float* rho_cell, int32_t* cell_of, int64_t cell_capacity,
                                   double* cell_table, int64_t* n_cells) {
    if (!valid_particles(p) || !has_vel(p) || !cp || !n_cells) return -1;
    if (!members_ok(p->n, n_hosts, host_offsets, host_members)) return -1;
    if (cp->nbins < 2 || cp->ncell_floor < 1 || cp->ncell_div < 1 || !(cp->f_cell > 0)) return -1;
    if (p->n > 0 && (!vbar || !sigma || !rho_cell || !cell_of)) return -1;
    const int32_t gb = p->grid_bits;
    const double unit = p->box / std::ldexp(1.0, gb);
    std::vector<HostCells> hcs(n_hosts);
    for (int32_t h = 0; h < n_hosts; ++h) {
        const int64_t NH = host_offsets[h + 1] - host_offsets[h];
        if (NH < cp->ncell_div) return -1;
    }
    std::vector<int64_t> cell_base(n_hosts + 1, 0);
    // Build each host's tree independently.
    parallel_for(n_hosts, [&](int64_t h) {
        const int32_t* mem = host_members + host_offsets[h];
        const int64_t NH = host_offsets[h + 1] - host_offsets[h];
        // Unwrap by the minimum image relative to the smallest-index member.
        std::vector<int64_t> u[3];
        std::vector<double> m(NH);
        std::vector<int32_t> gidx(NH);
        const uint32_t* q[3] = {p->qx, p->qy, p->qz};
        for (int d = 0; d < 3; ++d) {
            u[d].resize(NH);
            const int64_t ref = q[d][mem[0]];
            for (int64_t k = 0; k < NH; ++k) u[d][k] = ref + min_image(q[d][mem[k]], ref, gb);
        }
        for (int64_t k = 0; k < NH; ++k) { m[k] = mass_of(p, mem[k]); gidx[k] = mem[k]; }
        int64_t ncell = (int64_t)std::ceil(cp->f_cell * (double)NH);
        ncell = std::max<int64_t>(ncell, cp->ncell_floor);
        ncell = std::min<int64_t>(ncell, NH / cp->ncell_div);
        HostCells& hc = hcs[h];
        KdNode root;
        for (int d = 0; d < 3; ++d) {
            root.lo[d] = *std::min_element(u[d].begin(), u[d].end());
            root.hi[d] = *std::max_element(u[d].begin(), u[d].end());
        }
        root.mem.resize(NH);
        std::iota(root.mem.begin(), root.mem.end(), 0);
        hc.nodes.push_back(std::move(root));
        kd_split(hc, 0, u, m, gidx, ncell, cp);
        for (int i = 0; i < (int)hc.nodes.size(); ++i)
            if (hc.nodes[i].dim < 0) hc.leaves.push_back(i);
        std::sort(hc.leaves.begin(), hc.leaves.end(), [&](int a, int b) {
            return *std::min_element(hc.nodes[a].mem.begin(), hc.nodes[a].mem.end()) <
                   *std::min_element(hc.nodes[b].mem.begin(), hc.nodes[b].mem.end());
        });
    });
    for (int32_t h = 0; h < n_hosts; ++h) cell_base[h + 1] = cell_base[h] + (int64_t)hcs[h].leaves.size();
    *n_cells = cell_base[n_hosts];
    if (cell_table && cell_capacity < *n_cells) return -1;

    parallel_for(n_hosts, [&](int64_t h) {
        const int32_t* mem = host_members + host_offsets[h];
        const int64_t NH = host_offsets[h + 1] - host_offsets[h];
        const uint32_t* q[3] = {p->qx, p->qy, p->qz};
        const float* v[3] = {p->vx, p->vy, p->vz};
        std::vector<int64_t> u[3];
        for (int d = 0; d < 3; ++d) {
            u[d].resize(NH);
            const int64_t ref = q[d][mem[0]];
            for (int64_t k = 0; k < NH; ++k) u[d][k] = ref + min_image(q[d][mem[k]], ref, gb);
        }
        HostCells& hc = hcs[h];
        const int nleaf = (int)hc.leaves.size();
        std::vector<int> leaf_rank(hc.nodes.size(), -1);
        for (int c = 0; c < nleaf; ++c) leaf_rank[hc.leaves[c]] = c;
        struct Cell { double M, x[3], v[3], s[6], vol; int nbr[6]; };
        std::vector<Cell> cells(nleaf);
        for (int c = 0; c < nleaf; ++c) {
            const KdNode& nd = hc.nodes[hc.leaves[c]];
            Cell& C = cells[c];
            // Eqs. meanpos, meanvel: mass-weighted means.
            C.M = 0;
            for (int d = 0; d < 3; ++d) C.x[d] = C.v[d] = 0;
            for (int32_t k : nd.mem) {
                double mk = mass_of(p, mem[k]);
                C.M += mk;
                for (int d = 0; d < 3; ++d) {
                    C.x[d] += mk * ((double)u[d][k] * unit);
                    C.v[d] += mk * (double)v[d][mem[k]];
                }
            }
            for (int d = 0; d < 3; ++d) { C.x[d] /= C.M; C.v[d] /= C.M; }
            // Eq. meandispvel: biased (1/M) dispersion tensor about the mean.
            static const int I[6] = {0, 1, 2, 0, 0, 1}, J[6] = {0, 1, 2, 1, 2, 2};
            for (int a = 0; a < 6; ++a) C.s[a] = 0;
            for (int32_t k : nd.mem) {
                double mk = mass_of(p, mem[k]);
                double dv[3];
                for (int d = 0; d < 3; ++d) dv[d] = (double)v[d][mem[k]] - C.v[d];
                for (int a = 0; a < 6; ++a) C.s[a] += mk * dv[I[a]] * dv[J[a]];
            }
            for (int a = 0; a < 6; ++a) C.s[a] /= C.M;
            C.vol = 1.0;
            for (int d = 0; d < 3; ++d) C.vol *= (double)(nd.hi[d] - nd.lo[d] + 1) * unit;
            // Face neighbours: probe one grid unit outside each face at the
            // centre of the face, descend the tree to the leaf holding it.
            const KdNode& root = hc.nodes[0];
            for (int f = 0; f < 6; ++f) {
                const int d = f / 2;
                int64_t pt[3];
                for (int e = 0; e < 3; ++e) {
                    int64_t s = nd.lo[e] + nd.hi[e];
                    pt[e] = (s >= 0) ? s / 2 : -((-s + 1) / 2);  // floor((lo+hi)/2)
                }
                pt[d] = (f % 2 == 0) ? nd.lo[d] - 1 : nd.hi[d] + 1;
                bool inside = true;
                for (int e = 0; e < 3; ++e)
                    if (pt[e] < root.lo[e] || pt[e] > root.hi[e]) inside = false;
                C.nbr[f] = -1;
                if (!inside) continue;
                int cur = 0;
                while (hc.nodes[cur].dim >= 0)
                    cur = pt[hc.nodes[cur].dim] < hc.nodes[cur].t ? hc.nodes[cur].left : hc.nodes[cur].right;
                C.nbr[f] = leaf_rank[cur];
            }
        }
        // Eq. cellinterp: inverse-distance weights over the own cell and its
        // face neighbours, own cell first then -x,+x,-y,+y,-z,+z.
        for (int c = 0; c < nleaf; ++c) {
            const KdNode& nd = hc.nodes[hc.leaves[c]];
            int set[7], ns = 0;
            set[ns++] = c;
            for (int f = 0; f < 6; ++f)
                if (cells[c].nbr[f] >= 0) set[ns++] = cells[c].nbr[f];
            for (int32_t k : nd.mem) {
                const int32_t gi = mem[k];
                double xk[3];
                for (int d = 0; d < 3; ++d) xk[d] = (double)u[d][k] * unit;
                double w[7];
                int exact = -1;
                for (int a = 0; a < ns; ++a) {
                    const Cell& C = cells[set[a]];
                    double dx = xk[0] - C.x[0], dy = xk[1] - C.x[1], dz = xk[2] - C.x[2];
                    double r = std::sqrt(dx * dx + dy * dy + dz * dz);
                    if (r == 0.0) { exact = set[a]; break; }
                    w[a] = 1.0 / r;
                }
                double ov[3], os[6];
                if (exact >= 0) {
                    for (int d = 0; d < 3; ++d) ov[d] = cells[exact].v[d];
                    for (int e = 0; e < 6; ++e) os[e] = cells[exact].s[e];
                } else {
                    double wsum = 0, sv[3] = {0, 0, 0}, ss[6] = {0, 0, 0, 0, 0, 0};
                    for (int a = 0; a < ns; ++a) {
                        const Cell& C = cells[set[a]];
                        wsum += w[a];
                        for (int d = 0; d < 3; ++d) sv[d] += w[a] * C.v[d];
                        for (int e = 0; e < 6; ++e) ss[e] += w[a] * C.s[e];
                    }
                    for (int d = 0; d < 3; ++d) ov[d] = sv[d] / wsum;
                    for (int e = 0; e < 6; ++e) os[e] = ss[e] / wsum;
                }
                for (int d = 0; d < 3; ++d) vbar[(int64_t)d * p->n + gi] = (float)ov[d];
                for (int e = 0; e < 6; ++e) sigma[(int64_t)e * p->n + gi] = (float)os[e];
                rho_cell[gi] = (float)(cells[c].M / cells[c].vol);
                cell_of[gi] = (int32_t)(cell_base[h] + c);
            }
            if (cell_table) {
                double* row = cell_table + (cell_base[h] + c) * VR_REF_CELL_COLS;
                const Cell& C = cells[c];
                row[0] = (double)h;
                row[1] = (double)nd.mem.size();
                row[2] = C.M;
                for (int d = 0; d < 3; ++d) { row[3 + d] = C.x[d]; row[6 + d] = C.v[d]; }
                for (int e = 0; e < 6; ++e) row[9 + e] = C.s[e];
                for (int d = 0; d < 3; ++d) { row[15 + d] = (double)nd.lo[d]; row[18 + d] = (double)nd.hi[d]; }
                for (int f = 0; f < 6; ++f) row[21 + f] = C.nbr[f] >= 0 ? (double)(cell_base[h] + C.nbr[f]) : -1.0;
                row[27] = C.vol;
            }
        }
    });
    return 0;
}

// ---------------------------------------------------------------------------
// Local velocity density and the ratio R (Sec. 2.2).
extern "C" int vr_ref_local_vdensity(const vr_ref_particles* p, int32_t n_hosts,
                                     const int32_t* host_offsets, const int32_t* host_members,
                                     const float* vbar, const float* sigma, int32_t n_se,
                                     int32_t n_v, const int32_t* subset, int64_t n_subset,
                                     float* R, double* lnfl, double* lnfbg, int32_t* nbr_s,
                                     int32_t* nbr_v) {
    if (!valid_particles(p) || !has_vel(p)) return -1;
    if (!members_ok(p->n, n_hosts, host_offsets, host_members)) return -1;
    if (n_v < 2 || n_v > n_se || n_se > 256) return -1;
    if (p->n > 0 && (!vbar || !sigma || !R)) return -1;
    std::vector<int32_t> host_of(p->n, -1);
    for (int32_t h = 0; h < n_hosts; ++h) {
        if (host_offsets[h + 1] - host_offsets[h] < n_se) return -1;
        for (int32_t k = host_offsets[h]; k < host_offsets[h + 1]; ++k) host_of[host_members[k]] = h;
    }
    std::vector<int32_t> work;
    if (subset) {
        if (n_subset < 0) return -1;
        for (int64_t s = 0; s < n_subset; ++s) {
            if (subset[s] < 0 || subset[s] >= p->n || host_of[subset[s]] < 0) return -1;
            work.push_back(subset[s]);
        }
    } else {
        for (int32_t h = 0; h < n_hosts; ++h)
            for (int32_t k = host_offsets[h]; k < host_offsets[h + 1]; ++k) work.push_back(host_members[k]);
    }
    const double kW = 15.0 / (8.0 * M_PI);  // Epanechnikov normalisation in 3D
    const double ln2pi = std::log(2.0 * M_PI);
    parallel_for((int64_t)work.size(), [&](int64_t w) {
        const int32_t k = work[w];
        const int32_t h = host_of[k];
        const int32_t* mem = host_members + host_offsets[h];
        const int64_t NH = host_offsets[h + 1] - host_offsets[h];
        // S_k: the N_se members nearest in space (self included), by (d2, index).
        std::vector<std::pair<int64_t, int32_t>> ds(NH);
        for (int64_t a = 0; a < NH; ++a) ds[a] = {dist2_grid(p, k, mem[a]), mem[a]};
        std::partial_sort(ds.begin(), ds.begin() + n_se, ds.end());
        // V_k: the N_v elements of S_k nearest in velocity, by (dv2, index).
        std::vector<std::pair<double, int32_t>> vs(n_se);
        double msum_s = 0.0;
        for (int32_t a = 0; a < n_se; ++a) {
            vs[a] = {dv2_of(p, k, ds[a].second), ds[a].second};
            msum_s += mass_of(p, ds[a].second);
        }
        std::partial_sort(vs.begin(), vs.begin() + n_v, vs.end());
        if (nbr_s) for (int32_t a = 0; a < n_se; ++a) nbr_s[w * n_se + a] = ds[a].second;
        if (nbr_v) for (int32_t a = 0; a < n_v; ++a) nbr_v[w * n_v + a] = vs[a].second;
        // Bandwidth: distance to the N_v-th velocity neighbour.
        const double h2 = vs[n_v - 1].first;
        double lfl;
        if (h2 == 0.0) {
            lfl = std::numeric_limits<double>::infinity();
        } else {
            double sw = 0.0;
            for (int32_t a = 0; a < n_v; ++a) sw += mass_of(p, vs[a].second) * kW * (1.0 - vs[a].first / h2);
            lfl = std::log(sw) - 1.5 * std::log(h2) - std::log(msum_s);
        }
        // Background: multivariate Gaussian (Eq. fvbg) at the interpolated
        // mean velocity and dispersion tensor, through a 3x3 Cholesky factor.
        const int64_t n = p->n;
        double S00 = sigma[0 * n + k], S11 = sigma[1 * n + k], S22 = sigma[2 * n + k];
        double S10 = sigma[3 * n + k], S20 = sigma[4 * n + k], S21 = sigma[5 * n + k];
        double lfb = std::numeric_limits<double>::quiet_NaN();
        double r00 = S00;
        if (r00 > 0) {
            double L00 = std::sqrt(r00);
            double L10 = S10 / L00, L20 = S20 / L00;
            double r11 = S11 - L10 * L10;
            if (r11 > 0) {
                double L11 = std::sqrt(r11);
                double L21 = (S21 - L20 * L10) / L11;
                double r22 = S22 - L20 * L20 - L21 * L21;
                if (r22 > 0) {
                    double L22 = std::sqrt(r22);
                    double d0 = (double)p->vx[k] - (double)vbar[0 * n + k];
                    double d1 = (double)p->vy[k] - (double)vbar[1 * n + k];
                    double d2 = (double)p->vz[k] - (double)vbar[2 * n + k];
                    double y0 = d0 / L00;
                    double y1 = (d1 - L10 * y0) / L11;
                    double y2 = (d2 - L20 * y0 - L21 * y1) / L22;
                    double quad = y0 * y0 + y1 * y1 + y2 * y2;
                    double lndet = 2.0 * (std::log(L00) + std::log(L11) + std::log(L22));
                    lfb = -0.5 * quad - 1.5 * ln2pi - 0.5 * lndet;
                }
            }
        }
        if (lnfl) lnfl[k] = lfl;
        if (lnfbg) lnfbg[k] = lfb;
        R[k] = (float)(lfl - lfb);
    });
    return 0;
}

// Velocity linking length of a host (Sec. 2.1: ellv = alpha_v sigma_v).
extern "C" int vr_ref_host_ellv(const vr_ref_particles* p, int32_t n_hosts,
                                const int32_t* host_offsets, const int32_t* host_members,
                                double alpha_v, double* ellv_host) {
    if (!valid_particles(p) || !has_vel(p)) return -1;
    if (!members_ok(p->n, n_hosts, host_offsets, host_members)) return -1;
    if (n_hosts > 0 && !ellv_host) return -1;
    const float* v[3] = {p->vx, p->vy, p->vz};
    for (int32_t h = 0; h < n_hosts; ++h) {
        double M = 0, mv[3] = {0, 0, 0};
        for (int32_t k = host_offsets[h]; k < host_offsets[h + 1]; ++k) {
            double mk = mass_of(p, host_members[k]);
            M += mk;
            for (int d = 0; d < 3; ++d) mv[d] += mk * (double)v[d][host_members[k]];
        }
        if (!(M > 0)) return -1;
        for (int d = 0; d < 3; ++d) mv[d] /= M;
        double s[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int32_t k = host_offsets[h]; k < host_offsets[h + 1]; ++k) {
            double mk = mass_of(p, host_members[k]);
            double dv[3];
            for (int d = 0; d < 3; ++d) dv[d] = (double)v[d][host_members[k]] - mv[d];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) s[a][b] += mk * dv[a] * dv[b];
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) s[a][b] /= M;
        double det = s[0][0] * (s[1][1] * s[2][2] - s[1][2] * s[2][1]) -
                     s[0][1] * (s[1][0] * s[2][2] - s[1][2] * s[2][0]) +
                     s[0][2] * (s[1][0] * s[2][1] - s[1][1] * s[2][0]);
        ellv_host[h] = alpha_v * std::pow(det, 1.0 / 6.0);
    }
    return 0;
}

// 6D FOF over outliers (Eq. fof6d with the substructure linking length).
extern "C" int vr_ref_fof6d(const vr_ref_particles* p, const int32_t* host_of, int32_t n_hosts,
                            const double* ellv_host, double ellx_s, const float* R,
                            float R_threshold, int32_t* label6) {
    if (!valid_particles(p) || !has_vel(p) || (p->n > 0 && (!host_of || !ellv_host || !label6)))
        return -1;
    const double ell2 = vr_ref_ell2_grid(ellx_s, p->box, p->grid_bits);
    if (!(ell2 > 0) || !(std::sqrt(ell2) < std::ldexp(1.0, p->grid_bits - 1))) return -1;
    std::vector<int32_t> part;
    for (int64_t i = 0; i < p->n; ++i) {
        bool in = host_of[i] >= 0 && host_of[i] < n_hosts && (R == nullptr || R[i] >= R_threshold);
        if (in) {
            if (!(ellv_host[host_of[i]] > 0)) return -1;
            part.push_back((int32_t)i);
        }
    }
    MinUnionFind uf(p->n);
    for_grid_pairs(p, part, std::sqrt(ell2), [&](int32_t i, int32_t j) {
        if (host_of[i] != host_of[j]) return;
        const double ev = ellv_host[host_of[i]];
        const double t = (double)dist2_grid(p, i, j) / ell2 + dv2_of(p, i, j) / (ev * ev);
        if (t < 1.0) uf.unite(i, j);
    });
    for (int64_t i = 0; i < p->n; ++i) label6[i] = -1;
    for (int32_t i : part) label6[i] = uf.find(i);
    return 0;
}

// The paper's own substructure linker (Sec. 2.2, Eq. linkingcriteria): both
// particles significant outliers (L >= L_th), closer than the substructure
// linking length, speeds within a factor Vr and velocity directions within
// the opening angle, velocities taken relative to the local mean velocity.
extern "C" int vr_ref_fof_sub(const vr_ref_particles* p, const int32_t* host_of, int32_t n_hosts,
                              const float* vbar, double ellx_s, const float* L, float L_threshold, double Vr,
                              double cos_op, int32_t* label) {
    if (!valid_particles(p) || !has_vel(p) || (p->n > 0 && (!host_of || !vbar || !L || !label))) return -1;
    if (!(Vr >= 1.0) || !(cos_op >= -1.0 && cos_op <= 1.0) || n_hosts < 0) return -1;
    const double ell2 = vr_ref_ell2_grid(ellx_s, p->box, p->grid_bits);
    if (!(ell2 > 0) || !(std::sqrt(ell2) < std::ldexp(1.0, p->grid_bits - 1))) return -1;
    const int64_t n = p->n;
    std::vector<int32_t> part;
    for (int64_t i = 0; i < n; ++i)
        if (host_of[i] >= 0 && host_of[i] < n_hosts && L[i] >= L_threshold) part.push_back((int32_t)i);
    auto rel = [&](int64_t i, double* u) {
        u[0] = (double)p->vx[i] - (double)vbar[i];
        u[1] = (double)p->vy[i] - (double)vbar[n + i];
        u[2] = (double)p->vz[i] - (double)vbar[2 * n + i];
        return std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    };
    MinUnionFind uf(n);
    for_grid_pairs(p, part, std::sqrt(ell2), [&](int32_t i, int32_t j) {
        if (host_of[i] != host_of[j]) return;
        if (!((double)dist2_grid(p, i, j) < ell2)) return;
        double ui[3], uj[3];
        const double si = rel(i, ui), sj = rel(j, uj);
        if (!(si > 0 && sj > 0)) return;
        if (!(si <= Vr * sj && sj <= Vr * si)) return;
        const double dot = ui[0] * uj[0] + ui[1] * uj[1] + ui[2] * uj[2];
        if (dot >= cos_op * (si * sj)) uf.unite(i, j);
    });
    for (int64_t i = 0; i < n; ++i) label[i] = -1;
    for (int32_t i : part) label[i] = uf.find(i);
    return 0;
}

// Second stage of the paper's linker: the candidate groups grow through
// relaxed links into untagged outliers, and groups that the relaxed links
// connect strongly enough (f_merge of either group's first-stage size) join.
extern "C" int vr_ref_sub_grow(const vr_ref_particles* p, const int32_t* host_of, int32_t n_hosts,
                               const float* vbar, const float* L, float L_threshold, double gamma_L, double ellx_s,
                               double gamma_x, double Vr, double gamma_V, double cos_op_relaxed, double f_merge,
                               int32_t n_min, const int32_t* label1, int32_t* label_out, int32_t* rounds) {
    if (!valid_particles(p) || !has_vel(p) || (p->n > 0 && (!host_of || !vbar || !L || !label1 || !label_out)))
        return -1;
    if (!(gamma_L >= 1.0) || !(gamma_x >= 1.0) || !(gamma_V >= 1.0) || !(Vr >= 1.0) || n_min < 1 ||
        !(cos_op_relaxed >= -1.0 && cos_op_relaxed <= 1.0) || !(f_merge >= 0) || n_hosts < 0)
        return -1;
    const double ell2 = vr_ref_ell2_grid(gamma_x * ellx_s, p->box, p->grid_bits);
    if (!(ell2 > 0) || !(std::sqrt(ell2) < std::ldexp(1.0, p->grid_bits - 1))) return -1;
    const int64_t n = p->n;
    const double Vr2 = gamma_V * Vr;
    const float Lth2 = (float)((double)L_threshold / gamma_L);
    // first-stage groups of >= n_min members are the tagged candidates
    std::vector<int64_t> size(n, 0);
    for (int64_t i = 0; i < n; ++i)
        if (label1[i] >= 0) {
            if (label1[i] >= n) return -1;
            ++size[label1[i]];
        }
    std::vector<int32_t> tag(n, -1);
    for (int64_t i = 0; i < n; ++i)
        if (label1[i] >= 0 && size[label1[i]] >= n_min) tag[i] = label1[i];
    std::vector<int32_t> part;
    for (int64_t i = 0; i < n; ++i)
        if (host_of[i] >= 0 && host_of[i] < n_hosts && L[i] >= Lth2) part.push_back((int32_t)i);
        else if (tag[i] >= 0) return -1;  // a candidate member must be a relaxed participant
    auto rel = [&](int64_t i, double* u) {
        u[0] = (double)p->vx[i] - (double)vbar[i];
        u[1] = (double)p->vy[i] - (double)vbar[n + i];
        u[2] = (double)p->vz[i] - (double)vbar[2 * n + i];
        return std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    };
    // relaxed links as adjacency lists
    std::unordered_map<int32_t, std::vector<int32_t>> adj;
    std::vector<std::pair<int32_t, int32_t>> edges;
    for_grid_pairs(p, part, std::sqrt(ell2), [&](int32_t i, int32_t j) {
        if (host_of[i] != host_of[j]) return;
        if (!((double)dist2_grid(p, i, j) < ell2)) return;
        double ui[3], uj[3];
        const double si = rel(i, ui), sj = rel(j, uj);
        if (!(si > 0 && sj > 0)) return;
        if (!(si <= Vr2 * sj && sj <= Vr2 * si)) return;
        const double dot = ui[0] * uj[0] + ui[1] * uj[1] + ui[2] * uj[2];
        if (dot >= cos_op_relaxed * (si * sj)) {
            adj[i].push_back(j);
            adj[j].push_back(i);
            edges.push_back({i, j});
        }
    });
    // growth in synchronous rounds
    int32_t nr = 0;
    for (;;) {
        std::vector<std::pair<int32_t, int32_t>> upd;
        for (int32_t u : part) {
            if (tag[u] >= 0) continue;
            auto it = adj.find(u);
            if (it == adj.end()) continue;
            int32_t m = -1;
            for (int32_t t : it->second)
                if (tag[t] >= 0 && (m < 0 || tag[t] < m)) m = tag[t];
            if (m >= 0) upd.push_back({u, m});
        }
        if (upd.empty()) break;
        for (auto& um : upd) tag[um.first] = um.second;
        ++nr;
    }
    if (rounds) *rounds = nr;
    // relaxed links between different groups, per pair of groups
    std::map<std::pair<int32_t, int32_t>, int64_t> conn;
    for (auto& e : edges) {
        const int32_t a = tag[e.first], b = tag[e.second];
        if (a < 0 || b < 0 || a == b) continue;
        ++conn[{std::min(a, b), std::max(a, b)}];
    }
    MinUnionFind uf(n);
    for (auto& kv : conn) {
        const int32_t a = kv.first.first, b = kv.first.second;
        if ((double)kv.second > f_merge * (double)size[a] || (double)kv.second > f_merge * (double)size[b]) uf.unite(a, b);
    }
    // final label: the smallest index among the members of the joined groups
    std::vector<int32_t> low(n, INT32_MAX);
    for (int64_t i = 0; i < n; ++i)
        if (tag[i] >= 0) {
            const int32_t r = uf.find(tag[i]);
            low[r] = std::min(low[r], (int32_t)i);
        }
    for (int64_t i = 0; i < n; ++i) label_out[i] = tag[i] >= 0 ? low[uf.find(tag[i])] : -1;
    return 0;
}

// ---------------------------------------------------------------------------
// Two species (Sec. 2.1, DM+Baryons mode): dark matter links to dark matter
// and to baryons, baryons never link to each other.
extern "C" int vr_ref_fof3d_dm(const vr_ref_particles* p, double ellx, const uint8_t* is_baryon, int32_t* label) {
    if (!valid_particles(p) || (p->n > 0 && (!label || !is_baryon))) return -1;
    const double ell2 = vr_ref_ell2_grid(ellx, p->box, p->grid_bits);
    if (!(ell2 > 0) || !(std::sqrt(ell2) < std::ldexp(1.0, p->grid_bits - 1))) return -1;
    std::vector<int32_t> all(p->n);
    std::iota(all.begin(), all.end(), 0);
    MinUnionFind uf(p->n);
    for_grid_pairs(p, all, std::sqrt(ell2), [&](int32_t i, int32_t j) {
        if (is_baryon[i] && is_baryon[j]) return;
        if ((double)dist2_grid(p, i, j) < ell2) uf.unite(i, j);
    });
    for (int64_t i = 0; i < p->n; ++i) label[i] = uf.find((int32_t)i);
    return 0;
}

// Baryons take the substructure of the nearest dark-matter member of their
// host in phase space (Sec. 2.4, Eq. baryondist read with squared terms).
extern "C" int vr_ref_assign_baryons(const vr_ref_particles* p, int32_t n_hosts, const int32_t* host_offsets,
                                     const int32_t* host_members, const uint8_t* is_baryon, const int32_t* sub,
                                     double ellx, double sigma_v, int32_t* out) {
    if (!valid_particles(p) || !has_vel(p) || !members_ok(p->n, n_hosts, host_offsets, host_members)) return -1;
    if (n_hosts > 0 && (!is_baryon || !sub || !out)) return -1;
    const double ell2 = vr_ref_ell2_grid(ellx, p->box, p->grid_bits);
    if (!(ell2 > 0) || !(sigma_v > 0)) return -1;
    const double sv2 = sigma_v * sigma_v;
    parallel_for(n_hosts, [&](int64_t h) {
        std::vector<int32_t> dm;
        for (int32_t k = host_offsets[h]; k < host_offsets[h + 1]; ++k)
            if (!is_baryon[host_members[k]]) dm.push_back(host_members[k]);
        for (int32_t k = host_offsets[h]; k < host_offsets[h + 1]; ++k) {
            const int32_t i = host_members[k];
            if (!is_baryon[i]) {
                out[i] = sub[i];
                continue;
            }
            double best = std::numeric_limits<double>::infinity();
            int32_t bj = -1;
            for (int32_t j : dm) {
                const double D2 = (double)dist2_grid(p, i, j) / ell2 + dv2_of(p, i, j) / sv2;
                if (D2 < best || (D2 == best && j < bj)) {
                    best = D2;
                    bj = j;
                }
            }
            out[i] = bj >= 0 ? sub[bj] : -1;
        }
    });
    return 0;
}

// ---------------------------------------------------------------------------
// Unbinding (Sec. 2.2, Eq. binding): remove beta_E T + W >= 0, iterate until
// no particle is removed; the group is dissolved below N_min members.
extern "C" int vr_ref_unbind(const vr_ref_particles* p, int32_t n_groups, const int32_t* offsets,
                             const int32_t* members, const vr_ref_unbind_params* up,
                             uint8_t* bound, double* phi, int32_t* iters, double* min_margin) {
    if (!valid_particles(p) || !has_vel(p) || !up) return -1;
    if (!members_ok(p->n, n_groups, offsets, members)) return -1;
    if (n_groups > 0 && (!bound || !phi || !iters)) return -1;
    if (up->n_min < 1 || up->max_iter < 1 || !(up->eps >= 0) || up->n_ref_min < 1) return -1;
    const double unit = p->box / std::ldexp(1.0, p->grid_bits);
    const double eps2 = up->eps * up->eps;
    std::atomic<int> status(0);
    parallel_for(n_groups, [&](int64_t g) {
        std::vector<int32_t> S(members + offsets[g], members + offsets[g + 1]);
        double margin = std::numeric_limits<double>::infinity();
        for (int32_t i : S) { bound[i] = 0; phi[i] = std::numeric_limits<double>::quiet_NaN(); }
        int32_t pass = 0;
        bool done = (int64_t)S.size() < up->n_min;
        while (!done) {
            if (pass >= up->max_iter) { status.store(-5); break; }
            ++pass;
            const int64_t ns = (int64_t)S.size();
            std::vector<double> ph(ns, 0.0);
            // Direct-sum Plummer-softened potential of the current set.
            for (int64_t a = 0; a < ns; ++a) {
                double acc = 0.0;
                for (int64_t b = 0; b < ns; ++b) {
                    if (a == b) continue;
                    const int32_t i = S[a], j = S[b];
                    double dx = (double)min_image(p->qx[i], p->qx[j], p->grid_bits) * unit;
                    double dy = (double)min_image(p->qy[i], p->qy[j], p->grid_bits) * unit;
                    double dz = (double)min_image(p->qz[i], p->qz[j], p->grid_bits) * unit;
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (eps2 == 0.0 && r2 == 0.0) continue;
                    acc += mass_of(p, j) / std::sqrt(r2 + eps2);
                }
                ph[a] = -up->G * acc;
                phi[S[a]] = ph[a];
            }
            // Kinetic reference frame.
            double vref[3] = {0, 0, 0}, mref = 0;
            auto add_ref = [&](int32_t j) {
                double mj = mass_of(p, j);
                mref += mj;
                vref[0] += mj * (double)p->vx[j];
                vref[1] += mj * (double)p->vy[j];
                vref[2] += mj * (double)p->vz[j];
            };
            if (up->frame_type == 1) {
                int64_t pmin = 0;
                for (int64_t a = 1; a < ns; ++a)
                    if (ph[a] < ph[pmin]) pmin = a;  // ties keep the lowest index
                int64_t nref = (int64_t)std::ceil(up->frac_ref * (double)ns);
                nref = std::max<int64_t>(nref, up->n_ref_min);
                nref = std::min<int64_t>(nref, ns);
                std::vector<std::pair<int64_t, int32_t>> ds(ns);
                for (int64_t a = 0; a < ns; ++a) ds[a] = {dist2_grid(p, S[pmin], S[a]), S[a]};
                std::partial_sort(ds.begin(), ds.begin() + nref, ds.end());
                for (int64_t a = 0; a < nref; ++a) add_ref(ds[a].second);
            } else {
                for (int32_t j : S) add_ref(j);
            }
            for (int d = 0; d < 3; ++d) vref[d] /= mref;
            // Energies and the removal set.
            std::vector<int32_t> keep;
            for (int64_t a = 0; a < ns; ++a) {
                const int32_t i = S[a];
                const double mi = mass_of(p, i);
                double dx = (double)p->vx[i] - vref[0];
                double dy = (double)p->vy[i] - vref[1];
                double dz = (double)p->vz[i] - vref[2];
                double T = 0.5 * mi * (dx * dx + dy * dy + dz * dz);
                double W = mi * ph[a];
                double E = up->beta_E * T + W;
                if (W != 0.0) margin = std::min(margin, std::fabs(E) / std::fabs(W));
                if (!(E >= 0.0)) keep.push_back(i);
            }
            if ((int64_t)keep.size() == ns) {
                for (int32_t i : S) bound[i] = 1;
                done = true;
            } else if ((int64_t)keep.size() < up->n_min) {
                done = true;  // dissolved
            } else {
                S.swap(keep);
            }
        }
        iters[g] = pass;
        if (min_margin) min_margin[g] = margin;
    });
    return status.load();
}

// ---------------------------------------------------------------------------
// Normalised ratio L (Sec. 2.2, Eqs. skewgaus and ell): per host, a
// skew-Gaussian fitted to the binned R distribution gives its peak Rbar and
// the dispersion sigma_R of its upper side; L = (R - Rbar) / sigma_R.

extern "C" double vr_ref_ell_cost(int32_t nb, const double* x, const double* w, double c, double* apq) {
    double Sw = 0, Swu = 0, Swv = 0, Swuu = 0, Swvv = 0, Swy = 0, Swuy = 0, Swvy = 0;
    for (int32_t b = 0; b < nb; ++b) {
        const double d = x[b] - c;
        const double u = x[b] < c ? d * d : 0.0;
        const double v = x[b] < c ? 0.0 : d * d;
        const double y = std::log(w[b]);
        Sw += w[b];
        Swu += w[b] * u;
        Swv += w[b] * v;
        Swuu += w[b] * u * u;
        Swvv += w[b] * v * v;
        Swy += w[b] * y;
        Swuy += w[b] * u * y;
        Swvy += w[b] * v * y;
    }
    const double inf = std::numeric_limits<double>::infinity();
    if (!(Swuu > 0) || !(Swvv > 0)) return inf;
    // normal equations of min sum w (y - a + p u + q v)^2; p and q eliminated
    const double den = Sw - Swu * Swu / Swuu - Swv * Swv / Swvv;
    if (!(den > 0)) return inf;
    const double a = (Swy - Swu * Swuy / Swuu - Swv * Swvy / Swvv) / den;
    const double pp = (Swu * a - Swuy) / Swuu;
    const double qq = (Swv * a - Swvy) / Swvv;
    double J = 0;
    for (int32_t b = 0; b < nb; ++b) {
        const double d = x[b] - c;
        const double u = x[b] < c ? d * d : 0.0;
        const double v = x[b] < c ? 0.0 : d * d;
        const double r = std::log(w[b]) - a + pp * u + qq * v;
        J += w[b] * r * r;
    }
    if (apq) {
        apq[0] = a;
        apq[1] = pp;
        apq[2] = qq;
    }
    return J;
}

extern "C" int vr_ref_ell_fit(int64_t n, int32_t n_hosts, const int32_t* host_offsets,
                              const int32_t* host_members, const float* R, const vr_ref_ell_params* ep,
                              double* fit, int32_t* status, int32_t* merge, float* ell) {
    if (!ep || n < 0 || n_hosts < 0) return -1;
    if (!members_ok(n, n_hosts, host_offsets, host_members)) return -1;
    if (n_hosts > 0 && (!R || !fit || !status || !ell)) return -1;
    if (!(ep->width > 0) || ep->nbins < 1 || ep->max_merge < 1 || (ep->max_merge & (ep->max_merge - 1)) ||
        ep->nbins % ep->max_merge || ep->peak_min < 1 || ep->golden_iters < 0)
        return -1;
    const double inv_w = 1.0 / ep->width;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    parallel_for(n_hosts, [&](int64_t h) {
        // fine histogram of the finite values
        std::vector<int64_t> fine(ep->nbins, 0);
        for (int32_t k = host_offsets[h]; k < host_offsets[h + 1]; ++k) {
            const double r = (double)R[host_members[k]];
            if (!std::isfinite(r)) continue;
            const double t = std::floor((r - ep->lo) * inv_w);
            if (t >= 0 && t < ep->nbins) ++fine[(int64_t)t];
        }
        // merge pairs of bins until the fullest holds peak_min
        int32_t g = 1;
        std::vector<int64_t> cnt = fine;
        auto fullest = [](const std::vector<int64_t>& c) {
            int64_t m = 0;
            for (int64_t v : c) m = std::max(m, v);
            return m;
        };
        while (g < ep->max_merge && fullest(cnt) < ep->peak_min) {
            std::vector<int64_t> half(cnt.size() / 2);
            for (size_t b = 0; b < half.size(); ++b) half[b] = cnt[2 * b] + cnt[2 * b + 1];
            cnt.swap(half);
            g *= 2;
        }
        if (merge) merge[h] = g;
        const double step = ep->width * g;
        std::vector<double> x, w;
        int64_t bf = -1, bl = -1;
        for (int64_t b = 0; b < (int64_t)cnt.size(); ++b)
            if (cnt[b] > 0) {
                x.push_back(ep->lo + ((double)b + 0.5) * step);
                w.push_back((double)cnt[b]);
                if (bf < 0) bf = b;
                bl = b;
            }
        double* f = fit + 4 * h;
        if (x.empty()) {
            f[0] = f[1] = f[2] = f[3] = nan;
            status[h] = -1;
        } else {
            const int32_t nb = (int32_t)x.size();
            double best = std::numeric_limits<double>::infinity(), cbest = 0;
            if (nb >= 4)
                for (int64_t b = bf; b <= bl; ++b) {
                    const double c = ep->lo + ((double)b + 0.5) * step;
                    const double J = vr_ref_ell_cost(nb, x.data(), w.data(), c, nullptr);
                    if (J < best) {
                        best = J;
                        cbest = c;
                    }
                }
            bool ok = false;
            if (std::isfinite(best)) {
                // golden-section refinement over one merged bin either side
                const double phi = 0.6180339887498949;
                double lo = cbest - step, hi = cbest + step;
                double x1 = hi - phi * (hi - lo), x2 = lo + phi * (hi - lo);
                double f1 = vr_ref_ell_cost(nb, x.data(), w.data(), x1, nullptr);
                double f2 = vr_ref_ell_cost(nb, x.data(), w.data(), x2, nullptr);
                for (int32_t it = 0; it < ep->golden_iters; ++it) {
                    if (f1 < f2) {
                        hi = x2;
                        x2 = x1;
                        f2 = f1;
                        x1 = hi - phi * (hi - lo);
                        f1 = vr_ref_ell_cost(nb, x.data(), w.data(), x1, nullptr);
                    } else {
                        lo = x1;
                        x1 = x2;
                        f1 = f2;
                        x2 = lo + phi * (hi - lo);
                        f2 = vr_ref_ell_cost(nb, x.data(), w.data(), x2, nullptr);
                    }
                }
                double c = 0.5 * (lo + hi);
                if (!(vr_ref_ell_cost(nb, x.data(), w.data(), c, nullptr) <= best)) c = cbest;
                double apq[3];
                vr_ref_ell_cost(nb, x.data(), w.data(), c, apq);
                if (apq[1] > 0 && apq[2] > 0) {
                    f[0] = c;
                    f[1] = 1.0 / std::sqrt(2.0 * apq[2]);
                    f[2] = std::sqrt(apq[2] / apq[1]);
                    f[3] = std::exp(apq[0]);
                    ok = true;
                }
            }
            if (!ok) {
                // moments of the merged histogram
                double sw = 0, swx = 0, m = 0;
                for (int32_t b = 0; b < nb; ++b) {
                    sw += w[b];
                    swx += w[b] * x[b];
                    m = std::max(m, w[b]);
                }
                const double mean = swx / sw;
                double sxx = 0;
                for (int32_t b = 0; b < nb; ++b) sxx += w[b] * (x[b] - mean) * (x[b] - mean);
                const double sd = std::sqrt(sxx / sw);
                f[0] = mean;
                f[1] = sd > 0 ? sd : step;
                f[2] = 1.0;
                f[3] = m;
            }
            status[h] = ok ? 1 : 0;
        }
        for (int32_t k = host_offsets[h]; k < host_offsets[h + 1]; ++k) {
            const int32_t i = host_members[k];
            ell[i] = (float)(((double)R[i] - f[0]) / f[1]);
        }
    });
    return 0;
}

// Expected L of Gaussian chance outliers above ell_th (the closed form that
// follows Eq. ellsig: a truncated-Gaussian mean).
extern "C" double vr_ref_ell_mean(double ell_th) {
    const double pi = 3.14159265358979323846;
    return std::sqrt(2.0 / pi) * std::exp(-0.5 * ell_th * ell_th) / std::erfc(ell_th / std::sqrt(2.0));
}

// Significance cleaning (Eq. ellsig): members leave in order of smallest L
// until the mean L of the rest reaches Lbar (1 + beta / sqrt(N)).
extern "C" int vr_ref_ell_clean(int64_t n, int32_t n_groups, const int32_t* offsets, const int32_t* members,
                                const float* ell, double ell_th, double beta, int32_t n_min, int32_t* label,
                                int32_t* removed) {
    if (n < 0 || n_groups < 0 || n_min < 1) return -1;
    if (!members_ok(n, n_groups, offsets, members)) return -1;
    if (n_groups > 0 && (!ell || !label)) return -1;
    const double Lbar = vr_ref_ell_mean(ell_th);
    parallel_for(n_groups, [&](int64_t g) {
        std::vector<int32_t> S(members + offsets[g], members + offsets[g + 1]);
        std::vector<int32_t> order = S;
        std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return ell[a] < ell[b] || (ell[a] == ell[b] && a < b);
        });
        const int64_t N = (int64_t)order.size();
        double sum = 0;
        for (int32_t i : order) sum += (double)ell[i];
        int64_t k = 0;
        for (;;) {
            const int64_t m = N - k;
            if (m < n_min) {
                k = N;  // dissolved
                break;
            }
            if (sum / (double)m >= Lbar * (1.0 + beta / std::sqrt((double)m))) break;
            sum -= (double)ell[order[k]];
            ++k;
        }
        // S is ascending: the kept members in index order start at the root
        std::vector<char> gone(N, 0);
        for (int64_t r = 0; r < k; ++r)
            gone[std::lower_bound(S.begin(), S.end(), order[r]) - S.begin()] = 1;
        int32_t root = -1;
        for (int64_t a = 0; a < N; ++a) {
            if (gone[a]) {
                label[S[a]] = -1;
            } else {
                if (root < 0) root = S[a];
                label[S[a]] = root;
            }
        }
        if (removed) removed[g] = (int32_t)k;
    });
    return 0;
}
