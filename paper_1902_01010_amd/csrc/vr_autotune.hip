// vr_autotune.hip -- picks the launch-shape knobs of a context by timing the
// library's own entry points on synthetic device workloads, and keeps the
// choice in a small JSON cache keyed by the GPU architecture.
//
// Knobs never change integer results (FP64 sums only through their order):
//   unbind_tile, unbind_jchunk, unbind_bpc   persistent potential schedule
//   unbind_wide                              size class of the group kernel
//   knn_leaf, xcd_chunk                      neighbour-search tree and order
#include "vr_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <sstream>

namespace vr {
namespace {

// Counter-based uniform and normal variates (SplitMix64 finaliser on
// seed + index; Box-Muller for the normals).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double unif(uint64_t seed, uint64_t i, int k) {
    return ((double)(mix64(seed ^ (i * 8 + k) * 0xD1B54A32D192ED03ull) >> 11) + 0.5) * 0x1.0p-53;
}
__device__ __forceinline__ double gauss(uint64_t seed, uint64_t i, int k) {
    const double u1 = unif(seed, i, 2 * k), u2 = unif(seed, i, 2 * k + 1);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Particles of group g (members off[g] .. off[g+1]-1, contiguous): a
// Gaussian blob of radius rad(g) grid units around a random centre, and
// Gaussian velocities of dispersion sig.
__global__ void k_at_blobs(int ng, const int32_t* __restrict__ off, int gb, double rad0, double sig, uint64_t seed,
                           uint32_t* __restrict__ qx, uint32_t* __restrict__ qy, uint32_t* __restrict__ qz,
                           float* __restrict__ vx, float* __restrict__ vy, float* __restrict__ vz,
                           int32_t* __restrict__ mem) {
    const int g = blockIdx.x;
    if (g >= ng) return;
    const int s = off[g], e = off[g + 1];
    const double size = (double)(1u << gb);
    const double cx = unif(seed, g, 0) * size, cy = unif(seed, g, 1) * size, cz = unif(seed, g, 2) * size;
    const double rad = rad0 * cbrt((double)(e - s) / 1000.0);
    const uint32_t mask = (1u << gb) - 1u;
    for (int i = s + threadIdx.x; i < e; i += blockDim.x) {
        const uint64_t k = (uint64_t)i + 1000003ull * (uint64_t)g;
        const double x = cx + rad * gauss(seed + 1, k, 0), y = cy + rad * gauss(seed + 1, k, 1),
                     z = cz + rad * gauss(seed + 1, k, 2);
        qx[i] = (uint32_t)(int64_t)floor(x) & mask;
        qy[i] = (uint32_t)(int64_t)floor(y) & mask;
        qz[i] = (uint32_t)(int64_t)floor(z) & mask;
        vx[i] = (float)(sig * gauss(seed + 2, k, 0));
        vy[i] = (float)(sig * gauss(seed + 2, k, 1));
        vz[i] = (float)(sig * gauss(seed + 2, k, 2));
        mem[i] = i;
    }
}

// Particles of host g (members off[g] .. off[g+1]-1, contiguous) as a
// cusped halo: a Hernquist profile (density ~ r^-1 inside the scale radius,
// like NFW) with scale a = r200 / 10, cut at r200, around a random centre.
// r200 is that of N particles at 200 times the critical density when the
// mean spacing is sp grid units (matter density 0.3 critical); velocities
// Gaussian with dispersion 300 (N / 1e5)^(1/3).
__global__ void k_at_halos(int ng, const int32_t* __restrict__ off, int gb, double sp, uint64_t seed,
                           uint32_t* __restrict__ qx, uint32_t* __restrict__ qy, uint32_t* __restrict__ qz,
                           float* __restrict__ vx, float* __restrict__ vy, float* __restrict__ vz,
                           int32_t* __restrict__ mem) {
    const int g = blockIdx.x;
    if (g >= ng) return;
    const int s = off[g], e = off[g + 1];
    const double size = (double)(1u << gb), nh = (double)(e - s);
    const double cx = unif(seed, g, 0) * size, cy = unif(seed, g, 1) * size, cz = unif(seed, g, 2) * size;
    const double r200 = sp * cbrt(nh * 0.3 * 3.0 / (4.0 * 3.141592653589793 * 200.0));
    const double a = 0.1 * r200, smax = 10.0 / 11.0;
    const double sig = 300.0 * cbrt(nh / 1e5);
    const uint32_t mask = (1u << gb) - 1u;
    for (int i = s + threadIdx.x; i < e; i += blockDim.x) {
        const uint64_t k = (uint64_t)i + 1000003ull * (uint64_t)g;
        // enclosed-mass fraction u -> radius: (r / (r + a))^2 = u (r200 / (r200 + a))^2
        const double t = sqrt(unif(seed + 1, k, 0)) * smax, r = a * t / (1.0 - t);
        const double cth = 2.0 * unif(seed + 1, k, 1) - 1.0, ph = 6.283185307179586 * unif(seed + 1, k, 2);
        const double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
        const double x = cx + r * sth * cos(ph), y = cy + r * sth * sin(ph), z = cz + r * cth;
        qx[i] = (uint32_t)(int64_t)floor(x) & mask;
        qy[i] = (uint32_t)(int64_t)floor(y) & mask;
        qz[i] = (uint32_t)(int64_t)floor(z) & mask;
        vx[i] = (float)(sig * gauss(seed + 2, k, 0));
        vy[i] = (float)(sig * gauss(seed + 2, k, 1));
        vz[i] = (float)(sig * gauss(seed + 2, k, 2));
        mem[i] = i;
    }
}

struct Knobs {
    int unbind_tile = 256, unbind_jchunk = 4096, unbind_bpc = 0, unbind_wide = 4096, knn_leaf = 64, xcd_chunk = 64;
};

bool read_cache(const char* path, const char* arch, Knobs& k) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    if (s.find(std::string("\"arch\": \"") + arch + "\"") == std::string::npos) return false;
    auto get = [&](const char* key, int& v) {
        const std::string pat = std::string("\"") + key + "\": ";
        const size_t p = s.find(pat);
        if (p == std::string::npos) return false;
        v = std::atoi(s.c_str() + p + pat.size());
        return true;
    };
    return get("unbind_tile", k.unbind_tile) && get("unbind_jchunk", k.unbind_jchunk) &&
           get("unbind_bpc", k.unbind_bpc) && get("unbind_wide", k.unbind_wide) && get("knn_leaf", k.knn_leaf) &&
           get("xcd_chunk", k.xcd_chunk);
}

void apply(vr_ctx* ctx, const Knobs& k) {
    ctx->tuned_tile = k.unbind_tile;
    ctx->unbind_jchunk = k.unbind_jchunk;
    ctx->unbind_bpc = k.unbind_bpc;
    ctx->unbind_wide = k.unbind_wide;
    ctx->knn_leaf = k.knn_leaf;
    ctx->xcd_chunk = k.xcd_chunk;
}

struct DevBufs {
    std::vector<void*> ptrs;
    ~DevBufs() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <class T>
    T* get(size_t n) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return static_cast<T*>(p);
    }
};

}  // namespace
}  // namespace vr

using namespace vr;

extern "C" int vr_autotune(vr_ctx* ctx, const char* cache_path, int force) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipDeviceProp_t prop;
    VR_HIP(ctx, hipGetDeviceProperties(&prop, ctx->device));
    char arch[64];
    std::snprintf(arch, sizeof arch, "%.6s", prop.gcnArchName);
    Knobs best;
    if (!force && read_cache(cache_path, arch, best)) {
        apply(ctx, best);
        return VR_OK;
    }
    const int gb = 21;
    hipStream_t st = nullptr;
    VR_HIP(ctx, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } guard{st};
    hipEvent_t e0, e1;
    VR_HIP(ctx, hipEventCreate(&e0));
    VR_HIP(ctx, hipEventCreate(&e1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } eg{e0, e1};
    DevBufs mem;
    std::ostringstream log;

    // ---- unbinding: heavy-tailed group sizes 32 .. 32768 ------------------
    std::vector<int32_t> off{0};
    for (int k = 15; k >= 5; --k) {
        const int count = std::max(1, (1 << (15 - k)) / 2);
        for (int c = 0; c < count; ++c) off.push_back(off.back() + (1 << k));
    }
    const int ng = (int)off.size() - 1;
    const int64_t nu = off.back();
    uint32_t *qx = mem.get<uint32_t>(nu), *qy = mem.get<uint32_t>(nu), *qz = mem.get<uint32_t>(nu);
    float *vx = mem.get<float>(nu), *vy = mem.get<float>(nu), *vz = mem.get<float>(nu);
    int32_t *mb = mem.get<int32_t>(nu), *offd = mem.get<int32_t>(ng + 1), *iters = mem.get<int32_t>(ng);
    uint8_t* bound = mem.get<uint8_t>(nu);
    double* phi = mem.get<double>(nu);
    if (!qx || !qy || !qz || !vx || !vy || !vz || !mb || !offd || !iters || !bound || !phi)
        return set_err(ctx, VR_ERR_OUT_OF_MEMORY, "autotune workload allocation failed");
    VR_HIP(ctx, hipMemcpyAsync(offd, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_at_blobs, dim3(ng), dim3(256), 0, st, ng, offd, gb, 2000.0, 0.0, (uint64_t)77, qx, qy, qz,
                       vx, vy, vz, mb);
    VR_LAUNCH_CHECK(ctx);
    vr_particles P{};
    P.n = nu;
    P.qx = qx; P.qy = qy; P.qz = qz;
    P.vx = vx; P.vy = vy; P.vz = vz;
    P.mass = nullptr;
    P.mass_value = 1.0;
    P.box = 1.0;
    P.grid_bits = gb;
    vr_unbind_params up{};
    up.G = 1.0; up.eps = 1e-4; up.beta_E = 0.95; up.frac_ref = 0.1; up.n_min = 20; up.n_ref_min = 10;
    up.frame_type = 1; up.max_iter = 100; up.persistent = 1; up.tile = 0;
    const int saved_timing = ctx->timing;
    ctx->timing = 0;
    auto time_unbind = [&](float* ms) -> int {
        float bestms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            VR_HIP(ctx, hipEventRecord(e0, st));
            int rc = vr_unbind(ctx, &P, ng, offd, mb, &up, bound, phi, iters, st);
            if (rc) return rc;
            VR_HIP(ctx, hipEventRecord(e1, st));
            VR_HIP(ctx, hipEventSynchronize(e1));
            float t = 0;
            VR_HIP(ctx, hipEventElapsedTime(&t, e0, e1));
            if (rep > 0) bestms = std::min(bestms, t);
        }
        *ms = bestms;
        return VR_OK;
    };
    float best_ub = 1e30f;
    ctx->unbind_wide = best.unbind_wide;  // the default size class while the schedule is swept
    const int tiles[] = {64, 128, 256, 512, 1024};
    const int jchunks[] = {1024, 4096, 16384};
    const int bpcs[] = {0, 1, 2, 4};
    for (int t : tiles)
        for (int j : jchunks)
            for (int b : bpcs) {
                ctx->tuned_tile = t;
                ctx->unbind_jchunk = j;
                ctx->unbind_bpc = b;
                float ms = 0;
                int rc = time_unbind(&ms);
                if (rc) { ctx->timing = saved_timing; return rc; }
                log << "    {\"tile\": " << t << ", \"jchunk\": " << j << ", \"bpc\": " << b << ", \"ms\": " << ms
                    << "},\n";
                if (ms < best_ub) {
                    best_ub = ms;
                    best.unbind_tile = t;
                    best.unbind_jchunk = j;
                    best.unbind_bpc = b;
                }
            }
    apply(ctx, best);
    // then the size class at that schedule: the group kernel's 1024-thread
    // form for the leading groups from 1024 members up, ..., or for none
    std::ostringstream wlog;
    const int wides[] = {1024, 2048, 4096, 8192, 16384, 1 << 30};
    float best_w = 1e30f;
    for (int wm : wides) {
        ctx->unbind_wide = wm;
        float ms = 0;
        int rc = time_unbind(&ms);
        if (rc) { ctx->timing = saved_timing; return rc; }
        wlog << "    {\"wide\": " << wm << ", \"ms\": " << ms << "},\n";
        if (ms < best_w) {
            best_w = ms;
            best.unbind_wide = wm;
        }
    }
    apply(ctx, best);

    // ---- neighbour search: 2000 hosts, dN/dlnN ~ N^-0.9 on [256, 2^21] -----
    // Sizes at the mid-quantiles of that distribution (6.6 M members, largest
    // 1.07 M): the searched hosts of a 256^3 box, whose largest hosts set the
    // best leaf size.
    const int nh = 2000;
    std::vector<int32_t> hoff(nh + 1);
    hoff[0] = 0;
    {
        const double sl = 0.9, lo = std::pow(256.0, -sl), hi = std::pow(2097152.0, -sl);
        for (int h = 0; h < nh; ++h) {
            const double q = (h + 0.5) / nh;
            hoff[h + 1] = hoff[h] + (int32_t)std::floor(std::pow(lo - q * (lo - hi), -1.0 / sl));
        }
    }
    const int64_t nk = hoff[nh];
    uint32_t *kx = mem.get<uint32_t>(nk), *ky = mem.get<uint32_t>(nk), *kz = mem.get<uint32_t>(nk);
    float *kvx = mem.get<float>(nk), *kvy = mem.get<float>(nk), *kvz = mem.get<float>(nk);
    int32_t *kmem = mem.get<int32_t>(nk), *khoff = mem.get<int32_t>(nh + 1), *cof = mem.get<int32_t>(nk);
    float *vbar = mem.get<float>(3 * nk), *sig = mem.get<float>(6 * nk), *rho = mem.get<float>(nk),
          *R = mem.get<float>(nk);
    if (!kx || !ky || !kz || !kvx || !kvy || !kvz || !kmem || !khoff || !cof || !vbar || !sig || !rho || !R) {
        ctx->timing = saved_timing;
        return set_err(ctx, VR_ERR_OUT_OF_MEMORY, "autotune workload allocation failed");
    }
    VR_HIP(ctx, hipMemcpyAsync(khoff, hoff.data(), hoff.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_at_halos, dim3(nh), dim3(256), 0, st, nh, khoff, gb, (double)(1u << gb) / 256.0,
                       (uint64_t)91, kx, ky, kz, kvx, kvy, kvz, kmem);
    VR_LAUNCH_CHECK(ctx);
    vr_particles K{};
    K.n = nk;
    K.qx = kx; K.qy = ky; K.qz = kz;
    K.vx = kvx; K.vy = kvy; K.vz = kvz;
    K.mass = nullptr;
    K.mass_value = 1.0;
    K.box = 1.0;
    K.grid_bits = gb;
    vr_cell_params cp{0.01, 100, 8, 16, 0};
    int64_t ncells = 0;
    int rc = vr_cell_moments(ctx, &K, nh, khoff, kmem, &cp, vbar, sig, rho, cof, 0, nullptr, &ncells, st);
    if (rc) { ctx->timing = saved_timing; return rc; }
    float best_knn = 1e30f;
    std::ostringstream klog;
    struct KnnRun { int leaf, xchunk; float ms; };
    std::vector<KnnRun> kruns;
    const int leaves[] = {64, 96, 128, 192, 256};
    const int xchunks[] = {0, 16, 64, 256};
    for (int L : leaves)
        for (int X : xchunks) {
            ctx->knn_leaf = L;
            ctx->xcd_chunk = X;
            float bestms = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                VR_HIP(ctx, hipEventRecord(e0, st));
                rc = vr_local_vdensity(ctx, &K, nh, khoff, kmem, vbar, sig, 32, 8, nullptr, 0, R, st);
                if (rc) { ctx->timing = saved_timing; return rc; }
                VR_HIP(ctx, hipEventRecord(e1, st));
                VR_HIP(ctx, hipEventSynchronize(e1));
                float t = 0;
                VR_HIP(ctx, hipEventElapsedTime(&t, e0, e1));
                if (rep > 0) bestms = std::min(bestms, t);
            }
            klog << "    {\"leaf\": " << L << ", \"xcd_chunk\": " << X << ", \"ms\": " << bestms << "},\n";
            kruns.push_back({L, X, bestms});
            best_knn = std::min(best_knn, bestms);
        }
    // among the settings within 1% of the fastest (timing noise), the longest
    // XCD runs: the same speed with the fewest neighbour leaves fetched by
    // several XCDs
    {
        const KnnRun* pick = nullptr;
        for (const KnnRun& r : kruns)
            if (r.ms <= best_knn * 1.01f &&
                (!pick || r.xchunk > pick->xchunk || (r.xchunk == pick->xchunk && r.ms < pick->ms)))
                pick = &r;
        if (pick) {
            best.knn_leaf = pick->leaf;
            best.xcd_chunk = pick->xchunk;
        }
    }
    ctx->timing = saved_timing;
    apply(ctx, best);
    if (cache_path) {
        std::ofstream f(cache_path);
        if (!f) return set_err(ctx, VR_ERR_INVALID_ARG, "cannot write %s", cache_path);
        std::string a = log.str(), b = klog.str(), c = wlog.str();
        if (!a.empty()) a.erase(a.size() - 2, 1);  // trailing comma
        if (!b.empty()) b.erase(b.size() - 2, 1);
        if (!c.empty()) c.erase(c.size() - 2, 1);
        f << "{\n  \"arch\": \"" << arch << "\",\n"
          << "  \"unbind_tile\": " << best.unbind_tile << ",\n  \"unbind_jchunk\": " << best.unbind_jchunk
          << ",\n  \"unbind_bpc\": " << best.unbind_bpc << ",\n  \"unbind_wide\": " << best.unbind_wide
          << ",\n  \"knn_leaf\": " << best.knn_leaf
          << ",\n  \"xcd_chunk\": " << best.xcd_chunk << ",\n"
          << "  \"unbind_workload\": \"" << ng << " groups, " << nu << " particles, sizes 32..32768\",\n"
          << "  \"knn_workload\": \"" << nh << " Hernquist hosts, dN/dlnN ~ N^-0.9 on [256, 2^21], " << nk
          << " members, n_se 32, n_v 8\",\n"
          << "  \"unbind_sweep\": [\n" << a << "  ],\n  \"unbind_wide_sweep\": [\n" << c
          << "  ],\n  \"knn_sweep\": [\n" << b << "  ]\n}\n";
    }
    return VR_OK;
}
