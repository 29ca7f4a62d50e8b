// vr_internal.h -- shared internals of libvr (context, workspace, errors,
// device helpers).  gfx950 only: wave64, 160 KiB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/vr.h"

#define VR_WAVE 64

struct vr_buf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

struct vr_timer {
    std::string name;
    std::vector<hipEvent_t> pending;  // start/stop pairs not yet read
    std::vector<double> pending_work;
    int64_t launches = 0;
    double ms = 0.0;
    double work = 0.0;
};

struct vr_ctx {
    int timing = 0;
    std::vector<vr_timer> timers;
    std::vector<hipEvent_t> event_pool;
    int device = 0;
    int num_cus = 256;
    size_t max_ws = 0;      // 0 = no cap
    size_t held = 0;        // bytes currently held by slots
    std::vector<vr_buf> slots;
    std::string err;
    // host-pinned scalars for counts returned by syncing calls
    int64_t* pinned = nullptr;
    // host-pinned staging for copy_to_host (64 KB from creation, grown on demand)
    void* stage = nullptr;
    size_t stage_bytes = 0;
    // host-pinned staging for uploads, and the event after the last upload
    // that read it (upload_begin waits for that event before reusing it)
    void* up = nullptr;
    size_t up_bytes = 0;
    hipEvent_t up_event = nullptr;
    bool up_pending = false;
    int tuned_tile = 0;     // potential j-tile picked by the autotuner (0 = default)
    int knn_leaf = 64;      // members per leaf of the neighbour-search tree
    int unbind_jchunk = 4096;
    int unbind_bpc = 0;     // workgroups per CU of the persistent potential kernel (0 = occupancy limit)
    int unbind_wide = 4096; // members from which a leading group takes the 1024-thread group kernel
    int xcd_chunk = 64;     // consecutive workgroups per XCD in the neighbour sweeps (0 = hardware order)
    // while timing: candidate distances of the neighbour search (device counter)
    unsigned long long* knn_cand = nullptr;
    // the presorted member lists of the last KD build (workspace slot
    // WS_KD_PRE), kept for the next build over the same members: their
    // content hash, sizes and storage
    unsigned long long kd_pre_hash = 0;
    int64_t kd_pre_m = -1;
    int kd_pre_bits = 0;
    void* kd_pre_ptr = nullptr;
    // graph of the persistent unbinding passes, reused while its arguments match
    void* cap_stream = nullptr;
    void* ub_graph = nullptr;
    void* ub_exec = nullptr;
    std::string ub_key;
};

namespace vr {

// Workspace slot identifiers: every call takes its temporaries from fixed
// slots, grown on demand and reused across calls.
enum Slot {
    WS_SORT_KEYS_A, WS_SORT_KEYS_B, WS_SORT_VALS_A, WS_SORT_VALS_B, WS_SORT_HIST,
    WS_SCAN_TMP, WS_SCAN_TMP2,
    WS_A0, WS_A1, WS_A2, WS_A3, WS_A4, WS_A5, WS_A6, WS_A7, WS_A8, WS_A9,
    WS_B0, WS_B1, WS_B2, WS_B3, WS_B4, WS_B5, WS_B6, WS_B7, WS_B8, WS_B9,
    WS_C0, WS_C1, WS_C2, WS_C3, WS_C4, WS_C5, WS_C6, WS_C7, WS_C8, WS_C9,
    WS_D0, WS_D1, WS_D2, WS_D3, WS_D4, WS_D5, WS_D6, WS_D7, WS_D8, WS_D9,
    WS_FLAG, WS_FLAG2, WS_KD, WS_KD_HIST, WS_KD_S, WS_KD_PRE,
    WS_NSLOTS
};

// Carves aligned sub-arrays out of one workspace slot: call add() for every
// array (first pass sizes, second pass assigns), then alloc().
struct Carve {
    size_t bytes = 0;
    char* base = nullptr;
    template <class T>
    T* add(size_t count) {
        size_t off = bytes;
        bytes += (count * sizeof(T) + 255) & ~size_t(255);
        return base ? reinterpret_cast<T*>(base + off) : nullptr;
    }
};

int set_err(vr_ctx* ctx, int code, const char* fmt, ...);

// Grow-only workspace slot; returns nullptr (and sets the error) on failure.
void* ws(vr_ctx* ctx, int slot, size_t bytes);

template <class T>
inline T* wsT(vr_ctx* ctx, int slot, size_t count) {
    return static_cast<T*>(ws(ctx, slot, count * sizeof(T) + 16));
}

#define VR_HIP(ctx, call)                                                              \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::vr::set_err(ctx, VR_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// The last launch (or an earlier unchecked runtime call) failed; the message
// names the line that noticed it.
#define VR_LAUNCH_CHECK(ctx)                                                                       \
    do {                                                                                           \
        hipError_t e_ = hipGetLastError();                                                         \
        if (e_ != hipSuccess)                                                                      \
            return ::vr::set_err(ctx, VR_ERR_HIP, "launch check at %s:%d: %s", __FILE__, __LINE__, \
                                 hipGetErrorString(e_));                                           \
    } while (0)

#define VR_WS(ptr, ctx, T, slot, count)                       \
    T* ptr = ::vr::wsT<T>(ctx, slot, (size_t)(count));        \
    if (!ptr) return VR_ERR_OUT_OF_MEMORY;

inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

// Kernel timing (measurement support).  When ctx->timing is set, launches
// wrapped in VR_TIMED are bracketed by events on their stream and their
// durations and algorithmic work are accumulated under `name`.
hipEvent_t timer_event(vr_ctx* ctx);
void timer_push(vr_ctx* ctx, const char* name, hipEvent_t e0, hipEvent_t e1, double work);

#define VR_TIMED(ctx, name, st, work, ...)                                   \
    do {                                                                     \
        hipEvent_t e0_ = nullptr, e1_ = nullptr;                             \
        if ((ctx)->timing) {                                                 \
            e0_ = ::vr::timer_event(ctx);                                    \
            (void)hipEventRecord(e0_, st);                                   \
        }                                                                    \
        __VA_ARGS__;                                                         \
        if ((ctx)->timing) {                                                 \
            e1_ = ::vr::timer_event(ctx);                                    \
            (void)hipEventRecord(e1_, st);                                   \
            ::vr::timer_push(ctx, name, e0_, e1_, (double)(work));           \
        }                                                                    \
    } while (0)

// Records the device's address of the fixed scratch array of
// vr_relabel_min_noalloc (vr_species.hip); vr_create calls it with the
// device current.
int noalloc_scratch_init(int device);

// Drops the cached unbinding graph (vr_unbind.hip).
void unbind_release(vr_ctx* ctx);

// Host-side validation shared by the entry points.
int check_particles(vr_ctx* ctx, const vr_particles* p, bool need_vel);
int check_hosts(vr_ctx* ctx, int32_t n_hosts, const int32_t* off, const int32_t* mem);

// ---- device-wide primitives (vr_prims.hip) --------------------------------
// Exclusive prefix sum of n uint32 values (in may equal out).  Returns total
// through *total_dev (device pointer, may be null).
int scan_u32(vr_ctx* ctx, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev,
             hipStream_t s);
// Exclusive prefix sum of n bytes into n uint32 values (in and out distinct).
int scan_u8(vr_ctx* ctx, const uint8_t* in, uint32_t* out, int64_t n, hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on key bits [0, bits).  Keys
// and values are sorted in place (the buffers are overwritten).
int sort_pairs_u32(vr_ctx* ctx, uint32_t* keys, uint32_t* vals, int64_t n, int bits,
                   hipStream_t s);
int sort_pairs_u64(vr_ctx* ctx, uint64_t* keys, uint32_t* vals, int64_t n, int bits,
                   hipStream_t s);
// Where a producer should write the unsorted pairs so that the sort into
// (keys, vals) ends there without a final copy: the sort's own alternate
// buffers when it takes an odd number of 8-bit passes, else keys and vals.
// The pairs are then sorted by sort_pairs_*_from(kin, vin -> keys, vals)
// with the same n, bits and first_bit, and nothing may take workspace in
// between.  The _from sort orders by key bits [first_bit, bits); lower bits
// travel with their key (stable).
int sort_input_u64(vr_ctx* ctx, uint64_t* keys, uint32_t* vals, int64_t n, int bits, uint64_t** kin,
                   uint32_t** vin, int first_bit = 0);
int sort_pairs_u64_from(vr_ctx* ctx, uint64_t* kin, uint32_t* vin, uint64_t* keys, uint32_t* vals, int64_t n,
                        int bits, hipStream_t s, int first_bit = 0);
// The same for 32-bit keys.  The sort may take fewer pairs than the buffers
// were placed for (a producer that compacts): n of sort_input is then an
// upper bound of the sort's n, with the same bits.
int sort_input_u32(vr_ctx* ctx, uint32_t* keys, uint32_t* vals, int64_t n, int bits, uint32_t** kin,
                   uint32_t** vin);
int sort_pairs_u32_from(vr_ctx* ctx, uint32_t* kin, uint32_t* vin, uint32_t* keys, uint32_t* vals, int64_t n,
                        int bits, hipStream_t s);
// Fill helpers (kernels, never memset nodes, so they are safe to capture).
int fill_i32(vr_ctx* ctx, int32_t* p, int32_t v, int64_t n, hipStream_t s);
int fill_u32(vr_ctx* ctx, uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
int iota_u32(vr_ctx* ctx, uint32_t* p, int64_t n, hipStream_t s);
// Copy one device scalar to the host and wait.
int read_back(vr_ctx* ctx, const void* dev, void* host, size_t bytes, hipStream_t s);
// Copy bytes of device memory to (pageable) host memory through the
// context's pinned staging buffer, waiting for the stream; the buffer grows
// (hipHostMalloc) only for reads beyond its size.
int copy_to_host(vr_ctx* ctx, void* host, const void* dev, size_t bytes, hipStream_t s);
// Uploads without a sync: upload_begin returns the context's pinned upload
// buffer with room for bytes (null on failure, error set), once no earlier
// upload still reads it; the caller fills it, enqueues its host-to-device
// copies from it, and calls upload_end, which records the event they end at.
void* upload_begin(vr_ctx* ctx, size_t bytes);
int upload_end(vr_ctx* ctx, hipStream_t s);

// ---- device helpers --------------------------------------------------------
__device__ __forceinline__ int min_image(int d, int gb) {
    // ((d + half) mod size) - half for a power-of-two size
    const int half = 1 << (gb - 1);
    const int mask = (1 << gb) - 1;
    return ((d + half) & mask) - half;
}

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// The dispatcher deals workgroups to the eight XCDs in turn.  This renumbers
// workgroup b of nb so that each XCD takes runs of `chunk` consecutive
// workgroups: spatially neighbouring work shares one XCD's L2, while the
// runs still rotate over the XCDs, which keeps their loads balanced.  A
// bijection of [0, nb); chunk = 0 leaves the numbering alone.
__device__ __forceinline__ unsigned xcd_swizzle(unsigned b, unsigned nb, unsigned chunk) {
    if (chunk == 0) return b;
    const unsigned span = 8u * chunk;
    const unsigned full = nb - nb % span;
    if (b >= full) return b;
    const unsigned s = b / span, w = b % span;
    return s * span + (w & 7u) * chunk + (w >> 3);
}

// Symmetric 3x3 matrix [[a, d, e], [d, b, f], [e, f, c]]: its adjugate (the
// transposed cofactor matrix, itself symmetric) as (xx, yy, zz, xy, xz, yz),
// and its determinant by expansion along the first row.  With float entries
// promoted to double, each two-term cofactor is one rounding of exact
// products.
struct Sym3Adj {
    double xx, yy, zz, xy, xz, yz, det;
};
__device__ __forceinline__ Sym3Adj sym3_adjugate(double a, double b, double c, double d, double e, double f) {
    Sym3Adj r;
    r.xx = b * c - f * f;
    r.yy = a * c - e * e;
    r.zz = a * b - d * d;
    r.xy = e * f - d * c;
    r.xz = d * f - b * e;
    r.yz = d * e - a * f;
    r.det = a * r.xx + d * r.xy + e * r.xz;
    return r;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const unsigned l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

}  // namespace vr
