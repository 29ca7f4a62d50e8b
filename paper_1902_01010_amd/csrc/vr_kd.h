// vr_kd.h -- level-synchronous KD trees over the members of many hosts at
// once (shared by the entropy cells and the neighbour search).
#pragma once
#include "vr_internal.h"

namespace vr {

struct KdNode {
    int host, start, end, buf;
    int lo[3], hi[3];      // region (integer, inclusive) used for face probes and volumes
    int bmin[3], bmax[3];  // bounding box of the members
    int dim, t, left, right;
};

// Host members in structure-of-arrays form, unwrapped relative to the host's
// first member.  Positions are host_offsets positions.
struct Elems {
    int* u[3];
    int* gidx;
    float* mass;
};

enum KdMode { KD_MIN_ENTROPY = 0, KD_MAX_ENTROPY = 1, KD_WIDEST = 2 };

struct KdTree {
    KdNode* nodes = nullptr;
    int* leaves = nullptr;   // node ids of the leaves
    int n_leaves = 0;
    Elems F{};               // members in final (leaf-contiguous) order
    int use_mass = 0;
};

// Builds one tree per host: nodes with more than ncell[h] members are split
// at the median (rank floor(n/2) in (coordinate, index) order) of the
// dimension chosen by `mode`.  Root node of host h has id h.  Uses workspace
// slots A0..A8, B0..B5 and FLAG.
int kd_build(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts, const int32_t* host_offsets,
             const int32_t* host_members, const std::vector<int32_t>& off, const std::vector<int>& ncell,
             int mode, int nbins, KdTree& tree, hipStream_t st);

// host_offsets copied to the host, with validation (every host >= min_size).
int read_host_offsets(vr_ctx* ctx, int32_t n_hosts, const int32_t* host_offsets, int64_t n, int64_t min_size,
                      std::vector<int32_t>& off, hipStream_t st);

}  // namespace vr
