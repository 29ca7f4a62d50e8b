// vr_kd.h -- level-synchronous KD trees over the members of many hosts at
// once (shared by the entropy cells and the neighbour search).
#pragma once
#include "vr_internal.h"

namespace vr {

struct KdNode {
    int host, start, end, slot;  // slot: index among the active nodes of its level, -1 otherwise
    int lo[3], hi[3];            // region (integer, inclusive) used for face probes and volumes
    int bmin[3], bmax[3];        // bounding box of the members
    int dim, t, left, right;     // split dimension (-1 for a leaf) and value; children
};

// Members of the hosts.  "Element" e is a position in the caller's host
// member list (host h owns [off[h], off[h+1]) and its elements are in
// ascending particle-index order); the tree orders them into positions.
struct Elems {
    int* u[3];      // coordinates unwrapped relative to the host's first member
    int* gidx;      // particle index
    int* eid;       // element id
    float* mass;    // null for uniform mass
};

enum KdMode { KD_MIN_ENTROPY = 0, KD_MAX_ENTROPY = 1, KD_WIDEST = 2 };

struct KdTree {
    KdNode* nodes = nullptr;
    int* leaves = nullptr;     // node ids of the leaves
    int n_leaves = 0;
    int* seg_node = nullptr;   // position -> leaf node id
    int* leaf_min = nullptr;   // node id -> smallest particle index of the leaf
    Elems F{};                 // members by position (leaf segments are contiguous)
    int* elem_u[3] = {nullptr, nullptr, nullptr};  // coordinates by element id
    int* elem_host = nullptr;  // host by element id (= by position: hosts keep their ranges)
    int use_mass = 0;
};

// Builds one tree per host.  A node with more than ncell[h] members is split
// at the member of rank floor(n/2) in (coordinate, particle index) order of
// the dimension chosen by `mode`; the left child takes the members before it.
// The root of host h has node id h.
int kd_build(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts, const int32_t* host_offsets,
             const int32_t* host_members, const std::vector<int32_t>& off, const std::vector<int>& ncell,
             int mode, int nbins, KdTree& tree, hipStream_t st);

// host_offsets copied to the host, with validation (every host >= min_size).
int read_host_offsets(vr_ctx* ctx, int32_t n_hosts, const int32_t* host_offsets, int64_t n, int64_t min_size,
                      std::vector<int32_t>& off, hipStream_t st);

}  // namespace vr
