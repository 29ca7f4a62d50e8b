/*
 * vr.h -- C ABI of libvr, the MI355X (gfx950) hot path of the VELOCIraptor
 * phase-space halo finder (Elahi et al.): 3D friends-of-friends, entropy KD
 * cells with velocity moments, the local velocity-density ratio R, 6D
 * friends-of-friends over the outliers, and unbinding by summed potentials.
 *
 * Conventions shared by every call
 *  - Array arguments are DEVICE pointers, caller-owned, structure-of-arrays.
 *    The library never frees caller memory.  Particle counts n < 2^31.
 *  - Grid coordinates q are uint32 in [0, 2^grid_bits); one grid unit is
 *    box / 2^grid_bits length units; the box is periodic.
 *  - Every call enqueues its kernels on `stream` (a hipStream_t passed as
 *    void*, NULL = the default stream) and returns a status.  Arguments are
 *    validated on the host before any device work; outputs are undefined when
 *    a call returns non-zero; vr_last_error() gives the message.
 *  - Calls marked "syncs" wait for the stream because they return a count to
 *    the host.
 *  - Temporary device memory comes from the context's workspace pool, capped
 *    by max_workspace_bytes (VR_ERR_OUT_OF_MEMORY when exceeded).
 *  - A context serves one stream at a time and is not thread-safe; several
 *    contexts may coexist.
 *  - The KD builds of vr_cell_moments and vr_local_vdensity start from the
 *    host members sorted along each axis.  A context keeps the sorted lists
 *    of its last build and reuses them when the next build's members, hosts
 *    and (unwrapped) coordinates have the same 64-bit content hash; the
 *    lists take 12 bytes per member of workspace, and are simply not kept
 *    where the workspace cap leaves no room for them.
 */
#ifndef VR_H
#define VR_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VR_OK = 0,
    VR_ERR_INVALID_ARG = -1,
    VR_ERR_NO_DEVICE = -2,
    VR_ERR_OUT_OF_MEMORY = -3,
    VR_ERR_HIP = -4,
    VR_ERR_NOT_CONVERGED = -5,
    VR_ERR_UNSUPPORTED = -6
};

typedef struct vr_ctx vr_ctx;

/* Create a context on `device`.  max_workspace_bytes = 0 means no cap.
 * Returns VR_ERR_NO_DEVICE when no gfx950 device with that ordinal exists. */
int vr_create(vr_ctx** ctx, int device, size_t max_workspace_bytes);
void vr_destroy(vr_ctx* ctx);
/* Message for the last failure on ctx (or of vr_create when ctx is NULL). */
const char* vr_last_error(const vr_ctx* ctx);
/* Wait for the stream and report a pending asynchronous HIP error. */
int vr_sync(vr_ctx* ctx, void* stream);
/* Bytes of workspace currently held by the context. */
size_t vr_workspace_bytes(const vr_ctx* ctx);
/* Start of a new particle set: drops what the context carries from one call
 * to the next for the same particles (the sorted member lists kept from the
 * last KD build), so the next KD build sorts afresh.  Calls between two
 * vr_new_snapshot calls may still share those lists when their content
 * hashes match.  Host-only; never fails on a valid ctx. */
int vr_new_snapshot(vr_ctx* ctx);

/* Kernel timing, for measurement.  While enabled, the library brackets its
 * main kernels with HIP events recorded on the stream each kernel is
 * launched on, and accumulates per kernel name the number of launches, the
 * summed duration and the algorithmic work of the launches (the unit is per
 * kernel: "fof_link3d" particles, "kd_level" member visits, "knn" queries,
 * "fof_link6d" participants, "unbind_potential" ordered pairs i != j,
 * "unbind_group" members, "radix_scatter" keys, "unbind_persistent" ordered
 * pairs i != j, timed from the first to the last graph replay of one call).
 * The name "knn_candidates" reports the "knn" launches and time with, as the
 * work, the candidate distances the neighbour searches evaluated (summed by
 * the kernel itself while timing is on).  vr_set_timing also clears the
 * totals.  vr_kernel_time waits for the recorded events. */
int vr_set_timing(vr_ctx* ctx, int enabled);

/* Launch-shape knobs of the context (integer results never depend on them;
 * FP64 potentials only through the order of their partial sums):
 * "knn_leaf"      members per leaf of the neighbour-search tree (16..256, 64)
 * "unbind_tile"   j-tile of the potential kernel staged in LDS (64..4096, 256;
 *                 the persistent kernel uses at most 1024 per wavefront)
 * "unbind_jchunk" j-range of one potential work item (256..65536, 4096)
 * "unbind_bpc"    workgroups per CU of the persistent potential kernel
 *                 (0..8, 0 = as many as fit)
 * "unbind_wide"   size class of the persistent schedule: the leading groups
 *                 with at least this many members (up to the first smaller
 *                 one) take a 1024-thread workgroup per pass, the others
 *                 256 threads (256..2^30, 4096)
 * "xcd_chunk"     consecutive workgroups of the kNN and linking sweeps kept
 *                 on one XCD (0..4096, 64; 0 = the dispatcher's order)
 * Returns VR_ERR_INVALID_ARG for an unknown knob or a value out of range;
 * vr_get_tune reads a knob back. */
int vr_tune(vr_ctx* ctx, const char* knob, int value);
int vr_get_tune(const vr_ctx* ctx, const char* knob, int* value);

/* Autotuner of those knobs.  Unless force is set and if cache_path (may be
 * NULL) names a readable cache written for this GPU architecture, its knobs
 * are applied and nothing is timed.  Otherwise the call times vr_unbind
 * (persistent) over unbind_tile x unbind_jchunk x unbind_bpc, then over
 * unbind_wide at the fastest of those, on a synthetic heavy-tailed group set
 * (sizes 32 .. 32768) and vr_local_vdensity over
 * knn_leaf x xcd_chunk on synthetic hosts (2000 cusped halos whose sizes
 * follow dN/dlnN ~ N^-0.9 on [256, 2^21], 6.6 M members), applies the
 * fastest settings and writes them, with every timing, to cache_path as
 * JSON.  Allocates its workloads (freed before return); takes a few
 * seconds; syncs. */
int vr_autotune(vr_ctx* ctx, const char* cache_path, int force);
int vr_kernel_time(vr_ctx* ctx, const char* kernel, int64_t* launches, double* total_ms,
                   double* work);

/* Particle set.  mass == NULL means every particle has mass mass_value. */
typedef struct {
    int64_t n;
    const uint32_t *qx, *qy, *qz;
    const float *vx, *vy, *vz;
    const float *mass;
    double mass_value;
    double box;
    int32_t grid_bits;   /* 1..21 */
} vr_particles;

/* Quantisation onto the integer grid of the periodic box (the workloads fix
 * 2^21-grid coordinates): q = floor(x * 2^grid_bits / box) mod 2^grid_bits,
 * the scale computed once in FP64, x promoted exactly from float. */
int vr_quantize(vr_ctx* ctx, int64_t n, const float* x, const float* y, const float* z,
                double box, int32_t grid_bits, uint32_t* qx, uint32_t* qy, uint32_t* qz,
                void* stream);

/* 3D friends-of-friends (Sec. 2.1, Eq. fof3d): i and j are linked iff
 * |x_i - x_j|^2 < ellx^2 with the periodic minimum image.  The squared
 * distance is exact (integer grid); the test is (double)d2 < ell2 with
 * ell2 = (ellx * 2^grid_bits / box)^2 in FP64.  ellx is in length units and
 * must satisfy 0 < ellx < box/2.
 * label[i] (out, n int32) = smallest particle index of i's component. */
int vr_fof3d(vr_ctx* ctx, const vr_particles* p, double ellx, int32_t* label, void* stream);

/* Groups of a canonical labelling (label[label[i]] == label[i], or < 0 for
 * no group): components of at least n_min members (N_min, Sec. 2.2),
 * ordered by size descending then smallest member ascending; members
 * ascending inside a group.  Outputs: *n_groups (HOST), group_of[n] (group
 * id or -1), offsets[n_groups+1] (capacity n+1), members[offsets[n_groups]]
 * (capacity n).  Syncs. */
int vr_groups(vr_ctx* ctx, int64_t n, const int32_t* label, int32_t n_min, int32_t* n_groups,
              int32_t* group_of, int32_t* offsets, int32_t* members, void* stream);

typedef struct {
    double f_cell;        /* N_cell = f_cell N_H (0.01) ...                  */
    int32_t ncell_floor;  /* ... raised to at least this (100) ...           */
    int32_t ncell_div;    /* ... and capped at N_H / ncell_div (8)           */
    int32_t nbins;        /* bins of the entropy histogram (16, <= 64)       */
    int32_t split_rule;   /* 0 = split the minimum-entropy dimension, 1 = max */
} vr_cell_params;

#define VR_CELL_COLS 28

/* Entropy KD cells, per-cell moments and interpolation (Sec. 2.2, the
 * entropy equation and Eqs. meanpos, meanvel, meandispvel, cellinterp).
 * Hosts: host_offsets[n_hosts+1], host_members (ascending inside each host,
 * every host of at least ncell_div members).  Each host is unwrapped by the
 * minimum image relative to its first member, split recursively at the
 * median of the chosen dimension until a node holds at most N_cell members
 * (N_cell = min(max(ceil(f_cell N_H), ncell_floor), N_H / ncell_div)).  For
 * every host member writes vbar[n][3] and sigma[n][6] (particle-major:
 * vbar[3*i + d], sigma[6*i + e] with e over xx,yy,zz,xy,xz,yz, so one
 * member's values are contiguous), rho_cell[n] and cell_of[n] (either may
 * be NULL: not written); other entries are not touched.  Cells are numbered per host (hosts in order, cells by ascending
 * smallest member).  cell_table (may be NULL) receives VR_CELL_COLS doubles
 * per cell: host, n, M, xbar[3], vbar[3], sigma[6], lo[3], hi[3], face
 * neighbours[6] (-x,+x,-y,+y,-z,+z; -1 none), volume.  *n_cells (HOST).
 * Syncs. */
int vr_cell_moments(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts,
                    const int32_t* host_offsets, const int32_t* host_members,
                    const vr_cell_params* cp, float* vbar, float* sigma, float* rho_cell,
                    int32_t* cell_of, int64_t cell_capacity, double* cell_table,
                    int64_t* n_cells, void* stream);

/* Local velocity density ratio R = ln(f_l / f_bg) (Sec. 2.2, Eq. fvbg and
 * the ratio that follows the interpolation equation).  For particle k of a
 * host: S_k = the n_se members nearest in space (self included, ties by
 * index); V_k = the n_v members of S_k nearest in velocity; h = velocity
 * distance to the n_v-th; f_l = sum_V m_j W(|dv_j|/h) / (h^3 sum_S m_j) with
 * the 3D Epanechnikov kernel W(u) = 15/(8 pi) (1 - u^2); f_bg = Gaussian at
 * vbar(x_k), sigma(x_k) (vbar [n][3], sigma [n][6], particle-major as
 * vr_cell_moments writes them).  2 <= n_v <= n_se <= 256 and n_v <= 32 when
 * n_se > 64 (the paper's defaults, 256 and 32, are the largest case; beyond
 * n_se = 32 a workgroup's LDS heaps cut the occupancy), every host has
 * >= n_se members.  subset (may be NULL = all host members) lists the particles to
 * process; R is written only for them (NaN if sigma is not positive
 * definite, +inf if h = 0).  VR_ERR_INVALID_ARG, with nothing written to R,
 * if host_members lists a particle twice or one outside [0, n). */
int vr_local_vdensity(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts,
                      const int32_t* host_offsets, const int32_t* host_members,
                      const float* vbar, const float* sigma, int32_t n_se, int32_t n_v,
                      const int32_t* subset, int64_t n_subset, float* R, void* stream);

/* Velocity linking length per host (Sec. 2.1: ellv = alpha_v sigma_v with
 * sigma_v = (det Sigma_H)^(1/6), Sigma_H the mass-weighted dispersion tensor
 * of all members about their mass-weighted mean).  ellv_host[n_hosts].
 * Syncs once, before its kernels (the host offsets are validated on the
 * host); the result is ready when the stream reaches it. */
int vr_host_ellv(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts,
                 const int32_t* host_offsets, const int32_t* host_members, double alpha_v,
                 double* ellv_host, void* stream);

/* 6D friends-of-friends over outliers (Eq. fof6d with the substructure
 * linking length ellx_s = alpha_xS ellx): participants are particles with
 * 0 <= host_of[i] < n_hosts and R[i] >= R_threshold (all hosted ones if R is
 * NULL; other host_of values, e.g. -1 or the id of an unsearched group, do
 * not take part);
 * i and j are linked iff both participate, share a host h, and
 * d2/ells2 + dv2/ellv_host[h]^2 < 1 (FP64, that evaluation order).
 * label6[i] = smallest participant index of i's component, -1 otherwise. */
int vr_fof6d(vr_ctx* ctx, const vr_particles* p, const int32_t* host_of,
             const double* ellv_host, int32_t n_hosts, double ellx_s, const float* R,
             float R_threshold, int32_t* label6, void* stream);

/* The paper's own substructure linker (Sec. 2.2, Eq. linkingcriteria).
 * Participants: hosted particles (0 <= host_of[i] < n_hosts) with
 * L[i] >= L_threshold (L: [n], e.g. from vr_ell_fit).  With
 * u = v - vbar(x) in FP64 (vbar: [n][3] local mean velocity, as
 * vr_cell_moments gives it) and s = |u|, i and j link iff they share a
 * host, d2 < (ellx_s in grid units)^2 (exact integer d2), s_i, s_j > 0,
 * s_i <= Vr s_j and s_j <= Vr s_i, and u_i . u_j >= cos_theta_op (s_i s_j).
 * label[i] = smallest participant index of the component, -1 otherwise.
 * Vr >= 1, -1 <= cos_theta_op <= 1, 0 < ellx_s < box/2. */
int vr_fof_sub(vr_ctx* ctx, const vr_particles* p, const int32_t* host_of, int32_t n_hosts,
               const float* vbar, double ellx_s, const float* L, float L_threshold, double Vr,
               double cos_theta_op, int32_t* label, void* stream);

/* The paper's second, relaxed linking stage (Sec. 2.2, the two-stage
 * approach that follows Eq. linkingcriteria).  label1 (device [n]) holds
 * first-stage components (smallest index or -1, as vr_fof_sub gives them);
 * those with >= n_min members are the tagged candidate groups.  Relaxed
 * participants: hosted particles with L >= (float)(L_threshold / gamma_L);
 * relaxed links: the criteria of vr_fof_sub with linking length
 * gamma_x * ellx_s, speed ratio gamma_V * Vr and opening-angle cosine
 * cos_op_relaxed.  Growth runs in synchronous rounds until nothing changes:
 * each untagged relaxed participant with a relaxed link to a particle
 * tagged in the previous round takes the smallest such tag.  Then two
 * groups join (transitively) when the relaxed links between their members
 * outnumber f_merge times the first-stage size of either.  label_out
 * (device [n]) = smallest member index of the final group, -1 elsewhere;
 * *rounds (HOST, may be NULL) = rounds that tagged someone.  Every member
 * of a candidate group must be a relaxed participant (else
 * VR_ERR_INVALID_ARG).  Syncs the stream once per round. */
int vr_sub_grow(vr_ctx* ctx, const vr_particles* p, const int32_t* host_of, int32_t n_hosts,
                const float* vbar, const float* L, float L_threshold, double gamma_L, double ellx_s,
                double gamma_x, double Vr, double gamma_V, double cos_op_relaxed, double f_merge,
                int32_t n_min, const int32_t* label1, int32_t* label_out, int32_t* rounds, void* stream);

/* ---- two species: dark matter and baryons (DM+Baryons mode) -------------- */

/* 3D FOF seeded by dark matter (Sec. 2.1): is_baryon (device [n], 0 = dark
 * matter) marks baryons, which link to dark matter within ellx but never to
 * each other.  label[i] = smallest index of i's component (a baryon with no
 * dark matter within ellx stays alone).  With no baryons this is vr_fof3d. */
int vr_fof3d_dm(vr_ctx* ctx, const vr_particles* p, double ellx, const uint8_t* is_baryon, int32_t* label,
                void* stream);

/* Baryons to substructure (Sec. 2.4, Eq. baryondist read with squared
 * terms): within each host (offsets/members as vr_groups gives them; both
 * species), a baryon takes sub[j] of the host's dark-matter member j that
 * minimises D2 = d2 / ell2 + dv2 / sigma_v^2 (exact integer d2 in grid
 * units, ell2 = (ellx in grid units)^2, FP64 dv2 in x, y, z order; ties to
 * the smaller index), -1 when the host has no dark matter; dark-matter
 * members copy sub[j].  out (device [n]) is written for host members only.
 * sub: device [n].  sigma_v > 0 is used as given; sigma_v <= 0 asks for the
 * typical dispersion of the searched hosts, computed on the device: the
 * mean over hosts of ellv_host[h] / alpha_v (sigma_v,H of Sec. 2.1, as
 * vr_host_ellv gives ellv_host, device [n_hosts]) weighted by each host's
 * dark-matter member count.  *sigma_v_used (HOST, may be NULL) receives the
 * value used (0 when no host holds dark matter).  Errors:
 * VR_ERR_INVALID_ARG for ellx outside (0, box/2), sigma_v <= 0 without
 * ellv_host or alpha_v > 0, a computed sigma_v that is not positive, or
 * NULL arrays; VR_ERR_UNSUPPORTED when a host's dark matter would need a
 * search tree deeper than 8 levels of 64 (never below 2^48 members).
 * Syncs a few times (member counts, sigma_v, tree level sizes). */
int vr_assign_baryons(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts, const int32_t* host_offsets,
                      const int32_t* host_members, const uint8_t* is_baryon, const int32_t* sub, double ellx,
                      double sigma_v, const double* ellv_host, double alpha_v, double* sigma_v_used, int32_t* out,
                      void* stream);

/* Canonical labels: out[i] = smallest j with label[j] == label[i] when that
 * label (in [0, n)) holds >= min_size particles, else -1; label < 0 gives
 * -1.  A label >= n is an error (VR_ERR_INVALID_ARG).  Syncs. */
int vr_relabel_min(vr_ctx* ctx, int64_t n, const int32_t* label, int32_t min_size, int32_t* out, void* stream);

/* vr_relabel_min for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result, from the same kernels, but its per-label counts, minima
 * and error flag live in a fixed device array of the library (2 x
 * VR_NOALLOC_MAX_LABELS + 64 int32, about 32 MiB, held by each GPU the
 * library runs on until the process ends; its address is taken once per
 * device by vr_create).  The call allocates nothing: no hipMalloc, no
 * workspace growth, no host allocation; it clears what it uses with fill
 * kernels and syncs once (the error flag comes back through the context's
 * pinned host memory).  n > VR_NOALLOC_MAX_LABELS is VR_ERR_INVALID_ARG.
 * Every call on one GPU shares that GPU's array, which keeps the last
 * call's contents: calls that overlap on one GPU (several streams, threads
 * or contexts) race and must be serialised by the caller. */
#define VR_NOALLOC_MAX_LABELS 4194304
int vr_relabel_min_noalloc(vr_ctx* ctx, int64_t n, const int32_t* label, int32_t min_size, int32_t* out,
                           void* stream);

/* Members of each group (offsets/members, device CSR) without the particles
 * flagged in drop (device [n], e.g. is_baryon): out_offsets (device
 * [n_groups+1]) and out_members (device, capacity offsets[n_groups]), order
 * kept.  Syncs once (the offsets are validated on the host). */
int vr_select_members(vr_ctx* ctx, int64_t n, int32_t n_groups, const int32_t* offsets, const int32_t* members,
                      const uint8_t* drop, int32_t* out_offsets, int32_t* out_members, void* stream);

typedef struct {
    double G;          /* gravitational constant in the particle units       */
    double eps;        /* Plummer softening length                            */
    double beta_E;     /* remove beta_E T + W >= 0 (0.95)                     */
    double frac_ref;   /* fraction of members defining the velocity frame (0.1) */
    int32_t n_min;     /* dissolve below this many members (20)               */
    int32_t n_ref_min; /* at least this many frame members (10)               */
    int32_t frame_type;/* 1 = around the potential minimum, 0 = whole group    */
    int32_t max_iter;  /* VR_ERR_NOT_CONVERGED beyond this many passes (100)  */
    int32_t persistent;/* 1 = passes replayed from a cached graph, each with one
                          persistent potential launch over a work queue of
                          (group, 64-row tile, j-range) items for all groups;
                          0 = host-planned passes                           */
    int32_t tile;      /* j-tile of the potential kernel, 0 = autotuned       */
} vr_unbind_params;

/* Unbinding (Sec. 2.2, Eq. binding), groups treated in isolation: per pass,
 * phi_i = -G sum_{j != i} m_j / sqrt(r_ij^2 + eps^2) over the current set
 * (FP32 pair terms, FP64 accumulation), a velocity frame from the members
 * nearest the potential minimum, removal of beta_E T + W >= 0, repeated until
 * nothing is removed; a group falling below n_min is dissolved.
 * Outputs for every member: bound[i] (0/1), phi[i] (FP64, potential in the
 * last pass i took part in); iters[g] = passes run.  Syncs.  Returns
 * VR_ERR_NOT_CONVERGED if a group still loses members in pass max_iter. */
int vr_unbind(vr_ctx* ctx, const vr_particles* p, int32_t n_groups, const int32_t* offsets,
              const int32_t* members, const vr_unbind_params* up, uint8_t* bound, double* phi,
              int32_t* iters, void* stream);

/* ---- normalised ratio L and significance cleaning (Sec. 2.2) ---------------
 * The paper normalises R by a skew-Gaussian fitted to each host's binned R
 * distribution (Eq. skewgaus), L = (R - Rbar) / sigma_R (Eq. ell), thresholds
 * L, and cleans candidate groups by their mean L (Eq. ellsig and the
 * truncated-Gaussian mean that follows it). */
typedef struct {
    double lo;             /* lower edge of the fine R grid (-16) */
    double width;          /* fine bin width (1/32) */
    int32_t nbins;         /* fine bins (1024), a multiple of max_merge, <= 4096 */
    int32_t peak_min;      /* merge bin pairs until the fullest holds this many (32) */
    int32_t max_merge;     /* largest merge factor, a power of two (64) */
    int32_t golden_iters;  /* golden-section iterations refining the peak (48), <= 200 */
} vr_ell_params;

/* Per host h: the finite R of its members are counted on the fine grid
 * (bin floor((R - lo) / width); values off the grid are not counted); bin
 * pairs are merged until the fullest merged bin holds peak_min (or the
 * factor reaches max_merge).  On the non-empty merged bins (centres x_b,
 * counts n_b) the log model ln n = a - p (x-c)^2 [x<c] - q (x-c)^2 [x>=c] is
 * fitted by least squares weighted by n_b; for each c it is linear in
 * (a, p, q); c is the merged-bin centre of least cost, refined by
 * golden-section search over one merged bin either side.  Output (device):
 * fit[h][4] = Rbar = c, sigma_R = 1/sqrt(2q), s = sqrt(q/p), A = exp(a);
 * status[h] = 1 fitted; 0 when fewer than 4 bins are non-empty or p, q are
 * not positive: then Rbar, sigma_R are the mean and dispersion of the merged
 * histogram (the merged width if that is 0), s = 1, A = the fullest count;
 * -1 when no value was counted (Rbar = sigma_R = NaN).  merge[h] (may be
 * NULL) = merge factor.  ell[i] = (float)(((double)R[i] - Rbar) / sigma_R)
 * for every member i of every host (NaN stays NaN); other entries are left
 * alone.  Members of a host are distinct and ascending (as vr_groups gives
 * them); R, ell: [n] device arrays. */
int vr_ell_fit(vr_ctx* ctx, int64_t n, int32_t n_hosts, const int32_t* host_offsets,
               const int32_t* host_members, const float* R, const vr_ell_params* ep, double* fit,
               int32_t* status, int32_t* merge, float* ell, void* stream);

/* Significance cleaning of candidate groups (offsets/members as vr_groups
 * gives them): with Lbar = sqrt(2/pi) exp(-ell_th^2/2) / erfc(ell_th/sqrt 2),
 * a group of N members whose mean L is below Lbar (1 + beta / sqrt(N)) loses
 * its member of smallest L (ties: smaller index first), repeatedly; once
 * fewer than n_min remain it is dissolved.  label (device [n]) is updated
 * for the members of every group: removed -> -1, kept -> the smallest kept
 * index; other entries are left alone.  removed (device [n_groups], may be
 * NULL) = members removed per group (N when dissolved).  Means are FP64 sums
 * of the float L. */
int vr_ell_clean(vr_ctx* ctx, int64_t n, int32_t n_groups, const int32_t* offsets, const int32_t* members,
                 const float* ell, double ell_th, double beta, int32_t n_min, int32_t* label,
                 int32_t* removed, void* stream);

/* ---- learned surrogate of R ------------------------------------------------
 * Predicts the R of vr_local_vdensity from 12 cheap per-particle features
 * (no neighbour search) with a 12-64-64-64-1 ReLU network; particles whose
 * prediction lies within a margin of the threshold get the exact R. */

/* Features of every host member (rows in host_members order, m rows =
 * host_offsets[n_hosts], written to *n_rows; syncs), as BF16 bit patterns,
 * row-major [m][12], each (x - shift[k]) * scale[k] (shift, scale: HOST
 * arrays of 12, or NULL for 0 and 1).  vbar [n][3], sigma [n][6] and
 * rho_cell [n] as vr_cell_moments writes them.  With Sigma = sigma(x) of the particle
 * (eigenvalues l1 <= l2 <= l3, unit eigenvectors e_a), dv = v - vbar(x):
 *  0     ln rhat, rhat = (3 n_se / (4 pi nhat))^(1/3), nhat = the member count
 *        of the 27 cells of side f = 2^cell_bits grid units around the
 *        particle over their volume, or of the 27 cells of side 4f when the
 *        fine window holds fewer than n_se members;
 *  1..3  |dv . e_a| / sqrt(l_a);      4..6  ln l_a;      7  ln rho_cell;
 *  8..10 |(vloc - vbar) . e_a| / sqrt(l_a), vloc = mean velocity of the
 *        members in the particle's fine cell and its 6 face neighbours;
 *  11    |v - vloc| / sqrt((l1 + l2 + l3) / 3).
 * Cells count the members of all listed hosts.  Features 1..11 are NaN if
 * Sigma is not positive definite.  0 <= cell_bits <= grid_bits - 4. */
int vr_rs_features(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts, const int32_t* host_offsets,
                   const int32_t* host_members, const float* vbar, const float* sigma, const float* rho_cell,
                   int32_t n_se, int32_t cell_bits, const float* shift, const float* scale, uint16_t* feat,
                   int64_t* n_rows, void* stream);

/* Network parameters: one device FP32 vector of VR_MLP_PARAMS values,
 * W1[12][64], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], w4[64], b4
 * (W[i][o] connects input i to output o). */
#define VR_MLP_PARAMS 9217

/* Rhat[i] for the m feature rows: BF16 inputs, weights and hidden
 * activations on MFMA with FP32 accumulation, ReLU, FP32 last layer;
 * NaN for rows with a NaN feature. */
int vr_mlp_forward(vr_ctx* ctx, const float* weights, int64_t m, const uint16_t* feat, float* Rhat,
                   void* stream);

/* Gradient (device FP32 [VR_MLP_PARAMS]) of the mean squared error
 * mean_b (Rhat(row_b) - target[row_b])^2 over a batch of m rows; rows
 * (device, m entries) picks the rows of feat/target, NULL = rows 0..m-1.
 * The forward pass is that of vr_mlp_forward; errors flow down through BF16
 * MFMA products with FP32 accumulation.  loss (device, may be NULL)
 * receives the batch loss. */
int vr_mlp_grad(vr_ctx* ctx, const float* weights, int64_t m, const uint16_t* feat, const int32_t* rows,
                const float* target, float* grad, float* loss, void* stream);

typedef struct {
    float lr, beta1, beta2, eps;   /* Adam (Kingma & Ba), e.g. 1e-3, 0.9, 0.999, 1e-8 */
} vr_adam_params;

/* One Adam step (step >= 1, for the bias correction) on the FP32 master
 * weights with the vr_mlp_grad gradient of the batch; adam_state (device)
 * holds the first and second moments, 2 * VR_MLP_PARAMS floats, zero at
 * step 1. */
int vr_mlp_train_step(vr_ctx* ctx, float* weights, float* adam_state, int64_t m, const uint16_t* feat,
                      const int32_t* rows, const float* target, const vr_adam_params* ap, int32_t step,
                      float* loss, void* stream);

/* Band selection of the surrogate path: R[members[i]] = Rhat[i] for the m
 * rows, and subset receives (in row order) members[i] of the rows with
 * |Rhat[i] - R_threshold| < margin or Rhat[i] not finite; *n_subset (HOST)
 * counts them.  Running vr_local_vdensity on the subset then replaces those
 * entries by the exact R.  Syncs. */
int vr_rs_select(vr_ctx* ctx, int64_t m, const int32_t* members, const float* Rhat, float R_threshold,
                 float margin, float* R, int32_t* subset, int64_t* n_subset, void* stream);

#ifdef __cplusplus
}
#endif
#endif
