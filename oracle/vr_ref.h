/*
 * vr_ref.h -- CPU oracle for the phase-space halo-finder hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 reference written
 * from the paper (Elahi et al., "Hunting for Galaxies and Halos in
 * simulations with VELOCIraptor").  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * All pointers are HOST pointers owned by the caller.  Every function returns
 * 0 on success or a negative status (-1 invalid argument, -5 not converged).
 *
 * Parity caveats (also listed in the design notes): the face-neighbour rule
 * and the minimum-entropy split choice of the cell tree are readings of an
 * under-specified passage ("parity unpinned" by the paper itself; they are
 * pinned only by structural invariants).
 */
#ifndef VR_REF_H
#define VR_REF_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Particle set in structure-of-arrays form.  q* are grid coordinates in
 * [0, 2^grid_bits); one grid unit is box / 2^grid_bits length units.
 * mass == NULL means every particle has mass mass_value. */
typedef struct {
    int64_t n;
    const uint32_t *qx, *qy, *qz;
    const float *vx, *vy, *vz;
    const float *mass;
    double mass_value;
    double box;
    int32_t grid_bits;
} vr_ref_particles;

/* Number of worker threads used by the embarrassingly parallel loops
 * (per host, per particle, per group).  1 = serial.  Returns the value set. */
int vr_ref_set_threads(int n_threads);

/* Quantise positions: q = floor(x * 2^grid_bits / box) mod 2^grid_bits,
 * with the scale computed once in FP64. */
int vr_ref_quantize(int64_t n, const float* x, const float* y, const float* z,
                    double box, int32_t grid_bits,
                    uint32_t* qx, uint32_t* qy, uint32_t* qz);

/* Squared linking length in grid units: (ellx * 2^grid_bits / box)^2. */
double vr_ref_ell2_grid(double ell, double box, int32_t grid_bits);

/* 3D friends-of-friends (Eq. fof3d, Sec. 2.1): periodic minimum image,
 * exact integer squared distance, link iff (double)d2 < ell2.
 * label[i] = smallest particle index of i's component. */
int vr_ref_fof3d(const vr_ref_particles* p, double ellx, int32_t* label);

/* Groups of a labelling: components with size >= n_min (labels < 0 are
 * ignored), ordered by size descending then smallest member index ascending;
 * members ascending inside a group.  group_of[i] = group id or -1.
 * offsets has n_groups+1 entries. */
int vr_ref_groups(int64_t n, const int32_t* label, int32_t n_min,
                  int32_t* n_groups, int32_t* group_of,
                  int32_t* offsets, int32_t* members);

/* Entropy of a binned mass distribution (Sec. 2.2, unlabelled entropy
 * equation): S = -sum_k p_k ln p_k / ln nb, p_k = h_k / sum h. */
double vr_ref_entropy(int32_t nb, const double* hist);

typedef struct {
    double f_cell;        /* 0.01 */
    int32_t ncell_floor;  /* 100 */
    int32_t ncell_div;    /* 8 */
    int32_t nbins;        /* 16 */
    int32_t split_rule;   /* 0 = split the minimum-entropy dimension, 1 = maximum */
} vr_ref_cell_params;

#define VR_REF_CELL_COLS 28

/* Entropy KD cells, per-cell moments and inverse-distance interpolation
 * (Sec. 2.2, Eqs. meanpos, meanvel, meandispvel, cellinterp).
 * Hosts are given as ascending member lists.  For every host member writes
 * vbar[3*n] (component-major), sigma[6*n] (xx,yy,zz,xy,xz,yz), rho_cell[n],
 * cell_of[n].  Cells are numbered per host, hosts in the order given, and
 * inside a host by ascending smallest member index.  If cell_table != NULL it
 * receives VR_REF_CELL_COLS doubles per cell (layout in the .cpp). */
int vr_ref_cell_moments(const vr_ref_particles* p, int32_t n_hosts,
                        const int32_t* host_offsets, const int32_t* host_members,
                        const vr_ref_cell_params* cp,
                        float* vbar, float* sigma, float* rho_cell, int32_t* cell_of,
                        int64_t cell_capacity, double* cell_table, int64_t* n_cells);

/* Local velocity density ratio R = ln(f_l / f_bg) (Sec. 2.2, Eq. fvbg and
 * the unlabelled R equation).  Processes every member of every host, or only
 * the listed subset (each entry must be a host member).  Writes R only for
 * processed particles.  Optional FP64 side outputs (may be NULL):
 * lnfl[n], lnfbg[n]; nbr_s[n_proc*n_se] and nbr_v[n_proc*n_v] hold the
 * spatial and velocity neighbour sets of the processed particles in
 * processing order (ascending by their ordering key). */
int vr_ref_local_vdensity(const vr_ref_particles* p, int32_t n_hosts,
                          const int32_t* host_offsets, const int32_t* host_members,
                          const float* vbar, const float* sigma,
                          int32_t n_se, int32_t n_v,
                          const int32_t* subset, int64_t n_subset,
                          float* R, double* lnfl, double* lnfbg,
                          int32_t* nbr_s, int32_t* nbr_v);

/* Velocity linking length per host: alpha_v * (det Sigma_H)^(1/6), Sigma_H
 * the mass-weighted dispersion tensor of all host members about their
 * mass-weighted mean velocity (Sec. 2.1 with the sigV definition of the
 * property table). */
int vr_ref_host_ellv(const vr_ref_particles* p, int32_t n_hosts,
                     const int32_t* host_offsets, const int32_t* host_members,
                     double alpha_v, double* ellv_host);

/* 6D friends-of-friends over outliers (Eq. fof6d): participants are hosted
 * particles (0 <= host_of < n_hosts) with R >= R_threshold (all hosted ones
 * if R is NULL); link iff same host and d2/ellxs2 + dv2/ellv^2 < 1.
 * label6 = smallest participant index of the component, -1 otherwise. */
int vr_ref_fof6d(const vr_ref_particles* p, const int32_t* host_of, int32_t n_hosts,
                 const double* ellv_host, double ellx_s,
                 const float* R, float R_threshold, int32_t* label6);

/* The paper's substructure linker (Sec. 2.2, Eq. linkingcriteria):
 * participants are hosted particles with L >= L_threshold; i and j link iff
 * they share a host, d2 < (ellx_s in grid units)^2 (exact integer d2), and
 * with u = v - vbar(x) (FP64, per particle: vbar is [3][n], the local mean
 * velocity of Eq. cellinterp) and speeds s = |u| (both > 0):
 * s_i <= Vr s_j, s_j <= Vr s_i and u_i . u_j >= cos_op (s_i s_j).
 * label = smallest participant index of the component, -1 otherwise. */
int vr_ref_fof_sub(const vr_ref_particles* p, const int32_t* host_of, int32_t n_hosts,
                   const float* vbar, double ellx_s, const float* L, float L_threshold,
                   double Vr, double cos_op, int32_t* label);

/* Second, relaxed stage of the paper's linker (Sec. 2.2, the two-stage
 * approach after Eq. linkingcriteria).  label1 holds the first-stage
 * components (smallest index, -1); those of >= n_min members are the
 * candidate groups, tagged.  Relaxed participants: hosted particles with
 * L >= L_threshold / gamma_L; relaxed links: the criteria of vr_ref_fof_sub
 * with linking length gamma_x * ellx_s, speed ratio gamma_V * Vr and
 * opening angle of cosine cos_op_relaxed.  Growth, in synchronous rounds
 * until nothing changes: every untagged relaxed participant with a relaxed
 * link to a particle tagged in the previous round takes the smallest such
 * tag.  Then, for every pair of groups, the relaxed links between their
 * members are counted; two groups join when the count exceeds f_merge times
 * the first-stage size of either (joins are transitive).  label_out =
 * smallest member index of the final group, -1 for every other particle.
 * grown (may be NULL) receives the number of growth rounds. */
int vr_ref_sub_grow(const vr_ref_particles* p, const int32_t* host_of, int32_t n_hosts,
                    const float* vbar, const float* L, float L_threshold, double gamma_L,
                    double ellx_s, double gamma_x, double Vr, double gamma_V,
                    double cos_op_relaxed, double f_merge, int32_t n_min,
                    const int32_t* label1, int32_t* label_out, int32_t* rounds);

/* Two species (Sec. 2.1, DM+Baryons mode): 3D FOF in which a baryon
 * (is_baryon[i] != 0) never initiates links -- pairs link iff d2 < ell2 and
 * at least one of the two is dark matter.  label = smallest index of the
 * component (a baryon with no dark matter within ellx stays alone). */
int vr_ref_fof3d_dm(const vr_ref_particles* p, double ellx, const uint8_t* is_baryon, int32_t* label);

/* Baryons to substructure (Sec. 2.4, Eq. baryondist with squared terms):
 * within each host, every baryon takes the substructure label sub[j] of
 * the host's dark-matter member j nearest in phase space,
 * D2 = d2 / ell2 + dv2 / sigma_v^2 (exact integer d2, FP64 dv2 in x, y, z
 * order; ties to the smaller index); a host without dark matter gives -1.
 * Dark-matter members keep sub[j].  out[i] for host members only. */
int vr_ref_assign_baryons(const vr_ref_particles* p, int32_t n_hosts, const int32_t* host_offsets,
                          const int32_t* host_members, const uint8_t* is_baryon, const int32_t* sub,
                          double ellx, double sigma_v, int32_t* out);

typedef struct {
    double G, eps, beta_E, frac_ref;
    int32_t n_min, n_ref_min, frame_type, max_iter;
} vr_ref_unbind_params;

/* Unbinding (Sec. 2.2, Eq. binding) by direct FP64 summation of
 * Plummer-softened pair potentials.  bound[i] (0/1) for every member,
 * phi[i] = potential of i in the last pass it took part in, iters[g] =
 * passes run.  min_margin[g] (may be NULL) = smallest |beta_E T + W| / |W|
 * met in any pass of group g (used to excuse classifications that sit on
 * the threshold). */
int vr_ref_unbind(const vr_ref_particles* p, int32_t n_groups,
                  const int32_t* offsets, const int32_t* members,
                  const vr_ref_unbind_params* up,
                  uint8_t* bound, double* phi, int32_t* iters, double* min_margin);

/* ---- Normalised ratio L and significance cleaning (Sec. 2.2) ----------
 *
 * Per host, the finite R values of its members are binned on a fixed fine
 * grid (nbins bins of `width` from `lo`); adjacent bins are merged in pairs
 * until the fullest merged bin holds >= peak_min (merge factor <= max_merge).
 * The skew-Gaussian of Eq. skewgaus is fitted to the merged counts n_b at the
 * bin centres x_b by weighted least squares of ln n_b (weight n_b, the
 * inverse Poisson variance of ln n_b): for a peak position c the model
 * ln n = a - p (x-c)^2 [x<c] - q (x-c)^2 [x>=c] is linear in (a, p, q); c is
 * the merged-bin centre of least cost, refined by golden-section search over
 * one merged bin either side.  Then Rbar = c, sigma_R = 1/sqrt(2q),
 * s = sqrt(q/p), A = exp(a), and L = (R - Rbar) / sigma_R (Eq. ell), in FP64
 * rounded to float.  A host whose fit fails (fewer than 4 non-empty bins, or
 * p, q not positive) takes the mean and dispersion of its merged histogram
 * (status 0, s = 1); a host without binned values gets NaN (status -1). */
typedef struct {
    double lo;             /* lower edge of the fine grid (-16) */
    double width;          /* fine bin width (1/32) */
    int32_t nbins;         /* fine bins (1024), a multiple of max_merge */
    int32_t peak_min;      /* merge until the fullest merged bin holds this many (32) */
    int32_t max_merge;     /* largest merge factor, a power of two (64) */
    int32_t golden_iters;  /* golden-section iterations (48) */
} vr_ref_ell_params;

/* fit[h*4 + 0..3] = Rbar, sigma_R, s, A; status[h] = 1 fitted, 0 moments,
 * -1 no binned value; merge[h] (may be NULL) = merge factor; ell[i] for the
 * members of every host (other entries untouched). */
int vr_ref_ell_fit(int64_t n, int32_t n_hosts, const int32_t* host_offsets,
                   const int32_t* host_members, const float* R,
                   const vr_ref_ell_params* ep, double* fit, int32_t* status,
                   int32_t* merge, float* ell);

/* Least-squares cost of the log model at peak position c over nb bins
 * (centres x, counts w > 0); apq (may be NULL) receives a, p, q.  +inf when
 * a side of c holds no bin. */
double vr_ref_ell_cost(int32_t nb, const double* x, const double* w, double c, double* apq);

/* Mean L of a unit Gaussian above ell_th (the expected <L> of chance
 * outliers, the closed form following Eq. ellsig). */
double vr_ref_ell_mean(double ell_th);

/* Significance cleaning (Eq. ellsig): while a group's mean L is below
 * Lbar(ell_th) (1 + beta / sqrt(N)), remove its member of smallest L (ties:
 * smaller index first); below n_min members the group dissolves.  label is
 * updated in place for the members of every group: removed -> -1, kept ->
 * the smallest kept index.  removed[g] (may be NULL) = members removed. */
int vr_ref_ell_clean(int64_t n, int32_t n_groups, const int32_t* offsets,
                     const int32_t* members, const float* ell, double ell_th,
                     double beta, int32_t n_min, int32_t* label, int32_t* removed);

#ifdef __cplusplus
}
#endif
#endif
