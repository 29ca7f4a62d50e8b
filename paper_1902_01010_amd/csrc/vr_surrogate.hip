// vr_surrogate.hip -- the learned R surrogate: cheap per-particle features,
// a 12-64-64-64-1 ReLU network on BF16 MFMA (FP32 accumulation), its
// hand-written backward pass and Adam, and the band selection that sends
// uncertain particles back to the exact neighbour search.
//
// The exact R of Sec. 2.2 (local velocity density over the background
// Gaussian) needs an N_se-neighbour search per particle; the features here
// need none: window counts on two grid levels, the eigen-frame of the
// interpolated dispersion tensor and a local mean velocity.
#include "vr_internal.h"

#include <algorithm>
#include <cmath>

namespace vr {
namespace {

constexpr int NF = 12;            // features per particle
constexpr int H = 64;             // hidden width
// parameter offsets in the FP32 vector: W1[12][64] b1 W2[64][64] b2 W3[64][64] b3 w4[64] b4
constexpr int OW1 = 0, OB1 = OW1 + NF * H, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H * H,
              OW4 = OB3 + H, OB4 = OW4 + H, NPARAM = OB4 + 1;
static_assert(NPARAM == VR_MLP_PARAMS, "parameter layout");

typedef short bf8 __attribute__((ext_vector_type(8)));     // bits of 8 BF16 MFMA operands
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));   // the same, as the MFMA operand type
typedef float f16v __attribute__((ext_vector_type(16)));   // 32x32 accumulator slice of one lane

// FP32 -> BF16 bits, round to nearest even; NaN stays a (quiet) NaN.
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// D (32x32) += A (32x16) B (16x32) on gfx950's BF16 matrix cores: lane l
// gives row l%32 of A and column l%32 of B, eight K entries each, and the
// hardware pairs slot s of A's lane half h with slot s of B's lane half h.
// Which K index a (half, slot) stands for is the caller's choice, the same
// for both operands.
__device__ __forceinline__ f16v mfma(bf8 a, bf8 b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c, 0, 0,
                                                    0);
}

// ============================================================================
// features
// ============================================================================
__device__ __forceinline__ uint64_t cell_key(uint32_t cx, uint32_t cy, uint32_t cz, int b) {
    return ((uint64_t)cz << (2 * b)) | ((uint64_t)cy << b) | (uint64_t)cx;
}

__device__ __forceinline__ uint32_t hash64(uint64_t k, uint32_t mask) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return (uint32_t)k & mask;
}

constexpr uint64_t EMPTY64 = ~0ull;

__global__ void k_rs_keys(int64_t m, const int32_t* __restrict__ mem, const uint32_t* __restrict__ qx,
                          const uint32_t* __restrict__ qy, const uint32_t* __restrict__ qz, int cbits, int b,
                          uint64_t* __restrict__ keys, uint32_t* __restrict__ rows) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int g = mem[i];
    keys[i] = cell_key(qx[g] >> cbits, qy[g] >> cbits, qz[g] >> cbits, b);
    rows[i] = (uint32_t)i;
}

__global__ void k_rs_heads(int64_t m, const uint64_t* __restrict__ keys, uint32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ void k_rs_starts(int64_t m, const uint32_t* __restrict__ flag, const uint32_t* __restrict__ cid,
                            uint32_t* __restrict__ start, uint32_t ncells) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    if (flag[i]) start[cid[i]] = (uint32_t)i;
    if (i == 0) start[ncells] = (uint32_t)m;
}

__global__ void k_rs_clear(unsigned long long* __restrict__ hk, uint32_t size) {
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h < size) hk[h] = EMPTY64;
}

__global__ void k_rs_insert(uint32_t ncells, const uint64_t* __restrict__ keys, const uint32_t* __restrict__ start,
                            uint32_t hmask, unsigned long long* __restrict__ hk, uint32_t* __restrict__ hv) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const unsigned long long k = keys[start[c]];
    uint32_t h = hash64(k, hmask);
    for (;;) {
        const unsigned long long prev = atomicCAS(&hk[h], (unsigned long long)EMPTY64, k);
        if (prev == EMPTY64 || prev == k) {
            hv[h] = c;
            return;
        }
        h = (h + 1) & hmask;
    }
}

__device__ __forceinline__ int find64(const unsigned long long* __restrict__ hk, const uint32_t* __restrict__ hv,
                                      uint32_t hmask, uint64_t k) {
    uint32_t h = hash64(k, hmask);
    for (;;) {
        const unsigned long long kk = hk[h];
        if (kk == k) return (int)hv[h];
        if (kk == EMPTY64) return -1;
        h = (h + 1) & hmask;
    }
}

// velocity sums of the members of each fine cell, FP64, in sorted order
__global__ void k_rs_vsum(uint32_t ncells, const uint32_t* __restrict__ start, const uint32_t* __restrict__ rows,
                          const int32_t* __restrict__ mem, const float* __restrict__ vx, const float* __restrict__ vy,
                          const float* __restrict__ vz, double* __restrict__ vsum) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    double s0 = 0, s1 = 0, s2 = 0;
    for (uint32_t k = start[c]; k < start[c + 1]; ++k) {
        const int g = mem[rows[k]];
        s0 += (double)vx[g];
        s1 += (double)vy[g];
        s2 += (double)vz[g];
    }
    vsum[3 * (size_t)c] = s0;
    vsum[3 * (size_t)c + 1] = s1;
    vsum[3 * (size_t)c + 2] = s2;
}

struct Level {
    const unsigned long long* hk;
    const uint32_t* hv;
    uint32_t hmask;
    const uint32_t* start;
    int cbits, b;
};

// Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations
// (each rotation zeroes one off-diagonal pair); ascending eigenvalues, unit
// eigenvectors in the columns of V.
__device__ void jacobi3(double A[3][3], double lam[3], double V[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 12; ++sweep) {
        const double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
        const double dia = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
        if (off == 0.0 || off <= 1e-300 + 1e-18 * dia) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = A[p][q];
                if (apq == 0.0) continue;
                const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                // A <- J^T A J with J the rotation in the (p, q) plane
                for (int k = 0; k < 3; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                A[p][q] = A[q][p] = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    int o[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i) lam[i] = A[i][i];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2 - i; ++j)
            if (lam[o[j]] > lam[o[j + 1]]) { const int t = o[j]; o[j] = o[j + 1]; o[j + 1] = t; }
    double l2[3], V2[3][3];
    for (int a = 0; a < 3; ++a) {
        l2[a] = lam[o[a]];
        for (int k = 0; k < 3; ++k) V2[k][a] = V[k][o[a]];
    }
    for (int a = 0; a < 3; ++a) {
        lam[a] = l2[a];
        for (int k = 0; k < 3; ++k) V[k][a] = V2[k][a];
    }
}

// Members in the 27 cells around (cx, cy, cz).  Each z-layer's nine
// lookups go out together: the nine first-probe keys in one round trip,
// then the hits' values and member ranges; a probe continues one by one
// only past a collision.
__device__ __forceinline__ uint32_t window_count(const Level& L, uint32_t cx, uint32_t cy, uint32_t cz) {
    const uint32_t mask = (1u << L.b) - 1u;
    uint32_t n = 0;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
        uint64_t k[9];
        uint32_t h[9];
        unsigned long long kk[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int dy = j / 3 - 1, dx = j % 3 - 1;
            k[j] = cell_key((cx + dx) & mask, (cy + dy) & mask, (cz + dz) & mask, L.b);
            h[j] = hash64(k[j], L.hmask);
        }
#pragma unroll
        for (int j = 0; j < 9; ++j) kk[j] = L.hk[h[j]];
        int c[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            if (kk[j] == k[j]) c[j] = (int)L.hv[h[j]];
            else if (kk[j] == EMPTY64) c[j] = -1;
            else c[j] = find64(L.hk, L.hv, L.hmask, k[j]);  // past a collision
        }
#pragma unroll
        for (int j = 0; j < 9; ++j)
            if (c[j] >= 0) n += L.start[c[j] + 1] - L.start[c[j]];
    }
    return n;
}

struct FeatNorm {
    float shift[NF], scale[NF];
};

// Members in the 27-cell window of every occupied coarse cell (the fallback
// density of the fine cells inside it), once per coarse cell.
__global__ __launch_bounds__(256) void k_rs_coarsewin(uint32_t ncells, const uint64_t* __restrict__ keys,
                                                      Level coarse, uint32_t* __restrict__ cwin) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const uint64_t key = keys[coarse.start[c]];
    const uint32_t mask = (1u << coarse.b) - 1u;
    cwin[c] = window_count(coarse, (uint32_t)(key & mask), (uint32_t)((key >> coarse.b) & mask),
                           (uint32_t)(key >> (2 * coarse.b)));
}

// What a row's features take from its fine cell alone, once per occupied
// fine cell (rows of a cell share it): feature 0, the log radius holding
// n_se neighbours at the density of the 27-cell window (the coarse window
// where the fine one holds fewer than n_se), and the mean velocity of the
// cell and its six face neighbours.  cf[4 c .. 4 c + 3] = (f0, vloc).
__global__ __launch_bounds__(256) void k_rs_cellfeat(uint32_t ncells, const uint64_t* __restrict__ keys,
                                                     Level fine, Level coarse, const uint32_t* __restrict__ cwin,
                                                     const double* __restrict__ vsum, int n_se, double cell_len,
                                                     double* __restrict__ cf) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const uint64_t key = keys[fine.start[c]];
    const uint32_t mask = (1u << fine.b) - 1u;
    const uint32_t cx = (uint32_t)(key & mask), cy = (uint32_t)((key >> fine.b) & mask),
                   cz = (uint32_t)(key >> (2 * fine.b));
    const uint32_t nf = window_count(fine, cx, cy, cz);
    double nhat;
    if ((int)nf >= n_se) {
        nhat = (double)nf / (27.0 * cell_len * cell_len * cell_len);
    } else {
        // the coarse grid's cells are 4 fine cells a side; the one holding
        // this fine cell is occupied, and its window count is precomputed
        const uint32_t cmask = (1u << coarse.b) - 1u;
        const int c1 = find64(coarse.hk, coarse.hv, coarse.hmask,
                              cell_key((cx >> 2) & cmask, (cy >> 2) & cmask, (cz >> 2) & cmask, coarse.b));
        const uint32_t nc = c1 >= 0 ? cwin[c1] : 0u;
        const double L4 = 4.0 * cell_len;
        nhat = (double)nc / (27.0 * L4 * L4 * L4);
    }
    cf[4 * (size_t)c] = log(cbrt(3.0 * (double)n_se / (4.0 * M_PI * nhat)));
    const int fo[7][3] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    // the seven lookups go out together, as in window_count
    uint64_t fk[7];
    uint32_t fh[7];
    unsigned long long fkk[7];
    int fc[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        fk[k] = cell_key((cx + fo[k][0]) & mask, (cy + fo[k][1]) & mask, (cz + fo[k][2]) & mask, fine.b);
        fh[k] = hash64(fk[k], fine.hmask);
    }
#pragma unroll
    for (int k = 0; k < 7; ++k) fkk[k] = fine.hk[fh[k]];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        if (fkk[k] == fk[k]) fc[k] = (int)fine.hv[fh[k]];
        else if (fkk[k] == EMPTY64) fc[k] = -1;
        else fc[k] = find64(fine.hk, fine.hv, fine.hmask, fk[k]);
    }
    double s0 = 0, s1 = 0, s2 = 0, cnt = 0;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const int cc = fc[k];
        if (cc < 0) continue;
        cnt += (double)(fine.start[cc + 1] - fine.start[cc]);
        s0 += vsum[3 * (size_t)cc];
        s1 += vsum[3 * (size_t)cc + 1];
        s2 += vsum[3 * (size_t)cc + 2];
    }
    cf[4 * (size_t)c + 1] = s0 / cnt;
    cf[4 * (size_t)c + 2] = s1 / cnt;
    cf[4 * (size_t)c + 3] = s2 / cnt;
}

__global__ __launch_bounds__(256) void k_rs_features(int64_t m, const int32_t* __restrict__ mem,
                                                     const float* __restrict__ vx, const float* __restrict__ vy,
                                                     const float* __restrict__ vz, const float* __restrict__ vbar,
                                                     const float* __restrict__ sigma, const float* __restrict__ rho,
                                                     int64_t n, const uint32_t* __restrict__ head,
                                                     const uint32_t* __restrict__ cid, const double* __restrict__ cf,
                                                     FeatNorm nrm, const uint32_t* __restrict__ order,
                                                     uint16_t* __restrict__ feat) {
    // rows are taken in fine-cell order (position t of the sorted cell
    // keys), so neighbouring threads share their cell's values
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int64_t i = order[t];
    const int g = mem[i];
    const uint32_t c = head[t] ? cid[t] : cid[t] - 1;  // the row's fine cell (exclusive scan of the heads)
    double f[NF];
    f[0] = cf[4 * (size_t)c];
    f[8] = cf[4 * (size_t)c + 1];  // vloc, turned into features below
    f[9] = cf[4 * (size_t)c + 2];
    f[10] = cf[4 * (size_t)c + 3];
    const double vl[3] = {f[8], f[9], f[10]};
    double A[3][3];
    const float* sg = sigma + (int64_t)g * 6;  // particle-major
    A[0][0] = sg[0];
    A[1][1] = sg[1];
    A[2][2] = sg[2];
    A[0][1] = A[1][0] = sg[3];
    A[0][2] = A[2][0] = sg[4];
    A[1][2] = A[2][1] = sg[5];
    double lam[3], V[3][3];
    jacobi3(A, lam, V);
    const double vb[3] = {vbar[(int64_t)g * 3], vbar[(int64_t)g * 3 + 1], vbar[(int64_t)g * 3 + 2]};
    const double vv[3] = {vx[g], vy[g], vz[g]};
    const bool ok = lam[0] > 0.0;
    for (int a = 0; a < 3; ++a) {
        const double sl = sqrt(lam[a]);
        double pd = 0, pl = 0;
        for (int k = 0; k < 3; ++k) {
            pd += (vv[k] - vb[k]) * V[k][a];
            pl += (vl[k] - vb[k]) * V[k][a];
        }
        f[1 + a] = fabs(pd) / sl;
        f[4 + a] = log(lam[a]);
        f[8 + a] = fabs(pl) / sl;
    }
    f[7] = log((double)rho[g]);
    const double d0 = vv[0] - vl[0], d1 = vv[1] - vl[1], d2 = vv[2] - vl[2];
    f[11] = sqrt(d0 * d0 + d1 * d1 + d2 * d2) / sqrt((lam[0] + lam[1] + lam[2]) / 3.0);
    uint16_t* out = feat + i * NF;
    for (int k = 0; k < NF; ++k) {
        const double x = (!ok && k > 0) ? (double)NAN : (f[k] - (double)nrm.shift[k]) * (double)nrm.scale[k];
        out[k] = bf16_bits((float)x);
    }
}

// ============================================================================
// network
// ============================================================================
// K order of the layers: slot s of lane half h in k-block kb is index
// 16 kb + 8 (s / 4) + 4 h + s % 4.  That is where a lane's accumulator
// entries of one 32-unit tile already sit (entry j of tile t is unit
// 32 t + 8 (j / 4) + 4 h + j % 4, i.e. k-block 2 t + j / 8, slot j % 8), so
// one layer's output becomes the next layer's B operand in registers.
// BF16 weights pre-arranged as MFMA A operands, one 16-byte group per lane:
//  fwd1 [2 row tiles][1 k-block][64 lanes]   W1^T (inputs 12..15 are zero)
//  fwd2 [2][4][64], fwd3 [2][4][64]          W2^T, W3^T
//  bwd3 [2][4][64], bwd2 [2][4][64]          W3, W2 (propagate errors down)
// For lane l of row tile t and k-block kb the group holds row 32 t + l % 32
// of the matrix at the eight columns of that K order.
constexpr int PK_FWD1 = 0, PK_FWD2 = PK_FWD1 + 2 * 1 * 64, PK_FWD3 = PK_FWD2 + 2 * 4 * 64,
              PK_BWD3 = PK_FWD3 + 2 * 4 * 64, PK_BWD2 = PK_BWD3 + 2 * 4 * 64, PK_TOTAL = PK_BWD2 + 2 * 4 * 64;

__device__ __forceinline__ int layer_k(int kb, int half, int s) { return 16 * kb + 8 * (s >> 2) + 4 * half + (s & 3); }

__global__ void k_mlp_pack(const float* __restrict__ w, bf8* __restrict__ pk) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= PK_TOTAL) return;
    int base, nkb, which;
    if (e < PK_FWD2) { base = PK_FWD1; nkb = 1; which = 1; }
    else if (e < PK_FWD3) { base = PK_FWD2; nkb = 4; which = 2; }
    else if (e < PK_BWD3) { base = PK_FWD3; nkb = 4; which = 3; }
    else if (e < PK_BWD2) { base = PK_BWD3; nkb = 4; which = -3; }
    else { base = PK_BWD2; nkb = 4; which = -2; }
    const int r = e - base;
    const int lane = r & 63, kb = (r >> 6) % nkb, t = (r >> 6) / nkb;
    const int row = 32 * t + (lane & 31);
    bf8 v;
    for (int j = 0; j < 8; ++j) {
        const int col = layer_k(kb, lane >> 5, j);
        float x;
        if (which == 1) x = col < NF ? w[OW1 + col * H + row] : 0.f;          // W1^T[out=row][in=col]
        else if (which == 2) x = w[OW2 + col * H + row];                        // W2^T
        else if (which == 3) x = w[OW3 + col * H + row];                        // W3^T
        else if (which == -3) x = w[OW3 + row * H + col];                       // W3[in=row][out=col]
        else x = w[OW2 + row * H + col];                                        // W2
        v[j] = (short)bf16_bits(x);
    }
    pk[e] = v;
}

// Accumulator row of entry j of lane l in a 32x32 tile: 8 (j/4) + 4 (l/32) + j%4.
__device__ __forceinline__ int acc_row(int j, int lane) { return 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3); }

// The inputs of a 32-row tile as the B operand of the single k-block: lane
// l holds row r0 + l%32, inputs 4 (l/32) + 0..3 in slots 0..3 and
// 8 + 4 (l/32) + 0..3 in slots 4..7 (inputs 12..15 do not exist and are
// zero).  bad = some input is NaN.
__device__ __forceinline__ void load_inputs(const uint16_t* __restrict__ feat, int64_t row, bool valid, int lane,
                                            bf8& in, bool& bad) {
    const int half = lane >> 5;
    in = bf8{0, 0, 0, 0, 0, 0, 0, 0};
    bad = false;
    if (!valid) return;
    const uint16_t* fr = feat + row * NF;
    for (int j = 0; j < 4; ++j) {
        const uint16_t a = fr[4 * half + j];
        in[j] = (short)a;
        bad |= (a & 0x7FFFu) > 0x7F80u;
        if (half == 0) {
            const uint16_t b = fr[8 + j];
            in[4 + j] = (short)b;
            bad |= (b & 0x7FFFu) > 0x7F80u;
        }
    }
}

// One dense layer on a 32-row tile: out[t] (t = 2 row tiles of 32 hidden
// units) = bias + W^T x, x given as nkb B-operand k-blocks.
template <int NKB>
__device__ __forceinline__ void layer(const bf8* __restrict__ pk, const float* __restrict__ bias, const bf8* x,
                                      int lane, f16v out[2]) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f16v acc;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = bias ? bias[32 * t + acc_row(j, lane)] : 0.f;
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) acc = mfma(pk[(t * NKB + kb) * 64 + lane], x[kb], acc);
        out[t] = acc;
    }
}

// max(x, 0) for every non-NaN x in one integer max: a set sign bit is a
// negative integer (-0 gives +0).
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// Two FP32 values as packed BF16 bits (gfx950's v_cvt_pk_bf16_f32: round to
// nearest even, as bf16_bits for every non-NaN value).
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v){lo, hi}, bf2v));
}

// The BF16 B operands of the next layer (ReLU first when with_relu is set):
// entry j of row tile t is slot j % 8 of k-block 2 t + j / 8.
template <bool with_relu>
__device__ __forceinline__ void operands(f16v a[2], bf8 x[4]) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            uint32_t p[4];
#pragma unroll
            for (int s = 0; s < 8; s += 2) {
                const int j = 8 * b + s;
                if (with_relu) {
                    a[t][j] = relu(a[t][j]);
                    a[t][j + 1] = relu(a[t][j + 1]);
                }
                p[s >> 1] = bf16_pair(a[t][j], a[t][j + 1]);
            }
            x[2 * t + b] = __builtin_bit_cast(bf8, (uint4){p[0], p[1], p[2], p[3]});
        }
}
__device__ __forceinline__ void relu_to_operands(f16v a[2], bf8 x[4]) { operands<true>(a, x); }
// errors flowing down: signed, no ReLU
__device__ __forceinline__ void to_operands(f16v a[2], bf8 x[4]) { operands<false>(a, x); }

__device__ __forceinline__ float out_layer(const float* __restrict__ w, const f16v h3[2], int lane) {
    float y = 0.f;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 16; ++j) y = fmaf(w[OW4 + 32 * t + acc_row(j, lane)], h3[t][j], y);
    y += __shfl_xor(y, 32, 64);
    return y + w[OB4];
}

// Inference: every wavefront takes 32-row tiles until none are left.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ w, const bf8* __restrict__ pk,
                                                     int64_t m, const uint16_t* __restrict__ feat,
                                                     float* __restrict__ out) {
    const int lane = __lane_id();
    const int64_t ntiles = (m + 31) / 32;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t tile = wave; tile < ntiles; tile += nwaves) {
        const int64_t row = tile * 32 + (lane & 31);
        const bool valid = row < m;
        bf8 x0;
        bool bad;
        load_inputs(feat, row, valid, lane, x0, bad);
        f16v a[2];
        bf8 x[4];
        layer<1>(pk + PK_FWD1, w + OB1, &x0, lane, a);
        relu_to_operands(a, x);
        layer<4>(pk + PK_FWD2, w + OB2, x, lane, a);
        relu_to_operands(a, x);
        layer<4>(pk + PK_FWD3, w + OB3, x, lane, a);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int j = 0; j < 16; ++j) a[t][j] = relu(a[t][j]);
        const float y = out_layer(w, a, lane);
        bad |= __shfl_xor((int)bad, 32, 64) != 0;
        if (valid && lane < 32) out[row] = bad ? NAN : y;
    }
}

// ---- training -----------------------------------------------------------------
constexpr int GW = 4;                 // wavefronts per workgroup
constexpr int GROWS = 32 * GW;        // batch rows per workgroup
constexpr int NSLOT = NPARAM + 1;     // gradient + squared-error sum

// Store the lane's 32 accumulator entries (one per hidden unit, of its row)
// as BF16 into a [64 units][32 rows] tile in LDS.
__device__ __forceinline__ void stash(const f16v a[2], uint16_t* tile, int lane) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 16; ++j) tile[(32 * t + acc_row(j, lane)) * 32 + (lane & 31)] = bf16_bits(a[t][j]);
}

// dW^T[out][in] += sum over the tile's 32 rows of delta[out][row] act[in][row]
// (MFMA with the rows as the K dimension, slot s of lane half h in k-block
// kb = row 16 kb + 8 h + s), added into the LDS gradient at W[in][out];
// inputs in >= nin are skipped.
__device__ __forceinline__ void weight_grad(const uint16_t* dl, const uint16_t* ac, int nin, float* gw, int lane) {
    const int half = lane >> 5, l32 = lane & 31;
    const int ntin = (nin + 31) / 32;
#pragma unroll
    for (int t = 0; t < 2; ++t)
        for (int u = 0; u < ntin; ++u) {
            f16v acc;
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[j] = 0.f;
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const bf8 a = *reinterpret_cast<const bf8*>(dl + (32 * t + l32) * 32 + 16 * kb + 8 * half);
                const bf8 b = *reinterpret_cast<const bf8*>(ac + (32 * u + l32) * 32 + 16 * kb + 8 * half);
                acc = mfma(a, b, acc);
            }
            const int in = 32 * u + l32;
            if (in < nin)
#pragma unroll
                for (int j = 0; j < 16; ++j) atomicAdd(&gw[in * H + 32 * t + acc_row(j, lane)], acc[j]);
        }
}

__device__ __forceinline__ void bias_grad(const f16v d[2], float* gb, int lane, bool valid) {
    if (!valid) return;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 16; ++j) atomicAdd(&gb[32 * t + acc_row(j, lane)], d[t][j]);
}

// Gradient of the mean squared error over a batch of m rows (rows[] picks
// them from feat/target, or rows 0..m-1): each workgroup takes 128-row tiles
// and writes its partial sums (and its squared-error sum) to part[blockIdx].
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ w, const bf8* __restrict__ pk, int64_t m,
                                                  const uint16_t* __restrict__ feat, const int32_t* __restrict__ rows,
                                                  const float* __restrict__ target, float* __restrict__ part) {
    __shared__ float gacc[NSLOT];
    __shared__ uint16_t dl_all[GW][H * 32];
    __shared__ uint16_t ac_all[GW][H * 32];
    for (int k = threadIdx.x; k < NSLOT; k += blockDim.x) gacc[k] = 0.f;
    __syncthreads();
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    uint16_t* dl = dl_all[wv];
    uint16_t* ac = ac_all[wv];
    const float inv_m = 1.f / (float)m;
    // workgroups stride over 128-row tiles, so the partial sums stay one
    // slot vector per workgroup whatever the batch size
    for (int64_t tile = blockIdx.x; tile * GROWS < m; tile += gridDim.x) {
        const int64_t b = tile * GROWS + 32 * wv + (lane & 31);
        const bool valid = b < m;
        const int64_t row = valid ? (rows ? (int64_t)rows[b] : b) : 0;

        bf8 x0;
        bool bad;
        load_inputs(feat, row, valid, lane, x0, bad);
        f16v h1[2], h2[2], h3[2];
        bf8 x1[4], x2[4];
        layer<1>(pk + PK_FWD1, w + OB1, &x0, lane, h1);
        relu_to_operands(h1, x1);
        layer<4>(pk + PK_FWD2, w + OB2, x1, lane, h2);
        relu_to_operands(h2, x2);
        layer<4>(pk + PK_FWD3, w + OB3, x2, lane, h3);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int j = 0; j < 16; ++j) h3[t][j] = relu(h3[t][j]);
        const float y = out_layer(w, h3, lane);
        const float r = valid ? y - target[row] : 0.f;
        const float gout = 2.f * r * inv_m;              // d loss / d output of this row
        if (valid && lane < 32) {
            atomicAdd(&gacc[NPARAM], r * r);
            atomicAdd(&gacc[OB4], gout);
        }
        // layer 4 and the error at the pre-activations of layer 3
        f16v d3[2];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int u = 32 * t + acc_row(j, lane);
                if (valid) atomicAdd(&gacc[OW4 + u], gout * h3[t][j]);
                d3[t][j] = h3[t][j] > 0.f ? gout * w[OW4 + u] : 0.f;
            }
        bias_grad(d3, gacc + OB3, lane, valid);
        // W3: delta3 x h2
        stash(d3, dl, lane);
        stash(h2, ac, lane);
        __builtin_amdgcn_wave_barrier();
        weight_grad(dl, ac, H, gacc + OW3, lane);
        // delta2 = (W3 delta3) * [h2 > 0]
        bf8 xd[4];
        to_operands(d3, xd);
        f16v d2[2];
        layer<4>(pk + PK_BWD3, nullptr, xd, lane, d2);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int j = 0; j < 16; ++j) d2[t][j] = h2[t][j] > 0.f ? d2[t][j] : 0.f;
        bias_grad(d2, gacc + OB2, lane, valid);
        __builtin_amdgcn_wave_barrier();
        stash(d2, dl, lane);
        stash(h1, ac, lane);
        __builtin_amdgcn_wave_barrier();
        weight_grad(dl, ac, H, gacc + OW2, lane);
        // delta1 = (W2 delta2) * [h1 > 0]
        f16v d1[2];
        to_operands(d2, xd);
        layer<4>(pk + PK_BWD2, nullptr, xd, lane, d1);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int j = 0; j < 16; ++j) d1[t][j] = h1[t][j] > 0.f ? d1[t][j] : 0.f;
        bias_grad(d1, gacc + OB1, lane, valid);
        __builtin_amdgcn_wave_barrier();
        stash(d1, dl, lane);
        // the inputs as a [16][32] tile (rows of absent batch entries are zero)
        for (int j = 0; j < 4; ++j) {
            ac[(4 * (lane >> 5) + j) * 32 + (lane & 31)] = (uint16_t)x0[j];
            ac[(8 + 4 * (lane >> 5) + j) * 32 + (lane & 31)] = (uint16_t)x0[4 + j];
        }
        __builtin_amdgcn_wave_barrier();
        // inputs 16..31 of the B tile read the next rows of ac, but only inputs
        // < 12 are kept (MFMA output columns do not mix)
        weight_grad(dl, ac, NF, gacc + OW1, lane);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    float* dst = part + (int64_t)blockIdx.x * NSLOT;
    for (int k = threadIdx.x; k < NSLOT; k += blockDim.x) dst[k] = gacc[k];
}

// Sum of the workgroup partials, in workgroup order (deterministic).
__device__ __forceinline__ float part_sum(const float* __restrict__ part, int nwg, int k) {
    float s = 0.f;
    for (int g = 0; g < nwg; ++g) s += part[(int64_t)g * NSLOT + k];
    return s;
}

__global__ void k_mlp_reduce(const float* __restrict__ part, int nwg, int64_t m, float* __restrict__ grad,
                             float* __restrict__ loss) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < NPARAM && grad) grad[k] = part_sum(part, nwg, k);
    if (k == NPARAM && loss) *loss = part_sum(part, nwg, NPARAM) / (float)m;
}

__global__ void k_mlp_adam(const float* __restrict__ part, int nwg, int64_t m, float* __restrict__ w,
                           float* __restrict__ st, vr_adam_params ap, int step, float* __restrict__ loss) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == NPARAM && loss) *loss = part_sum(part, nwg, NPARAM) / (float)m;
    if (k >= NPARAM) return;
    const float g = part_sum(part, nwg, k);
    float* m1 = st;
    float* m2 = st + NPARAM;
    const float a = ap.beta1 * m1[k] + (1.f - ap.beta1) * g;
    const float b = ap.beta2 * m2[k] + (1.f - ap.beta2) * g * g;
    m1[k] = a;
    m2[k] = b;
    const float c1 = 1.f - powf(ap.beta1, (float)step), c2 = 1.f - powf(ap.beta2, (float)step);
    w[k] -= ap.lr * (a / c1) / (sqrtf(b / c2) + ap.eps);
}

// ---- band selection ---------------------------------------------------------------
__global__ void k_rs_band(int64_t m, const int32_t* __restrict__ mem, const float* __restrict__ rhat, float thr,
                          float margin, float* __restrict__ R, uint32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const float r = rhat[i];
    R[mem[i]] = r;
    flag[i] = (!isfinite(r) || fabsf(r - thr) < margin) ? 1u : 0u;
}

__global__ void k_rs_compact(int64_t m, const int32_t* __restrict__ mem, const uint32_t* __restrict__ flag,
                             const uint32_t* __restrict__ pos, int32_t* __restrict__ subset) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m || !flag[i]) return;
    subset[pos[i]] = mem[i];
}

int check_mlp(vr_ctx* ctx, const void* w, int64_t m, const uint16_t* feat) {
    if (!w) return set_err(ctx, VR_ERR_INVALID_ARG, "weights are NULL");
    if (m < 0 || m >= (int64_t(1) << 31)) return set_err(ctx, VR_ERR_INVALID_ARG, "m out of range");
    if (m > 0 && !feat) return set_err(ctx, VR_ERR_INVALID_ARG, "features are NULL");
    return VR_OK;
}

int pack_weights(vr_ctx* ctx, const float* w, bf8** out, hipStream_t st) {
    VR_WS(pk, ctx, bf8, WS_B9, PK_TOTAL);
    hipLaunchKernelGGL(k_mlp_pack, dim3(grid_for(PK_TOTAL, 256)), dim3(256), 0, st, w, pk);
    VR_LAUNCH_CHECK(ctx);
    *out = pk;
    return VR_OK;
}

int run_grad(vr_ctx* ctx, const float* w, int64_t m, const uint16_t* feat, const int32_t* rows,
             const float* target, float** part_out, int* nwg_out, hipStream_t st) {
    bf8* pk = nullptr;
    int rc = pack_weights(ctx, w, &pk, st);
    if (rc) return rc;
    const int nwg = (int)std::min<int64_t>((m + GROWS - 1) / GROWS, (int64_t)ctx->num_cus * 2);
    VR_WS(part, ctx, float, WS_B8, (size_t)nwg * NSLOT);
    VR_TIMED(ctx, "mlp_grad", st, m,
             hipLaunchKernelGGL(k_mlp_grad, dim3(nwg), dim3(64 * GW), 0, st, w, pk, m, feat, rows, target, part));
    VR_LAUNCH_CHECK(ctx);
    *part_out = part;
    *nwg_out = nwg;
    return VR_OK;
}

}  // namespace
}  // namespace vr

using namespace vr;

extern "C" {

int vr_rs_features(vr_ctx* ctx, const vr_particles* p, int32_t n_hosts, const int32_t* host_offsets,
                   const int32_t* host_members, const float* vbar, const float* sigma, const float* rho_cell,
                   int32_t n_se, int32_t cell_bits, const float* shift, const float* scale, uint16_t* feat,
                   int64_t* n_rows, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_particles(ctx, p, true);
    if (rc) return rc;
    if ((rc = check_hosts(ctx, n_hosts, host_offsets, host_members))) return rc;
    if (n_se < 1) return set_err(ctx, VR_ERR_INVALID_ARG, "n_se must be positive");
    if (cell_bits < 0 || cell_bits + 4 > p->grid_bits)
        return set_err(ctx, VR_ERR_INVALID_ARG, "cell_bits must be in [0, grid_bits - 4] (coarse grid >= 4 cells)");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    int32_t m32 = 0;
    if (n_hosts > 0) {
        rc = read_back(ctx, host_offsets + n_hosts, &m32, sizeof m32, st);
        if (rc) return rc;
    }
    if (n_rows) *n_rows = m32;
    const int64_t m = m32;
    if (m == 0) return VR_OK;
    if (!vbar || !sigma || !rho_cell || !feat) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    FeatNorm nrm;
    for (int k = 0; k < NF; ++k) {
        nrm.shift[k] = shift ? shift[k] : 0.f;
        nrm.scale[k] = scale ? scale[k] : 1.f;
    }
    Level lv[2];
    const int cb[2] = {cell_bits, cell_bits + 2};
    double* vsum = nullptr;
    const uint32_t* order = nullptr;
    const uint32_t* head0 = nullptr;
    const uint32_t* cid0 = nullptr;
    const uint64_t* keys0 = nullptr;
    const uint64_t* keys1 = nullptr;
    uint32_t ncell[2] = {0, 0};
    for (int L = 0; L < 2; ++L) {
        const int b = p->grid_bits - cb[L];
        VR_WS(keys, ctx, uint64_t, WS_A0 + 4 * L, m);
        VR_WS(rws, ctx, uint32_t, WS_A1 + 4 * L, m);
        VR_WS(flag, ctx, uint32_t, WS_A2 + 4 * L, m);
        VR_WS(cid, ctx, uint32_t, WS_A3 + 4 * L, m);
        uint64_t* kin;
        uint32_t* rin;
        if ((rc = sort_input_u64(ctx, keys, rws, m, 3 * b, &kin, &rin))) return rc;
        hipLaunchKernelGGL(k_rs_keys, dim3(grid_for(m, 256)), dim3(256), 0, st, m, host_members, p->qx, p->qy, p->qz,
                           cb[L], b, kin, rin);
        VR_LAUNCH_CHECK(ctx);
        if ((rc = sort_pairs_u64_from(ctx, kin, rin, keys, rws, m, 3 * b, st))) return rc;
        hipLaunchKernelGGL(k_rs_heads, dim3(grid_for(m, 256)), dim3(256), 0, st, m, keys, flag);
        VR_LAUNCH_CHECK(ctx);
        uint32_t* tot = reinterpret_cast<uint32_t*>(ctx->pinned);
        VR_WS(totd, ctx, uint32_t, WS_FLAG, 4);
        if ((rc = scan_u32(ctx, flag, cid, m, totd, st))) return rc;
        if ((rc = read_back(ctx, totd, tot, sizeof(uint32_t), st))) return rc;
        const uint32_t ncells = *tot;
        VR_WS(start, ctx, uint32_t, WS_B0 + 3 * L, (size_t)ncells + 1);
        hipLaunchKernelGGL(k_rs_starts, dim3(grid_for(m, 256)), dim3(256), 0, st, m, flag, cid, start, ncells);
        VR_LAUNCH_CHECK(ctx);
        uint32_t hsize = 64;
        while (hsize < 2u * ncells) hsize <<= 1;
        VR_WS(hk, ctx, unsigned long long, WS_B1 + 3 * L, hsize);
        VR_WS(hv, ctx, uint32_t, WS_B2 + 3 * L, hsize);
        hipLaunchKernelGGL(k_rs_clear, dim3(grid_for(hsize, 256)), dim3(256), 0, st, hk, hsize);
        VR_LAUNCH_CHECK(ctx);
        hipLaunchKernelGGL(k_rs_insert, dim3(grid_for(ncells, 256)), dim3(256), 0, st, ncells, keys, start, hsize - 1,
                           hk, hv);
        VR_LAUNCH_CHECK(ctx);
        lv[L] = Level{hk, hv, hsize - 1, start, cb[L], b};
        ncell[L] = ncells;
        if (L == 1) keys1 = keys;
        if (L == 0) {
            head0 = flag;
            cid0 = cid;
            keys0 = keys;
            VR_WS(vs, ctx, double, WS_B6, 3 * (size_t)ncells);
            hipLaunchKernelGGL(k_rs_vsum, dim3(grid_for(ncells, 256)), dim3(256), 0, st, ncells, start, rws,
                               host_members, p->vx, p->vy, p->vz, vs);
            VR_LAUNCH_CHECK(ctx);
            vsum = vs;
            order = rws;
        }
    }
    const double cell_len = ldexp(p->box, cell_bits - p->grid_bits);
    VR_WS(cf, ctx, double, WS_C0, 4 * (size_t)ncell[0]);
    VR_WS(cwin, ctx, uint32_t, WS_C1, (size_t)ncell[1]);
    VR_TIMED(ctx, "rs_features", st, 0,
             hipLaunchKernelGGL(k_rs_coarsewin, dim3(grid_for(ncell[1], 256)), dim3(256), 0, st, ncell[1], keys1, lv[1],
                                cwin));
    VR_LAUNCH_CHECK(ctx);
    VR_TIMED(ctx, "rs_features", st, 0,
             hipLaunchKernelGGL(k_rs_cellfeat, dim3(grid_for(ncell[0], 256)), dim3(256), 0, st, ncell[0], keys0, lv[0],
                                lv[1], cwin, vsum, n_se, cell_len, cf));
    VR_LAUNCH_CHECK(ctx);
    VR_TIMED(ctx, "rs_features", st, m,
             hipLaunchKernelGGL(k_rs_features, dim3(grid_for(m, 256)), dim3(256), 0, st, m, host_members, p->vx, p->vy,
                                p->vz, vbar, sigma, rho_cell, p->n, head0, cid0, cf, nrm, order, feat));
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

int vr_mlp_forward(vr_ctx* ctx, const float* weights, int64_t m, const uint16_t* feat, float* Rhat, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_mlp(ctx, weights, m, feat);
    if (rc) return rc;
    if (m == 0) return VR_OK;
    if (!Rhat) return set_err(ctx, VR_ERR_INVALID_ARG, "Rhat is NULL");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    bf8* pk = nullptr;
    if ((rc = pack_weights(ctx, weights, &pk, st))) return rc;
    const int64_t ntiles = (m + 31) / 32;
    const int64_t want = (ntiles + 3) / 4;
    const unsigned grid = (unsigned)std::min<int64_t>(want, (int64_t)ctx->num_cus * 8);
    VR_TIMED(ctx, "mlp_forward", st, m,
             hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(256), 0, st, weights, pk, m, feat, Rhat));
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

int vr_mlp_grad(vr_ctx* ctx, const float* weights, int64_t m, const uint16_t* feat, const int32_t* rows,
                const float* target, float* grad, float* loss, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_mlp(ctx, weights, m, feat);
    if (rc) return rc;
    if (m == 0) return set_err(ctx, VR_ERR_INVALID_ARG, "empty batch");
    if (!target || !grad) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL target or grad");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    float* part = nullptr;
    int nwg = 0;
    if ((rc = run_grad(ctx, weights, m, feat, rows, target, &part, &nwg, st))) return rc;
    hipLaunchKernelGGL(k_mlp_reduce, dim3(grid_for(NSLOT, 256)), dim3(256), 0, st, part, nwg, m, grad, loss);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

int vr_mlp_train_step(vr_ctx* ctx, float* weights, float* adam_state, int64_t m, const uint16_t* feat,
                      const int32_t* rows, const float* target, const vr_adam_params* ap, int32_t step, float* loss,
                      void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    int rc = check_mlp(ctx, weights, m, feat);
    if (rc) return rc;
    if (m == 0) return set_err(ctx, VR_ERR_INVALID_ARG, "empty batch");
    if (!target || !adam_state || !ap) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL target, state or params");
    if (step < 1) return set_err(ctx, VR_ERR_INVALID_ARG, "step counts from 1");
    if (!(ap->lr > 0) || !(ap->beta1 >= 0 && ap->beta1 < 1) || !(ap->beta2 >= 0 && ap->beta2 < 1) || !(ap->eps > 0))
        return set_err(ctx, VR_ERR_INVALID_ARG, "bad Adam parameters");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    float* part = nullptr;
    int nwg = 0;
    if ((rc = run_grad(ctx, weights, m, feat, rows, target, &part, &nwg, st))) return rc;
    hipLaunchKernelGGL(k_mlp_adam, dim3(grid_for(NSLOT, 256)), dim3(256), 0, st, part, nwg, m, weights, adam_state,
                       *ap, step, loss);
    VR_LAUNCH_CHECK(ctx);
    return VR_OK;
}

int vr_rs_select(vr_ctx* ctx, int64_t m, const int32_t* members, const float* Rhat, float R_threshold, float margin,
                 float* R, int32_t* subset, int64_t* n_subset, void* stream) {
    if (!ctx || !n_subset) return VR_ERR_INVALID_ARG;
    if (m < 0 || m >= (int64_t(1) << 31)) return set_err(ctx, VR_ERR_INVALID_ARG, "m out of range");
    if (!(margin >= 0)) return set_err(ctx, VR_ERR_INVALID_ARG, "margin must be >= 0");
    *n_subset = 0;
    if (m == 0) return VR_OK;
    if (!members || !Rhat || !R || !subset) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL array");
    VR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    VR_WS(flag, ctx, uint32_t, WS_A0, m);
    VR_WS(pos, ctx, uint32_t, WS_A1, m);
    VR_WS(tot, ctx, uint32_t, WS_FLAG, 4);
    hipLaunchKernelGGL(k_rs_band, dim3(grid_for(m, 256)), dim3(256), 0, st, m, members, Rhat, R_threshold, margin, R,
                       flag);
    VR_LAUNCH_CHECK(ctx);
    int rc = scan_u32(ctx, flag, pos, m, tot, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_rs_compact, dim3(grid_for(m, 256)), dim3(256), 0, st, m, members, flag, pos, subset);
    VR_LAUNCH_CHECK(ctx);
    uint32_t cnt = 0;
    if ((rc = read_back(ctx, tot, &cnt, sizeof cnt, st))) return rc;
    *n_subset = cnt;
    return VR_OK;
}

}  // extern "C"
