// Internal launch interface between the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace gbs {

constexpr int kMaxPairs = 32;       // n = N / 2 <= 32 (N <= 64)
constexpr int kBinomStride = 33;    // binomial table C(a, b), 0 <= a, b <= 32

// Offset of C (m x m, m even) in the P MR x Q MC register tile of a
// single-evaluation launch (MC = ceil(m / Q)): tiles of three or more local
// columns put their spare rows and columns in front (offset 2, 4 or 6 on
// 8-column grids, 2 on 4-column grids), which shortens the first Householder
// phase; smaller tiles, and every batch launch, keep them behind (offset 0).
// The offsets of two tile shapes stay 0 because those instances would spill
// registers: offset 2 with seven local columns on 8-column grids, and any
// offset with nine or ten local columns on 4-column grids.
__host__ __device__ constexpr bool charpoly_offset_ok(int Q, int MC, int o) {
    return o >= 0 && o < Q && (o == 0 || MC >= 3) && !(Q == 8 && MC == 7 && o == 2) && !(Q == 4 && MC >= 9 && o != 0);
}
__host__ __device__ constexpr int charpoly_front_offset(int P, int Q, int MR, int MC, int m) {
    const int o = (MC >= 3) ? ((P * MR < Q * MC ? P * MR : Q * MC) - m) : 0;
    return charpoly_offset_ok(Q, MC, o) ? o : 0;
}

// Largest subset matrix (m = 2s) the register-tile kernels take.  An 8 x 8
// tile of complex values per lane (m = 57..64) does not fit the register file
// without scratch spills; those subsets, at most C(32, 29) + C(32, 30) +
// C(32, 31) + 1 = 5489 of the 2^32 of an N = 64 loop hafnian, run on the
// LDS-resident FP64 kernel (launch_charpoly_lds) instead, and batch plans
// take items up to N = kMaxTileM.
constexpr int kMaxTileM = 56;
// Largest m on the 8 x 4 grid inside batch plans (its nine- and ten-column
// persistent instances spill).
constexpr int kMaxBatchM84 = 32;
// Subsets per launch of a single evaluation (one size class is split into
// launches of at most this many).  Larger launches spend less of their time in
// the partly empty last round of wavefronts and between launches; the
// coefficient buffer holds 2 (D + 1) complex values per subset (0.9 GB at
// N = 50, FP64).
constexpr uint64_t kSubsetsPerLaunch = 1ull << 20;

// Phase 1: one wavefront per pair subset of size s; writes, per subset, the
// D + 1 leading coefficients of det(xI - C) then of det(xI - C').
struct LaunchPhase1 {
    const double2* A0;     // Np x Np, zero diagonal
    const double2* dvec;   // Np loop weights
    int Np;                // even dimension
    int s;                 // subset size (1..n)
    uint64_t rank0;        // first colex rank (ignored when masks != nullptr)
    uint64_t count;        // subsets in this launch
    const uint64_t* masks; // explicit subset masks or nullptr
    const uint64_t* binom; // device binomial table
    int D;                 // n + 1
    void* Eout;            // count * 2 * (D + 1) complex (double2, or float2 when fp32)
    int fp32;              // La Budde in complex FP32
    const int4* lbmap;     // La Budde lane maps of every (team width, D) (lb_fill_table)
};

// Phase 2: one lane per subset; signed terms, compensated block partials.
struct LaunchPhase2 {
    const void* E;         // double2, or float2 when fp32
    int fp32;              // series and per-lane compensated sums in FP32
    uint64_t count;
    int D;
    double sign;        // (-1)^(n - s)
    int per_thread;     // subsets per lane
    double* partials;   // 5 doubles per block
    double2* terms;     // optional per-subset terms
};

// Lane grids of the per-subset kernel (rows x columns of lanes per subset).
// kLayout84T: the 8 x 4 grid with one 64-lane La Budde team serving both
// subsets of the wavefront in turn (half the LDS of two 32-lane teams).
enum { kLayout44 = 0, kLayout84 = 1, kLayout88 = 2, kLayout84T = 3, kNumLayouts = 4 };
bool charpoly_layout_ok(int m, int layout);
int charpoly_default_layout(int m);
hipError_t launch_charpoly(const LaunchPhase1& p, int layout, hipStream_t st);

// ---- batches of loop hafnians ----
struct BatchItem {
    const double2* A0;     // Np x Np, zero diagonal
    const double2* dvec;   // Np
    int Np, n;
};
// A run of `count` subsets of size s of one item, colex ranks rank0.. ;
// coefficients at Ebase + eoff (elements of the path's complex type).
struct BatchTile {
    uint64_t rank0;
    uint64_t count;
    uint64_t eoff;
    int item, s;
};
// One series block: up to 64 * per_thread subsets of a tile starting at sub0.
struct SeriesBlock {
    int tile;
    int pidx;
    uint64_t sub0;
};

// Persistent per-subset kernel over tiles that all use grid `layout` with the
// same (MR, MC) as subsets of size s_rep, the same La Budde team variant and C
// at tile offset `offset` (charpoly_front_offset of their m; 0 on the FP32
// path); D_max sizes the LDS.  The launch has as many wavefronts as the device
// holds at once for that kernel and LDS size (persistent_grid), at most
// max_grid.
hipError_t launch_charpoly_batch(int layout, int s_rep, int variant, int offset, int D_max, int fp32,
                                 const BatchTile* tiles, int ntiles, const BatchItem* items, const uint64_t* binom,
                                 const int4* lbmap, unsigned* counter, void* Ebase, int max_grid, hipStream_t st);

// Wavefronts (64-thread workgroups) of a persistent launch of `kernel` with
// `lds` bytes of dynamic LDS: the occupancy limit per CU (registers and LDS)
// times the CUs of the current device, at most max_grid and at least 1.
template <class K>
inline int persistent_grid(K kernel, size_t lds, int max_grid) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, lds) != hipSuccess || per_cu < 1) per_cu = 8;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    const long long g = (long long)per_cu * cus;
    return (int)std::max<long long>(1, std::min<long long>(g, max_grid));
}
// Kernel instance id (layout, MR, MC) of subsets of size s under `layout`.
int charpoly_instance(int layout, int s);
// La Budde team variant (0: teams of P Q lanes, 1: one team of 64 lanes) of an
// n-pair loop hafnian under `layout`.
int charpoly_variant(int layout, int n);
// La Budde lane maps for team widths 16, 32, 64 and D = 0..kMaxPairs+1:
// kLbTableEntries int4 (d, g, first k, last k) per team lane, d = -1 idle.
constexpr int kLbTableEntries = 3 * (kMaxPairs + 2) * 64;
void lb_fill_table(int4* out);
hipError_t launch_series_batch(int n, int fp32, const SeriesBlock* blocks, int nblocks, const BatchTile* tiles,
                               const BatchItem* items, const void* Ebase, int per_thread, double* partials,
                               hipStream_t st);
// Per-item fixed-order reduction of the partials; items with pairs but no
// partials (summed by launch_small_items) are left alone.
hipError_t launch_item_reduce(const int64_t* pbeg, int nitems, const double* partials, const BatchItem* items,
                              double2* out, double* abs_out, hipStream_t st);
// Whole loop hafnians of 1 <= n <= kSmallPairs pairs, one wavefront each
// (FP64): list holds the item indices, largest n first.
constexpr int kSmallPairs = 8;
hipError_t launch_small_items(const int* list, int count, const BatchItem* items, const uint64_t* binom,
                              const int4* lbmap, double2* out, double* abs_out, int grid, hipStream_t st);
hipError_t launch_batch_prep(const double2* mats, const int64_t* in_off, const int* N, BatchItem* items, int nitems,
                             hipStream_t st);
hipError_t launch_fill_u32(unsigned* p, int count, hipStream_t st);

// ---- subset terms with the matrix in LDS (double-double path, method comparison) ----
enum { kCharpolyLaBudde = 0, kCharpolyEigen = 1 };
constexpr int kMaxDdPairs = 28;  // N <= 56: the (m+1)^2 matrix and the La Budde ring fit in LDS in double-double
size_t dd_lds_bytes(int m, int D);
size_t lds_bytes(int m, int D, int prec_dd, int method);
// Largest n for the arithmetic / method (0 = unsupported pair).
int lds_max_pairs(int prec_dd, int method);
// Bytes per subset term in the terms buffer (32 double-double, 16 FP64).
size_t lds_term_bytes(int prec_dd);
// One workgroup per subset of size s; terms receive the signed subset terms
// (NaN for a subset whose QR iteration did not converge).
hipError_t launch_charpoly_lds(int prec_dd, int method, const double2* A0, const double2* dvec, int Np, int s,
                               uint64_t rank0, uint64_t count, const uint64_t* masks, const uint64_t* binom, int D,
                               double sign, void* terms, hipStream_t st);
hipError_t launch_charpoly_dd(const double2* A0, const double2* dvec, int Np, int s, uint64_t rank0, uint64_t count,
                              const uint64_t* masks, const uint64_t* binom, int D, double sign, void* terms,
                              hipStream_t st);
// Fixed-order double-double sums: blocks of 64 * per terms into partials (5
// doubles: re.hi, re.lo, im.hi, im.lo, sum |t|), optionally the terms rounded to double.
hipError_t launch_lds_block_reduce(int prec_dd, const void* terms, uint64_t count, int per, double* partials,
                                   double2* terms_out, hipStream_t st);
hipError_t launch_dd_block_reduce(const void* terms, uint64_t count, int per, double* partials, double2* terms_out,
                                  hipStream_t st);
hipError_t launch_dd_final_reduce(const double* partials, int64_t np, double2* out_hi, double2* out_lo, double* abs_out,
                                  hipStream_t st);

// ---- conditional sampling chain (Sec. III) ----
constexpr int kMaxSamplerModes = 128;  // modes of a sampled state
constexpr int kMaxCutoff = 64;         // photon-number cutoff per mode

// One lockstep step k (1-based) of the chain over nsamples samples: item
// b * (cutoff + 1) + j of the batch is the loop-hafnian matrix of pattern
// (s_1, .., s_{k-1}, j) of sample b's conditional state of modes 1..k.
struct SamplerStep {
    int M, k, cutoff, nsamples;
    const double2* Bk;      // k x k, B of the conditional state (heterodyne outcomes of modes k+1..M)
    const double2* ck;      // k: loop weights at zero outcome
    const double2* Fk;      // k x 2(M - k): gain of the loop weights on [beta_B; conj(beta_B)]
    const double2* beta;    // nsamples x (M - 1): outcomes of modes 2..M
    const int* samples;     // M x nsamples (mode-major): draws of modes 1..k-1
    const int64_t* in_off;  // per item: element offset of its matrix in mats
    const int* dims;        // per item: dimension
    double2* mats;          // packed matrices (output)
};
// beta[b * dim/2 + i] = x_i + i x_{dim/2 + i}, x = mean + L z_b, z_b = normals[b * dim ..]
hipError_t launch_heterodyne(const double* L, const double* mean, int dim, const double* normals, int nsamples,
                             double2* beta, hipStream_t st);
hipError_t launch_sampler_build(const SamplerStep& p, hipStream_t st);
// draw[b] from lh[b * (cutoff + 1) + j] and u[b]; probs (nullable) row b at probs + b * probs_stride.
hipError_t launch_sampler_draw(const double2* lh, int nsamples, int cutoff, const double* u, int* draw, double* probs,
                               int64_t probs_stride, hipStream_t st);
hipError_t launch_series(int n, const LaunchPhase2& p, hipStream_t st);
hipError_t launch_final_reduce(const double* partials, int64_t np, double2* out, double* abs_out, hipStream_t st);
// One partial record (5 doubles) from np records, same fixed order as launch_final_reduce.
hipError_t launch_partials_fold(const double* partials, int64_t np, double* record, hipStream_t st);
hipError_t launch_prep(const double2* A, int N, int64_t lda, int Np, double2* A0, double2* d, hipStream_t st);
hipError_t launch_scalar_set(double2* out, double2 v, double* abs_out, double a, hipStream_t st);
hipError_t launch_selftest(const double* in, double* out, hipStream_t st);

}  // namespace gbs
