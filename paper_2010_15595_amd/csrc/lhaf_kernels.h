// Internal launch interface between the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbs {

constexpr int kMaxPairs = 32;       // n = N / 2 <= 32 (N <= 64)
constexpr int kBinomStride = 33;    // binomial table C(a, b), 0 <= a, b <= 32

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
    double2* Eout;         // count * 2 * (D + 1)
};

// Phase 2: one lane per subset; signed terms, compensated block partials.
struct LaunchPhase2 {
    const double2* E;
    uint64_t count;
    int D;
    double sign;        // (-1)^(n - s)
    int per_thread;     // subsets per lane
    double* partials;   // 5 doubles per block
    double2* terms;     // optional per-subset terms
};

// Lane grids of the per-subset kernel (rows x columns of lanes per subset).
enum { kLayout44 = 0, kLayout84 = 1, kLayout88 = 2, kNumLayouts = 3 };
bool charpoly_layout_ok(int m, int layout);
int charpoly_default_layout(int m);
hipError_t launch_charpoly(const LaunchPhase1& p, int layout, hipStream_t st);
hipError_t launch_series(int n, const LaunchPhase2& p, hipStream_t st);
hipError_t launch_final_reduce(const double* partials, int64_t np, double2* out, double* abs_out, hipStream_t st);
hipError_t launch_prep(const double2* A, int N, int64_t lda, int Np, double2* A0, double2* d, hipStream_t st);
hipError_t launch_scalar_set(double2* out, double2 v, double* abs_out, double a, hipStream_t st);
hipError_t launch_selftest(const double* in, double* out, hipStream_t st);

}  // namespace gbs
