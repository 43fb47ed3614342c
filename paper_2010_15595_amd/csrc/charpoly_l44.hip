// Per-subset kernel instantiations for the 4 x 4 lanes per subset, four subsets per wavefront; MR = MC = ceil(m / 4).
#include <algorithm>

#include "lhaf_device.h"

namespace gbs {

template <int P, int Q, int MR, int MC>
static hipError_t launch_charpoly_t(const LaunchPhase1& p, hipStream_t st) {
    constexpr int G = P * Q;
    constexpr int W = 64 / G;
    const int T = (G >= p.D + 1) ? G : 64;
    const unsigned grid = (unsigned)((p.count + W - 1) / W);
    if (p.fp32) {
        const size_t lds = charpoly_lds_bytes(W, 64 / T, p.D, sizeof(float2));
        hipLaunchKernelGGL((charpoly_kernel<P, Q, MR, MC, float2>), dim3(grid), dim3(64), lds, st, p.A0, p.dvec, p.Np,
                           p.s, p.rank0, p.count, p.masks, p.binom, p.D, T, static_cast<float2*>(p.Eout));
    } else {
        const size_t lds = charpoly_lds_bytes(W, 64 / T, p.D, sizeof(double2));
        hipLaunchKernelGGL((charpoly_kernel<P, Q, MR, MC, double2>), dim3(grid), dim3(64), lds, st, p.A0, p.dvec,
                           p.Np, p.s, p.rank0, p.count, p.masks, p.binom, p.D, T, static_cast<double2*>(p.Eout));
    }
    return hipGetLastError();
}

hipError_t launch_charpoly_l44(const LaunchPhase1& p, hipStream_t st) {
    const int m = 2 * p.s;
    switch ((m + 3) / 4) {
        case 1: return launch_charpoly_t<4, 4, 1, 1>(p, st);
        case 2: return launch_charpoly_t<4, 4, 2, 2>(p, st);
        case 3: return launch_charpoly_t<4, 4, 3, 3>(p, st);
        case 4: return launch_charpoly_t<4, 4, 4, 4>(p, st);
        case 5: return launch_charpoly_t<4, 4, 5, 5>(p, st);
        case 6: return launch_charpoly_t<4, 4, 6, 6>(p, st);
    }
    return hipErrorInvalidValue;
}


template <int P, int Q, int MR, int MC>
static hipError_t launch_charpoly_batch_t(int D_max, int fp32, const BatchTile* tiles, int ntiles,
                                          const BatchItem* items, const uint64_t* binom, unsigned* counter,
                                          void* Ebase, int grid, hipStream_t st) {
    constexpr int G = P * Q;
    constexpr int W = 64 / G;
    // tiles with D + 1 <= G use W teams of G lanes (ring <= G x G), others one
    // team of 64 lanes; allocate the larger of the two layouts
    auto lds_for = [&](size_t vb) {
        const size_t a = charpoly_lds_bytes(W, W, std::min(D_max, G - 1), (int)vb);
        const size_t b = charpoly_lds_bytes(W, 1, D_max, (int)vb);
        return a > b ? a : b;
    };
    if (fp32) {
        const size_t lds = lds_for(sizeof(float2));
        hipLaunchKernelGGL((charpoly_batch_kernel<P, Q, MR, MC, float2>), dim3(grid), dim3(64), lds, st, tiles, ntiles,
                           items, binom, counter, static_cast<float2*>(Ebase));
    } else {
        const size_t lds = lds_for(sizeof(double2));
        hipLaunchKernelGGL((charpoly_batch_kernel<P, Q, MR, MC, double2>), dim3(grid), dim3(64), lds, st, tiles,
                           ntiles, items, binom, counter, static_cast<double2*>(Ebase));
    }
    return hipGetLastError();
}

hipError_t launch_charpoly_batch_l44(int s_rep, int D_max, int fp32, const BatchTile* tiles, int ntiles,
                                      const BatchItem* items, const uint64_t* binom, unsigned* counter, void* Ebase,
                                      int grid, hipStream_t st) {
    const int m = 2 * s_rep;
    switch ((m + 3) / 4) {
        case 1: return launch_charpoly_batch_t<4, 4, 1, 1>(D_max, fp32, tiles, ntiles, items, binom, counter, Ebase, grid, st);
        case 2: return launch_charpoly_batch_t<4, 4, 2, 2>(D_max, fp32, tiles, ntiles, items, binom, counter, Ebase, grid, st);
        case 3: return launch_charpoly_batch_t<4, 4, 3, 3>(D_max, fp32, tiles, ntiles, items, binom, counter, Ebase, grid, st);
        case 4: return launch_charpoly_batch_t<4, 4, 4, 4>(D_max, fp32, tiles, ntiles, items, binom, counter, Ebase, grid, st);
        case 5: return launch_charpoly_batch_t<4, 4, 5, 5>(D_max, fp32, tiles, ntiles, items, binom, counter, Ebase, grid, st);
        case 6: return launch_charpoly_batch_t<4, 4, 6, 6>(D_max, fp32, tiles, ntiles, items, binom, counter, Ebase, grid, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace gbs
