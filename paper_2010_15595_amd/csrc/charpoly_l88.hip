// Per-subset kernel instantiations for the 8 x 8 lanes per subset, one subset per wavefront; MR = MC = ceil(m / 8).
#include <algorithm>

#include "lhaf_device.h"

namespace gbs {

template <int P, int Q, int MR, int MC, int TEAM, int O>
static hipError_t launch_charpoly_inst(const LaunchPhase1& p, hipStream_t st) {
    constexpr int W = 64 / (P * Q);
    const unsigned grid = (unsigned)((p.count + W - 1) / W);
    const int4* lbm = p.lbmap + lb_table_offset(TEAM, p.D);
    if (p.fp32) {
        const size_t lds = charpoly_lds_bytes(W, TEAM, p.D, sizeof(float2));
        hipLaunchKernelGGL((charpoly_kernel<P, Q, MR, MC, float2, TEAM, O>), dim3(grid), dim3(64), lds, st, p.A0, p.dvec,
                           p.Np, p.s, p.rank0, p.count, p.masks, p.binom, p.D, lbm, static_cast<float2*>(p.Eout));
    } else {
        const size_t lds = charpoly_lds_bytes(W, TEAM, p.D, sizeof(double2));
        hipLaunchKernelGGL((charpoly_kernel<P, Q, MR, MC, double2, TEAM, O>), dim3(grid), dim3(64), lds, st, p.A0, p.dvec,
                           p.Np, p.s, p.rank0, p.count, p.masks, p.binom, p.D, lbm, static_cast<double2*>(p.Eout));
    }
    return hipGetLastError();
}

// Tile offset of C (charpoly_front_offset): even, below Q.
template <int P, int Q, int MR, int MC, int TEAM>
static hipError_t launch_charpoly_team(const LaunchPhase1& p, hipStream_t st) {
    if constexpr (MC >= 3) {
        switch (charpoly_front_offset(P, Q, MR, MC, 2 * p.s)) {
            case 0: return launch_charpoly_inst<P, Q, MR, MC, TEAM, 0>(p, st);
            case 2: return launch_charpoly_inst<P, Q, MR, MC, TEAM, 2>(p, st);
            case 4:
                if constexpr (Q == 8) return launch_charpoly_inst<P, Q, MR, MC, TEAM, 4>(p, st);
                break;
            case 6:
                if constexpr (Q == 8) return launch_charpoly_inst<P, Q, MR, MC, TEAM, 6>(p, st);
                break;
        }
        return hipErrorInvalidValue;
    }
    return launch_charpoly_inst<P, Q, MR, MC, TEAM, 0>(p, st);
}

template <int P, int Q, int MR, int MC>
static hipError_t launch_charpoly_t(const LaunchPhase1& p, hipStream_t st) {
    constexpr int G = P * Q;
    if (lb_variant(G, p.D) == 0) {
        if constexpr (G < 64) return launch_charpoly_team<P, Q, MR, MC, G>(p, st);
        return hipErrorInvalidValue;
    }
    return launch_charpoly_team<P, Q, MR, MC, 64>(p, st);
}

hipError_t launch_charpoly_l88(const LaunchPhase1& p, hipStream_t st) {
    const int m = 2 * p.s;
    switch ((m + 7) / 8) {
        case 1: return launch_charpoly_t<8, 8, 1, 1>(p, st);
        case 2: return launch_charpoly_t<8, 8, 2, 2>(p, st);
        case 3: return launch_charpoly_t<8, 8, 3, 3>(p, st);
        case 4: return launch_charpoly_t<8, 8, 4, 4>(p, st);
        case 5: return launch_charpoly_t<8, 8, 5, 5>(p, st);
        case 6: return launch_charpoly_t<8, 8, 6, 6>(p, st);
        case 7: return launch_charpoly_t<8, 8, 7, 7>(p, st);
    }
    return hipErrorInvalidValue;
}


template <int P, int Q, int MR, int MC, int TEAM, int O>
static hipError_t launch_charpoly_batch_inst(int D_max, int fp32, const BatchTile* tiles, int ntiles,
                                             const BatchItem* items, const uint64_t* binom, const int4* lbmap,
                                             unsigned* counter, void* Ebase, int max_grid, hipStream_t st) {
    constexpr int W = 64 / (P * Q);
    // every tile of the launch has D <= D_max and the launch's team layout;
    // the LDS size is non-decreasing in D
    const int D = (TEAM < 64) ? std::min(D_max, TEAM - 1) : D_max;
    if (fp32) {
        if constexpr (O == 0) {  // FP32 batches keep C at offset 0
            const size_t lds = charpoly_lds_bytes(W, TEAM, D, sizeof(float2));
            const auto k = charpoly_batch_kernel<P, Q, MR, MC, float2, TEAM, 0>;
            hipLaunchKernelGGL(k, dim3(persistent_grid(k, lds, max_grid)), dim3(64), lds, st, tiles, ntiles, items,
                               binom, lbmap, counter, static_cast<float2*>(Ebase));
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        const size_t lds = charpoly_lds_bytes(W, TEAM, D, sizeof(double2));
        const auto k = charpoly_batch_kernel<P, Q, MR, MC, double2, TEAM, O>;
        hipLaunchKernelGGL(k, dim3(persistent_grid(k, lds, max_grid)), dim3(64), lds, st, tiles, ntiles, items, binom,
                           lbmap, counter, static_cast<double2*>(Ebase));
    }
    return hipGetLastError();
}

// Tile offset of C (charpoly_front_offset of the launch's m).
template <int P, int Q, int MR, int MC, int TEAM>
static hipError_t launch_charpoly_batch_team(int offset, int D_max, int fp32, const BatchTile* tiles, int ntiles,
                                             const BatchItem* items, const uint64_t* binom, const int4* lbmap,
                                             unsigned* counter, void* Ebase, int max_grid, hipStream_t st) {
    switch (offset) {
        case 0:
            return launch_charpoly_batch_inst<P, Q, MR, MC, TEAM, 0>(D_max, fp32, tiles, ntiles, items, binom, lbmap,
                                                                     counter, Ebase, max_grid, st);
        case 2:
            if constexpr (charpoly_offset_ok(Q, MC, 2))
                return launch_charpoly_batch_inst<P, Q, MR, MC, TEAM, 2>(D_max, fp32, tiles, ntiles, items, binom,
                                                                         lbmap, counter, Ebase, max_grid, st);
            break;
        case 4:
            if constexpr (charpoly_offset_ok(Q, MC, 4))
                return launch_charpoly_batch_inst<P, Q, MR, MC, TEAM, 4>(D_max, fp32, tiles, ntiles, items, binom,
                                                                         lbmap, counter, Ebase, max_grid, st);
            break;
        case 6:
            if constexpr (charpoly_offset_ok(Q, MC, 6))
                return launch_charpoly_batch_inst<P, Q, MR, MC, TEAM, 6>(D_max, fp32, tiles, ntiles, items, binom,
                                                                         lbmap, counter, Ebase, max_grid, st);
            break;
    }
    return hipErrorInvalidValue;
}

// Every tile of one launch has team variant `variant` (lb_variant of P Q and
// its D).
template <int P, int Q, int MR, int MC>
static hipError_t launch_charpoly_batch_t(int variant, int offset, int D_max, int fp32, const BatchTile* tiles,
                                          int ntiles, const BatchItem* items, const uint64_t* binom, const int4* lbmap,
                                          unsigned* counter, void* Ebase, int max_grid, hipStream_t st) {
    constexpr int G = P * Q;
    if (variant == 0) {
        if constexpr (G < 64)
            return launch_charpoly_batch_team<P, Q, MR, MC, G>(offset, D_max, fp32, tiles, ntiles, items, binom, lbmap, counter,
                                                               Ebase, max_grid, st);
        return hipErrorInvalidValue;
    }
    return launch_charpoly_batch_team<P, Q, MR, MC, 64>(offset, D_max, fp32, tiles, ntiles, items, binom, lbmap, counter,
                                                        Ebase, max_grid, st);
}

hipError_t launch_charpoly_batch_l88(int s_rep, int variant, int offset, int D_max, int fp32, const BatchTile* tiles, int ntiles,
                                      const BatchItem* items, const uint64_t* binom, const int4* lbmap, unsigned* counter, void* Ebase,
                                      int max_grid, hipStream_t st) {
    const int m = 2 * s_rep;
    switch ((m + 7) / 8) {
        case 1: return launch_charpoly_batch_t<8, 8, 1, 1>(variant, offset, D_max, fp32, tiles, ntiles, items, binom, lbmap, counter, Ebase, max_grid, st);
        case 2: return launch_charpoly_batch_t<8, 8, 2, 2>(variant, offset, D_max, fp32, tiles, ntiles, items, binom, lbmap, counter, Ebase, max_grid, st);
        case 3: return launch_charpoly_batch_t<8, 8, 3, 3>(variant, offset, D_max, fp32, tiles, ntiles, items, binom, lbmap, counter, Ebase, max_grid, st);
        case 4: return launch_charpoly_batch_t<8, 8, 4, 4>(variant, offset, D_max, fp32, tiles, ntiles, items, binom, lbmap, counter, Ebase, max_grid, st);
        case 5: return launch_charpoly_batch_t<8, 8, 5, 5>(variant, offset, D_max, fp32, tiles, ntiles, items, binom, lbmap, counter, Ebase, max_grid, st);
        case 6: return launch_charpoly_batch_t<8, 8, 6, 6>(variant, offset, D_max, fp32, tiles, ntiles, items, binom, lbmap, counter, Ebase, max_grid, st);
        case 7: return launch_charpoly_batch_t<8, 8, 7, 7>(variant, offset, D_max, fp32, tiles, ntiles, items, binom, lbmap, counter, Ebase, max_grid, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace gbs
