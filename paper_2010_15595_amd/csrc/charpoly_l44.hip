// Per-subset kernel instantiations for the 4 x 4 lanes per subset, four subsets per wavefront; MR = MC = ceil(m / 4).
#include "lhaf_device.h"

namespace gbs {

template <int P, int Q, int MR, int MC>
static hipError_t launch_charpoly_t(const LaunchPhase1& p, hipStream_t st) {
    constexpr int G = P * Q;
    constexpr int W = 64 / G;
    const int T = (G >= p.D + 1) ? G : 64;
    const size_t lds = sizeof(double2) * lds_doubles2(W, 64 / T, p.D);
    const unsigned grid = (unsigned)((p.count + W - 1) / W);
    hipLaunchKernelGGL((charpoly_kernel<P, Q, MR, MC>), dim3(grid), dim3(64), lds, st, p.A0, p.dvec, p.Np, p.s,
                       p.rank0, p.count, p.masks, p.binom, p.D, T, p.Eout);
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

}  // namespace gbs
