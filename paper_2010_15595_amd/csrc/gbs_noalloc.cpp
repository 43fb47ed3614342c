// gbs_lhaf_device_noalloc: the device-pointer loop hafnian of gbs_lhaf_device
// for callers that cannot allocate device memory.  Every buffer the subset sum
// needs beyond the caller's input and outputs lives in one fixed device array
// (`scratch`, kScratchBytes per device, held until the process ends):
//
//   [A0 64x64 | d 64 | chunk partials | chunk records | coefficient chunk]
//
// The subset sum runs in chunks sized to fit the coefficient region.  Each
// chunk's compensated block partials are folded into one record (a fixed-order
// tree), and the records are folded into the result at the end, so the
// per-block partials of the whole sum never need to be stored.  Results agree
// with gbs_lhaf_device to rounding (the chunking changes the summation order).
// The kernels are those of gbs_lhaf_device; nothing here allocates.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "gbs_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // GBS_NOALLOC_SCRATCH_BYTES
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr size_t kOffA0 = 0;                                                   // 64 x 64 complex
constexpr size_t kOffD = kOffA0 + sizeof(double2) * GBS_MAX_DIM * GBS_MAX_DIM;  // 64 complex
constexpr size_t kOffPart = kOffD + 4096;                                      // partials of one chunk
constexpr uint64_t kMaxChunk = 1ull << 18;                                     // subsets per chunk, at most
constexpr int kPer = 8;                                                        // subsets per lane in the series
constexpr uint64_t kBlock = 64ull * kPer;                                      // subsets per partial record
constexpr size_t kRecord = 5 * sizeof(double);
constexpr size_t kOffRec = kOffPart + 32768;                                   // one record per chunk
constexpr size_t kRecBytes = size_t(8) << 20;
constexpr size_t kOffE = kOffRec + kRecBytes;                                  // coefficients of one chunk
constexpr size_t kEBytes = kScratchBytes - kOffE;
static_assert((kMaxChunk / kBlock) * kRecord <= kOffRec - kOffPart, "chunk partials region");
static_assert(kScratchBytes == (size_t)GBS_NOALLOC_SCRATCH_BYTES, "header and library agree on the size");

}  // namespace

namespace gbs_host {

// Device address of this device's scratch array (the host symbol is only a
// stand-in).  Called once per device, with that device current, when its
// context is created.
gbs_status noalloc_setup(DevCtx* c) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(GBS_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", c->device,
                    hipGetErrorString(e));
    c->na_scratch = p;
    return GBS_OK;
}

}  // namespace gbs_host

using namespace gbs_host;

extern "C" gbs_status gbs_lhaf_device_noalloc(const gbs_z* A_dev, int32_t N, gbs_precision prec, gbs_z* out_dev,
                                              double* abs_sum_dev, void* stream) {
    if (N < 0 || (N > 0 && !A_dev) || !out_dev) return fail(GBS_E_ARG, "bad device arguments");
    if (N > GBS_MAX_DIM) return fail(GBS_E_TOO_LARGE, "dimension %d exceeds %d", N, GBS_MAX_DIM);
    if (prec == GBS_DD) return fail(GBS_E_UNSUPPORTED, "the no-allocation entry point runs FP64 or FP32_COMP");
    if (prec != GBS_FP64 && prec != GBS_FP32_COMP) return fail(GBS_E_ARG, "bad precision %d", (int)prec);
    std::lock_guard<std::mutex> lock(g_mutex);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(GBS_E_DEVICE, "hipGetDevice failed");
    DevCtx* c = existing_ctx(dev);
    if (!c || !c->na_scratch)
        return fail(GBS_E_ARG, "gbs_init(%d) must precede gbs_lhaf_device_noalloc on device %d", dev, dev);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double2* out = reinterpret_cast<double2*>(out_dev);
    const int Np = N + (N & 1), n = Np / 2, D = n + 1;
    if (n == 0) {
        HIP_TRY(gbs::launch_scalar_set(out, make_double2(1.0, 0.0), abs_sum_dev, 1.0, st));
        return GBS_OK;
    }
    char* base = static_cast<char*>(c->na_scratch);
    double2* A0 = reinterpret_cast<double2*>(base + kOffA0);
    double2* dv = reinterpret_cast<double2*>(base + kOffD);
    double* part = reinterpret_cast<double*>(base + kOffPart);
    double* rec = reinterpret_cast<double*>(base + kOffRec);
    void* E = base + kOffE;
    const bool fp32 = prec == GBS_FP32_COMP;
    const size_t per_subset = std::max<size_t>(2 * (D + 1) * (fp32 ? sizeof(float2) : sizeof(double2)),
                                               gbs::lds_term_bytes(0));
    const uint64_t chunk = std::min<uint64_t>(kMaxChunk, (kEBytes / per_subset) / kBlock * kBlock);
    uint64_t nrec = 0;
    for (int s = 1; s <= n; ++s) nrec += (binom_host(n, s) + chunk - 1) / chunk;
    if (nrec * kRecord > kRecBytes)
        return fail(GBS_E_TOO_LARGE, "N = %d needs %llu chunk records, the scratch array holds %llu", N,
                    (unsigned long long)nrec, (unsigned long long)(kRecBytes / kRecord));
    HIP_TRY(gbs::launch_prep(reinterpret_cast<const double2*>(A_dev), N, N, Np, A0, dv, st));
    uint64_t r = 0;
    for (int s = 1; s <= n; ++s) {
        const uint64_t cnt = binom_host(n, s);
        const double sign = ((n - s) & 1) ? -1.0 : 1.0;
        for (uint64_t st0 = 0; st0 < cnt; st0 += chunk, ++r) {
            const uint64_t len = std::min(chunk, cnt - st0);
            const int64_t nb = (int64_t)((len + kBlock - 1) / kBlock);
            if (2 * s > gbs::kMaxTileM) {
                HIP_TRY(gbs::launch_charpoly_lds(0, gbs::kCharpolyLaBudde, A0, dv, Np, s, st0, len, nullptr, c->binom,
                                                 D, sign, E, st));
                HIP_TRY(gbs::launch_lds_block_reduce(0, E, len, kPer, part, nullptr, st));
            } else {
                gbs::LaunchPhase1 p1{A0, dv, Np, s, st0, len, nullptr, c->binom, D, E, fp32 ? 1 : 0, c->lbmap};
                HIP_TRY(gbs::launch_charpoly(p1, layout_for(c, n, s, false, fp32), st));
                gbs::LaunchPhase2 p2{E, fp32 ? 1 : 0, len, D, sign, kPer, part, nullptr};
                HIP_TRY(gbs::launch_series(n, p2, st));
            }
            HIP_TRY(gbs::launch_partials_fold(part, nb, rec + 5 * r, st));
        }
    }
    HIP_TRY(gbs::launch_final_reduce(rec, (int64_t)r, out, abs_sum_dev, st));
    return GBS_OK;
}
