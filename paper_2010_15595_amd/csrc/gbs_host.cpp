// Host side of the gbs_lhaf C ABI: argument validation, photon-pattern
// expansion, the pure-state parameters of Q (Cholesky factorisation on the
// host, O(M^3) for M <= a few hundred), device workspace and the launch
// schedule of the subset-sum kernels.  Every step of the subset sum itself runs
// in the HIP kernels of lhaf_kernels.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gbs_internal.h"

using cplx = std::complex<double>;

namespace gbs_host {

thread_local std::string g_last_error;

gbs_status fail(gbs_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

constexpr uint64_t kChunk = gbs::kSubsetsPerLaunch;  // subsets per phase-1 launch
constexpr size_t kConcurrentEBytes = (size_t)4 << 30;  // coefficient bytes of a loop hafnian whose classes run concurrently
constexpr int kPerThread = 8;            // subsets per lane in phase 2

uint64_t binom_host(int a, int b) {
    if (b < 0 || b > a) return 0;
    uint64_t r = 1;
    for (int i = 1; i <= b; ++i) r = r * (uint64_t)(a - b + i) / (uint64_t)i;
    return r;
}

int layout_for(const DevCtx* c, int n, int s, bool batch, bool fp32) {
    if (batch) {
        int v = c->layout_multi[n][s];
        // measured slower inside batches than the two-team 8x4 grid
        if (v < 0) v = (c->layout[n][s] == gbs::kLayout84T) ? gbs::kLayout84 : c->layout[n][s];
        if (v < 0) v = gbs::charpoly_default_layout(2 * s);
        // the persistent 8x4 instances above m = kMaxBatchM84 spill registers
        if ((v == gbs::kLayout84 || v == gbs::kLayout84T) && 2 * s > gbs::kMaxBatchM84) v = gbs::kLayout88;
        return v;
    }
    const int v = c->layout[n][s];
    // the tuner times the FP64 kernels; the FP32 La Budde instances of the
    // one-team 8x4 grid need 250-300 VGPRs (one or two waves per SIMD), and
    // the two-team grid ran N = 50 18% faster in FP32
    if (fp32 && v == gbs::kLayout84T) return gbs::kLayout84;
    return v >= 0 ? v : gbs::charpoly_default_layout(2 * s);
}

int layout_front_offset(int lay, int s) {
    const int P = (lay == gbs::kLayout44) ? 4 : 8, Q = (lay == gbs::kLayout88) ? 8 : 4, m = 2 * s;
    return gbs::charpoly_front_offset(P, Q, (m + P - 1) / P, (m + Q - 1) / Q, m);
}

std::mutex g_mutex;
std::map<int, DevCtx*> g_ctx;

// Optional per-launch timing (gbs_profile_enable / gbs_profile_read).
enum ProfKind { kProfCharpoly = 0, kProfSeries = 1, kProfReduce = 2 };
struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double flops, subsets;
    std::string kernel;  // instance name of a per-subset launch
};
// Both are touched only by calls that hold g_mutex.
bool g_prof = false;
std::vector<ProfRec> g_prof_recs;

double subset_flops(int n, int s) {
    const double m = 2.0 * s;
    return (40.0 / 3.0) * m * m * m + (4.0 / 3.0) * m * m * m + 8.0 * std::min(n - 1.0, m - 1.0) * m * m;
}

// Records an event pair around `launch` when profiling is on.
template <class F>
hipError_t timed_launch(int kind, double flops, double subsets, hipStream_t st, F&& launch,
                        const std::string& kernel = std::string()) {
    if (!g_prof) return launch();
    ProfRec r{kind, nullptr, nullptr, flops, subsets, kernel};
    hipError_t e = hipEventCreate(&r.a);
    if (e == hipSuccess) e = hipEventCreate(&r.b);
    if (e == hipSuccess) e = hipEventRecord(r.a, st);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(r.b, st);
    if (e != hipSuccess) {
        if (r.a) hipEventDestroy(r.a);
        if (r.b) hipEventDestroy(r.b);
        return e;
    }
    g_prof_recs.push_back(r);
    return e;
}

hipError_t dev_malloc(void** p, size_t bytes) {
    const char* f = std::getenv("GBS_TEST_FAIL_ALLOC");
    if (f && f[0] == '1' && f[1] == 0) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

bool profiling_on() { return g_prof; }

hipError_t prof_charpoly_launch(double flops, double subsets, hipStream_t st,
                                const std::function<hipError_t()>& launch, const std::string& kernel) {
    return timed_launch(kProfCharpoly, flops, subsets, st, launch, kernel);
}

gbs_status ensure_buffer(void** p, size_t* cap, size_t need, size_t elem) {
    if (*cap >= need) return GBS_OK;
    if (*p) hipFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = dev_malloc(p, need * elem);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(GBS_E_NOMEM, "hipMalloc(%zu bytes) failed: %s", need * elem, hipGetErrorString(e));
    }
    *cap = need;
    return GBS_OK;
}

void ctx_destroy(DevCtx* c);
gbs_status ctx_init(DevCtx* c);

gbs_status ctx_create(int device, DevCtx** out) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(GBS_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(GBS_E_DEVICE, "device %d out of range (%d devices)", device, count);
    HIP_TRY(hipSetDevice(device));
    DevCtx* c = new DevCtx();
    c->device = device;
    const gbs_status st = ctx_init(c);
    if (st != GBS_OK) {
        ctx_destroy(c);  // frees whatever was created before the failure
        return st;
    }
    *out = c;
    return GBS_OK;
}

gbs_status ctx_init(DevCtx* c) {
    const int device = c->device;
    HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&c->done, hipEventDisableTiming));
    HIP_TRY(hipEventCreate(&c->t0));
    HIP_TRY(hipEventCreate(&c->t1));
    HIP_TRY(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
    for (int i = 0; i < kAuxStreams; ++i) {
        HIP_TRY(hipStreamCreateWithFlags(&c->aux[i], hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming));
    }
    std::vector<uint64_t> tab(gbs::kBinomStride * gbs::kBinomStride, 0);
    for (int a = 0; a < gbs::kBinomStride; ++a)
        for (int b = 0; b < gbs::kBinomStride; ++b) tab[a * gbs::kBinomStride + b] = binom_host(a, b);
    HIP_TRY(dev_malloc((void**)&c->binom, tab.size() * sizeof(uint64_t)));
    HIP_TRY(hipMemcpy(c->binom, tab.data(), tab.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
    std::vector<int4> lbt(gbs::kLbTableEntries);
    gbs::lb_fill_table(lbt.data());
    HIP_TRY(dev_malloc((void**)&c->lbmap, lbt.size() * sizeof(int4)));
    HIP_TRY(hipMemcpy(c->lbmap, lbt.data(), lbt.size() * sizeof(int4), hipMemcpyHostToDevice));
    HIP_TRY(dev_malloc((void**)&c->A0, sizeof(double2) * GBS_MAX_DIM * GBS_MAX_DIM));
    HIP_TRY(dev_malloc((void**)&c->dvec, sizeof(double2) * GBS_MAX_DIM));
    HIP_TRY(dev_malloc((void**)&c->Ain, sizeof(double2) * GBS_MAX_DIM * GBS_MAX_DIM));
    HIP_TRY(dev_malloc((void**)&c->res, sizeof(double2) * 3));
    HIP_TRY(hipEventRecord(c->done, c->stream));
    const gbs_status na = noalloc_setup(c);
    if (na != GBS_OK) return na;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        snprintf(c->name, sizeof c->name, "%s", prop.gcnArchName);
        for (char* q = c->name; *q; ++q)
            if (*q == ' ' || *q == ':') *q = '_';
    }
    return GBS_OK;
}

void ctx_destroy(DevCtx* c) {
    if (!c) return;
    hipSetDevice(c->device);
    // device-pointer calls run on the callers' streams and read the context's
    // tables and workspace: let all of them finish first
    hipDeviceSynchronize();
    hipFree(c->binom);
    hipFree(c->lbmap);
    hipFree(c->A0);
    hipFree(c->dvec);
    hipFree(c->Ain);
    hipFree(c->res);
    hipFree(c->E);
    hipFree(c->partials);
    hipFree(c->masks);
    hipFree(c->terms);
    runner_free(c->runner);
    hipFree(c->smats);
    if (c->done) hipEventDestroy(c->done);
    if (c->t0) hipEventDestroy(c->t0);
    if (c->t1) hipEventDestroy(c->t1);
    if (c->fork) hipEventDestroy(c->fork);
    for (int i = 0; i < kAuxStreams; ++i) {
        if (c->join[i]) hipEventDestroy(c->join[i]);
        if (c->aux[i]) hipStreamDestroy(c->aux[i]);
    }
    if (c->stream) hipStreamDestroy(c->stream);
    delete c;
}

DevCtx* existing_ctx(int dev) {
    auto it = g_ctx.find(dev);
    return it == g_ctx.end() ? nullptr : it->second;
}

// Context of the current HIP device, created on first use.
gbs_status current_ctx(DevCtx** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(GBS_E_DEVICE, "hipGetDevice failed");
    auto it = g_ctx.find(dev);
    if (it != g_ctx.end()) {
        *out = it->second;
        return GBS_OK;
    }
    DevCtx* c = nullptr;
    gbs_status st = ctx_create(dev, &c);
    if (st != GBS_OK) return st;
    g_ctx[dev] = c;
    *out = c;
    return GBS_OK;
}

bool finite_z(const gbs_z& z) { return std::isfinite(z.re) && std::isfinite(z.im); }

gbs_status check_matrix(const gbs_z* A, int32_t N, int64_t lda, const char* what, bool need_sym) {
    if (N < 0) return fail(GBS_E_ARG, "%s: negative dimension %d", what, N);
    if (N == 0) return GBS_OK;
    if (!A) return fail(GBS_E_ARG, "%s: null pointer", what);
    if (lda < N) return fail(GBS_E_ARG, "%s: leading dimension %lld < %d", what, (long long)lda, N);
    double amax = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            const gbs_z& z = A[(int64_t)i * lda + j];
            if (!finite_z(z)) return fail(GBS_E_NONFINITE, "%s: non-finite entry at (%d, %d)", what, i, j);
            amax = std::max(amax, std::hypot(z.re, z.im));
        }
    if (need_sym) {
        const double tol = 1e-12 * amax;
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j) {
                const gbs_z& a = A[(int64_t)i * lda + j];
                const gbs_z& b = A[(int64_t)j * lda + i];
                if (std::hypot(a.re - b.re, a.im - b.im) > tol)
                    return fail(GBS_E_NOT_SYMMETRIC, "%s: entries (%d, %d) and (%d, %d) differ", what, i, j, j, i);
            }
    }
    return GBS_OK;
}

gbs_status expand_impl(const gbs_z* B, int32_t M, int64_t ldb, const gbs_z* gamma, const int32_t* mult,
                       std::vector<gbs_z>& out, int32_t* N_out) {
    if (M < 0) return fail(GBS_E_ARG, "negative M");
    if (M > 0 && !B) return fail(GBS_E_ARG, "null matrix");
    if (M > 0 && ldb < M) return fail(GBS_E_ARG, "leading dimension %lld < M = %d", (long long)ldb, M);
    gbs_status st = check_matrix(B, M, ldb, "A", true);
    if (st != GBS_OK) return st;
    int64_t N = 0;
    for (int i = 0; i < M; ++i) {
        const int s = mult ? mult[i] : 1;
        if (s < 0) return fail(GBS_E_ARG, "negative multiplicity %d at mode %d", s, i);
        N += s;
        if (N > GBS_MAX_DIM) return fail(GBS_E_TOO_LARGE, "expanded dimension exceeds %d", GBS_MAX_DIM);
    }
    if (gamma)
        for (int i = 0; i < M; ++i)
            if ((mult ? mult[i] : 1) > 0 && !finite_z(gamma[i]))
                return fail(GBS_E_NONFINITE, "non-finite loop weight at mode %d", i);
    std::vector<int> idx;
    idx.reserve(N);
    for (int i = 0; i < M; ++i)
        for (int r = 0; r < (mult ? mult[i] : 1); ++r) idx.push_back(i);
    out.assign((size_t)N * N, gbs_z{0.0, 0.0});
    for (int64_t a = 0; a < N; ++a)
        for (int64_t b = 0; b < N; ++b) out[a * N + b] = B[(int64_t)idx[a] * ldb + idx[b]];
    if (gamma)
        for (int64_t a = 0; a < N; ++a) out[a * N + a] = gamma[idx[a]];
    *N_out = (int32_t)N;
    return GBS_OK;
}

// Subset-sum schedule on prepared workspace (ctx->A0, ctx->dvec).
// Name of the per-subset kernel instance a launch of subsets of size s runs
// (as the profiler prints it), for per-instance timing.
std::string charpoly_instance_name(int lay, int s, int D, bool fp32) {
    const int P = (lay == gbs::kLayout44) ? 4 : 8, Q = (lay == gbs::kLayout88) ? 8 : 4, m = 2 * s;
    const int G = P * Q;
    const int team = gbs::charpoly_variant(lay, D - 1) != 0 ? 64 : G;
    char buf[96];
    snprintf(buf, sizeof buf, "charpoly_kernel<%d, %d, %d, %d, %s, %d, %d>", P, Q, (m + P - 1) / P, (m + Q - 1) / Q,
             fp32 ? "float2" : "double2", team, layout_front_offset(lay, s));
    return buf;
}

// Subset sum on the LDS-resident kernels (double-double, or FP64 with either
// characteristic-polynomial method): per size class and chunk, one workgroup
// per subset writes its term, a block reduction folds them into dd partials,
// and one final fixed-order dd reduction gives hi (out_dev) and lo (lo_dev).
gbs_status run_sum_lds(DevCtx* c, int Np, hipStream_t st, double2* out_dev, double2* lo_dev, double* abs_dev,
                       int* launches, int prec_dd, int method) {
    const int n = Np / 2, D = n + 1;
    const int maxp = gbs::lds_max_pairs(prec_dd, method);
    if (n > maxp)
        return fail(GBS_E_TOO_LARGE, "%s path: dimension %d exceeds %d",
                    prec_dd ? "double-double" : "LDS", Np, 2 * maxp);
    constexpr int kLdsPer = 8;  // terms per lane in the block reduction
    const uint64_t per_block = 64ull * kLdsPer;
    uint64_t max_len = 0, total_blocks = 0;
    for (int s = 1; s <= n; ++s) {
        const uint64_t cnt = binom_host(n, s);
        for (uint64_t st0 = 0; st0 < cnt; st0 += kChunk) {
            const uint64_t len = std::min(kChunk, cnt - st0);
            max_len = std::max(max_len, len);
            total_blocks += (len + per_block - 1) / per_block;
        }
    }
    gbs_status s1 = ensure_buffer(&c->E, &c->E_cap, (size_t)max_len * gbs::lds_term_bytes(prec_dd), 1);
    if (s1 != GBS_OK) return s1;
    s1 = ensure_buffer((void**)&c->partials, &c->partials_cap, (size_t)total_blocks * 5, sizeof(double));
    if (s1 != GBS_OK) return s1;
    uint64_t poff = 0;
    int nl = 0;
    for (int s = 1; s <= n; ++s) {
        const uint64_t cnt = binom_host(n, s);
        const double sign = ((n - s) & 1) ? -1.0 : 1.0;
        for (uint64_t st0 = 0; st0 < cnt; st0 += kChunk) {
            const uint64_t len = std::min(kChunk, cnt - st0);
            HIP_TRY(timed_launch(
                kProfCharpoly, subset_flops(n, s) * (double)len, (double)len, st,
                [&] {
                    return gbs::launch_charpoly_lds(prec_dd, method, c->A0, c->dvec, Np, s, st0, len, nullptr,
                                                    c->binom, D, sign, c->E, st);
                },
                prec_dd ? "charpoly_lds_kernel<ArDD, 0>"
                        : (method == gbs::kCharpolyEigen ? "charpoly_lds_kernel<ArF64, 1>" : "charpoly_lds_kernel<ArF64, 0>")));
            HIP_TRY(timed_launch(kProfSeries, 0.0, (double)len, st, [&] {
                return gbs::launch_lds_block_reduce(prec_dd, c->E, len, kLdsPer, c->partials + 5 * poff, nullptr, st);
            }));
            poff += (len + per_block - 1) / per_block;
            nl += 2;
        }
    }
    HIP_TRY(timed_launch(kProfReduce, 0.0, 0.0, st, [&] {
        return gbs::launch_dd_final_reduce(c->partials, (int64_t)poff, out_dev, lo_dev, abs_dev, st);
    }));
    if (launches) *launches = nl + 1;
    return GBS_OK;
}

// Colex ranks [lo, hi) of the size-s class taken by shard g of G: the shards
// split every class evenly, so each takes about 1/G of the work.
struct RankRange {
    uint64_t lo, hi;
};
RankRange shard_ranks(uint64_t cnt, int g, int G) {
    return RankRange{cnt * (uint64_t)g / (uint64_t)G, cnt * (uint64_t)(g + 1) / (uint64_t)G};
}

// lds_method >= 0 selects the LDS-resident kernels with that characteristic-polynomial method.
// Shard g of G (FP64 / FP32 paths only) sums its ranks of every class; with
// record_dev set, the compensated partial (sum, compensation re / im, sum |t|)
// is written there instead of the rounded result.
gbs_status run_sum(DevCtx* c, int Np, hipStream_t st, double2* out_dev, double* abs_dev, int* launches,
                   gbs_precision prec, double2* lo_dev = nullptr, int lds_method = -1, int shard = 0,
                   int nshards = 1, double* record_dev = nullptr) {
    const int n = Np / 2;
    int nl = 0;
    if (n == 0) {  // the empty matrix: one term, 1, in shard 0
        const double one = (shard == 0) ? 1.0 : 0.0;
        if (record_dev) {
            HIP_TRY(gbs::launch_scalar_set(reinterpret_cast<double2*>(record_dev), make_double2(one, 0.0),
                                           record_dev + 4, one, st));
            HIP_TRY(gbs::launch_scalar_set(reinterpret_cast<double2*>(record_dev + 2), make_double2(0.0, 0.0),
                                           nullptr, 0.0, st));
        } else {
            HIP_TRY(gbs::launch_scalar_set(out_dev, make_double2(one, 0.0), abs_dev, one, st));
        }
        if (lo_dev) HIP_TRY(gbs::launch_scalar_set(lo_dev, make_double2(0.0, 0.0), nullptr, 0.0, st));
        if (launches) *launches = 1;
        return GBS_OK;
    }
    if (prec == GBS_DD || lds_method >= 0)
        return run_sum_lds(c, Np, st, out_dev, lo_dev, abs_dev, launches, prec == GBS_DD ? 1 : 0,
                           lds_method >= 0 ? lds_method : gbs::kCharpolyLaBudde);
    if (lo_dev) HIP_TRY(gbs::launch_scalar_set(lo_dev, make_double2(0.0, 0.0), nullptr, 0.0, st));
    const bool fp32 = prec == GBS_FP32_COMP;
    const int D = n + 1;
    uint64_t max_len = 0, total_blocks = 0, total_len = 0;
    bool one_launch = true;  // every size class in one launch on the register-tile kernels
    const uint64_t per_block = 64ull * kPerThread;
    for (int s = 1; s <= n; ++s) {
        const RankRange rr = shard_ranks(binom_host(n, s), shard, nshards);
        if (rr.hi - rr.lo > kChunk || 2 * s > gbs::kMaxTileM) one_launch = false;
        total_len += rr.hi - rr.lo;
        for (uint64_t st0 = rr.lo; st0 < rr.hi; st0 += kChunk) {
            const uint64_t len = std::min(kChunk, rr.hi - st0);
            max_len = std::max(max_len, len);
            total_blocks += (len + per_block - 1) / per_block;
        }
    }
    const size_t vbytes = fp32 ? sizeof(float2) : sizeof(double2);
    const size_t per_subset = 2 * (size_t)(D + 1) * vbytes;
    // Small loop hafnians (every class one launch, all coefficient blocks in at
    // most kConcurrentEBytes): the size classes run concurrently on the
    // auxiliary streams, each on its own part of E, since one class alone
    // leaves most of the device idle.  Not while profiling, so that profiled
    // launches are timed one kernel at a time.  The partial records, and so the
    // result, are the same as in the one-stream order.
    const bool concurrent = one_launch && !g_prof && total_len * per_subset <= kConcurrentEBytes;
    gbs_status s1 = ensure_buffer(&c->E, &c->E_cap, (concurrent ? total_len : max_len) * per_subset, 1);
    if (s1 != GBS_OK) return s1;
    s1 = ensure_buffer((void**)&c->partials, &c->partials_cap, (size_t)total_blocks * 5, sizeof(double));
    if (s1 != GBS_OK) return s1;
    uint64_t poff = 0, eoff = 0;
    if (concurrent) {
        HIP_TRY(hipEventRecord(c->fork, st));
        for (int i = 0; i < kAuxStreams; ++i) HIP_TRY(hipStreamWaitEvent(c->aux[i], c->fork, 0));
    }
    auto enqueue_classes = [&]() -> gbs_status {
        for (int s = 1; s <= n; ++s) {
            const RankRange rr = shard_ranks(binom_host(n, s), shard, nshards);
            const double sign = ((n - s) & 1) ? -1.0 : 1.0;
            for (uint64_t st0 = rr.lo; st0 < rr.hi; st0 += kChunk) {
                const uint64_t len = std::min(kChunk, rr.hi - st0);
                if (2 * s > gbs::kMaxTileM) {
                    // beyond the register tiles: the LDS-resident FP64 kernel writes the
                    // signed terms, a block reduction folds them into the same partials
                    HIP_TRY(timed_launch(
                        kProfCharpoly, subset_flops(n, s) * (double)len, (double)len, st,
                        [&] {
                            return gbs::launch_charpoly_lds(0, gbs::kCharpolyLaBudde, c->A0, c->dvec, Np, s, st0, len,
                                                            nullptr, c->binom, D, sign, c->E, st);
                        },
                        "charpoly_lds_kernel<ArF64, 0>"));
                    HIP_TRY(timed_launch(kProfSeries, 0.0, (double)len, st, [&] {
                        return gbs::launch_lds_block_reduce(0, c->E, len, kPerThread, c->partials + 5 * poff, nullptr, st);
                    }));
                    poff += (len + per_block - 1) / per_block;
                    nl += 2;
                    continue;
                }
                const hipStream_t ls = concurrent ? c->aux[(s - 1) % kAuxStreams] : st;
                void* Es = concurrent ? static_cast<void*>(static_cast<char*>(c->E) + eoff * per_subset) : c->E;
                gbs::LaunchPhase1 p1{c->A0, c->dvec, Np, s, st0, len, nullptr, c->binom, D, Es, fp32 ? 1 : 0, c->lbmap};
                const int lay = layout_for(c, n, s, false, fp32);
                HIP_TRY(timed_launch(
                    kProfCharpoly, subset_flops(n, s) * (double)len, (double)len, ls,
                    [&] { return gbs::launch_charpoly(p1, lay, ls); }, charpoly_instance_name(lay, s, D, fp32)));
                gbs::LaunchPhase2 p2{Es, fp32 ? 1 : 0, len, D, sign, kPerThread, c->partials + 5 * poff, nullptr};
                HIP_TRY(timed_launch(kProfSeries, 0.0, (double)len, ls, [&] { return gbs::launch_series(n, p2, ls); }));
                poff += (len + per_block - 1) / per_block;
                eoff += len;
                nl += 2;
            }
        }
        return GBS_OK;
    };
    const gbs_status enq = enqueue_classes();
    if (concurrent) {
        // joined back into st even after a failed launch, so that later work on
        // st is ordered after everything already enqueued on the auxiliary streams
        hipError_t je = hipSuccess;
        for (int i = 0; i < kAuxStreams; ++i) {
            const hipError_t r = hipEventRecord(c->join[i], c->aux[i]);
            const hipError_t w = (r == hipSuccess) ? hipStreamWaitEvent(st, c->join[i], 0) : r;
            if (je == hipSuccess) je = w;
        }
        if (enq == GBS_OK) HIP_TRY(je);
    }
    if (enq != GBS_OK) return enq;
    if (record_dev) {
        HIP_TRY(timed_launch(kProfReduce, 0.0, 0.0, st, [&] {
            return gbs::launch_partials_fold(c->partials, (int64_t)poff, record_dev, st);
        }));
    } else {
        HIP_TRY(timed_launch(kProfReduce, 0.0, 0.0, st, [&] {
            return gbs::launch_final_reduce(c->partials, (int64_t)poff, out_dev, abs_dev, st);
        }));
    }
    if (launches) *launches = nl + 1;
    return GBS_OK;
}

// Full evaluation of an expanded host matrix (N x N, diagonal = loop weights).
gbs_status lhaf_host_matrix(const gbs_z* A, int32_t N, gbs_z* out, gbs_diag* diag, gbs_precision prec,
                            int lds_method = -1) {
    DevCtx* c = nullptr;
    gbs_status st = current_ctx(&c);
    if (st != GBS_OK) return st;
    const int Np = N + (N & 1);
    st = maybe_tune(c, Np / 2);
    if (st != GBS_OK) return st;
    HIP_TRY(hipStreamWaitEvent(c->stream, c->done, 0));
    if (N > 0) HIP_TRY(hipMemcpyAsync(c->Ain, A, sizeof(gbs_z) * (size_t)N * N, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipEventRecord(c->t0, c->stream));
    if (Np > 0) HIP_TRY(gbs::launch_prep(c->Ain, N, N, Np, c->A0, c->dvec, c->stream));
    int launches = 0;
    st = run_sum(c, Np, c->stream, c->res, reinterpret_cast<double*>(c->res + 1), &launches, prec, c->res + 2,
                 lds_method);
    if (st != GBS_OK) return st;
    HIP_TRY(hipEventRecord(c->t1, c->stream));
    double2 h[3];
    HIP_TRY(hipMemcpyAsync(h, c->res, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipEventRecord(c->done, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    out->re = h[0].x;
    out->im = h[0].y;
    if (diag) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, c->t0, c->t1);
        const double mag = std::hypot(h[0].x, h[0].y);
        diag->abs_sum = h[1].x;
        diag->kappa = mag > 0 ? h[1].x / mag : INFINITY;
        diag->subset_terms = (Np / 2) >= 64 ? 0 : (1ull << (Np / 2));
        diag->kernel_ms = ms;
        diag->n_pairs = Np / 2;
        diag->launches = launches;
        diag->lhaf_lo = gbs_z{h[2].x, h[2].y};
    }
    return GBS_OK;
}

// Cholesky factorisation Q = L L^H of a Hermitian matrix (row-major, n x n).
bool cholesky(std::vector<cplx>& L, int n) {
    for (int j = 0; j < n; ++j) {
        double d = L[j * n + j].real();
        for (int k = 0; k < j; ++k) d -= std::norm(L[j * n + k]);
        if (!(d > 0.0)) return false;
        const double ljj = std::sqrt(d);
        L[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            cplx s = L[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * std::conj(L[j * n + k]);
            L[i * n + j] = s / ljj;
        }
        for (int k = j + 1; k < n; ++k) L[j * n + k] = 0.0;
    }
    return true;
}

}  // namespace gbs_host

using namespace gbs_host;

extern "C" {

gbs_status gbs_init(int device) {
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_ctx.count(device)) {
        hipSetDevice(device);
        return GBS_OK;
    }
    DevCtx* c = nullptr;
    gbs_status st = ctx_create(device, &c);
    if (st != GBS_OK) return st;
    g_ctx[device] = c;
    return GBS_OK;
}

void gbs_finalize(void) {
    std::lock_guard<std::mutex> lock(g_mutex);
    for (auto& kv : g_ctx) ctx_destroy(kv.second);
    g_ctx.clear();
}

const char* gbs_status_string(gbs_status s) {
    switch (s) {
        case GBS_OK: return "ok";
        case GBS_E_ARG: return "invalid argument";
        case GBS_E_NOT_SYMMETRIC: return "matrix not symmetric";
        case GBS_E_NONFINITE: return "non-finite input";
        case GBS_E_TOO_LARGE: return "problem too large";
        case GBS_E_NOT_PURE: return "state is not pure";
        case GBS_E_NOT_PD: return "Q is not Hermitian positive definite";
        case GBS_E_DEVICE: return "GPU device error";
        case GBS_E_NOMEM: return "out of memory";
        case GBS_E_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

const char* gbs_last_error(void) { return g_last_error.c_str(); }

int32_t gbs_max_dim(void) { return GBS_MAX_DIM; }

gbs_status gbs_expand(const gbs_z* B, int32_t M, int64_t ldb, const gbs_z* gamma, const int32_t* mult, gbs_z* out,
                      int64_t out_cap, int32_t* N_out) {
    if (!N_out) return fail(GBS_E_ARG, "null N_out");
    std::vector<gbs_z> tmp;
    int32_t N = 0;
    gbs_status st = expand_impl(B, M, ldb, gamma, mult, tmp, &N);
    if (st != GBS_OK) return st;
    if ((int64_t)N * N > out_cap || (N > 0 && !out))
        return fail(GBS_E_ARG, "output capacity %lld < %d", (long long)out_cap, N * N);
    if (N > 0) std::memcpy(out, tmp.data(), sizeof(gbs_z) * tmp.size());
    *N_out = N;
    return GBS_OK;
}

}  // extern "C"

namespace gbs_host {

// Validated parameters of a Gaussian state from Q = Sigma + I/2 (2M x 2M,
// Hermitian positive definite) and alpha = [a; conj(a)] (nullable = 0):
// Q^-1, log det Q and Q^-1 alpha.  With `structured`, Q must also have the
// form [[K, L], [conj(L), conj(K)]] of a covariance in the (a, a^dagger) basis,
// so that A = X (I - Q^-1) is symmetric.
struct GaussParams {
    int M = 0;
    std::vector<cplx> Qi;  // 2M x 2M
    std::vector<cplx> qa;  // Q^-1 alpha
    std::vector<cplx> al;
    double logdet = 0.0;
    cplx quad = 0.0;       // alpha^H Q^-1 alpha
    // A = X (I - Q^-1): rows of the two halves swapped (Eq. (4))
    cplx A(int i, int j) const {
        const int n = 2 * M;
        const int xi = i < M ? i + M : i - M;
        return ((xi == j) ? cplx(1.0) : cplx(0.0)) - Qi[xi * n + j];
    }
};

gbs_status gauss_params(const gbs_z* Q, const gbs_z* alpha, int32_t M, bool structured, GaussParams& G) {
    if (M < 0) return fail(GBS_E_ARG, "negative M");
    if (M > 0 && !Q) return fail(GBS_E_ARG, "null Q");
    const int n = 2 * M;
    G.M = M;
    for (int i = 0; i < n * n; ++i)
        if (!finite_z(Q[i])) return fail(GBS_E_NONFINITE, "non-finite Q entry %d", i);
    if (alpha)
        for (int i = 0; i < n; ++i)
            if (!finite_z(alpha[i])) return fail(GBS_E_NONFINITE, "non-finite alpha entry %d", i);
    double qmax = 0.0;
    for (int i = 0; i < n * n; ++i) qmax = std::max(qmax, std::hypot(Q[i].re, Q[i].im));
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) {
            const gbs_z a = Q[i * n + j], b = Q[j * n + i];
            if (std::hypot(a.re - b.re, a.im + b.im) > 1e-12 * std::max(1.0, qmax))
                return fail(GBS_E_NOT_PD, "Q is not Hermitian at (%d, %d)", i, j);
        }
    if (structured)
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < n; ++j) {
                // Q[i + M][j'] = conj(Q[i][j]) with j' the partner of j
                const int jp = j < M ? j + M : j - M;
                const gbs_z a = Q[i * n + j], b = Q[(i + M) * n + jp];
                if (std::hypot(a.re - b.re, a.im + b.im) > 1e-12 * std::max(1.0, qmax))
                    return fail(GBS_E_ARG, "Q lacks the [[K, L], [conj(L), conj(K)]] form at (%d, %d)", i, j);
            }
    G.al.assign(n, 0.0);
    if (alpha) {
        double amax = 0.0;
        for (int i = 0; i < n; ++i) amax = std::max(amax, std::hypot(alpha[i].re, alpha[i].im));
        for (int i = 0; i < M; ++i) {
            const gbs_z a = alpha[i], b = alpha[M + i];
            if (std::hypot(a.re - b.re, a.im + b.im) > 1e-12 * std::max(1.0, amax))
                return fail(GBS_E_ARG, "alpha is not of the form [a; conj(a)] at mode %d", i);
        }
        for (int i = 0; i < n; ++i) G.al[i] = cplx(alpha[i].re, alpha[i].im);
    }
    std::vector<cplx> L(n * n);
    for (int i = 0; i < n * n; ++i) L[i] = cplx(Q[i].re, Q[i].im);
    if (!cholesky(L, n)) return fail(GBS_E_NOT_PD, "Q is not positive definite");
    // Q^-1 = L^-H L^-1, column by column
    G.Qi.assign(n * n, 0.0);
    std::vector<cplx> col(n);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            cplx s = (i == j) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * col[k];
            col[i] = s / L[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            cplx s = col[i];
            for (int k = i + 1; k < n; ++k) s -= std::conj(L[k * n + i]) * col[k];
            col[i] = s / L[i * n + i].real();
        }
        for (int i = 0; i < n; ++i) G.Qi[i * n + j] = col[i];
    }
    G.logdet = 0.0;
    for (int i = 0; i < n; ++i) G.logdet += 2.0 * std::log(L[i * n + i].real());
    G.qa.assign(n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) G.qa[i] += G.Qi[i * n + j] * G.al[j];
    G.quad = 0.0;
    for (int i = 0; i < n; ++i) G.quad += std::conj(G.al[i]) * G.qa[i];
    return GBS_OK;
}

double lfactorial_sum(const int32_t* pattern, int M) {
    double lf = 0.0;
    for (int i = 0; i < M; ++i) lf += std::lgamma((double)pattern[i] + 1.0);
    return lf;
}

}  // namespace gbs_host

extern "C" {

gbs_status gbs_pure_state(const gbs_z* Q, const gbs_z* alpha, int32_t M, gbs_z* B_out, gbs_z* gamma_out,
                          double* p_vac_out) {
    if (M > 0 && (!Q || !alpha)) return fail(GBS_E_ARG, "null Q or alpha");
    GaussParams G;
    gbs_status st = gauss_params(Q, alpha, M, false, G);
    if (st != GBS_OK) return st;
    double anorm = 0.0, offb = 0.0, diffb = 0.0;
    const int n = 2 * M;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) anorm = std::max(anorm, std::abs(G.A(i, j)));
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            offb = std::max(offb, std::abs(G.A(i, M + j)));
            offb = std::max(offb, std::abs(G.A(M + i, j)));
            diffb = std::max(diffb, std::abs(G.A(M + i, M + j) - std::conj(G.A(i, j))));
        }
    if (offb > 1e-10 * std::max(1.0, anorm) || diffb > 1e-10 * std::max(1.0, anorm))
        return fail(GBS_E_NOT_PURE, "A = X(I - Q^-1) is not B (+) conj(B) (off-block %.3g, mismatch %.3g)", offb, diffb);
    if (B_out)
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                const cplx b = G.A(i, j);
                B_out[i * M + j] = gbs_z{b.real(), b.imag()};
            }
    // the loop weights pairing with B are the second half of Q^-1 alpha
    if (gamma_out)
        for (int i = 0; i < M; ++i) gamma_out[i] = gbs_z{G.qa[M + i].real(), G.qa[M + i].imag()};
    if (p_vac_out) *p_vac_out = std::exp(-0.5 * G.quad.real() - 0.5 * G.logdet);
    return GBS_OK;
}

gbs_status gbs_probability_mixed(const gbs_z* Q, const gbs_z* alpha, const int32_t* pattern, int32_t M,
                                 gbs_precision prec, double* p_out, gbs_z* lhaf_out, gbs_diag* diag) {
    if (!p_out || (M > 0 && !pattern)) return fail(GBS_E_ARG, "null output or pattern");
    if (prec != GBS_FP64 && prec != GBS_FP32_COMP && prec != GBS_DD) return fail(GBS_E_ARG, "bad precision %d", (int)prec);
    int64_t photons = 0;
    for (int i = 0; i < M; ++i) {
        if (pattern[i] < 0) return fail(GBS_E_ARG, "negative photon number at mode %d", i);
        photons += pattern[i];
    }
    if (2 * photons > GBS_MAX_DIM)
        return fail(GBS_E_TOO_LARGE, "%lld photons need a %lld x %lld loop hafnian (max %d)", (long long)photons,
                    (long long)(2 * photons), (long long)(2 * photons), GBS_MAX_DIM);
    GaussParams G;
    gbs_status st = gauss_params(Q, alpha, M, true, G);
    if (st != GBS_OK) return st;
    // rows/columns i and i + M repeated s_i times: first-half copies, then second-half copies
    std::vector<int> idx;
    for (int half = 0; half < 2; ++half)
        for (int i = 0; i < M; ++i)
            for (int c = 0; c < pattern[i]; ++c) idx.push_back(i + half * M);
    const int N = (int)idx.size();
    std::vector<gbs_z> As((size_t)N * N);
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            cplx v;
            if (a == b) {
                // loop weight of index k: the entry of Q^-1 alpha of its partner index (X Q^-1 alpha)
                const int k = idx[a];
                v = G.qa[k < M ? k + M : k - M];
            } else {
                v = G.A(idx[a], idx[b]);
            }
            As[(size_t)a * N + b] = gbs_z{v.real(), v.imag()};
        }
    gbs_z lh{1.0, 0.0};
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        st = lhaf_host_matrix(As.data(), N, &lh, diag, prec);
    }
    if (st != GBS_OK) return st;
    const double scale = std::exp(-0.5 * G.quad.real() - 0.5 * G.logdet - lfactorial_sum(pattern, M));
    *p_out = scale * lh.re;
    if (lhaf_out) *lhaf_out = lh;
    return GBS_OK;
}

gbs_status gbs_lhaf(const gbs_z* A, int32_t M, int64_t lda, const gbs_z* gamma, const int32_t* mult,
                    gbs_precision prec, gbs_z* out, gbs_diag* diag) {
    if (!out) return fail(GBS_E_ARG, "null output");
    if (prec != GBS_FP64 && prec != GBS_FP32_COMP && prec != GBS_DD) return fail(GBS_E_ARG, "bad precision %d", (int)prec);
    std::vector<gbs_z> Aexp;
    int32_t N = 0;
    gbs_status st = expand_impl(A, M, lda, gamma, mult, Aexp, &N);
    if (st != GBS_OK) return st;
    std::lock_guard<std::mutex> lock(g_mutex);
    return lhaf_host_matrix(Aexp.data(), N, out, diag, prec);
}

gbs_status gbs_haf(const gbs_z* A, int32_t N, int64_t lda, gbs_precision prec, gbs_z* out, gbs_diag* diag) {
    if (!out) return fail(GBS_E_ARG, "null output");
    if (prec != GBS_FP64 && prec != GBS_FP32_COMP && prec != GBS_DD) return fail(GBS_E_ARG, "bad precision %d", (int)prec);
    gbs_status st = check_matrix(A, N, lda, "A", true);
    if (st != GBS_OK) return st;
    if (N > GBS_MAX_DIM) return fail(GBS_E_TOO_LARGE, "dimension %d exceeds %d", N, GBS_MAX_DIM);
    if (N & 1) {
        out->re = 0.0;
        out->im = 0.0;
        if (diag) std::memset(diag, 0, sizeof *diag);
        return GBS_OK;
    }
    std::vector<gbs_z> A0((size_t)N * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) A0[(size_t)i * N + j] = (i == j) ? gbs_z{0.0, 0.0} : A[(int64_t)i * lda + j];
    std::lock_guard<std::mutex> lock(g_mutex);
    return lhaf_host_matrix(A0.data(), N, out, diag, prec);
}

gbs_status gbs_lhaf_method(const gbs_z* A, int32_t N, int64_t lda, gbs_precision prec, gbs_charpoly method,
                           gbs_z* out, gbs_diag* diag) {
    if (!out) return fail(GBS_E_ARG, "null output");
    if (method != GBS_CHARPOLY_LABUDDE && method != GBS_CHARPOLY_EIGEN) return fail(GBS_E_ARG, "bad method %d", (int)method);
    if (prec == GBS_FP32_COMP || (prec == GBS_DD && method == GBS_CHARPOLY_EIGEN))
        return fail(GBS_E_UNSUPPORTED, "the reference kernels run La Budde in FP64 or double-double, eigenvalues in FP64");
    if (prec != GBS_FP64 && prec != GBS_DD) return fail(GBS_E_ARG, "bad precision %d", (int)prec);
    gbs_status st = check_matrix(A, N, lda, "A", true);
    if (st != GBS_OK) return st;
    if (N > GBS_MAX_DIM) return fail(GBS_E_TOO_LARGE, "dimension %d exceeds %d", N, GBS_MAX_DIM);
    std::vector<gbs_z> Ah((size_t)N * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) Ah[(size_t)i * N + j] = A[(int64_t)i * lda + j];
    gbs_z v{0.0, 0.0};
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        st = lhaf_host_matrix(Ah.data(), N, &v, diag, prec,
                              method == GBS_CHARPOLY_EIGEN ? gbs::kCharpolyEigen : gbs::kCharpolyLaBudde);
    }
    if (st != GBS_OK) return st;
    if (!std::isfinite(v.re) || !std::isfinite(v.im))
        return fail(GBS_E_NONFINITE, "a subset's QR iteration did not converge (or the result overflowed)");
    *out = v;
    return GBS_OK;
}

gbs_status gbs_probability(const gbs_z* Q, const gbs_z* alpha, const int32_t* pattern, int32_t M,
                           gbs_precision prec, double* p_out, gbs_z* lhaf_out, gbs_diag* diag) {
    if (!p_out || (M > 0 && !pattern)) return fail(GBS_E_ARG, "null output or pattern");
    if (prec != GBS_FP64 && prec != GBS_FP32_COMP && prec != GBS_DD) return fail(GBS_E_ARG, "bad precision %d", (int)prec);
    std::vector<gbs_z> B((size_t)M * M), gamma(M);
    double pvac = 0.0;
    gbs_status st = gbs_pure_state(Q, alpha, M, B.data(), gamma.data(), &pvac);
    if (st != GBS_OK) return st;
    std::vector<gbs_z> Aexp;
    int32_t N = 0;
    st = expand_impl(B.data(), M, M, gamma.data(), pattern, Aexp, &N);
    if (st != GBS_OK) return st;
    gbs_z lh{1.0, 0.0};
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        st = lhaf_host_matrix(Aexp.data(), N, &lh, diag, prec);
    }
    if (st != GBS_OK) return st;
    *p_out = pvac * (lh.re * lh.re + lh.im * lh.im) * std::exp(-lfactorial_sum(pattern, M));
    if (lhaf_out) *lhaf_out = lh;
    return GBS_OK;
}

gbs_status gbs_lhaf_terms(const gbs_z* A, int32_t N, int64_t lda, const uint64_t* masks, int64_t count,
                          gbs_precision prec, gbs_z* terms_out) {
    if (count < 0 || (count > 0 && (!masks || !terms_out))) return fail(GBS_E_ARG, "bad mask list");
    if (prec != GBS_FP64 && prec != GBS_FP32_COMP && prec != GBS_DD) return fail(GBS_E_ARG, "bad precision %d", (int)prec);
    gbs_status st = check_matrix(A, N, lda, "A", true);
    if (st != GBS_OK) return st;
    if (N < 1) return fail(GBS_E_ARG, "terms need N >= 1");
    if (N > GBS_MAX_DIM) return fail(GBS_E_TOO_LARGE, "dimension %d exceeds %d", N, GBS_MAX_DIM);
    const int Np = N + (N & 1), n = Np / 2;
    const bool fp32 = prec == GBS_FP32_COMP, dd = prec == GBS_DD;
    if (dd && n > gbs::kMaxDdPairs)
        return fail(GBS_E_TOO_LARGE, "double-double path: dimension %d exceeds %d", N, 2 * gbs::kMaxDdPairs);
    for (int64_t j = 0; j < count; ++j)
        if (n < 64 && (masks[j] >> n) != 0) return fail(GBS_E_ARG, "mask %lld has bits beyond n = %d", (long long)j, n);
    std::lock_guard<std::mutex> lock(g_mutex);
    DevCtx* c = nullptr;
    st = current_ctx(&c);
    if (st != GBS_OK) return st;
    std::vector<gbs_z> Ah((size_t)N * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) Ah[(size_t)i * N + j] = A[(int64_t)i * lda + j];
    st = maybe_tune(c, n);
    if (st != GBS_OK) return st;
    HIP_TRY(hipStreamWaitEvent(c->stream, c->done, 0));
    HIP_TRY(hipMemcpyAsync(c->Ain, Ah.data(), sizeof(gbs_z) * Ah.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(gbs::launch_prep(c->Ain, N, N, Np, c->A0, c->dvec, c->stream));
    const int D = n + 1;
    for (int s = 0; s <= n; ++s) {
        std::vector<int64_t> pos;
        std::vector<uint64_t> grp;
        for (int64_t j = 0; j < count; ++j)
            if (__builtin_popcountll(masks[j]) == s) {
                pos.push_back(j);
                grp.push_back(masks[j]);
            }
        if (grp.empty()) continue;
        if (s == 0) {  // the empty subset contributes [eta^n] exp(0) = 0 for n >= 1
            for (int64_t j : pos) terms_out[j] = gbs_z{0.0, 0.0};
            continue;
        }
        for (size_t off = 0; off < grp.size(); off += kChunk) {
            const size_t len = std::min<size_t>(kChunk, grp.size() - off);
            st = ensure_buffer((void**)&c->masks, &c->masks_cap, len, sizeof(uint64_t));
            if (st != GBS_OK) return st;
            st = ensure_buffer((void**)&c->terms, &c->terms_cap, len, sizeof(double2));
            if (st != GBS_OK) return st;
            const bool lds_route = !dd && 2 * s > gbs::kMaxTileM;
            const size_t ebytes = dd ? len * 4 * sizeof(double)
                                     : len * std::max<size_t>(2 * (D + 1) * (fp32 ? sizeof(float2) : sizeof(double2)),
                                                              gbs::lds_term_bytes(0));
            st = ensure_buffer(&c->E, &c->E_cap, ebytes, 1);
            if (st != GBS_OK) return st;
            const size_t nblk = (len + 64 * kPerThread - 1) / (64 * kPerThread);
            st = ensure_buffer((void**)&c->partials, &c->partials_cap, nblk * 5, sizeof(double));
            if (st != GBS_OK) return st;
            HIP_TRY(hipMemcpyAsync(c->masks, grp.data() + off, sizeof(uint64_t) * len, hipMemcpyHostToDevice, c->stream));
            const double sign = ((n - s) & 1) ? -1.0 : 1.0;
            if (dd) {
                HIP_TRY(gbs::launch_charpoly_dd(c->A0, c->dvec, Np, s, 0, len, c->masks, c->binom, D, sign, c->E,
                                                c->stream));
                HIP_TRY(gbs::launch_dd_block_reduce(c->E, len, kPerThread, c->partials, c->terms, c->stream));
            } else if (lds_route) {
                HIP_TRY(gbs::launch_charpoly_lds(0, gbs::kCharpolyLaBudde, c->A0, c->dvec, Np, s, 0, len, c->masks,
                                                 c->binom, D, sign, c->E, c->stream));
                HIP_TRY(gbs::launch_lds_block_reduce(0, c->E, len, kPerThread, c->partials, c->terms, c->stream));
            } else {
                gbs::LaunchPhase1 p1{c->A0, c->dvec, Np, s, 0, len, c->masks, c->binom, D, c->E, fp32 ? 1 : 0,
                                     c->lbmap};
                HIP_TRY(gbs::launch_charpoly(p1, layout_for(c, n, s, false, fp32), c->stream));
                gbs::LaunchPhase2 p2{c->E, fp32 ? 1 : 0, len, D, sign, kPerThread, c->partials, c->terms};
                HIP_TRY(gbs::launch_series(n, p2, c->stream));
            }
            std::vector<double2> th(len);
            HIP_TRY(hipMemcpyAsync(th.data(), c->terms, sizeof(double2) * len, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
            for (size_t q = 0; q < len; ++q) terms_out[pos[off + q]] = gbs_z{th[q].x, th[q].y};
        }
    }
    HIP_TRY(hipEventRecord(c->done, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return GBS_OK;
}

gbs_status gbs_lhaf_device(const gbs_z* A_dev, int32_t N, gbs_precision prec, gbs_z* out_dev, double* abs_sum_dev,
                           void* stream) {
    if (N < 0 || (N > 0 && !A_dev) || !out_dev) return fail(GBS_E_ARG, "bad device arguments");
    if (N > GBS_MAX_DIM) return fail(GBS_E_TOO_LARGE, "dimension %d exceeds %d", N, GBS_MAX_DIM);
    if (prec != GBS_FP64 && prec != GBS_FP32_COMP && prec != GBS_DD) return fail(GBS_E_ARG, "bad precision %d", (int)prec);
    std::lock_guard<std::mutex> lock(g_mutex);
    DevCtx* c = nullptr;
    gbs_status st = current_ctx(&c);
    if (st != GBS_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int Np = N + (N & 1);
    st = maybe_tune(c, Np / 2);
    if (st != GBS_OK) return st;
    HIP_TRY(hipStreamWaitEvent(s, c->done, 0));
    if (Np > 0)
        HIP_TRY(gbs::launch_prep(reinterpret_cast<const double2*>(A_dev), N, N, Np, c->A0, c->dvec, s));
    st = run_sum(c, Np, s, reinterpret_cast<double2*>(out_dev), abs_sum_dev, nullptr, prec);
    if (st != GBS_OK) return st;
    HIP_TRY(hipEventRecord(c->done, s));
    return GBS_OK;
}

gbs_status gbs_lhaf_device_shard(const gbs_z* A_dev, int32_t N, gbs_precision prec, int32_t shard, int32_t nshards,
                                 double* partial_dev, void* stream) {
    if (N < 0 || (N > 0 && !A_dev) || !partial_dev) return fail(GBS_E_ARG, "bad device arguments");
    if (nshards < 1 || nshards > GBS_MAX_SHARDS || shard < 0 || shard >= nshards)
        return fail(GBS_E_ARG, "bad shard %d of %d (1 <= shards <= %d)", shard, nshards, GBS_MAX_SHARDS);
    if (N > GBS_MAX_DIM) return fail(GBS_E_TOO_LARGE, "dimension %d exceeds %d", N, GBS_MAX_DIM);
    if (prec == GBS_DD) return fail(GBS_E_UNSUPPORTED, "shards take GBS_FP64 or GBS_FP32_COMP");
    if (prec != GBS_FP64 && prec != GBS_FP32_COMP) return fail(GBS_E_ARG, "bad precision %d", (int)prec);
    std::lock_guard<std::mutex> lock(g_mutex);
    DevCtx* c = nullptr;
    gbs_status st = current_ctx(&c);
    if (st != GBS_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int Np = N + (N & 1);
    st = maybe_tune(c, Np / 2);
    if (st != GBS_OK) return st;
    HIP_TRY(hipStreamWaitEvent(s, c->done, 0));
    if (Np > 0)
        HIP_TRY(gbs::launch_prep(reinterpret_cast<const double2*>(A_dev), N, N, Np, c->A0, c->dvec, s));
    st = run_sum(c, Np, s, nullptr, nullptr, nullptr, prec, nullptr, -1, shard, nshards, partial_dev);
    if (st != GBS_OK) return st;
    HIP_TRY(hipEventRecord(c->done, s));
    return GBS_OK;
}

gbs_status gbs_combine_partials(const double* partials, int32_t count, gbs_z* out, double* abs_sum) {
    if (count < 1 || !partials || !out) return fail(GBS_E_ARG, "bad partial records");
    auto two_sum = [](double a, double b, double& e) {
        const double s = a + b;
        const double bb = s - a;
        e = (a - (s - bb)) + (b - bb);
        return s;
    };
    double sr = partials[0], cr = partials[1], si = partials[2], ci = partials[3], ab = partials[4];
    for (int32_t g = 1; g < count; ++g) {
        const double* p = partials + 5 * (size_t)g;
        double e;
        sr = two_sum(sr, p[0], e);
        cr = cr + p[1] + e;
        si = two_sum(si, p[2], e);
        ci = ci + p[3] + e;
        ab += p[4];
    }
    out->re = sr + cr;
    out->im = si + ci;
    if (abs_sum) *abs_sum = ab;
    return GBS_OK;
}

gbs_status gbs_profile_enable(int on) {
    std::lock_guard<std::mutex> lock(g_mutex);
    for (auto& r : g_prof_recs) {
        hipEventSynchronize(r.b);
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    g_prof_recs.clear();
    g_prof = on != 0;
    return GBS_OK;
}

gbs_status gbs_profile_read(gbs_profile* out) {
    if (!out) return fail(GBS_E_ARG, "null output");
    std::lock_guard<std::mutex> lock(g_mutex);
    gbs_profile p{};
    struct Inst {
        double ms = 0.0, flops = 0.0;
        int64_t launches = 0;
    };
    std::map<std::string, Inst> inst;
    for (auto& r : g_prof_recs) {
        HIP_TRY(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        if (r.kind == kProfCharpoly) {
            p.charpoly_ms += ms;
            p.charpoly_launches += 1;
            p.charpoly_flops += r.flops;
            p.subset_terms += r.subsets;
            Inst& q = inst[r.kernel];
            q.ms += ms;
            q.flops += r.flops;
            q.launches += 1;
        } else if (r.kind == kProfSeries) {
            p.series_ms += ms;
            p.series_launches += 1;
        } else {
            p.reduce_ms += ms;
            p.reduce_launches += 1;
        }
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    g_prof_recs.clear();
    // the instance with the largest summed duration
    const Inst* best = nullptr;
    for (const auto& kv : inst)
        if (!best || kv.second.ms > best->ms) {
            best = &kv.second;
            snprintf(p.dominant_kernel, sizeof p.dominant_kernel, "%s", kv.first.c_str());
        }
    if (best) {
        p.dominant_ms = best->ms;
        p.dominant_flops = best->flops;
        p.dominant_launches = best->launches;
    }
    *out = p;
    return GBS_OK;
}

double gbs_yardstick_flops(int32_t N) {
    if (N < 0 || N > GBS_MAX_DIM) return 0.0;
    const int n = (N + 1) / 2;
    double f = 0.0;
    for (int s = 1; s <= n; ++s) f += (double)binom_host(n, s) * subset_flops(n, s);
    return f;
}

gbs_status gbs_set_layout(int32_t n, int32_t s, int32_t layout) {
    if (n < 0 || n > gbs::kMaxPairs || s < 0 || s > gbs::kMaxPairs) return fail(GBS_E_ARG, "bad (n, s)");
    if (layout < -1 || layout >= gbs::kNumLayouts) return fail(GBS_E_ARG, "bad layout %d", layout);
    if (s > 0 && layout >= 0 && !gbs::charpoly_layout_ok(2 * s, layout))
        return fail(GBS_E_ARG, "layout %d cannot hold m = %d", layout, 2 * s);
    std::lock_guard<std::mutex> lock(g_mutex);
    DevCtx* c = nullptr;
    gbs_status st = current_ctx(&c);
    if (st != GBS_OK) return st;
    for (int nn = (n ? n : 1); nn <= (n ? n : gbs::kMaxPairs); ++nn)
        for (int ss = (s ? s : 1); ss <= (s ? s : nn); ++ss)
            if (layout < 0 || gbs::charpoly_layout_ok(2 * ss, layout)) c->layout[nn][ss] = c->layout_multi[nn][ss] = layout;
    return GBS_OK;
}

}  // extern "C"

namespace gbs_host {

// Reads "<arch> <n> <s> <layout>" lines of the autotune cache for this device.
bool cache_load(DevCtx* c, int n) {
    const char* path = std::getenv("GBS_AUTOTUNE_CACHE");
    if (!path || !*path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[256], arch[64];
    int nn, ss, lay, lay_multi;
    bool any = false;
    auto ok = [&](int l) { return l >= 0 && l < gbs::kNumLayouts && gbs::charpoly_layout_ok(2 * ss, l); };
    // "<arch> <n> <s> <layout> [<batch layout>]"
    while (std::fgets(line, sizeof line, f)) {
        const int k = std::sscanf(line, "%63s %d %d %d %d", arch, &nn, &ss, &lay, &lay_multi);
        if (k < 4 || nn != n || std::strcmp(arch, c->name) != 0 || ss < 1 || ss > n || !ok(lay)) continue;
        c->layout[n][ss] = lay;
        c->layout_multi[n][ss] = (k == 5 && ok(lay_multi)) ? lay_multi : -1;
        any = true;
    }
    std::fclose(f);
    return any;
}

void cache_store(const DevCtx* c, int n) {
    const char* path = std::getenv("GBS_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    for (int s = 1; s <= n; ++s)
        std::fprintf(f, "%s %d %d %d %d\n", c->name, n, s, c->layout[n][s], c->layout_multi[n][s]);
    std::fclose(f);
}

// Times each valid lane grid per subset size on a synthetic matrix.
gbs_status autotune_impl(DevCtx* c, int n, gbs_tune_report* rep) {
    const int Np = 2 * n, D = n + 1;
    std::vector<gbs_z> Ah((size_t)Np * Np);
    uint64_t x = 0x9E3779B97F4A7C15ull;
    auto rnd = [&]() {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        return (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    };
    for (int i = 0; i < Np; ++i)
        for (int j = 0; j <= i; ++j) {
            const gbs_z z{0.3 * rnd(), 0.3 * rnd()};
            Ah[(size_t)i * Np + j] = z;
            Ah[(size_t)j * Np + i] = z;
        }
    HIP_TRY(hipStreamWaitEvent(c->stream, c->done, 0));
    HIP_TRY(hipMemcpyAsync(c->Ain, Ah.data(), sizeof(gbs_z) * Ah.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(gbs::launch_prep(c->Ain, Np, Np, Np, c->A0, c->dvec, c->stream));
    const uint64_t sample_cap = 1ull << 16;
    uint64_t max_len = 0;
    for (int s = 1; s <= n; ++s) max_len = std::max(max_len, std::min(sample_cap, binom_host(n, s)));
    gbs_status st = ensure_buffer(&c->E, &c->E_cap, (size_t)max_len * 2 * (D + 1) * sizeof(double2), 1);
    if (st != GBS_OK) return st;
    if (rep) {
        std::memset(rep, 0, sizeof *rep);
        rep->n = n;
    }
    // GBS_AUTOTUNE_LAYOUTS: bit mask of the lane grids the tuner may choose (default: all)
    unsigned mask = (1u << gbs::kNumLayouts) - 1u;
    if (const char* e = std::getenv("GBS_AUTOTUNE_LAYOUTS")) {
        const unsigned v = (unsigned)strtoul(e, nullptr, 0) & mask;
        if (v) mask = v;
    }
    for (int s = 1; s <= n; ++s) {
        const uint64_t len = std::min(sample_cap, binom_host(n, s));
        double best = 1e300, best_multi = 1e300;
        int best_lay = gbs::charpoly_default_layout(2 * s), best_lay_multi = -1;
        for (int lay = 0; lay < gbs::kNumLayouts; ++lay) {
            if (!gbs::charpoly_layout_ok(2 * s, lay) || !((mask >> lay) & 1u)) continue;
            gbs::LaunchPhase1 p1{c->A0, c->dvec, Np, s, 0, len, nullptr, c->binom, D, c->E, 0, c->lbmap};
            auto time_ns = [&](double* ns) -> hipError_t {
                hipError_t e = gbs::launch_charpoly(p1, lay, c->stream);  // warm-up
                if (e != hipSuccess) return e;
                if ((e = hipEventRecord(c->t0, c->stream)) != hipSuccess) return e;
                const int reps = 3;
                for (int r = 0; r < reps; ++r)
                    if ((e = gbs::launch_charpoly(p1, lay, c->stream)) != hipSuccess) return e;
                if ((e = hipEventRecord(c->t1, c->stream)) != hipSuccess) return e;
                if ((e = hipEventSynchronize(c->t1)) != hipSuccess) return e;
                float ms = 0.f;
                if ((e = hipEventElapsedTime(&ms, c->t0, c->t1)) != hipSuccess) return e;
                *ns = 1e6 * ms / (reps * (double)len);
                return hipSuccess;
            };
            double ns = 0.0;
            HIP_TRY(time_ns(&ns));
            if (rep) rep->ns_per_subset[s][lay] = ns;
            if (ns < best) {
                best = ns;
                best_lay = lay;
            }
            if (lay == gbs::kLayout84T) continue;
            // FP64 batch tiles keep C at the same tile offset: the batch choice
            // is the fastest grid other than the one-team 8x4 grid
            if (ns < best_multi) {
                best_multi = ns;
                best_lay_multi = lay;
            }
        }
        c->layout[n][s] = best_lay;
        c->layout_multi[n][s] = best_lay_multi;
        if (rep) rep->layout[s] = best_lay;
    }
    HIP_TRY(hipEventRecord(c->done, c->stream));
    c->tuned[n] = true;
    cache_store(c, n);
    return GBS_OK;
}

gbs_status maybe_tune(DevCtx* c, int n) {
    if (n < 1 || n > gbs::kMaxPairs || c->tuned[n]) return GBS_OK;
    c->tuned[n] = true;
    if (cache_load(c, n)) return GBS_OK;
    const char* at = std::getenv("GBS_AUTOTUNE");
    if (at && (std::strcmp(at, "1") == 0 || std::strcmp(at, "force") == 0)) return autotune_impl(c, n, nullptr);
    return GBS_OK;
}

}  // namespace gbs_host

extern "C" {

gbs_status gbs_autotune(int32_t n, gbs_tune_report* report) {
    if (n < 1 || n > gbs::kMaxPairs) return fail(GBS_E_ARG, "n = %d out of range", n);
    std::lock_guard<std::mutex> lock(g_mutex);
    DevCtx* c = nullptr;
    gbs_status st = current_ctx(&c);
    if (st != GBS_OK) return st;
    return autotune_impl(c, n, report);
}

gbs_status gbs_selftest(int32_t* failures) {
    if (!failures) return fail(GBS_E_ARG, "null output");
    std::lock_guard<std::mutex> lock(g_mutex);
    DevCtx* c = nullptr;
    gbs_status st = current_ctx(&c);
    if (st != GBS_OK) return st;
    double hin[64], hout[1408];
    for (int l = 0; l < 64; ++l) hin[l] = std::ldexp(1.0, l % 20) + 0.25 * l;
    double *din = nullptr, *dout = nullptr;
    hipError_t e = dev_malloc((void**)&din, sizeof hin);
    if (e == hipSuccess) e = dev_malloc((void**)&dout, sizeof hout);
    if (e == hipSuccess) e = hipMemcpy(din, hin, sizeof hin, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = gbs::launch_selftest(din, dout, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(hout, dout, sizeof hout, hipMemcpyDeviceToHost);
    hipFree(din);
    hipFree(dout);
    HIP_TRY(e);
    int bad = 0;
    for (int l = 0; l < 64; ++l) {
        double so = 0.0, ss = 0.0;
        for (int q = 0; q < 8; ++q) so += hin[(l & ~7) + q];
        for (int q = 0; q < 8; ++q) ss += hin[(l & 7) + 8 * q];
        if (std::fabs(hout[l] - so) > 1e-12 * std::fabs(so)) ++bad;
        if (std::fabs(hout[64 + l] - ss) > 1e-12 * std::fabs(ss)) ++bad;
        if (hout[128 + l] != hin[37]) ++bad;
        if (l >= 1 && hout[192 + l] != hin[l - 1]) ++bad;
        // swap16: x <- [x.r0, y.r0, x.r2, y.r2], y <- [x.r1, y.r1, x.r3, y.r3] with y = -x
        const int row = l / 16, li = l % 16;
        const double sx = (row % 2 == 0) ? hin[l] : -hin[(row - 1) * 16 + li];
        const double sy = (row % 2 == 0) ? hin[(row + 1) * 16 + li] : -hin[l];
        if (hout[256 + l] != sx || hout[320 + l] != sy) ++bad;
        // swap32: x <- [x.lo, y.lo], y <- [x.hi, y.hi]
        const double tx = (l < 32) ? hin[l] : -hin[l - 32];
        const double ty = (l < 32) ? hin[l + 32] : -hin[l];
        if (hout[384 + l] != tx || hout[448 + l] != ty) ++bad;
        // grouped row sums over lanes {l mod 8 + 8q} (8x8) and {l mod 8 + 8q} within 32-lane halves (8x4)
        const double f8[6] = {1.0, 2.0, 3.0, -1.0, 0.5, 7.0};
        for (int j = 0; j < 6; ++j)
            if (std::fabs(hout[512 + 64 * j + l] - f8[j] * ss) > 1e-12 * std::fabs(f8[j] * ss)) ++bad;
        double s4 = 0.0;
        for (int q = 0; q < 4; ++q) s4 += hin[(l & 7) + 8 * q + (l & 32)];
        const double f4[4] = {1.0, -2.0, 3.0, 0.25};
        for (int j = 0; j < 4; ++j)
            if (std::fabs(hout[896 + 64 * j + l] - f4[j] * s4) > 1e-12 * std::fabs(f4[j] * s4)) ++bad;
        // sums over the lane quad {4 (l / 4) + q}: row sums of the column-swap 8x4 map
        double sq = 0.0;
        for (int q = 0; q < 4; ++q) sq += hin[(l & ~3) + q];
        const double fq[4] = {1.0, 0.5, -3.0, 2.0};
        for (int j = 0; j < 4; ++j)
            if (std::fabs(hout[1152 + 64 * j + l] - fq[j] * sq) > 1e-12 * std::fabs(fq[j] * sq)) ++bad;
    }
    *failures = bad;
    return GBS_OK;
}

}  // extern "C"
