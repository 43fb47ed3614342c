// Internal declarations shared by the host translation units of libgbs_lhaf.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gbs_lhaf.h"
#include "lhaf_kernels.h"

namespace gbs_host {

// Sets the thread-local error text and returns st.
gbs_status fail(gbs_status st, const char* fmt, ...);

#define HIP_TRY(call)                                                                                         \
    do {                                                                                                      \
        hipError_t e_ = (call);                                                                               \
        if (e_ != hipSuccess)                                                                                 \
            return gbs_host::fail(e_ == hipErrorOutOfMemory ? GBS_E_NOMEM : GBS_E_DEVICE, "%s: %s (%s:%d)", \
                                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                          \
    } while (0)

uint64_t binom_host(int a, int b);
// Cholesky factorisation Q = L L^H of a Hermitian matrix (row-major n x n, in
// place, lower triangle); false when not positive definite.
bool cholesky(std::vector<std::complex<double>>& L, int n);
// Flop yardstick of one subset of size s of an n-pair loop hafnian.
double subset_flops(int n, int s);

struct BatchRunner;

// Per-device workspace.  All library calls take g_mutex, so one context is
// used by one call at a time; `done` orders reuse across caller streams.
constexpr int kAuxStreams = 4;  // streams that run the size classes of a small loop hafnian concurrently

struct DevCtx {
    int device = -1;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr, t0 = nullptr, t1 = nullptr;
    hipStream_t aux[kAuxStreams] = {};     // default priority, created with the context
    hipEvent_t fork = nullptr, join[kAuxStreams] = {};
    uint64_t* binom = nullptr;
    int4* lbmap = nullptr;      // La Budde lane maps (gbs::lb_fill_table)
    double2* A0 = nullptr;      // 64 x 64
    double2* dvec = nullptr;    // 64
    double2* Ain = nullptr;     // host-call staging, 64 x 64
    double2* res = nullptr;     // [0] lhaf, [1] (abs_sum, -)
    void* E = nullptr;
    size_t E_cap = 0;           // bytes
    double* partials = nullptr;
    size_t partials_cap = 0;    // partial records
    uint64_t* masks = nullptr;
    double2* terms = nullptr;
    size_t masks_cap = 0, terms_cap = 0;
    BatchRunner* runner = nullptr;  // eager batch runner of the sampling chain, created on first use
    void* smats = nullptr;          // packed loop-hafnian matrices of one sampling step
    size_t smats_cap = 0;           // bytes
    void* na_scratch = nullptr;     // device address of this device's no-allocation scratch array
    // lane grid per (n, s); -1 = heuristic default.  layout_multi is the
    // choice for batch plans, where many launches share the device: the
    // tuner's best among the grids with one La Budde team per subset group
    int layout[gbs::kMaxPairs + 1][gbs::kMaxPairs + 1];
    int layout_multi[gbs::kMaxPairs + 1][gbs::kMaxPairs + 1];
    bool tuned[gbs::kMaxPairs + 1];
    char name[64] = {0};
    DevCtx() {
        for (auto& row : layout)
            for (int& v : row) v = -1;
        for (auto& row : layout_multi)
            for (int& v : row) v = -1;
        for (bool& t : tuned) t = false;
    }
};

extern std::mutex g_mutex;  // serialises every library call

gbs_status current_ctx(DevCtx** out);
// Context of device `dev` if gbs_init (or an earlier call) created it, else
// nullptr; never creates one (caller holds g_mutex).
DevCtx* existing_ctx(int dev);
// Looks up this device's no-allocation scratch array (gbs_noalloc.cpp).
gbs_status noalloc_setup(DevCtx* c);
// Lane grid of subsets of size s of an n-pair loop hafnian; batch = true
// gives the batch-plan choice.
int layout_for(const DevCtx* c, int n, int s, bool batch = false, bool fp32 = false);
// Tile offset of C for size-s subsets on `lay` (charpoly_front_offset of m = 2s).
int layout_front_offset(int lay, int s);
// Consults the autotune cache / runs the tuner once per n (uses the workspace,
// so it is called before the caller's matrix is prepared).
gbs_status maybe_tune(DevCtx* c, int n);
gbs_status ensure_buffer(void** p, size_t* cap, size_t need, size_t elem);
// Every device allocation of the library goes through here.  Test hook for the
// out-of-memory paths: while the environment variable GBS_TEST_FAIL_ALLOC is
// "1", it fails (nullptr, hipErrorOutOfMemory) without allocating.
hipError_t dev_malloc(void** p, size_t bytes);
// Times each valid lane grid per subset size of an n-pair loop hafnian.
gbs_status autotune_impl(DevCtx* c, int n, gbs_tune_report* rep);

// ---- batches of loop hafnians (gbs_batch.cpp) ----

// One persistent per-subset launch of a batch schedule.
struct CharpolyLaunch {
    int round, layout, s_rep, inst, variant, offset;
    int tile_begin, ntiles;  // range in the device tile array
    int counter;
    double flops = 0.0, subsets = 0.0;  // yardstick flops and subsets of its tiles
    std::string kernel;                 // kernel instance name (as the profiler prints it)
};
// One series launch (all blocks of one round and one n).
struct SeriesLaunch {
    int round, n;
    int block_begin, nblocks;
};

// Host-side schedule of a batch of loop hafnians of dimensions `dims`:
// tiles, rounds over two coefficient buffers, launches, and the sizes of the
// device arrays they need.  Built without touching the device.
struct BatchSchedule {
    int count = 0;
    bool fp32 = false;
    int64_t tile_subsets = 0;
    int series_per_thread = 8;  // subsets per lane of a series block (64 lanes; a block never spans tiles)
    int rounds = 0;
    int max_n = 0;
    int64_t subset_terms = 0;
    double flops = 0.0;
    int64_t in_elems = 0, a0_elems = 0, d_elems = 0;  // packed input, padded A0 blocks, loop weights
    int64_t ebuf_bytes = 16;                          // per coefficient buffer
    std::vector<int> dims, npair;
    std::vector<int64_t> in_off, a0_off, d_off;
    std::vector<gbs::BatchTile> tiles;  // device order: (round, instance), largest first
    std::vector<gbs::SeriesBlock> sblocks;
    std::vector<int64_t> pbeg;          // partial records of item i: [pbeg[i], pbeg[i+1])
    std::vector<CharpolyLaunch> cp;
    std::vector<SeriesLaunch> se;
    std::vector<int> small;             // FP64 items with 1 <= n <= kSmallPairs, largest n first: one wavefront each
};
// tile_offsets: FP64 tiles keep C at the front tile offset of their m (one
// persistent launch per offset); captured plans use it, the sampler's eagerly
// run steps do not (the extra launches cost it more than the offset saves).
void batch_schedule(const DevCtx* c, const std::vector<int>& dims, bool fp32, int64_t tile_subsets,
                    int64_t round_bytes, bool tile_offsets, BatchSchedule& S);

// Device arrays a schedule runs on.  `mats` is the packed input.
struct BatchDev {
    const double2* mats = nullptr;
    double2 *a0 = nullptr, *dv = nullptr;
    gbs::BatchItem* items = nullptr;
    int64_t* in_off = nullptr;
    int* dims = nullptr;
    gbs::BatchTile* tiles = nullptr;
    gbs::SeriesBlock* sblocks = nullptr;
    int64_t* pbeg = nullptr;
    double* partials = nullptr;
    unsigned* counters = nullptr;
    void* ebuf[2] = {nullptr, nullptr};
    double2* out = nullptr;
    double* abs = nullptr;
    int* small = nullptr;
    const uint64_t* binom = nullptr;  // binomial table (kBinomStride^2)
    const int4* lbmap = nullptr;      // La Budde lane maps (gbs::lb_fill_table)
};
constexpr int kBatchBranches = 4;  // parallel streams of the per-subset launches of one round
// Issues the whole schedule: counter fill, prep, rounds of per-subset launches
// on the branch streams (joined into `cs` through events from `new_event`),
// series launches and the per-item reduction, all ordered after prior work on
// `cs`.  Works eagerly and under stream capture alike.
// With `prof`, per-subset launches are timed when gbs_profile_enable is on
// (never under stream capture).
gbs_status batch_enqueue(DevCtx* c, const BatchSchedule& S, const BatchDev& d, hipStream_t cs, hipStream_t* br,
                         const std::function<hipError_t(hipEvent_t*)>& new_event, bool prof);

// Per-launch timing (gbs_profile_*): true while profiling is on.
bool profiling_on();
// Runs `launch`; while profiling is on, brackets it with a HIP event pair on
// `st`, recorded as a per-subset kernel launch of instance `kernel`.
hipError_t prof_charpoly_launch(double flops, double subsets, hipStream_t st,
                                const std::function<hipError_t()>& launch, const std::string& kernel);

// Eager runner of batch schedules on reusable, growing device buffers, for
// callers whose batches change from one run to the next.
struct BatchRunner;
gbs_status runner_create(DevCtx* c, BatchRunner** out);
void runner_free(BatchRunner* r);
// Runs the batch of dimensions S.dims on packed matrices mats_dev (device).
// The meta arrays (items, offsets, tiles) are uploaded first; `before_sum`
// (optional) is then enqueued on `st` so that it can fill mats_dev from them
// (it receives the device in_off and dims arrays).  Results: out[i] and
// abs[i] in the runner's device buffers (runner_out / runner_abs), valid
// after `st` completes.
gbs_status runner_run(BatchRunner* r, const BatchSchedule& S, const double2* mats_dev, hipStream_t st,
                      const std::function<gbs_status(const int64_t* in_off_dev, const int* dims_dev)>& before_sum);
double2* runner_out(BatchRunner* r);

}  // namespace gbs_host
