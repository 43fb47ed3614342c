// Internal declarations shared by the host translation units of libgbs_lhaf.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

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
// Flop yardstick of one subset of size s of an n-pair loop hafnian.
double subset_flops(int n, int s);

// Per-device workspace.  All library calls take g_mutex, so one context is
// used by one call at a time; `done` orders reuse across caller streams.
struct DevCtx {
    int device = -1;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr, t0 = nullptr, t1 = nullptr;
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
    size_t masks_cap = 0;
    // lane grid per (n, s); -1 = heuristic default
    int layout[gbs::kMaxPairs + 1][gbs::kMaxPairs + 1];
    bool tuned[gbs::kMaxPairs + 1];
    char name[64] = {0};
    DevCtx() {
        for (auto& row : layout)
            for (int& v : row) v = -1;
        for (bool& t : tuned) t = false;
    }
};

extern std::mutex g_mutex;  // serialises every library call

gbs_status current_ctx(DevCtx** out);
int layout_for(const DevCtx* c, int n, int s);
// Consults the autotune cache / runs the tuner once per n (uses the workspace,
// so it is called before the caller's matrix is prepared).
gbs_status maybe_tune(DevCtx* c, int n);
gbs_status ensure_buffer(void** p, size_t* cap, size_t need, size_t elem);
// Times each valid lane grid per subset size of an n-pair loop hafnian.
gbs_status autotune_impl(DevCtx* c, int n, gbs_tune_report* rep);

}  // namespace gbs_host
