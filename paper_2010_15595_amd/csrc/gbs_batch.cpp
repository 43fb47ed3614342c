// Batched loop hafnians (C ABI gbs_batch_*): a plan splits the subset sums of
// many loop hafnians of uneven size into tiles, assigns them to rounds over two
// alternating coefficient buffers, and captures the whole schedule into one
// HIP graph:
//
//   fill counters -> prep all items
//   round r: one persistent per-subset launch per kernel instance (parallel
//            graph branches; each waits for the series of round r-2, which
//            read the same buffer) -> series launches per n
//   per-item fixed-order compensated reduction
//
// Tiles within a launch are ordered largest first, so the device counter
// hands out long work first (longest-processing-time schedule).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <numeric>
#include <vector>

#include "gbs_internal.h"

using namespace gbs_host;

namespace {

constexpr int kSeriesPerThread = 8;                   // most subsets per lane in the series kernel
constexpr int kPersistentWaves = 256 * 8;             // wavefronts of the small-item launch

}  // namespace

struct gbs_plan {
    int device = 0;
    BatchSchedule S;
    double tune_ms = 0.0;
    size_t bytes = 0;
    BatchDev d;
    double2* staging = nullptr;  // packed input copy (the graph reads a fixed address)
    hipStream_t cs = nullptr;
    hipStream_t br[kBatchBranches] = {};
    std::vector<hipEvent_t> events;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    std::vector<hipEvent_t> eager_events;  // events of profiled eager runs, reused run to run
};

namespace gbs_host {

void batch_schedule(const DevCtx* c, const std::vector<int>& dims, bool fp32, int64_t tile_subsets,
                    int64_t round_bytes, bool tile_offsets, BatchSchedule& S) {
    S = BatchSchedule();
    S.count = (int)dims.size();
    S.fp32 = fp32;
    S.tile_subsets = tile_subsets;
    // series blocks stay within one tile: small tiles get fewer subsets per lane
    S.series_per_thread = (int)std::max<int64_t>(1, std::min<int64_t>(kSeriesPerThread, (tile_subsets + 63) / 64));
    const int64_t sblock = 64 * (int64_t)S.series_per_thread;
    S.dims = dims;
    const int64_t vbytes = fp32 ? (int64_t)sizeof(float2) : (int64_t)sizeof(double2);
    const int nitems = S.count;

    // items (flop yardstick per dimension computed once)
    double flops_of[GBS_MAX_DIM + 1];
    bool have_flops[GBS_MAX_DIM + 1] = {};
    S.in_off.resize(nitems);
    S.a0_off.resize(nitems);
    S.d_off.resize(nitems);
    S.npair.resize(nitems);
    for (int i = 0; i < nitems; ++i) {
        const int N = dims[i], Np = N + (N & 1);
        S.npair[i] = Np / 2;
        S.in_off[i] = S.in_elems;
        S.a0_off[i] = S.a0_elems;
        S.d_off[i] = S.d_elems;
        S.in_elems += (int64_t)N * N;
        S.a0_elems += (int64_t)Np * Np;
        S.d_elems += Np;
        S.max_n = std::max(S.max_n, Np / 2);
        S.subset_terms += (int64_t)1 << (Np / 2);
        if (!have_flops[N]) {
            flops_of[N] = gbs_yardstick_flops(N);
            have_flops[N] = true;
        }
        S.flops += flops_of[N];
    }

    // tiles: (item, s, rank range); series blocks and partial ranges per item
    struct HostTile {
        gbs::BatchTile t;
        int inst, layout, variant, offset;
        double cost;
        int round;
    };
    // items with n <= small_pairs pairs are summed whole by one wavefront each
    // (GBS_SMALL_PAIRS overrides the default kSmallPairs; 0 disables)
    int small_pairs = gbs::kSmallPairs;
    if (const char* e = std::getenv("GBS_SMALL_PAIRS")) small_pairs = std::max(0, std::min(gbs::kSmallPairs, atoi(e)));
    std::vector<HostTile> ht;
    for (int i = 0; i < nitems; ++i) {
        const int n = S.npair[i];
        if (!fp32 && n >= 1 && n <= small_pairs) {
            S.small.push_back(i);
            continue;
        }
        for (int s = 1; s <= n; ++s) {
            const uint64_t cnt = binom_host(n, s);
            const int lay = layout_for(c, n, s, true);
            for (uint64_t r0 = 0; r0 < cnt; r0 += (uint64_t)tile_subsets) {
                HostTile h{};
                h.t.rank0 = r0;
                h.t.count = std::min<uint64_t>((uint64_t)tile_subsets, cnt - r0);
                h.t.item = i;
                h.t.s = s;
                h.layout = lay;
                h.variant = gbs::charpoly_variant(lay, n);
                // with tile_offsets, FP64 tiles keep C at the front offset of
                // their m (a launch per offset); FP32 tiles at offset 0
                h.offset = (tile_offsets && !fp32) ? layout_front_offset(lay, s) : 0;
                h.inst = 32 * gbs::charpoly_instance(lay, s) + 8 * h.variant + h.offset;
                h.cost = subset_flops(n, s) * (double)h.t.count;
                ht.push_back(h);
            }
        }
    }
    {  // largest n first, stable: a counting sort over n = 1..small_pairs
        std::vector<int> by_n[gbs::kSmallPairs + 1];
        for (int i : S.small) by_n[S.npair[i]].push_back(i);
        S.small.clear();
        for (int n = gbs::kSmallPairs; n >= 1; --n) S.small.insert(S.small.end(), by_n[n].begin(), by_n[n].end());
    }
    // partials: per item contiguous, in (item, s, rank) order
    S.pbeg.assign(nitems + 1, 0);
    std::vector<int64_t> tile_pidx(ht.size());
    {
        int64_t pi = 0;
        size_t k = 0;
        for (int i = 0; i < nitems; ++i) {
            S.pbeg[i] = pi;
            while (k < ht.size() && ht[k].t.item == i) {
                tile_pidx[k] = pi;
                pi += (int64_t)((ht[k].t.count + sblock - 1) / sblock);
                ++k;
            }
        }
        S.pbeg[nitems] = pi;
    }
    // rounds: tiles in decreasing cost, filled up to round_bytes of coefficients
    std::vector<size_t> order(ht.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return ht[a].cost > ht[b].cost; });
    std::vector<int64_t> round_fill;
    for (size_t k : order) {
        const int64_t need = (int64_t)ht[k].t.count * 2 * (S.npair[ht[k].t.item] + 2) * vbytes;
        int r = (int)round_fill.size() - 1;
        if (r < 0 || round_fill[r] + need > round_bytes) {
            round_fill.push_back(0);
            r = (int)round_fill.size() - 1;
        }
        ht[k].t.eoff = (uint64_t)(round_fill[r] / vbytes);
        round_fill[r] += need;
        ht[k].round = r;
    }
    S.rounds = (int)round_fill.size();
    S.ebuf_bytes = round_fill.empty() ? 16 : *std::max_element(round_fill.begin(), round_fill.end());

    // device tile array: grouped by (round, instance), largest first inside a group
    std::vector<size_t> dorder(order);
    std::stable_sort(dorder.begin(), dorder.end(), [&](size_t a, size_t b) {
        if (ht[a].round != ht[b].round) return ht[a].round < ht[b].round;
        return ht[a].inst < ht[b].inst;  // stable: cost order kept inside
    });
    S.tiles.resize(dorder.size());
    std::vector<int> pos_of(ht.size());
    for (size_t q = 0; q < dorder.size(); ++q) {
        S.tiles[q] = ht[dorder[q]].t;
        pos_of[dorder[q]] = (int)q;
    }
    for (size_t q = 0; q < dorder.size();) {
        size_t e = q;
        while (e < dorder.size() && ht[dorder[e]].round == ht[dorder[q]].round &&
               ht[dorder[e]].inst == ht[dorder[q]].inst)
            ++e;
        const HostTile& h = ht[dorder[q]];
        CharpolyLaunch L{h.round, h.layout, h.t.s, h.inst, h.variant, h.offset, (int)q, (int)(e - q), (int)S.cp.size()};
        for (size_t k = q; k < e; ++k) {
            L.flops += ht[dorder[k]].cost;
            L.subsets += (double)ht[dorder[k]].t.count;
        }
        {
            const int P = (h.layout == gbs::kLayout44) ? 4 : 8, Q = (h.layout == gbs::kLayout88) ? 8 : 4;
            const int m = 2 * h.t.s, team = h.variant ? 64 : P * Q;
            char buf[96];
            snprintf(buf, sizeof buf, "charpoly_batch_kernel<%d, %d, %d, %d, %s, %d, %d>", P, Q, (m + P - 1) / P,
                     (m + Q - 1) / Q, fp32 ? "float2" : "double2", team, h.offset);
            L.kernel = buf;
        }
        S.cp.push_back(L);
        q = e;
    }
    // series blocks grouped by (round, n)
    std::map<std::pair<int, int>, std::vector<gbs::SeriesBlock>> by;
    for (size_t k = 0; k < ht.size(); ++k) {
        const int n = S.npair[ht[k].t.item];
        auto& v = by[{ht[k].round, n}];
        int64_t pi = tile_pidx[k];
        for (uint64_t s0 = 0; s0 < ht[k].t.count; s0 += (uint64_t)sblock)
            v.push_back(gbs::SeriesBlock{pos_of[k], (int)pi++, s0});
    }
    for (auto& kv : by) {
        S.se.push_back(SeriesLaunch{kv.first.first, kv.first.second, (int)S.sblocks.size(), (int)kv.second.size()});
        S.sblocks.insert(S.sblocks.end(), kv.second.begin(), kv.second.end());
    }
}

gbs_status batch_enqueue(DevCtx* c, const BatchSchedule& S, const BatchDev& d, hipStream_t cs, hipStream_t* br,
                         const std::function<hipError_t(hipEvent_t*)>& new_event, bool prof) {
    (void)c;
    const int nitems = S.count;
    HIP_TRY(gbs::launch_fill_u32(d.counters, (int)std::max<size_t>(1, S.cp.size()), cs));
    HIP_TRY(gbs::launch_batch_prep(d.mats, d.in_off, d.dims, d.items, nitems, cs));
    hipEvent_t ev_prep;
    HIP_TRY(new_event(&ev_prep));
    HIP_TRY(hipEventRecord(ev_prep, cs));
    hipEvent_t ev_small = nullptr;
    if (!S.small.empty()) {
        hipStream_t bs = br[kBatchBranches - 1];
        HIP_TRY(hipStreamWaitEvent(bs, ev_prep, 0));
        HIP_TRY(gbs::launch_small_items(d.small, (int)S.small.size(), d.items, d.binom, d.lbmap, d.out, d.abs,
                                        kPersistentWaves, bs));
        HIP_TRY(new_event(&ev_small));
        HIP_TRY(hipEventRecord(ev_small, bs));
    }
    std::vector<hipEvent_t> ev_series(S.rounds, nullptr);
    size_t ci = 0, si = 0;
    for (int r = 0; r < S.rounds; ++r) {
        void* E = d.ebuf[r % 2];
        std::vector<hipEvent_t> joins;
        int b = 0;
        for (; ci < S.cp.size() && S.cp[ci].round == r; ++ci, ++b) {
            const CharpolyLaunch& L = S.cp[ci];
            hipStream_t bs = br[b % kBatchBranches];
            HIP_TRY(hipStreamWaitEvent(bs, ev_prep, 0));
            if (r >= 2) HIP_TRY(hipStreamWaitEvent(bs, ev_series[r - 2], 0));
            // as many wavefronts as fit on the device, no more than there are tiles
            auto launch = [&]() {
                return gbs::launch_charpoly_batch(L.layout, L.s_rep, L.variant, L.offset, S.max_n + 1, S.fp32 ? 1 : 0,
                                                  d.tiles + L.tile_begin, L.ntiles, d.items, d.binom, d.lbmap,
                                                  d.counters + L.counter, E, L.ntiles, bs);
            };
            if (prof && profiling_on())
                HIP_TRY(prof_charpoly_launch(L.flops, L.subsets, bs, launch, L.kernel));
            else
                HIP_TRY(launch());
            hipEvent_t ej;
            HIP_TRY(new_event(&ej));
            HIP_TRY(hipEventRecord(ej, bs));
            joins.push_back(ej);
        }
        for (hipEvent_t ej : joins) HIP_TRY(hipStreamWaitEvent(cs, ej, 0));
        for (; si < S.se.size() && S.se[si].round == r; ++si) {
            const SeriesLaunch& L = S.se[si];
            HIP_TRY(gbs::launch_series_batch(L.n, S.fp32 ? 1 : 0, d.sblocks + L.block_begin, L.nblocks, d.tiles,
                                             d.items, E, S.series_per_thread, d.partials, cs));
        }
        HIP_TRY(new_event(&ev_series[r]));
        HIP_TRY(hipEventRecord(ev_series[r], cs));
    }
    if (ev_small) HIP_TRY(hipStreamWaitEvent(cs, ev_small, 0));
    HIP_TRY(gbs::launch_item_reduce(d.pbeg, nitems, d.partials, d.items, d.out, d.abs, cs));
    return GBS_OK;
}

}  // namespace gbs_host

namespace {

template <class T>
gbs_status upload(T** dst, const std::vector<T>& src, size_t* bytes) {
    const size_t nb = std::max<size_t>(1, src.size()) * sizeof(T);
    hipError_t e = dev_malloc((void**)dst, nb);
    if (e != hipSuccess) return fail(GBS_E_NOMEM, "hipMalloc(%zu) failed: %s", nb, hipGetErrorString(e));
    *bytes += nb;
    if (!src.empty()) HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return GBS_OK;
}

gbs_status dmalloc(void** dst, size_t nb, size_t* bytes) {
    nb = std::max<size_t>(nb, 16);
    hipError_t e = dev_malloc(dst, nb);
    if (e != hipSuccess) return fail(GBS_E_NOMEM, "hipMalloc(%zu) failed: %s", nb, hipGetErrorString(e));
    *bytes += nb;
    return GBS_OK;
}

void plan_free(gbs_plan* p) {
    if (!p) return;
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    for (hipEvent_t e : p->events) hipEventDestroy(e);
    for (hipEvent_t e : p->eager_events) hipEventDestroy(e);
    if (p->t0) hipEventDestroy(p->t0);
    if (p->t1) hipEventDestroy(p->t1);
    for (hipStream_t s : p->br)
        if (s) hipStreamDestroy(s);
    if (p->cs) hipStreamDestroy(p->cs);
    const BatchDev& d = p->d;
    void* bufs[] = {p->staging, d.a0,       d.dv,       d.items,   d.in_off,  d.dims, d.tiles,
                    d.sblocks,  d.pbeg,     d.partials, d.counters, d.ebuf[0], d.ebuf[1], d.out,
                    d.abs,      d.small,    const_cast<uint64_t*>(d.binom), const_cast<int4*>(d.lbmap)};
    for (void* b : bufs)
        if (b) hipFree(b);
    delete p;
}

std::vector<gbs::BatchItem> item_table(const BatchSchedule& S, double2* a0, double2* dv) {
    std::vector<gbs::BatchItem> items(S.count);
    for (int i = 0; i < S.count; ++i)
        items[i] = gbs::BatchItem{a0 + S.a0_off[i], dv + S.d_off[i], 2 * S.npair[i], S.npair[i]};
    return items;
}

// Builds schedule, buffers and graph for one tile size into p (freed by the
// caller on failure).
gbs_status plan_build_into(DevCtx* c, const std::vector<int>& dims, bool fp32, int64_t tile_subsets,
                           int64_t round_bytes, gbs_plan* p) {
    p->device = c->device;
    BatchSchedule& S = p->S;
    batch_schedule(c, dims, fp32, tile_subsets, round_bytes, true, S);
    const int nitems = S.count;
    gbs_status st;
    size_t& B = p->bytes;
    BatchDev& d = p->d;
    if ((st = dmalloc((void**)&p->staging, sizeof(double2) * (size_t)S.in_elems, &B)) != GBS_OK) return st;
    d.mats = p->staging;
    if ((st = dmalloc((void**)&d.a0, sizeof(double2) * (size_t)S.a0_elems, &B)) != GBS_OK) return st;
    if ((st = dmalloc((void**)&d.dv, sizeof(double2) * (size_t)S.d_elems, &B)) != GBS_OK) return st;
    if ((st = upload(&d.items, item_table(S, d.a0, d.dv), &B)) != GBS_OK) return st;
    if ((st = upload(&d.in_off, S.in_off, &B)) != GBS_OK) return st;
    if ((st = upload(&d.dims, S.dims, &B)) != GBS_OK) return st;
    if ((st = upload(&d.tiles, S.tiles, &B)) != GBS_OK) return st;
    if ((st = upload(&d.sblocks, S.sblocks, &B)) != GBS_OK) return st;
    if ((st = upload(&d.pbeg, S.pbeg, &B)) != GBS_OK) return st;
    if ((st = upload(&d.small, S.small, &B)) != GBS_OK) return st;
    {  // the plan's own copies of the context's tables: a plan outlives gbs_finalize
        void* tb = nullptr;
        const size_t nb = sizeof(uint64_t) * gbs::kBinomStride * gbs::kBinomStride;
        if ((st = dmalloc(&tb, nb, &B)) != GBS_OK) return st;
        d.binom = static_cast<uint64_t*>(tb);
        HIP_TRY(hipMemcpy(tb, c->binom, nb, hipMemcpyDeviceToDevice));
        const size_t nl = sizeof(int4) * gbs::kLbTableEntries;
        tb = nullptr;
        if ((st = dmalloc(&tb, nl, &B)) != GBS_OK) return st;
        d.lbmap = static_cast<int4*>(tb);
        HIP_TRY(hipMemcpy(tb, c->lbmap, nl, hipMemcpyDeviceToDevice));
    }
    if ((st = dmalloc((void**)&d.partials, sizeof(double) * 5 * (size_t)std::max<int64_t>(1, S.pbeg[nitems]), &B)) !=
        GBS_OK)
        return st;
    if ((st = dmalloc((void**)&d.counters, sizeof(unsigned) * std::max<size_t>(1, S.cp.size()), &B)) != GBS_OK)
        return st;
    for (int b = 0; b < 2 && b < S.rounds; ++b)
        if ((st = dmalloc(&d.ebuf[b], (size_t)S.ebuf_bytes, &B)) != GBS_OK) return st;
    if ((st = dmalloc((void**)&d.out, sizeof(double2) * nitems, &B)) != GBS_OK) return st;
    if ((st = dmalloc((void**)&d.abs, sizeof(double) * nitems, &B)) != GBS_OK) return st;

    // graph capture
    HIP_TRY(hipStreamCreateWithFlags(&p->cs, hipStreamNonBlocking));
    for (hipStream_t& s : p->br) HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    HIP_TRY(hipEventCreate(&p->t0));
    HIP_TRY(hipEventCreate(&p->t1));
    auto new_event = [p](hipEvent_t* e) -> hipError_t {
        hipError_t r = hipEventCreateWithFlags(e, hipEventDisableTiming);
        if (r == hipSuccess) p->events.push_back(*e);
        return r;
    };
    HIP_TRY(hipStreamBeginCapture(p->cs, hipStreamCaptureModeThreadLocal));
    if ((st = batch_enqueue(c, S, d, p->cs, p->br, new_event, false)) != GBS_OK) return st;
    HIP_TRY(hipStreamEndCapture(p->cs, &p->graph));
    HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return GBS_OK;
}

gbs_status plan_build(DevCtx* c, const std::vector<int>& dims, bool fp32, int64_t tile_subsets, int64_t round_bytes,
                      gbs_plan** out) {
    gbs_plan* p = new gbs_plan();
    const gbs_status st = plan_build_into(c, dims, fp32, tile_subsets, round_bytes, p);
    if (st != GBS_OK) {
        // a failed capture leaves the stream capturing: end it and drop the partial graph
        hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
        if (p->cs && hipStreamIsCapturing(p->cs, &cst) == hipSuccess && cst != hipStreamCaptureStatusNone) {
            hipGraph_t g = nullptr;
            hipStreamEndCapture(p->cs, &g);
            if (g) hipGraphDestroy(g);
        }
        plan_free(p);
        return st;
    }
    *out = p;
    return GBS_OK;
}

}  // namespace

// ---- eager runner -----------------------------------------------------------

struct gbs_host::BatchRunner {
    DevCtx* c = nullptr;
    hipStream_t br[kBatchBranches] = {};
    std::vector<hipEvent_t> events;
    size_t ev_next = 0;
    hipEvent_t upload_done = nullptr;
    bool uploaded = false;
    char* host_meta = nullptr;  // pinned staging of the meta arrays
    size_t host_meta_cap = 0;
    void* meta = nullptr;
    size_t meta_cap = 0;
    void *a0 = nullptr, *dv = nullptr, *partials = nullptr, *counters = nullptr, *out = nullptr, *abs = nullptr;
    size_t a0_cap = 0, dv_cap = 0, partials_cap = 0, counters_cap = 0, out_cap = 0, abs_cap = 0;
    void* ebuf[2] = {nullptr, nullptr};
    size_t ebuf_cap[2] = {0, 0};
};

namespace gbs_host {

gbs_status runner_create(DevCtx* c, BatchRunner** out) {
    BatchRunner* r = new BatchRunner();
    r->c = c;
    *out = r;
    for (hipStream_t& s : r->br) HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&r->upload_done, hipEventDisableTiming));
    return GBS_OK;
}

void runner_free(BatchRunner* r) {
    if (!r) return;
    for (hipStream_t s : r->br)
        if (s) hipStreamSynchronize(s);
    for (hipEvent_t e : r->events) hipEventDestroy(e);
    if (r->upload_done) hipEventDestroy(r->upload_done);
    for (hipStream_t s : r->br)
        if (s) hipStreamDestroy(s);
    if (r->host_meta) hipHostFree(r->host_meta);
    void* bufs[] = {r->meta, r->a0, r->dv, r->partials, r->counters, r->out, r->abs, r->ebuf[0], r->ebuf[1]};
    for (void* b : bufs)
        if (b) hipFree(b);
    delete r;
}

double2* runner_out(BatchRunner* r) { return static_cast<double2*>(r->out); }

gbs_status runner_run(BatchRunner* r, const BatchSchedule& S, const double2* mats_dev, hipStream_t st,
                      const std::function<gbs_status(const int64_t* in_off_dev, const int* dims_dev)>& before_sum) {
    if (S.count == 0) return GBS_OK;
    // the pinned staging and the buffers may be reused only once the previous run has finished with them
    if (r->uploaded) HIP_TRY(hipEventSynchronize(r->upload_done));
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t n_items = sizeof(gbs::BatchItem) * S.count, n_inoff = sizeof(int64_t) * S.in_off.size(),
                 n_dims = sizeof(int) * S.dims.size(), n_tiles = sizeof(gbs::BatchTile) * S.tiles.size(),
                 n_sb = sizeof(gbs::SeriesBlock) * S.sblocks.size(), n_pbeg = sizeof(int64_t) * S.pbeg.size(),
                 n_small = sizeof(int) * S.small.size();
    const size_t o_items = 0, o_inoff = align(o_items + n_items), o_dims = align(o_inoff + n_inoff),
                 o_tiles = align(o_dims + n_dims), o_sb = align(o_tiles + n_tiles), o_pbeg = align(o_sb + n_sb),
                 o_small = align(o_pbeg + n_pbeg), total = align(o_small + n_small);
    const size_t npart = 5 * (size_t)std::max<int64_t>(1, S.pbeg[S.count]);
    const bool grow = r->meta_cap < total || r->a0_cap < sizeof(double2) * (size_t)S.a0_elems ||
                      r->dv_cap < sizeof(double2) * (size_t)S.d_elems || r->partials_cap < sizeof(double) * npart ||
                      r->counters_cap < sizeof(unsigned) * std::max<size_t>(1, S.cp.size()) ||
                      r->out_cap < sizeof(double2) * S.count || r->abs_cap < sizeof(double) * S.count ||
                      r->ebuf_cap[0] < (size_t)S.ebuf_bytes || (S.rounds > 1 && r->ebuf_cap[1] < (size_t)S.ebuf_bytes);
    if (grow) {
        // buffers still in use by earlier work on st are released only after it
        HIP_TRY(hipStreamSynchronize(st));
        gbs_status e;
        if ((e = ensure_buffer(&r->meta, &r->meta_cap, total, 1)) != GBS_OK) return e;
        if ((e = ensure_buffer(&r->a0, &r->a0_cap, sizeof(double2) * std::max<size_t>(1, S.a0_elems), 1)) != GBS_OK)
            return e;
        if ((e = ensure_buffer(&r->dv, &r->dv_cap, sizeof(double2) * std::max<size_t>(1, S.d_elems), 1)) != GBS_OK)
            return e;
        if ((e = ensure_buffer(&r->partials, &r->partials_cap, sizeof(double) * npart, 1)) != GBS_OK) return e;
        if ((e = ensure_buffer(&r->counters, &r->counters_cap, sizeof(unsigned) * std::max<size_t>(1, S.cp.size()),
                               1)) != GBS_OK)
            return e;
        if ((e = ensure_buffer(&r->out, &r->out_cap, sizeof(double2) * S.count, 1)) != GBS_OK) return e;
        if ((e = ensure_buffer(&r->abs, &r->abs_cap, sizeof(double) * S.count, 1)) != GBS_OK) return e;
        for (int b = 0; b < 2 && b < S.rounds; ++b)
            if ((e = ensure_buffer(&r->ebuf[b], &r->ebuf_cap[b], (size_t)S.ebuf_bytes, 1)) != GBS_OK) return e;
    }
    if (r->host_meta_cap < total) {
        if (r->host_meta) HIP_TRY(hipHostFree(r->host_meta));
        r->host_meta = nullptr;
        r->host_meta_cap = 0;
        HIP_TRY(hipHostMalloc((void**)&r->host_meta, total, hipHostMallocDefault));
        r->host_meta_cap = total;
    }
    const std::vector<gbs::BatchItem> items = item_table(S, (double2*)r->a0, (double2*)r->dv);
    char* h = r->host_meta;
    std::memcpy(h + o_items, items.data(), n_items);
    std::memcpy(h + o_inoff, S.in_off.data(), n_inoff);
    std::memcpy(h + o_dims, S.dims.data(), n_dims);
    if (n_tiles) std::memcpy(h + o_tiles, S.tiles.data(), n_tiles);
    if (n_sb) std::memcpy(h + o_sb, S.sblocks.data(), n_sb);
    std::memcpy(h + o_pbeg, S.pbeg.data(), n_pbeg);
    if (n_small) std::memcpy(h + o_small, S.small.data(), n_small);
    HIP_TRY(hipMemcpyAsync(r->meta, h, total, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(r->upload_done, st));
    r->uploaded = true;

    char* m = static_cast<char*>(r->meta);
    BatchDev d;
    d.mats = mats_dev;
    d.a0 = (double2*)r->a0;
    d.dv = (double2*)r->dv;
    d.items = (gbs::BatchItem*)(m + o_items);
    d.in_off = (int64_t*)(m + o_inoff);
    d.dims = (int*)(m + o_dims);
    d.tiles = (gbs::BatchTile*)(m + o_tiles);
    d.sblocks = (gbs::SeriesBlock*)(m + o_sb);
    d.pbeg = (int64_t*)(m + o_pbeg);
    d.small = (int*)(m + o_small);
    d.partials = (double*)r->partials;
    d.counters = (unsigned*)r->counters;
    d.ebuf[0] = r->ebuf[0];
    d.ebuf[1] = r->ebuf[1];
    d.out = (double2*)r->out;
    d.abs = (double*)r->abs;
    d.binom = r->c->binom;  // the runner lives and dies with its context
    d.lbmap = r->c->lbmap;
    if (before_sum) {
        const gbs_status e = before_sum(d.in_off, d.dims);
        if (e != GBS_OK) return e;
    }
    r->ev_next = 0;
    auto new_event = [r](hipEvent_t* e) -> hipError_t {
        if (r->ev_next == r->events.size()) {
            hipEvent_t ev;
            const hipError_t err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (err != hipSuccess) return err;
            r->events.push_back(ev);
        }
        *e = r->events[r->ev_next++];
        return hipSuccess;
    };
    // while per-launch profiling is on, every branch runs on st (each launch timed alone)
    hipStream_t serial[kBatchBranches];
    for (hipStream_t& b : serial) b = st;
    return batch_enqueue(r->c, S, d, st, profiling_on() ? serial : r->br, new_event, true);
}

}  // namespace gbs_host

namespace {

int kernel_nodes_of(const gbs_plan* p) { return 3 + (int)p->S.cp.size() + (int)p->S.se.size(); }

gbs_status plan_run(gbs_plan* p, const gbs_z* mats_dev, gbs_z* out_dev, double* abs_dev, hipStream_t s,
                    bool prof = false) {
    if (p->S.in_elems > 0)
        HIP_TRY(hipMemcpyAsync(p->staging, mats_dev, sizeof(double2) * (size_t)p->S.in_elems, hipMemcpyDeviceToDevice,
                               s));
    if (prof && profiling_on()) {
        // the captured schedule issued eagerly with every branch on the caller's
        // stream, so each per-subset launch is timed alone on the whole device (as
        // single evaluations time theirs), not while it shares the device with
        // the other branches
        hipStream_t serial[kBatchBranches];
        for (hipStream_t& b : serial) b = s;
        size_t next = 0;
        auto new_event = [p, &next](hipEvent_t* e) -> hipError_t {
            if (next == p->eager_events.size()) {
                hipEvent_t ev;
                const hipError_t err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
                if (err != hipSuccess) return err;
                p->eager_events.push_back(ev);
            }
            *e = p->eager_events[next++];
            return hipSuccess;
        };
        const gbs_status st = batch_enqueue(nullptr, p->S, p->d, s, serial, new_event, true);
        if (st != GBS_OK) return st;
    } else {
        HIP_TRY(hipGraphLaunch(p->exec, s));
    }
    if (out_dev) HIP_TRY(hipMemcpyAsync(out_dev, p->d.out, sizeof(double2) * p->S.count, hipMemcpyDeviceToDevice, s));
    if (abs_dev) HIP_TRY(hipMemcpyAsync(abs_dev, p->d.abs, sizeof(double) * p->S.count, hipMemcpyDeviceToDevice, s));
    return GBS_OK;
}

}  // namespace

extern "C" {

gbs_status gbs_batch_plan_create(const int32_t* dims, int32_t count, gbs_precision prec, int32_t flags,
                                 gbs_plan** plan) {
    if (!plan || count < 0 || (count > 0 && !dims)) return fail(GBS_E_ARG, "bad batch arguments");
    if (prec == GBS_DD) return fail(GBS_E_UNSUPPORTED, "batch plans run in FP64 or FP32_COMP");
    if (prec != GBS_FP64 && prec != GBS_FP32_COMP) return fail(GBS_E_ARG, "bad precision %d", (int)prec);
    std::vector<int> dv(count);
    for (int i = 0; i < count; ++i) {
        if (dims[i] < 0) return fail(GBS_E_ARG, "negative dimension at item %d", i);
        if (dims[i] > gbs::kMaxTileM)
            return fail(GBS_E_TOO_LARGE, "dimension %d at item %d exceeds %d (batch plans run the register-tile kernels)",
                        dims[i], i, gbs::kMaxTileM);
        dv[i] = dims[i];
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    DevCtx* c = nullptr;
    gbs_status st = current_ctx(&c);
    if (st != GBS_OK) return st;
    std::vector<bool> seen(gbs::kMaxPairs + 1, false);
    for (int N : dv) {
        const int n = (N + 1) / 2;
        if (n >= 1 && !seen[n]) {
            seen[n] = true;
            st = (flags & GBS_PLAN_AUTOTUNE) ? autotune_impl(c, n, nullptr) : maybe_tune(c, n);
            if (st != GBS_OK) return st;
        }
    }
    int64_t round_bytes = (int64_t)4 << 30;  // per coefficient buffer
    if (const char* e = std::getenv("GBS_BATCH_ROUND_MB")) round_bytes = std::max<int64_t>(1, atoll(e)) << 20;
    if (!(flags & GBS_PLAN_AUTOTUNE)) {
        gbs_plan* p = nullptr;
        st = plan_build(c, dv, prec == GBS_FP32_COMP, 256, round_bytes, &p);
        if (st != GBS_OK) return st;
        *plan = p;
        return GBS_OK;
    }
    // autotune the tile size on a synthetic batch of the same shape
    int64_t in_elems = 0;
    for (int N : dv) in_elems += (int64_t)N * N;
    std::vector<gbs_z> hin((size_t)std::max<int64_t>(1, in_elems));
    {
        uint64_t x = 0x2545F4914F6CDD1Dull;
        int64_t o = 0;
        for (int N : dv) {
            for (int i = 0; i < N; ++i)
                for (int j = 0; j <= i; ++j) {
                    x ^= x << 13;
                    x ^= x >> 7;
                    x ^= x << 17;
                    const double re = (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
                    const double im = (double)((x * 0x9E3779B97F4A7C15ull) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
                    hin[o + (int64_t)i * N + j] = hin[o + (int64_t)j * N + i] = gbs_z{0.3 * re, 0.3 * im};
                }
            o += (int64_t)N * N;
        }
    }
    gbs_z* din = nullptr;
    HIP_TRY(dev_malloc((void**)&din, sizeof(gbs_z) * hin.size()));
    if (hipMemcpy(din, hin.data(), sizeof(gbs_z) * hin.size(), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(din);
        return fail(GBS_E_DEVICE, "copy of the tuning batch failed");
    }
    // Candidates in increasing tile size; the replay time is taken to be
    // unimodal in it, so the search stops at the first candidate slower than
    // the best so far.  Only the first candidate gets an untimed warm replay
    // (code objects and caches are warm for the later ones).
    gbs_plan* best = nullptr;
    float best_ms = 1e30f;
    bool warm = false;
    for (int64_t ts : {64, 128, 256, 1024, 4096, 16384, 65536}) {
        gbs_plan* p = nullptr;
        st = plan_build(c, dv, prec == GBS_FP32_COMP, ts, round_bytes, &p);
        if (st != GBS_OK) break;
        float ms = 1e30f;
        if (!warm) {
            st = plan_run(p, din, nullptr, nullptr, p->cs);
            warm = true;
        }
        if (st == GBS_OK && hipEventRecord(p->t0, p->cs) != hipSuccess) st = fail(GBS_E_DEVICE, "event record failed");
        if (st == GBS_OK) st = plan_run(p, din, nullptr, nullptr, p->cs);
        if (st == GBS_OK && hipEventRecord(p->t1, p->cs) != hipSuccess) st = fail(GBS_E_DEVICE, "event failed");
        if (st == GBS_OK && hipEventSynchronize(p->t1) != hipSuccess) st = fail(GBS_E_DEVICE, "sync failed");
        if (st == GBS_OK) hipEventElapsedTime(&ms, p->t0, p->t1);
        if (st != GBS_OK) {
            plan_free(p);
            break;
        }
        if (ms < best_ms) {
            if (best) plan_free(best);
            best = p;
            best_ms = ms;
        } else {
            plan_free(p);
            break;
        }
    }
    hipFree(din);
    if (st != GBS_OK) {
        if (best) plan_free(best);
        return st;
    }
    best->tune_ms = best_ms;
    *plan = best;
    return GBS_OK;
}

gbs_status gbs_batch_plan_info(const gbs_plan* plan, gbs_batch_info* info) {
    if (!plan || !info) return fail(GBS_E_ARG, "null plan or info");
    info->items = plan->S.count;
    info->tiles = (int)plan->S.tiles.size();
    info->rounds = plan->S.rounds;
    info->kernel_nodes = kernel_nodes_of(plan);
    info->subset_terms = plan->S.subset_terms;
    info->tile_subsets = plan->S.tile_subsets;
    info->workspace_bytes = (int64_t)plan->bytes;
    info->yardstick_flops = plan->S.flops;
    info->tune_ms = plan->tune_ms;
    return GBS_OK;
}

gbs_status gbs_batch_run(gbs_plan* plan, const gbs_z* mats_dev, gbs_z* out_dev, double* abs_sum_dev, void* stream) {
    if (!plan || (!mats_dev && plan->S.in_elems > 0) || (!out_dev && plan->S.count > 0))
        return fail(GBS_E_ARG, "bad batch run arguments");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (hipSetDevice(plan->device) != hipSuccess) return fail(GBS_E_DEVICE, "hipSetDevice failed");
    // while per-launch profiling is on, the schedule runs eagerly with every
    // per-subset launch timed (same launches and arguments as the graph)
    return plan_run(plan, mats_dev, out_dev, abs_sum_dev, reinterpret_cast<hipStream_t>(stream), true);
}

void gbs_batch_plan_destroy(gbs_plan* plan) {
    if (!plan) return;
    std::lock_guard<std::mutex> lock(g_mutex);
    hipSetDevice(plan->device);
    hipDeviceSynchronize();
    plan_free(plan);
}

}  // extern "C"
