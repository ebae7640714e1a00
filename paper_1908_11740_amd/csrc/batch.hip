// Many independent joins in one replayable launch (hipGraph).
//
// Tiles are independent tasks (Sec. 3.4); so are whole joins.  A batch
// plans every join once -- grid choice (learned picker or rule), buffer
// capacities, the workgroups of every partition in the batched launches --
// and records one hipGraph per batch:
//   * the partitioning sequence once for all 2n inputs: every launch runs
//     the workgroups of all partitions (each finds its partition in a prefix
//     of the per-partition workgroup counts), then one classification
//     launch over all joins, which appends every join's work records (span
//     units of small tiles, medium tiles, dense tiles), tagged with the
//     join's index, to one set of work lists shared by the whole batch
//     (inputs too large for the batched scans run per join instead, on a
//     few streams, longest first);
//   * then, once, the join launches over the shared lists: persistent
//     workgroups take the work units of all joins (round-robin over stripes
//     of consecutive records, which mostly belong to one join); the waves
//     stage pairs into scratch chunks that each hold the pairs of one join,
//     and a compaction moves every chunk to its join's output region at a
//     position reserved on the join's fill counter (count-only batches add
//     per-wave counts to the fill counters instead).
// A replay is one graph launch and one status readback for the whole
// batch.  Capacities are bounds checked on the device, as in the single-join
// path; when a join outgrows them (new data in the same buffers) its buffers
// grow, the shared lists are resized, the batch runs again eagerly and the
// graph is recorded again; so does the pair scratch, from the chunk counters
// of the run that outgrew it.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "plan.hpp"
#include "sj_internal.hpp"
#include "sj_prof.hpp"

namespace sj {
int64_t classify_chunk_tiles();
int lds_medium_entries();
int batch_medium_entries();
int scratch_totals();
int scratch_regions();
int scratch_chunk_pairs();
int lds_unit_tiles(int block);

namespace {

constexpr int kLanes = 4;  // concurrent graph branches (HIP's hardware queues per process)
// Grids chosen for a batch: at most this many tiles per input rectangle
// (K^2 <= (nR + nS) / 4).  Of the caps 8, 4, 2, 1, 1/2, 1/4, 1/8, 1/16, 1/32
// timed on a batch of 256 joins drawn like the 256-join benchmark batch but
// from other seeds, 1/4 replayed fastest.
constexpr double kBatchTilesPerRect = 0.25;

template <class T>
hipError_t grow_buf(T*& p, int64_t& cap, int64_t need, bool zero = false) {
    if (need <= cap && p) return hipSuccess;
    const int64_t nc = std::max<int64_t>({need, cap + cap / 4, 1});
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc((void**)&p, (size_t)nc * sizeof(T));
    if (e != hipSuccess) return e;
    if (zero && (e = hipMemset(p, 0, (size_t)nc * sizeof(T))) != hipSuccess) return e;
    cap = nc;
    return hipSuccess;
}

void free_part(Part& P) {  // st belongs to the batch's status array
    void* bufs[] = {P.h1, P.e1, P.e1i, P.cp, P.chunk_cell, P.h2, P.entb, P.enti, P.off,
                    P.scan_tmp};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    P = Part{};
}

void free_work(BatchWork& bw) {
    JoinWork& w = bw.w;
    void* bufs[] = {w.uspan, w.units, w.med, w.medt, w.dense, w.dense_unit_prefix, w.dgrp, w.dmj,
                    w.dbox, w.didf, w.dtmp, w.ctr, w.st, w.sc_total, w.sc_buf, w.sc_fills,
                    w.sc_ctr, bw.ujob, bw.mjob, bw.djob, bw.jobs, bw.fill, bw.sc_job};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    bw = BatchWork{};
}

sj_status from_hip_err(hipError_t e) {
    if (e == hipSuccess) return SJ_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SJ_ERR_OOM;
    return SJ_ERR_DEVICE;
}

// The schedule of one join in a batch: the small-tile workgroup shape is the
// batch's (one launch serves all joins), the caps its defaults, the split
// threshold and the flags the join's grid's; the plain schedule does not
// apply (every join is batched).
JoinParams batch_join_params(const sj_grid& g, bool count_only) {
    sj_grid q = g;
    q.flags &= ~(uint32_t)(SJ_PLAIN | SJ_TWO_PASS);
    JoinParams p = api_join_params(q, count_only);
    p.block = batch_block();
    const int E = 4 * p.block;
    p.small_cap = E / 4;
    p.unit_cap = E - p.small_cap;
    p.unit_tiles = lds_unit_tiles(p.block);
    p.med_cap = batch_medium_entries();
    return p;
}

}  // namespace
}  // namespace sj

struct sj_batch {
    int device = 0;
    int n = 0;
    int num_cus = 0;
    bool count_only = false;
    std::vector<sj::Part> R, S;
    std::vector<const float4*> rin, sin;
    std::vector<int64_t> nr, ns, off, need_m1R, need_mR, need_m1S, need_mS;
    std::vector<sj_grid> grid;
    std::vector<sj::JoinParams> jp;
    std::vector<int> lane;
    std::vector<std::vector<int>> lane_jobs;
    sj_pair* out = nullptr;
    sj::DevStatus* dst = nullptr;  // [3n]: R partitions, S partitions, joins
    sj::DevStatus* hst = nullptr;  // pinned mirror
    sj::BatchWork bw;              // the shared work lists and the job descriptors
    sj::PartBatch pb;              // all partitions as one set of launches
    uint32_t* cls_pre = nullptr;   // device [n + 1]: classification workgroups per join, prefix
    uint32_t cls_blocks = 0;
    bool fused = false;            // partitions and classification batched (else per join on lanes)
    int64_t units_bound = 0, med_bound = 0;
    int64_t need_sc_nch = 0;  // scratch chunks per region a run needed (0: none yet)
    bool any_axis = false;
    hipStream_t ls[sj::kLanes] = {};
    hipEvent_t fork = nullptr, done[sj::kLanes] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace sj {
namespace {

int64_t cap_of(const sj_batch* b, int j) {
    return b->out ? b->off[j + 1] - b->off[j] : 0;
}

// Size every join's partition buffers from its current needs, the shared
// work lists from the sum of the joins' bounds, and write the job
// descriptors.  Buffers may move: a recorded graph is stale afterwards.
sj_status prepare_all(sj_batch* b) {
    hipError_t e;
    BatchWork& bw = b->bw;
    JoinWork& w = bw.w;
    int64_t units = 1, med = 1, dense = 2, dent = 1, dunits = 1;
    bool any_gbda = false;
    b->any_axis = false;
    std::vector<Job> jobs((size_t)std::max(b->n, 1));
    for (int j = 0; j < b->n; ++j) {
        Part& R = b->R[j];
        Part& S = b->S[j];
        if ((e = api_part_prepare(R, b->nr[j], b->need_m1R[j], b->need_mR[j])) != hipSuccess ||
            (e = api_part_prepare(S, b->ns[j], b->need_m1S[j], b->need_mS[j])) != hipSuccess)
            return from_hip_err(e);
        JoinParams p = batch_join_params(b->grid[j], b->count_only);
        p.C = (int64_t)R.bl.cells() * R.bl.tiles_per_cell();
        const int64_t m = R.cap_m + S.cap_m, active = std::min<int64_t>(p.C, std::min(R.cap_m, S.cap_m)) + 1;
        p.units_bound = std::min<int64_t>(
            active, plan::span_units_bound(p.C, m, plan::SpanRules{p.small_cap, p.unit_cap,
                                                                  p.unit_tiles,
                                                                  classify_chunk_tiles()}));
        p.med_bound = std::min<int64_t>(active, m / (p.small_cap + 1) + 1);
        const int64_t nd = m / (p.med_cap + 1) + 2;
        units += p.units_bound;
        med += p.med_bound;
        dense += nd;
        dent += m;
        dunits += (p.gbda ? 4 : 1) * m / std::max(1, p.split_tau) + (p.gbda ? 9 : 1) * nd + 1;
        any_gbda = any_gbda || p.gbda;
        b->any_axis = b->any_axis || p.axis_model;
        b->jp[j] = p;
        Job& J = jobs[(size_t)j];
        J = Job{};
        J.offR = R.off;
        J.offS = S.off;
        J.entR = R.entb;
        J.entS = S.entb;
        J.idR = R.enti;
        J.idS = S.enti;
        J.out = b->out ? (unsigned long long*)(b->out + b->off[j]) : nullptr;
        J.capacity = cap_of(b, j);
        J.st = b->dst + 2 * (int64_t)b->n + j;
        J.stR = R.st;
        J.stS = S.st;
        J.e2 = 0.0;
        J.split_tau = p.split_tau;
        J.flags = (p.axis_model ? kJobAxis : 0u) | (p.gbda ? kJobGbda : 0u);
        J.gd = R.gd;
        J.bl = R.bl;
        J.C = p.C;
    }
    b->units_bound = units;
    b->med_bound = med;
    int64_t c1 = 0, c2 = 0, c3 = 0;
    if ((e = grow_buf(w.units, w.cap_units, units)) != hipSuccess ||
        (e = grow_buf(w.uspan, w.cap_uspan, w.cap_units)) != hipSuccess ||
        (e = grow_buf(bw.ujob, bw.cap_ujob, w.cap_units)) != hipSuccess ||
        (e = grow_buf(w.med, w.cap_med, med)) != hipSuccess ||
        (e = grow_buf(w.medt, w.cap_medt, w.cap_med)) != hipSuccess ||
        (e = grow_buf(bw.mjob, bw.cap_mjob, w.cap_med)) != hipSuccess ||
        (e = grow_buf(w.dense, w.cap_dense, dense)) != hipSuccess ||
        (e = grow_buf(bw.djob, bw.cap_djob, w.cap_dense)) != hipSuccess ||
        (e = grow_buf(w.dense_unit_prefix, w.cap_prefix, w.cap_dense + 1)) != hipSuccess)
        return from_hip_err(e);
    w.cap_dunits = std::max(w.cap_dunits, dunits);
    if (any_gbda && ((e = grow_buf(w.dgrp, w.cap_dgrp, 10 * w.cap_dense)) != hipSuccess ||
                     (e = grow_buf(w.dmj, w.cap_dmj, 10 * w.cap_dense)) != hipSuccess))
        return from_hip_err(e);
    if (dent > w.cap_dent || !w.dbox) {
        if (w.dbox) (void)hipFree(w.dbox);
        if (w.didf) (void)hipFree(w.didf);
        if (w.dtmp) (void)hipFree(w.dtmp);
        w.dbox = nullptr;
        w.didf = nullptr;
        w.dtmp = nullptr;
        w.cap_dent = 0;
        if ((e = grow_buf(w.dbox, c1, dent)) != hipSuccess ||
            (e = grow_buf(w.didf, c2, c1)) != hipSuccess ||
            (e = grow_buf(w.dtmp, c3, 2 * c1)) != hipSuccess)
            return from_hip_err(e);
        w.cap_dent = c1;
    }
    if (!b->count_only) {
        int64_t pairs = 0;
        for (int j = 0; j < b->n; ++j) pairs += cap_of(b, j);
        const int64_t regions = scratch_regions(), cp = scratch_chunk_pairs();
        const int64_t nch = std::max(b->need_sc_nch,
                                     batch_scratch_chunks(pairs, units, med, b->num_cus));
        int64_t cap_ctr = w.sc_ctr ? regions : 0;
        if ((e = grow_buf(w.sc_buf, w.cap_sc_pairs, regions * nch * cp)) != hipSuccess ||
            (e = grow_buf(w.sc_fills, w.cap_sc_fills, regions * nch)) != hipSuccess ||
            (e = grow_buf(bw.sc_job, bw.cap_sc_job, regions * nch)) != hipSuccess ||
            (e = grow_buf(w.sc_ctr, cap_ctr, regions)) != hipSuccess)
            return from_hip_err(e);
        w.sc_nch = nch;
    }
    if ((e = grow_buf(bw.jobs, bw.cap_jobs, (int64_t)jobs.size())) != hipSuccess ||
        (e = grow_buf(bw.fill, bw.cap_fill, (int64_t)jobs.size())) != hipSuccess)
        return from_hip_err(e);
    for (int j = 0; j < b->n; ++j) jobs[(size_t)j].fill = bw.fill + j;
    if (b->n > 0 &&
        (e = hipMemcpy(bw.jobs, jobs.data(), sizeof(Job) * (size_t)b->n, hipMemcpyHostToDevice)) !=
            hipSuccess)
        return from_hip_err(e);
    // all partitions and classifications as single launches when every
    // partition's scans take the direct form (else each join on its lane)
    b->fused = b->n > 0;
    for (int j = 0; j < b->n && b->fused; ++j)
        b->fused = part_batchable(b->R[j], b->nr[j]) && part_batchable(b->S[j], b->ns[j]);
    if (b->fused) {
        std::vector<Part*> parts;
        std::vector<const float4*> rects;
        std::vector<int64_t> ns;
        for (int j = 0; j < b->n; ++j) {
            parts.push_back(&b->R[j]);
            rects.push_back(b->rin[j]);
            ns.push_back(b->nr[j]);
            parts.push_back(&b->S[j]);
            rects.push_back(b->sin[j]);
            ns.push_back(b->ns[j]);
        }
        if ((e = part_batch_plan(b->pb, parts.data(), rects.data(), ns.data(), (int)parts.size(),
                                 b->num_cus)) != hipSuccess)
            return from_hip_err(e);
        std::vector<uint32_t> pre((size_t)b->n + 1, 0u);
        int64_t acc = 0;
        for (int j = 0; j < b->n; ++j) {
            pre[(size_t)j] = (uint32_t)acc;
            acc += classify_blocks(b->jp[j].C);
        }
        if (acc >= ((int64_t)1 << 31)) return SJ_ERR_TOO_LARGE;
        pre[(size_t)b->n] = (uint32_t)acc;
        b->cls_blocks = (uint32_t)acc;
        if (b->cls_pre) (void)hipFree(b->cls_pre);
        b->cls_pre = nullptr;
        if ((e = hipMalloc((void**)&b->cls_pre, sizeof(uint32_t) * pre.size())) != hipSuccess ||
            (e = hipMemcpy(b->cls_pre, pre.data(), sizeof(uint32_t) * pre.size(),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return from_hip_err(e);
    }
    return SJ_OK;
}

// The whole batch on stream s: clear the shared counters, then per lane each
// join's partitions and classification, then the shared join launches.
hipError_t enqueue_all(sj_batch* b, hipStream_t s) {
    hipError_t e;
    if ((e = batch_reset(b->bw, b->n, s)) != hipSuccess) return e;
    if (b->fused) {
        if ((e = run_partition_batch(b->pb, s)) != hipSuccess ||
            (e = batch_classify_all(b->bw, b->jp[0], b->cls_pre, b->n, b->cls_blocks, s)) !=
                hipSuccess)
            return e;
        return batch_join(b->bw, b->n, b->any_axis, !b->count_only, b->units_bound, b->med_bound,
                          s);
    }
    if ((e = hipEventRecord(b->fork, s)) != hipSuccess) return e;
    for (int l = 0; l < kLanes; ++l) {
        if ((e = hipStreamWaitEvent(b->ls[l], b->fork, 0)) != hipSuccess) return e;
        for (int j : b->lane_jobs[l]) {
            if ((e = run_partition(b->R[j], b->rin[j], b->nr[j], b->num_cus, b->ls[l])) != hipSuccess ||
                (e = run_partition(b->S[j], b->sin[j], b->ns[j], b->num_cus, b->ls[l])) != hipSuccess ||
                (e = batch_classify(b->bw, b->R[j], b->S[j], b->jp[j], (uint32_t)j, b->ls[l])) !=
                    hipSuccess)
                return e;
        }
        if ((e = hipEventRecord(b->done[l], b->ls[l])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, b->done[l], 0)) != hipSuccess) return e;
    }
    return batch_join(b->bw, b->n, b->any_axis, !b->count_only, b->units_bound, b->med_bound, s);
}

hipError_t read_all(sj_batch* b, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(b->hst, b->dst, sizeof(DevStatus) * 3 * (size_t)b->n,
                                  hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// After a run: raise the needs of what overflowed.  *again: something must
// grow and the batch run again.
sj_status check(sj_batch* b, bool* again) {
    *again = false;
    bool scratch = false;
    const int n = b->n;
    for (int j = 0; j < n; ++j) {
        const DevStatus& r = b->hst[j];
        const DevStatus& s = b->hst[n + j];
        const DevStatus& q = b->hst[2 * n + j];
        const uint32_t f = r.flags | s.flags | q.flags;
        if (f & kStatBadRect) return SJ_ERR_RECT;
        if (f & kStatTooLarge) return SJ_ERR_TOO_LARGE;
        if (f & kStatInternal) {
            api_set_error("batch: internal status flag");
            return SJ_ERR_DEVICE;
        }
        if (r.flags & kStatCapacity) {
            b->need_m1R[j] = std::max<int64_t>(b->need_m1R[j], (int64_t)r.m1_total + 1);
            if (r.m_total) b->need_mR[j] = std::max<int64_t>(b->need_mR[j], (int64_t)r.m_total + 1);
            *again = true;
        }
        if (s.flags & kStatCapacity) {
            b->need_m1S[j] = std::max<int64_t>(b->need_m1S[j], (int64_t)s.m1_total + 1);
            if (s.m_total) b->need_mS[j] = std::max<int64_t>(b->need_mS[j], (int64_t)s.m_total + 1);
            *again = true;
        }
        // the shared lists are sized from bounds of the partitions' capacities,
        // so they overflow only after a partition did (re-sized above)
        if (q.flags & kStatCapacity) *again = true;
        scratch = scratch || (q.flags & kStatScratch);
    }
    if (scratch) {
        // the waves that found the scratch full stopped reserving, so the
        // counters undercount: at least double
        int64_t used = 0;
        if (batch_scratch_used(b->bw, &used) != hipSuccess) return SJ_ERR_DEVICE;
        b->need_sc_nch = std::max(2 * b->bw.w.sc_nch, used + used / 4 + 2);
        *again = true;
    }
    return SJ_OK;
}

void drop_graph(sj_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

hipError_t capture(sj_batch* b) {
    drop_graph(b);
    const bool was = prof_pause(true);
    hipError_t e = hipStreamBeginCapture(b->ls[0], hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e2 = enqueue_all(b, b->ls[0]);
        e = hipStreamEndCapture(b->ls[0], &b->graph);
        if (e2 != hipSuccess) e = e2;
    }
    prof_pause(was);
    if (e != hipSuccess) {
        drop_graph(b);
        return e;
    }
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) drop_graph(b);
    return e;
}

// Size everything and run the batch eagerly until every join fits.  Sizing
// may free and reallocate buffers, so a recorded graph holds stale kernel
// arguments afterwards: it is dropped, and the next replay records a new one.
sj_status settle(sj_batch* b, hipStream_t s) {
    drop_graph(b);
    if (b->n == 0) return prepare_all(b);
    for (int attempt = 0; attempt < 4; ++attempt) {
        sj_status st = prepare_all(b);
        if (st != SJ_OK) return st;
        hipError_t e = enqueue_all(b, s);
        if (e == hipSuccess) e = read_all(b, s);
        if (e != hipSuccess) return from_hip_err(e);
        bool again = false;
        st = check(b, &again);
        if (st != SJ_OK) return st;
        if (!again) return SJ_OK;
    }
    api_set_error("batch: buffers still too small after regrowth");
    return SJ_ERR_DEVICE;
}

void destroy(sj_batch* b) {
    if (!b) return;
    drop_graph(b);
    for (auto& P : b->R) free_part(P);
    for (auto& P : b->S) free_part(P);
    free_work(b->bw);
    for (int l = 0; l < kLanes; ++l) {
        if (b->ls[l]) (void)hipStreamDestroy(b->ls[l]);
        if (b->done[l]) (void)hipEventDestroy(b->done[l]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->dst) (void)hipFree(b->dst);
    if (b->hst) (void)hipHostFree(b->hst);
    if (b->cls_pre) (void)hipFree(b->cls_pre);
    part_batch_free(b->pb);
    delete b;
}

}  // namespace
}  // namespace sj

using namespace sj;

extern "C" {

sj_status sj_batch_create(int32_t n_joins, const float* const* R, const int64_t* nR,
                          const float* const* S, const int64_t* nS, const sj_grid* grids,
                          sj_pair* out, const int64_t* out_offsets, sj_batch** batch,
                          void* stream) {
    if (!batch || n_joins < 0 || (n_joins > 0 && (!R || !nR || !S || !nS))) return SJ_ERR_ARG;
    if (out && !out_offsets) return SJ_ERR_ARG;
    for (int j = 0; j < n_joins; ++j) {
        if (nR[j] < 0 || nS[j] < 0 || (nR[j] > 0 && !R[j]) || (nS[j] > 0 && !S[j])) return SJ_ERR_ARG;
        if (((uintptr_t)R[j] & 15u) || ((uintptr_t)S[j] & 15u)) return SJ_ERR_ARG;
        if (nR[j] >= ((int64_t)1 << 30) || nS[j] >= ((int64_t)1 << 30)) return SJ_ERR_TOO_LARGE;
        if (out && out_offsets[j + 1] < out_offsets[j]) return SJ_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    sj_batch* b = new (std::nothrow) sj_batch();
    if (!b) return SJ_ERR_OOM;
    auto fail = [&](sj_status st) {
        destroy(b);
        return st;
    };
    if (hipGetDevice(&b->device) != hipSuccess) return fail(SJ_ERR_DEVICE);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) return fail(SJ_ERR_DEVICE);
    b->num_cus = prop.multiProcessorCount;
    const int n = n_joins;
    b->n = n;
    b->out = out;
    b->count_only = (out == nullptr);
    b->R.resize(n);
    b->S.resize(n);
    b->grid.resize(n);
    b->jp.resize(n);
    b->lane.resize(n);
    b->lane_jobs.resize(kLanes);
    b->rin.assign(n, nullptr);
    b->sin.assign(n, nullptr);
    b->nr.assign(nR, nR + n);
    b->ns.assign(nS, nS + n);
    b->off.assign(n + 1, 0);
    if (out)
        for (int j = 0; j <= n; ++j) b->off[j] = out_offsets[j];
    if (n > 0) {
        if (hipMalloc((void**)&b->dst, sizeof(DevStatus) * 3 * (size_t)n) != hipSuccess ||
            hipMemset(b->dst, 0, sizeof(DevStatus) * 3 * (size_t)n) != hipSuccess)
            return fail(SJ_ERR_OOM);
        if (hipHostMalloc((void**)&b->hst, sizeof(DevStatus) * 3 * (size_t)n,
                          hipHostMallocDefault) != hipSuccess) {
            b->hst = nullptr;
            return fail(SJ_ERR_OOM);
        }
    }
    for (int l = 0; l < kLanes; ++l) {
        if (hipStreamCreateWithFlags(&b->ls[l], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->done[l], hipEventDisableTiming) != hipSuccess)
            return fail(SJ_ERR_DEVICE);
    }
    {
        JoinWork& w = b->bw.w;
        w.device = b->device;
        w.num_cus = b->num_cus;
        int64_t cap = 0;
        if (grow_buf(w.ctr, cap, 16, true) != hipSuccess) return fail(SJ_ERR_OOM);
        cap = 0;
        if (grow_buf(w.st, cap, 1, true) != hipSuccess) return fail(SJ_ERR_OOM);
        cap = 0;
        if (grow_buf(w.sc_total, cap, (int64_t)scratch_totals(), true) != hipSuccess)
            return fail(SJ_ERR_OOM);
    }
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
        return fail(SJ_ERR_DEVICE);
    // 1. grids: the caller's, else the picker's / the rule's
    std::vector<int64_t> work(n);
    for (int j = 0; j < n; ++j) {
        sj_grid g{};
        if (grids) g = grids[j];
        b->rin[j] = (const float4*)R[j];
        b->sin[j] = (const float4*)S[j];
        if (g.k == 0 || g.split_tau == 0) {
            const bool chosen_k = g.k == 0;
            sj_status st = sj_choose_grid(R[j], nR[j], S[j], nS[j], &g, nullptr, stream);
            if (st != SJ_OK) return fail(st);
            // inside one replay a join's per-tile passes are not hidden behind
            // call overhead: a chosen 2-D grid keeps K^2 <= (nR + nS) / 4
            if (chosen_k && !(g.flags & SJ_STRIPES)) {
                const double c = std::floor(std::sqrt(kBatchTilesPerRect * (double)(nR[j] + nS[j])));
                g.k = std::max(1, std::min(g.k, (int32_t)c));
            }
        }
        GridDev gd;
        sj_grid rg;
        sj_status st = api_resolve_grid(&g, rg, gd);
        if (st != SJ_OK) return fail(st);
        b->grid[j] = rg;
        for (Part* P : {&b->R[j], &b->S[j]}) {
            P->device = b->device;
            P->grid = rg;
            P->gd = gd;
            // coarse cells sized for the join's larger input, so that the
            // small joins of a batch fill their level-2 chunks
            P->bl = blocking_for(gd.kx, gd.ky, std::max(nR[j], nS[j]));
        }
        b->R[j].n = nR[j];
        b->S[j].n = nS[j];
        b->R[j].st = b->dst + j;
        b->S[j].st = b->dst + n + j;
        work[j] = nR[j] + nS[j];
    }
    b->need_m1R.resize(n);
    b->need_mR.resize(n);
    b->need_m1S.resize(n);
    b->need_mS.resize(n);
    for (int j = 0; j < n; ++j) {
        b->need_m1R[j] = nR[j] + nR[j] / 4 + 4096;
        b->need_mR[j] = 2 * nR[j] + 4096;
        b->need_m1S[j] = nS[j] + nS[j] / 4 + 4096;
        b->need_mS[j] = 2 * nS[j] + 4096;
    }
    // 2. longest processing time first onto the least-loaded lane
    std::vector<int> order(n);
    for (int j = 0; j < n; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work[a] > work[c]; });
    int64_t load[kLanes] = {0, 0, 0, 0};
    for (int j : order) {
        const int l = (int)(std::min_element(load, load + kLanes) - load);
        b->lane[j] = l;
        b->lane_jobs[l].push_back(j);
        load[l] += work[j];
    }
    // 3. size everything, run once eagerly (capacities checked), record the graph
    sj_status st = settle(b, s);
    if (st != SJ_OK) return fail(st);
    if (capture(b) != hipSuccess) {
        api_set_error("batch: graph capture failed");
        return fail(SJ_ERR_DEVICE);
    }
    *batch = b;
    return SJ_OK;
}

sj_status sj_batch_run(sj_batch* b, int64_t* n_pairs, void* stream) {
    if (!b) return SJ_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (b->n == 0) return SJ_OK;
    if (!b->exec && capture(b) != hipSuccess) return SJ_ERR_DEVICE;
    if (hipGraphLaunch(b->exec, s) != hipSuccess || read_all(b, s) != hipSuccess)
        return SJ_ERR_DEVICE;
    bool again = false;
    sj_status st = check(b, &again);
    if (st != SJ_OK) return st;
    if (again) {
        st = settle(b, s);
        if (st != SJ_OK) return st;
    }
    bool over = false;
    for (int j = 0; j < b->n; ++j) {
        const int64_t np = (int64_t)b->hst[2 * b->n + j].n_pairs;
        if (n_pairs) n_pairs[j] = np;
        if (!b->count_only && np > cap_of(b, j)) over = true;
    }
    return over ? SJ_ERR_CAPACITY : SJ_OK;
}

sj_status sj_batch_run_eager(sj_batch* b, int64_t* n_pairs, void* stream) {
    if (!b) return SJ_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (b->n == 0) return SJ_OK;
    if (enqueue_all(b, s) != hipSuccess || read_all(b, s) != hipSuccess) return SJ_ERR_DEVICE;
    bool again = false;
    sj_status st = check(b, &again);
    if (st != SJ_OK) return st;
    if (again) {
        st = settle(b, s);
        if (st != SJ_OK) return st;
    }
    bool over = false;
    for (int j = 0; j < b->n; ++j) {
        const int64_t np = (int64_t)b->hst[2 * b->n + j].n_pairs;
        if (n_pairs) n_pairs[j] = np;
        if (!b->count_only && np > cap_of(b, j)) over = true;
    }
    return over ? SJ_ERR_CAPACITY : SJ_OK;
}

sj_status sj_batch_stats(const sj_batch* b, sj_join_stats* o) {
    if (!b || !o) return SJ_ERR_ARG;
    std::memset(o, 0, sizeof(*o));
    if (hipDeviceSynchronize() != hipSuccess) return SJ_ERR_DEVICE;
    if (join_stats(b->bw.w, true, o) != hipSuccess) return SJ_ERR_DEVICE;
    for (int j = 0; j < b->n; ++j) o->n_pairs += (int64_t)b->hst[2 * b->n + j].n_pairs;
    const int E = 4 * batch_block();  // entries of a span unit
    o->single_pass = 1;
    o->small_cap = E / 4;
    o->med_cap = batch_medium_entries();
    return SJ_OK;
}

sj_status sj_batch_entries(const sj_batch* b, int64_t* m1, int64_t* m) {
    if (!b) return SJ_ERR_ARG;
    for (int i = 0; i < 2 * b->n; ++i) {
        if (m1) m1[i] = (int64_t)b->hst[i].m1_total;
        if (m) m[i] = (int64_t)b->hst[i].m_total;
    }
    return SJ_OK;
}

sj_status sj_batch_info(const sj_batch* b, int32_t* k, int32_t* split_tau) {
    if (!b) return SJ_ERR_ARG;
    for (int j = 0; j < b->n; ++j) {
        if (k) k[j] = b->grid[j].k;
        if (split_tau) split_tau[j] = b->grid[j].split_tau;
    }
    return SJ_OK;
}

void sj_batch_free(sj_batch* b) { destroy(b); }

sj_status sj_batch_join(int32_t n_joins, const float* const* R, const int64_t* nR,
                        const float* const* S, const int64_t* nS, const sj_grid* grids,
                        sj_pair* out, const int64_t* out_offsets, int64_t* n_pairs, void* stream) {
    sj_batch* b = nullptr;
    sj_status st = sj_batch_create(n_joins, R, nR, S, nS, grids, out, out_offsets, &b, stream);
    if (st != SJ_OK) return st;
    // the creation run already produced every join's result
    bool over = false;
    for (int j = 0; j < b->n; ++j) {
        const int64_t np = (int64_t)b->hst[2 * b->n + j].n_pairs;
        if (n_pairs) n_pairs[j] = np;
        if (!b->count_only && np > cap_of(b, j)) over = true;
    }
    destroy(b);
    return over ? SJ_ERR_CAPACITY : SJ_OK;
}

}  // extern "C"
