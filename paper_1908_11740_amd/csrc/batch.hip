// Many independent joins in one replayable launch (hipGraph).
//
// Tiles are independent tasks (Sec. 3.4); so are whole joins.  A batch
// plans every join once -- grid choice (learned picker or rule), buffer
// capacities, a longest-processing-time assignment of the joins to a few
// streams -- and records the partition and join kernels of all joins into
// one hipGraph whose branches (one per stream) run concurrently, so small
// joins fill the GPU together instead of paying one launch sequence and
// one host synchronisation each.  A replay is one graph launch and one
// status readback for the whole batch.  Capacities are bounds, checked on
// the device as in the single-join path; a join that outgrew them (new
// data in the same buffers) is re-run alone with grown buffers and the
// graph is recorded again.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "sj_internal.hpp"
#include "sj_prof.hpp"

namespace sj {
namespace {

constexpr int kLanes = 4;  // concurrent graph branches (HIP's hardware queues per process)

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

void free_work(JoinWork& w) {
    void* bufs[] = {w.uspan, w.units, w.med, w.medt, w.dense, w.dense_unit_prefix, w.dgrp, w.dmj,
                    w.ucnt, w.scan_tmp,
                    w.dbox, w.didf, w.dtmp, w.sc_buf, w.sc_fills, w.sc_ctr, w.sc_total, w.ctr};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    w = JoinWork{};
}

sj_status from_hip_err(hipError_t e) {
    if (e == hipSuccess) return SJ_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SJ_ERR_OOM;
    return SJ_ERR_DEVICE;
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
    sj::JoinWork work[sj::kLanes];
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

sj_status prepare_join(sj_batch* b, int j) {
    Part& R = b->R[j];
    Part& S = b->S[j];
    hipError_t e;
    if ((e = api_part_prepare(R, b->nr[j], b->need_m1R[j], b->need_mR[j])) != hipSuccess ||
        (e = api_part_prepare(S, b->ns[j], b->need_m1S[j], b->need_mS[j])) != hipSuccess)
        return from_hip_err(e);
    JoinParams p = api_join_params(b->grid[j], b->count_only);
    const int64_t C = (int64_t)R.bl.cells() * R.bl.tiles_per_cell();
    sj_status st = api_join_prepare(b->work[b->lane[j]], p, C, R.cap_m, S.cap_m, cap_of(b, j));
    if (st != SJ_OK) return st;
    b->jp[j] = p;
    return SJ_OK;
}

hipError_t enqueue_join(sj_batch* b, int j, hipStream_t s) {
    hipError_t e;
    if ((e = run_partition(b->R[j], b->rin[j], b->nr[j], b->num_cus, s)) != hipSuccess) return e;
    if ((e = run_partition(b->S[j], b->sin[j], b->ns[j], b->num_cus, s)) != hipSuccess) return e;
    JoinWork w = b->work[b->lane[j]];
    w.st = b->dst + 2 * (int64_t)b->n + j;
    return run_join(b->R[j], b->S[j], b->jp[j], w, b->out ? b->out + b->off[j] : nullptr,
                    cap_of(b, j), s);
}

// All joins, one stream per lane, forked from and joined back into s.
hipError_t enqueue_all(sj_batch* b, hipStream_t s) {
    hipError_t e;
    if ((e = hipEventRecord(b->fork, s)) != hipSuccess) return e;
    for (int l = 0; l < kLanes; ++l) {
        if ((e = hipStreamWaitEvent(b->ls[l], b->fork, 0)) != hipSuccess) return e;
        for (int j : b->lane_jobs[l])
            if ((e = enqueue_join(b, j, b->ls[l])) != hipSuccess) return e;
        if ((e = hipEventRecord(b->done[l], b->ls[l])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, b->done[l], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t read_all(sj_batch* b, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(b->hst, b->dst, sizeof(DevStatus) * 3 * (size_t)b->n,
                                  hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// After a run: grow what overflowed.  Returns SJ_OK when every join fitted,
// SJ_ERR_CAPACITY (internal) when some were regrown and must run again.
sj_status check(sj_batch* b, std::vector<int>& redo) {
    redo.clear();
    const int n = b->n;
    for (int j = 0; j < n; ++j) {
        const DevStatus& r = b->hst[j];
        const DevStatus& s = b->hst[n + j];
        const DevStatus& q = b->hst[2 * n + j];
        const uint32_t f = r.flags | s.flags | q.flags;
        if (f & kStatBadRect) return SJ_ERR_RECT;
        if (f & kStatTooLarge) return SJ_ERR_TOO_LARGE;
        if (f & kStatInternal) return SJ_ERR_DEVICE;
        bool again = false;
        if (r.flags & kStatCapacity) {
            b->need_m1R[j] = std::max<int64_t>(b->need_m1R[j], (int64_t)r.m1_total + 1);
            if (r.m_total) b->need_mR[j] = std::max<int64_t>(b->need_mR[j], (int64_t)r.m_total + 1);
            again = true;
        }
        if (s.flags & kStatCapacity) {
            b->need_m1S[j] = std::max<int64_t>(b->need_m1S[j], (int64_t)s.m1_total + 1);
            if (s.m_total) b->need_mS[j] = std::max<int64_t>(b->need_mS[j], (int64_t)s.m_total + 1);
            again = true;
        }
        if (!again && (q.flags & kStatCapacity)) again = true;  // join bounds: exact m next time
        if (!again && (q.flags & kStatScratch) && (int64_t)q.n_pairs <= cap_of(b, j)) {
            b->grid[j].flags |= SJ_TWO_PASS;
            again = true;
        }
        if (again) redo.push_back(j);
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

// Eager runs of the given joins (on their lanes) until every one fits.
// Re-preparing a join may free and reallocate its partition buffers and its
// lane's work lists, and may switch it to two passes, so a recorded graph
// holds stale kernel arguments after any job is prepared again: it is
// dropped here, and the next replay records a new one.
sj_status settle(sj_batch* b, std::vector<int> jobs, hipStream_t s) {
    if (!jobs.empty()) drop_graph(b);
    for (int attempt = 0; attempt < 4 && !jobs.empty(); ++attempt) {
        for (int j : jobs) {
            sj_status st = prepare_join(b, j);
            if (st != SJ_OK) return st;
        }
        hipError_t e = hipEventRecord(b->fork, s);
        for (int j : jobs) {
            if (e == hipSuccess) e = hipStreamWaitEvent(b->ls[b->lane[j]], b->fork, 0);
            if (e == hipSuccess) e = enqueue_join(b, j, b->ls[b->lane[j]]);
        }
        for (int l = 0; l < kLanes && e == hipSuccess; ++l) {
            e = hipEventRecord(b->done[l], b->ls[l]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, b->done[l], 0);
        }
        if (e == hipSuccess) e = read_all(b, s);
        if (e != hipSuccess) return from_hip_err(e);
        sj_status st = check(b, jobs);
        if (st != SJ_OK) return st;
    }
    if (!jobs.empty()) {
        api_set_error("batch: buffers still too small after regrowth");
        return SJ_ERR_DEVICE;
    }
    return SJ_OK;
}

void destroy(sj_batch* b) {
    if (!b) return;
    drop_graph(b);
    for (auto& P : b->R) free_part(P);
    for (auto& P : b->S) free_part(P);
    for (auto& w : b->work) free_work(w);
    for (int l = 0; l < kLanes; ++l) {
        if (b->ls[l]) (void)hipStreamDestroy(b->ls[l]);
        if (b->done[l]) (void)hipEventDestroy(b->done[l]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->dst) (void)hipFree(b->dst);
    if (b->hst) (void)hipHostFree(b->hst);
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
        JoinWork& w = b->work[l];
        w.device = b->device;
        w.num_cus = b->num_cus;
        int64_t cap = 0;
        if (grow_buf(w.ctr, cap, 16, true) != hipSuccess) return fail(SJ_ERR_OOM);
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
            sj_status st = sj_choose_grid(R[j], nR[j], S[j], nS[j], &g, nullptr, stream);
            if (st != SJ_OK) return fail(st);
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
            P->bl = blocking_for(gd.kx, gd.ky);
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
    sj_status st = settle(b, order, s);
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
    std::vector<int> redo;
    sj_status st = check(b, redo);
    if (st != SJ_OK) return st;
    if (!redo.empty()) {
        st = settle(b, redo, s);
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
