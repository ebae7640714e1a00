// C ABI of libsj (declared in include/sj.h): argument checks, handle and
// workspace management, kernel sequencing and the one status readback per
// call.  No exception crosses the ABI.
#include <algorithm>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "plan.hpp"
#include "sj_internal.hpp"
#include "sj_prof.hpp"

struct sj_part : public sj::Part {};

namespace sj {

int lds_unit_entries(int block);
int lds_unit_tiles(int block);
int lds_medium_entries();
int64_t classify_blocks(int64_t C);
int64_t classify_chunk_tiles();

namespace {

std::mutex g_mu;
thread_local char g_err[256] = "";

void set_err(const char* what, hipError_t e) {
    snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
}

template <class T>
hipError_t grow(T*& p, int64_t& cap, int64_t need, bool zero = false) {
    if (need <= cap && p) return hipSuccess;
    int64_t nc = std::max<int64_t>(need, cap + cap / 4);
    if (nc < 1) nc = 1;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc((void**)&p, (size_t)nc * sizeof(T));
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
    if (zero) {
        e = hipMemset(p, 0, (size_t)nc * sizeof(T));
        if (e != hipSuccess) return e;
    }
    cap = nc;
    return hipSuccess;
}

sj_status from_hip(hipError_t e) {
    if (e == hipSuccess) return SJ_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SJ_ERR_OOM;
    return SJ_ERR_DEVICE;
}

// Resolve the grid of a call: K range, default domain, float32 scales.
sj_status resolve_grid(const sj_grid* g, sj_grid& out, GridDev& gd) {
    if (!g) return SJ_ERR_ARG;
    out = *g;
    if (out.k < 1 || out.k > SJ_K_MAX) return SJ_ERR_ARG;
    if (out.domain[0] == 0.f && out.domain[1] == 0.f && out.domain[2] == 0.f &&
        out.domain[3] == 0.f) {
        out.domain[2] = 1.f;
        out.domain[3] = 1.f;
    }
    const float w = out.domain[2] - out.domain[0], h = out.domain[3] - out.domain[1];
    if (!std::isfinite(w) || !std::isfinite(h) || !(w > 0.f) || !(h > 0.f)) return SJ_ERR_ARG;
    if (out.flags & SJ_STRIPES) {
        // K vertical stripes swept along y: a 1 x K grid on the transposed
        // input (partition axes: x' = y, y' = x)
        gd.transpose = 1;
        gd.x0 = out.domain[1];
        gd.y0 = out.domain[0];
        gd.sx = 1.0f / h;
        gd.sy = (float)out.k / w;
        gd.kx = 1;
        gd.ky = out.k;
    } else {
        gd.transpose = 0;
        gd.x0 = out.domain[0];
        gd.y0 = out.domain[1];
        gd.sx = (float)out.k / w;
        gd.sy = (float)out.k / h;
        gd.kx = out.k;
        gd.ky = out.k;
    }
    if (!std::isfinite(gd.sx) || !std::isfinite(gd.sy)) return SJ_ERR_ARG;
    return SJ_OK;
}

bool same_grid(const sj_grid& a, const sj_grid& b) {
    return a.k == b.k && std::memcmp(a.domain, b.domain, sizeof(a.domain)) == 0 &&
           (a.flags & SJ_STRIPES) == (b.flags & SJ_STRIPES);
}

struct DeviceState {
    JoinWork w;
    PartBatch pb;  // the two partitions of sj_join_rects as one set of launches
    DevStatus* host = nullptr;  // pinned [3]: readbacks; [0] ends as the last join's status
    bool init = false;
};

std::map<int, DeviceState> g_dev;

sj_status device_state(int dev, DeviceState** out) {
    DeviceState& d = g_dev[dev];
    if (!d.init) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return SJ_ERR_DEVICE;
        d.w.device = dev;
        d.w.num_cus = prop.multiProcessorCount;
        if (hipHostMalloc((void**)&d.host, 3 * sizeof(DevStatus), hipHostMallocDefault) != hipSuccess)
            return SJ_ERR_OOM;
        int64_t cap = 0;
        if (grow(d.w.ctr, cap, 16, true) != hipSuccess) return SJ_ERR_OOM;
        DevStatus* st = nullptr;
        cap = 0;
        if (grow(st, cap, 1, true) != hipSuccess) return SJ_ERR_OOM;
        d.w.st = st;
        d.init = true;
    }
    *out = &d;
    return SJ_OK;
}

sj_status current_device(int* dev) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return SJ_ERR_DEVICE;
    if (hipGetDevice(dev) != hipSuccess) return SJ_ERR_DEVICE;
    return SJ_OK;
}

// Architecture name of a device without feature suffixes ("gfx950").
void arch_name(const hipDeviceProp_t& prop, char* out, size_t cap) {
    size_t i = 0;
    for (; i + 1 < cap && prop.gcnArchName[i] && prop.gcnArchName[i] != ':'; ++i)
        out[i] = prop.gcnArchName[i];
    out[i] = '\0';
}

hipError_t read_status(const DevStatus* dst, DevStatus* host, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(host, dst, sizeof(DevStatus), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// Autotuner cache: launch shape of the small-tile kernel, LDS slab caps and
// split threshold per (device, K, log2 entries of R and S, mode).
struct TuneKey {
    int dev, k, lr, ls, count_only;
    bool operator<(const TuneKey& o) const {
        return std::tie(dev, k, lr, ls, count_only) < std::tie(o.dev, o.k, o.lr, o.ls, o.count_only);
    }
};
std::map<TuneKey, sj_tuning> g_tune;

int log2_bucket(int64_t m) {
    int b = 0;
    while (b < 62 && ((int64_t)1 << b) < m) ++b;
    return b;
}

// mode: bit 0 count only, bit 1 distance join; the grid adds bit 2 for
// stripes and bit 3 for GBDA dense tiles (each tuned apart: a 1 x K grid of
// dense stripes shares K and entry counts with a K x K grid)
TuneKey tune_key(int dev, const sj_grid& g, int64_t mR, int64_t mS, int mode) {
    mode |= ((g.flags & SJ_STRIPES) ? 4 : 0) | ((g.flags & SJ_GBDA) ? 8 : 0);
    return TuneKey{dev, g.k, log2_bucket(mR), log2_bucket(mS), mode};
}

// Schedule parameters of a join.
JoinParams join_params(const sj_grid& g, bool count_only) {
    JoinParams p{};
    p.K = g.k;
    p.C = (int64_t)g.k * g.k;
    p.plain = (g.flags & SJ_PLAIN) != 0;
    p.count_only = count_only;
    p.block = 256;  // span units of the small tiles
    const int E = lds_unit_entries(p.block);
    const int E_plain = lds_unit_entries(256);  // LDS entries of the plain per-tile kernel
    p.small_cap = p.plain ? E_plain : E / 4;
    p.unit_cap = p.plain ? E_plain : E - p.small_cap;
    p.unit_tiles = lds_unit_tiles(p.block);
    p.med_cap = p.plain ? E_plain : lds_medium_entries();
    p.split_tau = g.split_tau > 0 ? g.split_tau : 256;
    if (p.plain || g.split_tau == INT32_MAX) p.split_tau = INT32_MAX;
    p.single = !p.plain && !count_only && (g.flags & SJ_TWO_PASS) == 0;
    // the model picks between x and y; stripes sweep along y by construction
    p.axis_model = !p.plain && (g.flags & (SJ_SWEEP_X | SJ_STRIPES)) == 0;
    p.gbda = !p.plain && (g.flags & SJ_GBDA) != 0;
    return p;
}

// Apply a tuning (block shape, caps; split threshold unless the grid fixes one).
void apply_tuning(JoinParams& p, const sj_grid& g, const sj_tuning& t) {
    if (p.plain) return;
    p.block = t.block;
    const int E = lds_unit_entries(p.block);
    p.small_cap = std::min(t.small_cap, E / 2 + E / 4);
    p.unit_cap = E - p.small_cap;
    p.unit_tiles = lds_unit_tiles(p.block);
    p.med_cap = std::max(p.small_cap, std::min(t.med_cap, lds_medium_entries()));
    if (g.split_tau == 0 && t.split_tau > 0) p.split_tau = t.split_tau;
}

JoinParams tuned_params(int dev, const sj_grid& g, int64_t mR, int64_t mS, bool count_only,
                        bool dist = false) {
    JoinParams p = join_params(g, count_only);
    auto it = g_tune.find(tune_key(dev, g, mR, mS, (count_only ? 1 : 0) | (dist ? 2 : 0)));
    if (it != g_tune.end()) apply_tuning(p, g, it->second);
    return p;
}

// Bounds of a join's work lists and growth of the workspace to hold them
// (tile entries mR, mS: exact after a partition, or capacity bounds).
sj_status join_prepare(JoinWork& w, JoinParams& p, int64_t C, int64_t mR, int64_t mS,
                       int64_t capacity) {
    p.C = C;
    const int64_t active = std::min<int64_t>(p.C, std::min(mR, mS)) + 1;
    p.units_bound = std::min<int64_t>(
        active, plan::span_units_bound(p.C, mR + mS,
                                       plan::SpanRules{p.small_cap, p.unit_cap, p.unit_tiles,
                                                       classify_chunk_tiles()}));
    p.med_bound = std::min<int64_t>(active, (mR + mS) / (p.small_cap + 1) + 1);
    const int64_t ndense = (mR + mS) / (p.med_cap + 1) + 2;
    hipError_t e = hipSuccess;
    if (!p.plain) {
        if ((e = grow(w.units, w.cap_units, p.units_bound)) != hipSuccess) return from_hip(e);
        if ((e = grow(w.uspan, w.cap_uspan, w.cap_units)) != hipSuccess) return from_hip(e);
        if ((e = grow(w.med, w.cap_med, p.med_bound)) != hipSuccess) return from_hip(e);
        if ((e = grow(w.medt, w.cap_medt, w.cap_med)) != hipSuccess) return from_hip(e);
        if ((e = grow(w.med_lpt, w.cap_med_lpt, w.cap_med)) != hipSuccess) return from_hip(e);
    }
    if ((e = grow(w.dense, w.cap_dense, ndense)) != hipSuccess) return from_hip(e);
    // dense units: ceil(list / tau) per tile; with GBDA ceil per mini-join,
    // where each class group takes part in at most 4 of the 9
    w.cap_dunits = std::max<int64_t>(
        w.cap_dunits, p.plain ? w.cap_dense
                              : (p.gbda ? 4 : 1) * (mR + mS) / std::max(1, p.split_tau) +
                                    (p.gbda ? 9 : 1) * w.cap_dense + 1);
    if (p.gbda) {
        if ((e = grow(w.dgrp, w.cap_dgrp, 10 * w.cap_dense)) != hipSuccess) return from_hip(e);
        if ((e = grow(w.dmj, w.cap_dmj, 10 * w.cap_dense)) != hipSuccess) return from_hip(e);
    }
    {
        const int64_t slots = join_slots(p, w);
        if ((e = grow(w.ucnt, w.cap_ucnt, slots + 1)) != hipSuccess) return from_hip(e);
        if ((e = grow(w.scan_tmp, w.cap_scan, scan_block_sums_needed(slots))) != hipSuccess)
            return from_hip(e);
    }
    if ((e = grow(w.dense_unit_prefix, w.cap_prefix, w.cap_dense + 1)) != hipSuccess)
        return from_hip(e);
    {
        const int64_t need = std::max<int64_t>(mR + mS, 1);
        if (need > w.cap_dent || !w.dbox) {
            if (w.dbox) (void)hipFree(w.dbox);
            if (w.didf) (void)hipFree(w.didf);
            if (w.dtmp) (void)hipFree(w.dtmp);
            w.dbox = nullptr;
            w.didf = nullptr;
            w.dtmp = nullptr;
            w.cap_dent = 0;
            int64_t c1 = 0, c2 = 0, c3 = 0;
            if ((e = grow(w.dbox, c1, need)) != hipSuccess) return from_hip(e);
            if ((e = grow(w.didf, c2, c1)) != hipSuccess) return from_hip(e);
            if ((e = grow(w.dtmp, c3, 2 * c1)) != hipSuccess) return from_hip(e);
            w.cap_dent = c1;
        }
    }
    if (p.single) {
        // scratch of the single pass: the caller's capacity (at most 2^27
        // pairs) spread over the regions with 25% headroom, plus one partly
        // filled chunk per resident wavefront of the three sweep kernels
        const int64_t regions = scratch_regions(), cp = scratch_chunk_pairs();
        const int64_t want = std::min<int64_t>(capacity, (int64_t)1 << 27);
        const int64_t waves = 3LL * w.num_cus * 32;
        int64_t nch = (want + want / 4) / (regions * cp) + (waves + regions - 1) / regions + 2;
        // test hook: a tiny scratch forces the two-pass retry
        const char* dbg = std::getenv("SJ_DEBUG_SCRATCH_CHUNKS");
        if (dbg) nch = std::max(1, std::atoi(dbg));
        if ((e = grow(w.sc_buf, w.cap_sc_pairs, regions * nch * cp)) != hipSuccess ||
            (e = grow(w.sc_fills, w.cap_sc_fills, regions * nch + 1)) != hipSuccess ||
            (e = grow(w.scan_tmp, w.cap_scan, scan_block_sums_needed(regions * nch))) != hipSuccess)
            return from_hip(e);
        if (!w.sc_ctr) {
            int64_t c1 = 0, c2 = 0;
            if ((e = grow(w.sc_ctr, c1, regions)) != hipSuccess ||
                (e = grow(w.sc_total, c2, scratch_totals())) != hipSuccess)
                return from_hip(e);
        }
        w.sc_nch = dbg ? nch : std::max<int64_t>(w.sc_nch, nch);
    }
    return SJ_OK;
}

// Grow the buffers of a partitioned input for n rectangles with level-1 and
// tile-entry capacities of at least need_m1 and need_m (P.bl set).
hipError_t part_prepare(Part& Pr, int64_t n, int64_t need_m1, int64_t need_m) {
    Part* P = &Pr;
    hipError_t e = hipSuccess;
    const Blocking bl = P->bl;
    const int64_t G1 = bl.cells(), B2 = bl.tiles_per_cell(), Cb = G1 * B2;
    const int64_t ch1 = l1_chunk(n, G1);
    const int64_t nb1 = n > 0 ? (n + ch1 - 1) / ch1 : 1;
    const int64_t need_chunks = need_m1 / kChunk2 + G1 + 2;
    if ((e = grow(P->h1, P->cap_h1, G1 * nb1 + 1)) != hipSuccess ||
        (e = grow(P->cp, P->cap_cp, G1 + 1)) != hipSuccess ||
        (e = grow(P->chunk_cell, P->cap_chunks, need_chunks)) != hipSuccess ||
        (e = grow(P->h2, P->cap_h2, B2 * P->cap_chunks + 1)) != hipSuccess ||
        (e = grow(P->off, P->cap_off, Cb + 1)) != hipSuccess ||
        (e = grow(P->scan_tmp, P->cap_scan,
                  scan_block_sums_needed(std::max(G1 * nb1, B2 * P->cap_chunks)))) !=
            hipSuccess)
        return e;
    if ((e = grow(P->e1, P->cap_m1, need_m1)) != hipSuccess) return e;
    if ((e = grow(P->e1i, P->cap_m1i, P->cap_m1)) != hipSuccess) return e;
    if ((e = grow(P->entb, P->cap_m, need_m)) != hipSuccess) return e;
    if ((e = grow(P->enti, P->cap_mi, P->cap_m)) != hipSuccess) return e;
    return hipSuccess;
}

// Debug mode (environment SJ_CHECK_WORKLISTS=1): after a join, read the
// span units and both partitions' tile offsets back and check them on the
// host (plan::check_units).  Costs a full download per join.
bool check_worklists_enabled() {
    const char* v = std::getenv("SJ_CHECK_WORKLISTS");
    return v && v[0] && v[0] != '0';
}

sj_status check_worklists(const Part& R, const Part& S, const JoinParams& p, const JoinWork& w) {
    sj_join_stats js{};
    if (join_stats(w, false, &js) != hipSuccess) return SJ_ERR_DEVICE;
    const int64_t n = js.small_units, C = (int64_t)R.bl.cells() * R.bl.tiles_per_cell();
    if (n > w.cap_units) {
        snprintf(g_err, sizeof(g_err), "work-list check: %lld span units > capacity %lld",
                 (long long)n, (long long)w.cap_units);
        return SJ_ERR_DEVICE;
    }
    std::vector<uint32_t> offR((size_t)C + 1), offS((size_t)C + 1);
    std::vector<uint4> sp((size_t)n);
    std::vector<uint2> ut((size_t)n);
    if (hipMemcpy(offR.data(), R.off, (C + 1) * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(offS.data(), S.off, (C + 1) * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        (n && hipMemcpy(sp.data(), w.uspan, n * sizeof(uint4), hipMemcpyDeviceToHost) != hipSuccess) ||
        (n && hipMemcpy(ut.data(), w.units, n * sizeof(uint2), hipMemcpyDeviceToHost) != hipSuccess))
        return SJ_ERR_DEVICE;
    if (offR[C] != (uint32_t)R.m || offS[C] != (uint32_t)S.m || R.m > R.cap_m || S.m > S.cap_m) {
        snprintf(g_err, sizeof(g_err), "work-list check: tile offsets end past the entries");
        return SJ_ERR_DEVICE;
    }
    std::vector<plan::Unit> u((size_t)n);
    for (int64_t i = 0; i < n; ++i)
        u[(size_t)i] = plan::Unit{sp[i].x, sp[i].y, sp[i].z, sp[i].w, ut[i].x, ut[i].y};
    const plan::SpanRules rules{p.small_cap, p.unit_cap, p.unit_tiles, classify_chunk_tiles()};
    const int64_t max_e = std::min<int64_t>(plan::span_unit_max_entries(rules), lds_unit_entries(p.block));
    const char* why = "";
    const int64_t bad = plan::check_units(offR.data(), offS.data(), C, u.data(), n, max_e,
                                          p.unit_tiles, p.small_cap, &why);
    if (bad >= 0) {
        snprintf(g_err, sizeof(g_err), "work-list check: span unit %lld: %s", (long long)bad, why);
        return SJ_ERR_DEVICE;
    }
    return SJ_OK;
}

// After a join's status readback: false if it must run again (the scratch
// of the single pass ran out although the output fits: two passes then).
bool join_done(JoinWork& w, JoinParams& p, const DevStatus& hs, int64_t capacity) {
    w.last_single = p.single;
    w.last_small_cap = p.plain ? 0 : p.small_cap;
    w.last_med_cap = p.plain ? 0 : p.med_cap;
    if (p.single && (hs.flags & kStatScratch) && !(hs.flags & ~kStatScratch) &&
        (int64_t)hs.n_pairs <= capacity) {
        p.single = false;
        return false;
    }
    return true;
}

// The result of a finished join from its status (partition flags folded
// in): the error it maps to, the pair count, the optional sort.
sj_status join_outcome(const Part& R, const Part& S, const JoinParams& p, const JoinWork& w,
                       const DevStatus& hs, sj_pair* out, int64_t capacity, int64_t* n_pairs,
                       bool count_only, int64_t* cand, hipStream_t s) {
    const uint32_t flags = hs.flags;
    if (flags & kStatTooLarge) return SJ_ERR_TOO_LARGE;
    if (flags & (kStatInternal | kStatCapacity)) {
        snprintf(g_err, sizeof(g_err), "join: internal status flags 0x%x", flags);
        return SJ_ERR_DEVICE;
    }
    if (!p.plain && check_worklists_enabled()) {
        sj_status st = check_worklists(R, S, p, w);
        if (st != SJ_OK) return st;
    }
    *n_pairs = (int64_t)hs.n_pairs;
    if (cand) *cand = (int64_t)hs.n_cand;
    if (!count_only && (int64_t)hs.n_pairs > capacity) return SJ_ERR_CAPACITY;
    if (!count_only && (R.grid.flags & SJ_SORTED_OUTPUT))
        return sj_sort_pairs(out, *n_pairs, R.n, S.n, s);
    return SJ_OK;
}

// e2 non-null: distance join of two partitions of anchored squares (pairs
// with dx*dx + dy*dy <= *e2); *cand then receives the filter's pair count.
sj_status do_join(const sj_part* R, const sj_part* S, sj_pair* out, int64_t capacity,
                  int64_t* n_pairs, bool count_only, hipStream_t s, const double* e2 = nullptr,
                  int64_t* cand = nullptr) {
    if (!R || !S || !n_pairs || capacity < 0) return SJ_ERR_ARG;
    if (!count_only && capacity > 0 && !out) return SJ_ERR_ARG;
    if (!same_grid(R->grid, S->grid)) return SJ_ERR_GRID_MISMATCH;
    if (R->device != S->device) return SJ_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return SJ_ERR_DEVICE;
    if (cur != R->device && hipSetDevice(R->device) != hipSuccess) return SJ_ERR_DEVICE;
    DeviceState* ds = nullptr;
    sj_status st = device_state(R->device, &ds);
    if (st != SJ_OK) return st;
    JoinWork& w = ds->w;
    JoinParams p = tuned_params(R->device, R->grid, R->m, S->m, count_only, e2 != nullptr);
    if (e2) {
        p.dist = true;
        p.e2 = *e2;
    }
    st = join_prepare(w, p, (int64_t)R->bl.cells() * R->bl.tiles_per_cell(), R->m, S->m, capacity);
    if (st != SJ_OK) return st;
    hipError_t e = hipSuccess;
    DevStatus hs{};
    for (int attempt = 0; attempt < 2; ++attempt) {
        e = run_join(*R, *S, p, w, count_only ? nullptr : out, count_only ? 0 : capacity, s);
        if (e != hipSuccess) {
            set_err("join launch", e);
            return from_hip(e);
        }
        // fold the partition-time flags of both inputs into the status word
        e = read_status(w.st, ds->host, s);
        if (e != hipSuccess) {
            set_err("join status readback", e);
            return from_hip(e);
        }
        hs = *ds->host;
        if (!join_done(w, p, hs, capacity)) continue;
        break;
    }
    return join_outcome(*R, *S, p, w, hs, out, capacity, n_pairs, count_only, cand, s);
}

// Partitions of both inputs and their join with one status readback (see
// sj_join_rects): capacities are bounds, checked on the device; when a
// partition outgrows them, its buffers grow and the sequence runs again.
// e2 non-null: distance join of two sets of anchored squares, as do_join.
sj_status fused_join(const float* Rr, int64_t nR, const float* Sr, int64_t nS, const sj_grid* g,
                     sj_part** pr, sj_part** ps, sj_pair* out, int64_t capacity,
                     int64_t* n_pairs, bool count_only, hipStream_t s, const double* e2 = nullptr,
                     int64_t* cand = nullptr) {
    if (!pr || !ps || !n_pairs || nR < 0 || nS < 0 || capacity < 0) return SJ_ERR_ARG;
    if ((nR > 0 && !Rr) || (nS > 0 && !Sr) || (!count_only && capacity > 0 && !out))
        return SJ_ERR_ARG;
    if ((((uintptr_t)Rr | (uintptr_t)Sr) & 15u) != 0) return SJ_ERR_ARG;
    if (nR >= ((int64_t)1 << 30) || nS >= ((int64_t)1 << 30)) return SJ_ERR_TOO_LARGE;
    sj_grid grid;
    GridDev gd;
    sj_status rs = resolve_grid(g, grid, gd);
    if (rs != SJ_OK) return rs;
    if (grid.flags & SJ_PLAIN) return SJ_ERR_ARG;  // the plain schedule reads the offsets unguarded
    int dev = 0;
    if (current_device(&dev) != SJ_OK) return SJ_ERR_DEVICE;
    sj_part* P[2] = {*pr, *ps};
    const bool fresh[2] = {P[0] == nullptr, P[1] == nullptr};
    const float* rin[2] = {Rr, Sr};
    const int64_t nn[2] = {nR, nS};
    auto fail = [&](sj_status e) {
        for (int i = 0; i < 2; ++i)
            if (fresh[i] && P[i]) sj_part_free(P[i]);
        return e;
    };
    for (int i = 0; i < 2; ++i) {
        if (!P[i]) {
            P[i] = new (std::nothrow) sj_part();
            if (!P[i]) return fail(SJ_ERR_OOM);
            P[i]->device = dev;
        } else if (P[i]->device != dev) {
            return fail(SJ_ERR_ARG);
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceState* ds = nullptr;
    sj_status st = device_state(dev, &ds);
    if (st != SJ_OK) return fail(st);
    JoinWork& w = ds->w;
    // the tuning key: the entries of the last run on these handles when it
    // partitioned the same sizes on the same grid, else the rectangle counts
    int64_t mkey[2], need_m1[2], need_m[2];
    for (int i = 0; i < 2; ++i) {
        Part& Q = *P[i];
        const bool same = Q.st && Q.n == nn[i] && same_grid(Q.grid, grid) && Q.m > 0;
        mkey[i] = same ? Q.m : nn[i];
        need_m1[i] = std::max<int64_t>(Q.cap_m1, nn[i] + nn[i] / 4 + 4096);
        need_m[i] = std::max<int64_t>(Q.cap_m, 2 * nn[i] + 4096);
        if (!Q.st) {
            int64_t cap = 0;
            hipError_t e = grow(Q.st, cap, 1, true);
            if (e != hipSuccess) return fail(from_hip(e));
        }
        Q.bl = blocking_for(gd.kx, gd.ky);
        Q.gd = gd;
        Q.grid = grid;
    }
    JoinParams p = tuned_params(dev, grid, mkey[0], mkey[1], count_only, e2 != nullptr);
    if (e2) {
        p.dist = true;
        p.e2 = *e2;
    }
    DevStatus hs[3] = {};
    bool parts_done = false;
    for (int attempt = 0; attempt < 6; ++attempt) {
        hipError_t e = hipSuccess;
        if (!parts_done) {
            for (int i = 0; i < 2; ++i)
                if ((e = part_prepare(*P[i], nn[i], need_m1[i], need_m[i])) != hipSuccess)
                    return fail(from_hip(e));
            // both inputs in one set of launches where the batched scans take
            // them (their small launches then fill the GPU together)
            if (part_batchable(*P[0], nn[0]) && part_batchable(*P[1], nn[1])) {
                const float4* rr[2] = {(const float4*)rin[0], (const float4*)rin[1]};
                Part* pp[2] = {P[0], P[1]};
                e = part_batch_plan(ds->pb, pp, rr, nn, 2, w.num_cus);
                if (e == hipSuccess) e = run_partition_batch(ds->pb, s);
            } else {
                for (int i = 0; i < 2 && e == hipSuccess; ++i)
                    e = run_partition(*P[i], (const float4*)rin[i], nn[i], w.num_cus, s);
            }
            if (e != hipSuccess) {
                set_err("partition launch", e);
                return fail(from_hip(e));
            }
        }
        // work lists sized from the partitions' capacities (bounds of their entries)
        st = join_prepare(w, p, (int64_t)P[0]->bl.cells() * P[0]->bl.tiles_per_cell(),
                          P[0]->cap_m, P[1]->cap_m, capacity);
        if (st != SJ_OK) return fail(st);
        e = run_join(*P[0], *P[1], p, w, count_only ? nullptr : out, count_only ? 0 : capacity, s);
        if (e != hipSuccess) {
            set_err("join launch", e);
            return fail(from_hip(e));
        }
        // the one readback: both partitions' status and the join's
        if ((e = hipMemcpyAsync(&ds->host[0], P[0]->st, sizeof(DevStatus), hipMemcpyDeviceToHost,
                                s)) != hipSuccess ||
            (e = hipMemcpyAsync(&ds->host[1], P[1]->st, sizeof(DevStatus), hipMemcpyDeviceToHost,
                                s)) != hipSuccess ||
            (e = hipMemcpyAsync(&ds->host[2], w.st, sizeof(DevStatus), hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess) {
            set_err("status readback", e);
            return fail(from_hip(e));
        }
        for (int i = 0; i < 3; ++i) hs[i] = ds->host[i];
        bool regrow = false;
        for (int i = 0; i < 2; ++i) {
            const uint32_t f = hs[i].flags;
            if (f & kStatBadRect) return fail(SJ_ERR_RECT);
            if (f & kStatTooLarge) return fail(SJ_ERR_TOO_LARGE);
            if (f & kStatInternal) {
                snprintf(g_err, sizeof(g_err), "partition: internal status flags 0x%x", f);
                return fail(SJ_ERR_DEVICE);
            }
            if (f & kStatCapacity) {
                need_m1[i] = std::max<int64_t>(need_m1[i], (int64_t)hs[i].m1_total + 1);
                if (hs[i].m_total) need_m[i] = std::max<int64_t>(need_m[i], (int64_t)hs[i].m_total + 1);
                regrow = true;
            }
        }
        if (regrow) continue;
        parts_done = true;
        for (int i = 0; i < 2; ++i) {
            P[i]->n = nn[i];
            P[i]->m = (int64_t)hs[i].m_total;
            P[i]->m1 = (int64_t)hs[i].m1_total;
        }
        if (!join_done(w, p, hs[2], capacity)) continue;
        ds->host[0] = hs[2];  // the last join's status, as sj_join leaves it
        *pr = P[0];
        *ps = P[1];
        return join_outcome(*P[0], *P[1], p, w, hs[2], out, capacity, n_pairs, count_only,
                            cand, s);
    }
    snprintf(g_err, sizeof(g_err), "fused join: buffers still too small after regrowth");
    return fail(SJ_ERR_DEVICE);
}


// The schedule search of sj_tune; e2 non-null: of the distance join.
sj_status tune_impl(const sj_part* R, const sj_part* S, sj_pair* out, int64_t capacity,
                    int32_t reps, sj_tuning* best, void* stream, const double* e2) {
    if (!R || !S || capacity < 0 || reps < 1 || (capacity > 0 && !out)) return SJ_ERR_ARG;
    if (!same_grid(R->grid, S->grid)) return SJ_ERR_GRID_MISMATCH;
    if (R->grid.flags & SJ_PLAIN) return SJ_ERR_ARG;
    const bool count_only = (out == nullptr);
    const int mode = (count_only ? 1 : 0) | (e2 ? 2 : 0);
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SJ_ERR_DEVICE;
    const int blocks[] = {64, 128, 256, 512};
    const int taus[] = {128, 256, 1024};
    sj_tuning win{};
    win.ms = -1.0;
    sj_status rs = SJ_OK;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tune.erase(tune_key(R->device, R->grid, R->m, S->m, mode));
    }
    for (int blk : blocks) {
        const int E = lds_unit_entries(blk);
        for (int sc : {E / 4, E / 2}) {
            for (int mc : {1024, 2048}) {
                for (int tau : taus) {
                    if (R->grid.split_tau != 0 && tau != taus[0]) continue;  // fixed by the grid
                    sj_tuning t{blk, sc, mc, R->grid.split_tau != 0 ? 0 : tau, 0.0};
                    {
                        std::lock_guard<std::mutex> lk(g_mu);
                        g_tune[tune_key(R->device, R->grid, R->m, S->m, mode)] = t;
                    }
                    int64_t np = 0;
                    float ms = 0.f, tot = 0.f;
                    sj_status st = do_join(R, S, out, capacity, &np, count_only, s, e2);  // warm-up
                    for (int r = 0; r < reps && (st == SJ_OK || st == SJ_ERR_CAPACITY); ++r) {
                        if (hipEventRecord(e0, s) != hipSuccess) st = SJ_ERR_DEVICE;
                        if (st != SJ_ERR_DEVICE)
                            st = do_join(R, S, out, capacity, &np, count_only, s, e2);
                        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                            st = SJ_ERR_DEVICE;
                        tot += ms;
                    }
                    if (st != SJ_OK && st != SJ_ERR_CAPACITY) {
                        rs = st;
                        break;
                    }
                    t.ms = tot / reps;
                    if (win.ms < 0 || t.ms < win.ms) win = t;
                }
                if (rs != SJ_OK) break;
            }
            if (rs != SJ_OK) break;
        }
        if (rs != SJ_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_mu);
    const TuneKey key = tune_key(R->device, R->grid, R->m, S->m, mode);
    if (rs != SJ_OK) {
        g_tune.erase(key);
        return rs;
    }
    g_tune[key] = win;
    if (best) *best = win;
    return SJ_OK;
}
}  // namespace

// Entry points for the batch driver (batch.hip).
std::mutex& api_mutex() { return g_mu; }
void api_set_error(const char* msg) { snprintf(g_err, sizeof(g_err), "%s", msg); }
sj_status api_workspace(int dev, JoinWork** w, int* num_cus) {
    DeviceState* ds = nullptr;
    sj_status st = device_state(dev, &ds);
    if (st != SJ_OK) return st;
    *w = &ds->w;
    *num_cus = ds->w.num_cus;
    return SJ_OK;
}
sj_status api_resolve_grid(const sj_grid* g, sj_grid& out, GridDev& gd) {
    return resolve_grid(g, out, gd);
}
JoinParams api_join_params(const sj_grid& g, bool count_only) { return join_params(g, count_only); }
sj_status api_join_prepare(JoinWork& w, JoinParams& p, int64_t C, int64_t mR, int64_t mS,
                           int64_t capacity) {
    return join_prepare(w, p, C, mR, mS, capacity);
}
hipError_t api_part_prepare(Part& P, int64_t n, int64_t need_m1, int64_t need_m) {
    return part_prepare(P, n, need_m1, need_m);
}
sj_status api_distance_pairs(const sj_part* R, const sj_part* S, double e2, sj_pair* out,
                             int64_t capacity, int64_t* n_pairs, int64_t* cand, hipStream_t s) {
    return do_join(R, S, out, capacity, n_pairs, out == nullptr, s, &e2, cand);
}
sj_status api_distance_fused(const float* R, int64_t nR, const float* S, int64_t nS,
                             const sj_grid* g, sj_part** pr, sj_part** ps, double e2, sj_pair* out,
                             int64_t capacity, int64_t* n_pairs, int64_t* cand, hipStream_t s) {
    return fused_join(R, nR, S, nS, g, pr, ps, out, capacity, n_pairs, out == nullptr, s, &e2,
                      cand);
}
sj_status api_distance_tune(const sj_part* R, const sj_part* S, double e2, sj_pair* out,
                            int64_t capacity, int32_t reps, sj_tuning* best, hipStream_t s) {
    return tune_impl(R, S, out, capacity, reps, best, s, &e2);
}

}  // namespace sj

using namespace sj;

extern "C" {

sj_status sj_partition(const float* rects, int64_t n, const sj_grid* g, sj_part** out,
                       void* stream) {
    if (!out || n < 0 || (n > 0 && !rects)) return SJ_ERR_ARG;
    if (((uintptr_t)rects & 15u) != 0) return SJ_ERR_ARG;
    if (n >= ((int64_t)1 << 30)) return SJ_ERR_TOO_LARGE;
    sj_grid grid;
    GridDev gd;
    sj_status rs = resolve_grid(g, grid, gd);
    if (rs != SJ_OK) return rs;
    int dev = 0;
    if (current_device(&dev) != SJ_OK) return SJ_ERR_DEVICE;
    hipStream_t s = (hipStream_t)stream;

    sj_part* P = *out;
    const bool fresh = (P == nullptr);
    if (fresh) {
        P = new (std::nothrow) sj_part();
        if (!P) return SJ_ERR_OOM;
        P->device = dev;
    } else if (P->device != dev) {
        return SJ_ERR_ARG;
    }
    auto fail = [&](sj_status e) {
        if (fresh) sj_part_free(P);
        return e;
    };
    DeviceState* ds = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        sj_status st = device_state(dev, &ds);
        if (st != SJ_OK) return fail(st);
    }
    const Blocking bl = blocking_for(gd.kx, gd.ky);
    const int64_t G1 = bl.cells(), B2 = bl.tiles_per_cell(), Cb = G1 * B2;
    const int64_t ch1 = l1_chunk(n, G1);
    const int64_t nb1 = n > 0 ? (n + ch1 - 1) / ch1 : 1;
    int64_t need_m1 = std::max<int64_t>(P->cap_m1, n + n / 4 + 4096);
    int64_t need_m = std::max<int64_t>(P->cap_m, 2 * n + 4096);
    hipError_t e;
    if (!P->st) {
        int64_t cap = 0;
        if ((e = grow(P->st, cap, 1, true)) != hipSuccess) return fail(from_hip(e));
    }
    P->bl = bl;
    P->gd = gd;
    P->grid = grid;
    for (int attempt = 0; attempt < 4; ++attempt) {
        if ((e = part_prepare(*P, n, need_m1, need_m)) != hipSuccess) return fail(from_hip(e));
        if ((e = run_partition(*P, (const float4*)rects, n, ds->w.num_cus, s)) != hipSuccess) {
            set_err("partition launch", e);
            return fail(from_hip(e));
        }
        if ((e = read_status(P->st, ds->host, s)) != hipSuccess) {
            set_err("partition status readback", e);
            return fail(from_hip(e));
        }
        const DevStatus hs = *ds->host;
        if (hs.flags & kStatBadRect) return fail(SJ_ERR_RECT);
        if (hs.flags & kStatTooLarge) return fail(SJ_ERR_TOO_LARGE);
        if (hs.flags & kStatInternal) {
            snprintf(g_err, sizeof(g_err), "partition: internal status flags 0x%x", hs.flags);
            return fail(SJ_ERR_DEVICE);
        }
        if (hs.flags & kStatCapacity) {
            need_m1 = std::max<int64_t>(need_m1, (int64_t)hs.m1_total + 1);
            if (hs.m_total) need_m = std::max<int64_t>(need_m, (int64_t)hs.m_total + 1);
            continue;
        }
        P->n = n;
        P->m = (int64_t)hs.m_total;
        P->m1 = (int64_t)hs.m1_total;
        *out = P;
        return SJ_OK;
    }
    snprintf(g_err, sizeof(g_err), "partition: buffers still too small after regrowth");
    return fail(SJ_ERR_DEVICE);
}

sj_status sj_join(const sj_part* R, const sj_part* S, sj_pair* out, int64_t capacity,
                  int64_t* n_pairs, void* stream) {
    return do_join(R, S, out, capacity, n_pairs, false, (hipStream_t)stream);
}

sj_status sj_tune(const sj_part* R, const sj_part* S, sj_pair* out, int64_t capacity,
                  int32_t reps, sj_tuning* best, void* stream) {
    return tune_impl(R, S, out, capacity, reps, best, stream, nullptr);
}

sj_status sj_tune_set(const sj_part* R, const sj_part* S, int32_t count_only,
                      const sj_tuning* t) {
    if (!R || !S || !t) return SJ_ERR_ARG;
    if (t->block != 64 && t->block != 128 && t->block != 256 && t->block != 512) return SJ_ERR_ARG;
    if (t->small_cap < 2 || t->med_cap < 2 || t->split_tau < 0) return SJ_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    g_tune[tune_key(R->device, R->grid, R->m, S->m, count_only != 0)] = *t;
    return SJ_OK;
}

void sj_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tune.clear();
}

sj_status sj_tune_lookup(const sj_part* R, const sj_part* S, int32_t count_only, sj_tuning* t) {
    if (!R || !S || !t) return SJ_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tune.find(tune_key(R->device, R->grid, R->m, S->m, count_only != 0));
    if (it == g_tune.end()) return SJ_ERR_ARG;
    *t = it->second;
    return SJ_OK;
}

sj_status sj_tune_save(const char* path) {
    if (!path) return SJ_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return SJ_ERR_ARG;
    std::fprintf(f, "# arch k log2_mR log2_mS mode block small_cap med_cap split_tau ms\n");
    for (const auto& kv : g_tune) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, kv.first.dev) != hipSuccess) continue;
        plan::TuneLine t{};
        arch_name(prop, t.arch, sizeof(t.arch));
        t.k = kv.first.k;
        t.lr = kv.first.lr;
        t.ls = kv.first.ls;
        t.mode = kv.first.count_only;
        t.block = kv.second.block;
        t.small_cap = kv.second.small_cap;
        t.med_cap = kv.second.med_cap;
        t.split_tau = kv.second.split_tau;
        t.ms = kv.second.ms;
        char line[256];
        plan::format_tune_line(t, line, sizeof(line));
        std::fputs(line, f);
    }
    const bool ok = std::fclose(f) == 0;
    return ok ? SJ_OK : SJ_ERR_ARG;
}

sj_status sj_tune_load(const char* path, int32_t* n_loaded) {
    if (n_loaded) *n_loaded = 0;
    if (!path) return SJ_ERR_ARG;
    int dev = 0;
    if (current_device(&dev) != SJ_OK) return SJ_ERR_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return SJ_ERR_DEVICE;
    char mine[64];
    arch_name(prop, mine, sizeof(mine));
    FILE* f = std::fopen(path, "r");
    if (!f) return SJ_ERR_ARG;
    std::vector<std::pair<TuneKey, sj_tuning>> got;
    char line[512];
    bool bad = false;
    while (std::fgets(line, sizeof(line), f)) {
        plan::TuneLine t;
        const int r = plan::parse_tune_line(line, SJ_K_MAX, &t);
        if (r < 0) {
            bad = true;
            break;
        }
        if (r == 0 || std::strcmp(t.arch, mine) != 0) continue;
        got.emplace_back(TuneKey{dev, t.k, t.lr, t.ls, t.mode},
                         sj_tuning{t.block, t.small_cap, t.med_cap, t.split_tau, t.ms});
    }
    std::fclose(f);
    if (bad) {
        snprintf(g_err, sizeof(g_err), "sj_tune_load: malformed line in %s", path);
        return SJ_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : got) g_tune[kv.first] = kv.second;
    if (n_loaded) *n_loaded = (int32_t)got.size();
    return SJ_OK;
}

sj_status sj_join_count(const sj_part* R, const sj_part* S, int64_t* n_pairs, void* stream) {
    return do_join(R, S, nullptr, 0, n_pairs, true, (hipStream_t)stream);
}

sj_status sj_join_rects(const float* R, int64_t nR, const float* S, int64_t nS, const sj_grid* g,
                        sj_part** pr, sj_part** ps, sj_pair* out, int64_t capacity,
                        int64_t* n_pairs, void* stream) {
    return fused_join(R, nR, S, nS, g, pr, ps, out, capacity, n_pairs, out == nullptr,
                      (hipStream_t)stream);
}

sj_status sj_part_info(const sj_part* P, int64_t* n_rects, int64_t* n_entries, sj_grid* g) {
    if (!P) return SJ_ERR_ARG;
    if (n_rects) *n_rects = P->n;
    if (n_entries) *n_entries = P->m;
    if (g) *g = P->grid;
    return SJ_OK;
}

sj_status sj_part_stats(const sj_part* P, int64_t* level1_entries, int64_t* level2_chunks) {
    if (!P) return SJ_ERR_ARG;
    if (level1_entries) *level1_entries = P->m1;
    if (level2_chunks) {
        uint32_t nc = 0;
        if (P->st && hipMemcpy(&nc, &P->st->n_chunks, 4, hipMemcpyDeviceToHost) != hipSuccess)
            return SJ_ERR_DEVICE;
        *level2_chunks = nc;
    }
    return SJ_OK;
}

sj_status sj_part_download(const sj_part* P, int64_t* offsets, int32_t* ids, void* stream) {
    if (!P) return SJ_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipStreamSynchronize(s) != hipSuccess) return SJ_ERR_DEVICE;
    const int kx = P->gd.kx, ky = P->gd.ky;
    const Blocking bl = P->bl;
    const int64_t B2 = bl.tiles_per_cell();
    const int64_t Cb = (int64_t)bl.cells() * B2;
    std::vector<uint32_t> off((size_t)Cb + 1);
    std::vector<uint32_t> raw((size_t)std::max<int64_t>(P->m, 1));
    if (hipMemcpy(off.data(), P->off, (size_t)(Cb + 1) * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return SJ_ERR_DEVICE;
    if (P->m > 0 &&
        hipMemcpy(raw.data(), P->enti, (size_t)P->m * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return SJ_ERR_DEVICE;
    // regroup from the blocked tile order into row-major tile order of the
    // partition grid (stripes: kx = 1, one row per stripe)
    int64_t at = 0;
    for (int ty = 0; ty < ky; ++ty)
        for (int tx = 0; tx < kx; ++tx) {
            const int gx = tx / bl.Bx, gy = ty / bl.By;
            const int64_t bt = ((int64_t)gy * bl.Gx + gx) * B2 +
                               (int64_t)(ty - gy * bl.By) * bl.Bx + (tx - gx * bl.Bx);
            if (offsets) offsets[(int64_t)ty * kx + tx] = at;
            for (uint32_t q = off[bt]; q < off[bt + 1]; ++q, ++at)
                if (ids) ids[at] = (int32_t)(raw[q] & kIdMask);
        }
    if (offsets) offsets[(int64_t)kx * ky] = at;
    return SJ_OK;
}

void sj_part_free(sj_part* P) {
    if (!P) return;
    void* bufs[] = {P->h1, P->e1, P->e1i, P->cp, P->chunk_cell, P->h2, P->entb, P->enti, P->off,
                    P->scan_tmp, P->st};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    delete P;
}

const char* sj_status_string(sj_status s) {
    switch (s) {
        case SJ_OK: return "ok";
        case SJ_ERR_ARG: return "invalid argument";
        case SJ_ERR_RECT: return "invalid rectangle (NaN, infinite or inverted)";
        case SJ_ERR_CAPACITY: return "output capacity too small";
        case SJ_ERR_GRID_MISMATCH: return "inputs partitioned on different grids";
        case SJ_ERR_OOM: return "device out of memory";
        case SJ_ERR_DEVICE: return "HIP device error";
        case SJ_ERR_TOO_LARGE: return "input too large";
    }
    return "unknown status";
}

const char* sj_version(void) { return "sj 0.1 (gfx950)"; }

const char* sj_last_error(void) { return g_err; }

sj_status sj_last_join_stats(sj_join_stats* out) {
    if (!out) return SJ_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SJ_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev.find(dev);
    if (it == g_dev.end() || !it->second.init) return SJ_ERR_ARG;
    std::memset(out, 0, sizeof(*out));
    const JoinWork& w = it->second.w;
    if (hipDeviceSynchronize() != hipSuccess) return SJ_ERR_DEVICE;
    if (join_stats(w, w.last_single, out) != hipSuccess) return SJ_ERR_DEVICE;
    out->n_pairs = (int64_t)it->second.host->n_pairs;
    out->single_pass = w.last_single ? 1 : 0;
    out->small_cap = w.last_small_cap;
    out->med_cap = w.last_med_cap;
    return SJ_OK;
}

sj_status sj_sweep_axis(const sj_part* R, const sj_part* S, const int32_t* tiles, int64_t n,
                        int64_t* out, void* stream) {
    if (!R || !S || n < 0 || (n > 0 && (!tiles || !out))) return SJ_ERR_ARG;
    if (!same_grid(R->grid, S->grid)) return SJ_ERR_GRID_MISMATCH;
    if (R->device != S->device || (R->grid.flags & SJ_STRIPES)) return SJ_ERR_ARG;
    const int K = R->grid.k;
    for (int64_t j = 0; j < n; ++j)
        if (tiles[2 * j] < 0 || tiles[2 * j] >= K || tiles[2 * j + 1] < 0 || tiles[2 * j + 1] >= K)
            return SJ_ERR_ARG;
    if (n == 0) return SJ_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceState* ds = nullptr;
    sj_status st = device_state(R->device, &ds);
    if (st != SJ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    int32_t* dt = nullptr;
    int64_t* dout = nullptr;
    hipError_t e = hipMalloc((void**)&dt, (size_t)n * 2 * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&dout, (size_t)n * 4 * sizeof(int64_t));
    if (e == hipSuccess)
        e = hipMemcpyAsync(dt, tiles, (size_t)n * 2 * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = axis_query(*R, *S, dt, n, dout, ds->w.num_cus, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, dout, (size_t)n * 4 * sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (dt) (void)hipFree(dt);
    if (dout) (void)hipFree(dout);
    if (e != hipSuccess) set_err("sweep axis", e);
    return from_hip(e);
}

}  // extern "C"
