// C ABI of libsj (declared in include/sj.h): argument checks, handle and
// workspace management, kernel sequencing and the one status readback per
// call.  No exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>

#include "sj_internal.hpp"
#include "sj_prof.hpp"

struct sj_part : public sj::Part {};

namespace sj {

int lds_unit_entries(int block);

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
    gd.x0 = out.domain[0];
    gd.y0 = out.domain[1];
    gd.sx = (float)out.k / w;
    gd.sy = (float)out.k / h;
    gd.K = out.k;
    if (!std::isfinite(gd.sx) || !std::isfinite(gd.sy)) return SJ_ERR_ARG;
    return SJ_OK;
}

bool same_grid(const sj_grid& a, const sj_grid& b) {
    return a.k == b.k && std::memcmp(a.domain, b.domain, sizeof(a.domain)) == 0;
}

struct DeviceState {
    JoinWork w;
    DevStatus* host = nullptr;  // pinned
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
        if (hipHostMalloc((void**)&d.host, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess)
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

hipError_t read_status(const DevStatus* dst, DevStatus* host, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(host, dst, sizeof(DevStatus), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// Schedule parameters of a join.
JoinParams join_params(const sj_grid& g, bool count_only) {
    JoinParams p{};
    p.K = g.k;
    p.C = (int64_t)g.k * g.k;
    p.plain = (g.flags & SJ_PLAIN) != 0;
    p.count_only = count_only;
    p.block = 256;
    const int E = lds_unit_entries(p.block);
    p.small_cap = p.plain ? E : E / 4;
    p.unit_cap = E - p.small_cap;
    p.split_tau = g.split_tau > 0 ? g.split_tau : 256;
    if (p.plain || g.split_tau == INT32_MAX) p.split_tau = INT32_MAX;
    return p;
}

sj_status do_join(const sj_part* R, const sj_part* S, sj_pair* out, int64_t capacity,
                  int64_t* n_pairs, bool count_only, hipStream_t s) {
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
    JoinParams p = join_params(R->grid, count_only);
    const int E = lds_unit_entries(p.block);
    const int64_t mR = R->m, mS = S->m;
    const int64_t active = std::min<int64_t>(p.C, std::min(mR, mS)) + 1;
    const int64_t dense_thr = p.plain ? E : p.small_cap;
    const int64_t ndense = (mR + mS) / (dense_thr + 1) + 2;
    hipError_t e = hipSuccess;
    if (!p.plain) {
        if ((e = grow(w.tiles, w.cap_tiles, active)) != hipSuccess) return from_hip(e);
        if ((e = grow(w.units, w.cap_units, active)) != hipSuccess) return from_hip(e);
    }
    if ((e = grow(w.dense, w.cap_dense, ndense)) != hipSuccess) return from_hip(e);
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
    const DevStatus hs = *ds->host;
    const uint32_t flags = hs.flags;
    if (flags & (kStatInternal | kStatCapacity)) {
        snprintf(g_err, sizeof(g_err), "join: internal status flags 0x%x", flags);
        return SJ_ERR_DEVICE;
    }
    *n_pairs = (int64_t)hs.n_pairs;
    if (!count_only && (int64_t)hs.n_pairs > capacity) return SJ_ERR_CAPACITY;
    return SJ_OK;
}

}  // namespace
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
    const int64_t C = (int64_t)grid.k * grid.k;

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
    hipError_t e;
    if (!P->st) {
        int64_t cap = 0;
        if ((e = grow(P->st, cap, 1, true)) != hipSuccess) return fail(from_hip(e));
    }
    {
        int64_t cc = P->cap_c;
        if (C > cc || !P->cnt) {
            if ((e = grow(P->cnt, P->cap_c, C, true)) != hipSuccess) return fail(from_hip(e));
            int64_t co = 0;
            if (P->off) (void)hipFree(P->off);
            P->off = nullptr;
            if ((e = grow(P->off, co, P->cap_c + 1)) != hipSuccess) return fail(from_hip(e));
        }
        if ((e = grow(P->scan_tmp, P->cap_scan, scan_block_sums_needed(P->cap_c))) != hipSuccess)
            return fail(from_hip(e));
    }
    DeviceState* ds = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        sj_status st = device_state(dev, &ds);
        if (st != SJ_OK) return fail(st);
    }
    const float4* r4 = (const float4*)rects;
    if ((e = launch_fill_u32((uint32_t*)P->st, 0u, sizeof(DevStatus) / 4, s)) != hipSuccess)
        return fail(from_hip(e));
    {
        ProfRange pr("k_count", s);
        if ((e = launch_count(r4, n, gd, P->cnt, P->st, s)) != hipSuccess) return fail(from_hip(e));
    }
    {
        ProfRange pr("k_scan", s);
        if ((e = launch_scan(P->cnt, C, P->off, P->scan_tmp, P->st, s)) != hipSuccess)
            return fail(from_hip(e));
    }
    if ((e = read_status(P->st, ds->host, s)) != hipSuccess) return fail(from_hip(e));
    const DevStatus hs = *ds->host;
    if (hs.flags & (kStatBadRect | kStatCapacity)) {
        // restore the all-zero count invariant before reporting
        (void)launch_fill_u32(P->cnt, 0u, C, s);
        (void)launch_fill_u32((uint32_t*)P->st, 0u, sizeof(DevStatus) / 4, s);
        (void)hipStreamSynchronize(s);
        return fail((hs.flags & kStatBadRect) ? SJ_ERR_RECT : SJ_ERR_TOO_LARGE);
    }
    const int64_t M = (int64_t)hs.m_total;
    if (M > P->cap_m || !P->box) {
        if (P->box) (void)hipFree(P->box);
        if (P->idf) (void)hipFree(P->idf);
        P->box = nullptr;
        P->idf = nullptr;
        P->cap_m = 0;
        int64_t c1 = 0, c2 = 0;
        if ((e = grow(P->box, c1, std::max<int64_t>(M, 1))) != hipSuccess ||
            (e = grow(P->idf, c2, c1)) != hipSuccess) {
            (void)launch_fill_u32(P->cnt, 0u, C, s);
            (void)hipStreamSynchronize(s);
            return fail(from_hip(e));
        }
        P->cap_m = c1;
    }
    {
        ProfRange pr("k_scatter", s);
        if ((e = launch_scatter(r4, n, gd, P->cnt, P->off, P->box, P->idf, P->cap_m, P->st, s)) !=
            hipSuccess)
            return fail(from_hip(e));
    }
    P->grid = grid;
    P->gd = gd;
    P->n = n;
    P->m = M;
    *out = P;
    return SJ_OK;
}

sj_status sj_join(const sj_part* R, const sj_part* S, sj_pair* out, int64_t capacity,
                  int64_t* n_pairs, void* stream) {
    return do_join(R, S, out, capacity, n_pairs, false, (hipStream_t)stream);
}

sj_status sj_join_count(const sj_part* R, const sj_part* S, int64_t* n_pairs, void* stream) {
    return do_join(R, S, nullptr, 0, n_pairs, true, (hipStream_t)stream);
}

sj_status sj_part_info(const sj_part* P, int64_t* n_rects, int64_t* n_entries, sj_grid* g) {
    if (!P) return SJ_ERR_ARG;
    if (n_rects) *n_rects = P->n;
    if (n_entries) *n_entries = P->m;
    if (g) *g = P->grid;
    return SJ_OK;
}

sj_status sj_part_download(const sj_part* P, int64_t* offsets, int32_t* ids, void* stream) {
    if (!P) return SJ_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipStreamSynchronize(s) != hipSuccess) return SJ_ERR_DEVICE;
    const int64_t C = (int64_t)P->grid.k * P->grid.k;
    if (offsets) {
        uint32_t* tmp = (uint32_t*)malloc((size_t)(C + 1) * 4);
        if (!tmp) return SJ_ERR_OOM;
        if (hipMemcpy(tmp, P->off, (size_t)(C + 1) * 4, hipMemcpyDeviceToHost) != hipSuccess) {
            free(tmp);
            return SJ_ERR_DEVICE;
        }
        for (int64_t i = 0; i <= C; ++i) offsets[i] = tmp[i];
        free(tmp);
    }
    if (ids && P->m > 0) {
        if (hipMemcpy(ids, P->idf, (size_t)P->m * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return SJ_ERR_DEVICE;
        for (int64_t i = 0; i < P->m; ++i) ids[i] = (int32_t)((uint32_t)ids[i] & kIdMask);
    }
    return SJ_OK;
}

void sj_part_free(sj_part* P) {
    if (!P) return;
    if (P->cnt) (void)hipFree(P->cnt);
    if (P->off) (void)hipFree(P->off);
    if (P->box) (void)hipFree(P->box);
    if (P->idf) (void)hipFree(P->idf);
    if (P->scan_tmp) (void)hipFree(P->scan_tmp);
    if (P->st) (void)hipFree(P->st);
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

}  // extern "C"
