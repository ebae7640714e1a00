// Epsilon-distance join of two point sets on top of the MBR join: the
// filter-and-refine reduction of Sec. 1.  Every point becomes a square of
// side eps centred on it, the squares of P and Q are partitioned and joined
// like any rectangles, and each candidate pair is then refined by its
// distance.
//
// Result: every (i, j) with D(p_i, q_j) <= E, where, in float64 from the
// float32 inputs, dx = p.x - q.x, dy = p.y - q.y, D = dx*dx + dy*dy and
// E = eps*eps, each operation rounded once (no fused multiply-add).  The set
// is a pure function of the inputs: it depends on no grid, schedule or
// launch shape.
//
// Filter soundness.  The squares are widened before they are rounded
// outward to float32: half-side eps/2 plus m = (|c| + eps/2) * 2^-44 per
// coordinate c.  D <= E implies |c_p - c_q| <= eps * (1 + 2^-50) on each
// axis (every float64 rounding above is a relative error of at most 2^-53),
// while two widened squares overlap on an axis whenever their centres are
// within eps + (m_p + m_q)(1 - 2^-7) >= eps * (1 + 2^-45) on it (the
// roundings of the bounds cost less than m / 128), so every accepted pair is
// a candidate.  The filter also keeps pairs farther than eps (the squares'
// corners, the margin); the refinement drops them.
#include <cmath>
#include <map>
#include <mutex>

#include "sj_internal.hpp"
#include "sj_prof.hpp"

namespace sj {
namespace {

// Neighbouring float32 values by stepping the bit pattern (IEEE-754 order);
// called only on values that have a finite neighbour in that direction.
__device__ __forceinline__ float step_down(float f) {
    if (f == 0.f) return -__int_as_float(1);
    const int b = __float_as_int(f);
    return __int_as_float(f > 0.f ? b - 1 : b + 1);
}

__device__ __forceinline__ float step_up(float f) {
    if (f == 0.f) return __int_as_float(1);
    const int b = __float_as_int(f);
    return __int_as_float(f > 0.f ? b + 1 : b - 1);
}

// Largest float32 <= v and smallest float32 >= v (v float64).
__device__ __forceinline__ float down_f(double v) {
    const float f = (float)v;
    return (double)f > v ? step_down(f) : f;
}

__device__ __forceinline__ float up_f(double v) {
    const float f = (float)v;
    return (double)f < v ? step_up(f) : f;
}

__device__ __forceinline__ void widen(float c, double h, float& lo, float& hi) {
    const double cd = (double)c;
    const double m = __dmul_rn(__dadd_rn(fabs(cd), h), 0x1p-44);
    lo = down_f(__dsub_rn(__dsub_rn(cd, h), m));
    hi = up_f(__dadd_rn(__dadd_rn(cd, h), m));
}

// One thread per point: the widened, outward-rounded square of side eps.  A
// non-finite coordinate gives a non-finite bound, which the partition
// rejects with SJ_ERR_RECT.
__global__ __launch_bounds__(256) void k_point_squares(const float2* __restrict__ pts, int64_t n,
                                                       float eps, float4* __restrict__ box) {
    const double h = 0.5 * (double)eps;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float2 p = pts[i];
        float4 b;
        widen(p.x, h, b.x, b.z);
        widen(p.y, h, b.y, b.w);
        box[i] = b;
    }
}

// Refinement: keep the candidates (r, s) with D <= E.  The two point reads
// per candidate are random gathers, so each thread takes kRefineU candidates
// (strided by the block size, so the candidate reads coalesce) and issues all
// of their gathers before the first test, to keep many in flight.  A
// wavefront's kept pairs are placed with one atomic and a lane prefix sum of
// the per-lane counts; positions at or beyond `capacity` are counted, not
// written.
constexpr int kRefineU = 8;
constexpr int kRefineBlock = 256;

__global__ __launch_bounds__(kRefineBlock) void k_refine(const sj_pair* __restrict__ cand,
                                                         int64_t nc,
                                                         const float2* __restrict__ P,
                                                         const float2* __restrict__ Q, float eps,
                                                         sj_pair* __restrict__ out,
                                                         int64_t capacity,
                                                         unsigned long long* __restrict__ count) {
    const double e2 = __dmul_rn((double)eps, (double)eps);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t span = (int64_t)kRefineBlock * kRefineU;
    for (int64_t base = (int64_t)blockIdx.x * span; base < nc; base += (int64_t)gridDim.x * span) {
        // slots past the end read candidate (0, 0) (both sets are non-empty
        // when there is a candidate) and are masked out of the result
        sj_pair c[kRefineU];
        float2 p[kRefineU], q[kRefineU];
        uint32_t valid = 0;
#pragma unroll
        for (int u = 0; u < kRefineU; ++u) {
            const int64_t i = base + (int64_t)u * kRefineBlock + threadIdx.x;
            const bool in = i < nc;
            c[u] = cand[in ? i : 0];
            valid |= (uint32_t)in << u;
        }
#pragma unroll
        for (int u = 0; u < kRefineU; ++u) {
            p[u] = P[c[u].r];
            q[u] = Q[c[u].s];
        }
        uint32_t keep = 0;
#pragma unroll
        for (int u = 0; u < kRefineU; ++u) {
            const double dx = __dsub_rn((double)p[u].x, (double)q[u].x);
            const double dy = __dsub_rn((double)p[u].y, (double)q[u].y);
            if (__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)) <= e2) keep |= 1u << u;
        }
        keep &= valid;
        const int cnt = __popc(keep);
        int incl = cnt;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int t = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += t;
        }
        const int total = __shfl(incl, kWave - 1, kWave);
        if (total == 0) continue;
        unsigned long long wbase = 0;
        if (lane == kWave - 1) wbase = atomicAdd(count, (unsigned long long)total);
        wbase = __shfl(wbase, kWave - 1, kWave);
        unsigned long long at = wbase + (unsigned long long)(incl - cnt);
#pragma unroll
        for (int u = 0; u < kRefineU; ++u) {
            if (keep >> u & 1u) {
                if (at < (unsigned long long)capacity) out[at] = c[u];
                ++at;
            }
        }
    }
}

// Library-owned state per device: the squares of both inputs, their
// partitions and the candidate buffer, reused (and grown) across calls.
struct DistState {
    float4* sqP = nullptr;
    float4* sqQ = nullptr;
    int64_t capP = 0, capQ = 0;
    sj_pair* cand = nullptr;
    int64_t cap_cand = 0;
    unsigned long long* count = nullptr;
    unsigned long long* host = nullptr;
    sj_part* PP = nullptr;
    sj_part* PQ = nullptr;
    int64_t last_candidates = 0;
};

std::mutex g_dmu;
std::map<int, DistState> g_ds;

template <class T>
hipError_t grow_to(T*& p, int64_t& cap, int64_t need) {
    if (p && need <= cap) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    const int64_t nc = need + need / 4 + 1024;
    const hipError_t e = hipMalloc((void**)&p, (size_t)nc * sizeof(T));
    if (e == hipSuccess) cap = nc;
    return e;
}

unsigned blocks_for(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384));
}

}  // namespace
}  // namespace sj

using namespace sj;

extern "C" {

namespace {

// Squares of both point sets, the grid (chosen when g->k is 0) and the two
// partitions, in the device state d.  The caller holds g_dmu.
sj_status prepare(DistState& d, const float* P, int64_t nP, const float* Q, int64_t nQ, float eps,
                  sj_grid* g, hipStream_t s) {
    if (!d.count) {
        if (hipMalloc((void**)&d.count, sizeof(unsigned long long)) != hipSuccess) return SJ_ERR_OOM;
        if (hipHostMalloc((void**)&d.host, sizeof(unsigned long long), hipHostMallocDefault) !=
            hipSuccess) {
            d.host = nullptr;
            (void)hipFree(d.count);
            d.count = nullptr;
            return SJ_ERR_OOM;
        }
    }
    if (grow_to(d.sqP, d.capP, std::max<int64_t>(nP, 1)) != hipSuccess ||
        grow_to(d.sqQ, d.capQ, std::max<int64_t>(nQ, 1)) != hipSuccess)
        return SJ_ERR_OOM;
    {
        ProfRange pr("k_point_squares", s);
        if (nP > 0)
            hipLaunchKernelGGL(k_point_squares, dim3(blocks_for(nP)), dim3(256), 0, s,
                               (const float2*)P, nP, eps, d.sqP);
        if (nQ > 0)
            hipLaunchKernelGGL(k_point_squares, dim3(blocks_for(nQ)), dim3(256), 0, s,
                               (const float2*)Q, nQ, eps, d.sqQ);
        if (hipGetLastError() != hipSuccess) return SJ_ERR_DEVICE;
    }
    sj_status st = SJ_OK;
    if (g->k == 0) {
        st = sj_choose_grid((const float*)d.sqP, nP, (const float*)d.sqQ, nQ, g, nullptr, s);
        if (st != SJ_OK) return st;
    }
    st = sj_partition((const float*)d.sqP, nP, g, &d.PP, s);
    if (st != SJ_OK) return st;
    return sj_partition((const float*)d.sqQ, nQ, g, &d.PQ, s);
}

sj_status check_args(const float* P, int64_t nP, const float* Q, int64_t nQ, float eps,
                     const sj_grid* g) {
    if (!g || nP < 0 || nQ < 0 || (nP > 0 && !P) || (nQ > 0 && !Q) || !(eps >= 0.f) ||
        !std::isfinite(eps))
        return SJ_ERR_ARG;
    if (((uintptr_t)P & 7u) || ((uintptr_t)Q & 7u)) return SJ_ERR_ARG;
    if (nP >= ((int64_t)1 << 30) || nQ >= ((int64_t)1 << 30)) return SJ_ERR_TOO_LARGE;
    return SJ_OK;
}

}  // namespace

sj_status sj_distance_join(const float* P, int64_t nP, const float* Q, int64_t nQ, float eps,
                           sj_grid* g, sj_pair* out, int64_t capacity, int64_t* n_pairs,
                           void* stream) {
    sj_status st = check_args(P, nP, Q, nQ, eps, g);
    if (st != SJ_OK) return st;
    if (!n_pairs || capacity < 0 || (!out && capacity != 0)) return SJ_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SJ_ERR_DEVICE;
    const hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_dmu);
    DistState& d = g_ds[dev];
    st = prepare(d, P, nP, Q, nQ, eps, g, s);
    if (st != SJ_OK) return st;
    int64_t nc = 0;
    st = sj_join(d.PP, d.PQ, d.cand, d.cap_cand, &nc, stream);
    if (st == SJ_ERR_CAPACITY) {
        if (grow_to(d.cand, d.cap_cand, nc) != hipSuccess) return SJ_ERR_OOM;
        st = sj_join(d.PP, d.PQ, d.cand, d.cap_cand, &nc, stream);
    }
    if (st != SJ_OK) return st;
    d.last_candidates = nc;
    {
        ProfRange pr("k_refine", s);
        if (hipMemsetAsync(d.count, 0, sizeof(unsigned long long), s) != hipSuccess)
            return SJ_ERR_DEVICE;
        const int64_t span = (int64_t)kRefineBlock * kRefineU;
        const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nc + span - 1) / span, 8192));
        if (nc > 0)
            hipLaunchKernelGGL(k_refine, dim3(nb), dim3(kRefineBlock), 0, s, d.cand, nc,
                               (const float2*)P, (const float2*)Q, eps, out, capacity, d.count);
        if (hipGetLastError() != hipSuccess) return SJ_ERR_DEVICE;
    }
    if (hipMemcpyAsync(d.host, d.count, sizeof(unsigned long long), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SJ_ERR_DEVICE;
    *n_pairs = (int64_t)*d.host;
    if (out && *n_pairs > capacity) return SJ_ERR_CAPACITY;
    if (out && (g->flags & SJ_SORTED_OUTPUT)) return sj_sort_pairs(out, *n_pairs, nP, nQ, stream);
    return SJ_OK;
}

sj_status sj_distance_tune(const float* P, int64_t nP, const float* Q, int64_t nQ, float eps,
                           sj_grid* g, int32_t reps, sj_tuning* best, void* stream) {
    sj_status st = check_args(P, nP, Q, nQ, eps, g);
    if (st != SJ_OK) return st;
    if (reps < 1) return SJ_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SJ_ERR_DEVICE;
    const hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_dmu);
    DistState& d = g_ds[dev];
    st = prepare(d, P, nP, Q, nQ, eps, g, s);
    if (st != SJ_OK) return st;
    // the candidate buffer holds every candidate, so each schedule is timed
    // with its full output
    int64_t nc = 0;
    st = sj_join_count(d.PP, d.PQ, &nc, stream);
    if (st != SJ_OK) return st;
    if (grow_to(d.cand, d.cap_cand, std::max<int64_t>(nc, 1)) != hipSuccess) return SJ_ERR_OOM;
    return sj_tune(d.PP, d.PQ, d.cand, d.cap_cand, reps, best, stream);
}

sj_status sj_distance_last_info(sj_distance_info* info) {
    if (!info) return SJ_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SJ_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_dmu);
    *info = sj_distance_info{};
    const auto it = g_ds.find(dev);
    if (it == g_ds.end() || !it->second.PP || !it->second.PQ) return SJ_OK;
    const DistState& d = it->second;
    info->candidates = d.last_candidates;
    sj_status st = sj_part_info(d.PP, nullptr, &info->entries_p, nullptr);
    if (st == SJ_OK) st = sj_part_info(d.PQ, nullptr, &info->entries_q, nullptr);
    if (st == SJ_OK) st = sj_part_stats(d.PP, &info->level1_entries_p, nullptr);
    if (st == SJ_OK) st = sj_part_stats(d.PQ, &info->level1_entries_q, nullptr);
    return st;
}

}  // extern "C"
