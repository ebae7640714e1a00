// Epsilon-distance join of two point sets on top of the MBR join: the
// filter-and-refine reduction of Sec. 1.  Every point becomes a square of
// side eps, the squares of P and Q are partitioned and joined like any
// rectangles, and each pair the filter passes is refined by its distance.
//
// Result: every (i, j) with D(p_i, q_j) <= E, where, in float64 from the
// float32 inputs, dx = p.x - q.x, dy = p.y - q.y, D = dx*dx + dy*dy and
// E = eps*eps, each operation rounded once (no fused multiply-add).  The set
// is a pure function of the inputs: it depends on no grid, schedule or
// launch shape.
//
// Squares.  The square of a point c is anchored at it: [c, u(c)] on each
// axis, with u(c) = c + eps + m, m = (|c| + eps) * 2^-44, summed in float64
// and rounded up to float32.  Two squares meet on an axis iff their lower
// ends are at most the side apart, as for squares centred on the points, so
// the filter is the same; and the lower corner of every entry is its input
// point exactly, so the join tests D <= E on the two boxes it has in hand
// (no candidate list, no gathers of the points).
//
// Filter soundness.  D <= E implies |c_p - c_q| <= eps * (1 + 2^-50) on each
// axis (every float64 rounding above is a relative error of at most 2^-53).
// The two float64 additions of u(c) lose at most 2^-52 (|c| + eps) < m, so
// u(c) >= c + eps * (1 + 2^-45): the squares of every accepted pair overlap,
// and the pair is examined in the tile of its reference point.  The filter
// also passes pairs farther than eps (the squares' corners, the margin);
// the distance test drops them.
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

// Upper end of the anchored square of c (see above).
__device__ __forceinline__ float upper_end(float c, double eps) {
    const double cd = (double)c;
    const double m = __dmul_rn(__dadd_rn(fabs(cd), eps), 0x1p-44);
    return up_f(__dadd_rn(__dadd_rn(cd, eps), m));
}

// One thread per point: its anchored, outward-rounded square of side eps.  A
// non-finite coordinate gives a non-finite bound, which the partition
// rejects with SJ_ERR_RECT.
__global__ __launch_bounds__(256) void k_point_squares(const float2* __restrict__ pts, int64_t n,
                                                       float eps, float4* __restrict__ box) {
    const double e = (double)eps;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float2 p = pts[i];
        box[i] = make_float4(p.x, p.y, upper_end(p.x, e), upper_end(p.y, e));
    }
}

// Library-owned state per device: the squares of both inputs, their
// partitions and the tuner's pair buffer, reused (and grown) across calls.
struct DistState {
    float4* sqP = nullptr;
    float4* sqQ = nullptr;
    int64_t capP = 0, capQ = 0;
    sj_pair* tune_out = nullptr;
    int64_t cap_tune = 0;
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

// Squares of both point sets and the grid (chosen when g->k is 0), and,
// with partition, the two partitions, in the device state d.  The caller
// holds g_dmu.
sj_status prepare(DistState& d, const float* P, int64_t nP, const float* Q, int64_t nQ, float eps,
                  sj_grid* g, hipStream_t s, bool partition = true) {
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
    if (!partition) return SJ_OK;
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

// E = eps * eps in float64 (one rounding)
double eps_sq(float eps) { return (double)eps * (double)eps; }

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
    st = prepare(d, P, nP, Q, nQ, eps, g, s, (g->flags & SJ_PLAIN) != 0);
    if (st != SJ_OK) return st;
    // the join tests the distance of every filter pair and writes the result
    // (sorted by (i, j) when the grid asks for it); both partitions and the
    // join with one status readback, except on the plain schedule
    int64_t cand = 0;
    if (g->flags & SJ_PLAIN)
        st = api_distance_pairs(d.PP, d.PQ, eps_sq(eps), out, capacity, n_pairs, &cand, s);
    else
        st = api_distance_fused((const float*)d.sqP, nP, (const float*)d.sqQ, nQ, g, &d.PP,
                                &d.PQ, eps_sq(eps), out, capacity, n_pairs, &cand, s);
    if (st == SJ_OK || st == SJ_ERR_CAPACITY) d.last_candidates = cand;
    return st;
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
    // every schedule is timed with its full output, in a library buffer
    const double e2 = eps_sq(eps);
    int64_t np = 0, cand = 0;
    st = api_distance_pairs(d.PP, d.PQ, e2, nullptr, 0, &np, &cand, s);
    if (st != SJ_OK) return st;
    if (grow_to(d.tune_out, d.cap_tune, std::max<int64_t>(np, 1)) != hipSuccess) return SJ_ERR_OOM;
    return api_distance_tune(d.PP, d.PQ, e2, d.tune_out, d.cap_tune, reps, best, s);
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
