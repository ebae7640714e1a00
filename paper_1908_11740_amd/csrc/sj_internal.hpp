// Internal declarations shared by the HIP translation units of libsj.
// Device code targets gfx950 (CDNA4): 64-wide wavefronts, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sj.h"

namespace sj {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Grid and cell function (PBSM uniform grid, Sec. 2.2).
// cell(v) = clamp(floor((v - lo) * scale), 0, K - 1), evaluated with explicit
// round-to-nearest intrinsics so that every kernel computes bit-identical
// cell indices (no contraction into an FMA in one kernel but not another).
// It is monotone non-decreasing in v, which makes the integer form of the
// duplicate test exact: cell(max(a, b)) = max(cell(a), cell(b)).
// ---------------------------------------------------------------------------
struct GridDev {
    float x0, y0;  // lower corner of the gridded domain
    float sx, sy;  // K / domain width, K / domain height
    int K;
};

__device__ __forceinline__ int cell_of(float v, float lo, float scale, int K) {
    float f = floorf(__fmul_rn(__fsub_rn(v, lo), scale));
    f = fminf(fmaxf(f, 0.0f), (float)(K - 1));
    return (int)f;
}

// Order-preserving map float32 -> uint32 (after -0.0 -> +0.0).
__device__ __forceinline__ uint32_t order_key(float x) {
    uint32_t u = __float_as_uint(x + 0.0f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Entry id word: rectangle position in bits 0..29; bit 30 = the rectangle's
// x_l falls in this tile's column (cell(x_l) == tx); bit 31 = its y_l falls
// in this tile's row (cell(y_l) == ty).  For a pair found in tile T, the
// reference point (max x_l, max y_l) of Eq. (1) lies in T iff
// (bx_r | bx_s) & (by_r | by_s).
constexpr uint32_t kIdMask = 0x3FFFFFFFu;
constexpr uint32_t kBx = 0x40000000u;
constexpr uint32_t kBy = 0x80000000u;

// Device-side status word bits.
constexpr uint32_t kStatBadRect = 1u;
constexpr uint32_t kStatCapacity = 2u;  // an internal buffer was too small
constexpr uint32_t kStatInternal = 4u;  // broken invariant (count/scatter mismatch)

// Counters written by the device and read back once per call.
struct DevStatus {
    unsigned long long n_pairs;  // pairs found (may exceed the output capacity)
    unsigned long long m_total;  // entries of the partitioned side(s)
    uint32_t flags;              // kStat* bits
    uint32_t n_dense;            // dense tiles found by the join classification
    uint32_t n_units;            // LDS units built by the classification
    uint32_t pad;
};

// ---------------------------------------------------------------------------
// Partitioned input (device buffers) -- the opaque sj_part.
// ---------------------------------------------------------------------------
struct Part {
    int device = 0;
    sj_grid grid{};
    GridDev gd{};
    int64_t n = 0;         // rectangles
    int64_t m = 0;         // entries
    int64_t cap_c = 0;     // capacity of cnt / off (tiles)
    int64_t cap_m = 0;     // capacity of box / idf (entries)
    uint32_t* cnt = nullptr;   // [cap_c]    per-tile counts, all zero between calls
    uint32_t* off = nullptr;   // [cap_c+1]  exclusive prefix of counts
    float4* box = nullptr;     // [cap_m]    (x_l, y_l, x_u, y_u) per entry
    uint32_t* idf = nullptr;   // [cap_m]    id word per entry
    uint32_t* scan_tmp = nullptr;  // block sums of the scan
    int64_t cap_scan = 0;
    DevStatus* st = nullptr;   // device status
};

// Launch helpers implemented in partition.hip
hipError_t launch_count(const float4* rects, int64_t n, GridDev g, uint32_t* cnt, DevStatus* st,
                        hipStream_t s);
hipError_t launch_scan(const uint32_t* cnt, int64_t C, uint32_t* off, uint32_t* block_sums,
                       DevStatus* st, hipStream_t s);
int64_t scan_block_sums_needed(int64_t C);
hipError_t launch_scatter(const float4* rects, int64_t n, GridDev g, uint32_t* cnt,
                          const uint32_t* off, float4* box, uint32_t* idf, int64_t cap_m,
                          DevStatus* st, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// Join workspace and launch helpers implemented in join.hip
// ---------------------------------------------------------------------------
struct JoinParams {
    int K;
    int64_t C;
    int split_tau;   // pivots per dense unit
    int unit_cap;    // LDS unit entry budget
    int small_cap;   // tiles with more entries than this are dense
    int block;       // threads per workgroup for the sweep kernels
    bool plain;      // one workgroup per tile, no batching, no splitting
    bool count_only;
};

struct JoinWork {
    int device = 0;
    // classification outputs
    uint32_t* tiles = nullptr;      // [cap_tiles] tile ids of LDS units (grouped)
    uint2* units = nullptr;         // [cap_units] (first index into tiles, count)
    uint4* dense = nullptr;         // [cap_dense] (tile, base in dense buffer, nr, ns)
    uint32_t* dense_unit_prefix = nullptr;  // [cap_dense+1]
    int64_t cap_tiles = 0, cap_units = 0, cap_dense = 0, cap_prefix = 0;
    // globally sorted dense segments
    float4* dbox = nullptr;         // [cap_dent]
    uint32_t* didf = nullptr;       // [cap_dent]
    unsigned long long* dtmp = nullptr;  // [2 * cap_dent] merge-sort scratch
    int64_t cap_dent = 0;
    // queue counters: [0] LDS units taken, [1] dense sort taken, [2] dense units taken,
    // [3] tiles written, [4] units written, [5] dense entries allocated, [6] dense units
    uint32_t* ctr = nullptr;
    DevStatus* st = nullptr;
    void* host_status = nullptr;    // pinned DevStatus mirror
    int num_cus = 0;
};

hipError_t run_join(const Part& R, const Part& S, const JoinParams& p, JoinWork& w,
                    sj_pair* out, int64_t capacity, hipStream_t s);

}  // namespace sj
