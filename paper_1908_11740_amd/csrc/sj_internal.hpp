// Internal declarations shared by the HIP translation units of libsj.
// Device code targets gfx950 (CDNA4): 64-wide wavefronts, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

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
    float x0, y0;   // lower corner of the gridded domain (partition axes)
    float sx, sy;   // kx / domain width, ky / domain height
    int kx, ky;     // cells along x and y
    int transpose;  // 1: each rectangle's x and y are swapped on load (stripes, see sj.h)
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
constexpr uint32_t kStatCapacity = 2u;  // an internal buffer was too small (sizes reported)
constexpr uint32_t kStatInternal = 4u;  // broken invariant
constexpr uint32_t kStatTooLarge = 8u;  // more than 2^31 - 1 entries
constexpr uint32_t kStatScratch = 16u;  // single-pass pair scratch ran out (two-pass retry)

// Counters written by the device and read back once per call.
struct DevStatus {
    unsigned long long n_pairs;   // pairs found (may exceed the output capacity)
    unsigned long long m_total;   // tile entries of the partitioned input
    unsigned long long m1_total;  // coarse-cell entries (level 1)
    uint32_t flags;               // kStat* bits
    uint32_t n_dense;             // dense tiles found by the join classification
    uint32_t n_units;             // LDS units built by the classification
    uint32_t n_chunks;            // level-2 chunks of the partition
    unsigned long long n_cand;    // distance join: pairs passed by the filter
};

// Two-level blocking of the K x K grid: G x G coarse cells of B x B tiles.
constexpr int kCoarseMax = 64;    // G <= 64: level-1 LDS histogram <= 16 KB
constexpr int kCoarsePref = 32;   // preferred G (longer level-1 write runs)
constexpr int kMaxB = (SJ_K_MAX + kCoarseMax - 1) / kCoarseMax;  // B <= 128: level-2 LDS <= 64 KB
constexpr uint32_t kChunk2 = 4096;  // level-1 entries per level-2 chunk
constexpr int64_t kL1Blocks = 1024;  // level-1 workgroups per input (upper bound: 4 per CU)
constexpr int64_t kL1MinChunk = 2048;
constexpr int kL1StageChunk = 4096;     // level-1 chunk of the staged scatter (rectangles)
constexpr int kL1StageMaxG1 = 1024;     // coarse cells the staged level-1 scatter handles
constexpr int64_t kL1StageMaxChunks = 16384;  // ... and chunks (inputs up to 64M rectangles)

struct Blocking {
    int Gx, Gy;  // coarse cells along x and y
    int Bx, By;  // tiles per coarse cell along x and y
    __host__ __device__ int cells() const { return Gx * Gy; }
    __host__ __device__ int tiles_per_cell() const { return Bx * By; }
};

Blocking blocking_for(int kx, int ky);
// The same grid with coarse cells sized for inputs of about m_side
// rectangles (both inputs of a join must use one blocking).
Blocking blocking_for(int kx, int ky, int64_t m_side);
int64_t l1_chunk(int64_t n, int64_t G1);

// ---------------------------------------------------------------------------
// Partitioned input (device buffers) -- the opaque sj_part.
// Tile segments are stored in blocked tile order (see partition.hip).
// ---------------------------------------------------------------------------
struct Part {
    int device = 0;
    sj_grid grid{};
    GridDev gd{};
    Blocking bl{1, 1};
    int64_t n = 0;          // rectangles
    int64_t m = 0;          // tile entries
    int64_t m1 = 0;         // coarse-cell entries
    int64_t nb1 = 0;        // level-1 workgroups of the last call
    uint32_t* h1 = nullptr;   // [cap_h1]  level-1 histograms -> offsets (scanned in place)
    int64_t cap_h1 = 0;
    float4* e1 = nullptr;     // [cap_m1]  level-1 entries: boxes ...
    uint32_t* e1i = nullptr;  // [cap_m1]  ... and rectangle indices
    int64_t cap_m1 = 0, cap_m1i = 0;
    uint32_t* cp = nullptr;   // [G*G + 1] chunk prefix per coarse cell
    int64_t cap_cp = 0;
    uint32_t* chunk_cell = nullptr;  // [cap_chunks] coarse cell of each chunk
    int64_t cap_chunks = 0;
    uint32_t* h2 = nullptr;   // [B*B*cap_chunks + 1] level-2 histograms -> offsets
    int64_t cap_h2 = 0;
    float4* entb = nullptr;   // [cap_m]   tile entries: boxes ...
    uint32_t* enti = nullptr; // [cap_m]   ... and id words (position | start bits)
    int64_t cap_m = 0, cap_mi = 0;
    uint32_t* off = nullptr;  // [G*G*B*B + 1] segment start per blocked tile
    int64_t cap_off = 0;
    uint32_t* scan_tmp = nullptr;
    int64_t cap_scan = 0;
    DevStatus* st = nullptr;
};

// ---------------------------------------------------------------------------
// One join of a batch as the shared join kernels see it (device memory,
// 256 bytes).  Every work record of a batch (span unit, medium tile, dense
// tile) carries its join's index into an array of these; a kernel that
// pipelines its loads reads a record's descriptor one lane per word and
// takes fields with readlane where it needs them.
// ---------------------------------------------------------------------------
constexpr uint32_t kJobAxis = 1u, kJobGbda = 2u, kJobDist = 4u;
struct __attribute__((aligned(256))) Job {
    const uint32_t* offR;       // tile offsets of the two partitions
    const uint32_t* offS;
    float4* entR;               // tile slabs: boxes ...
    float4* entS;
    uint32_t* idR;              // ... and id words
    uint32_t* idS;
    unsigned long long* out;    // this join's output region: pairs (r | s << 32)
    unsigned long long* fill;   // pairs found so far = next output position
    DevStatus* st;              // this join's status
    const DevStatus* stR;       // partition status of the two inputs
    const DevStatus* stS;
    int64_t capacity;           // pairs the output region holds
    double e2;                  // distance join: keep dx*dx + dy*dy <= e2
    int32_t split_tau;          // pivots per dense unit
    uint32_t flags;             // kJobAxis | kJobGbda | kJobDist
    GridDev gd;                 // grid and blocking of the two partitions
    Blocking bl;
    int64_t C;                  // tiles of the grid
};
static_assert(sizeof(Job) == 256, "a job descriptor is 64 words");

// Implemented in partition.hip
int64_t scan_block_sums_needed(int64_t C);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t run_partition(Part& P, const float4* rects, int64_t n, int num_cus, hipStream_t s);

// Many partitions in one set of launches (a batch of joins): each launch of
// the partitioning sequence runs the workgroups of every partition, and a
// workgroup finds its partition in a prefix of the per-partition workgroup
// counts.  PartJob is one partition as the kernels see it (device memory).
struct PartJob {
    const float4* rects;
    int64_t n, ch1, nb1;
    GridDev gd;
    Blocking bl;
    uint32_t* h1;
    float4* e1;
    uint32_t* e1i;
    uint32_t* cp;
    uint32_t* chunk_cell;
    uint32_t* h2;
    float4* entb;
    uint32_t* enti;
    uint32_t* off;
    uint32_t* scan_tmp;
    int64_t cap_m1, cap_m, cap_chunks;
    DevStatus* st;
};
enum PartLaunch : int {
    kPlL1Count = 0, kPlScan1, kPlL1Direct, kPlL1Staged, kPlL2Count, kPlScan2, kPlL2Direct,
    kPlL2Staged, kPlOffsets, kPlLaunches
};
// A workgroup of a batched launch: workgroup blk belongs to the job j with
// pre[j] <= blk < pre[j + 1] (jobs without workgroups have equal prefixes)
// and is that job's workgroup wg of nwg.
struct JobSlot {
    int j;
    uint32_t wg, nwg;
};

__device__ __forceinline__ JobSlot job_slot(const uint32_t* pre, int nj) {
    const uint32_t blk = blockIdx.x;
    int lo = 0, hi = nj;  // pre[lo] <= blk < pre[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= blk) lo = mid;
        else hi = mid;
    }
    return JobSlot{lo, blk - pre[lo], pre[lo + 1] - pre[lo]};
}

struct PartBatch {
    int n = 0;                      // partitions
    PartJob* jobs = nullptr;        // device [cap]
    uint32_t* pre = nullptr;        // device [kPlLaunches][cap + 1] workgroup prefixes
    int64_t cap = 0;
    uint32_t blocks[kPlLaunches] = {};  // workgroups of every launch
    int max_g1 = 1, max_b2 = 1;     // LDS histogram sizes of the direct kernels
    std::vector<PartJob> hjobs;     // host copies of the uploaded tables: a plan
    std::vector<uint32_t> hpre;     //   equal to the last one is not uploaded again
};
// Whether the batched form serves a partition of n rectangles (prepared
// buffers): its scans must take the direct form.
bool part_batchable(const Part& P, int64_t n);
// Write the job table and workgroup prefixes (host -> device, synchronous).
hipError_t part_batch_plan(PartBatch& b, Part* const* parts, const float4* const* rects,
                           const int64_t* n, int count, int num_cus);
hipError_t run_partition_batch(const PartBatch& b, hipStream_t s);
void part_batch_free(PartBatch& b);

// ---------------------------------------------------------------------------
// Join workspace and launch helpers implemented in join.hip
// ---------------------------------------------------------------------------
struct JoinParams {
    int K;
    int64_t C;
    int split_tau;   // pivots per dense unit
    int unit_cap;    // span units are cut where their running entry count crosses a multiple of this
    int unit_tiles;  // ... and hold at most this many tiles
    int small_cap;   // tiles with at most this many entries are batched
    int med_cap;     // tiles above small_cap and up to med_cap: one per workgroup
    int block;       // threads per workgroup for the small-unit kernel
    int64_t units_bound;  // upper bound on small units
    int64_t med_bound;    // upper bound on medium tiles
    bool plain;      // one workgroup per tile, no batching, no splitting
    bool count_only;
    bool single;     // one sweep into scratch chunks + compaction (else count, scan, write)
    bool axis_model; // medium and dense tiles choose their sweeping axis (Eq. (2))
    bool gbda;       // dense tiles: the 9 GBDA class mini-joins, no duplicate test
    bool dist;       // distance join: boxes are squares anchored at their points, and
    double e2;       // a pair is kept only if dx*dx + dy*dy <= e2 (float64, no FMA)
};

struct JoinWork {
    int device = 0;
    // classification outputs
    uint4* uspan = nullptr;         // [cap_uspan] small units: (R start, NR, S start, NS)
    int64_t cap_uspan = 0;
    uint2* units = nullptr;         // [cap_units] small units: (first blocked tile, tile count)
    uint4* med = nullptr;           // [cap_med] medium-tile segments
    int64_t cap_med = 0;
    uint32_t* medt = nullptr;       // [cap_medt] blocked tile index of each medium tile
    int64_t cap_medt = 0;
    uint4* med_lpt = nullptr;       // [cap_med_lpt] medium records, largest first
    int64_t cap_med_lpt = 0;
    uint4* dense = nullptr;         // [cap_dense] (tile, base in dense buffer, nr, ns)
    uint32_t* dense_unit_prefix = nullptr;  // [cap_dense+1]
    uint32_t* dgrp = nullptr;       // [cap_dgrp] GBDA class group starts, 10 per dense tile
    uint32_t* dmj = nullptr;        // [cap_dmj] GBDA mini-join unit prefix, 10 per dense tile
    int64_t cap_dgrp = 0, cap_dmj = 0;
    int64_t cap_units = 0, cap_dense = 0, cap_prefix = 0, cap_dunits = 0;
    uint32_t* ucnt = nullptr;       // per-unit pair counts -> output offsets
    int64_t cap_ucnt = 0;
    uint32_t* scan_tmp = nullptr;   // block sums of the pair-count scan
    int64_t cap_scan = 0;
    // globally sorted dense segments
    float4* dbox = nullptr;         // [cap_dent]
    uint32_t* didf = nullptr;       // [cap_dent]
    unsigned long long* dtmp = nullptr;  // [2 * cap_dent] merge-sort scratch
    int64_t cap_dent = 0;
    // queue counters: [0] LDS units taken, [1] dense sort taken, [2] dense units taken,
    // [3] tiles written, [4] units written, [5] dense entries allocated, [6] dense units
    // single-pass pair scratch: scratch_regions() regions of sc_nch chunks
    unsigned long long* sc_buf = nullptr;  // [regions * sc_nch * scratch_chunk_pairs()]
    int64_t cap_sc_pairs = 0;
    uint32_t* sc_fills = nullptr;   // [regions * sc_nch + 1] chunk fill levels -> offsets
    int64_t cap_sc_fills = 0;
    uint32_t* sc_ctr = nullptr;     // [regions] chunks reserved per region
    unsigned long long* sc_total = nullptr;  // [scratch_totals()] pair totals
    int64_t sc_nch = 0;
    bool last_single = false;       // the last join ran in one pass
    int last_small_cap = 0, last_med_cap = 0;  // class bounds of the last join
    uint32_t* ctr = nullptr;
    DevStatus* st = nullptr;
    void* host_status = nullptr;    // pinned DevStatus mirror
    int num_cus = 0;
};

hipError_t run_join(const Part& R, const Part& S, const JoinParams& p, JoinWork& w,
                    sj_pair* out, int64_t capacity, hipStream_t s);

// Work lists shared by the joins of a batch (join.hip): the classification
// of every join appends records tagged with the join's index, one sequence
// of join launches consumes them all (capacities: sums over the joins).
struct BatchWork {
    JoinWork w;                 // lists, counters and dense buffers
    uint32_t* ujob = nullptr;   // [cap_ujob] join of each span unit
    uint32_t* mjob = nullptr;   // [cap_mjob] ... medium tile
    uint32_t* djob = nullptr;   // [cap_djob] ... dense tile
    int64_t cap_ujob = 0, cap_mjob = 0, cap_djob = 0;
    Job* jobs = nullptr;        // [cap_jobs] device descriptors
    unsigned long long* fill = nullptr;  // [cap_jobs] pairs found per join
    int64_t cap_jobs = 0, cap_fill = 0;
    // pair scratch (the batch's joins with output): w.sc_buf / sc_fills /
    // sc_ctr / sc_nch as in a single join, plus the join of every chunk
    uint32_t* sc_job = nullptr;  // [cap_sc_job]
    int64_t cap_sc_job = 0;
};
int batch_block();  // the small-tile workgroup shape of a batch
hipError_t batch_reset(BatchWork& b, int n_jobs, hipStream_t s);
hipError_t batch_classify(BatchWork& b, const Part& R, const Part& S, const JoinParams& p,
                          uint32_t jid, hipStream_t s);
// every join's classification in one launch: p (any join's parameters) gives
// the batch-wide caps, the job table the rest; pre: device [n_jobs + 1]
// prefix of classify_blocks(C) per join
hipError_t batch_classify_all(BatchWork& b, const JoinParams& p, const uint32_t* pre, int n_jobs,
                              uint32_t blocks, hipStream_t s);
int64_t classify_blocks(int64_t C);
hipError_t batch_join(BatchWork& b, int n_jobs, bool any_axis, bool pairs, int64_t units_bound,
                      int64_t med_bound, hipStream_t s);
int64_t batch_scratch_chunks(int64_t pairs, int64_t units, int64_t med, int num_cus);
// chunks reserved per scratch region by the last batch run (host copy)
hipError_t batch_scratch_used(const BatchWork& b, int64_t* max_chunks);
int64_t join_slots(const JoinParams& p, const JoinWork& w);
hipError_t join_stats(const JoinWork& w, bool single, sj_join_stats* out);
// Eq. (2) for the listed tiles (device: n x (tx, ty) int32 in, n x 4 int64
// out: divisions k, I^x, I^y, axis) on the grid of R and S.
hipError_t axis_query(const Part& R, const Part& S, const int32_t* tiles, int64_t n, int64_t* out,
                      int num_cus, hipStream_t s);
int scratch_regions();
int scratch_chunk_pairs();
int scratch_totals();

// Helpers of the API layer (sj_api.hip) used by the batch driver.
std::mutex& api_mutex();
void api_set_error(const char* msg);
sj_status api_workspace(int dev, JoinWork** w, int* num_cus);
sj_status api_resolve_grid(const sj_grid* g, sj_grid& out, GridDev& gd);
JoinParams api_join_params(const sj_grid& g, bool count_only);
sj_status api_join_prepare(JoinWork& w, JoinParams& p, int64_t C, int64_t mR, int64_t mS,
                           int64_t capacity);
hipError_t api_part_prepare(Part& P, int64_t n, int64_t need_m1, int64_t need_m);
// distance join of two partitions of anchored squares (distance.hip): pairs
// with dx*dx + dy*dy <= e2 straight into out (out NULL: count only); cand
// receives the pairs the filter passed to the distance test
sj_status api_distance_pairs(const sj_part* R, const sj_part* S, double e2, sj_pair* out,
                             int64_t capacity, int64_t* n_pairs, int64_t* cand, hipStream_t s);
// both partitions of the squares and the distance join with one status readback
sj_status api_distance_fused(const float* R, int64_t nR, const float* S, int64_t nS,
                             const sj_grid* g, sj_part** pr, sj_part** ps, double e2, sj_pair* out,
                             int64_t capacity, int64_t* n_pairs, int64_t* cand, hipStream_t s);
sj_status api_distance_tune(const sj_part* R, const sj_part* S, double e2, sj_pair* out,
                            int64_t capacity, int32_t reps, sj_tuning* best, hipStream_t s);
bool prof_pause(bool pause);  // prof.hip: suspend event brackets (graph capture)

}  // namespace sj
