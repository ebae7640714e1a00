// Joining phase of the PBSM join (Sec. 3.4 steps 5-6) on gfx950.
//
// Per tile T the join sorts R_T and S_T by lower x-endpoint and runs the
// forward-scan plane sweep of Algorithm 1, keeping a pair only when the
// reference point of Eq. (1) lies in T.  Algorithm 1 is run in its
// per-pivot form: with both lists sorted by x_l (ties broken arbitrarily),
// the merge of Algorithm 1 makes
//   * each r the pivot of a forward scan over the s with  r.x_l < s.x_l <= r.x_u,
//   * each s the pivot of a forward scan over the r with  s.x_l <= r.x_l <= s.x_u,
// so every pivot's scan can start at its own binary-searched position and
// all pivots of all tiles run independently (one lane per pivot).  Every
// scanned candidate gets the closed y-interval test and the reference-point
// test; the union over pivots is exactly Algorithm 1's output for the tile.
//
// Work units
//   small:   tiles with both lists non-empty and at most `small_cap` entries
//            are batched into LDS units of about `unit_cap` entries; a unit
//            is staged, sorted per tile segment and swept in LDS, either by
//            one wavefront (64-thread schedule: wave-level fences only, the
//            next unit staged while the current one is swept) or by one
//            workgroup of 128 / 256 / 512 threads.
//   medium:  tiles up to `med_cap` entries, one per workgroup, same code with
//            a larger LDS slab (large lists bitonic-sorted in LDS).
//   dense:   larger tiles are sorted into a global buffer and swept by units
//            of at most `split_tau` pivots, so one tile is shared by many CUs.
//   plain:   (baseline) one workgroup per tile for every tile, LDS up to
//            1024 entries, larger tiles dense without splitting.
//
// Output without a shared counter (a device-wide atomic on one address
// serialises at roughly 80 M/s on this GPU).  Every wave stages its pairs in
// LDS (ballot + masked popcount give the slots) and flushes them:
//   single pass (default): into 512-pair chunks of a scratch buffer that the
//            wave reserves from one of 32 spread counters; chunk fill levels
//            are scanned and the chunks compacted into the caller's buffer.
//            Exact totals are kept even if the scratch runs out, and the call
//            then joins again in two passes.
//   two passes: a counting pass writes each unit's pair count to its own
//            slot, an exclusive scan gives every unit its output region and
//            the writing pass fills it.  Count-only joins stop after the scan.
#include <algorithm>

#include "sj_internal.hpp"
#include "sj_prof.hpp"

namespace sj {

hipError_t scan_u32(uint32_t* data, int64_t len, uint32_t* bs, unsigned long long* total,
                    DevStatus* st, hipStream_t s);

namespace {

enum Ctr : int {
    kTilesWritten = 0,
    kUnitsWritten = 1,
    kMedCount = 2,
    kDenseCount = 3,
    kDenseEntries = 4,
    kDenseUnits = 5,
    kSmallEntries = 6,  // statistics: entries of the small and medium tiles
    kMedEntries = 7,
    kAxisTiles = 8,     // statistics: tiles that evaluated the sweeping-axis model ...
    kAxisY = 9,         // ... and those of them swept along y
    kMedTaken = 10,     // single join: medium tiles claimed (counting or single pass) ...
    kMedTaken2 = 11,    // ... and by the writing pass
    kDenseTaken = 12,   // single join: dense units claimed (counting or single pass) ...
    kDenseTaken2 = 13,  // ... and by the writing pass
    kNumCtr = 14
};
static_assert(kNumCtr <= 16, "the join's counter array holds 16 words");
// k_classify adds to each of these pairs of counters with one 64-bit atomic
static_assert(kUnitsWritten == kTilesWritten + 1 && kTilesWritten % 2 == 0, "tile/unit pair");
static_assert(kMedEntries == kSmallEntries + 1 && kSmallEntries % 2 == 0, "statistics pair");

constexpr int kWaveBuf = 256;        // staged pairs per wave (>= 64 lanes x kCand)
constexpr int kUnitWaveBuf = 128;    // LDS units emit one candidate per lane and call
constexpr int kSpanWaveBuf = 96;     // ... span units (LDS holds their tile tables)
constexpr int kSpanTQ = 2;           // tile-table words per thread: span units of
                                     // up to kSpanTQ * NT - 1 tiles
constexpr int kMedNT = 512;          // workgroup of the medium-tile kernel
constexpr int kBatchBlock = 256;     // small-tile workgroup of a batch of joins
constexpr int kMedE = 2048;          // LDS entries of a medium tile
constexpr int kBatchMedNT = 256;     // medium tiles of a batch: the half-size slab, whose
constexpr int kBatchMedE = 1024;     // ... 4 workgroups per CU beat the full slab's 2
constexpr int kDenseSortMax = 8192;  // entries sorted in LDS by the dense sort
constexpr int kDenseSortNT = 1024;
constexpr int kDenseNT = 256;

struct Args {
    const uint32_t* offR;
    const uint32_t* offS;
    float4* entR;     // tile slabs: boxes; the counting pass writes each slab back sorted
    float4* entS;
    uint32_t* idR;    // ... and id words (position | start bits)
    uint32_t* idS;
    int64_t C;        // blocked tiles
    int small_cap;    // small tiles: nr + ns <= small_cap
    int unit_cap;     // entries per small unit (target)
    int med_cap;      // medium tiles: small_cap < nr + ns <= med_cap
    int split_tau;    // pivots per dense unit
    int plain;
    int unit_tiles;   // tiles per small unit (at most)
    uint4* uspan;     // small units: (R start, NR, S start, NS) of the unit's entry spans
    uint2* units;     // small units: (first blocked tile, tile count)
    uint4* med;       // medium tiles: (R start, nr, S start, ns)
    uint4* med_lpt;   // single join: the medium records by decreasing entry count
                      // (k_med_order), claimed one at a time by the workgroups
    uint4* dense;     // dense tiles: (tile, base in dense buffer, nr, ns)
    uint32_t* dprefix;  // dense units before each dense tile
    int64_t cap_units, cap_med, cap_dense, cap_dent, cap_dunits;
    float4* dbox;
    uint32_t* didf;
    unsigned long long* dtmp;
    uint32_t* ucnt;   // per-unit pair counts, then (scanned) output offsets
    int64_t base_med;    // slot of medium tile m: base_med + m
    int64_t base_dense;  // slot of dense unit u: base_dense + u
    uint32_t* ctr;
    DevStatus* st;
    const DevStatus* stR;  // partition-time status of the two inputs
    const DevStatus* stS;
    unsigned long long* out;  // pairs as (r | s << 32)
    int64_t capacity;
    int writeback;            // counting pass leaves the slabs sorted for a second pass
    unsigned long long* sc_buf;   // single-pass scratch: kRegions x sc_nch chunks of kChunkP
    uint32_t* sc_fills;           // fill level of every chunk, then their exclusive prefix
    uint32_t* sc_ctr;             // [kRegions] chunks reserved per region
    unsigned long long* sc_total; // [kTotals] hit totals
    int64_t sc_nch;               // chunks per region
    int cls;                      // work class of the launch (pair totals per class)
    uint32_t* medt;               // blocked tile index of each medium tile (axis model)
    int axis_model;               // medium / dense tiles choose their sweeping axis
    GridDev gd;                   // grid and blocking of the two partitions
    Blocking bl;
    int gbda;                     // dense tiles: the 9 class-class mini-joins, no duplicate test
    uint32_t* dgrp;               // [cap_dense * 10] class group starts of each dense tile (R, S)
    uint32_t* dmj;                // [cap_dense * 10] units before each mini-join of a dense tile
    int dist;                     // distance join (boxes: squares anchored at their points)
    double e2;                    // ... keep a pair only if dx*dx + dy*dy <= e2
    // batch of joins: the lists hold the records of many joins, each tagged
    // with its join's index into jobs (slabs, output region, flags); the
    // fields above that describe one join are then those of jid (k_classify)
    int batch;
    uint32_t jid;
    const Job* jobs;
    uint32_t* ujob;               // join of each span unit
    uint32_t* mjob;               // ... medium tile
    uint32_t* djob;               // ... dense tile
    uint32_t* sc_job;             // join of each scratch chunk (single pass)
};

// One join's tile offsets and slabs: from the arguments (single join) or
// from the descriptor of a record's join (batch).
struct Src {
    const uint32_t* offR;
    const uint32_t* offS;
    float4* entR;
    float4* entS;
    uint32_t* idR;
    uint32_t* idS;
};

__device__ __forceinline__ Src src_of(const Args& a) {
    return Src{a.offR, a.offS, a.entR, a.entS, a.idR, a.idS};
}
__device__ __forceinline__ Src src_of(const Job& j) {
    return Src{j.offR, j.offS, j.entR, j.entS, j.idR, j.idS};
}

// Per-join schedule fields of a record: its job's (batch) or the arguments'.
struct JobFlags {
    int dist, gbda, plain, split_tau;
    double e2;
};
__device__ __forceinline__ JobFlags flags_of(const Args& a, uint32_t job) {
    if (!a.batch) return JobFlags{a.dist, a.gbda, a.plain, a.split_tau, a.e2};
    const Job& j = a.jobs[job];
    return JobFlags{(j.flags & kJobDist) ? 1 : 0, (j.flags & kJobGbda) ? 1 : 0, 0, j.split_tau, j.e2};
}

// GBDA classes of an entry in its tile, from the start bits of Eq. (1):
// A = both projections begin in the tile, B = only x, C = only y, D = neither.
// The 9 class pairs (R class, S class) that can hold a pair whose reference
// point lies in the tile: some rectangle begins in it along x, some along y.
__device__ __forceinline__ uint32_t gbda_class(uint32_t idw) {
    return ((idw & kBx) ? 0u : 2u) + ((idw & kBy) ? 0u : 1u);
}
__constant__ uint8_t kMiniJoin[9][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {1, 0},
                                         {1, 2}, {2, 0}, {2, 1}, {3, 0}};

// A medium or dense tile record carries its sweeping axis in bit 31 of one
// field (set by k_axis): medium (R start, nr | axis, S start, ns), dense
// (tile | axis, base, nr, ns).  Counts and blocked tile indices stay below
// 2^31.
constexpr uint32_t kAxisBit = 0x80000000u;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ void lds_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup"); }

// The i-th work unit of workgroup g of G: round-robin over stripes of S
// consecutive units.  S = 1 for a single join; a batch uses longer stripes,
// since consecutive units mostly belong to one join and a wave then rarely
// changes joins.  Increasing in i.
__device__ __forceinline__ uint32_t unit_of(uint32_t i, uint32_t g, uint32_t G, uint32_t S) {
    return ((i / S) * G + g) * S + i % S;
}
constexpr uint32_t kSpanStripe = 16;  // batch stripes: span units
constexpr uint32_t kMedStripe = 2;    // ... medium tiles
constexpr uint32_t kDenseStripe = 1;  // ... dense units

// ---------------------------------------------------------------------------
// Pair sink.  Three modes:
//   kCount   per-lane counters, reduced into the unit's slot of the count
//            array (first pass of the two-pass output; count-only joins).
//   kWrite   second pass: per-wave LDS staging flushed into the unit's own
//            output region (exclusive prefix of the counts), space reserved
//            with an LDS atomic.
//   kSingle  one pass: per-wave LDS staging flushed into scratch chunks of
//            kChunkP pairs that the wave reserves from one of kRegions
//            counters (a spread of addresses: a single device-wide counter
//            serialises); chunk fill levels are compacted into the caller's
//            buffer afterwards.  Every hit is counted even if the scratch
//            runs out, so the exact count is always known.
//   kAppend  batch of joins, count only: per-lane counters, added to the
//            fill counter of the join with one atomic per wave whenever the
//            wave moves on to a unit of another join, and at the end.
// In a batch of joins, kSingle keeps one open scratch chunk per wave for the
// join of its current unit: the staged pairs are flushed and the chunk is
// closed when the wave moves on to a unit of another join, so a chunk holds
// the pairs of one join (tagged in sc_job); the compaction places every
// chunk into its join's output region with one atomic per chunk.
// BLOCK: the unit is processed by a whole workgroup (end() has barriers);
// otherwise by one wavefront.
// ---------------------------------------------------------------------------
enum Mode : int { kCount = 0, kWrite = 1, kSingle = 2, kAppend = 3 };
constexpr int kRegions = 32;    // scratch regions / reservation counters
constexpr int kChunkP = 512;    // pairs per scratch chunk
constexpr int kTotals = 64;     // spread counters of the per-wave hit totals
constexpr int kTotalsPer = 16;  // ... per work class (small, medium, dense)

// ROTATE: every new chunk from the next region (else a wave keeps its
// region); the single-join small-tile kernel keeps its region, since its
// many waves of modest output fill the regions evenly and the kernel's
// register allocation is tighter without the rotation.
template <int MODE, bool BLOCK, bool ROTATE = true>
struct Sink {
    unsigned long long* buf;  // this wave's LDS staging buffer
    uint32_t* s_acc;          // LDS word: pair count (kCount) or fill counter (kWrite)
    uint32_t bufcap;          // staging capacity
    uint32_t n;               // staged pairs (wave-uniform)
    uint32_t cnt;             // this lane's pair count (kCount)
    unsigned long long base;  // first output slot of the unit (kWrite)
    uint32_t region, chunk, cfill;  // current scratch chunk (kSingle)
    bool have, ok;
    unsigned long long total;       // hits seen by this wave (kSingle)
    uint32_t cand;                  // this lane's filter pairs (distance join; not kWrite)
    uint32_t cjob;                  // batch: the join of the current unit

    __device__ void init(uint32_t wave_gid) {
        n = 0;
        cnt = 0;
        base = 0;
        region = wave_gid % kRegions;
        chunk = 0;
        cfill = 0;
        have = false;
        ok = true;
        total = 0;
        cand = 0;
        cjob = 0;
    }

    // Batch, every lane of the wave: the join of the following units.  On a
    // change, the pairs of the previous join leave the wave: kAppend adds
    // its count to the join's fill counter, kSingle flushes the staged pairs
    // and closes the open chunk.
    __device__ void set_job(const Args& a, uint32_t j) {
        if (j == cjob) return;
        if (MODE == kAppend) {
            drain_count(a);
        } else if (MODE == kSingle) {
            if (n) flush(a);
            if (have && lane_id() == 0) a.sc_fills[(size_t)region * a.sc_nch + chunk] = cfill;
            have = false;
        }
        cjob = j;
    }

    // kAppend: the wave's count of the current join into its fill counter
    __device__ void drain_count(const Args& a) {
        uint32_t v = cnt;
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
        if (lane_id() == 0 && v) atomicAdd(a.jobs[cjob].fill, (unsigned long long)v);
        total += v;
        cnt = 0;
    }

    __device__ void begin(const Args& a, int64_t slot) {
        if (MODE != kAppend) cnt = 0;
        if (MODE != kSingle) n = 0;
        if (MODE == kWrite) {
            base = a.ucnt[slot];
            cfill = 0;
        }
        if ((MODE == kCount || MODE == kWrite) && BLOCK && threadIdx.x == 0) *s_acc = 0u;
    }

    __device__ void flush(const Args& a) {
        lds_fence();
        if (MODE == kWrite) {
            uint32_t b = cfill;  // one wave per unit: a register counter
            if (BLOCK) {
                if (lane_id() == 0) b = atomicAdd(s_acc, n);
                b = __shfl(b, 0, kWave);
            }
            cfill += n;
            for (uint32_t q = lane_id(); q < n; q += kWave) {
                const unsigned long long idx = base + b + q;
                if (idx < (unsigned long long)a.capacity) a.out[idx] = buf[q];
            }
        } else if (MODE == kSingle) {
            uint32_t done = 0;
            while (ok && done < n) {
                if (!have || cfill == (uint32_t)kChunkP) {
                    if (have && lane_id() == 0)
                        a.sc_fills[(size_t)region * a.sc_nch + chunk] = (uint32_t)kChunkP;
                    // each new chunk from the next region in turn: waves differ
                    // widely in output, and a wave that kept one region could
                    // fill it while others have room
                    if (ROTATE && have) region = (region + 1u) % (uint32_t)kRegions;
                    uint32_t k = 0;
                    if (lane_id() == 0) {
                        k = atomicAdd(&a.sc_ctr[region], 1u);
                        if (a.batch && (int64_t)k < a.sc_nch) a.sc_job[(size_t)region * a.sc_nch + k] = cjob;
                    }
                    k = __shfl(k, 0, kWave);
                    have = true;
                    chunk = k;
                    cfill = 0;
                    if ((int64_t)k >= a.sc_nch) {
                        ok = false;
                        have = false;
                        if (lane_id() == 0) atomicOr(&a.st->flags, kStatScratch);
                        break;
                    }
                }
                const uint32_t take = min(n - done, (uint32_t)kChunkP - cfill);
                unsigned long long* dst =
                    a.sc_buf + ((size_t)region * a.sc_nch + chunk) * kChunkP + cfill;
                for (uint32_t q = lane_id(); q < take; q += kWave) dst[q] = buf[done + q];
                cfill += take;
                done += take;
            }
        }
        lds_fence();
        n = 0;
    }

    // Emit up to N pairs per lane (hit k -> (r[k], s[k])).  Every lane calls
    // it; one flush check per call.
    template <int N>
    __device__ __forceinline__ void emit(const Args& a, const bool (&hit)[N], const uint32_t (&r)[N],
                                         const uint32_t (&s)[N]) {
        if (MODE == kCount || MODE == kAppend) {
#pragma unroll
            for (int k = 0; k < N; ++k) cnt += hit[k] ? 1u : 0u;
            return;
        }
        unsigned long long m[N];
        uint32_t nh = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            m[k] = __ballot(hit[k]);
            nh += (uint32_t)__popcll(m[k]);
        }
        if (nh == 0u) return;
        if (MODE == kSingle) total += nh;
        if (n + nh > bufcap) flush(a);
        uint32_t at = n;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (hit[k]) buf[at + lanes_below(m[k])] = (unsigned long long)r[k] | ((unsigned long long)s[k] << 32);
            at += (uint32_t)__popcll(m[k]);
        }
        n += nh;
    }

    __device__ void end(const Args& a, int64_t slot) {
        if (MODE == kWrite) {
            if (n) flush(a);
        } else if (MODE == kCount) {
            uint32_t v = cnt;
            for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
            if (BLOCK) {
                if (lane_id() == 0 && v) atomicAdd(s_acc, v);
            } else if (lane_id() == 0) {
                a.ucnt[slot] = v;
            }
        }
        if (BLOCK) {
            __syncthreads();
            if (MODE == kCount && threadIdx.x == 0) a.ucnt[slot] = *s_acc;
            __syncthreads();
        }
    }

    // kernel end, every lane: the last staged pairs and the wave's totals
    __device__ void finish(const Args& a, uint32_t wave_gid) {
        if (MODE != kWrite && a.dist) {
            unsigned long long v = cand;
            for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
            if (lane_id() == 0 && v) atomicAdd(&a.st->n_cand, v);
        }
        if (MODE != kSingle && MODE != kAppend) return;
        if (MODE == kAppend) drain_count(a);
        if (n) flush(a);
        if (lane_id() == 0) {
            if (MODE == kSingle && have && ok) a.sc_fills[(size_t)region * a.sc_nch + chunk] = cfill;
            if (total) atomicAdd(&a.sc_total[a.cls * kTotalsPer + wave_gid % kTotalsPer], total);
        }
    }
};

// Reference-point test of Eq. (1) on the start bits of the two entries.
__device__ __forceinline__ bool ref_point_here(uint32_t ida, uint32_t idb) {
    return ((ida | idb) & (kBx | kBy)) == (kBx | kBy);
}

// Distance join (Sec. 1): the squares are anchored at their points, so the
// lower corners (x_l, y_l) are the input points themselves.  The refinement
// of a filter pair, in float64 with every operation rounded once (no fused
// multiply-add); symmetric in x and y and in the two points, so it holds for
// boxes taken with x and y exchanged.
__device__ __forceinline__ bool within_eps(const float4& p, const float4& q, double e2) {
    const double dx = __dsub_rn((double)p.x, (double)q.x);
    const double dy = __dsub_rn((double)p.y, (double)q.y);
    return __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)) <= e2;
}

// First index in [lo, hi) whose x_l is > v (upper) or >= v (lower).
template <class F>
__device__ __forceinline__ int search_x(const F& xl, int lo, int hi, float v, bool upper) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const float x = xl(mid);
        const bool go_right = upper ? (x <= v) : (x < v);
        if (go_right) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// The sweep over one batch of pivots [p_begin, p_end).  Acc provides the
// candidate entries of the batch's storage (box(j) = (x_l, y_l, x_u, y_u),
// id(j)) and, for a pivot p, its setup (own rectangle; start and end of its
// scan in the other list).  Each iteration examines up to kCand consecutive
// candidates per lane, so their loads are in flight together.  Idle lanes
// claim the next pivots from a workgroup-wide LDS counter (*next, zero on
// entry; one atomic per wave and round), so scans of very different lengths
// spread over all lanes of the workgroup.
// ---------------------------------------------------------------------------
constexpr int kCand = 4;
constexpr int kChunkC = 8;  // consecutive candidates per lane and round (LDS units)

template <int MODE, bool BLOCK, bool REF = true, class Acc>
__device__ void sweep_pivots(const Args& a, const Acc& acc, int p_begin, int p_end, uint32_t* next,
                             Sink<MODE, BLOCK>& sk, bool dist, double e2) {
    bool scanning = false, exhausted = false, isR = false;
    int j = 0, jend = 0;
    float pxl = 0.f, pxu = 0.f, pyl = 0.f, pyu = 0.f;
    uint32_t pid = 0;
    const int lane = lane_id();
    while (true) {
        // idle lanes claim pivots and find where their scans start
        const bool need = !scanning && !exhausted;
        const unsigned long long m = __ballot(need);
        if (m) {
            const int leader = __builtin_ctzll(m);
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(next, (uint32_t)__popcll(m));
            base = __shfl(base, leader, kWave);
            if (need) {
                const int p = p_begin + (int)(base + lanes_below(m));
                if (p < p_end) {
                    acc.setup(p, isR, j, jend, pxl, pxu, pyl, pyu, pid);
                    scanning = j < jend;
                } else {
                    exhausted = true;
                }
            }
        }
        // every scanning lane tests its next kCand candidates
        bool hit[kCand];
        uint32_t er[kCand], es[kCand];
#pragma unroll
        for (int k = 0; k < kCand; ++k) {
            hit[k] = false;
            er[k] = 0;
            es[k] = 0;
        }
        if (scanning) {
            float4 c[kCand];
            uint32_t qid[kCand];
#pragma unroll
            for (int k = 0; k < kCand; ++k) {
                const int idx = min(j + k, jend - 1);
                c[k] = acc.box(idx);
                qid[k] = acc.id(idx);
            }
            bool go = true;
            int used = 0;
            const uint32_t me = pid & kIdMask;
#pragma unroll
            for (int k = 0; k < kCand; ++k) {
                go = go && (j + k < jend) && (c[k].x <= pxu);
                const bool f = go && (pyl <= c[k].w) && (c[k].y <= pyu) &&
                               (!REF || ref_point_here(pid, qid[k]));
                hit[k] = f && (!dist || within_eps(make_float4(pxl, pyl, pxu, pyu), c[k], e2));
                if (MODE != kWrite) sk.cand += (dist && f) ? 1u : 0u;
                used += go ? 1 : 0;
                const uint32_t other = qid[k] & kIdMask;
                er[k] = isR ? me : other;
                es[k] = isR ? other : me;
            }
            j += used;
            scanning = go && j < jend;  // a candidate beyond x_u ends the scan
        }
        sk.template emit<kCand>(a, hit, er, es);
        if (__ballot(scanning || !exhausted) == 0ull) break;
    }
}

// ---------------------------------------------------------------------------
// LDS unit: a batch of tiles staged, sorted and swept in LDS.
// ---------------------------------------------------------------------------
struct LdsLayout {
    unsigned long long* wbuf;  // [nwaves * kUnitWaveBuf]
    uint32_t* acc;             // [0] sink accumulator, [1] next pivot to claim
    uint32_t* rg;  // [tc+1] global start of each tile's R segment
    uint32_t* rl;  // [tc+1] local start (prefix) of each tile's R segment
    uint32_t* sg;
    uint32_t* sl;
    uint32_t* key;  // [E] unsorted order keys
    uint16_t* tk;   // [E] local tile of each entry
    float4* bx;     // [E] sorted boxes (R part first, then S part)
    uint32_t* id;   // [E] sorted id words
};

__host__ __device__ inline size_t lds_bytes(int nt, int E, int tc) {
    size_t b = 0;
    b += (size_t)(nt / kWave) * kUnitWaveBuf * 8;
    b += 16;
    b += (size_t)4 * (tc + 1) * 4;
    b = (b + 15) / 16 * 16;
    b += (size_t)E * 16;                  // boxes
    b += (size_t)E * 4;                   // ids
    b += (size_t)(E + 8) * 4;             // keys (+8: 128-bit loads past the end)
    b += (size_t)((E * 2 + 15) / 16) * 16;  // tile indices
    return b;
}

__device__ inline LdsLayout carve(unsigned char* p, int nt, int E, int tc) {
    LdsLayout L;
    L.wbuf = (unsigned long long*)p;
    p += (size_t)(nt / kWave) * kUnitWaveBuf * 8;
    L.acc = (uint32_t*)p; p += 16;
    L.rg = (uint32_t*)p; p += (size_t)(tc + 1) * 4;
    L.rl = (uint32_t*)p; p += (size_t)(tc + 1) * 4;
    L.sg = (uint32_t*)p; p += (size_t)(tc + 1) * 4;
    L.sl = (uint32_t*)p; p += (size_t)(tc + 1) * 4;
    {
        const size_t used = (size_t)((nt / kWave) * kUnitWaveBuf * 8 + 16 + 4 * (tc + 1) * 4);
        p += ((used + 15) / 16 * 16) - used;  // 16-byte alignment of the boxes
    }
    L.bx = (float4*)p; p += (size_t)E * 16;
    L.id = (uint32_t*)p; p += (size_t)E * 4;
    L.key = (uint32_t*)p; p += (size_t)(E + 8) * 4;
    L.tk = (uint16_t*)p;
    return L;
}

// tile-table capacity of an LDS unit of E entries (every tile has >= 2)
__host__ __device__ constexpr int tc_for(int E, bool batched) { return batched ? E / 2 + 2 : 2; }

template <int MODE>
__device__ inline Sink<MODE, true> make_sink(const LdsLayout& L) {
    Sink<MODE, true> sk;
    sk.buf = L.wbuf + (threadIdx.x / kWave) * kUnitWaveBuf;
    sk.s_acc = L.acc;
    sk.bufcap = kUnitWaveBuf;
    sk.init(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
    return sk;
}

// Rank of (key[e], e) among the entries [lo, hi): the sorted position of e
// within its segment (ties broken by position).  Eight keys per two 128-bit
// LDS loads; key[] is 16-byte aligned and readable 8 entries past the end.
// A position j counts if key[j] < key[e], or key[j] == key[e] and j < e,
// i.e. if key[j] < key[e] + (j < e) (finite order keys stay below 2^32 - 1).
// Only the first and last groups of eight need the segment bounds.
__device__ __forceinline__ int seg_rank(const uint32_t* key, int lo, int hi, int e) {
    const uint32_t my = key[e];
    const uint4* k4 = (const uint4*)key;
    int rank = 0;
    int jb = lo & ~3;
    auto group = [&](int j0, bool bounded) {
        const uint4 A = k4[j0 >> 2], B = k4[(j0 >> 2) + 1];
        const uint32_t kk[8] = {A.x, A.y, A.z, A.w, B.x, B.y, B.z, B.w};
        const int d = e - j0;  // positions u < d precede e
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const bool c = kk[u] < my + (u < d ? 1u : 0u);
            rank += (bounded ? (c && j0 + u >= lo && j0 + u < hi) : c) ? 1 : 0;
        }
    };
    group(jb, true);  // head: may start before lo and end after hi
    for (jb += 8; jb + 8 <= hi; jb += 8) group(jb, false);
    if (jb < hi) group(jb, true);
    return rank;
}

// Stage tiles [0, c) -- segment bounds from tile_of(k, k / NT) -- in LDS, sort every
// tile segment by x_l and sweep.  Every thread of the workgroup calls it.
// prefetch() runs once the unit's entries have arrived: the caller issues
// the loads of its next unit there, so they overlap this unit's sort and
// sweep.
//
// swap: the unit is one tile swept along y (sweeping-axis model): every box
// is taken with x and y exchanged, so the sort and the sweep below run along
// y; the write-back exchanges them again.  The duplicate test of Eq. (1) is
// symmetric in x and y, so the pairs reported do not change.
template <int NT, int Q, int TC, int MODE, class TileOf, class Prefetch>
__device__ __forceinline__ void run_lds_unit(const Args& a, const Src& src, bool dist, double e2,
                                             const LdsLayout& L, int c, const TileOf& tile_of,
                                             const Prefetch& prefetch, Sink<MODE, true>& sk,
                                             bool swap = false) {
    constexpr int E = NT * Q;
    const int tid = threadIdx.x;
    if (c > TC) {  // more tiles than the LDS tile table holds: cannot happen
        if (tid == 0) atomicOr(&a.st->flags, kStatInternal);
        return;
    }
    __shared__ uint32_t s_tot[2];
    __shared__ uint32_t s_wsum[2][NT / kWave + 1];
    __shared__ uint32_t s_wq[Q][NT / kWave];  // range-length sums per round and wave
    // 1. tile table with local prefixes (chunks of NT tiles; unrolled, so
    //    the chunk index is a constant for tile_of)
    uint32_t carry_r = 0, carry_s = 0;
#pragma unroll
    for (int jc = 0; jc < (TC + NT - 1) / NT; ++jc) {
        const int k0 = jc * NT;
        if (k0 >= c) break;
        const int k = k0 + tid;
        uint32_t nr = 0, ns = 0, r0 = 0, s0 = 0;
        if (k < c) {
            const uint4 ti = tile_of(k, jc);  // (R start, nr, S start, ns)
            r0 = ti.x;
            nr = ti.y;
            s0 = ti.z;
            ns = ti.w;
        }
        const int lane = lane_id(), w = tid / kWave;
        uint32_t ir = nr, is = ns;
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t tr = __shfl_up(ir, d, kWave), ts = __shfl_up(is, d, kWave);
            if (lane >= d) {
                ir += tr;
                is += ts;
            }
        }
        if (lane == kWave - 1) {
            s_wsum[0][w] = ir;
            s_wsum[1][w] = is;
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t ar = 0, as = 0;
            for (int q = 0; q < NT / kWave; ++q) {
                const uint32_t vr = s_wsum[0][q], vs = s_wsum[1][q];
                s_wsum[0][q] = ar;
                s_wsum[1][q] = as;
                ar += vr;
                as += vs;
            }
            s_tot[0] = ar;
            s_tot[1] = as;
        }
        __syncthreads();
        if (k < c) {
            L.rg[k] = r0;
            L.sg[k] = s0;
            L.rl[k] = carry_r + s_wsum[0][w] + ir - nr;
            L.sl[k] = carry_s + s_wsum[1][w] + is - ns;
        }
        carry_r += s_tot[0];
        carry_s += s_tot[1];
        __syncthreads();
    }
    const int NR = (int)carry_r, NS = (int)carry_s, NE = NR + NS;
    if (tid == 0) {
        L.rl[c] = NR;
        L.sl[c] = NS;
        L.acc[1] = 0u;  // pivot counter of the sweep
    }
    if (NE > E) {  // cannot happen for units built with unit_cap + small_cap <= E
        if (tid == 0) atomicOr(&a.st->flags, kStatInternal);
        __syncthreads();
        return;
    }
    // 1b. local tile of every entry: mark each segment's first entry with its
    //     tile (R part: k, S part: c + k, so the values rise along the array),
    //     then an inclusive max-scan fills the segments
#pragma unroll
    for (int q = 0; q < Q; ++q) L.tk[tid * Q + q] = 0;
    __syncthreads();
    for (int k = tid; k < c; k += NT) {
        if (L.rl[k + 1] > L.rl[k]) L.tk[L.rl[k]] = (uint16_t)k;
        if (L.sl[k + 1] > L.sl[k]) L.tk[NR + L.sl[k]] = (uint16_t)(c + k);
    }
    __syncthreads();
    {
        uint32_t v[Q];
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const uint32_t x = L.tk[tid * Q + q];
            run = x > run ? x : run;
            v[q] = run;
        }
        const int lane = lane_id(), w = tid / kWave;
        uint32_t inc = run;
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t t = __shfl_up(inc, d, kWave);
            if (lane >= d) inc = t > inc ? t : inc;
        }
        if (lane == kWave - 1) s_wsum[0][w] = inc;
        uint32_t ex = __shfl_up(inc, 1, kWave);
        if (lane == 0) ex = 0;
        __syncthreads();
        for (int q = 0; q < w; ++q) ex = s_wsum[0][q] > ex ? s_wsum[0][q] : ex;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = tid * Q + q;
            const uint32_t t = v[q] > ex ? v[q] : ex;
            if (i < NE) L.tk[i] = (uint16_t)(i < NR ? t : t - (uint32_t)c);
        }
    }
    __syncthreads();
    // 2. load entries (coalesced within each tile segment).  All loads are
    //    issued before the first LDS store that uses one, so the Q gathers
    //    are in flight together (an LDS store between them would order the
    //    next address computation after the previous load's return).
    float4 pb[Q];
    uint32_t pi[Q], pg[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e = tid + q * NT;
        pg[q] = 0xFFFFFFFFu;
        if (e < NE) {
            const bool isR = e < NR;
            const int k = L.tk[e];
            const uint32_t g = isR ? L.rg[k] + (uint32_t)e - L.rl[k]
                                   : L.sg[k] + (uint32_t)(e - NR) - L.sl[k];
            pb[q] = (isR ? src.entR : src.entS)[g];
            pi[q] = (isR ? src.idR : src.idS)[g];
            pg[q] = g;
        }
    }
    if (swap) {
#pragma unroll
        for (int q = 0; q < Q; ++q) pb[q] = make_float4(pb[q].y, pb[q].x, pb[q].w, pb[q].z);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e = tid + q * NT;
        if (e < NE) {
            if (MODE == kWrite) {  // the counting pass left every slab sorted
                L.bx[e] = make_float4(pb[q].x, pb[q].y, pb[q].z, pb[q].w);
                L.id[e] = pi[q];
            } else {
                L.key[e] = order_key(pb[q].x);
            }
        }
    }
    prefetch();
    __syncthreads();
    if (MODE != kWrite) {
        // 3. sort within each tile segment, write the sorted payload to LDS
        //    and back to the slab in global memory.  Batched small tiles:
        //    rank sort (each entry counts the smaller keys of its segment).
        //    One large tile (TC == 2): a rank sort is quadratic, so both lists
        //    are bitonic-sorted as (key, position) words in the box area,
        //    and the sorted positions are inverted into ranks.
        int pos[Q];
        if (TC == 2 && (NR > 64 || NS > 64)) {
            unsigned long long* kw = (unsigned long long*)L.bx;  // 2E words fit E boxes
            int PR = 1, PS = 1;
            while (PR < NR) PR <<= 1;
            while (PS < NS) PS <<= 1;
            for (int i = tid; i < PR + PS; i += NT) {
                const bool r = i < PR;
                const int j = r ? i : i - PR;
                const int n = r ? NR : NS;
                kw[i] = j < n ? ((unsigned long long)L.key[r ? j : NR + j] << 32) | (uint32_t)j
                              : ~0ull;
            }
            __syncthreads();
            // both networks at once: pair index i < PR/2 belongs to R's
            for (int size = 2; size <= (PR > PS ? PR : PS); size <<= 1) {
                for (int stride = size >> 1; stride > 0; stride >>= 1) {
                    for (int i = tid; i < (PR + PS) / 2; i += NT) {
                        const bool r = i < PR / 2;
                        const int P = r ? PR : PS;
                        if (size > P) continue;
                        const int ii = r ? i : i - PR / 2;
                        const int lo = 2 * ii - (ii & (stride - 1));
                        const int hi = lo + stride;
                        const bool up = (lo & size) == 0;
                        unsigned long long* w = r ? kw : kw + PR;
                        const unsigned long long x = w[lo], y = w[hi];
                        if ((x > y) == up) {
                            w[lo] = y;
                            w[hi] = x;
                        }
                    }
                    __syncthreads();
                }
            }
            for (int i = tid; i < NE; i += NT) {  // rank of each entry (keys are no longer needed)
                const bool r = i < NR;
                const uint32_t src = (uint32_t)kw[r ? i : PR + (i - NR)];
                L.key[r ? src : NR + src] = (uint32_t)i;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int e = tid + q * NT;
                pos[q] = e < NE ? (int)L.key[e] : -1;
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int e = tid + q * NT;
                pos[q] = -1;
                if (e < NE) {
                    const bool isR = e < NR;
                    const int k = L.tk[e];
                    const int lo = isR ? (int)L.rl[k] : NR + (int)L.sl[k];
                    const int hi = isR ? (int)L.rl[k + 1] : NR + (int)L.sl[k + 1];
                    pos[q] = lo + seg_rank(L.key, lo, hi, e);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (pos[q] >= 0) {
                L.bx[pos[q]] = make_float4(pb[q].x, pb[q].y, pb[q].z, pb[q].w);
                L.id[pos[q]] = pi[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = tid + q * NT;
            if (MODE == kCount && a.writeback && e < NE) {
                float4 b = L.bx[e];
                if (swap) b = make_float4(b.y, b.x, b.w, b.z);
                if (e < NR) {
                    src.entR[pg[q]] = b;
                    src.idR[pg[q]] = L.id[e];
                } else {
                    src.entS[pg[q]] = b;
                    src.idS[pg[q]] = L.id[e];
                }
            }
        }
    }
    // 4. sweep
    __syncthreads();
    // 4a. exact forward-scan range [j0, j1) of every pivot p in the other
    //     list of its tile: R pivot: the s with  r.x_l < s.x_l <= r.x_u,
    //     S pivot: the r with  s.x_l <= r.x_l <= s.x_u.  The range length
    //     goes to cnt[p] (in place of the sort keys), j0 to js[p] (in place
    //     of the tile index, read first by the same thread).
    uint32_t* cnt = L.key;
    uint16_t* js = L.tk;
    auto X = [&](int q) { return L.bx[q].x; };
    //     Thread tid takes the pivots p = q * NT + tid, so that the lanes of
    //     a wave read consecutive boxes (no LDS bank conflicts).
    uint32_t v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int p = q * NT + tid;
        v[q] = 0;
        if (p < NE) {
            const int k = L.tk[p];
            const float4 b = L.bx[p];
            const bool isR = p < NR;
            const int lo = isR ? NR + (int)L.sl[k] : (int)L.rl[k];
            const int hi = isR ? NR + (int)L.sl[k + 1] : (int)L.rl[k + 1];
            const int j0 = search_x(X, lo, hi, b.x, isR);
            const int j1 = search_x(X, j0, hi, b.z, true);
            v[q] = (uint32_t)(j1 - j0);
            js[p] = (uint16_t)j0;
        }
    }
    // 4b. exclusive prefix of the range lengths in pivot order (candidate
    //     index space): round q of NT pivots after the rounds before it
    {
        const int lane = lane_id(), w = tid / kWave;
        uint32_t inc[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            inc[q] = v[q];
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t t = __shfl_up(inc[q], d, kWave);
                if (lane >= d) inc[q] += t;
            }
        }
        if (lane == kWave - 1) {
#pragma unroll
            for (int q = 0; q < Q; ++q) s_wq[q][w] = inc[q];
        }
        __syncthreads();
        uint32_t before = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            uint32_t wpre = 0, rtot = 0;
#pragma unroll
            for (int x = 0; x < NT / kWave; ++x) {
                const uint32_t y = s_wq[q][x];
                wpre += x < w ? y : 0u;
                rtot += y;
            }
            const int p = q * NT + tid;
            if (p < NE) cnt[p] = before + wpre + inc[q] - v[q];
            before += rtot;
        }
        if (tid == 0) cnt[NE] = before;
    }
    __syncthreads();
    // 4c. every lane takes chunks of kUnitChunk consecutive candidates, so
    //     long scans are shared by many lanes; each candidate gets the closed
    //     y-test and the reference-point test of Eq. (1).  A batch of small
    //     tiles has few candidates per pivot: shorter chunks leave fewer lanes
    //     idle in the last round (measured: 4 beats 2 and 8 there; one medium
    //     tile keeps 8)
    constexpr int kUnitChunk = TC == 2 ? kChunkC : kChunkC / 2;
    const uint32_t T = cnt[NE];
    // the trip count is uniform over the workgroup (the sink needs all lanes)
    for (uint32_t it = 0; it * (uint32_t)(NT * kUnitChunk) < T; ++it) {
        const uint32_t c0 = it * (uint32_t)(NT * kUnitChunk) + (uint32_t)tid * kUnitChunk;
        const uint32_t cs = c0 < T ? c0 : T - 1u;
        int lo = 0, hi = NE;  // pivot of candidate cs: last p with cnt[p] <= cs
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cnt[mid] <= cs) lo = mid;
            else hi = mid;
        }
        int p = lo;
        uint32_t pend = cnt[p + 1];
        float4 pb4 = L.bx[p];
        uint32_t pid = L.id[p];
#pragma unroll
        for (int i = 0; i < kUnitChunk; ++i) {
            const uint32_t cc = c0 + (uint32_t)i;
            const bool valid = cc < T;
            if (valid && cc >= pend) {
                do {
                    ++p;
                    pend = cnt[p + 1];
                } while (cc >= pend);
                pb4 = L.bx[p];
                pid = L.id[p];
            }
            bool hit[1] = {false};
            uint32_t er[1] = {0}, es[1] = {0};
            if (valid) {
                const int j = (int)js[p] + (int)(cc - cnt[p]);
                const float4 q4 = L.bx[j];
                const uint32_t qid = L.id[j];
                const bool f = (pb4.y <= q4.w) && (q4.y <= pb4.w) && ref_point_here(pid, qid);
                hit[0] = f && (!dist || within_eps(pb4, q4, e2));
                if (MODE != kWrite) sk.cand += (dist && f) ? 1u : 0u;
                const bool isR = p < NR;
                er[0] = (isR ? pid : qid) & kIdMask;
                es[0] = (isR ? qid : pid) & kIdMask;
            }
            sk.template emit<1>(a, hit, er, es);
        }
    }
}

// ---------------------------------------------------------------------------
// Span units: the small tiles.  k_classify cuts the blocked tile order into
// runs of consecutive tiles of at most small_cap entries each (a tile with
// one empty list rides along: its entries are loaded but never swept), so a
// unit's R entries and its S entries are each one contiguous span of the
// tile slabs.  A unit record is (R start, NR, S start, NS) and (first tile,
// tile count); the gather needs no tile table, so the kernel issues the next
// unit's gather (and its table of tile offsets) as soon as the current
// unit's entries sit sorted in LDS, and the loads travel while the current
// unit is swept.  The tile of an entry is found by a binary search in the
// offset table (a position keeps its tile through the sort, which stays
// inside tile segments), the candidate prefix of the sweep is taken per
// wavefront over the wave's own pivots, and a unit costs three workgroup
// barriers: table and keys staged, boxes sorted, LDS free again.
// ---------------------------------------------------------------------------
struct SpanLayout {
    unsigned long long* wbuf;  // [NT / 64 * kSpanWaveBuf] pair staging per wave
    uint32_t* acc;             // [0] sink accumulator
    uint16_t* rl;              // [kSpanTQ * NT] local start of each tile's R segment (c + 1 used)
    uint16_t* sl;              // [kSpanTQ * NT] ... of its S segment
    float4* bx;                // [E] sorted boxes (R part, then S part)
    uint32_t* id;              // [E] sorted id words
    uint32_t* key;             // [E + 8] sort keys; then per wave the candidate prefix
    uint16_t* js;              // [E] per wave: first candidate of each pivot's scan
};

__host__ __device__ constexpr size_t span_lds_bytes(int nt, int e) {
    return (size_t)(nt / kWave) * kSpanWaveBuf * 8 + 16 + (size_t)kSpanTQ * nt * 4 +  // staging, acc, tables
           (size_t)e * 16 + (size_t)e * 4 + (size_t)(e + 8) * 4 + (size_t)e * 2;
}

__device__ inline SpanLayout carve_span(unsigned char* p, int nt, int e) {
    SpanLayout L;
    L.wbuf = (unsigned long long*)p;
    p += (size_t)(nt / kWave) * kSpanWaveBuf * 8;
    L.acc = (uint32_t*)p;
    p += 16;
    L.rl = (uint16_t*)p;
    p += (size_t)kSpanTQ * nt * 2;
    L.sl = (uint16_t*)p;
    p += (size_t)kSpanTQ * nt * 2;  // nt is a multiple of 64: the boxes stay 16-byte aligned
    L.bx = (float4*)p;
    p += (size_t)e * 16;
    L.id = (uint32_t*)p;
    p += (size_t)e * 4;
    L.key = (uint32_t*)p;
    p += (size_t)(e + 8) * 4;
    L.js = (uint16_t*)p;
    return L;
}

__device__ __forceinline__ void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v, int lane) {
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

// Last k in [0, c) with T[k] <= v: the segment holding local position v
// (T non-decreasing, T[0] = 0 <= v < T[c]; empty segments are skipped).
__device__ __forceinline__ int segment_of(const uint16_t* T, int c, int v) {
    int lo = 0, hi = c;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int)T[mid] <= v) lo = mid;
        else hi = mid;
    }
    return lo;
}

typedef float vf4 __attribute__((ext_vector_type(4)));  // a box held in registers

// Issue the loads of a staged span unit: thread tid's words t = tid + k * NT
// of the tile offset tables (raw: made local to the spans only when the unit
// is staged, so that no instruction here waits for a load) and its entries
// e = tid + q * NT.
template <int NT, int Q>
__device__ __forceinline__ void span_issue(const Src& a, int tid, const uint4& sp, const uint2& ut,
                                           uint32_t (&tr)[kSpanTQ], uint32_t (&ts)[kSpanTQ],
                                           vf4 (&pb)[Q], uint32_t (&pi)[Q]) {
#pragma unroll
    for (int k = 0; k < kSpanTQ; ++k) {
        const int t = tid + k * NT;
        if (t <= (int)ut.y) {
            tr[k] = a.offR[ut.x + t];
            ts[k] = a.offS[ut.x + t];
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint32_t e = (uint32_t)(tid + q * NT);
        if (e < sp.y) {
            pb[q] = ((const vf4*)a.entR)[sp.x + e];
            pi[q] = a.idR[sp.x + e];
        } else if (e < sp.y + sp.w) {
            pb[q] = ((const vf4*)a.entS)[sp.z + (e - sp.y)];
            pi[q] = a.idS[sp.z + (e - sp.y)];
        }
    }
}

// waves per SIMD that the LDS slab allows: the register budget the compiler
// is held to, so that registers do not lower the occupancy further
__host__ __device__ constexpr int span_waves(int nt, int q) {
    const int per_cu = (int)(163840 / span_lds_bytes(nt, nt * q));
    const int w = per_cu * (nt / kWave) / 4;
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// BATCH: the units of a batch of joins (job records, stripes); a separate
// instantiation, so that the single-join kernel carries none of it.
template <int NT, int Q, int MODE, bool BATCH>
__global__ __launch_bounds__(NT, span_waves(NT, Q)) void k_span_units(Args a) {
    constexpr int E = NT * Q;
    constexpr int PW = Q * kWave;  // pivots of one wavefront
    constexpr int kCh = kChunkC / 2;  // consecutive candidates per lane and round
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const SpanLayout L = carve_span(smem, NT, E);
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const uint32_t nu = min(a.ctr[kUnitsWritten], (uint32_t)a.cap_units);
    const uint32_t G = gridDim.x;
    Sink<MODE, true, BATCH> sk;
    sk.buf = L.wbuf + w * kSpanWaveBuf;
    sk.s_acc = L.acc;
    sk.bufcap = kSpanWaveBuf;
    sk.init(blockIdx.x * (NT / kWave) + w);
    const uint32_t S = BATCH ? kSpanStripe : 1u;
    // Unit records of this workgroup, kWave at a time: lane l holds the record
    // of the workgroup's unit i0 + l, read with readlane.  No memory wait
    // falls inside the loop: vector loads retire in order, so waiting for a
    // record loaded after the next unit's entries would wait for the entries
    // too.
    uint4 rsp = make_uint4(0, 0, 0, 0);
    uint2 rut = make_uint2(0, 0);
    uint32_t rjob = 0;
    int i0 = 0;
    auto load_records = [&](int base) {
        i0 = base;
        const uint32_t uu = unit_of((uint32_t)(base + lane), blockIdx.x, G, S);
        if (uu < nu) {
            rsp = a.uspan[uu];
            rut = a.units[uu];
            if (BATCH) rjob = a.ujob[uu];
        }
    };
    auto record = [&](int i, uint4& s, uint2& t, uint32_t& j) {  // i0 <= i < i0 + kWave
        const int l = i - i0;
        s = make_uint4(__builtin_amdgcn_readlane(rsp.x, l), __builtin_amdgcn_readlane(rsp.y, l),
                       __builtin_amdgcn_readlane(rsp.z, l), __builtin_amdgcn_readlane(rsp.w, l));
        t = make_uint2(__builtin_amdgcn_readlane(rut.x, l), __builtin_amdgcn_readlane(rut.y, l));
        j = BATCH ? __builtin_amdgcn_readlane(rjob, l) : 0u;
    };
    // a batch's job descriptors: scalar loads at every use (kept in
    // registers across units, they would crowd out the sweep's)
    auto src_for = [&](uint32_t j) { return BATCH ? src_of(a.jobs[j]) : src_of(a); };
    // staged unit: record, join, this thread's table words and entries (in flight)
    uint4 sp = make_uint4(0, 0, 0, 0);
    uint2 ut = make_uint2(0, 0);
    uint32_t sjob = 0;
    uint32_t tr[kSpanTQ] = {}, ts[kSpanTQ] = {};
    vf4 pb[Q];
    uint32_t pi[Q];
    uint32_t u = unit_of(0, blockIdx.x, G, S);
    int i = 0;
    if (u < nu) {
        load_records(0);
        record(0, sp, ut, sjob);
        span_issue<NT, Q>(src_for(sjob), tid, sp, ut, tr, ts, pb, pi);
        sk.cjob = sjob;  // nothing staged yet
    }
    for (; u < nu; ++i, u = unit_of((uint32_t)i, blockIdx.x, G, S)) {
        const uint4 cur = sp;
        const uint32_t cjob = sjob;
        const JobFlags jf = flags_of(a, cjob);
        const int NR = (int)cur.y, NE = (int)(cur.y + cur.w), c = (int)ut.y;
        if (NE > E || c < 1 || c >= kSpanTQ * NT) {  // cannot happen for units built by k_classify
            if (tid == 0) atomicOr(&a.st->flags, kStatInternal);
            break;
        }
        sk.begin(a, u);  // per-unit count / output region; thread 0 clears the accumulator
        // 1. tile table and sort keys (the writing pass reads slabs left sorted)
#pragma unroll
        for (int k = 0; k < kSpanTQ; ++k) {
            const int t = tid + k * NT;
            if (t <= c) {
                L.rl[t] = (uint16_t)(tr[k] - cur.x);
                L.sl[t] = (uint16_t)(ts[k] - cur.z);
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = tid + q * NT;
            if (e < NE) {
                if (MODE == kWrite) {
                    ((vf4*)L.bx)[e] = pb[q];
                    L.id[e] = pi[q];
                } else {
                    L.key[e] = order_key(pb[q].x);
                }
            }
        }
        __syncthreads();
        // 2. tile of each entry; rank sort inside its segment
        int tk[Q];
        {
            int ev[Q], pe[Q];
            bool isR[Q], act[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                pe[q] = tid + q * NT;
                act[q] = pe[q] < NE;
                isR[q] = pe[q] < NR;
                ev[q] = isR[q] ? pe[q] : pe[q] - NR;
                ev[q] = act[q] ? ev[q] : 0;
            }
#pragma unroll
            for (int q = 0; q < Q; ++q)
                tk[q] = isR[q] ? segment_of(L.rl, c, ev[q]) : segment_of(L.sl, c, ev[q]);
            if (MODE != kWrite) {
                int lo[Q], hi[Q], rk[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int k = tk[q];
                    lo[q] = isR[q] ? (int)L.rl[k] : NR + (int)L.sl[k];
                    hi[q] = isR[q] ? (int)L.rl[k + 1] : NR + (int)L.sl[k + 1];
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) rk[q] = act[q] ? seg_rank(L.key, lo[q], hi[q], pe[q]) : 0;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    if (act[q]) {
                        ((vf4*)L.bx)[lo[q] + rk[q]] = pb[q];
                        L.id[lo[q] + rk[q]] = pi[q];
                    }
                }
            }
        }
        // the staged registers are free: start the next unit's loads
        if (unit_of((uint32_t)i + 1u, blockIdx.x, G, S) < nu) {
            if (i + 1 - i0 >= kWave) load_records(i + 1);
            record(i + 1, sp, ut, sjob);
            span_issue<NT, Q>(src_for(sjob), tid, sp, ut, tr, ts, pb, pi);
        }
        __syncthreads();
        if (MODE == kCount && a.writeback) {  // slabs left sorted for the writing pass
            const Src cs = src_for(cjob);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int e = tid + q * NT;
                if (e < NR) {
                    cs.entR[cur.x + e] = L.bx[e];
                    cs.idR[cur.x + e] = L.id[e];
                } else if (e < NE) {
                    cs.entS[cur.z + (e - NR)] = L.bx[e];
                    cs.idS[cur.z + (e - NR)] = L.id[e];
                }
            }
        }
        // 3. exact forward-scan range of this thread's pivots p = tid + q * NT
        //    (R pivot: the s with r.x_l < s.x_l <= r.x_u; S pivot: the r with
        //    s.x_l <= r.x_l <= s.x_u), and the wave's exclusive prefix of the
        //    range lengths (slot q * 64 + lane)
        uint32_t* cw = L.key + w * (PW + 1);
        uint16_t* jw = L.js + w * PW;
        uint32_t run = 0;
        {
            int lo[Q], hi[Q], j0[Q], j1[Q];
            float xl[Q], xu[Q];
            bool isR[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int p = tid + q * NT;
                isR[q] = p < NR;
                lo[q] = hi[q] = 0;
                xl[q] = xu[q] = 0.f;
                if (p < NE) {
                    const int k = tk[q];
                    const float4 b = L.bx[p];
                    xl[q] = b.x;
                    xu[q] = b.z;
                    lo[q] = isR[q] ? NR + (int)L.sl[k] : (int)L.rl[k];
                    hi[q] = isR[q] ? NR + (int)L.sl[k + 1] : (int)L.rl[k + 1];
                }
            }
            auto X = [&](int j) { return L.bx[j].x; };
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                j0[q] = search_x(X, lo[q], hi[q], xl[q], isR[q]);
                j1[q] = search_x(X, j0[q], hi[q], xu[q], true);
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const uint32_t v = (uint32_t)(j1[q] - j0[q]);
                const uint32_t inc = wave_incl_sum(v, lane);
                cw[q * kWave + lane] = run + inc - v;
                jw[q * kWave + lane] = (uint16_t)j0[q];
                run += __shfl(inc, kWave - 1, kWave);
            }
        }
        if (lane == 0) cw[PW] = run;
        wave_fence();
        // 4. the wave's candidates, kCh consecutive ones per lane and round;
        //    each gets the closed y-test and the reference-point test of Eq. (1)
        const uint32_t T = run;
        for (uint32_t it = 0; it * (uint32_t)(kWave * kCh) < T; ++it) {
            const uint32_t c0 = it * (uint32_t)(kWave * kCh) + (uint32_t)lane * kCh;
            const uint32_t cs = c0 < T ? c0 : T - 1u;
            int lo = 0, hi = PW;  // slot of candidate cs: last slot with cw[slot] <= cs
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (cw[mid] <= cs) lo = mid;
                else hi = mid;
            }
            int sl = lo;
            uint32_t pend = cw[sl + 1];
            int p = (sl / kWave) * NT + w * kWave + (sl % kWave);
            float4 pb4 = L.bx[p];
            uint32_t pid = L.id[p];
#pragma unroll
            for (int i = 0; i < kCh; ++i) {
                const uint32_t cc = c0 + (uint32_t)i;
                const bool valid = cc < T;
                if (valid && cc >= pend) {
                    do {
                        ++sl;
                        pend = cw[sl + 1];
                    } while (cc >= pend);
                    p = (sl / kWave) * NT + w * kWave + (sl % kWave);
                    pb4 = L.bx[p];
                    pid = L.id[p];
                }
                bool hit[1] = {false};
                uint32_t er[1] = {0}, es[1] = {0};
                if (valid) {
                    const int j = (int)jw[sl] + (int)(cc - cw[sl]);
                    const float4 q4 = L.bx[j];
                    const uint32_t qid = L.id[j];
                    const bool f = (pb4.y <= q4.w) && (q4.y <= pb4.w) && ref_point_here(pid, qid);
                    hit[0] = f && (!jf.dist || within_eps(pb4, q4, jf.e2));
                    if (MODE != kWrite) sk.cand += (jf.dist && f) ? 1u : 0u;
                    const bool isR = p < NR;
                    er[0] = (isR ? pid : qid) & kIdMask;
                    es[0] = (isR ? qid : pid) & kIdMask;
                }
                sk.template emit<1>(a, hit, er, es);
            }
        }
        // 5. unit end: counts / remaining staged pairs, then LDS is free; a
        //    batch's pairs leave the wave when the next unit (staged above)
        //    belongs to another join
        if (MODE == kWrite && sk.n) sk.flush(a);
        if (BATCH && sjob != cjob) sk.set_job(a, sjob);
        if (MODE == kCount) {
            uint32_t v = sk.cnt;
            for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
            if (lane == 0 && v) atomicAdd(L.acc, v);
        }
        __syncthreads();
        if (MODE == kCount && tid == 0) a.ucnt[u] = *L.acc;
    }
    sk.finish(a, blockIdx.x * (NT / kWave) + w);
}

// ---------------------------------------------------------------------------
// k_classify: sort the tiles into three classes by entry count n = nr + ns
// and build the work lists of the join.  One workgroup covers kClassChunk
// consecutive tiles of the blocked order (kClassPer per thread).
//   small:  both lists non-empty, n <= small_cap.  Cut into span units:
//           maximal runs of consecutive tiles with n <= small_cap (tiles
//           with one empty list ride along), also cut where the running
//           entry count of the run crosses a multiple of unit_cap and every
//           unit_tiles tiles.  A unit therefore holds at most
//           unit_cap - 1 + small_cap entries and unit_tiles tiles, and its R
//           and S entries are contiguous.  Runs without a joinable tile are
//           dropped.
//   medium: both lists non-empty, small_cap < n <= med_cap: one record each.
//   dense:  both lists non-empty, n > med_cap: sorted globally and split.
// A tile's segment bounds are written with its record, so the join kernels
// need no dependent loads of the offset arrays.
// ---------------------------------------------------------------------------
constexpr int kClassNT = 256;
constexpr int kClassPer = 16;
constexpr int kClassChunk = kClassNT * kClassPer;

__device__ __forceinline__ void append_dense(const Args& a, uint32_t t, uint32_t nr, uint32_t ns) {
    const uint32_t d = atomicAdd(&a.ctr[kDenseCount], 1u);
    const uint32_t base = atomicAdd(&a.ctr[kDenseEntries], nr + ns);
    if (d < (uint32_t)a.cap_dense && (int64_t)base + nr + ns <= a.cap_dent) {
        a.dense[d] = make_uint4(t, base, nr, ns);
        if (a.batch) a.djob[d] = a.jid;
    } else
        atomicOr(&a.st->flags, kStatCapacity);
}

// Block-wide exclusive sums of four per-thread values (kClassNT threads);
// tot receives the block totals.
__device__ __forceinline__ void block_excl4(uint32_t (&v)[4], uint32_t (&tot)[4],
                                            uint32_t (*s_ws)[kClassNT / kWave]) {
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    uint32_t inc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        inc[i] = v[i];
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t t = __shfl_up(inc[i], d, kWave);
            if (lane >= d) inc[i] += t;
        }
        if (lane == kWave - 1) s_ws[i][w] = inc[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint32_t before = 0, all = 0;
        for (int q = 0; q < kClassNT / kWave; ++q) {
            const uint32_t y = s_ws[i][q];
            before += q < w ? y : 0u;
            all += y;
        }
        v[i] = before + inc[i] - v[i];
        tot[i] = all;
    }
    __syncthreads();
}

__device__ __forceinline__ void classify_body(const Args& a, uint32_t blk) {
    __shared__ uint16_t s_j[kClassChunk + 1];  // joinable small tiles before each tile of the chunk
    __shared__ uint32_t s_ws[4][kClassNT / kWave];
    __shared__ uint32_t s_fc[kClassNT / kWave];  // first cut of each wave
    __shared__ uint32_t s_base[2];
    // an input whose partition failed or overflowed holds no valid tile
    // offsets: no work (the join's status carries its flags)
    if ((a.stR->flags | a.stS->flags) & (kStatBadRect | kStatCapacity | kStatTooLarge)) return;
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const int64_t c0 = (int64_t)blk * kClassChunk;  // first tile of the chunk
    const int tl0 = tid * kClassPer;                        // this thread's first local tile
    const int64_t t0 = c0 + tl0;
    const uint32_t SC = (uint32_t)a.small_cap, B = (uint32_t)a.unit_cap;
    const int TC = a.unit_tiles;
    // offsets of tiles t0 - 1 .. t0 + kClassPer (index i <-> tile t0 - 1 + i)
    uint32_t oR[kClassPer + 2], oS[kClassPer + 2];
#pragma unroll
    for (int i = 0; i < kClassPer + 2; ++i) {
        const int64_t t = t0 - 1 + i;
        const bool in = t >= 0 && t <= a.C;
        oR[i] = in ? a.offR[t] : 0u;
        oS[i] = in ? a.offS[t] : 0u;
    }
    // per tile (bit i <-> index i; index 0 is the tile before this thread's
    // range): cuts a span run (a tile of more than small_cap entries, or past
    // the grid), joinable small tile; a run tile weighs its entry count
    auto n_of = [&](int i) { return (oR[i + 1] - oR[i]) + (oS[i + 1] - oS[i]); };
    uint32_t brkm = 0, joinm = 0;
    uint32_t nj = 0, je = 0, nmed = 0, med_e = 0, wsum = 0;
#pragma unroll
    for (int i = 0; i <= kClassPer; ++i) {
        const int64_t t = t0 - 1 + i;
        const bool exists = t >= 0 && t < a.C;
        const uint32_t nr = oR[i + 1] - oR[i], ns = oS[i + 1] - oS[i], n = nr + ns;
        if (!exists || n > SC) brkm |= 1u << i;
        if (i == 0 || !exists) continue;
        if (n <= SC) wsum += n;
        if (nr && ns) {
            if (n <= SC) {
                joinm |= 1u << (i - 1);
                ++nj;
                je += n;
            } else if (n <= (uint32_t)a.med_cap) {
                ++nmed;
                med_e += n;
            } else {
                append_dense(a, (uint32_t)t, nr, ns);
            }
        }
    }
    // block prefixes: run weights, joinable tiles, medium tiles, their entries
    uint32_t v[4] = {wsum, nj, nmed, med_e}, tot[4];
    block_excl4(v, tot, s_ws);
    const uint32_t wpre = v[0], jpre = v[1], mpre = v[2];
    // unit starts (bit q <-> tile t0 + q); joinable prefix per tile into LDS
    uint32_t startm = 0;
    uint32_t first_cut = kClassChunk;
    {
        uint32_t pre = wpre, jrun = jpre;
        uint32_t pre_prev = wpre - ((brkm & 1u) ? 0u : n_of(0));
#pragma unroll
        for (int q = 0; q < kClassPer; ++q) {
            const int tl = tl0 + q;
            const bool brk = (brkm >> (q + 1)) & 1u, brk_prev = (brkm >> q) & 1u;
            const bool st = !brk && (tl == 0 || brk_prev || pre / B != pre_prev / B || tl % TC == 0);
            startm |= st ? 1u << q : 0u;
            if ((brk || st) && first_cut == (uint32_t)kClassChunk) first_cut = tl;
            s_j[tl] = (uint16_t)jrun;
            jrun += (joinm >> q) & 1u;
            pre_prev = pre;
            pre += brk ? 0u : n_of(q + 1);
        }
        if (tid == kClassNT - 1) s_j[kClassChunk] = (uint16_t)jrun;
    }
    const uint32_t cutm = startm | (brkm >> 1);
    // first cut after this thread's range: suffix minimum over later threads
    uint32_t m = first_cut;
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t t = __shfl_down(m, d, kWave);
        if (lane + d < kWave) m = t < m ? t : m;
    }
    if (lane == 0) s_fc[w] = m;
    uint32_t after = __shfl_down(m, 1, kWave);
    if (lane == kWave - 1) after = kClassChunk;
    __syncthreads();
    for (int q = w + 1; q < kClassNT / kWave; ++q) after = s_fc[q] < after ? s_fc[q] : after;
    // a unit [start, next cut) is kept if it holds a joinable tile
    uint32_t keepm = 0, nu = 0;
    {
        uint32_t next = after;
#pragma unroll
        for (int q = kClassPer - 1; q >= 0; --q) {
            if (((startm >> q) & 1u) && s_j[next] != s_j[tl0 + q]) {
                keepm |= 1u << q;
                ++nu;
            }
            if ((cutm >> q) & 1u) next = (uint32_t)(tl0 + q);
        }
    }
    uint32_t vu[4] = {nu, je, 0, 0}, totu[4];
    block_excl4(vu, totu, s_ws);
    const uint32_t total_units = totu[0], total_j = tot[1], total_med = tot[2];
    if (tid == 0) {
        // joinable tiles and units reserved with one 64-bit add, the entry
        // statistics of the small and medium tiles added with another (every
        // workgroup adds to the same words, so the atomics serialise; the low
        // words never carry)
        const unsigned long long add =
            (unsigned long long)total_j | ((unsigned long long)total_units << 32);
        const unsigned long long tu =
            add ? atomicAdd((unsigned long long*)&a.ctr[kTilesWritten], add) : 0ull;
        s_base[0] = (uint32_t)(tu >> 32);
        s_base[1] = total_med ? atomicAdd(&a.ctr[kMedCount], total_med) : 0u;
        const unsigned long long both = (unsigned long long)totu[1] | ((unsigned long long)tot[3] << 32);
        if (both) atomicAdd((unsigned long long*)&a.ctr[kSmallEntries], both);
    }
    __syncthreads();
    const uint32_t ub = s_base[0], mb = s_base[1];
    if ((int64_t)ub + total_units > a.cap_units || (int64_t)mb + total_med > a.cap_med) {
        if (tid == 0) atomicOr(&a.st->flags, kStatCapacity);
        return;
    }
    {
        // unit records, last first (the end of a unit is the next cut)
        uint32_t ui = ub + vu[0] + nu, next = after;
#pragma unroll
        for (int q = kClassPer - 1; q >= 0; --q) {
            if ((keepm >> q) & 1u) {
                const int64_t t = t0 + q, te = c0 + next;  // te <= C: tiles past the grid cut runs
                const uint32_t rend = a.offR[te], send = a.offS[te];  // (cached: read by this block)
                --ui;
                a.uspan[ui] = make_uint4(oR[q + 1], rend - oR[q + 1], oS[q + 1], send - oS[q + 1]);
                a.units[ui] = make_uint2((uint32_t)t, (uint32_t)(te - t));
                if (a.batch) a.ujob[ui] = a.jid;
            }
            if ((cutm >> q) & 1u) next = (uint32_t)(tl0 + q);
        }
    }
    uint32_t mi = mb + mpre;
#pragma unroll
    for (int q = 0; q < kClassPer; ++q) {
        const int64_t t = t0 + q;
        const uint32_t nr = oR[q + 2] - oR[q + 1], ns = oS[q + 2] - oS[q + 1];
        if (t < a.C && nr && ns && nr + ns > SC && nr + ns <= (uint32_t)a.med_cap) {
            if (a.axis_model) a.medt[mi] = (uint32_t)t;
            if (a.batch) a.mjob[mi] = a.jid;
            a.med[mi++] = make_uint4(oR[q + 1], nr, oS[q + 1], ns);
        }
    }
}

__global__ __launch_bounds__(kClassNT) void k_classify(Args a) { classify_body(a, blockIdx.x); }

// Every join of a batch in one launch: the workgroups of join j classify its
// grid's chunks (job_slot over the prefix of their counts).
__global__ __launch_bounds__(kClassNT) void k_classify_b(Args a, const uint32_t* __restrict__ pre,
                                                         int nj) {
    const JobSlot t = job_slot(pre, nj);
    const Job& J = a.jobs[t.j];
    Args b = a;
    b.offR = J.offR;
    b.offS = J.offS;
    b.stR = J.stR;
    b.stS = J.stS;
    b.C = J.C;
    b.jid = (uint32_t)t.j;
    b.axis_model = (J.flags & kJobAxis) ? 1 : 0;
    classify_body(b, t.wg);
}

// ---------------------------------------------------------------------------
// Sweeping-axis model (Sec. 3.3, Eq. (2)) of one tile, evaluated by one
// workgroup of kAxisNT threads.  Sample: the entries whose rectangle index is
// a multiple of phi = 100.  k divisions per tile extent, k = clamp(floor(
// tile extent / mean sampled extent), 1, 1000), the mean of (w + h) / 2 in
// cell units from exact integer sums in units of 2^-30 of a cell (128-bit),
// so it does not depend on the order of the tile's list.  An extent is
// capped at 2^32 cells first: one such extent makes the sum >= 2^62, more
// than 2 n 2^30 for any sample size n < 2^31, so k = 1 with or without it.  Per axis
// and side a histogram counts the sampled rectangles meeting each division
// (difference array in LDS, then a prefix sum); I = sum_i H_R[i] * H_S[i].
// ---------------------------------------------------------------------------
constexpr int kAxisNT = 256;
constexpr uint32_t kAxisPhi = 100;
constexpr int kAxisKMax = 1000;
constexpr int kAxisPer = (kAxisKMax + kAxisNT - 1) / kAxisNT;  // divisions per thread

typedef unsigned __int128 u128;

struct AxisLds {
    int hist[4][kAxisKMax + 1];  // difference arrays: R x, R y, S x, S y
    int wsum[kAxisNT / kWave][4];
    unsigned long long red[kAxisNT / kWave][2];
    u128 ext[kAxisNT / kWave];
    uint32_t cnt[kAxisNT / kWave][2];
};

struct AxisOut {
    int k;
    unsigned long long ix, iy;
};

// extent hi - lo in cell units, capped at 2^32 cells, in units of 2^-30 cell
// (< 2^63: the scaling by 2^30 is exact, the conversion truncates = floor)
__device__ __forceinline__ unsigned long long fixed_extent(float lo, float hi, float scale) {
    const float e = fminf(__fmul_rn(__fsub_rn(hi, lo), scale), 4294967296.0f);
    return (unsigned long long)__fmul_rn(e, 1073741824.0f);
}

__device__ __forceinline__ u128 shfl_xor_u128(u128 v, int d) {
    const unsigned long long lo = __shfl_xor((unsigned long long)v, d, kWave);
    const unsigned long long hi = __shfl_xor((unsigned long long)(v >> 64), d, kWave);
    return ((u128)hi << 64) | lo;
}

// division of coordinate v in tile column t
__device__ __forceinline__ int division(float v, float origin, float scale, int t, int k) {
    const float u = __fmul_rn(__fsub_rn(v, origin), scale);
    float f = floorf(__fmul_rn(__fsub_rn(u, (float)t), (float)k));
    f = fminf(fmaxf(f, 0.0f), (float)(k - 1));
    return (int)f;
}

__device__ __forceinline__ void blocked_xy(const Blocking& bl, uint32_t t, int& tx, int& ty) {
    const uint32_t B2 = (uint32_t)bl.tiles_per_cell();
    const uint32_t cell = t / B2, r = t % B2;
    tx = (int)(cell % (uint32_t)bl.Gx) * bl.Bx + (int)(r % (uint32_t)bl.Bx);
    ty = (int)(cell / (uint32_t)bl.Gx) * bl.By + (int)(r / (uint32_t)bl.Bx);
}

__device__ AxisOut axis_eval(const float4* __restrict__ bR, const uint32_t* __restrict__ iR,
                             uint32_t nr, const float4* __restrict__ bS,
                             const uint32_t* __restrict__ iS, uint32_t ns, int tx, int ty,
                             const GridDev& g, AxisLds& L) {
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    constexpr int NW = kAxisNT / kWave;
    const uint32_t n = nr + ns;
    // A. sample sizes and fixed-point extent sum
    uint32_t cR = 0, cS = 0;
    u128 ext = 0;
    for (uint32_t i = tid; i < n; i += kAxisNT) {
        const bool isR = i < nr;
        const uint32_t j = isR ? i : i - nr;
        if (((isR ? iR : iS)[j] & kIdMask) % kAxisPhi == 0u) {
            const float4 b = (isR ? bR : bS)[j];
            ext += (u128)fixed_extent(b.x, b.z, g.sx) + (u128)fixed_extent(b.y, b.w, g.sy);
            if (isR) ++cR;
            else ++cS;
        }
    }
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        cR += __shfl_xor(cR, d, kWave);
        cS += __shfl_xor(cS, d, kWave);
        ext += shfl_xor_u128(ext, d);
    }
    if (lane == 0) {
        L.cnt[w][0] = cR;
        L.cnt[w][1] = cS;
        L.ext[w] = ext;
    }
    __syncthreads();
    uint32_t nRs = 0, nSs = 0;
    u128 tot = 0;
    for (int q = 0; q < NW; ++q) {
        nRs += L.cnt[q][0];
        nSs += L.cnt[q][1];
        tot += L.ext[q];
    }
    __syncthreads();
    AxisOut o{0, 0ull, 0ull};
    if (nRs == 0 || nSs == 0) return o;  // the same for every thread
    int k = kAxisKMax;
    if (tot) {
        const u128 q = ((u128)(2ull * (nRs + nSs)) << 30) / tot;
        k = q < 1 ? 1 : (q > (u128)kAxisKMax ? kAxisKMax : (int)q);
    }
    // B. difference arrays of the four histograms
    for (int i = tid; i < 4 * (kAxisKMax + 1); i += kAxisNT) (&L.hist[0][0])[i] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kAxisNT) {
        const bool isR = i < nr;
        const uint32_t j = isR ? i : i - nr;
        if (((isR ? iR : iS)[j] & kIdMask) % kAxisPhi == 0u) {
            const float4 b = (isR ? bR : bS)[j];
            int* hx = L.hist[isR ? 0 : 2];
            int* hy = L.hist[isR ? 1 : 3];
            atomicAdd(&hx[division(b.x, g.x0, g.sx, tx, k)], 1);
            atomicAdd(&hx[division(b.z, g.x0, g.sx, tx, k) + 1], -1);
            atomicAdd(&hy[division(b.y, g.y0, g.sy, ty, k)], 1);
            atomicAdd(&hy[division(b.w, g.y0, g.sy, ty, k) + 1], -1);
        }
    }
    __syncthreads();
    // C. prefix sums over the divisions (thread j owns kAxisPer of them) and
    //    the products of Eq. (2)
    const int d0 = tid * kAxisPer;
    int part[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kAxisPer; ++q) {
        const int d = d0 + q;
        if (d < k) {
#pragma unroll
            for (int h = 0; h < 4; ++h) part[h] += L.hist[h][d];
        }
    }
    int inc[4] = {part[0], part[1], part[2], part[3]};
    for (int d = 1; d < kWave; d <<= 1) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int t = __shfl_up(inc[h], d, kWave);
            if (lane >= d) inc[h] += t;
        }
    }
    if (lane == kWave - 1) {
#pragma unroll
        for (int h = 0; h < 4; ++h) L.wsum[w][h] = inc[h];
    }
    __syncthreads();
    int run[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        run[h] = inc[h] - part[h];
        for (int q = 0; q < w; ++q) run[h] += L.wsum[q][h];
    }
    unsigned long long ix = 0, iy = 0;
#pragma unroll
    for (int q = 0; q < kAxisPer; ++q) {
        const int d = d0 + q;
        if (d < k) {
#pragma unroll
            for (int h = 0; h < 4; ++h) run[h] += L.hist[h][d];
            ix += (unsigned long long)run[0] * (unsigned long long)run[2];
            iy += (unsigned long long)run[1] * (unsigned long long)run[3];
        }
    }
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        ix += __shfl_xor(ix, d, kWave);
        iy += __shfl_xor(iy, d, kWave);
    }
    if (lane == 0) {
        L.red[w][0] = ix;
        L.red[w][1] = iy;
    }
    __syncthreads();
    o.k = k;
    for (int q = 0; q < NW; ++q) {
        o.ix += L.red[q][0];
        o.iy += L.red[q][1];
    }
    __syncthreads();
    return o;
}

// The join's medium and dense tiles: evaluate the model, mark the tiles to
// sweep along y (bit 31 of the record), count both.
__global__ __launch_bounds__(kAxisNT) void k_axis(Args a) {
    __shared__ AxisLds L;
    const uint32_t nm = min(a.ctr[kMedCount], (uint32_t)a.cap_med);
    const uint32_t nd = min(a.ctr[kDenseCount], (uint32_t)a.cap_dense);
    uint32_t nt = 0, ny = 0;
    for (uint32_t j = blockIdx.x; j < nm + nd; j += gridDim.x) {
        const bool med = j < nm;
        const uint32_t job = a.batch ? (med ? a.mjob[j] : a.djob[j - nm]) : 0u;
        if (a.batch && !(a.jobs[job].flags & kJobAxis)) continue;  // (uniform per block)
        const Src src = a.batch ? src_of(a.jobs[job]) : src_of(a);
        const GridDev gd = a.batch ? a.jobs[job].gd : a.gd;
        const Blocking bl = a.batch ? a.jobs[job].bl : a.bl;
        const uint4 rec = med ? a.med[j] : a.dense[j - nm];
        uint32_t t, nr, ns, r0, s0;
        if (med) {
            t = a.medt[j];
            r0 = rec.x;
            nr = rec.y;
            s0 = rec.z;
            ns = rec.w;
        } else {
            t = rec.x;
            r0 = src.offR[t];
            nr = rec.z;
            s0 = src.offS[t];
            ns = rec.w;
        }
        int tx, ty;
        blocked_xy(bl, t, tx, ty);
        const AxisOut o = axis_eval(src.entR + r0, src.idR + r0, nr, src.entS + s0, src.idS + s0, ns,
                                    tx, ty, gd, L);
        if (threadIdx.x == 0) {
            ++nt;
            if (o.iy < o.ix) {
                ++ny;
                if (med) a.med[j].y = rec.y | kAxisBit;
                else a.dense[j - nm].x = rec.x | kAxisBit;
            }
        }
    }
    if (threadIdx.x == 0 && nt) {
        atomicAdd(&a.ctr[kAxisTiles], nt);
        if (ny) atomicAdd(&a.ctr[kAxisY], ny);
    }
}

// The model for listed tiles (sj_sweep_axis).
__global__ __launch_bounds__(kAxisNT) void k_axis_query(const uint32_t* __restrict__ offR,
                                                        const uint32_t* __restrict__ offS,
                                                        const float4* __restrict__ entR,
                                                        const uint32_t* __restrict__ idR,
                                                        const float4* __restrict__ entS,
                                                        const uint32_t* __restrict__ idS, GridDev gd,
                                                        Blocking bl, const int2* __restrict__ tiles,
                                                        int64_t n, long long* __restrict__ out) {
    __shared__ AxisLds L;
    for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
        const int2 xy = tiles[j];
        const uint32_t cell = (uint32_t)(xy.y / bl.By) * (uint32_t)bl.Gx + (uint32_t)(xy.x / bl.Bx);
        const uint32_t t = cell * (uint32_t)bl.tiles_per_cell() +
                           (uint32_t)(xy.y % bl.By) * (uint32_t)bl.Bx + (uint32_t)(xy.x % bl.Bx);
        const uint32_t r0 = offR[t], s0 = offS[t];
        const AxisOut o =
            axis_eval(entR + r0, idR + r0, offR[t + 1] - r0, entS + s0, idS + s0, offS[t + 1] - s0,
                      xy.x, xy.y, gd, L);
        if (threadIdx.x == 0) {
            out[4 * j] = o.k;
            out[4 * j + 1] = (long long)o.ix;
            out[4 * j + 2] = (long long)o.iy;
            out[4 * j + 3] = o.iy < o.ix ? 1 : 0;
        }
    }
}

// ---------------------------------------------------------------------------
// k_lds_medium: one workgroup per medium tile (persistent workgroups, tiles
// assigned round-robin; the record of the next tile is loaded while the
// current one is sorted and swept).  The grid is an upper bound on the tile
// count; surplus workgroups exit at once.
// ---------------------------------------------------------------------------
template <int NT, int Q, int MODE>
__global__ __launch_bounds__(NT) void k_lds_medium(Args a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int TC = tc_for(NT * Q, false);
    const uint32_t nu = min(a.ctr[kMedCount], (uint32_t)a.cap_med);
    const LdsLayout L = carve(smem, NT, NT * Q, TC);
    Sink<MODE, true> sk = make_sink<MODE>(L);
    __shared__ uint4 s_rec;
    __shared__ uint32_t s_u;
    const uint32_t G = gridDim.x;
    const uint32_t SP = a.batch ? kMedStripe : 1u;
    // a single join claims its tiles largest first (LPT order); thread 0
    // claims the next one as the current one starts and loads its record
    // during the sweep, so neither wait is exposed
    const bool dyn = !a.batch && a.med_lpt;
    uint32_t* taken = &a.ctr[MODE == kWrite ? kMedTaken2 : kMedTaken];
    uint32_t i = 0, u;
    uint4 pf = make_uint4(0, 0, 0, 0);
    if (dyn) {
        if (threadIdx.x == 0) {
            const uint32_t f = atomicAdd(taken, 1u);
            s_u = f;
            if (f < nu) s_rec = a.med_lpt[f];
        }
        __syncthreads();
        u = s_u;
        pf = s_rec;
    } else {
        u = unit_of(0, blockIdx.x, G, SP);
        if (u < nu) pf = a.med[u];
    }
    while (u < nu) {
        const int64_t slot = a.base_med + u;
        const uint32_t job = a.batch ? a.mjob[u] : 0u;
        const JobFlags jf = flags_of(a, job);
        const Src src = a.batch ? src_of(a.jobs[job]) : src_of(a);
        if (a.batch) sk.set_job(a, job);
        uint4 c0 = pf;
        const bool swap = (c0.y & kAxisBit) != 0;  // sweeping axis in bit 31 of the R count
        c0.y &= ~kAxisBit;
        uint32_t nx = 0;
        uint4 nrec = make_uint4(0, 0, 0, 0);
        if (dyn && threadIdx.x == 0) nx = atomicAdd(taken, 1u);
        const uint32_t un = dyn ? 0u : unit_of(i + 1, blockIdx.x, G, SP);
        auto prefetch = [&]() {
            if (dyn) {
                if (threadIdx.x == 0 && nx < nu) nrec = a.med_lpt[nx];
            } else if (un < nu) {
                pf = a.med[un];
            }
        };
        sk.begin(a, slot);
        run_lds_unit<NT, Q, TC, MODE>(a, src, jf.dist, jf.e2, L, 1, [&](int, int) { return c0; },
                                      prefetch, sk, swap);
        sk.end(a, slot);  // ends with a workgroup barrier: s_u and s_rec are free
        if (dyn) {
            if (threadIdx.x == 0) {
                s_u = nx;
                s_rec = nrec;
            }
            __syncthreads();
            u = s_u;
            pf = s_rec;
        } else {
            u = unit_of(++i, blockIdx.x, G, SP);
        }
    }
    sk.finish(a, blockIdx.x * (NT / kWave) + threadIdx.x / kWave);
}

// ---------------------------------------------------------------------------
// k_med_order (single join, one workgroup): the medium records in
// decreasing order of their entry counts, by a counting sort over 64
// classes of 32 entries, into med_lpt.  Largest first, the tiles claimed
// last are the shortest, so the workgroups finish together.
// ---------------------------------------------------------------------------
constexpr int kOrderNT = 1024;
constexpr int kOrderClasses = 64;

__device__ __forceinline__ uint32_t med_class(const uint4& r) {
    const uint32_t n = (r.y & ~kAxisBit) + r.w;  // <= med_cap <= kMedE
    const uint32_t c = (n - 1u) / 32u;
    return (uint32_t)kOrderClasses - 1u - (c < (uint32_t)kOrderClasses ? c : (uint32_t)kOrderClasses - 1u);
}

__global__ __launch_bounds__(kOrderNT) void k_med_order(Args a) {
    __shared__ uint32_t s_cnt[kOrderClasses];
    const uint32_t nm = min(a.ctr[kMedCount], (uint32_t)a.cap_med);
    const int tid = threadIdx.x;
    if (tid < kOrderClasses) s_cnt[tid] = 0u;
    __syncthreads();
    for (uint32_t m = tid; m < nm; m += kOrderNT) atomicAdd(&s_cnt[med_class(a.med[m])], 1u);
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0;
        for (int c = 0; c < kOrderClasses; ++c) {
            const uint32_t v = s_cnt[c];
            s_cnt[c] = acc;
            acc += v;
        }
    }
    __syncthreads();
    for (uint32_t m = tid; m < nm; m += kOrderNT) {
        const uint4 r = a.med[m];
        a.med_lpt[atomicAdd(&s_cnt[med_class(r)], 1u)] = r;
    }
}

// ---------------------------------------------------------------------------
// k_plain_tiles (baseline): one workgroup per tile, slot = tile id.
// ---------------------------------------------------------------------------
template <int NT, int Q, int MODE>
__global__ __launch_bounds__(NT) void k_plain_tiles(Args a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int TC = tc_for(NT * Q, false);
    const LdsLayout L = carve(smem, NT, NT * Q, TC);
    Sink<MODE, true> sk = make_sink<MODE>(L);
    // one workgroup per tile; a grid-stride loop only when K*K exceeds the grid
    for (int64_t t = blockIdx.x; t < a.C; t += gridDim.x) {
        const uint32_t nr = a.offR[t + 1] - a.offR[t];
        const uint32_t ns = a.offS[t + 1] - a.offS[t];
        if (nr == 0 || ns == 0) continue;
        if (nr + ns > (uint32_t)(NT * Q)) {
            if (MODE == kCount && threadIdx.x == 0) append_dense(a, (uint32_t)t, nr, ns);
            continue;
        }
        const uint4 ti = make_uint4(a.offR[t], nr, a.offS[t], ns);
        sk.begin(a, t);
        run_lds_unit<NT, Q, TC, MODE>(a, src_of(a), a.dist, a.e2, L, 1, [&](int, int) { return ti; },
                                      [] {}, sk);
        sk.end(a, t);
    }
    sk.finish(a, blockIdx.x * (NT / kWave) + threadIdx.x / kWave);
}

// ---------------------------------------------------------------------------
// Dense tiles: sort each list into the global dense buffer ...
// ---------------------------------------------------------------------------
__device__ void bitonic_lds(unsigned long long* k, int P) {
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = ((lo & size) == 0);
                const unsigned long long x = k[lo], y = k[hi];
                if ((x > y) == up) {
                    k[lo] = y;
                    k[hi] = x;
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ float lower_edge(const float4& b, bool y) { return y ? b.y : b.x; }

__global__ __launch_bounds__(kDenseSortNT) void k_dense_sort(Args a) {
    __shared__ unsigned long long keys[kDenseSortMax];
    __shared__ uint32_t s_cls[4];
    const uint32_t nd = min(a.ctr[kDenseCount], (uint32_t)a.cap_dense);
    for (uint32_t seg = blockIdx.x; seg < 2 * nd; seg += gridDim.x) {
        const uint4 dd = a.dense[seg >> 1];
        const uint32_t job = a.batch ? a.djob[seg >> 1] : 0u;
        const Src sj = a.batch ? src_of(a.jobs[job]) : src_of(a);
        const bool gbda = flags_of(a, job).gbda != 0;
        const bool sideS = seg & 1;
        const bool swap = (dd.x & kAxisBit) != 0;  // swept along y: sort by y_l
        const uint32_t tile = dd.x & ~kAxisBit;
        const uint32_t src = sideS ? sj.offS[tile] : sj.offR[tile];
        const uint32_t L = sideS ? dd.w : dd.z;
        const uint32_t dst = dd.y + (sideS ? dd.z : 0u);
        const float4* ent = sideS ? sj.entS : sj.entR;
        const uint32_t* eid = sideS ? sj.idS : sj.idR;
        // key: (GBDA class,) order key of the lower edge, position
        auto key_of = [&](uint32_t i) -> unsigned long long {
            const unsigned long long ok = order_key(lower_edge(ent[src + i], swap));
            return gbda ? ((unsigned long long)gbda_class(eid[src + i]) << 62) | (ok << 30) | i
                        : (ok << 32) | i;
        };
        const unsigned long long pos_mask = gbda ? 0x3FFFFFFFull : 0xFFFFFFFFull;
        if (gbda) {  // class group starts of this list
            if (threadIdx.x < 4) s_cls[threadIdx.x] = 0u;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < L; i += blockDim.x)
                atomicAdd(&s_cls[gbda_class(eid[src + i])], 1u);
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t* g = a.dgrp + (size_t)(seg >> 1) * 10 + (sideS ? 5 : 0);
                uint32_t acc = 0;
                for (int c = 0; c < 4; ++c) {
                    g[c] = acc;
                    acc += s_cls[c];
                }
                g[4] = acc;
            }
        }
        const unsigned long long* fin;  // final sorted keys (low 32 bits = position)
        if (L <= (uint32_t)kDenseSortMax) {
            int P = 1;
            while (P < (int)L) P <<= 1;
            for (int i = threadIdx.x; i < P; i += blockDim.x) keys[i] = i < (int)L ? key_of(i) : ~0ull;
            __syncthreads();
            bitonic_lds(keys, P);
            fin = keys;
        } else if (L <= 2u * (uint32_t)kDenseSortMax) {
            // two sorted runs: the first kDenseSortMax keys, kept in global
            // memory, and the rest, kept in LDS.  A key's place in the merged
            // order is its index in its run plus the number of smaller keys
            // in the other run (keys are distinct: they carry the position),
            // and its entry is written there at once: a list of up to twice
            // the LDS size needs no merge pass through global memory.
            unsigned long long* A = a.dtmp + 2ull * dst;
            const uint32_t n2 = L - (uint32_t)kDenseSortMax;
            for (int i = threadIdx.x; i < kDenseSortMax; i += blockDim.x) keys[i] = key_of((uint32_t)i);
            __syncthreads();
            bitonic_lds(keys, kDenseSortMax);
            for (int i = threadIdx.x; i < kDenseSortMax; i += blockDim.x) A[i] = keys[i];
            __syncthreads();
            int P = 1;
            while (P < (int)n2) P <<= 1;
            for (int i = threadIdx.x; i < P; i += blockDim.x)
                keys[i] = i < (int)n2 ? key_of((uint32_t)kDenseSortMax + (uint32_t)i) : ~0ull;
            __syncthreads();
            bitonic_lds(keys, P);
            auto place = [&](unsigned long long v, uint32_t at) {
                const uint32_t q = (uint32_t)(v & pos_mask);
                const float4 b = ent[src + q];
                a.dbox[dst + at] = swap ? make_float4(b.y, b.x, b.w, b.z) : b;
                a.didf[dst + at] = eid[src + q];
            };
            for (uint32_t i = threadIdx.x; i < (uint32_t)kDenseSortMax; i += blockDim.x) {
                const unsigned long long v = A[i];
                uint32_t b0 = 0, b1 = n2;  // keys of the LDS run below v
                while (b0 < b1) {
                    const uint32_t m = (b0 + b1) >> 1;
                    if (keys[m] < v) b0 = m + 1;
                    else b1 = m;
                }
                place(v, i + b0);
            }
            for (uint32_t j = threadIdx.x; j < n2; j += blockDim.x) {
                const unsigned long long v = keys[j];
                uint32_t b0 = 0, b1 = (uint32_t)kDenseSortMax;  // keys of the global run below v
                while (b0 < b1) {
                    const uint32_t m = (b0 + b1) >> 1;
                    if (A[m] < v) b0 = m + 1;
                    else b1 = m;
                }
                place(v, j + b0);
            }
            __syncthreads();
            continue;
        } else {
            // sorted runs of kDenseSortMax in LDS, then merge passes in global
            // memory (rank of each key in the partner run by binary search;
            // keys are distinct because they carry the position).
            unsigned long long* A = a.dtmp + 2ull * dst;
            unsigned long long* Bf = A + L;
            for (uint32_t c0 = 0; c0 < L; c0 += kDenseSortMax) {
                const int n = (int)min((uint32_t)kDenseSortMax, L - c0);
                for (int i = threadIdx.x; i < kDenseSortMax; i += blockDim.x)
                    keys[i] = i < n ? key_of(c0 + (uint32_t)i) : ~0ull;
                __syncthreads();
                bitonic_lds(keys, kDenseSortMax);
                for (int i = threadIdx.x; i < n; i += blockDim.x) A[c0 + i] = keys[i];
                __syncthreads();
            }
            for (uint32_t wdt = kDenseSortMax; wdt < L; wdt <<= 1) {
                for (uint32_t i = threadIdx.x; i < L; i += blockDim.x) {
                    const uint32_t run = i / (2 * wdt);
                    const uint32_t lo = run * 2 * wdt;
                    const uint32_t mid = min(lo + wdt, L), hi = min(lo + 2 * wdt, L);
                    const unsigned long long v = A[i];
                    uint32_t olo, ohi, mine;
                    if (i < mid) {
                        olo = mid;
                        ohi = hi;
                        mine = i - lo;
                    } else {
                        olo = lo;
                        ohi = mid;
                        mine = i - mid;
                    }
                    uint32_t b0 = olo, b1 = ohi;
                    while (b0 < b1) {
                        const uint32_t m = (b0 + b1) >> 1;
                        if (A[m] < v) b0 = m + 1;
                        else b1 = m;
                    }
                    Bf[lo + mine + (b0 - olo)] = v;
                }
                __syncthreads();
                unsigned long long* tmp = A;
                A = Bf;
                Bf = tmp;
            }
            fin = A;
        }
        for (uint32_t i = threadIdx.x; i < L; i += blockDim.x) {
            const uint32_t q = (uint32_t)(fin[i] & pos_mask);
            const float4 b = ent[src + q];
            a.dbox[dst + i] = swap ? make_float4(b.y, b.x, b.w, b.z) : b;
            a.didf[dst + i] = eid[src + q];
        }
        __syncthreads();
    }
}

// ... plan the dense units (one block) ...
__global__ __launch_bounds__(1024) void k_dense_plan(Args a) {
    __shared__ uint32_t lds[1024 / kWave + 1];
    const uint32_t nd = min(a.ctr[kDenseCount], (uint32_t)a.cap_dense);
    const int lane = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    uint32_t carry = 0;
    for (uint32_t d0 = 0; d0 < nd; d0 += blockDim.x) {
        const uint32_t d = d0 + threadIdx.x;
        uint32_t v = 0;
        if (d < nd) {
            const uint4 dd = a.dense[d];
            const uint32_t n = dd.z + dd.w;
            const JobFlags jf = flags_of(a, a.batch ? a.djob[d] : 0u);
            if (jf.gbda) {
                // units of the 9 mini-joins (R class X x S class Y), each split
                // into ranges of split_tau pivots; units before each in dmj
                const uint32_t* g = a.dgrp + (size_t)d * 10;
                uint32_t* mj = a.dmj + (size_t)d * 10;
                for (int j = 0; j < 9; ++j) {
                    mj[j] = v;
                    const int X = kMiniJoin[j][0], Y = kMiniJoin[j][1];
                    const uint32_t nx = g[X + 1] - g[X], ny = g[5 + Y + 1] - g[5 + Y];
                    if (nx && ny) v += (nx + ny + (uint32_t)jf.split_tau - 1u) / (uint32_t)jf.split_tau;
                }
                mj[9] = v;
            } else {
                v = jf.plain ? 1u : (n + (uint32_t)jf.split_tau - 1u) / (uint32_t)jf.split_tau;
            }
        }
        uint32_t inc = v;
        for (int s = 1; s < kWave; s <<= 1) {
            const uint32_t t = __shfl_up(inc, s, kWave);
            if (lane >= s) inc += t;
        }
        if (lane == kWave - 1) lds[w] = inc;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t acc = 0;
            for (int q = 0; q < nw; ++q) {
                const uint32_t x = lds[q];
                lds[q] = acc;
                acc += x;
            }
            lds[nw] = acc;
        }
        __syncthreads();
        if (d < nd) a.dprefix[d] = carry + lds[w] + inc - v;
        carry += lds[nw];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.dprefix[nd] = carry;
        a.ctr[kDenseUnits] = carry;
        if ((int64_t)carry > a.cap_dunits) atomicOr(&a.st->flags, kStatCapacity);
    }
}

// ... and sweep them: one unit = a contiguous range of pivots of one tile.
struct GlobAcc {
    const float4* bxs;
    const uint32_t* idf;
    int base, nr, ns;  // R entries at [base, base+nr), S at [base+nr, base+nr+ns)
    __device__ float4 box(int j) const { return bxs[j]; }
    __device__ uint32_t id(int j) const { return idf[j]; }
    __device__ bool setup(int p, bool& isR, int& j, int& jend, float& pxl, float& pxu, float& pyl,
                          float& pyu, uint32_t& pid) const {
        const int e = base + p;  // pivots: R entries then S entries
        const float4 b = bxs[e];
        pxl = b.x;
        pxu = b.z;
        pyl = b.y;
        pyu = b.w;
        pid = idf[e];
        auto X = [&](int q) { return bxs[q].x; };
        isR = p < nr;
        const int lo = isR ? base + nr : base;
        const int hi = isR ? base + nr + ns : base + nr;
        j = search_x(X, lo, hi, b.x, isR);
        jend = hi;
        return true;
    }
};

// One GBDA mini-join of a dense tile: R class group [rb, rb+nr), S class
// group [sb, sb+ns) of the sorted dense buffer; pivots: R group, then S group.
struct GbdaAcc {
    const float4* bxs;
    const uint32_t* idf;
    int rb, nr, sb, ns;
    __device__ float4 box(int j) const { return bxs[j]; }
    __device__ uint32_t id(int j) const { return idf[j]; }
    __device__ bool setup(int p, bool& isR, int& j, int& jend, float& pxl, float& pxu, float& pyl,
                          float& pyu, uint32_t& pid) const {
        isR = p < nr;
        const int e = isR ? rb + p : sb + (p - nr);
        const float4 b = bxs[e];
        pxl = b.x;
        pxu = b.z;
        pyl = b.y;
        pyu = b.w;
        pid = idf[e];
        auto X = [&](int q) { return bxs[q].x; };
        const int lo = isR ? sb : rb;
        const int hi = isR ? sb + ns : rb + nr;
        j = search_x(X, lo, hi, b.x, isR);
        jend = hi;
        return true;
    }
};

template <int MODE>
__global__ __launch_bounds__(kDenseNT) void k_dense_sweep(Args a) {
    __shared__ unsigned long long wbuf[(kDenseNT / kWave) * kWaveBuf];
    __shared__ uint32_t s_acc;
    __shared__ uint32_t s_next;
    const uint32_t wg = blockIdx.x * (kDenseNT / kWave) + threadIdx.x / kWave;
    Sink<MODE, true> sk;
    sk.buf = wbuf + (threadIdx.x / kWave) * kWaveBuf;
    sk.s_acc = &s_acc;
    sk.bufcap = kWaveBuf;
    sk.init(wg);
    const uint32_t nd = min(a.ctr[kDenseCount], (uint32_t)a.cap_dense);
    const uint32_t nu = min(a.ctr[kDenseUnits], (uint32_t)a.cap_dunits);
    const uint32_t G = gridDim.x, SP = a.batch ? kDenseStripe : 1u;
    // a single join's workgroups claim the units from a counter (their scans
    // differ widely in length); thread 0 claims the next one as a unit starts
    __shared__ uint32_t s_u;
    const bool dyn = !a.batch;
    uint32_t* taken = &a.ctr[MODE == kWrite ? kDenseTaken2 : kDenseTaken];
    uint32_t u;
    if (dyn) {
        if (threadIdx.x == 0) s_u = atomicAdd(taken, 1u);
        __syncthreads();
        u = s_u;
    } else {
        u = unit_of(0, blockIdx.x, G, SP);
    }
    for (uint32_t i = 0; u < nu; ++i) {
        uint32_t nx = 0;
        if (dyn && threadIdx.x == 0) nx = atomicAdd(taken, 1u);
        // dense tile of unit u: last d with dprefix[d] <= u
        uint32_t lo = 0, hi = nd;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.dprefix[mid] <= u) lo = mid;
            else hi = mid;
        }
        const uint4 dd = a.dense[lo];
        const int64_t slot = a.base_dense + u;
        const uint32_t job = a.batch ? a.djob[lo] : 0u;
        const JobFlags jf = flags_of(a, job);
        sk.begin(a, slot);
        if (a.batch) sk.set_job(a, job);
        if (threadIdx.x == 0) s_next = 0u;
        __syncthreads();
        if (jf.gbda) {
            // mini-join j of the tile and its range of pivots
            const uint32_t r = u - a.dprefix[lo];
            const uint32_t* mj = a.dmj + (size_t)lo * 10;
            int jm = 0;
            while (jm < 8 && mj[jm + 1] <= r) ++jm;
            const int X = kMiniJoin[jm][0], Y = kMiniJoin[jm][1];
            const uint32_t* g = a.dgrp + (size_t)lo * 10;
            const int nx = (int)(g[X + 1] - g[X]), ny = (int)(g[5 + Y + 1] - g[5 + Y]);
            const int p0 = (int)(r - mj[jm]) * jf.split_tau;
            const int p1 = min(p0 + jf.split_tau, nx + ny);
            GbdaAcc acc{a.dbox, a.didf, (int)(dd.y + g[X]), nx, (int)(dd.y + dd.z + g[5 + Y]), ny};
            sweep_pivots<MODE, true, false>(a, acc, p0, p1, &s_next, sk, jf.dist, jf.e2);
        } else {
            const int n = (int)(dd.z + dd.w);
            int p0 = 0, p1 = n;
            if (!jf.plain) {
                p0 = (int)(u - a.dprefix[lo]) * jf.split_tau;
                p1 = min(p0 + jf.split_tau, n);
            }
            GlobAcc acc{a.dbox, a.didf, (int)dd.y, (int)dd.z, (int)dd.w};
            sweep_pivots<MODE, true>(a, acc, p0, p1, &s_next, sk, jf.dist, jf.e2);
        }
        sk.end(a, slot);  // ends with a workgroup barrier: s_u is free
        if (dyn) {
            if (threadIdx.x == 0) s_u = nx;
            __syncthreads();
            u = s_u;
        } else {
            u = unit_of(i + 1, blockIdx.x, G, SP);
        }
    }
    sk.finish(a, wg);
}

// ---------------------------------------------------------------------------
// Single-pass output compaction: chunk fill levels were scanned into output
// offsets (fills[g] = first output slot of chunk g, fills[total] = pairs
// stored); one wavefront copies one chunk.
// ---------------------------------------------------------------------------
constexpr int kCompactNT = 256;

__global__ __launch_bounds__(kCompactNT) void k_compact(Args a) {
    const int64_t nch = (int64_t)kRegions * a.sc_nch;
    const int64_t g = (int64_t)blockIdx.x * (kCompactNT / kWave) + threadIdx.x / kWave;
    if (g >= nch) return;
    const uint32_t o0 = a.sc_fills[g], o1 = a.sc_fills[g + 1];
    const unsigned long long* src = a.sc_buf + (size_t)g * kChunkP;
    for (uint32_t q = lane_id(); q < o1 - o0; q += kWave) {
        const unsigned long long idx = (unsigned long long)o0 + q;
        if (idx < (unsigned long long)a.capacity) a.out[idx] = src[q];
    }
}

__global__ void k_reset(uint32_t* ctr, DevStatus* st, uint32_t* sc_ctr,
                        unsigned long long* sc_total) {
    if (threadIdx.x < kNumCtr) ctr[threadIdx.x] = 0u;
    if (sc_ctr && threadIdx.x < kRegions) sc_ctr[threadIdx.x] = 0u;
    if (sc_total && threadIdx.x < kTotals) sc_total[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) {
        st->n_pairs = 0ull;
        st->m_total = 0ull;
        st->flags = 0u;
        st->n_dense = 0u;
        st->n_units = 0u;
        st->n_cand = 0ull;
    }
}

// Single pass: the exact pair count is the sum of the per-wave totals; with
// no scratch overflow it must equal the pairs stored (m_total holds those).
__global__ void k_finish(const uint32_t* ctr, DevStatus* st, const DevStatus* stR,
                         const DevStatus* stS, const unsigned long long* sc_total) {
    st->n_dense = ctr[kDenseCount];
    st->n_units = ctr[kUnitsWritten] + ctr[kMedCount];
    st->flags |= stR->flags | stS->flags;
    if (sc_total) {
        unsigned long long t = 0;
        for (int i = 0; i < kTotals; ++i) t += sc_total[i];
        st->n_pairs = t;
        if (!(st->flags & kStatScratch) && t != st->m_total) st->flags |= kStatInternal;
    }
}

// Batch of joins: clear the shared counters and every join's fill counter
// and status (grid-stride over the joins).
__global__ void k_batch_reset(uint32_t* ctr, DevStatus* st, unsigned long long* totals,
                              uint32_t* sc_ctr, const Job* jobs, int n_jobs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kNumCtr) ctr[i] = 0u;
    if (i < kTotals) totals[i] = 0ull;
    if (sc_ctr && i < kRegions) sc_ctr[i] = 0u;
    if (i == 0) *st = DevStatus{};
    for (int j = i; j < n_jobs; j += gridDim.x * blockDim.x) {
        *jobs[j].fill = 0ull;
        *jobs[j].st = DevStatus{};
    }
}

// Batch compaction: every scratch chunk reserved in the run (the first
// sc_ctr[r] of region r) goes to the output region of its join, at a
// position reserved with one atomic on the join's fill counter; pairs past
// the join's capacity are counted, not stored.  One wavefront per chunk,
// grid-strided.
__global__ __launch_bounds__(kCompactNT) void k_compact_batch(Args a) {
    const uint32_t per = kCompactNT / kWave;
    const uint32_t nch = (uint32_t)(kRegions * a.sc_nch);
    for (uint32_t g = blockIdx.x * per + threadIdx.x / kWave; g < nch; g += gridDim.x * per) {
        const uint32_t r = g / (uint32_t)a.sc_nch, k = g % (uint32_t)a.sc_nch;
        if (k >= a.sc_ctr[r]) continue;
        const uint32_t f = a.sc_fills[g];
        const Job& J = a.jobs[a.sc_job[g]];
        unsigned long long b = 0;
        if (lane_id() == 0) b = atomicAdd(J.fill, (unsigned long long)f);
        b = __shfl(b, 0, kWave);
        const unsigned long long* src = a.sc_buf + (size_t)g * kChunkP;
        for (uint32_t q = lane_id(); q < f; q += kWave)
            if (b + q < (unsigned long long)J.capacity) J.out[b + q] = src[q];
    }
}

// ... and after the join: every join's pair count (its fill counter) and
// status (its partitions' flags and the flags of the shared lists).
__global__ void k_batch_finish(const DevStatus* st, const Job* jobs, int n_jobs) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_jobs) return;
    const Job& J = jobs[j];
    J.st->n_pairs = *J.fill;
    J.st->flags |= J.stR->flags | J.stS->flags | st->flags;
}

template <class F>
hipError_t set_lds(F* kern, size_t lds) {
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

template <int NT, int Q, int MODE>
hipError_t launch_plain(const Args& a, hipStream_t s) {
    const size_t lds = lds_bytes(NT, NT * Q, tc_for(NT * Q, false));
    hipError_t e = set_lds(k_plain_tiles<NT, Q, MODE>, lds);
    if (e != hipSuccess) return e;
    // HIP limits a grid to fewer than 2^32 work-items
    const int64_t max_blocks = ((int64_t)1 << 31) / NT;
    const int64_t nb = a.C < max_blocks ? a.C : max_blocks;
    hipLaunchKernelGGL((k_plain_tiles<NT, Q, MODE>), dim3((unsigned)nb), dim3(NT), lds, s, a);
    return hipGetLastError();
}

// grid = min(bound, resident workgroups): persistent workgroups
template <class K>
hipError_t launch_persistent(K* kern, int nt, size_t lds, int64_t bound, int num_cus, int& per_cu,
                             const Args& a, hipStream_t s) {
    if (bound <= 0) return hipSuccess;
    if (per_cu == 0) {
        hipError_t e = set_lds(kern, lds);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
    }
    const int64_t grid = std::min<int64_t>(bound, (int64_t)num_cus * per_cu);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(nt), lds, s, a);
    return hipGetLastError();
}

template <int NT, int Q, int MODE>
hipError_t launch_medium(const Args& a, int64_t bound, int num_cus, hipStream_t s) {
    static int per_cu = 0;  // resident workgroups per CU (computed once per instantiation)
    return launch_persistent(k_lds_medium<NT, Q, MODE>, NT, lds_bytes(NT, NT * Q, tc_for(NT * Q, false)),
                             bound, num_cus, per_cu, a, s);
}

template <int NT, int Q, int MODE, bool BATCH = false>
hipError_t launch_span(const Args& a, int64_t bound, int num_cus, hipStream_t s) {
    static int per_cu = 0;
    return launch_persistent(k_span_units<NT, Q, MODE, BATCH>, NT, span_lds_bytes(NT, NT * Q), bound,
                             num_cus, per_cu, a, s);
}

// small-tile units: block threads and entries per unit (see lds_unit_entries)
template <int MODE>
hipError_t launch_small(const Args& a, int block, int64_t bound, int num_cus, hipStream_t s) {
    switch (block) {
        case 64: return launch_span<64, 4, MODE>(a, bound, num_cus, s);
        case 128: return launch_span<128, 8, MODE>(a, bound, num_cus, s);
        case 512: return launch_span<512, 4, MODE>(a, bound, num_cus, s);
        default: return launch_span<256, 4, MODE>(a, bound, num_cus, s);
    }
}

constexpr const char* mode_tag(int mode, const char* count, const char* write, const char* single) {
    return mode == kCount ? count : (mode == kWrite ? write : single);
}

// one pass (count, write or single) over every unit
template <int MODE>
hipError_t join_pass(const Args& a0, const JoinParams& p, const JoinWork& w, hipStream_t s) {
    hipError_t e = hipSuccess;
    Args a = a0;
    a.cls = 0;
    if (p.plain) {
        ProfRange pr(mode_tag(MODE, "k_plain_tiles_count", "k_plain_tiles_write",
                              "k_plain_tiles_single"), s);
        e = launch_plain<256, 4, MODE>(a, s);
    } else {
        {
            ProfRange pr(mode_tag(MODE, "k_span_units_count", "k_span_units_write",
                                  "k_span_units_single"), s);
            e = launch_small<MODE>(a, p.block, std::min<int64_t>(p.units_bound, w.cap_units),
                                   w.num_cus, s);
        }
        if (e == hipSuccess) {
            a.cls = 1;
            ProfRange pr(mode_tag(MODE, "k_lds_medium_count", "k_lds_medium_write",
                                  "k_lds_medium_single"), s);
            // medium tiles up to 1024 entries: a half-size slab, twice the
            // workgroups per CU
            const int64_t mb = std::min<int64_t>(p.med_bound, w.cap_med);
            e = p.med_cap <= 1024 ? launch_medium<256, 4, MODE>(a, mb, w.num_cus, s)
                                  : launch_medium<kMedNT, kMedE / kMedNT, MODE>(a, mb, w.num_cus, s);
        }
    }
    if (e != hipSuccess) return e;
    a.cls = 2;
    ProfRange pr(mode_tag(MODE, "k_dense_sweep_count", "k_dense_sweep_write",
                          "k_dense_sweep_single"), s);
    hipLaunchKernelGGL(k_dense_sweep<MODE>, dim3(w.num_cus * 4), dim3(kDenseNT), 0, s, a);
    return hipGetLastError();
}

}  // namespace

int lds_unit_entries(int block) { return block == 128 ? 1024 : block * 4; }
int batch_block() { return kBatchBlock; }
int lds_unit_tiles(int block) { return kSpanTQ * block - 1; }
int lds_medium_entries() { return kMedE; }
int batch_medium_entries() { return kBatchMedE; }
int64_t classify_blocks(int64_t C) { return (C + kClassChunk - 1) / kClassChunk; }
int64_t classify_chunk_tiles() { return kClassChunk; }

// Slots of the per-unit count array: small units, medium tiles, dense units
// (tuned) or one per tile plus dense units (plain).
int64_t join_slots(const JoinParams& p, const JoinWork& w) {
    return (p.plain ? p.C : w.cap_units + w.cap_med) + w.cap_dunits;
}

// Kernel arguments of one join over the work lists of w.
Args join_args(const Part& R, const Part& S, const JoinParams& p, const JoinWork& w) {
    Args a{};
    a.offR = R.off;
    a.offS = S.off;
    a.entR = R.entb;
    a.entS = S.entb;
    a.idR = R.enti;
    a.idS = S.enti;
    a.C = p.C;
    a.small_cap = p.small_cap;
    a.unit_cap = p.unit_cap;
    a.med_cap = p.med_cap;
    a.split_tau = p.split_tau;
    a.plain = p.plain ? 1 : 0;
    a.unit_tiles = p.unit_tiles;
    a.uspan = w.uspan;
    a.units = w.units;
    a.med = w.med;
    a.med_lpt = p.plain ? nullptr : w.med_lpt;
    a.dense = w.dense;
    a.dprefix = w.dense_unit_prefix;
    a.cap_units = w.cap_units;
    a.cap_med = w.cap_med;
    a.cap_dense = w.cap_dense;
    a.cap_dent = w.cap_dent;
    a.cap_dunits = w.cap_dunits;
    a.dbox = w.dbox;
    a.didf = w.didf;
    a.dtmp = w.dtmp;
    a.ucnt = w.ucnt;
    a.base_med = p.plain ? 0 : w.cap_units;
    a.base_dense = p.plain ? p.C : w.cap_units + w.cap_med;
    a.ctr = w.ctr;
    a.st = w.st;
    a.stR = R.st;
    a.stS = S.st;
    a.axis_model = (p.axis_model && !p.plain) ? 1 : 0;
    a.gbda = (p.gbda && !p.plain) ? 1 : 0;
    a.dist = p.dist ? 1 : 0;
    a.e2 = p.e2;
    a.dgrp = w.dgrp;
    a.dmj = w.dmj;
    a.medt = w.medt;
    a.gd = R.gd;
    a.bl = R.bl;
    return a;
}

hipError_t run_join(const Part& R, const Part& S, const JoinParams& p, JoinWork& w, sj_pair* out,
                    int64_t capacity, hipStream_t s) {
    Args a = join_args(R, S, p, w);
    a.out = (unsigned long long*)out;
    a.capacity = out ? capacity : 0;
    const bool single = p.single && !p.plain && !p.count_only && w.sc_nch > 0;
    a.writeback = (!single && !p.count_only) ? 1 : 0;
    if (single) {
        a.sc_buf = w.sc_buf;
        a.sc_fills = w.sc_fills;
        a.sc_ctr = w.sc_ctr;
        a.sc_total = w.sc_total;
        a.sc_nch = w.sc_nch;
    }
    const int64_t nslots = join_slots(p, w);
    const int64_t nchunks = (int64_t)kRegions * w.sc_nch;

    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, w.ctr, w.st, single ? w.sc_ctr : nullptr,
                       single ? w.sc_total : nullptr);
    hipError_t e = single ? launch_fill_u32(w.sc_fills, 0u, nchunks + 1, s)
                          : launch_fill_u32(w.ucnt, 0u, nslots + 1, s);
    if (e != hipSuccess) return e;
    if (p.plain) {
        // the plain counting pass lists the dense tiles itself
        ProfRange pr("k_plain_tiles_count", s);
        e = launch_plain<256, 4, kCount>(a, s);
        if (e != hipSuccess) return e;
    } else {
        ProfRange pr("k_classify", s);
        hipLaunchKernelGGL(k_classify, dim3((unsigned)classify_blocks(p.C)), dim3(kClassNT), 0, s,
                           a);
    }
    if (a.axis_model) {
        ProfRange pr("k_axis", s);
        hipLaunchKernelGGL(k_axis, dim3(w.num_cus * 4), dim3(kAxisNT), 0, s, a);
    }
    {
        ProfRange pr("k_dense_sort", s);
        hipLaunchKernelGGL(k_dense_sort, dim3(w.num_cus * 2), dim3(kDenseSortNT), 0, s, a);
    }
    hipLaunchKernelGGL(k_dense_plan, dim3(1), dim3(1024), 0, s, a);
    if (a.med_lpt) {
        ProfRange pr("k_med_order", s);
        hipLaunchKernelGGL(k_med_order, dim3(1), dim3(kOrderNT), 0, s, a);
    }
    if (single) {
        e = join_pass<kSingle>(a, p, w, s);
        if (e != hipSuccess) return e;
        {
            ProfRange pr("k_scan_chunks", s);
            e = scan_u32(w.sc_fills, nchunks, w.scan_tmp, &w.st->m_total, w.st, s);
            if (e != hipSuccess) return e;
        }
        ProfRange pr("k_compact", s);
        const int64_t per = kCompactNT / kWave;
        hipLaunchKernelGGL(k_compact, dim3((unsigned)((nchunks + per - 1) / per)), dim3(kCompactNT),
                           0, s, a);
    } else {
        if (p.plain) {
            ProfRange pr("k_dense_sweep_count", s);
            hipLaunchKernelGGL(k_dense_sweep<kCount>, dim3(w.num_cus * 4), dim3(kDenseNT), 0, s, a);
        } else {
            e = join_pass<kCount>(a, p, w, s);
            if (e != hipSuccess) return e;
        }
        {
            ProfRange pr("k_scan_pairs", s);
            e = scan_u32(w.ucnt, nslots, w.scan_tmp, &w.st->n_pairs, w.st, s);
            if (e != hipSuccess) return e;
        }
        if (!p.count_only) {
            e = join_pass<kWrite>(a, p, w, s);
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1), 0, s, w.ctr, w.st, R.st, S.st,
                       single ? w.sc_total : nullptr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batch of joins.  The classification of every join appends its records,
// tagged with the join's index, to one set of work lists; one sequence of
// join launches consumes the records of all joins (the joins' units are the
// work queue of the persistent workgroups).  Pairs go to scratch chunks of
// one join each and k_compact_batch moves the chunks into the joins' output
// regions (kSingle); count-only batches add per-wave counts to the joins'
// fill counters (kAppend).
// ---------------------------------------------------------------------------
namespace {
Args batch_args(BatchWork& b) {
    Args a{};
    JoinWork& w = b.w;
    a.batch = 1;
    a.jobs = b.jobs;
    a.ujob = b.ujob;
    a.mjob = b.mjob;
    a.djob = b.djob;
    a.uspan = w.uspan;
    a.units = w.units;
    a.med = w.med;
    a.medt = w.medt;
    a.dense = w.dense;
    a.dprefix = w.dense_unit_prefix;
    a.cap_units = w.cap_units;
    a.cap_med = w.cap_med;
    a.cap_dense = w.cap_dense;
    a.cap_dent = w.cap_dent;
    a.cap_dunits = w.cap_dunits;
    a.dbox = w.dbox;
    a.didf = w.didf;
    a.dtmp = w.dtmp;
    a.dgrp = w.dgrp;
    a.dmj = w.dmj;
    a.ctr = w.ctr;
    a.st = w.st;
    a.sc_total = w.sc_total;  // pairs per work class
    return a;
}
}  // namespace

hipError_t batch_reset(BatchWork& b, int n_jobs, hipStream_t s) {
    const int nb = std::max(1, std::min(64, (n_jobs + 255) / 256));
    hipLaunchKernelGGL(k_batch_reset, dim3(nb), dim3(256), 0, s, b.w.ctr, b.w.st, b.w.sc_total,
                       b.w.sc_ctr, b.jobs, n_jobs);
    return hipGetLastError();
}

// Scratch chunks per region for a batch run: the pairs the outputs can hold
// with 25% headroom, plus the partly filled chunks that waves close when
// they move on to another join (at most one per wave and stripe, estimated
// from the list bounds and capped: a run that outgrows the scratch reports
// it and the batch grows the scratch from the counters).
int64_t batch_scratch_chunks(int64_t pairs, int64_t units, int64_t med, int num_cus) {
    const int64_t waves = (int64_t)kBatchBlock / kWave;
    int64_t partial = waves * (units / kSpanStripe + med / kMedStripe) + 3LL * num_cus * 32;
    partial = std::min<int64_t>(partial, 65536);
    const int64_t full = (pairs + pairs / 4) / kChunkP;
    return (full + partial + kRegions - 1) / kRegions + 2;
}

hipError_t batch_scratch_used(const BatchWork& b, int64_t* max_chunks) {
    uint32_t c[kRegions];
    *max_chunks = 0;
    if (!b.w.sc_ctr) return hipSuccess;
    hipError_t e = hipMemcpy(c, b.w.sc_ctr, sizeof(c), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    for (int r = 0; r < kRegions; ++r) *max_chunks = std::max<int64_t>(*max_chunks, c[r]);
    return hipSuccess;
}

hipError_t batch_classify(BatchWork& b, const Part& R, const Part& S, const JoinParams& p,
                          uint32_t jid, hipStream_t s) {
    Args a = join_args(R, S, p, b.w);
    a.batch = 1;
    a.jid = jid;
    a.jobs = b.jobs;
    a.ujob = b.ujob;
    a.mjob = b.mjob;
    a.djob = b.djob;
    ProfRange pr("k_classify", s);
    hipLaunchKernelGGL(k_classify, dim3((unsigned)classify_blocks(p.C)), dim3(kClassNT), 0, s, a);
    return hipGetLastError();
}

hipError_t batch_classify_all(BatchWork& b, const JoinParams& p, const uint32_t* pre, int n_jobs,
                              uint32_t blocks, hipStream_t s) {
    if (n_jobs == 0 || blocks == 0) return hipSuccess;
    Args a{};
    JoinWork& w = b.w;
    a.batch = 1;
    a.jobs = b.jobs;
    a.ujob = b.ujob;
    a.mjob = b.mjob;
    a.djob = b.djob;
    a.small_cap = p.small_cap;
    a.unit_cap = p.unit_cap;
    a.med_cap = p.med_cap;
    a.unit_tiles = p.unit_tiles;
    a.uspan = w.uspan;
    a.units = w.units;
    a.med = w.med;
    a.medt = w.medt;
    a.dense = w.dense;
    a.cap_units = w.cap_units;
    a.cap_med = w.cap_med;
    a.cap_dense = w.cap_dense;
    a.cap_dent = w.cap_dent;
    a.ctr = w.ctr;
    a.st = w.st;
    ProfRange pr("k_classify", s);
    hipLaunchKernelGGL(k_classify_b, dim3(blocks), dim3(kClassNT), 0, s, a, pre, n_jobs);
    return hipGetLastError();
}

hipError_t batch_join(BatchWork& b, int n_jobs, bool any_axis, bool pairs, int64_t units_bound,
                      int64_t med_bound, hipStream_t s) {
    Args a = batch_args(b);
    pairs = pairs && b.w.sc_nch > 0;
    if (pairs) {
        a.sc_buf = b.w.sc_buf;
        a.sc_fills = b.w.sc_fills;
        a.sc_ctr = b.w.sc_ctr;
        a.sc_nch = b.w.sc_nch;
        a.sc_job = b.sc_job;
    }
    const int ncu = b.w.num_cus;
    if (any_axis) {
        ProfRange pr("k_axis", s);
        hipLaunchKernelGGL(k_axis, dim3(ncu * 4), dim3(kAxisNT), 0, s, a);
    }
    {
        ProfRange pr("k_dense_sort", s);
        hipLaunchKernelGGL(k_dense_sort, dim3(ncu * 2), dim3(kDenseSortNT), 0, s, a);
    }
    hipLaunchKernelGGL(k_dense_plan, dim3(1), dim3(1024), 0, s, a);
    hipError_t e;
    const int64_t ub = std::min<int64_t>(units_bound, b.w.cap_units);
    const int64_t mb = std::min<int64_t>(med_bound, b.w.cap_med);
    {
        ProfRange pr("k_span_units_batch", s);
        a.cls = 0;
        static_assert(kBatchBlock == 256, "the batch's span kernel is instantiated for 256 threads");
        e = pairs ? launch_span<256, 4, kSingle, true>(a, ub, ncu, s)
                  : launch_span<256, 4, kAppend, true>(a, ub, ncu, s);
        if (e != hipSuccess) return e;
    }
    {
        ProfRange pr("k_lds_medium_batch", s);
        a.cls = 1;
        e = pairs ? launch_medium<kBatchMedNT, kBatchMedE / kBatchMedNT, kSingle>(a, mb, ncu, s)
                  : launch_medium<kBatchMedNT, kBatchMedE / kBatchMedNT, kAppend>(a, mb, ncu, s);
        if (e != hipSuccess) return e;
    }
    {
        ProfRange pr("k_dense_sweep_batch", s);
        a.cls = 2;
        if (pairs)
            hipLaunchKernelGGL(k_dense_sweep<kSingle>, dim3(ncu * 4), dim3(kDenseNT), 0, s, a);
        else
            hipLaunchKernelGGL(k_dense_sweep<kAppend>, dim3(ncu * 4), dim3(kDenseNT), 0, s, a);
    }
    if (pairs) {
        ProfRange pr("k_compact_batch", s);
        const int64_t per = kCompactNT / kWave;
        const int64_t need = (kRegions * b.w.sc_nch + per - 1) / per;
        hipLaunchKernelGGL(k_compact_batch, dim3((unsigned)std::min<int64_t>(need, ncu * 8)),
                           dim3(kCompactNT), 0, s, a);
    }
    if (n_jobs > 0)
        hipLaunchKernelGGL(k_batch_finish, dim3((unsigned)((n_jobs + 255) / 256)), dim3(256), 0, s,
                           b.w.st, b.jobs, n_jobs);
    return hipGetLastError();
}

hipError_t join_stats(const JoinWork& w, bool single, sj_join_stats* o) {
    uint32_t c[kNumCtr];
    unsigned long long t[kTotals];
    hipError_t e = hipMemcpy(c, w.ctr, sizeof(c), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    if (single && w.sc_total) {
        e = hipMemcpy(t, w.sc_total, sizeof(t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return e;
    }
    o->small_tiles = c[kTilesWritten];
    o->small_units = c[kUnitsWritten];
    o->medium_tiles = c[kMedCount];
    o->dense_tiles = c[kDenseCount];
    o->dense_units = c[kDenseUnits];
    o->small_entries = c[kSmallEntries];
    o->medium_entries = c[kMedEntries];
    o->dense_entries = c[kDenseEntries];
    int64_t pc[3] = {-1, -1, -1};
    if (single && w.sc_total)
        for (int k = 0; k < 3; ++k) {
            pc[k] = 0;
            for (int i = 0; i < kTotalsPer; ++i) pc[k] += (int64_t)t[k * kTotalsPer + i];
        }
    o->pairs_small = pc[0];
    o->pairs_medium = pc[1];
    o->pairs_dense = pc[2];
    o->axis_tiles = c[kAxisTiles];
    o->axis_y = c[kAxisY];
    return hipSuccess;
}

hipError_t axis_query(const Part& R, const Part& S, const int32_t* tiles, int64_t n, int64_t* out,
                      int num_cus, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>(n, (int64_t)num_cus * 8);
    hipLaunchKernelGGL(k_axis_query, dim3(g), dim3(kAxisNT), 0, s, R.off, S.off, R.entb, R.enti,
                       S.entb, S.enti, R.gd,
                       R.bl, (const int2*)tiles, n, (long long*)out);
    return hipGetLastError();
}

int scratch_regions() { return kRegions; }
int scratch_chunk_pairs() { return kChunkP; }
int scratch_totals() { return kTotals; }

}  // namespace sj
