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
// Schedules
//   tuned:  tiles with both lists non-empty and at most `small_cap` entries
//           are batched into LDS units of about `unit_cap` entries (built by
//           k_classify); a persistent workgroup pulls units off an atomic
//           queue, stages the unit's tile slabs in LDS, sorts every tile
//           segment in LDS and sweeps from LDS.  Larger ("dense") tiles are
//           sorted into a global buffer and swept by units of at most
//           `split_tau` pivots, so one dense tile is shared by many CUs.
//   plain:  one workgroup per tile (grid = K*K); tiles that fit LDS are
//           sorted and swept there, larger tiles are sorted globally and
//           swept by one workgroup each (no splitting).
//
// Pairs leave through a per-wave LDS staging buffer: lanes with a hit take
// slots by ballot + masked popcount, and a full buffer is flushed with one
// global atomic per wave and coalesced 8-byte stores.
#include "sj_internal.hpp"
#include "sj_prof.hpp"

namespace sj {

namespace {

enum Ctr : int {
    kUnitsTaken = 0,
    kDenseSortTaken = 1,
    kDenseUnitsTaken = 2,
    kTilesWritten = 3,
    kUnitsWritten = 4,
    kDenseEntries = 5,
    kDenseUnits = 6,
    kDenseCount = 7,
    kNumCtr = 8
};

constexpr int kWaveBuf = 256;    // staged pairs per wave
constexpr int kDenseSortMax = 8192;  // entries sorted in LDS by the dense sort

struct Args {
    const uint32_t* offR;
    const uint32_t* offS;
    const float4* boxR;
    const uint32_t* idfR;
    const float4* boxS;
    const uint32_t* idfS;
    int64_t C;
    int small_cap;   // LDS tiles: nr + ns <= small_cap
    int unit_cap;    // entries per LDS unit (target)
    int split_tau;
    int plain;
    int count_only;
    uint32_t* tiles;
    uint2* units;
    uint4* dense;
    uint32_t* dprefix;
    int64_t cap_tiles, cap_units, cap_dense, cap_dent;
    float4* dbox;
    uint32_t* didf;
    unsigned long long* dtmp;
    uint32_t* ctr;
    DevStatus* st;
    const DevStatus* stR;  // partition-time status of the two inputs
    const DevStatus* stS;
    unsigned long long* out;  // pairs as (r | s << 32)
    int64_t capacity;
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
}

// ---------------------------------------------------------------------------
// Per-wave pair emitter (wave-uniform state; every lane calls emit()).
// ---------------------------------------------------------------------------
struct Emitter {
    unsigned long long* buf;  // this wave's LDS buffer
    uint32_t n;               // staged pairs (uniform)
    unsigned long long cnt;   // pairs counted in count-only mode (uniform)

    __device__ void flush(const Args& a) {
        wave_lds_fence();
        unsigned long long base = 0;
        if (lane_id() == 0) base = atomicAdd(&a.st->n_pairs, (unsigned long long)n);
        base = __shfl(base, 0, kWave);
        for (uint32_t q = lane_id(); q < n; q += kWave) {
            unsigned long long idx = base + q;
            if (idx < (unsigned long long)a.capacity) a.out[idx] = buf[q];
        }
        wave_lds_fence();
        n = 0;
    }

    __device__ __forceinline__ void emit(const Args& a, bool hit, uint32_t r, uint32_t s) {
        unsigned long long m = __ballot(hit);
        if (m == 0ull) return;
        uint32_t c = (uint32_t)__popcll(m);
        if (a.count_only) {
            cnt += c;
            return;
        }
        if (n + c > (uint32_t)kWaveBuf) flush(a);
        if (hit) buf[n + lanes_below(m)] = (unsigned long long)r | ((unsigned long long)s << 32);
        n += c;
    }

    __device__ void finish(const Args& a) {
        if (a.count_only) {
            if (cnt && lane_id() == 0) atomicAdd(&a.st->n_pairs, cnt);
            cnt = 0;
        } else if (n) {
            flush(a);
        }
    }
};

// Reference-point test of Eq. (1) on the start bits of the two entries.
__device__ __forceinline__ bool ref_point_here(uint32_t ida, uint32_t idb) {
    return ((ida | idb) & (kBx | kBy)) == (kBx | kBy);
}

// ---------------------------------------------------------------------------
// The sweep over one batch of pivots.  Acc provides, for entry j of the
// batch's storage: xl(j), xu(j), yl(j), yu(j), id(j); and for a pivot p its
// setup (own rectangle, other list's segment).  Lanes that finish a scan pick
// the next pivot (p += stride), so a wave keeps all 64 lanes busy until the
// batch runs dry.
// ---------------------------------------------------------------------------
template <class Acc>
__device__ void sweep_pivots(const Args& a, const Acc& acc, int p_begin, int p_end, int stride,
                             Emitter& em) {
    int p = p_begin;
    bool alive = false, isR = false;
    int j = 0, jend = 0;
    float pxu = 0.f, pyl = 0.f, pyu = 0.f;
    uint32_t pid = 0;
    if (p < p_end) alive = acc.setup(p, isR, j, jend, pxu, pyl, pyu, pid);
    while (true) {
        bool hit = false;
        uint32_t rr = 0, ss = 0;
        if (alive) {
            if (j < jend && acc.xl(j) <= pxu) {
                float ql = acc.yl(j), qu = acc.yu(j);
                uint32_t qid = acc.id(j);
                hit = (pyl <= qu) && (ql <= pyu) && ref_point_here(pid, qid);
                rr = (isR ? pid : qid) & kIdMask;
                ss = (isR ? qid : pid) & kIdMask;
                ++j;
            } else {
                p += stride;
                alive = (p < p_end) && acc.setup(p, isR, j, jend, pxu, pyl, pyu, pid);
            }
        }
        em.emit(a, hit, rr, ss);
        if (__ballot(alive) == 0ull) break;
    }
}

// First index in [lo, hi) whose x_l is > v (upper) or >= v (lower).
template <class F>
__device__ __forceinline__ int search_x(const F& xl, int lo, int hi, float v, bool upper) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        float x = xl(mid);
        bool go_right = upper ? (x <= v) : (x < v);
        if (go_right) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// LDS unit: a batch of tiles staged, sorted and swept in LDS.
// ---------------------------------------------------------------------------
struct LdsLayout {
    unsigned long long* wbuf;  // [nwaves * kWaveBuf]
    uint32_t* rg;  // [tc+1] global start of each tile's R segment
    uint32_t* rl;  // [tc+1] local start (prefix) of each tile's R segment
    uint32_t* sg;
    uint32_t* sl;
    uint32_t* key;  // [E] unsorted order keys
    uint16_t* tk;   // [E] local tile of each entry
    float* xl;      // [E] sorted payload (R part first, then S part)
    float* yl;
    float* xu;
    float* yu;
    uint32_t* id;
};

__host__ __device__ inline size_t lds_bytes(int nt, int E) {
    const int tc = E / 2 + 2;
    size_t b = 0;
    b += (size_t)(nt / kWave) * kWaveBuf * 8;
    b += (size_t)4 * (tc + 1) * 4;
    b += (size_t)E * 4;                  // key
    b += (size_t)((E * 2 + 7) / 8) * 8;  // tk
    b += (size_t)5 * E * 4;              // payload
    return b;
}

__device__ inline LdsLayout carve(unsigned char* p, int nt, int E) {
    const int tc = E / 2 + 2;
    LdsLayout L;
    L.wbuf = (unsigned long long*)p;
    p += (size_t)(nt / kWave) * kWaveBuf * 8;
    L.rg = (uint32_t*)p; p += (size_t)(tc + 1) * 4;
    L.rl = (uint32_t*)p; p += (size_t)(tc + 1) * 4;
    L.sg = (uint32_t*)p; p += (size_t)(tc + 1) * 4;
    L.sl = (uint32_t*)p; p += (size_t)(tc + 1) * 4;
    L.key = (uint32_t*)p; p += (size_t)E * 4;
    L.tk = (uint16_t*)p; p += (size_t)((E * 2 + 7) / 8) * 8;
    L.xl = (float*)p; p += (size_t)E * 4;
    L.yl = (float*)p; p += (size_t)E * 4;
    L.xu = (float*)p; p += (size_t)E * 4;
    L.yu = (float*)p; p += (size_t)E * 4;
    L.id = (uint32_t*)p;
    return L;
}

struct LdsAcc {
    const LdsLayout* L;
    int NR;  // R entries of the unit; S entries start at NR
    __device__ float xl(int j) const { return L->xl[j]; }
    __device__ float yl(int j) const { return L->yl[j]; }
    __device__ float yu(int j) const { return L->yu[j]; }
    __device__ uint32_t id(int j) const { return L->id[j]; }
    __device__ bool setup(int p, bool& isR, int& j, int& jend, float& pxu, float& pyl, float& pyu,
                          uint32_t& pid) const {
        const int k = L->tk[p];
        pxu = L->xu[p];
        pyl = L->yl[p];
        pyu = L->yu[p];
        pid = L->id[p];
        const float px = L->xl[p];
        auto X = [&](int q) { return L->xl[q]; };
        if (p < NR) {  // R pivot: scan S from the first s with s.x_l > r.x_l
            isR = true;
            int lo = NR + (int)L->sl[k], hi = NR + (int)L->sl[k + 1];
            j = search_x(X, lo, hi, px, true);
            jend = hi;
        } else {  // S pivot: scan R from the first r with r.x_l >= s.x_l
            isR = false;
            int lo = (int)L->rl[k], hi = (int)L->rl[k + 1];
            j = search_x(X, lo, hi, px, false);
            jend = hi;
        }
        return true;
    }
};

// Stage tiles [0, c) -- given by tile_of(k) -- in LDS, sort every tile
// segment by x_l and sweep.  Returns false if the unit did not fit (cannot
// happen for units built by k_classify / the plain kernel).
template <int NT, int Q, class TileOf>
__device__ void run_lds_unit(const Args& a, const LdsLayout& L, int c, const TileOf& tile_of,
                             Emitter& em) {
    constexpr int E = NT * Q;
    const int tid = threadIdx.x;
    if (c > E / 2 + 1) {  // more tiles than the LDS tile table holds: cannot happen
        if (tid == 0) atomicOr(&a.st->flags, kStatInternal);
        return;
    }
    __shared__ uint32_t s_tot[2];
    __shared__ uint32_t s_wsum[2][NT / kWave + 1];
    // 1. tile table with local prefixes (chunks of NT tiles)
    uint32_t carry_r = 0, carry_s = 0;
    for (int k0 = 0; k0 < c; k0 += NT) {
        const int k = k0 + tid;
        uint32_t nr = 0, ns = 0, r0 = 0, s0 = 0;
        if (k < c) {
            const uint32_t t = tile_of(k);
            r0 = a.offR[t];
            nr = a.offR[t + 1] - r0;
            s0 = a.offS[t];
            ns = a.offS[t + 1] - s0;
        }
        // block exclusive scan of (nr, ns)
        const int lane = lane_id(), w = tid / kWave;
        uint32_t ir = nr, is = ns;
        for (int d = 1; d < kWave; d <<= 1) {
            uint32_t tr = __shfl_up(ir, d, kWave), ts = __shfl_up(is, d, kWave);
            if (lane >= d) { ir += tr; is += ts; }
        }
        if (lane == kWave - 1) { s_wsum[0][w] = ir; s_wsum[1][w] = is; }
        __syncthreads();
        if (tid == 0) {
            uint32_t ar = 0, as = 0;
            for (int q = 0; q < NT / kWave; ++q) {
                uint32_t vr = s_wsum[0][q], vs = s_wsum[1][q];
                s_wsum[0][q] = ar; s_wsum[1][q] = as;
                ar += vr; as += vs;
            }
            s_tot[0] = ar; s_tot[1] = as;
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
    }
    if (NE > E) {  // cannot happen for units built with unit_cap + small_cap <= E
        if (tid == 0) atomicOr(&a.st->flags, kStatInternal);
        __syncthreads();
        return;
    }
    __syncthreads();
    // 2. load entries (coalesced within each tile segment), keep payload in
    //    registers, publish keys and tile indices
    float4 pb[Q];
    uint32_t pi[Q];
    int pk[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e = tid + q * NT;
        pk[q] = -1;
        if (e < NE) {
            const bool isR = e < NR;
            const int le = isR ? e : e - NR;
            const uint32_t* loc = isR ? L.rl : L.sl;
            // tile k: last k with loc[k] <= le
            int lo = 0, hi = c;  // loc[c] = total > le
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (loc[mid] <= (uint32_t)le) lo = mid;
                else hi = mid;
            }
            const int k = lo;
            const uint32_t g = (isR ? L.rg[k] : L.sg[k]) + (uint32_t)le - loc[k];
            pb[q] = isR ? a.boxR[g] : a.boxS[g];
            pi[q] = isR ? a.idfR[g] : a.idfS[g];
            pk[q] = k;
            L.key[e] = order_key(pb[q].x);
            L.tk[e] = (uint16_t)k;
        }
    }
    __syncthreads();
    // 3. rank sort within each tile segment, write sorted payload
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e = tid + q * NT;
        if (e < NE) {
            const bool isR = e < NR;
            const int k = pk[q];
            const int lo = isR ? (int)L.rl[k] : NR + (int)L.sl[k];
            const int hi = isR ? (int)L.rl[k + 1] : NR + (int)L.sl[k + 1];
            const uint32_t my = L.key[e];
            int rank = 0;
            for (int j = lo; j < hi; ++j) {
                const uint32_t kj = L.key[j];
                rank += (kj < my) || (kj == my && j < e);
            }
            const int pos = lo + rank;
            L.xl[pos] = pb[q].x;
            L.yl[pos] = pb[q].y;
            L.xu[pos] = pb[q].z;
            L.yu[pos] = pb[q].w;
            L.id[pos] = pi[q];
        }
    }
    __syncthreads();
    // 4. sweep: one lane per pivot, pivots = all entries of the unit
    LdsAcc acc{&L, NR};
    sweep_pivots(a, acc, tid, NE, NT, em);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// k_classify (tuned schedule): find active tiles, batch the small ones into
// LDS units, list the dense ones.  One block covers kClassChunk tiles; units
// never cross block chunks.
// ---------------------------------------------------------------------------
constexpr int kClassNT = 256;
constexpr int kClassPer = 8;
constexpr int kClassChunk = kClassNT * kClassPer;

__global__ __launch_bounds__(kClassNT) void k_classify(Args a) {
    __shared__ uint32_t s_uidx[kClassChunk];  // unit index of the k-th small tile
    __shared__ uint32_t s_ws[3][kClassNT / kWave];
    __shared__ uint32_t s_base[2];
    const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const int64_t t0 = (int64_t)blockIdx.x * kClassChunk + (int64_t)tid * kClassPer;
    uint32_t nsmall = 0, size_small = 0;
    uint32_t sz[kClassPer];
    uint8_t cls[kClassPer];  // 0 none, 1 small, 2 dense
#pragma unroll
    for (int q = 0; q < kClassPer; ++q) {
        const int64_t t = t0 + q;
        cls[q] = 0;
        sz[q] = 0;
        if (t < a.C) {
            const uint32_t nr = a.offR[t + 1] - a.offR[t];
            const uint32_t ns = a.offS[t + 1] - a.offS[t];
            if (nr && ns) {
                sz[q] = nr + ns;
                if (nr + ns <= (uint32_t)a.small_cap) {
                    cls[q] = 1;
                    ++nsmall;
                    size_small += nr + ns;
                } else {
                    cls[q] = 2;
                    uint32_t d = atomicAdd(&a.ctr[kDenseCount], 1u);
                    uint32_t base = atomicAdd(&a.ctr[kDenseEntries], nr + ns);
                    if (d < (uint32_t)a.cap_dense && (int64_t)base + nr + ns <= a.cap_dent)
                        a.dense[d] = make_uint4((uint32_t)t, base, nr, ns);
                    else
                        atomicOr(&a.st->flags, kStatCapacity);
                }
            }
        }
    }
    // block exclusive scans of nsmall and size_small
    uint32_t in = nsmall, isz = size_small;
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t tn = __shfl_up(in, d, kWave), ts = __shfl_up(isz, d, kWave);
        if (lane >= d) { in += tn; isz += ts; }
    }
    if (lane == kWave - 1) { s_ws[0][w] = in; s_ws[1][w] = isz; }
    __syncthreads();
    if (tid == 0) {
        uint32_t an = 0, as = 0;
        for (int q = 0; q < kClassNT / kWave; ++q) {
            uint32_t vn = s_ws[0][q], vs = s_ws[1][q];
            s_ws[0][q] = an; s_ws[1][q] = as;
            an += vn; as += vs;
        }
        s_ws[2][0] = an;
    }
    __syncthreads();
    const uint32_t total_small = s_ws[2][0];
    uint32_t rank = s_ws[0][w] + in - nsmall;
    uint32_t spre = s_ws[1][w] + isz - size_small;
    const uint32_t B = (uint32_t)a.unit_cap;
#pragma unroll
    for (int q = 0; q < kClassPer; ++q) {
        if (cls[q] == 1) {
            s_uidx[rank] = spre / B;
            ++rank;
            spre += sz[q];
        }
    }
    __syncthreads();
    if (total_small == 0) return;
    const uint32_t nunits = s_uidx[total_small - 1] + 1;
    if (tid == 0) {
        s_base[0] = atomicAdd(&a.ctr[kTilesWritten], total_small);
        s_base[1] = atomicAdd(&a.ctr[kUnitsWritten], nunits);
    }
    __syncthreads();
    const uint32_t tb = s_base[0], ub = s_base[1];
    if ((int64_t)tb + total_small > a.cap_tiles || (int64_t)ub + nunits > a.cap_units) {
        if (tid == 0) atomicOr(&a.st->flags, kStatCapacity);
        return;
    }
    rank = s_ws[0][w] + in - nsmall;
#pragma unroll
    for (int q = 0; q < kClassPer; ++q) {
        if (cls[q] == 1) {
            a.tiles[tb + rank] = (uint32_t)(t0 + q);
            const uint32_t u = s_uidx[rank];
            if (rank == 0 || s_uidx[rank - 1] != u) {
                // first tile of unit u: count the tiles of the unit
                uint32_t lo = rank, hi = total_small;
                while (hi - lo > 1) {
                    uint32_t mid = (lo + hi) >> 1;
                    if (s_uidx[mid] == u) lo = mid;
                    else hi = mid;
                }
                a.units[ub + u] = make_uint2(tb + rank, lo - rank + 1);
            }
            ++rank;
        }
    }
}

// ---------------------------------------------------------------------------
// k_lds_units (tuned): persistent workgroups over the LDS unit queue.
// ---------------------------------------------------------------------------
template <int NT, int Q>
__global__ __launch_bounds__(NT) void k_lds_units(Args a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const LdsLayout L = carve(smem, NT, NT * Q);
    Emitter em{L.wbuf + (threadIdx.x / kWave) * kWaveBuf, 0u, 0ull};
    __shared__ uint32_t s_u;
    const uint32_t nunits = a.ctr[kUnitsWritten];
    while (true) {
        if (threadIdx.x == 0) s_u = atomicAdd(&a.ctr[kUnitsTaken], 1u);
        __syncthreads();
        const uint32_t u = s_u;
        __syncthreads();
        if (u >= nunits || u >= (uint32_t)a.cap_units) break;
        const uint2 ud = a.units[u];
        const uint32_t* tl = a.tiles + ud.x;
        run_lds_unit<NT, Q>(a, L, (int)ud.y, [&](int k) { return tl[k]; }, em);
    }
    em.finish(a);
}

// ---------------------------------------------------------------------------
// k_plain_tiles (plain): one workgroup per tile.
// ---------------------------------------------------------------------------
template <int NT, int Q>
__global__ __launch_bounds__(NT) void k_plain_tiles(Args a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const LdsLayout L = carve(smem, NT, NT * Q);
    Emitter em{L.wbuf + (threadIdx.x / kWave) * kWaveBuf, 0u, 0ull};
    // one workgroup per tile; a grid-stride loop only when K*K exceeds the grid
    for (int64_t t = blockIdx.x; t < a.C; t += gridDim.x) {
        const uint32_t nr = a.offR[t + 1] - a.offR[t];
        const uint32_t ns = a.offS[t + 1] - a.offS[t];
        if (nr == 0 || ns == 0) continue;
        if (nr + ns > (uint32_t)(NT * Q)) {
            if (threadIdx.x == 0) {
                uint32_t d = atomicAdd(&a.ctr[kDenseCount], 1u);
                uint32_t base = atomicAdd(&a.ctr[kDenseEntries], nr + ns);
                if (d < (uint32_t)a.cap_dense && (int64_t)base + nr + ns <= a.cap_dent)
                    a.dense[d] = make_uint4((uint32_t)t, base, nr, ns);
                else
                    atomicOr(&a.st->flags, kStatCapacity);
            }
            continue;
        }
        const uint32_t tt = (uint32_t)t;
        run_lds_unit<NT, Q>(a, L, 1, [&](int) { return tt; }, em);
    }
    em.finish(a);
}

// ---------------------------------------------------------------------------
// Dense tiles: sort each list into the global dense buffer ...
// ---------------------------------------------------------------------------
constexpr int kDenseSortNT = 1024;

__device__ void bitonic_lds(unsigned long long* k, int P) {
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = ((lo & size) == 0);
                unsigned long long x = k[lo], y = k[hi];
                if ((x > y) == up) {
                    k[lo] = y;
                    k[hi] = x;
                }
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kDenseSortNT) void k_dense_sort(Args a) {
    __shared__ unsigned long long keys[kDenseSortMax];
    __shared__ uint32_t s_seg;
    const uint32_t nd = min(a.ctr[kDenseCount], (uint32_t)a.cap_dense);
    while (true) {
        if (threadIdx.x == 0) s_seg = atomicAdd(&a.ctr[kDenseSortTaken], 1u);
        __syncthreads();
        const uint32_t seg = s_seg;
        __syncthreads();
        if (seg >= 2 * nd) break;
        const uint4 dd = a.dense[seg >> 1];
        const bool sideS = seg & 1;
        const uint32_t src = sideS ? a.offS[dd.x] : a.offR[dd.x];
        const uint32_t L = sideS ? dd.w : dd.z;
        const uint32_t dst = dd.y + (sideS ? dd.z : 0u);
        const float4* box = sideS ? a.boxS : a.boxR;
        const uint32_t* idf = sideS ? a.idfS : a.idfR;
        const unsigned long long* fin;  // final sorted keys (low 32 bits = position)
        if (L <= (uint32_t)kDenseSortMax) {
            int P = 1;
            while (P < (int)L) P <<= 1;
            for (int i = threadIdx.x; i < P; i += blockDim.x)
                keys[i] = i < (int)L ? ((unsigned long long)order_key(box[src + i].x) << 32) | (uint32_t)i
                                     : ~0ull;
            __syncthreads();
            bitonic_lds(keys, P);
            fin = keys;
        } else {
            // sorted runs of kDenseSortMax in LDS, then merge passes in global
            // memory (rank of each key in the partner run by binary search;
            // keys are distinct because they carry the position).
            unsigned long long* A = a.dtmp + 2ull * dst;
            unsigned long long* Bf = A + L;
            for (uint32_t c0 = 0; c0 < L; c0 += kDenseSortMax) {
                const int n = (int)min((uint32_t)kDenseSortMax, L - c0);
                for (int i = threadIdx.x; i < kDenseSortMax; i += blockDim.x)
                    keys[i] = i < n ? ((unsigned long long)order_key(box[src + c0 + i].x) << 32) |
                                          (c0 + (uint32_t)i)
                                    : ~0ull;
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
                    if (i < mid) { olo = mid; ohi = hi; mine = i - lo; }
                    else { olo = lo; ohi = mid; mine = i - mid; }
                    uint32_t b0 = olo, b1 = ohi;
                    while (b0 < b1) {
                        uint32_t m = (b0 + b1) >> 1;
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
            const uint32_t q = (uint32_t)fin[i];
            a.dbox[dst + i] = box[src + q];
            a.didf[dst + i] = idf[src + q];
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
            v = a.plain ? 1u : (n + (uint32_t)a.split_tau - 1u) / (uint32_t)a.split_tau;
        }
        uint32_t inc = v;
        for (int s = 1; s < kWave; s <<= 1) {
            uint32_t t = __shfl_up(inc, s, kWave);
            if (lane >= s) inc += t;
        }
        if (lane == kWave - 1) lds[w] = inc;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t acc = 0;
            for (int q = 0; q < nw; ++q) {
                uint32_t x = lds[q];
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
    }
}

// ... and sweep them, one unit = a contiguous range of pivots of one tile.
struct GlobAcc {
    const float4* box;
    const uint32_t* idf;
    int base, nr, ns;  // R entries at [base, base+nr), S at [base+nr, base+nr+ns)
    __device__ float xl(int j) const { return box[j].x; }
    __device__ float yl(int j) const { return box[j].y; }
    __device__ float yu(int j) const { return box[j].w; }
    __device__ uint32_t id(int j) const { return idf[j]; }
    __device__ bool setup(int p, bool& isR, int& j, int& jend, float& pxu, float& pyl, float& pyu,
                          uint32_t& pid) const {
        const int e = base + p;  // pivots: R entries then S entries
        const float4 b = box[e];
        pxu = b.z;
        pyl = b.y;
        pyu = b.w;
        pid = idf[e];
        auto X = [&](int q) { return box[q].x; };
        if (p < nr) {
            isR = true;
            j = search_x(X, base + nr, base + nr + ns, b.x, true);
            jend = base + nr + ns;
        } else {
            isR = false;
            j = search_x(X, base, base + nr, b.x, false);
            jend = base + nr;
        }
        return true;
    }
};

template <int NT>
__global__ __launch_bounds__(NT) void k_dense_sweep(Args a) {
    __shared__ unsigned long long wbuf[(NT / kWave) * kWaveBuf];
    __shared__ uint32_t s_u;
    Emitter em{wbuf + (threadIdx.x / kWave) * kWaveBuf, 0u, 0ull};
    const uint32_t nd = min(a.ctr[kDenseCount], (uint32_t)a.cap_dense);
    const uint32_t nu = a.ctr[kDenseUnits];
    while (true) {
        if (threadIdx.x == 0) s_u = atomicAdd(&a.ctr[kDenseUnitsTaken], 1u);
        __syncthreads();
        const uint32_t u = s_u;
        __syncthreads();
        if (u >= nu) break;
        // dense tile of unit u: last d with dprefix[d] <= u
        uint32_t lo = 0, hi = nd;
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (a.dprefix[mid] <= u) lo = mid;
            else hi = mid;
        }
        const uint4 dd = a.dense[lo];
        const int n = (int)(dd.z + dd.w);
        int p0 = 0, p1 = n;
        if (!a.plain) {
            p0 = (int)(u - a.dprefix[lo]) * a.split_tau;
            p1 = min(p0 + a.split_tau, n);
        }
        GlobAcc acc{a.dbox, a.didf, (int)dd.y, (int)dd.z, (int)dd.w};
        sweep_pivots(a, acc, p0 + (int)threadIdx.x, p1, NT, em);
    }
    em.finish(a);
}

__global__ void k_reset(uint32_t* ctr, DevStatus* st) {
    if (threadIdx.x < kNumCtr) ctr[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        st->n_pairs = 0ull;
        st->flags = 0u;
        st->n_dense = 0u;
        st->n_units = 0u;
    }
}

__global__ void k_finish(const uint32_t* ctr, DevStatus* st, const DevStatus* stR,
                         const DevStatus* stS) {
    st->n_dense = ctr[kDenseCount];
    st->n_units = ctr[kUnitsWritten];
    st->flags |= stR->flags | stS->flags;
}

template <int NT, int Q>
hipError_t launch_units(const Args& a, int num_cus, bool plain, hipStream_t s) {
    const size_t lds = lds_bytes(NT, NT * Q);
    if (plain) {
        hipError_t e = hipFuncSetAttribute((const void*)k_plain_tiles<NT, Q>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        // HIP limits a grid to fewer than 2^32 work-items
        const int64_t max_blocks = ((int64_t)1 << 31) / NT;
        const int64_t nb = a.C < max_blocks ? a.C : max_blocks;
        hipLaunchKernelGGL((k_plain_tiles<NT, Q>), dim3((unsigned)nb), dim3(NT), lds, s, a);
        return hipGetLastError();
    }
    int per_cu = 0;
    hipError_t e = hipFuncSetAttribute((const void*)k_lds_units<NT, Q>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_lds_units<NT, Q>, NT, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    hipLaunchKernelGGL((k_lds_units<NT, Q>), dim3((unsigned)(num_cus * per_cu)), dim3(NT), lds, s, a);
    return hipGetLastError();
}

}  // namespace

int lds_unit_entries(int block) { return block == 64 ? 64 * 16 : (block == 128 ? 128 * 8 : (block == 512 ? 512 * 4 : 256 * 4)); }

hipError_t run_join(const Part& R, const Part& S, const JoinParams& p, JoinWork& w, sj_pair* out,
                    int64_t capacity, hipStream_t s) {
    Args a{};
    a.offR = R.off;
    a.offS = S.off;
    a.boxR = R.box;
    a.idfR = R.idf;
    a.boxS = S.box;
    a.idfS = S.idf;
    a.C = p.C;
    a.small_cap = p.small_cap;
    a.unit_cap = p.unit_cap;
    a.split_tau = p.split_tau;
    a.plain = p.plain ? 1 : 0;
    a.count_only = p.count_only ? 1 : 0;
    a.tiles = w.tiles;
    a.units = w.units;
    a.dense = w.dense;
    a.dprefix = w.dense_unit_prefix;
    a.cap_tiles = w.cap_tiles;
    a.cap_units = w.cap_units;
    a.cap_dense = w.cap_dense;
    a.cap_dent = w.cap_dent;
    a.dbox = w.dbox;
    a.didf = w.didf;
    a.dtmp = w.dtmp;
    a.ctr = w.ctr;
    a.st = w.st;
    a.stR = R.st;
    a.stS = S.st;
    a.out = (unsigned long long*)out;
    a.capacity = out ? capacity : 0;

    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, w.ctr, w.st);
    if (!p.plain) {
        ProfRange pr("k_classify", s);
        const unsigned nb = (unsigned)((p.C + kClassChunk - 1) / kClassChunk);
        hipLaunchKernelGGL(k_classify, dim3(nb), dim3(kClassNT), 0, s, a);
    }
    hipError_t e;
    {
    ProfRange pr(p.plain ? "k_plain_tiles" : "k_lds_units", s);
    switch (p.block) {
        case 64: e = launch_units<64, 16>(a, w.num_cus, p.plain, s); break;
        case 128: e = launch_units<128, 8>(a, w.num_cus, p.plain, s); break;
        case 512: e = launch_units<512, 4>(a, w.num_cus, p.plain, s); break;
        default: e = launch_units<256, 4>(a, w.num_cus, p.plain, s); break;
    }
    }
    if (e != hipSuccess) return e;
    const int nsort = w.num_cus * 2;
    {
        ProfRange pr("k_dense_sort", s);
        hipLaunchKernelGGL(k_dense_sort, dim3(nsort), dim3(kDenseSortNT), 0, s, a);
    }
    hipLaunchKernelGGL(k_dense_plan, dim3(1), dim3(1024), 0, s, a);
    {
        ProfRange pr("k_dense_sweep", s);
        hipLaunchKernelGGL(k_dense_sweep<256>, dim3(w.num_cus * 4), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1), 0, s, w.ctr, w.st, R.st, S.st);
    return hipGetLastError();
}

}  // namespace sj
