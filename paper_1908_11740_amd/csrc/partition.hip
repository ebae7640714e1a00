// Partitioning phase of the PBSM join (Sec. 3.4 steps 1-4) on gfx950.
//
//   count    one thread per rectangle: validate it, compute its cell range and
//            add 1 to the count of every tile it covers (step 2; the per-thread
//            private counts of the paper become device-wide atomics).
//   scan     exclusive prefix sum of the counts = per-tile segment offsets
//            (step 3: "sum the counts, allocate one segment per tile").
//   scatter  second read of the input: each rectangle is written into a slot
//            of the segment of every tile it covers (step 4).  The slot is
//            taken by an atomic decrement of the tile's count, which leaves
//            every count at zero again for the next call.
//
// All loads of the input are 16-byte float4 loads by consecutive lanes
// (coalesced).  The scatter stores a float4 box and a 32-bit id word per
// entry.
#include "sj_internal.hpp"

namespace sj {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ bool rect_ok(float4 a) {
    return isfinite(a.x) && isfinite(a.y) && isfinite(a.z) && isfinite(a.w) && a.x <= a.z &&
           a.y <= a.w;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__global__ __launch_bounds__(kBlock) void k_count(const float4* __restrict__ rects, int64_t n,
                                                 GridDev g, uint32_t* __restrict__ cnt,
                                                 DevStatus* __restrict__ st) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float4 a = rects[i];
        if (!rect_ok(a)) {
            bad = true;
            continue;
        }
        int cx0 = cell_of(a.x, g.x0, g.sx, g.K), cx1 = cell_of(a.z, g.x0, g.sx, g.K);
        int cy0 = cell_of(a.y, g.y0, g.sy, g.K), cy1 = cell_of(a.w, g.y0, g.sy, g.K);
        for (int cy = cy0; cy <= cy1; ++cy) {
            uint32_t* row = cnt + (int64_t)cy * g.K;
            for (int cx = cx0; cx <= cx1; ++cx) atomicAdd(row + cx, 1u);
        }
    }
    if (bad) atomicOr(&st->flags, kStatBadRect);
}

__global__ __launch_bounds__(kBlock) void k_scatter(const float4* __restrict__ rects, int64_t n,
                                                   GridDev g, uint32_t* __restrict__ cnt,
                                                   const uint32_t* __restrict__ off,
                                                   float4* __restrict__ box,
                                                   uint32_t* __restrict__ idf, int64_t cap_m,
                                                   DevStatus* __restrict__ st) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t err = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float4 a = rects[i];
        if (!rect_ok(a)) continue;
        a.x += 0.0f;  // -0.0 -> +0.0
        a.y += 0.0f;
        a.z += 0.0f;
        a.w += 0.0f;
        int cx0 = cell_of(a.x, g.x0, g.sx, g.K), cx1 = cell_of(a.z, g.x0, g.sx, g.K);
        int cy0 = cell_of(a.y, g.y0, g.sy, g.K), cy1 = cell_of(a.w, g.y0, g.sy, g.K);
        for (int cy = cy0; cy <= cy1; ++cy) {
            const int64_t rowt = (int64_t)cy * g.K;
            const uint32_t by = (cy == cy0) ? kBy : 0u;
            for (int cx = cx0; cx <= cx1; ++cx) {
                const int64_t t = rowt + cx;
                uint32_t old = atomicSub(cnt + t, 1u);
                if (old == 0u) {  // more scatters than counts: cannot happen
                    atomicAdd(cnt + t, 1u);
                    err |= kStatInternal;
                    continue;
                }
                uint64_t pos = (uint64_t)off[t] + old - 1u;
                if (pos >= (uint64_t)cap_m) {
                    err |= kStatCapacity;
                    continue;
                }
                box[pos] = a;
                idf[pos] = (uint32_t)i | by | ((cx == cx0) ? kBx : 0u);
            }
        }
    }
    if (err) atomicOr(&st->flags, err);
}

// ---- exclusive scan of per-tile counts (reduce, top-level scan, down-sweep) ----
constexpr int kScanItems = 16;
constexpr int kScanChunk = kBlock * kScanItems;  // counts per block

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan over the block; returns the block total in `total`.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds, uint32_t& total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    uint32_t inc = wave_incl_scan(v, lane);
    if (lane == kWave - 1) lds[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint32_t x = lane < nw ? lds[lane] : 0u;
        uint32_t xi = wave_incl_scan(x, lane);
        if (lane < nw) lds[lane] = xi - x;
        if (lane == nw - 1) lds[nw] = xi;
    }
    __syncthreads();
    uint32_t res = inc - v + lds[w];
    total = lds[nw];
    __syncthreads();
    return res;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ cnt,
                                                       int64_t C, uint32_t* __restrict__ bs) {
    __shared__ uint32_t red[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        if (i < C) s += cnt[i];
    }
    s = wave_sum_u32(s);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kBlock / kWave; ++k) t += red[k];
        bs[blockIdx.x] = t;
    }
}

// One block: exclusive scan of the nb block sums in place (64-bit carry to
// detect totals beyond 2^31 - 1); writes off[C] and the entry total.
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* __restrict__ bs, int64_t nb,
                                                  uint32_t* __restrict__ off, int64_t C,
                                                  DevStatus* __restrict__ st) {
    __shared__ uint32_t lds[1024 / kWave + 1];
    unsigned long long carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += blockDim.x) {
        int64_t i = b0 + threadIdx.x;
        uint32_t v = i < nb ? bs[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, lds, tot);
        if (i < nb) bs[i] = (uint32_t)(carry + ex);
        carry += tot;
    }
    if (threadIdx.x == 0) {
        if (carry >= 0x7FFFFFFFull) {
            atomicOr(&st->flags, kStatCapacity);
            off[C] = 0x7FFFFFFFu;
        } else {
            off[C] = (uint32_t)carry;
        }
        st->m_total = carry;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_down(const uint32_t* __restrict__ cnt, int64_t C,
                                                     const uint32_t* __restrict__ bs,
                                                     uint32_t* __restrict__ off) {
    __shared__ uint32_t lds[kBlock / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = i < C ? cnt[i] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(s, lds, tot) + bs[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < C) off[i] = ex;
        ex += v[k];
    }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

int grid_for(int64_t n, int block, int max_blocks) {
    int64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

}  // namespace

int64_t scan_block_sums_needed(int64_t C) { return (C + kScanChunk - 1) / kScanChunk + 1; }

hipError_t launch_count(const float4* rects, int64_t n, GridDev g, uint32_t* cnt, DevStatus* st,
                        hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_count, dim3(grid_for(n, kBlock, 1 << 20)), dim3(kBlock), 0, s, rects, n,
                       g, cnt, st);
    return hipGetLastError();
}

hipError_t launch_scan(const uint32_t* cnt, int64_t C, uint32_t* off, uint32_t* block_sums,
                       DevStatus* st, hipStream_t s) {
    int64_t nb = (C + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, cnt, C, block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, block_sums, nb, off, C, st);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kBlock), 0, s, cnt, C, block_sums,
                       off);
    return hipGetLastError();
}

hipError_t launch_scatter(const float4* rects, int64_t n, GridDev g, uint32_t* cnt,
                          const uint32_t* off, float4* box, uint32_t* idf, int64_t cap_m,
                          DevStatus* st, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, kBlock, 1 << 20)), dim3(kBlock), 0, s, rects,
                       n, g, cnt, off, box, idf, cap_m, st);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, kBlock, 65536)), dim3(kBlock), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace sj
