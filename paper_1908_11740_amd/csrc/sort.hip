// Canonical order of a pair list: lexicographic by (r, s), the order in which
// the result set J is written out when it must be reproducible (a join's pair
// order otherwise depends on the schedule).
//
// Least-significant-digit radix sort of the 64-bit keys (r << 32) | s with
// 8-bit digits, only over the bits that r < nR and s < nS can set (for 10M x
// 10M: 3 digits of s, then 3 of r).  A pair in memory is (r, s) as two
// int32, i.e. a little-endian u64 with r in the low word, so the key is that
// word pair exchanged; the exchange is its own inverse and is applied before
// the first and after the last pass.  Every pass:
//   k_rs_hist     per tile of kRsTile keys, an LDS histogram of the digit,
//                 stored digit-major (digit * tiles + tile);
//   scan          exclusive prefix over all (digit, tile) counts: the first
//                 destination of every tile's keys of every digit;
//   k_rs_scatter  per tile, in rounds of one key per thread (index order),
//                 the stable rank of each key among the round's keys with the
//                 same digit (wavefront ballots over the 8 digit bits, then a
//                 prefix over the workgroup's waves), added to the tile's
//                 running offset of that digit.
// Passes alternate between the caller's buffer and one library buffer.
#include <map>
#include <mutex>

#include "sj_internal.hpp"
#include "sj_prof.hpp"

namespace sj {

hipError_t scan_u32(uint32_t* data, int64_t len, uint32_t* bs, unsigned long long* total,
                    DevStatus* st, hipStream_t s);

namespace {

constexpr int kRsNT = 256;
constexpr int kRsWaves = kRsNT / kWave;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsNT * kRsItems;
constexpr int kRsDigits = 256;

// in and out may be the same buffer (each element is read and written by one thread)
__global__ __launch_bounds__(256) void k_rs_swap(const unsigned long long* in,
                                                 unsigned long long* out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long v = in[i];
        out[i] = (v << 32) | (v >> 32);
    }
}

__global__ __launch_bounds__(kRsNT) void k_rs_hist(const unsigned long long* __restrict__ key,
                                                   int64_t n, int shift, int64_t tiles,
                                                   uint32_t* __restrict__ hist) {
    __shared__ uint32_t cnt[kRsDigits];
    cnt[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        const int64_t i = base + (int64_t)k * kRsNT + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(uint32_t)(key[i] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kRsNT) void k_rs_scatter(const unsigned long long* __restrict__ in,
                                                      unsigned long long* __restrict__ out,
                                                      int64_t n, int shift, int64_t tiles,
                                                      const uint32_t* __restrict__ offs) {
    __shared__ uint32_t run[kRsDigits];              // next destination of each digit
    __shared__ uint32_t wcnt[kRsWaves][kRsDigits];   // keys of each digit per wave (this round)
    __shared__ uint32_t woff[kRsWaves][kRsDigits];   // first destination per wave and digit
    const int tid = threadIdx.x, w = tid / kWave;
    run[tid] = offs[(int64_t)tid * tiles + blockIdx.x];
#pragma unroll
    for (int q = 0; q < kRsWaves; ++q) wcnt[q][tid] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int k = 0; k < kRsItems; ++k) {
        const int64_t i = base + (int64_t)k * kRsNT + tid;
        const bool valid = i < n;
        const unsigned long long v = valid ? in[i] : 0ull;
        const uint32_t d = (uint32_t)(v >> shift) & 0xFFu;
        // lanes of this wave with the same digit
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const unsigned long long m = __ballot(valid && ((d >> b) & 1u));
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(peers >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
        if (valid && below == 0u) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {  // thread tid owns digit tid: offsets of the waves, then clear
            uint32_t acc = run[tid];
#pragma unroll
            for (int q = 0; q < kRsWaves; ++q) {
                woff[q][tid] = acc;
                acc += wcnt[q][tid];
                wcnt[q][tid] = 0u;
            }
            run[tid] = acc;
        }
        __syncthreads();
        if (valid) out[woff[w][d] + below] = v;
        __syncthreads();
    }
}

struct SortState {
    unsigned long long* tmp = nullptr;
    int64_t cap_tmp = 0;
    uint32_t* hist = nullptr;
    int64_t cap_hist = 0;
    uint32_t* bs = nullptr;
    int64_t cap_bs = 0;
    DevStatus* st = nullptr;  // always clear: the scan's abort word
    hipEvent_t done = nullptr;  // end of the last sort's work: the next one waits for it
};

std::mutex g_smu;
std::map<int, SortState> g_ss;

template <class T>
hipError_t ensure(T*& p, int64_t& cap, int64_t need) {
    if (p && need <= cap) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    const hipError_t e = hipMalloc((void**)&p, (size_t)std::max<int64_t>(need, 1) * sizeof(T));
    if (e == hipSuccess) cap = std::max<int64_t>(need, 1);
    return e;
}

int bits_for(int64_t n) {  // bits of the largest index n - 1
    int b = 0;
    while (b < 31 && ((int64_t)1 << b) < n) ++b;
    return b;
}

unsigned grid_of(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384));
}

sj_status check_args(const sj_pair* pairs, int64_t n, int64_t n_r, int64_t n_s) {
    if (n < 0 || (n > 0 && !pairs) || n_r < 0 || n_s < 0 || n_r > ((int64_t)1 << 31) ||
        n_s > ((int64_t)1 << 31))
        return SJ_ERR_ARG;
    if ((uintptr_t)pairs & 7u) return SJ_ERR_ARG;
    if (n >= ((int64_t)1 << 32)) return SJ_ERR_TOO_LARGE;
    return SJ_OK;
}

// The passes of the sort over n >= 2 pairs with the given work buffers:
// tmp (n keys), hist (256 * tiles + 1 counters), bs (the scan's block sums),
// st (a status word whose flags are clear).  Launches only.
hipError_t sort_passes(unsigned long long* buf, int64_t n, int64_t n_r, int64_t n_s,
                       unsigned long long* tmp, uint32_t* hist, uint32_t* bs, DevStatus* st,
                       hipStream_t s) {
    const int64_t tiles = (n + kRsTile - 1) / kRsTile;
    const int64_t hlen = (int64_t)kRsDigits * tiles;
    // digit positions of the key (r << 32) | s that can be non-zero
    int shifts[8];
    int np = 0;
    for (int b = 0; b < bits_for(n_s); b += 8) shifts[np++] = b;
    for (int b = 0; b < bits_for(n_r); b += 8) shifts[np++] = 32 + b;
    hipLaunchKernelGGL(k_rs_swap, dim3(grid_of(n)), dim3(256), 0, s, buf, tmp, n);
    unsigned long long* src = tmp;
    unsigned long long* dst = buf;
    for (int p = 0; p < np; ++p) {
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)tiles), dim3(kRsNT), 0, s, src, n, shifts[p],
                           tiles, hist);
        const hipError_t e = scan_u32(hist, hlen, bs, &st->n_pairs, st, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)tiles), dim3(kRsNT), 0, s, src, dst, n,
                           shifts[p], tiles, hist);
        std::swap(src, dst);
    }
    // the sorted keys are in src; back to pairs in the caller's buffer
    hipLaunchKernelGGL(k_rs_swap, dim3(grid_of(n)), dim3(256), 0, s, src, buf, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Work buffers of sj_sort_pairs_noalloc: one fixed array per GPU, resident
// until the process ends (see include/sj.h).  In host code `scratch` names a
// host-side stand-in, not device memory: its device address is taken once per
// device with hipGetSymbolAddress, and only that address is used.
// ---------------------------------------------------------------------------
constexpr int64_t kNaTiles = (SJ_SORT_NOALLOC_MAX + kRsTile - 1) / kRsTile;
constexpr int64_t kNaHist = kRsDigits * kNaTiles + 1;
constexpr int64_t kNaTmpBytes = SJ_SORT_NOALLOC_MAX * 8;
constexpr int64_t kNaHistOff = kNaTmpBytes;
constexpr int64_t kNaBsOff = (kNaHistOff + kNaHist * 4 + 255) / 256 * 256;
constexpr int64_t kNaBsWords = (kRsDigits * kNaTiles + 8191) / 8192 + 1;  // >= scan block sums
constexpr int64_t kNaStOff = (kNaBsOff + kNaBsWords * 4 + 255) / 256 * 256;
constexpr int64_t kNaBytes = kNaStOff + (int64_t)((sizeof(DevStatus) + 255) / 256 * 256);

__device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kNaMaxDevices = 64;
std::mutex g_namu;
unsigned char* g_na_ptr[kNaMaxDevices] = {};  // device address of scratch per device

}  // namespace
}  // namespace sj

using namespace sj;

extern "C" sj_status sj_sort_pairs(sj_pair* pairs, int64_t n, int64_t n_r, int64_t n_s,
                                   void* stream) {
    const sj_status as = check_args(pairs, n, n_r, n_s);
    if (as != SJ_OK) return as;
    if (n < 2) return SJ_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SJ_ERR_DEVICE;
    const hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_smu);
    SortState& S = g_ss[dev];
    const int64_t tiles = (n + kRsTile - 1) / kRsTile;
    const int64_t hlen = (int64_t)kRsDigits * tiles;
    int64_t one = 0;
    if (ensure(S.tmp, S.cap_tmp, n) != hipSuccess || ensure(S.hist, S.cap_hist, hlen + 1) != hipSuccess ||
        ensure(S.bs, S.cap_bs, scan_block_sums_needed(hlen)) != hipSuccess)
        return SJ_ERR_OOM;
    if (!S.st) {
        if (ensure(S.st, one, 1) != hipSuccess) return SJ_ERR_OOM;
        if (hipMemset(S.st, 0, sizeof(DevStatus)) != hipSuccess) return SJ_ERR_DEVICE;
    }
    if (!S.done && hipEventCreateWithFlags(&S.done, hipEventDisableTiming) != hipSuccess) {
        S.done = nullptr;
        return SJ_ERR_DEVICE;
    }
    // the library buffers are shared by every sort on this device: a sort
    // enqueued on another stream runs after the previous one
    if (hipStreamWaitEvent(s, S.done, 0) != hipSuccess) return SJ_ERR_DEVICE;
    ProfRange pr("k_sort_pairs", s);
    if (sort_passes((unsigned long long*)pairs, n, n_r, n_s, S.tmp, S.hist, S.bs, S.st, s) !=
            hipSuccess ||
        hipEventRecord(S.done, s) != hipSuccess)
        return SJ_ERR_DEVICE;
    return SJ_OK;
}

extern "C" sj_status sj_sort_pairs_noalloc(sj_pair* pairs, int64_t n, int64_t n_r, int64_t n_s,
                                           void* stream) {
    const sj_status as = check_args(pairs, n, n_r, n_s);
    if (as != SJ_OK) return as;
    if (n > SJ_SORT_NOALLOC_MAX) {
        api_set_error("sj_sort_pairs_noalloc: more pairs than the fixed work buffer holds "
                      "(SJ_SORT_NOALLOC_MAX)");
        return SJ_ERR_TOO_LARGE;
    }
    if (n < 2) return SJ_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SJ_ERR_DEVICE;
    if (dev < 0 || dev >= kNaMaxDevices) return SJ_ERR_DEVICE;
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_namu);
        if (!g_na_ptr[dev]) {
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
                api_set_error("sj_sort_pairs_noalloc: no device address for the work buffer");
                return SJ_ERR_DEVICE;
            }
            g_na_ptr[dev] = (unsigned char*)p;
        }
        base = g_na_ptr[dev];
    }
    const hipStream_t s = (hipStream_t)stream;
    DevStatus* st = (DevStatus*)(base + kNaStOff);
    // the status word keeps the last call's contents: clear it (a fill
    // kernel, so the call can also be recorded into a graph)
    hipError_t e = launch_fill_u32((uint32_t*)st, 0u, (int64_t)(sizeof(DevStatus) / 4), s);
    if (e == hipSuccess)
        e = sort_passes((unsigned long long*)pairs, n, n_r, n_s, (unsigned long long*)base,
                        (uint32_t*)(base + kNaHistOff), (uint32_t*)(base + kNaBsOff), st, s);
    return e == hipSuccess ? SJ_OK : SJ_ERR_DEVICE;
}
