// Choosing the grid: data statistics, the paper's rule of thumb and the
// learned picker.
//
// Rule (Sec. 4.3.1 and 4.3.3): the tiles should be about one order of
// magnitude larger than the rectangles, i.e. with e = mean over R and S of
// the rectangle extent (w + h) / 2 in domain units,
//   K = clamp(round(1 / (10 e)), 1, SJ_K_MAX)  (square grid).
// The paper leaves the dense-tile split threshold open (it has none); the
// rule keeps the library default.
//
// Features (input of the learned picker), per side (R then S):
//   [0] log2(n + 1)
//   [1] log2(mean w + 1e-9), [2] log2(mean h + 1e-9)    (domain units)
//   [3] log2(std w + 1e-9),  [4] log2(std h + 1e-9)
//   [5 + 32 cy + cx] log2(1 + 1024 * share of the sampled centres in cell
//       (cx, cy) of a 32 x 32 grid over the domain); every phi-th rectangle
//       (phi = 100) is sampled, as the paper samples for its sweep-axis
//       histograms (Sec. 3.3).
// Moments are over every rectangle, accumulated in float64 with a fixed
// reduction order, so features and the rule's K are deterministic.
#include <cmath>
#include <map>
#include <mutex>

#include "sj_internal.hpp"
#include "sj_prof.hpp"

namespace sj {

int64_t mlp_params(int D);
hipError_t mlp_forward(const float* P, int D, const float* X, const float* mu, const float* sd,
                       int B, float* Y, float* act, hipStream_t s, float* h1_scratch);

namespace {

constexpr int kHist = 32;
constexpr int kPhi = 100;
constexpr int kSide = SJ_FEAT_SIDE;
constexpr int kFeatDim = SJ_FEAT_DIM;
constexpr int kFeatNT = 256;
constexpr int kFeatBlocks = 2048;
static_assert(kSide == 5 + kHist * kHist, "feature layout");

struct ChooseOut {
    double ebar, ebar_x;
    int32_t k_rule, k_pick, tau_pick, invalid, k_rule_x, pad;
    float y[2];
};

__device__ __forceinline__ bool rect_valid(const float4 r) {
    return isfinite(r.x) && isfinite(r.y) && isfinite(r.z) && isfinite(r.w) && r.x <= r.z &&
           r.y <= r.w;
}

// Per-block float64 partial sums (w, h, w^2, h^2) and the sampled centre
// histogram (integer atomics: order-independent).
__global__ __launch_bounds__(kFeatNT) void k_feat_partial(const float4* __restrict__ rects,
                                                         int64_t n, float x0, float y0, double iw,
                                                         double ih, double* __restrict__ part,
                                                         uint32_t* __restrict__ hist,
                                                         uint32_t* __restrict__ invalid) {
    __shared__ uint32_t h[kHist * kHist];
    __shared__ double red[4][kFeatNT / kWave];
    for (int i = threadIdx.x; i < kHist * kHist; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    double sw = 0, sh = 0, sww = 0, shh = 0;
    uint32_t bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float4 nxt = i < n ? rects[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    for (; i < n; i += stride) {
        const float4 r = nxt;  // the next rectangle is loaded while this one is summed
        if (i + stride < n) nxt = rects[i + stride];
        if (!rect_valid(r)) {
            ++bad;
            continue;
        }
        const double w = ((double)r.z - (double)r.x) * iw, hh = ((double)r.w - (double)r.y) * ih;
        sw += w;
        sh += hh;
        sww += w * w;
        shh += hh * hh;
    }
    // the sampled centres: rectangles phi * j (a strided pass over 1/phi of the input)
    const int64_t ns = (n + kPhi - 1) / kPhi;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ns;
         j += (int64_t)gridDim.x * blockDim.x) {
        const float4 r = rects[j * kPhi];
        if (!rect_valid(r)) continue;
        // explicit roundings (no FMA contraction): the cell decision is exact
        const double cx = __dmul_rn(__dmul_rn(__dsub_rn(__dmul_rn(0.5, __dadd_rn(r.x, r.z)), x0), iw), kHist);
        const double cy = __dmul_rn(__dmul_rn(__dsub_rn(__dmul_rn(0.5, __dadd_rn(r.y, r.w)), y0), ih), kHist);
        const int bx = (int)fmin(fmax(floor(cx), 0.0), (double)(kHist - 1));
        const int by = (int)fmin(fmax(floor(cy), 0.0), (double)(kHist - 1));
        atomicAdd(&h[by * kHist + bx], 1u);
    }
    double v[4] = {sw, sh, sww, shh};
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        for (int d = kWave / 2; d >= 1; d >>= 1) v[k] += __shfl_down(v[k], d, kWave);
        if (lane == 0) red[k][w] = v[k];
    }
    if (bad) atomicAdd(invalid, bad);
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0;
        for (int q = 0; q < kFeatNT / kWave; ++q) s += red[threadIdx.x][q];
        part[(int64_t)blockIdx.x * 4 + threadIdx.x] = s;
    }
    for (int i = threadIdx.x; i < kHist * kHist; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ __launch_bounds__(1024) void k_feat_final(const double* __restrict__ part, int nbR,
                                                     int nbS, int64_t nR, int64_t nS,
                                                     const uint32_t* __restrict__ hist,
                                                     const uint32_t* __restrict__ invalid,
                                                     float* __restrict__ feat,
                                                     ChooseOut* __restrict__ out) {
    __shared__ double s[2][4];
    __shared__ double red[8][128];
    {
        // 128 threads per (side, moment): strided partial sums, then a tree
        // (fixed order for a given block count)
        const int sk = threadIdx.x >> 7, l = threadIdx.x & 127;
        const int side = sk >> 2, k = sk & 3;
        const int nb = side == 0 ? nbR : nbS;
        const double* base = side == 0 ? part : part + (int64_t)nbR * 4;
        double acc = 0;
        for (int b = l; b < nb; b += 128) acc += base[(int64_t)b * 4 + k];
        red[sk][l] = acc;
        __syncthreads();
        for (int h = 64; h >= 1; h >>= 1) {
            if (l < h) red[sk][l] += red[sk][l + h];
            __syncthreads();
        }
        if (l == 0) s[side][k] = red[sk][0];
    }
    __syncthreads();
    for (int side = 0; side < 2; ++side) {
        const int64_t n = side == 0 ? nR : nS;
        float* f = feat + side * kSide;
        const uint32_t* hs = hist + side * kHist * kHist;
        const double nn = n > 0 ? (double)n : 1.0;
        if (threadIdx.x == 0) {
            const double mw = s[side][0] / nn, mh = s[side][1] / nn;
            const double vw = fmax(s[side][2] / nn - mw * mw, 0.0);
            const double vh = fmax(s[side][3] / nn - mh * mh, 0.0);
            f[0] = (float)log2((double)n + 1.0);
            f[1] = (float)log2(mw + 1e-9);
            f[2] = (float)log2(mh + 1e-9);
            f[3] = (float)log2(sqrt(vw) + 1e-9);
            f[4] = (float)log2(sqrt(vh) + 1e-9);
        }
        const int64_t sampled = n > 0 ? (n + kPhi - 1) / kPhi : 0;
        const double scale = sampled > 0 ? (double)(kHist * kHist) / (double)sampled : 0.0;
        for (int b = threadIdx.x; b < kHist * kHist; b += blockDim.x)
            f[5 + b] = (float)log2(1.0 + scale * (double)hs[b]);
    }
    if (threadIdx.x == 0) {
        const int64_t n = nR + nS;
        const double e = n > 0 ? (s[0][0] + s[0][1] + s[1][0] + s[1][1]) / (2.0 * (double)n) : 0.0;
        int k = 1;
        if (n > 0) {
            const double kk = e > 0 ? floor(1.0 / (10.0 * e) + 0.5) : (double)SJ_K_MAX;
            k = (int)fmin(fmax(kk, 1.0), (double)SJ_K_MAX);
        }
        out->ebar = e;
        out->k_rule = k;
        // 1-D partitioning (Sec. 4.3.1): stripes ten times the mean x-extent
        const double ex = n > 0 ? (s[0][0] + s[1][0]) / (double)n : 0.0;
        int kx1 = 1;
        if (n > 0) {
            const double kk = ex > 0 ? floor(1.0 / (10.0 * ex) + 0.5) : (double)SJ_K_MAX;
            kx1 = (int)fmin(fmax(kk, 1.0), (double)SJ_K_MAX);
        }
        out->ebar_x = ex;
        out->k_rule_x = kx1;
        out->k_pick = 0;
        out->tau_pick = 0;
        out->invalid = (int32_t)*invalid;
        out->y[0] = out->y[1] = 0.f;
    }
}

// Learned pick from the network output y (standardised targets):
//   log2 K = y0 * sd0 + mu0,  log2 tau = y1 * sd1 + mu1.
__global__ void k_pick(const float* __restrict__ Y, const float* __restrict__ ystat,
                       ChooseOut* __restrict__ out) {
    const float l2k = Y[0] * ystat[2] + ystat[0];
    const float l2t = Y[1] * ystat[3] + ystat[1];
    out->y[0] = l2k;
    out->y[1] = l2t;
    const float k = rintf(exp2f(fminf(fmaxf(l2k, 0.f), 13.f)));
    const float t = rintf(exp2f(fminf(fmaxf(l2t, 3.f), 20.f)));
    out->k_pick = (int32_t)fminf(fmaxf(k, 1.f), (float)SJ_K_MAX);
    out->tau_pick = (int32_t)t;
}

// zero the histograms, the invalid count and (empty sides) the partial sums
// with a kernel rather than a memset node, so the sequence can be captured
__global__ void k_feat_zero(uint32_t* __restrict__ hist, int nh, double* __restrict__ pR,
                            double* __restrict__ pS) {
    for (int i = threadIdx.x; i < nh; i += blockDim.x) hist[i] = 0u;
    if (threadIdx.x < 4) {
        if (pR) pR[threadIdx.x] = 0.0;
        if (pS) pS[threadIdx.x] = 0.0;
    }
}

template <class T>
hipError_t alloc(T*& p, int64_t n) {
    if (p) return hipSuccess;
    return hipMalloc((void**)&p, (size_t)n * sizeof(T));
}

struct ChooseState {
    float* feat = nullptr;       // [kFeatDim]
    double* part = nullptr;      // [2 * kFeatBlocks * 4]
    uint32_t* hist = nullptr;    // [2 * 1024 + 1]  (last word: invalid-rect count)
    ChooseOut* out = nullptr;
    ChooseOut* host = nullptr;   // pinned
    float* y = nullptr;          // [2]
    float* h1 = nullptr;         // [64] hidden layer of the picker
    float* picker = nullptr;     // mu | sd | ystat | params
    int64_t picker_n = 0;
    bool loaded = false;
};

std::mutex g_cmu;
std::map<int, ChooseState> g_cs;

sj_status state_for(int dev, ChooseState** out) {
    ChooseState& c = g_cs[dev];
    if (!c.host) {
        if (alloc(c.feat, kFeatDim) != hipSuccess || alloc(c.part, 2 * kFeatBlocks * 4) != hipSuccess ||
            alloc(c.hist, 2 * kHist * kHist + 1) != hipSuccess || alloc(c.out, 1) != hipSuccess ||
            alloc(c.y, 2) != hipSuccess || alloc(c.h1, 64) != hipSuccess)
            return SJ_ERR_OOM;
        if (hipHostMalloc((void**)&c.host, sizeof(ChooseOut), hipHostMallocDefault) != hipSuccess) {
            c.host = nullptr;
            return SJ_ERR_OOM;
        }
    }
    *out = &c;
    return SJ_OK;
}

int feat_blocks(int64_t n) {
    const int64_t b = (n + kFeatNT * 4 - 1) / (kFeatNT * 4);
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), kFeatBlocks);
}

sj_status domain_of(const sj_grid* g, float d[4]) {
    d[0] = 0.f;
    d[1] = 0.f;
    d[2] = 1.f;
    d[3] = 1.f;
    if (g && !(g->domain[0] == 0.f && g->domain[1] == 0.f && g->domain[2] == 0.f &&
               g->domain[3] == 0.f)) {
        for (int i = 0; i < 4; ++i) d[i] = g->domain[i];
    }
    const float w = d[2] - d[0], h = d[3] - d[1];
    if (!std::isfinite(w) || !std::isfinite(h) || !(w > 0.f) || !(h > 0.f)) return SJ_ERR_ARG;
    return SJ_OK;
}

// Features of (R, S) into c.feat and the rule into c.out (no synchronisation).
hipError_t launch_features(ChooseState& c, const float* R, int64_t nR, const float* S, int64_t nS,
                           const float d[4], hipStream_t s) {
    ProfRange pr("k_features", s);
    const double iw = 1.0 / ((double)d[2] - (double)d[0]), ih = 1.0 / ((double)d[3] - (double)d[1]);
    const int nbR = feat_blocks(nR), nbS = feat_blocks(nS);
    hipLaunchKernelGGL(k_feat_zero, dim3(1), dim3(1024), 0, s, c.hist, 2 * kHist * kHist + 1,
                       nR > 0 ? nullptr : c.part, nS > 0 ? nullptr : c.part + (int64_t)nbR * 4);
    if (nR > 0)
        hipLaunchKernelGGL(k_feat_partial, dim3(nbR), dim3(kFeatNT), 0, s, (const float4*)R, nR, d[0],
                           d[1], iw, ih, c.part, c.hist, c.hist + 2 * kHist * kHist);
    if (nS > 0)
        hipLaunchKernelGGL(k_feat_partial, dim3(nbS), dim3(kFeatNT), 0, s, (const float4*)S, nS, d[0],
                           d[1], iw, ih, c.part + (int64_t)nbR * 4, c.hist + kHist * kHist,
                           c.hist + 2 * kHist * kHist);
    hipLaunchKernelGGL(k_feat_final, dim3(1), dim3(1024), 0, s, c.part, nbR, nbS, nR, nS, c.hist,
                       c.hist + 2 * kHist * kHist, c.feat, c.out);
    return hipGetLastError();
}

bool args_ok(const float* R, int64_t nR, const float* S, int64_t nS) {
    if (nR < 0 || nS < 0 || (nR > 0 && !R) || (nS > 0 && !S)) return false;
    if (((uintptr_t)R & 15u) || ((uintptr_t)S & 15u)) return false;
    return true;
}

}  // namespace
}  // namespace sj

using namespace sj;

extern "C" {

int32_t sj_rule_k(double mean_extent) {
    if (!(mean_extent > 0.0)) return mean_extent == 0.0 ? SJ_K_MAX : 1;
    const double k = std::floor(1.0 / (10.0 * mean_extent) + 0.5);
    return (int32_t)std::fmin(std::fmax(k, 1.0), (double)SJ_K_MAX);
}

sj_status sj_features(const float* R, int64_t nR, const float* S, int64_t nS, const sj_grid* g,
                      float* feat, double* mean_extent, void* stream) {
    if (!args_ok(R, nR, S, nS) || !feat) return SJ_ERR_ARG;
    float d[4];
    if (domain_of(g, d) != SJ_OK) return SJ_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SJ_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_cmu);
    ChooseState* c = nullptr;
    sj_status st = state_for(dev, &c);
    if (st != SJ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (launch_features(*c, R, nR, S, nS, d, s) != hipSuccess) return SJ_ERR_DEVICE;
    if (hipMemcpyAsync(feat, c->feat, kFeatDim * sizeof(float), hipMemcpyDeviceToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(c->host, c->out, sizeof(ChooseOut), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SJ_ERR_DEVICE;
    if (c->host->invalid) return SJ_ERR_RECT;
    if (mean_extent) *mean_extent = c->host->ebar;
    return SJ_OK;
}

sj_status sj_picker_load(const float* blob, int64_t n) {
    const int64_t need = 2 * (int64_t)kFeatDim + 4 + mlp_params(kFeatDim);
    if (!blob || n != need) return SJ_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SJ_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_cmu);
    ChooseState* c = nullptr;
    sj_status st = state_for(dev, &c);
    if (st != SJ_OK) return st;
    if (alloc(c->picker, need) != hipSuccess) return SJ_ERR_OOM;
    if (hipMemcpy(c->picker, blob, (size_t)need * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return SJ_ERR_DEVICE;
    c->picker_n = need;
    c->loaded = true;
    return SJ_OK;
}

void sj_picker_unload(void) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_cmu);
    auto it = g_cs.find(dev);
    if (it != g_cs.end()) it->second.loaded = false;
}

int32_t sj_picker_loaded(void) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_cmu);
    auto it = g_cs.find(dev);
    return it != g_cs.end() && it->second.loaded ? 1 : 0;
}

sj_status sj_choose_grid(const float* R, int64_t nR, const float* S, int64_t nS, sj_grid* g,
                         sj_choice* info, void* stream) {
    if (!g || !args_ok(R, nR, S, nS)) return SJ_ERR_ARG;
    if (g->k < 0 || g->k > SJ_K_MAX || g->split_tau < 0) return SJ_ERR_ARG;
    float d[4];
    if (domain_of(g, d) != SJ_OK) return SJ_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SJ_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_cmu);
    ChooseState* c = nullptr;
    sj_status st = state_for(dev, &c);
    if (st != SJ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (launch_features(*c, R, nR, S, nS, d, s) != hipSuccess) return SJ_ERR_DEVICE;
    const bool stripes = (g->flags & SJ_STRIPES) != 0;
    const bool learned = c->loaded && !(g->flags & SJ_RULE_ONLY) && !stripes;
    if (learned) {
        ProfRange pr("k_picker", s);
        const float* mu = c->picker;
        const float* sd = mu + kFeatDim;
        const float* ystat = sd + kFeatDim;
        const float* P = ystat + 4;
        if (mlp_forward(P, kFeatDim, c->feat, mu, sd, 1, c->y, nullptr, s, c->h1) != hipSuccess)
            return SJ_ERR_DEVICE;
        hipLaunchKernelGGL(k_pick, dim3(1), dim3(1), 0, s, c->y, ystat, c->out);
    }
    if (hipMemcpyAsync(c->host, c->out, sizeof(ChooseOut), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SJ_ERR_DEVICE;
    const ChooseOut o = *c->host;
    if (o.invalid) return SJ_ERR_RECT;
    // a K x K grid costs O(K^2) per pass whatever the input size, so a chosen
    // 2-D grid keeps K^2 <= 8 (nR + nS): the fastest measured grid of every
    // picker-corpus instance has fewer tiles than that, and inputs far smaller
    // than the corpus's (a batch's small joins) get no grid of mostly empty tiles
    int32_t kcap = SJ_K_MAX;
    if (!stripes) {
        const double c = std::floor(std::sqrt(8.0 * (double)(nR + nS)));
        kcap = (int32_t)std::max(1.0, std::min(c, (double)SJ_K_MAX));
    }
    if (g->k == 0) g->k = std::min(learned ? o.k_pick : (stripes ? o.k_rule_x : o.k_rule), kcap);
    if (g->split_tau == 0 && learned) g->split_tau = o.tau_pick;
    if (info) {
        info->mean_extent = o.ebar;
        info->k_rule = stripes ? o.k_rule_x : o.k_rule;
        info->mean_x_extent = o.ebar_x;
        info->k_learned = learned ? o.k_pick : 0;
        info->tau_learned = learned ? o.tau_pick : 0;
        info->used_learned = learned ? 1 : 0;
        info->k_cap = kcap;
    }
    return SJ_OK;
}

}  // extern "C"
