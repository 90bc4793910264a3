// Learned pruning threshold: pair features and a 256-128-128-1 MLP with BF16
// weights and inputs and FP32 accumulation, trained on the GPU.
//
// Features of a pair (A, B), 256 floats:
//  [0,128)   shared 4-mer spectrum folded by base complement: 4-mer code
//            c = 4 two-bit codes (A0 C1 G2 T3, first base high); class
//            q = c if c < 128 else c ^ 0xFF; f_X[q] = count / (|X| - 3);
//            x[q] = 128 * min(f_A[q], f_B[q]).
//  [128,254) diagonal 12-mer hit histogram: every (i, j) with equal 12-mers
//            at A[i..] and B[j..], ignoring 12-mers occurring more than 64
//            times in A; hits counted per diagonal band b = (j - i + |A|) / 64;
//            band count c -> bin floor(log2((1 + c)^4)) capped at 125 (exact
//            integer arithmetic); x[128 + bin] = ln(1 + number of bands in bin).
//  [254,256) ln|A|, ln|B| divided by ln(4e6).
// The model standardises features with stored means and deviations, rounds to
// BF16 (round to nearest even), runs ReLU layers in FP32 and predicts
// y = ln(1 + S); the threshold is T = floor(0.9 * (exp(y) - 1)).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "swmi.h"
#include "swmi_host.h"
#include "swmi_internal.h"

using namespace swmi;

#define HIP_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(SW_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

namespace swmi {

constexpr int kFeat = 256, kHid = 128;
constexpr int kK12 = 1 << 24;     // 12-mer codes
constexpr int kCap = 64;          // 12-mers more frequent than this in A are ignored
constexpr int kBins = 126;
// parameter vector: W1[256][128], b1[128], W2[128][128], b2[128], W3[128], b3
constexpr int64_t kOffW1 = 0, kOffB1 = kOffW1 + kFeat * kHid, kOffW2 = kOffB1 + kHid,
                  kOffB2 = kOffW2 + kHid * kHid, kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid,
                  kNParams = kOffB3 + 1;

__device__ __host__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

__device__ __host__ __forceinline__ float bf16_to_f32(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// ------------------------------------------------------------------------ feature kernels

// 4-mer class counts of one sequence into cnt[128].
__global__ __launch_bounds__(256) void kmer4_kernel(const uint8_t* __restrict__ codes, int64_t n,
                                                    unsigned int* __restrict__ cnt) {
    __shared__ unsigned int h[128];
    if (threadIdx.x < 128) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p + 3 < n; p += (int64_t)gridDim.x * blockDim.x) {
        const unsigned c = ((unsigned)codes[p] << 6) | ((unsigned)codes[p + 1] << 4) | ((unsigned)codes[p + 2] << 2) |
                           (unsigned)codes[p + 3];
        atomicAdd(&h[c < 128 ? c : (c ^ 0xFFu)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 128 && h[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
}

__device__ __forceinline__ uint32_t kmer12(const uint8_t* c, int64_t p) {
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) v = (v << 2) | c[p + k];
    return v;
}

__global__ void k12_count_kernel(const uint8_t* __restrict__ a, int64_t n, unsigned int* __restrict__ counts) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p + 11 < n; p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&counts[kmer12(a, p)], 1u);
}

// For every 12-mer of B: hits against A's 12-mer counts, but only for codes seen
// at most kCap times; band counts by diagonal. Needs the positions of A's
// 12-mers: we scan A's positions per code through a bucket index.
__global__ void k12_fill_kernel(const uint8_t* __restrict__ a, int64_t n, const unsigned int* __restrict__ start,
                                unsigned int* __restrict__ cursor, unsigned int* __restrict__ pos) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p + 11 < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = kmer12(a, p);
        const unsigned int slot = atomicAdd(&cursor[k], 1u);
        pos[start[k] + slot] = (unsigned int)p;
    }
}

__global__ void k12_hits_kernel(const uint8_t* __restrict__ b, int64_t nb, int64_t na,
                                const unsigned int* __restrict__ counts, const unsigned int* __restrict__ start,
                                const unsigned int* __restrict__ pos, unsigned int* __restrict__ band) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j + 11 < nb; j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = kmer12(b, j);
        const unsigned int c = counts[k];
        if (c == 0 || c > (unsigned)kCap) continue;
        const unsigned int s0 = start[k];
        for (unsigned int t = 0; t < c; ++t) {
            const int64_t i = pos[s0 + t];
            atomicAdd(&band[(j - i + na) / 64], 1u);
        }
    }
}

// Exclusive scan of the 2^24 12-mer counts (one block per 4096-entry tile, then a fix-up).
__global__ __launch_bounds__(256) void scan_tiles_kernel(const unsigned int* __restrict__ in, unsigned int* __restrict__ out,
                                                         unsigned int* __restrict__ tile_sum) {
    __shared__ unsigned int s[256];
    const int64_t base = (int64_t)blockIdx.x * 4096;
    unsigned int v[16];
    unsigned int acc = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        v[k] = in[base + threadIdx.x * 16 + k];
        acc += v[k];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned int x = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += x;
        __syncthreads();
    }
    unsigned int run = s[threadIdx.x] - acc;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        out[base + threadIdx.x * 16 + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) tile_sum[blockIdx.x] = s[255];
}

__global__ __launch_bounds__(1024) void scan_sums_kernel(unsigned int* __restrict__ tile_sum, int n) {
    // single block: exclusive scan of n <= 4096 tile sums
    __shared__ unsigned int s[4096];
    for (int i = threadIdx.x; i < n; i += blockDim.x) s[i] = tile_sum[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int run = 0;
        for (int i = 0; i < n; ++i) {
            const unsigned int x = s[i];
            s[i] = run;
            run += x;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) tile_sum[i] = s[i];
}

__global__ void scan_fix_kernel(unsigned int* __restrict__ out, const unsigned int* __restrict__ tile_sum) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < kK12) out[i] += tile_sum[i / 4096];
}

__device__ __forceinline__ int log_bin(unsigned int c) {
    // floor(log2((1 + c)^4)), exact, capped at kBins - 1
    const unsigned __int128 x = (unsigned __int128)(1ull + c);
    const unsigned __int128 x4 = x * x * x * x;
    const uint64_t hi = (uint64_t)(x4 >> 64), lo = (uint64_t)x4;
    const int lg = hi ? 127 - __clzll((long long)hi) : 63 - __clzll((long long)lo);
    return lg < kBins - 1 ? lg : kBins - 1;
}

__global__ void band_hist_kernel(const unsigned int* __restrict__ band, int64_t nbands, unsigned int* __restrict__ hist) {
    __shared__ unsigned int h[kBins];
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nbands; k += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[log_bin(band[k])], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ void feature_finish_kernel(const unsigned int* __restrict__ cnt_a, const unsigned int* __restrict__ cnt_b,
                                      const unsigned int* __restrict__ hist, int64_t na, int64_t nb,
                                      float* __restrict__ out) {
    const int t = threadIdx.x;
    if (t < 128) {
        const double fa = na >= 4 ? (double)cnt_a[t] / (double)(na - 3) : 0.0;
        const double fb = nb >= 4 ? (double)cnt_b[t] / (double)(nb - 3) : 0.0;
        out[t] = (float)(128.0 * (fa < fb ? fa : fb));
    } else if (t < 128 + kBins) {
        out[t] = (float)log1p((double)hist[t - 128]);
    } else if (t == 254) {
        out[t] = (float)(log((double)(na > 0 ? na : 1)) / log(4.0e6));
    } else if (t == 255) {
        out[t] = (float)(log((double)(nb > 0 ? nb : 1)) / log(4.0e6));
    }
}

// ------------------------------------------------------------------------ MLP kernels

// One block of 128 threads per sample.  x: bf16 [n][256]; activations h1, h2
// are stored rounded to bf16 (the next layer's input) as float.
__global__ __launch_bounds__(128) void mlp_fwd_kernel(const uint16_t* __restrict__ x, int n,
                                                      const uint16_t* __restrict__ w, const float* __restrict__ p,
                                                      float* __restrict__ h1, float* __restrict__ h2,
                                                      float* __restrict__ y) {
    __shared__ float xs[kFeat];
    __shared__ float a1[kHid];
    __shared__ float a2[kHid];
    const int t = threadIdx.x;
    for (int s = blockIdx.x; s < n; s += gridDim.x) {
        xs[t] = bf16_to_f32(x[(int64_t)s * kFeat + t]);
        xs[t + 128] = bf16_to_f32(x[(int64_t)s * kFeat + t + 128]);
        __syncthreads();
        float acc = p[kOffB1 + t];
        for (int i = 0; i < kFeat; ++i) acc = fmaf(xs[i], bf16_to_f32(w[kOffW1 + i * kHid + t]), acc);
        const float r1 = bf16_to_f32(f32_to_bf16(acc > 0.f ? acc : 0.f));
        a1[t] = r1;
        h1[(int64_t)s * kHid + t] = r1;
        __syncthreads();
        float acc2 = p[kOffB2 + t];
        for (int i = 0; i < kHid; ++i) acc2 = fmaf(a1[i], bf16_to_f32(w[kOffW2 + i * kHid + t]), acc2);
        const float r2 = bf16_to_f32(f32_to_bf16(acc2 > 0.f ? acc2 : 0.f));
        a2[t] = r2;
        h2[(int64_t)s * kHid + t] = r2;
        __syncthreads();
        if (t == 0) {
            float acc3 = p[kOffB3];
            for (int i = 0; i < kHid; ++i) acc3 = fmaf(a2[i], bf16_to_f32(w[kOffW3 + i]), acc3);
            y[s] = acc3;
        }
        __syncthreads();
    }
}

// Per-sample deltas of the MSE loss mean((y - t)^2): d3 = dL/dy, d2 = dL/dz2, d1 = dL/dz1.
// dLoss/dy per sample: squared error (quantile <= 0) or pinball loss at the quantile.
__device__ __forceinline__ float loss_grad(float y, float t, float quantile, int n) {
    if (quantile <= 0.f) return 2.f * (y - t) / (float)n;
    const float g = y > t ? 1.f - quantile : (y < t ? -quantile : 0.f);
    return g / (float)n;
}

__global__ __launch_bounds__(128) void mlp_delta_kernel(int n, const uint16_t* __restrict__ w,
                                                        const float* __restrict__ h1, const float* __restrict__ h2,
                                                        const float* __restrict__ y, const float* __restrict__ tgt,
                                                        float quantile, float* __restrict__ d3,
                                                        float* __restrict__ d2, float* __restrict__ d1) {
    __shared__ float s2[kHid];
    const int t = threadIdx.x;
    for (int s = blockIdx.x; s < n; s += gridDim.x) {
        const float dy = loss_grad(y[s], tgt[s], quantile, n);
        if (t == 0) d3[s] = dy;
        const float g2 = h2[(int64_t)s * kHid + t] > 0.f ? bf16_to_f32(w[kOffW3 + t]) * dy : 0.f;
        s2[t] = g2;
        d2[(int64_t)s * kHid + t] = g2;
        __syncthreads();
        float acc = 0.f;
        for (int k = 0; k < kHid; ++k) acc = fmaf(bf16_to_f32(w[kOffW2 + t * kHid + k]), s2[k], acc);
        d1[(int64_t)s * kHid + t] = h1[(int64_t)s * kHid + t] > 0.f ? acc : 0.f;
        __syncthreads();
    }
}

// Parameter gradients, one thread per parameter, samples summed in index order.
__global__ void mlp_grad_kernel(int n, const uint16_t* __restrict__ x, const float* __restrict__ h1,
                                const float* __restrict__ h2, const float* __restrict__ d3,
                                const float* __restrict__ d2, const float* __restrict__ d1, float* __restrict__ grad) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= kNParams) return;
    float acc = 0.f;
    if (q < kOffB1) {
        const int i = (int)(q / kHid), j = (int)(q % kHid);
        for (int s = 0; s < n; ++s) acc = fmaf(bf16_to_f32(x[(int64_t)s * kFeat + i]), d1[(int64_t)s * kHid + j], acc);
    } else if (q < kOffW2) {
        const int j = (int)(q - kOffB1);
        for (int s = 0; s < n; ++s) acc += d1[(int64_t)s * kHid + j];
    } else if (q < kOffB2) {
        const int i = (int)((q - kOffW2) / kHid), j = (int)((q - kOffW2) % kHid);
        for (int s = 0; s < n; ++s) acc = fmaf(h1[(int64_t)s * kHid + i], d2[(int64_t)s * kHid + j], acc);
    } else if (q < kOffW3) {
        const int j = (int)(q - kOffB2);
        for (int s = 0; s < n; ++s) acc += d2[(int64_t)s * kHid + j];
    } else if (q < kOffB3) {
        const int i = (int)(q - kOffW3);
        for (int s = 0; s < n; ++s) acc = fmaf(h2[(int64_t)s * kHid + i], d3[s], acc);
    } else {
        for (int s = 0; s < n; ++s) acc += d3[s];
    }
    grad[q] = acc;
}

// Adam on FP32 master parameters; refreshes the BF16 copies of the weights
// (biases stay FP32 and are read from the master vector).
__global__ void adam_kernel(float* __restrict__ master, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps,
                            float bc1, float bc2, uint16_t* __restrict__ wbf) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    const float upd = lr * (mq / bc1) / (sqrtf(vq / bc2) + eps);
    const float w = master[q] - upd;
    master[q] = w;
    wbf[q] = f32_to_bf16(w);
}

// Standardise, round to bf16.
__global__ void standardize_kernel(const float* __restrict__ f, int64_t n, const float* __restrict__ mean,
                                   const float* __restrict__ inv_std, uint16_t* __restrict__ xb) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * kFeat) return;
    const int k = (int)(i % kFeat);
    xb[i] = f32_to_bf16((f[i] - mean[k]) * inv_std[k]);
}

}  // namespace swmi

// ------------------------------------------------------------------------ model object

struct sw_model {
    std::vector<float> mean, inv_std;  // 256 each
    std::vector<float> params;          // kNParams, FP32 master values
};

// ------------------------------------------------------------------------ host helpers

namespace {

// Feature workspace for one pair: codes, 4-mer counts, 12-mer index, bands.
size_t feat_ws(int64_t na, int64_t nb) {
    const int64_t nbands = (na + nb) / 64 + 2;
    return align_up((size_t)na + 64, 256) + align_up((size_t)nb + 64, 256) + 2 * 512 + align_up(kBins * 4, 256) +
           3 * (size_t)kK12 * 4 + 4096 * 4 + align_up((size_t)na * 4 + 64, 256) + align_up((size_t)nbands * 4, 256) + 256;
}

sw_status features_one(sw_context* ctx, const uint8_t* d_a, int64_t na, const uint8_t* d_b, int64_t nb,
                       float* d_out, uint8_t* ws) {
    hipStream_t s = ctx->stream;
    const int64_t nbands = (na + nb) / 64 + 2;
    uint8_t* ca = ws;
    uint8_t* cb = ca + align_up((size_t)na + 64, 256);
    unsigned int* cnt_a = (unsigned int*)(cb + align_up((size_t)nb + 64, 256));
    unsigned int* cnt_b = cnt_a + 128;
    unsigned int* hist = cnt_b + 128;
    unsigned int* counts = (unsigned int*)((uint8_t*)hist + align_up(kBins * 4, 256));
    unsigned int* start = counts + kK12;
    unsigned int* cursor = start + kK12;
    unsigned int* tiles = cursor + kK12;
    unsigned int* pos = tiles + 4096;
    unsigned int* band = (unsigned int*)((uint8_t*)pos + align_up((size_t)na * 4 + 64, 256));
    unsigned long long* bad = (unsigned long long*)((uint8_t*)band + align_up((size_t)nbands * 4, 256));
    HIP_TRY(launch_zero(bad, 16, s));
    const sw_scoring dna{1, 3, 5, 2, nullptr};  // the features are DNA k-mers
    const EncTable et = enc_table(&dna);
    HIP_TRY(launch_encode(d_a, na, ca, 0, 64, 0, et, bad, s));
    HIP_TRY(launch_encode(d_b, nb, cb, 0, 64, 0, et, bad + 1, s));
    HIP_TRY(launch_zero(cnt_a, 2 * 512 + align_up(kBins * 4, 256), s));
    HIP_TRY(launch_zero(counts, (size_t)kK12 * 4, s));
    HIP_TRY(launch_zero(cursor, (size_t)kK12 * 4, s));
    HIP_TRY(launch_zero(band, (size_t)nbands * 4, s));
    const int g = 2048;
    hipLaunchKernelGGL(kmer4_kernel, dim3(g), dim3(256), 0, s, ca, na, cnt_a);
    hipLaunchKernelGGL(kmer4_kernel, dim3(g), dim3(256), 0, s, cb, nb, cnt_b);
    hipLaunchKernelGGL(k12_count_kernel, dim3(g), dim3(256), 0, s, ca, na, counts);
    hipLaunchKernelGGL(scan_tiles_kernel, dim3(kK12 / 4096), dim3(256), 0, s, counts, start, tiles);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, tiles, kK12 / 4096);
    hipLaunchKernelGGL(scan_fix_kernel, dim3(kK12 / 256), dim3(256), 0, s, start, tiles);
    hipLaunchKernelGGL(k12_fill_kernel, dim3(g), dim3(256), 0, s, ca, na, start, cursor, pos);
    hipLaunchKernelGGL(k12_hits_kernel, dim3(g), dim3(256), 0, s, cb, nb, na, counts, start, pos, band);
    hipLaunchKernelGGL(band_hist_kernel, dim3(256), dim3(256), 0, s, band, nbands, hist);
    hipLaunchKernelGGL(feature_finish_kernel, dim3(1), dim3(256), 0, s, cnt_a, cnt_b, hist, na, nb, d_out);
    HIP_TRY(hipGetLastError());
    return SW_OK;
}

}  // namespace

// ------------------------------------------------------------------------ C ABI

extern "C" size_t sw_features_workspace_size(sw_context* ctx, const int64_t* offs_a, const int64_t* offs_b,
                                             int32_t n_pairs) {
    if (!ctx || n_pairs < 0 || (n_pairs && (!offs_a || !offs_b))) return 0;
    size_t m = 0;
    for (int32_t p = 0; p < n_pairs; ++p)
        m = std::max(m, feat_ws(offs_a[p + 1] - offs_a[p], offs_b[p + 1] - offs_b[p]));
    return m;
}

extern "C" sw_status sw_features_dev(sw_context* ctx, const uint8_t* d_seqs_a, const int64_t* offs_a,
                                     const uint8_t* d_seqs_b, const int64_t* offs_b, int32_t n_pairs, float* d_out,
                                     void* d_workspace, size_t workspace_bytes) {
    if (!ctx || n_pairs < 0 || (n_pairs && (!offs_a || !offs_b || !d_seqs_a || !d_seqs_b || !d_out)))
        return fail(SW_EINVAL, "sw_features_dev: bad arguments");
    const size_t need = sw_features_workspace_size(ctx, offs_a, offs_b, n_pairs);
    if (n_pairs && (!d_workspace || workspace_bytes < need))
        return fail(SW_ENOMEM, "sw_features_dev: workspace of %zu bytes, need %zu", workspace_bytes, need);
    HIP_TRY(hipSetDevice(ctx->device));
    for (int32_t p = 0; p < n_pairs; ++p) {
        const int64_t na = offs_a[p + 1] - offs_a[p], nb = offs_b[p + 1] - offs_b[p];
        if (na < 0 || nb < 0) return fail(SW_EINVAL, "sw_features_dev: offsets of pair %d decrease", p);
        if (na >= ((int64_t)1 << 32) || nb >= ((int64_t)1 << 32))
            return fail(SW_EUNSUPPORTED, "sw_features_dev: sequence of 2^32 or more");
        sw_status st = features_one(ctx, d_seqs_a + offs_a[p], na, d_seqs_b + offs_b[p], nb,
                                    d_out + (int64_t)p * kFeat, (uint8_t*)d_workspace);
        if (st != SW_OK) return st;
    }
    return SW_OK;
}

extern "C" sw_status sw_mlp_forward_dev(sw_context* ctx, const uint16_t* d_x, int32_t n, const uint16_t* d_wbf,
                                        const float* d_params, float* d_h1, float* d_h2, float* d_y) {
    if (!ctx || n < 0 || (n && (!d_x || !d_wbf || !d_params || !d_h1 || !d_h2 || !d_y)))
        return fail(SW_EINVAL, "sw_mlp_forward_dev: bad arguments");
    if (!n) return SW_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(std::min(n, 8192)), dim3(128), 0, ctx->stream, d_x, n, d_wbf, d_params,
                       d_h1, d_h2, d_y);
    HIP_TRY(hipGetLastError());
    return SW_OK;
}

extern "C" sw_status sw_mlp_backward_dev(sw_context* ctx, const uint16_t* d_x, int32_t n, const uint16_t* d_wbf,
                                         const float* d_h1, const float* d_h2, const float* d_y,
                                         const float* d_target, float quantile, float* d_scratch, float* d_grad) {
    if (!ctx || n <= 0 || !d_x || !d_wbf || !d_h1 || !d_h2 || !d_y || !d_target || !d_scratch || !d_grad)
        return fail(SW_EINVAL, "sw_mlp_backward_dev: bad arguments");
    if (!(quantile < 1.f)) return fail(SW_EINVAL, "sw_mlp_backward_dev: quantile must be < 1");
    HIP_TRY(hipSetDevice(ctx->device));
    float* d3 = d_scratch;
    float* d2 = d3 + align_up((size_t)n, 64);
    float* d1 = d2 + (size_t)n * kHid;
    hipLaunchKernelGGL(mlp_delta_kernel, dim3(std::min(n, 8192)), dim3(128), 0, ctx->stream, n, d_wbf, d_h1, d_h2,
                       d_y, d_target, quantile, d3, d2, d1);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)((kNParams + 255) / 256)), dim3(256), 0, ctx->stream, n, d_x,
                       d_h1, d_h2, d3, d2, d1, d_grad);
    HIP_TRY(hipGetLastError());
    return SW_OK;
}

extern "C" sw_status sw_mlp_adam_dev(sw_context* ctx, float* d_params, float* d_m, float* d_v, const float* d_grad,
                                     int32_t step, float lr, float beta1, float beta2, float eps, uint16_t* d_wbf) {
    if (!ctx || !d_params || !d_m || !d_v || !d_grad || !d_wbf || step < 1)
        return fail(SW_EINVAL, "sw_mlp_adam_dev: bad arguments");
    HIP_TRY(hipSetDevice(ctx->device));
    const float bc1 = 1.f - powf(beta1, (float)step), bc2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((kNParams + 255) / 256)), dim3(256), 0, ctx->stream, d_params, d_m,
                       d_v, d_grad, kNParams, lr, beta1, beta2, eps, bc1, bc2, d_wbf);
    HIP_TRY(hipGetLastError());
    return SW_OK;
}

extern "C" sw_status sw_mlp_standardize_dev(sw_context* ctx, const float* d_feat, int32_t n, const float* d_mean,
                                            const float* d_inv_std, uint16_t* d_x) {
    if (!ctx || n < 0 || (n && (!d_feat || !d_mean || !d_inv_std || !d_x)))
        return fail(SW_EINVAL, "sw_mlp_standardize_dev: bad arguments");
    if (!n) return SW_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    const int64_t tot = (int64_t)n * kFeat;
    hipLaunchKernelGGL(standardize_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream, d_feat,
                       (int64_t)n, d_mean, d_inv_std, d_x);
    HIP_TRY(hipGetLastError());
    return SW_OK;
}

extern "C" int64_t sw_mlp_param_count(void) { return kNParams; }

// Model file: "SWMLP001", int32 256, int32 128, float mean[256], float inv_std[256], float params[kNParams].
extern "C" sw_status sw_model_load(sw_context* ctx, const char* path, sw_model** out) {
    (void)ctx;
    if (!path || !out) return fail(SW_EINVAL, "sw_model_load: NULL argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(SW_EINVAL, "sw_model_load: cannot open %s", path);
    char magic[8];
    int32_t dims[2];
    sw_model* m = new (std::nothrow) sw_model();
    bool ok = m && std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "SWMLP001", 8) == 0 &&
              std::fread(dims, 4, 2, f) == 2 && dims[0] == kFeat && dims[1] == kHid;
    if (ok) {
        m->mean.resize(kFeat);
        m->inv_std.resize(kFeat);
        m->params.resize(kNParams);
        ok = std::fread(m->mean.data(), 4, kFeat, f) == (size_t)kFeat &&
             std::fread(m->inv_std.data(), 4, kFeat, f) == (size_t)kFeat &&
             std::fread(m->params.data(), 4, kNParams, f) == (size_t)kNParams;
    }
    std::fclose(f);
    if (!ok) {
        delete m;
        return fail(SW_EINVAL, "sw_model_load: %s is not a 256-128-128-1 threshold model", path);
    }
    *out = m;
    return SW_OK;
}

extern "C" sw_status sw_model_free(sw_model* m) {
    delete m;
    return SW_OK;
}

namespace swmi {

size_t predict_workspace_size(int64_t max_M, int64_t max_N, int32_t n) {
    const size_t fws = feat_ws(max_M, max_N);
    const size_t feat = align_up((size_t)n * kFeat * 4, 256), xb = align_up((size_t)n * kFeat * 2, 256);
    const size_t act = align_up((size_t)n * kHid * 4, 256), ys = align_up((size_t)n * 4, 256);
    const size_t prm = align_up((size_t)kNParams * 4, 256), wbf = align_up((size_t)kNParams * 2, 256);
    return fws + feat + xb + 2 * act + ys + prm + wbf + 2 * 1024;
}

// Threshold of every pair from the model: features -> standardise -> MLP -> T.
sw_status predict_thresholds(sw_context* ctx, const sw_model* m, const uint8_t* d_a, const int64_t* offs_a,
                             const uint8_t* d_b, const int64_t* offs_b, int32_t n, void* ws, size_t ws_bytes,
                             std::vector<int32_t>& T) {
    T.assign((size_t)n, 0);
    if (!n) return SW_OK;
    int64_t mM = 0, mN = 0;
    for (int32_t k = 0; k < n; ++k) {
        mM = std::max(mM, offs_a[k + 1] - offs_a[k]);
        mN = std::max(mN, offs_b[k + 1] - offs_b[k]);
    }
    if (ws_bytes < predict_workspace_size(mM, mN, n))
        return fail(SW_ENOMEM, "threshold prediction: workspace of %zu bytes, need %zu", ws_bytes,
                    predict_workspace_size(mM, mN, n));
    const size_t fws = feat_ws(mM, mN);
    const size_t feat = align_up((size_t)n * kFeat * 4, 256), xb = align_up((size_t)n * kFeat * 2, 256);
    const size_t act = align_up((size_t)n * kHid * 4, 256), ys = align_up((size_t)n * 4, 256);
    const size_t prm = align_up((size_t)kNParams * 4, 256), wbf = align_up((size_t)kNParams * 2, 256);
    uint8_t* p = (uint8_t*)ws;
    uint8_t* fw = p;
    float* d_feat = (float*)(p + fws);
    uint16_t* d_x = (uint16_t*)((uint8_t*)d_feat + feat);
    float* d_h1 = (float*)((uint8_t*)d_x + xb);
    float* d_h2 = (float*)((uint8_t*)d_h1 + act);
    float* d_y = (float*)((uint8_t*)d_h2 + act);
    float* d_p = (float*)((uint8_t*)d_y + ys);
    uint16_t* d_w = (uint16_t*)((uint8_t*)d_p + prm);
    float* d_mean = (float*)((uint8_t*)d_w + wbf);
    float* d_inv = d_mean + kFeat;
    std::vector<uint16_t> hw((size_t)kNParams);
    for (int64_t q = 0; q < kNParams; ++q) hw[(size_t)q] = f32_to_bf16(m->params[(size_t)q]);
    hipStream_t s = ctx->stream;
    HIP_TRY(hipMemcpyAsync(d_p, m->params.data(), (size_t)kNParams * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_w, hw.data(), (size_t)kNParams * 2, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_mean, m->mean.data(), kFeat * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_inv, m->inv_std.data(), kFeat * 4, hipMemcpyHostToDevice, s));
    sw_status st;
    if ((st = sw_features_dev(ctx, d_a, offs_a, d_b, offs_b, n, d_feat, fw, fws)) != SW_OK) return st;
    if ((st = sw_mlp_standardize_dev(ctx, d_feat, n, d_mean, d_inv, d_x)) != SW_OK) return st;
    if ((st = sw_mlp_forward_dev(ctx, d_x, n, d_w, d_p, d_h1, d_h2, d_y)) != SW_OK) return st;
    std::vector<float> y((size_t)n);
    HIP_TRY(hipMemcpyAsync(y.data(), d_y, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int32_t k = 0; k < n; ++k) {
        const double sh = std::exp((double)y[(size_t)k]) - 1.0;
        const double t = std::floor(0.9 * sh);
        // A threshold below t_min = 0.01 * |A||B| / (|A| + |B|) can only skip the
        // strips of that width along the last rows and columns, under 2 % of the
        // cells: not worth the risk of a rerun, so none is set.
        const double la = (double)(offs_a[k + 1] - offs_a[k]), lb = (double)(offs_b[k + 1] - offs_b[k]);
        const double tmin = la + lb > 0 ? 0.01 * la * lb / (la + lb) : 0.0;
        T[(size_t)k] = (t < 1.0 || t < tmin) ? 0 : (t > 1.0e9 ? 1000000000 : (int32_t)t);
    }
    return SW_OK;
}

}  // namespace swmi
