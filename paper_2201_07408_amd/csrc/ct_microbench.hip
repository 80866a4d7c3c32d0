// Measured ceilings of the device: HBM streaming rates, FP32 vector issue
// rates and the rate of bilinear samples of the kind the projectors take
// (two plane coordinates, their integer and fraction parts, four taps, three
// linear interpolations and an accumulate), with the taps read from an LDS
// tile or gathered from an array that stays in L2.  These are the constants
// the kernels' rooflines are measured against; they are not an operation of
// the method.
#include "ct_common.h"

#include <algorithm>

namespace ct {
namespace {

constexpr int kMbThreads = 256;
constexpr int kTileRows = 64, kTileStride = 80;   // LDS tile: 64 rows of 80 floats (stride 16 mod 32 banks)
constexpr int kL2Side = 512;                      // L2 array: 512 x 512 floats (1 MiB)
constexpr int kSteps = 48;                        // samples per walk

__global__ __launch_bounds__(kMbThreads) void k_mb_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                        size_t n4) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ __launch_bounds__(kMbThreads) void k_mb_read(const float4 *__restrict__ src, size_t n4,
                                                        float *__restrict__ out) {
    float s = 0.0f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
        const float4 v = src[i];
        s += (v.x + v.y) + (v.z + v.w);
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// eight independent chains per work-item, 16 steps per iteration
__global__ __launch_bounds__(kMbThreads) void k_mb_fma(float *__restrict__ out, float a, float b, int iters) {
    float c[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = (float)(threadIdx.x + i) * 1e-3f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
#pragma unroll
            for (int i = 0; i < 8; ++i) c[i] = fmaf(c[i], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += c[i];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(kMbThreads) void k_mb_add(float *__restrict__ out, float a, int iters) {
    float c[8];
    const float av = (float)threadIdx.x * 1e-7f + a;
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = (float)(threadIdx.x + i) * 1e-3f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
#pragma unroll
            for (int i = 0; i < 8; ++i) c[i] = c[i] + av;
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += c[i];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Start and slope of a work-item's walk: the 64 lanes of a wavefront start
// on a 16 x 4 grid of cells half a cell apart (like neighbouring rays), with
// slopes in [0.5, 1); starts lie in [2, 10), so 48 steps stay below 58 and
// every tap (integer part + 1) below 59 in both coordinates.
__device__ __forceinline__ void walk_start(int tid, float &b0, float &c0, float &gb, float &gc) {
    const int lane = tid & 63, wave = tid >> 6;
    b0 = 2.0f + 0.5f * (float)(lane & 15);
    c0 = 2.0f + 0.5f * (float)(lane >> 4) + 0.25f * (float)(wave & 3);
    gb = 0.5f + 0.03125f * (float)((tid * 7) & 15);
    gc = 0.5f + 0.03125f * (float)((tid * 11) & 15);
}

// One bilinear sample at (fb, fc) from rows of `stride` floats at t0.
template <typename P>
__device__ __forceinline__ float bilinear(P t0, int stride, float fb, float fc) {
    const int ib = (int)fb, ic = (int)fc;
    const float wb = __builtin_amdgcn_fractf(fb), wc = __builtin_amdgcn_fractf(fc);
    const P t = t0 + (ic * stride + ib);
    const float a = fmaf(wb, t[1] - t[0], t[0]);
    const float b = fmaf(wb, t[stride + 1] - t[stride], t[stride]);
    return fmaf(wc, b - a, a);
}

__global__ __launch_bounds__(kMbThreads) void k_mb_lds_bilinear(float *__restrict__ out, int reps) {
    __shared__ float tile[kTileRows * kTileStride];
    for (int i = threadIdx.x; i < kTileRows * kTileStride; i += blockDim.x)
        tile[i] = (float)((i * 2654435761u) >> 20) * 1e-3f;
    __syncthreads();
    float b0, c0, gb, gc;
    walk_start(threadIdx.x, b0, c0, gb, gc);
    float acc = 0.0f;
    for (int r = 0; r < reps; ++r) {
        // the start moves with the running sum (within [0, 0.25) of a cell)
        // so that the walk cannot be hoisted out of the repetitions
        const float sb = b0 + 0.25f * __builtin_amdgcn_fractf(acc);
#pragma unroll 8
        for (int j = 0; j < kSteps; ++j)
            acc += bilinear((const float *)tile, kTileStride, fmaf((float)j, gb, sb), fmaf((float)j, gc, c0));
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// The same walks over a window of an L2-resident array; the window's
// origin (below 448 in both coordinates) differs from workgroup to
// workgroup, and the walk stays within 60 cells of it.
__global__ __launch_bounds__(kMbThreads) void k_mb_l2_bilinear(const float *__restrict__ arr, float *__restrict__ out,
                                                               int reps) {
    const int ox = (int)((blockIdx.x * 37u) % 448u), oy = (int)((blockIdx.x * 53u) % 448u);
    const float *t0 = arr + (size_t)oy * kL2Side + ox;
    float b0, c0, gb, gc;
    walk_start(threadIdx.x, b0, c0, gb, gc);
    float acc = 0.0f;
    for (int r = 0; r < reps; ++r) {
        const float sb = b0 + 0.25f * __builtin_amdgcn_fractf(acc);
#pragma unroll 8
        for (int j = 0; j < kSteps; ++j) acc += bilinear(t0, kL2Side, fmaf((float)j, gb, sb), fmaf((float)j, gc, c0));
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// Tap reads alone (the gather bandwidth of the bilinear access pattern):
// per sample the address steps by one row and/or one column (integer add)
// and the four taps are read and summed; the walk starts at row 8 and
// column 10 at most (the column shifted by 0 or 1 per repetition) and takes
// 47 steps of at most one row and one column, so no tap lies beyond row 56
// or column 58.
__device__ __forceinline__ void tap_walk(int tid, int stride, int &start, int &step) {
    const int lane = tid & 63;
    start = (2 + (lane >> 4) + (tid >> 6)) * stride + 2 + (lane & 15) / 2;
    step = ((tid * 7) & 1 ? stride : 0) + (((tid * 11) & 3) != 0 ? 1 : 0);
}

__global__ __launch_bounds__(kMbThreads) void k_mb_lds_gather(float *__restrict__ out, int reps) {
    __shared__ float tile[kTileRows * kTileStride];
    for (int i = threadIdx.x; i < kTileRows * kTileStride; i += blockDim.x)
        tile[i] = (float)((i * 2654435761u) >> 20) * 1e-3f;
    __syncthreads();
    int start, step;
    tap_walk(threadIdx.x, kTileStride, start, step);
    float acc = 0.0f;
    for (int r = 0; r < reps; ++r) {
        // the start moves with the running sum (by 0 or 1 column) so that
        // the reads cannot be hoisted out of the repetitions
        int idx = start + ((int)acc & 1);
#pragma unroll 8
        for (int j = 0; j < kSteps - 1; ++j, idx += step)
            acc += (tile[idx] + tile[idx + 1]) + (tile[idx + kTileStride] + tile[idx + kTileStride + 1]);
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kMbThreads) void k_mb_l2_gather(const float *__restrict__ arr, float *__restrict__ out,
                                                             int reps) {
    const int ox = (int)((blockIdx.x * 37u) % 448u), oy = (int)((blockIdx.x * 53u) % 448u);
    const float *t0 = arr + (size_t)oy * kL2Side + ox;
    int start, step;
    tap_walk(threadIdx.x, kL2Side, start, step);
    float acc = 0.0f;
    for (int r = 0; r < reps; ++r) {
        int idx = start + ((int)acc & 1);
#pragma unroll 8
        for (int j = 0; j < kSteps - 1; ++j, idx += step)
            acc += (t0[idx] + t0[idx + 1]) + (t0[idx + kL2Side] + t0[idx + kL2Side + 1]);
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// LDS read bandwidth without bank conflicts: each lane reads 16 consecutive
// bytes, a wavefront 1 KiB of consecutive addresses, 14 reads per
// repetition at fixed offsets from a base of at most 127 float4s into a
// 1024-float4 tile (the last read ends below float4 959).
__global__ __launch_bounds__(kMbThreads) void k_mb_lds_peak(float *__restrict__ out, int reps) {
    __shared__ float4 tile4[1024];
    for (int i = threadIdx.x; i < 1024; i += blockDim.x) {
        const float v = (float)((i * 2654435761u) >> 20) * 1e-3f;
        tile4[i] = make_float4(v, v + 1.0f, v + 2.0f, v + 3.0f);
    }
    __syncthreads();
    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const int lane = (int)(threadIdx.x & 63);
    for (int r = 0; r < reps; ++r) {
        const int base = lane + 64 * ((int)acc.x & 1);
#pragma unroll
        for (int j = 0; j < 14; ++j) {
            const float4 v = tile4[base + 64 * j];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = (acc.x + acc.y) + (acc.z + acc.w);
}

__global__ void k_mb_fill(float *__restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = (float)((i * 2654435761u) >> 22) * 1e-3f;
}

// Best (shortest) of `reps` timed launches after one warm-up, in ms.
template <typename Launch>
int best_ms(Launch launch, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, double &ms) {
    launch();
    CT_LAUNCH_CHECK();
    ms = 1e300;
    for (int r = 0; r < reps; ++r) {
        CT_HIP_CHECK(hipEventRecord(e0, s));
        launch();
        CT_LAUNCH_CHECK();
        CT_HIP_CHECK(hipEventRecord(e1, s));
        CT_HIP_CHECK(hipEventSynchronize(e1));
        float t = 0.0f;
        CT_HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
        ms = std::min(ms, (double)t);
    }
    return CT_OK;
}

struct MbBuffers {
    float *big = nullptr, *res = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~MbBuffers() {
        if (big) (void)hipFree(big);
        if (res) (void)hipFree(res);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

int measure(ct_ceilings *out, hipStream_t s) {
    constexpr size_t kHalf = (size_t)1 << 27;           // floats per copy half (512 MiB)
    constexpr unsigned kBlocks = 4096;                   // compute and gather launches
    constexpr int kReps = 5;
    MbBuffers m;
    if (hipMalloc(&m.big, 2 * kHalf * sizeof(float)) != hipSuccess ||
        hipMalloc(&m.res, (size_t)kBlocks * kMbThreads * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("ct_measure_ceilings: cannot allocate 1 GiB of device memory");
        return CT_ERR_ALLOC;
    }
    CT_HIP_CHECK(hipEventCreate(&m.e0));
    CT_HIP_CHECK(hipEventCreate(&m.e1));
    hipLaunchKernelGGL(k_mb_fill, dim3(4096), dim3(kMbThreads), 0, s, m.big, 2 * kHalf);
    CT_LAUNCH_CHECK();
    const float4 *src = reinterpret_cast<const float4 *>(m.big);
    float4 *dst = reinterpret_cast<float4 *>(m.big + kHalf);
    const size_t n4 = kHalf / 4;
    // streaming grids: two rounds of resident workgroups on 256 CUs
    const unsigned sblk = 256 * 8 * 2;
    double ms = 0.0;
    CT_TRY(best_ms([&] { hipLaunchKernelGGL(k_mb_copy, dim3(sblk), dim3(kMbThreads), 0, s, src, dst, n4); }, s, m.e0,
                   m.e1, kReps, ms));
    out->hbm_copy_gbs = 2.0 * kHalf * sizeof(float) / (ms * 1e-3) / 1e9;
    CT_TRY(best_ms([&] { hipLaunchKernelGGL(k_mb_read, dim3(kBlocks), dim3(kMbThreads), 0, s, src, 2 * n4, m.res); },
                   s, m.e0, m.e1, kReps, ms));
    out->hbm_read_gbs = 2.0 * kHalf * sizeof(float) / (ms * 1e-3) / 1e9;
    const int iters = 256;
    const double chain_ops = (double)kBlocks * kMbThreads * iters * 16 * 8;
    CT_TRY(best_ms([&] { hipLaunchKernelGGL(k_mb_fma, dim3(kBlocks), dim3(kMbThreads), 0, s, m.res, 0.999f, 1e-3f,
                                            iters); },
                   s, m.e0, m.e1, kReps, ms));
    out->fp32_fma_tflops = 2.0 * chain_ops / (ms * 1e-3) / 1e12;
    CT_TRY(best_ms([&] { hipLaunchKernelGGL(k_mb_add, dim3(kBlocks), dim3(kMbThreads), 0, s, m.res, 1e-3f, iters); },
                   s, m.e0, m.e1, kReps, ms));
    out->fp32_add_tflops = chain_ops / (ms * 1e-3) / 1e12;
    const int reps_lds = 64, reps_l2 = 16;
    CT_TRY(best_ms([&] { hipLaunchKernelGGL(k_mb_lds_bilinear, dim3(kBlocks), dim3(kMbThreads), 0, s, m.res,
                                            reps_lds); },
                   s, m.e0, m.e1, kReps, ms));
    out->lds_bilinear_gsps = (double)kBlocks * kMbThreads * reps_lds * kSteps / (ms * 1e-3) / 1e9;
    // the L2 array is the first 1 MiB of the filled buffer
    CT_TRY(best_ms([&] { hipLaunchKernelGGL(k_mb_l2_bilinear, dim3(kBlocks), dim3(kMbThreads), 0, s, m.big, m.res,
                                            reps_l2); },
                   s, m.e0, m.e1, kReps, ms));
    out->l2_bilinear_gsps = (double)kBlocks * kMbThreads * reps_l2 * kSteps / (ms * 1e-3) / 1e9;
    // tap bytes: four floats per sample
    CT_TRY(best_ms([&] { hipLaunchKernelGGL(k_mb_lds_gather, dim3(kBlocks), dim3(kMbThreads), 0, s, m.res,
                                            reps_lds); },
                   s, m.e0, m.e1, kReps, ms));
    out->lds_gather_gbs = 16.0 * kBlocks * kMbThreads * reps_lds * (kSteps - 1) / (ms * 1e-3) / 1e9;
    CT_TRY(best_ms([&] { hipLaunchKernelGGL(k_mb_l2_gather, dim3(kBlocks), dim3(kMbThreads), 0, s, m.big, m.res,
                                            reps_l2); },
                   s, m.e0, m.e1, kReps, ms));
    out->l2_gather_gbs = 16.0 * kBlocks * kMbThreads * reps_l2 * (kSteps - 1) / (ms * 1e-3) / 1e9;
    const int reps_peak = 128;
    CT_TRY(best_ms([&] { hipLaunchKernelGGL(k_mb_lds_peak, dim3(kBlocks), dim3(kMbThreads), 0, s, m.res,
                                            reps_peak); },
                   s, m.e0, m.e1, kReps, ms));
    out->lds_peak_gbs = 16.0 * 14 * kBlocks * kMbThreads * reps_peak / (ms * 1e-3) / 1e9;
    return CT_OK;
}

}  // namespace
}  // namespace ct

extern "C" int ct_measure_ceilings(ct_ceilings *out, void *stream) {
    ct::clear_error();
    CT_ARG_CHECK(out, "ct_measure_ceilings: NULL output");
    ct_ceilings r{};
    const int st = ct::measure(&r, (hipStream_t)stream);
    if (st == CT_OK) *out = r;
    return st;
}
