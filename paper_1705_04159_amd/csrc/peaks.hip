// peaks.hip -- micro-benchmarks for the measured peaks of the current device:
// HBM (stream triad), FP32 vector FMA, FP32 / BF16 / FP64 matrix cores, and
// random K-wide row gathers from sources that fit in one XCD's L2, in the
// Infinity Cache or only in HBM.  The row update's roofline (Sec. II: a few
// K x K operations per row, fed by gathered rows of the other factor) is
// stated against these as well as against the spec sheet.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bpmf.h"
#include "../../include/bpmf_peaks.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kBlocks = 2048;  // 8 wavefronts per SIMD on 256 CUs
constexpr int kAcc = 8;        // independent accumulators per wavefront (matrix cores)

__global__ __launch_bounds__(kThreads) void triad(int64_t n4, const float4 *__restrict__ b,
                                                  const float4 *__restrict__ c, float4 *__restrict__ a,
                                                  float s)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n4) return;
    const float4 x = b[i], y = c[i];
    a[i] = make_float4(x.x + s * y.x, x.y + s * y.y, x.z + s * y.z, x.w + s * y.w);
}

// Eight independent FMA chains per lane, sixteen steps per iteration.
__global__ __launch_bounds__(kThreads) void valu_fma(int iters, float *__restrict__ out)
{
    float a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = 1.0f + 1e-6f * (float)(threadIdx.x + k);
    const float m = 0.9999999f, d = 1e-7f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] = fmaf(a[k], m, d);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += a[k];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

// kAcc independent accumulators per wavefront on each matrix-core kind.
__global__ __launch_bounds__(kThreads) void mfma_f32(int iters, float *__restrict__ out)
{
    floatx4 acc[kAcc] = {};
    const float a = 1e-3f * (float)(threadIdx.x & 63), b = 1e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < kAcc; ++r) acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[r], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int r = 0; r < kAcc; ++r) s += acc[r][0] + acc[r][1] + acc[r][2] + acc[r][3];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void mfma_bf16(int iters, float *__restrict__ out)
{
    floatx4 acc[kAcc] = {};
    // BF16 bit patterns of 1/128 (0x3c00) and of a lane-dependent small value
    u32x4 ua, ub;
    const uint32_t lo = 0x3c00u + (threadIdx.x & 63);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        ua[e] = lo | (lo << 16);
        ub[e] = 0x3c003c00u;
    }
    const bf16x8 a = __builtin_bit_cast(bf16x8, ua), b = __builtin_bit_cast(bf16x8, ub);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < kAcc; ++r) acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[r], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int r = 0; r < kAcc; ++r) s += acc[r][0] + acc[r][1] + acc[r][2] + acc[r][3];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void mfma_f64(int iters, float *__restrict__ out)
{
    doublex4 acc[kAcc] = {};
    const double a = 1e-3 * (double)(threadIdx.x & 63), b = 1e-3;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < kAcc; ++r) acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[r], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < kAcc; ++r) s += acc[r][0] + acc[r][1] + acc[r][2] + acc[r][3];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = (float)s;
}

// A 32-bit integer mixer (xor-shift / multiply rounds, the "lowbias32"
// constants published by C. Wellons): consecutive gather indices land on
// unrelated rows.
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Each wavefront reads `per_wave` whole rows per step (lanes_per_row lanes
// of 16 B each per row), four steps in flight.
__global__ __launch_bounds__(kThreads) void gather_rows(const float4 *__restrict__ src, uint32_t src_rows,
                                                        int lanes_per_row, int per_wave, int64_t n_rows,
                                                        float *__restrict__ out)
{
    constexpr int U = 4;
    const int lane = threadIdx.x & 63;
    const int sub = lane / lanes_per_row, part = lane - sub * lanes_per_row;
    const bool active = sub < per_wave;
    const int64_t wave = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
    const int64_t n_waves = (int64_t)gridDim.x * (kThreads / 64);
    const int64_t step = (int64_t)per_wave * U;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t base = wave * step; base < n_rows; base += n_waves * step) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t g = base + (int64_t)u * per_wave + sub;
            v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (active && g < n_rows) {
                const uint32_t r = __umulhi(mix32((uint32_t)g), src_rows);
                v[u] = src[(size_t)r * lanes_per_row + part];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc.x += v[u].x;
            acc.y += v[u].y;
            acc.z += v[u].z;
            acc.w += v[u].w;
        }
    }
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

// Device buffers and events of one measurement, released on every path.
struct Bench {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *buf[3] = {nullptr, nullptr, nullptr};
    ~Bench()
    {
        for (void *p : buf)
            if (p) (void)hipFree(p);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
    }
    int init()
    {
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return BPMF_E_DEVICE;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return BPMF_E_DEVICE;
        return BPMF_OK;
    }
    int alloc(int q, size_t bytes)
    {
        if (hipMalloc(&buf[q], bytes) != hipSuccess) {
            buf[q] = nullptr;
            (void)hipGetLastError();
            return BPMF_E_NOMEM;
        }
        return hipMemsetAsync(buf[q], 0, bytes, s) == hipSuccess ? BPMF_OK : BPMF_E_DEVICE;
    }
    // One warm-up launch, then `reps` timed ones; *best = shortest, in ms.
    template <typename F>
    int time(int reps, F launch, float *best)
    {
        launch(s);
        if (hipGetLastError() != hipSuccess) return BPMF_E_DEVICE;
        *best = 1e30f;
        for (int r = 0; r < reps; ++r) {
            if (hipEventRecord(e0, s) != hipSuccess) return BPMF_E_DEVICE;
            launch(s);
            if (hipGetLastError() != hipSuccess) return BPMF_E_DEVICE;
            if (hipEventRecord(e1, s) != hipSuccess) return BPMF_E_DEVICE;
            if (hipEventSynchronize(e1) != hipSuccess) return BPMF_E_DEVICE;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return BPMF_E_DEVICE;
            if (ms < *best) *best = ms;
        }
        return BPMF_OK;
    }
};

}  // namespace

extern "C" int bpmf_peak_triad(int64_t bytes_per_array, int32_t reps, double *gbs)
{
    if (!gbs || reps < 1 || bytes_per_array < (1 << 20) || bytes_per_array % 16) return BPMF_E_INVAL;
    Bench b;
    int rc;
    if ((rc = b.init()) != BPMF_OK) return rc;
    for (int q = 0; q < 3; ++q)
        if ((rc = b.alloc(q, (size_t)bytes_per_array)) != BPMF_OK) return rc;
    const int64_t n4 = bytes_per_array / 16;
    const unsigned grid = (unsigned)((n4 + kThreads - 1) / kThreads);
    float ms = 0.f;
    rc = b.time(reps, [&](hipStream_t s) {
        triad<<<grid, kThreads, 0, s>>>(n4, (const float4 *)b.buf[1], (const float4 *)b.buf[2],
                                        (float4 *)b.buf[0], 0.5f);
    }, &ms);
    if (rc != BPMF_OK) return rc;
    *gbs = 3.0 * (double)bytes_per_array / (ms * 1e-3) / 1e9;
    return BPMF_OK;
}

extern "C" int bpmf_peak_compute(int32_t kind, int32_t reps, double *tflops)
{
    if (!tflops || reps < 1 || kind < BPMF_PEAK_FP32_VALU || kind > BPMF_PEAK_FP64_MFMA) return BPMF_E_INVAL;
    Bench b;
    int rc;
    if ((rc = b.init()) != BPMF_OK) return rc;
    if ((rc = b.alloc(0, sizeof(float) * kBlocks * kThreads)) != BPMF_OK) return rc;
    float *out = (float *)b.buf[0];
    const double waves = (double)kBlocks * kThreads / 64;
    int iters = 0;
    double flop = 0.0;  // per launch
    float ms = 0.f;
    switch (kind) {
    case BPMF_PEAK_FP32_VALU:
        iters = 2048;
        flop = 2.0 * 16 * 8 * iters * (double)kBlocks * kThreads;
        rc = b.time(reps, [&](hipStream_t s) { valu_fma<<<kBlocks, kThreads, 0, s>>>(iters, out); }, &ms);
        break;
    case BPMF_PEAK_FP32_MFMA:
        iters = 4096;
        flop = (double)kAcc * 2 * 16 * 16 * 4 * iters * waves;
        rc = b.time(reps, [&](hipStream_t s) { mfma_f32<<<kBlocks, kThreads, 0, s>>>(iters, out); }, &ms);
        break;
    case BPMF_PEAK_BF16_MFMA:
        iters = 8192;
        flop = (double)kAcc * 2 * 16 * 16 * 32 * iters * waves;
        rc = b.time(reps, [&](hipStream_t s) { mfma_bf16<<<kBlocks, kThreads, 0, s>>>(iters, out); }, &ms);
        break;
    default:
        iters = 2048;
        flop = (double)kAcc * 2 * 16 * 16 * 4 * iters * waves;
        rc = b.time(reps, [&](hipStream_t s) { mfma_f64<<<kBlocks, kThreads, 0, s>>>(iters, out); }, &ms);
        break;
    }
    if (rc != BPMF_OK) return rc;
    *tflops = flop / (ms * 1e-3) / 1e12;
    return BPMF_OK;
}

extern "C" int bpmf_peak_gather(int64_t src_bytes, int32_t row_bytes, int64_t n_rows, int32_t reps, double *gbs)
{
    if (!gbs || reps < 1 || row_bytes < 16 || row_bytes > 1024 || row_bytes % 16 || src_bytes < row_bytes ||
        n_rows < 1 || src_bytes / row_bytes > (int64_t)UINT32_MAX)
        return BPMF_E_INVAL;
    Bench b;
    int rc;
    if ((rc = b.init()) != BPMF_OK) return rc;
    const int64_t src_rows = src_bytes / row_bytes;
    if ((rc = b.alloc(0, (size_t)(src_rows * row_bytes))) != BPMF_OK) return rc;
    if ((rc = b.alloc(1, sizeof(float) * kBlocks * kThreads)) != BPMF_OK) return rc;
    const int lanes = row_bytes / 16;  // 1..64
    const int per_wave = 64 / lanes;
    float ms = 0.f;
    rc = b.time(reps, [&](hipStream_t s) {
        gather_rows<<<kBlocks, kThreads, 0, s>>>((const float4 *)b.buf[0], (uint32_t)src_rows, lanes, per_wave,
                                                 n_rows, (float *)b.buf[1]);
    }, &ms);
    if (rc != BPMF_OK) return rc;
    *gbs = (double)n_rows * row_bytes / (ms * 1e-3) / 1e9;
    return BPMF_OK;
}
