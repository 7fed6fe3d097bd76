// misc.hip -- initialisation, prediction/RMSE and small bookkeeping kernels.
//
// Prediction follows Algorithm 1's last loop ("predict rating and compute
// RMSE" over all test points): p = u_row . v_col + mean rating; the running
// mean of p over sweeps t > burn_in is kept in FP64; the two RMSEs (running
// mean, current sample) are reduced in a fixed order (per-block tree, then
// one block over the block sums), so they are bit-reproducible.
#include <mutex>

#include "../../include/bpmf.h"
#include "internal.h"
#include "rng_device.h"

namespace bpmf {
namespace {

constexpr int kGroup = 16;  // lanes per test pair

// Staging area of bpmf_predict_noalloc: row ids, column ids and predictions
// of at most kScratchPairs pairs (6 MiB).  Each GPU the library runs on holds
// its own copy until the process ends; host code reaches it only through
// the per-device address from hipGetSymbolAddress (scratch_dev below), never
// through the symbol itself.
constexpr int64_t kScratchPairs = 1 << 19;
static __device__ __align__(256) unsigned char scratch[kScratchPairs * 12];
constexpr int kMaxDevices = 64;
void *scratch_dev[kMaxDevices] = {};
std::mutex scratch_mu;

__device__ __forceinline__ double as_f64(float v) { return (double)v; }
__device__ __forceinline__ double as_f64(double v) { return v; }

// X_ik = scale * z(stream, t = 0, row i, k); padding columns are zeroed.
template <typename T>
__global__ void init_factor(int K, int ld, int64_t rows, double scale, uint64_t seed,
                            uint32_t stream, T *__restrict__ X)
{
    const int nb = (K + 3) / 4;
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= rows * nb) return;
    int64_t row = q / nb;
    int blk = (int)(q - row * nb);
    double z[4];
    normals_block(seed, (uint32_t)row, 0u, stream, (uint32_t)blk, 0u, z);
    for (int l = 0; l < 4; ++l) {
        int k = 4 * blk + l;
        if (k < ld) X[(size_t)row * ld + k] = k < K ? (T)(scale * z[l]) : T(0);
    }
}

template <typename T>
__device__ __forceinline__ double group_dot(int K, const T *u, const T *v, int g)
{
    T s = T(0);
    for (int k = g; k < K; k += kGroup) s += u[k] * v[k];
#pragma unroll
    for (int off = kGroup / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kGroup);
    return as_f64(s);
}

// One group of G lanes per test pair, grid-stride over pairs with a fixed
// grid, four pairs per group in flight (their ids, values and running sums
// are loaded before any row, so the dependent loads of the four overlap).
// Writes per-block sums of squared errors (running mean, sample).  FP32
// factors are read as float4 (rows are padded to a multiple of 4).
template <typename T, int G>
__global__ __launch_bounds__(256) void predict_test(
    int K, int ld, int64_t n, const int32_t *__restrict__ row, const int32_t *__restrict__ col,
    const float *__restrict__ val, const T *__restrict__ U, const T *__restrict__ V, double rbar,
    double *__restrict__ pred_sum, const uint32_t *__restrict__ ctr, int burn_in,
    double *__restrict__ part)
{
    constexpr int GPB = 256 / G;  // groups per block
    constexpr int P = 4;          // pairs per group in flight
    __shared__ double red[2][GPB];
    const uint32_t t = ctr[0];
    const uint32_t cnt = ctr[2];
    const bool use = (int64_t)t > (int64_t)burn_in;
    const int g = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int64_t groups_total = (int64_t)gridDim.x * GPB;
    double sa = 0.0, sl = 0.0;
    // a group takes P consecutive pairs: the pairs are in user order, so
    // they mostly share the user's row (cache hits after the first)
    for (int64_t e0 = ((int64_t)blockIdx.x * GPB + grp) * P; e0 < n; e0 += P * groups_total) {
        int64_t e[P];
        bool ok[P];
        int32_t ri[P], ci[P];
        float rv[P];
        double prev[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            e[q] = e0 + q;
            ok[q] = e[q] < n;
            ri[q] = ok[q] ? row[e[q]] : 0;
            ci[q] = ok[q] ? col[e[q]] : 0;
            rv[q] = ok[q] ? val[e[q]] : 0.f;
            prev[q] = ok[q] && (use || cnt) ? pred_sum[e[q]] : 0.0;
        }
        T s[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const T *u = U + (size_t)ri[q] * ld;
            const T *v = V + (size_t)ci[q] * ld;
            s[q] = T(0);
            if constexpr (sizeof(T) == 4) {
                for (int k = 4 * g; k < K; k += 4 * G) {
                    const float4 a = *reinterpret_cast<const float4 *>(u + k);
                    const float4 b = *reinterpret_cast<const float4 *>(v + k);
                    s[q] += a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;  // padding entries are 0
                }
            } else {
                for (int k = g; k < K; k += G) s[q] += u[k] * v[k];
            }
        }
#pragma unroll
        for (int q = 0; q < P; ++q) {
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) s[q] += __shfl_xor(s[q], off, G);
            if (!ok[q]) continue;
            const double p = (double)s[q] + rbar;
            double avg;
            if (use) {
                const double ps = prev[q] + p;
                avg = ps / (double)(cnt + 1);
                if (g == 0) pred_sum[e[q]] = ps;
            } else {
                avg = cnt ? prev[q] / (double)cnt : p;
            }
            const double r = (double)rv[q];
            sa += (avg - r) * (avg - r);
            sl += (p - r) * (p - r);
        }
    }
    if (g == 0) {
        red[0][grp] = sa;
        red[1][grp] = sl;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double s2 = 0.0;
        for (int q = 0; q < GPB; ++q) s2 += red[threadIdx.x][q];
        part[2 * blockIdx.x + threadIdx.x] = s2;
    }
}

// One block: sum the per-block partials (each thread a fixed strided subset,
// then a fixed tree), store the RMSEs of this sweep in hist[slot],
// slot = t - t0, and count the sweep into the running mean if t > burn_in.
__global__ __launch_bounds__(256) void predict_finalize(int nblk, int64_t n,
                                                        const double *__restrict__ part,
                                                        uint32_t *__restrict__ ctr, int burn_in,
                                                        double *__restrict__ hist, int64_t hist_cap)
{
    __shared__ double red[2][256];
    const int tid = threadIdx.x;
    double sa = 0.0, sl = 0.0;
#pragma unroll 8
    for (int b = tid; b < nblk; b += 256) {
        sa += part[2 * b];
        sl += part[2 * b + 1];
    }
    red[0][tid] = sa;
    red[1][tid] = sl;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            red[0][tid] += red[0][tid + w];
            red[1][tid] += red[1][tid + w];
        }
        __syncthreads();
    }
    if (tid != 0) return;
    const uint32_t t = ctr[0];
    int64_t slot = (int64_t)t - (int64_t)ctr[1];
    if (slot < 0 || slot >= hist_cap) slot = hist_cap - 1;
    const double dn = n > 0 ? (double)n : 1.0;
    hist[2 * slot] = sqrt(red[0][0] / dn);
    hist[2 * slot + 1] = sqrt(red[1][0] / dn);
    if ((int64_t)t > (int64_t)burn_in) ctr[2] += 1;
}

template <typename T>
__global__ void predict_pairs(int K, int ld, int64_t n, const int32_t *__restrict__ row,
                              const int32_t *__restrict__ col, const T *__restrict__ U,
                              const T *__restrict__ V, double rbar, float *__restrict__ out)
{
    const int g = threadIdx.x % kGroup;
    int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kGroup;
    if (e >= n) return;
    double p = group_dot<T>(K, U + (size_t)row[e] * ld, V + (size_t)col[e] * ld, g) + rbar;
    if (g == 0) out[e] = (float)p;
}

__global__ void set_counter(uint32_t *ctr, int idx, uint32_t v) { ctr[idx] = v; }
__global__ void advance_t(uint32_t *ctr) { ctr[0] += 1u; }

__global__ void fill_f64(double *p, int64_t n, double v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Round-to-nearest-even FP32 -> BF16.
__global__ void to_bf16(const float *__restrict__ x, uint16_t *__restrict__ y, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t u = __float_as_uint(x[i]);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    y[i] = (uint16_t)(u >> 16);
}

// r = hi + mid + lo, each part a BF16 value (round to nearest even at each
// step; exact: hi keeps the top 8 significant bits of r, mid the next 8 of
// the remainder and lo the rest, which fits), stored as three planes of
// n + 32 values, each ending in 32 zeros.
__device__ __forceinline__ uint16_t bf16_rne_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ void split_ratings(const float *__restrict__ rc, uint16_t *__restrict__ rc3, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t plane = n + 32;
    if (i >= plane) return;
    if (i >= n) {
        rc3[i] = rc3[plane + i] = rc3[2 * plane + i] = 0;
        return;
    }
    float r = rc[i];
    const uint16_t hi = bf16_rne_bits(r);
    r -= __uint_as_float((uint32_t)hi << 16);
    const uint16_t mid = bf16_rne_bits(r);
    r -= __uint_as_float((uint32_t)mid << 16);
    rc3[i] = hi;
    rc3[plane + i] = mid;
    rc3[2 * plane + i] = bf16_rne_bits(r);
}

}  // namespace

hipError_t launch_init_factor(bpmf_ctx *c, int side_id, hipStream_t s)
{
    Side &sd = c->side[side_id];
    const int nb = (c->K + 3) / 4;
    int64_t total = sd.rows * nb;
    double scale = pow((double)c->K, -0.25);
    unsigned grid = (unsigned)((total + 255) / 256);
    if (grid == 0) return hipSuccess;
    if (c->prec == 0)
        hipLaunchKernelGGL((init_factor<double>), dim3(grid), dim3(256), 0, s, c->K, c->ld,
                           sd.rows, scale, c->seed, sd.stream_init, (double *)sd.X);
    else
        hipLaunchKernelGGL((init_factor<float>), dim3(grid), dim3(256), 0, s, c->K, c->ld,
                           sd.rows, scale, c->seed, sd.stream_init, (float *)sd.X);
    return hipGetLastError();
}

hipError_t launch_predict_test(bpmf_ctx *c, hipStream_t s)
{
    int nblk = c->rmse_blocks;
    if (c->prec == 0)
        hipLaunchKernelGGL((predict_test<double, 16>), dim3(nblk), dim3(256), 0, s, c->K, c->ld,
                           c->n_test, c->test_row, c->test_col, c->test_val,
                           (const double *)c->side[0].X, (const double *)c->side[1].X, c->rbar,
                           c->pred_sum, c->ctr, c->burn_in, c->rmse_part);
    else if (c->ld <= 32)  // four lanes per pair: twice the pairs in flight per wavefront
        hipLaunchKernelGGL((predict_test<float, 4>), dim3(nblk), dim3(256), 0, s, c->K, c->ld,
                           c->n_test, c->test_row, c->test_col, c->test_val,
                           (const float *)c->side[0].X, (const float *)c->side[1].X, c->rbar,
                           c->pred_sum, c->ctr, c->burn_in, c->rmse_part);
    else  // eight lanes per pair, several float4 steps each
        hipLaunchKernelGGL((predict_test<float, 8>), dim3(nblk), dim3(256), 0, s, c->K, c->ld,
                           c->n_test, c->test_row, c->test_col, c->test_val,
                           (const float *)c->side[0].X, (const float *)c->side[1].X, c->rbar,
                           c->pred_sum, c->ctr, c->burn_in, c->rmse_part);
    hipLaunchKernelGGL(predict_finalize, dim3(1), dim3(256), 0, s, nblk, c->n_test, c->rmse_part,
                       c->ctr, c->burn_in, c->rmse_hist, c->hist_cap);
    return hipGetLastError();
}

hipError_t launch_predict_pairs(bpmf_ctx *c, int64_t n, const int32_t *row, const int32_t *col,
                                float *out, hipStream_t s)
{
    unsigned grid = (unsigned)((n * kGroup + 255) / 256);
    if (grid == 0) return hipSuccess;
    if (c->prec == 0)
        hipLaunchKernelGGL((predict_pairs<double>), dim3(grid), dim3(256), 0, s, c->K, c->ld, n,
                           row, col, (const double *)c->side[0].X, (const double *)c->side[1].X,
                           c->rbar, out);
    else
        hipLaunchKernelGGL((predict_pairs<float>), dim3(grid), dim3(256), 0, s, c->K, c->ld, n,
                           row, col, (const float *)c->side[0].X, (const float *)c->side[1].X,
                           c->rbar, out);
    return hipGetLastError();
}

// Caller ids to internal rows for a relabelled context, in place.  The ids
// were range-checked on the host, so every table read is in bounds.
__global__ void map_pairs(int64_t n, int32_t *__restrict__ row, int32_t *__restrict__ col,
                          const int32_t *__restrict__ urow, const int32_t *__restrict__ vrow)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    row[e] = urow[row[e]];
    col[e] = vrow[col[e]];
}

hipError_t launch_map_pairs(bpmf_ctx *c, int64_t n, int32_t *row, int32_t *col, hipStream_t s)
{
    if (!c->relabel || n == 0) return hipSuccess;
    hipLaunchKernelGGL(map_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, row, col,
                       (const int32_t *)c->d_int_of[0], (const int32_t *)c->d_int_of[1]);
    return hipGetLastError();
}

// The device address of this GPU's staging area, looked up once per device
// with that device current (called by bpmf_create).
hipError_t predict_scratch_init(bpmf_ctx *c)
{
    if (c->device < 0 || c->device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(scratch_mu);
    if (!scratch_dev[c->device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_dev[c->device] = p;
    }
    c->scratch = scratch_dev[c->device];
    return hipSuccess;
}

hipError_t launch_set_counter(uint32_t *ctr, int idx, uint32_t value, hipStream_t s)
{
    hipLaunchKernelGGL(set_counter, dim3(1), dim3(1), 0, s, ctr, idx, value);
    return hipGetLastError();
}

hipError_t launch_advance_t(uint32_t *ctr, hipStream_t s)
{
    hipLaunchKernelGGL(advance_t, dim3(1), dim3(1), 0, s, ctr);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_to_bf16(bpmf_ctx *c, int side_id, hipStream_t s)
{
    Side &sd = c->side[side_id];
    int64_t n = sd.rows * c->ld;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (const float *)sd.X, sd.Xbf, n);
    return hipGetLastError();
}

hipError_t launch_split_ratings(bpmf_ctx *c, int side_id, hipStream_t s)
{
    Side &sd = c->side[side_id];
    if (!sd.rc3) return hipSuccess;
    const int64_t n = c->nnz;
    hipLaunchKernelGGL(split_ratings, dim3((unsigned)((n + 32 + 255) / 256)), dim3(256), 0, s,
                       (const float *)sd.rc, sd.rc3, n);
    return hipGetLastError();
}

}  // namespace bpmf

extern "C" int bpmf_predict_noalloc(bpmf_ctx *c, int64_t n, const int32_t *row, const int32_t *col,
                                    float *out)
{
    using namespace bpmf;
    if (!c) return BPMF_E_INVAL;
    if (c->sticky) {
        c->err = "context unusable after a device error: " + c->err;
        return BPMF_E_DEVICE;
    }
    if (n < 0 || (n > 0 && (!row || !col || !out))) {
        c->err = "bpmf_predict_noalloc: bad pair arrays";
        return BPMF_E_INVAL;
    }
    if (n > kScratchPairs) {
        c->err = "bpmf_predict_noalloc: at most " + std::to_string(kScratchPairs) +
                 " pairs per call (its staging area is a fixed device array)";
        return BPMF_E_TOOBIG;
    }
    if (!c->scratch) {
        c->err = "bpmf_predict_noalloc: no staging area on this device";
        return BPMF_E_INVAL;
    }
    for (int64_t e = 0; e < n; ++e)
        if (row[e] < 0 || row[e] >= c->M || col[e] < 0 || col[e] >= c->N) {
            c->err = "bpmf_predict_noalloc: pair " + std::to_string(e) + " out of range";
            return BPMF_E_RANGE;
        }
    if (n == 0) return BPMF_OK;
    int32_t *d_row = (int32_t *)c->scratch;
    int32_t *d_col = d_row + kScratchPairs;
    float *d_out = (float *)(d_col + kScratchPairs);
    hipError_t e = hipMemcpyAsync(d_row, row, sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_col, col, sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_map_pairs(c, n, d_row, d_col, c->stream);
    if (e == hipSuccess) e = launch_predict_pairs(c, n, d_row, d_col, d_out, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->err = std::string("bpmf_predict_noalloc: ") + hipGetErrorString(e);
        c->sticky = true;
        return BPMF_E_DEVICE;
    }
    return BPMF_OK;
}
