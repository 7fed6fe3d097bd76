// row_generic.hip -- reference-shaped row update for any K <= 128 and every
// precision: one workgroup of 256 threads per work item, Gram accumulated
// from LDS tiles of gathered neighbour rows, Cholesky and both triangular
// solves in LDS.  It is the FP64 path and the fallback for shapes the
// matrix-core kernels do not cover.
//
// Per row (Algorithm 1, the body of the movie and user loops; the
// conditional is BPMF's):  P = Lambda + alpha sum_j y_j y_j^T,
// b = Lambda mu + alpha sum_j r'_j y_j, P = L L^T, y = L^-1 b,
// x = L^-T (y + z), z = Philox normals of counter (row, t, stream<<24|blk, 0).
#include "internal.h"
#include "rng_device.h"

namespace bpmf {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxK = 128;
constexpr int kMaxE = (kMaxK * (kMaxK + 1) / 2 + kThreads - 1) / kThreads;  // 33

__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }

// Inverse of e = i(i+1)/2 + j, 0 <= j <= i.
__device__ __forceinline__ void tri_index(int e, int &i, int &j)
{
    int ii = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
    while (ii * (ii + 1) / 2 > e) --ii;
    i = ii;
    j = e - ii * (ii + 1) / 2;
}

__device__ __forceinline__ float load_y(const float *p) { return *p; }
__device__ __forceinline__ double load_y(const double *p) { return *p; }
__device__ __forceinline__ float load_y(const uint16_t *p) { return __uint_as_float((uint32_t)(*p) << 16); }

__host__ __device__ constexpr int tile_for(int K) { return K <= 64 ? 64 : 32; }

template <typename T>
struct Smem {
    T *P;          // packed lower K(K+1)/2
    T *b;          // K
    T *Y;          // tile * K
    T *r;          // tile
    int32_t *idx;  // tile
};

template <typename T>
__device__ __forceinline__ Smem<T> carve(char *base, int K)
{
    Smem<T> s;
    int tile = tile_for(K);
    int KK2 = K * (K + 1) / 2;
    s.P = (T *)base;
    s.b = s.P + KK2;
    s.Y = s.b + K;
    s.r = s.Y + tile * K;
    s.idx = (int32_t *)(s.r + tile);
    return s;
}

// Cholesky of the packed lower P (in place), forward solve of b, add the
// row's normals, back solve; the result is left in s.b.  A non-positive
// pivot clears *status and propagates NaN into the row.
template <typename T>
__device__ void factor_and_sample(int K, Smem<T> s, uint64_t seed, uint32_t stream, uint32_t t,
                                  uint32_t row, int *__restrict__ status)
{
    const int tid = threadIdx.x;
    for (int k = 0; k < K; ++k) {
        if (tid == 0) {
            T d = s.P[pk(k, k)];
            if (!(d > T(0))) *status = 0;
            s.P[pk(k, k)] = d > T(0) ? sqrt(d) : T(NAN);
        }
        __syncthreads();
        T dk = s.P[pk(k, k)];
        for (int i = k + 1 + tid; i < K; i += kThreads) s.P[pk(i, k)] /= dk;
        __syncthreads();
        int m = K - k - 1;
        int n = m * (m + 1) / 2;
        for (int q = tid; q < n; q += kThreads) {
            int ii, jj;
            tri_index(q, ii, jj);
            int i = k + 1 + ii, j = k + 1 + jj;
            s.P[pk(i, j)] -= s.P[pk(i, k)] * s.P[pk(j, k)];
        }
        __syncthreads();
    }
    // y = L^-1 b
    for (int k = 0; k < K; ++k) {
        if (tid == 0) s.b[k] /= s.P[pk(k, k)];
        __syncthreads();
        T yk = s.b[k];
        for (int i = k + 1 + tid; i < K; i += kThreads) s.b[i] -= s.P[pk(i, k)] * yk;
        __syncthreads();
    }
    // y += z
    for (int blk = tid; 4 * blk < K; blk += kThreads) {
        double z[4];
        normals_block(seed, row, t, stream, (uint32_t)blk, 0u, z);
        for (int l = 0; l < 4 && 4 * blk + l < K; ++l) s.b[4 * blk + l] += (T)z[l];
    }
    __syncthreads();
    // x = L^-T y
    for (int k = K - 1; k >= 0; --k) {
        if (tid == 0) s.b[k] /= s.P[pk(k, k)];
        __syncthreads();
        T xk = s.b[k];
        for (int i = tid; i < k; i += kThreads) s.b[i] -= s.P[pk(k, i)] * xk;
        __syncthreads();
    }
}

template <typename T, typename YT>
__global__ __launch_bounds__(kThreads) void row_update_generic(
    int K, T alpha, const RowItem *__restrict__ items, const int32_t *__restrict__ nbr,
    const T *__restrict__ rc, const YT *__restrict__ Y, int ldy, const T *__restrict__ Lam,
    const T *__restrict__ Lmu, T *__restrict__ X, int ldx, T *__restrict__ part, uint64_t seed,
    uint32_t stream, const uint32_t *__restrict__ ctr, int *__restrict__ status)
{
    extern __shared__ __align__(16) char smem_raw[];
    Smem<T> s = carve<T>(smem_raw, K);
    const int tid = threadIdx.x;
    const int tile = tile_for(K);
    const int KK2 = K * (K + 1) / 2;
    const RowItem it = items[blockIdx.x];

    int ij[kMaxE];
    T acc[kMaxE];
#pragma unroll
    for (int m = 0; m < kMaxE; ++m) {
        int e = tid + m * kThreads, i = 0, j = 0;
        if (e < KK2) tri_index(e, i, j);
        ij[m] = (i << 16) | j;
        acc[m] = T(0);
    }
    T bacc = T(0);

    for (int64_t base = it.beg; base < it.end; base += tile) {
        int cnt = (int)min<int64_t>(tile, it.end - base);
        if (tid < tile) {
            s.idx[tid] = tid < cnt ? nbr[base + tid] : 0;
            s.r[tid] = tid < cnt ? rc[base + tid] : T(0);
        }
        __syncthreads();
        for (int q = tid; q < tile * K; q += kThreads) {
            int tt = q / K, k = q - tt * K;
            s.Y[q] = tt < cnt ? (T)load_y(Y + (size_t)s.idx[tt] * ldy + k) : T(0);
        }
        __syncthreads();
        for (int tt = 0; tt < cnt; ++tt) {
            const T *y = s.Y + tt * K;
#pragma unroll
            for (int m = 0; m < kMaxE; ++m) {
                if (tid + m * kThreads < KK2) {
                    int i = ij[m] >> 16, j = ij[m] & 0xffff;
                    acc[m] += y[i] * y[j];
                }
            }
            if (tid < K) bacc += s.r[tt] * y[tid];
        }
        __syncthreads();
    }

    if (it.slot >= 0) {  // partial of a split row
        T *dst = part + (size_t)it.slot * (KK2 + K);
#pragma unroll
        for (int m = 0; m < kMaxE; ++m)
            if (tid + m * kThreads < KK2) dst[tid + m * kThreads] = acc[m];
        if (tid < K) dst[KK2 + tid] = bacc;
        return;
    }
#pragma unroll
    for (int m = 0; m < kMaxE; ++m) {
        int e = tid + m * kThreads;
        if (e < KK2) {
            int i = ij[m] >> 16, j = ij[m] & 0xffff;
            s.P[e] = Lam[i * K + j] + alpha * acc[m];
        }
    }
    if (tid < K) s.b[tid] = Lmu[tid] + alpha * bacc;
    __syncthreads();
    factor_and_sample<T>(K, s, seed, stream, ctr[0], (uint32_t)it.row, status);
    if (tid < K) X[(size_t)it.row * ldx + tid] = s.b[tid];
}

// Finish split rows: sum their partial slots in slot order, add the prior,
// factor and sample.
template <typename T>
__global__ __launch_bounds__(kThreads) void row_finish_generic(
    int K, T alpha, const FinishItem *__restrict__ fin, const T *__restrict__ part,
    const T *__restrict__ Lam, const T *__restrict__ Lmu, T *__restrict__ X, int ldx,
    uint64_t seed, uint32_t stream, const uint32_t *__restrict__ ctr, int *__restrict__ status)
{
    extern __shared__ __align__(16) char smem_raw[];
    Smem<T> s = carve<T>(smem_raw, K);
    const int tid = threadIdx.x;
    const int KK2 = K * (K + 1) / 2;
    const FinishItem f = fin[blockIdx.x];
    for (int e = tid; e < KK2 + K; e += kThreads) {
        T sum = T(0);
        for (int q = 0; q < f.count; ++q) sum += part[(size_t)(f.first + q) * (KK2 + K) + e];
        if (e < KK2) {
            int i, j;
            tri_index(e, i, j);
            s.P[e] = Lam[i * K + j] + alpha * sum;
        } else {
            s.b[e - KK2] = Lmu[e - KK2] + alpha * sum;
        }
    }
    __syncthreads();
    factor_and_sample<T>(K, s, seed, stream, ctr[0], (uint32_t)f.row, status);
    if (tid < K) X[(size_t)f.row * ldx + tid] = s.b[tid];
}

template <typename T>
size_t lds_bytes(int K)
{
    int tile = tile_for(K);
    return sizeof(T) * ((size_t)K * (K + 1) / 2 + K + (size_t)tile * K + tile) + 4 * tile + 16;
}

}  // namespace

size_t row_generic_lds_bytes(int K, int prec)
{
    return prec == 0 ? lds_bytes<double>(K) : lds_bytes<float>(K);
}

// One workgroup per work item; every item (segments and whole rows) in the
// segments stage, the split rows in the finishing stage.
hipError_t launch_row_generic(bpmf_ctx *c, int side_id, hipStream_t s, int stage)
{
    Side &sd = c->side[side_id];
    Side &ot = c->side[1 - side_id];
    const int K = c->K;
    // this kernel draws every work item: a side must not also have rows on
    // the rank-one path (lowrank_available excludes every case that lands here)
    if (sd.n_low != 0) return hipErrorInvalidValue;
    if (c->prec == 0) {
        size_t lds = lds_bytes<double>(K);
        if (stage == kStageSegments && sd.n_items > 0)
            hipLaunchKernelGGL((row_update_generic<double, double>), dim3((unsigned)sd.n_items),
                               dim3(kThreads), lds, s, K, c->alpha, sd.items, sd.nbr,
                               (const double *)sd.rc, (const double *)ot.X, c->ld,
                               (const double *)sd.Lam_w, (const double *)sd.Lmu_w,
                               (double *)sd.X, c->ld, (double *)c->part, c->seed, sd.stream_row,
                               c->ctr, c->hyp_status + 1);
        if (stage == kStageFinish && sd.n_fin > 0)
            hipLaunchKernelGGL((row_finish_generic<double>), dim3((unsigned)sd.n_fin),
                               dim3(kThreads), lds, s, K, c->alpha, sd.fin,
                               (const double *)c->part, (const double *)sd.Lam_w,
                               (const double *)sd.Lmu_w, (double *)sd.X, c->ld, c->seed,
                               sd.stream_row, c->ctr, c->hyp_status + 1);
    } else {
        size_t lds = lds_bytes<float>(K);
        if (stage == kStageSegments && sd.n_items > 0) {
            if (c->prec == 2)
                hipLaunchKernelGGL((row_update_generic<float, uint16_t>),
                                   dim3((unsigned)sd.n_items), dim3(kThreads), lds, s, K,
                                   (float)c->alpha, sd.items, sd.nbr, (const float *)sd.rc,
                                   (const uint16_t *)ot.Xbf, c->ld, (const float *)sd.Lam_w,
                                   (const float *)sd.Lmu_w, (float *)sd.X, c->ld,
                                   (float *)c->part, c->seed, sd.stream_row, c->ctr,
                                   c->hyp_status + 1);
            else
                hipLaunchKernelGGL((row_update_generic<float, float>), dim3((unsigned)sd.n_items),
                                   dim3(kThreads), lds, s, K, (float)c->alpha, sd.items, sd.nbr,
                                   (const float *)sd.rc, (const float *)ot.X, c->ld,
                                   (const float *)sd.Lam_w, (const float *)sd.Lmu_w,
                                   (float *)sd.X, c->ld, (float *)c->part, c->seed,
                                   sd.stream_row, c->ctr, c->hyp_status + 1);
        }
        if (stage == kStageFinish && sd.n_fin > 0)
            hipLaunchKernelGGL((row_finish_generic<float>), dim3((unsigned)sd.n_fin),
                               dim3(kThreads), lds, s, K, (float)c->alpha, sd.fin,
                               (const float *)c->part, (const float *)sd.Lam_w,
                               (const float *)sd.Lmu_w, (float *)sd.X, c->ld, c->seed,
                               sd.stream_row, c->ctr, c->hyp_status + 1);
    }
    return hipGetLastError();
}

}  // namespace bpmf
