// hyper.hip -- FP64 Normal-Wishart hyperparameter draw of one side on the GPU.
//
// Algorithm 1 samples the movie hyperparameters from V before the movie loop
// and the user hyperparameters from U before the user loop.  With the
// Normal-Wishart hyperprior of BPMF (mu0, beta0, W0, nu0) and the n rows x_i
// of the side's factor, the conjugate posterior is
//   beta* = beta0 + n,  nu* = nu0 + n,  mu* = (beta0 mu0 + n xbar) / beta*,
//   W*^-1 = W0^-1 + S + beta0 n / beta* (xbar - mu0)(xbar - mu0)^T,
//   S = sum_i (x_i - xbar)(x_i - xbar)^T,
// and the draw is Lambda ~ Wishart(W*, nu*) by the Bartlett decomposition
// (Lambda = (L_W A)(L_W A)^T, L_W = chol(W*), A lower triangular with
// A_kk = sqrt(chi2(nu* - k)), k = 0..K-1, and N(0,1) below the diagonal in
// row-major order), then mu = mu* + chol(beta* Lambda)^-T z.
//
// Three launches: per-block FP64 moment sums over row chunks, an
// entry-parallel fixed-order reduction of the block sums, and one workgroup
// for the K x K algebra.  S is formed as sum x x^T - n xbar xbar^T.
#include "internal.h"
#include "rng_device.h"

namespace bpmf {
namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerTile = 32;

__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }

__device__ __forceinline__ void tri_index(int e, int &i, int &j)
{
    int ii = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
    while (ii * (ii + 1) / 2 > e) --ii;
    i = ii;
    j = e - ii * (ii + 1) / 2;
}

__device__ __forceinline__ double as_f64(float v) { return (double)v; }
__device__ __forceinline__ double as_f64(double v) { return v; }

// Block b sums rows [b*chunk, min(rows, (b+1)*chunk)):  entries e < K are
// sum x_e, entries K + pk(i,j) are sum x_i x_j.
template <typename XT>
__global__ __launch_bounds__(kThreads) void hyper_moments(int K, const XT *__restrict__ X, int ld,
                                                          int64_t rows, int64_t chunk,
                                                          double *__restrict__ part)
{
    extern __shared__ __align__(16) char smem_raw[];
    double *tileX = (double *)smem_raw;  // kRowsPerTile * K
    const int tid = threadIdx.x;
    const int E = K + K * (K + 1) / 2;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = min<int64_t>(rows, r0 + chunk);
    constexpr int kMaxE = (128 + 128 * 129 / 2 + kThreads - 1) / kThreads;  // 33
    double acc[kMaxE];
    int ia[kMaxE], ja[kMaxE];
#pragma unroll
    for (int m = 0; m < kMaxE; ++m) {
        acc[m] = 0.0;
        int e = tid + m * kThreads, i = -1, j = -1;
        if (e < K) {
            i = e;
            j = -1;
        } else if (e < E) {
            tri_index(e - K, i, j);
        }
        ia[m] = i;
        ja[m] = j;
    }
    for (int64_t base = r0; base < r1; base += kRowsPerTile) {
        int cnt = (int)min<int64_t>(kRowsPerTile, r1 - base);
        for (int q = tid; q < cnt * K; q += kThreads) {
            int rr = q / K, k = q - rr * K;
            tileX[q] = as_f64(X[(size_t)(base + rr) * ld + k]);
        }
        __syncthreads();
        for (int rr = 0; rr < cnt; ++rr) {
            const double *x = tileX + rr * K;
#pragma unroll
            for (int m = 0; m < kMaxE; ++m) {
                if (ia[m] >= 0) acc[m] += ja[m] < 0 ? x[ia[m]] : x[ia[m]] * x[ja[m]];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < kMaxE; ++m) {
        int e = tid + m * kThreads;
        if (e < E) part[(size_t)blockIdx.x * E + e] = acc[m];
    }
}

// stats[e] = sum over blocks b (in order) of part[b][e].
__global__ void hyper_reduce(int E, int nblk, const double *__restrict__ part,
                             double *__restrict__ stats)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * E + e];
    stats[e] = s;
}

// In-place Cholesky of a packed lower K x K matrix in LDS by the whole
// workgroup.  Clears *ok on a non-positive pivot.
__device__ void chol_packed(int K, double *P, int *ok)
{
    const int tid = threadIdx.x;
    for (int k = 0; k < K; ++k) {
        if (tid == 0) {
            double d = P[pk(k, k)];
            if (!(d > 0.0)) {
                *ok = 0;
                d = 1.0;
            }
            P[pk(k, k)] = sqrt(d);
        }
        __syncthreads();
        double dk = P[pk(k, k)];
        for (int i = k + 1 + tid; i < K; i += kThreads) P[pk(i, k)] /= dk;
        __syncthreads();
        int m = K - k - 1;
        int n = m * (m + 1) / 2;
        for (int q = tid; q < n; q += kThreads) {
            int ii, jj;
            tri_index(q, ii, jj);
            int i = k + 1 + ii, j = k + 1 + jj;
            P[pk(i, j)] -= P[pk(i, k)] * P[pk(j, k)];
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void hyper_draw(
    int K, int64_t n, const double *__restrict__ stats, const double *__restrict__ mu0,
    const double *__restrict__ W0inv, double beta0, double nu0, uint64_t seed, uint32_t stream,
    const uint32_t *__restrict__ ctr, double *__restrict__ G0, double *__restrict__ G1,
    double *__restrict__ mu_out, double *__restrict__ Lam_out, T *__restrict__ Lam_w,
    T *__restrict__ Lmu_w, int *__restrict__ status)
{
    extern __shared__ __align__(16) char smem_raw[];
    const int KK2 = K * (K + 1) / 2;
    double *Mp = (double *)smem_raw;  // packed lower
    double *xbar = Mp + KK2;
    double *mus = xbar + K;
    double *zv = mus + K;
    double *mu = zv + K;
    __shared__ int ok;
    const int tid = threadIdx.x;
    const uint32_t t = ctr[0];
    const double dn = (double)n;
    const double beta_s = beta0 + dn;
    const double nu_s = nu0 + dn;
    const double shrink = beta0 * dn / beta_s;
    if (tid == 0) ok = 1;
    for (int k = tid; k < K; k += kThreads) {
        xbar[k] = stats[k] / dn;
        mus[k] = (beta0 * mu0[k] + dn * xbar[k]) / beta_s;
    }
    __syncthreads();
    // W*^-1 (packed lower)
    for (int e = tid; e < KK2; e += kThreads) {
        int i, j;
        tri_index(e, i, j);
        double S = stats[K + e] - dn * xbar[i] * xbar[j];
        Mp[e] = W0inv[i * K + j] + S + shrink * (xbar[i] - mu0[i]) * (xbar[j] - mu0[j]);
    }
    __syncthreads();
    chol_packed(K, Mp, &ok);
    // G0 = R^-1 (lower), one column per thread
    for (int j = tid; j < K; j += kThreads) {
        for (int i = 0; i < j; ++i) G0[i * K + j] = 0.0;
        G0[j * K + j] = 1.0 / Mp[pk(j, j)];
        for (int i = j + 1; i < K; ++i) {
            double s = 0.0;
            for (int k = j; k < i; ++k) s += Mp[pk(i, k)] * G0[k * K + j];
            G0[i * K + j] = -s / Mp[pk(i, i)];
        }
    }
    __syncthreads();
    // W* = R^-T R^-1 into Mp
    for (int e = tid; e < KK2; e += kThreads) {
        int a, b;
        tri_index(e, a, b);  // a >= b
        double s = 0.0;
        for (int k = a; k < K; ++k) s += G0[k * K + a] * G0[k * K + b];
        Mp[e] = s;
    }
    __syncthreads();
    chol_packed(K, Mp, &ok);  // Mp = L_W
    // Bartlett factor A into G1 (full, upper zero)
    for (int q = tid; q < K * K; q += kThreads) G1[q] = 0.0;
    __syncthreads();
    for (int k = tid; k < K; k += kThreads)
        G1[k * K + k] = sqrt(chi_square(seed, stream, t, (uint32_t)k, nu_s - (double)k, &ok));
    const int n_low = K * (K - 1) / 2;
    for (int blk = tid; 4 * blk < n_low; blk += kThreads) {
        double z[4];
        normals_block(seed, (uint32_t)blk, t, stream, 1u, 0u, z);
        for (int l = 0; l < 4 && 4 * blk + l < n_low; ++l) {
            int e = 4 * blk + l, r, c;
            tri_index(e, r, c);  // e = r(r+1)/2 + c with c <= r: shift to strict lower
            // strict-lower row-major index: e = r'(r'-1)/2 + c', r' = r + 1 when c <= r
            G1[(r + 1) * K + c] = z[l];
        }
    }
    __syncthreads();
    // B = L_W A into G0 (lower)
    for (int q = tid; q < K * K; q += kThreads) {
        int r = q / K, c = q - r * K;
        double s = 0.0;
        if (c <= r)
            for (int m = c; m <= r; ++m) s += Mp[pk(r, m)] * G1[m * K + c];
        G0[q] = s;
    }
    __syncthreads();
    // Lambda = B B^T; Mp <- beta* Lambda (packed)
    for (int e = tid; e < KK2; e += kThreads) {
        int r, c;
        tri_index(e, r, c);
        double s = 0.0;
        for (int m = 0; m <= c; ++m) s += G0[r * K + m] * G0[c * K + m];
        Lam_out[r * K + c] = s;
        Lam_out[c * K + r] = s;
    }
    __syncthreads();
    for (int e = tid; e < KK2; e += kThreads) {
        int r, c;
        tri_index(e, r, c);
        Mp[e] = beta_s * Lam_out[r * K + c];
    }
    __syncthreads();
    chol_packed(K, Mp, &ok);
    for (int blk = tid; 4 * blk < K; blk += kThreads) {
        double z[4];
        normals_block(seed, (uint32_t)blk, t, stream, 2u, 0u, z);
        for (int l = 0; l < 4 && 4 * blk + l < K; ++l) zv[4 * blk + l] = z[l];
    }
    __syncthreads();
    // x = L^-T z (column oriented), in zv
    for (int i = K - 1; i >= 0; --i) {
        if (tid == 0) zv[i] /= Mp[pk(i, i)];
        __syncthreads();
        double xi = zv[i];
        for (int j = tid; j < i; j += kThreads) zv[j] -= Mp[pk(i, j)] * xi;
        __syncthreads();
    }
    for (int k = tid; k < K; k += kThreads) {
        mu[k] = mus[k] + zv[k];
        mu_out[k] = mu[k];
    }
    __syncthreads();
    for (int i = tid; i < K; i += kThreads) {
        double s = 0.0;
        for (int j = 0; j < K; ++j) s += Lam_out[i * K + j] * mu[j];
        Lmu_w[i] = (T)s;
    }
    for (int q = tid; q < K * K; q += kThreads) Lam_w[q] = (T)Lam_out[q];
    if (tid == 0 && !ok) *status = 0;
}

// Working-precision prior from FP64 (mu, Lambda) set by the host.
template <typename T>
__global__ void prior_to_working(int K, const double *__restrict__ mu, const double *__restrict__ Lam,
                                 T *__restrict__ Lam_w, T *__restrict__ Lmu_w)
{
    int tid = threadIdx.x;
    for (int i = tid; i < K; i += blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < K; ++j) s += Lam[i * K + j] * mu[j];
        Lmu_w[i] = (T)s;
    }
    for (int q = tid; q < K * K; q += blockDim.x) Lam_w[q] = (T)Lam[q];
}

}  // namespace

hipError_t launch_hyper(bpmf_ctx *c, int side_id, hipStream_t s)
{
    Side &sd = c->side[side_id];
    const int K = c->K;
    const int E = K + K * (K + 1) / 2;
    int64_t rows = sd.rows;
    int nblk = c->hyp_blocks;
    int64_t chunk = (rows + nblk - 1) / nblk;
    if (chunk < 1) chunk = 1;
    int used = (int)((rows + chunk - 1) / chunk);
    if (used < 1) used = 1;
    size_t lds1 = sizeof(double) * kRowsPerTile * K;
    if (c->prec == 0)
        hipLaunchKernelGGL((hyper_moments<double>), dim3(used), dim3(kThreads), lds1, s, K,
                           (const double *)sd.X, c->ld, rows, chunk, c->hyp_part);
    else
        hipLaunchKernelGGL((hyper_moments<float>), dim3(used), dim3(kThreads), lds1, s, K,
                           (const float *)sd.X, c->ld, rows, chunk, c->hyp_part);
    hipLaunchKernelGGL(hyper_reduce, dim3((E + 255) / 256), dim3(256), 0, s, E, used, c->hyp_part,
                       c->hyp_stats);
    size_t lds2 = sizeof(double) * ((size_t)K * (K + 1) / 2 + 4 * (size_t)K);
    double *G0 = c->hyp_scratch, *G1 = G0 + (size_t)K * K;
    if (c->prec == 0)
        hipLaunchKernelGGL((hyper_draw<double>), dim3(1), dim3(kThreads), lds2, s, K, rows,
                           c->hyp_stats, c->d_mu0, c->d_W0inv, c->beta0, c->nu0, c->seed,
                           sd.stream_hyp, c->ctr, G0, G1, sd.mu, sd.Lam, (double *)sd.Lam_w,
                           (double *)sd.Lmu_w, c->hyp_status);
    else
        hipLaunchKernelGGL((hyper_draw<float>), dim3(1), dim3(kThreads), lds2, s, K, rows,
                           c->hyp_stats, c->d_mu0, c->d_W0inv, c->beta0, c->nu0, c->seed,
                           sd.stream_hyp, c->ctr, G0, G1, sd.mu, sd.Lam, (float *)sd.Lam_w,
                           (float *)sd.Lmu_w, c->hyp_status);
    return hipGetLastError();
}

hipError_t prepare_hyper(bpmf_ctx *c)
{
    const int K = c->K;
    size_t lds2 = sizeof(double) * ((size_t)K * (K + 1) / 2 + 4 * (size_t)K);
    if (lds2 <= 65536) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void *)hyper_draw<double>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)hyper_draw<float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
}

hipError_t launch_prior_to_working(bpmf_ctx *c, int side_id, hipStream_t s)
{
    Side &sd = c->side[side_id];
    if (c->prec == 0)
        hipLaunchKernelGGL((prior_to_working<double>), dim3(1), dim3(256), 0, s, c->K, sd.mu,
                           sd.Lam, (double *)sd.Lam_w, (double *)sd.Lmu_w);
    else
        hipLaunchKernelGGL((prior_to_working<float>), dim3(1), dim3(256), 0, s, c->K, sd.mu,
                           sd.Lam, (float *)sd.Lam_w, (float *)sd.Lmu_w);
    return hipGetLastError();
}

}  // namespace bpmf
