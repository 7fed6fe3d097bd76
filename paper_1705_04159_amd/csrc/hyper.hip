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
// Three launches: per-block FP64 moment sums over row chunks (S is formed as
// sum x x^T - n xbar xbar^T; on the FP64 matrix cores for K <= 112), a
// fixed-order reduction of the block sums (coalesced over entries), and one
// workgroup for the K x K algebra.  The
// algebra avoids forming W* and two of the three factorisations:
//   * L_W is obtained from one Cholesky of the index-reversed W*^-1:
//     J W*^-1 J = C C^T gives W*^-1 = (J C J)(J C J)^T with J C J upper
//     triangular, hence W* = (J C J)^-T (J C J)^-1 and, by uniqueness of the
//     Cholesky factor, L_W = J C^-T J, i.e. L_W[i][j] = (C^-1)[K-1-j][K-1-i];
//   * B = L_W A is lower triangular with a positive diagonal, so it is the
//     Cholesky factor of Lambda, and chol(beta* Lambda) = sqrt(beta*) B:
//     mu = mu* + B^-T z / sqrt(beta*).
// All K x K matrices are packed lower triangles in LDS when they fit.
#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "rng_device.h"

namespace bpmf {
namespace {

constexpr int kThreads = 256;      // moment sums (non-matrix-core path)
constexpr int kDrawThreads = 1024;  // the K x K algebra of the draw (one workgroup)

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

// Block b sums rows [b*chunk, min(rows, (b+1)*chunk)).  Entry e < K is
// sum x_e (taken as x_e * 1 with a constant 1 appended to each staged row),
// entry K + pk(i,j) is sum x_i x_j.  NE = entries per thread.
template <int NE, typename XT>
__global__ __launch_bounds__(kThreads) void hyper_moments(int K, const XT *__restrict__ X, int ld,
                                                          int64_t rows, int64_t chunk,
                                                          int tile_rows, double *__restrict__ part)
{
    extern __shared__ __align__(16) char smem_raw[];
    double *tileX = (double *)smem_raw;  // tile_rows * (K + 1)
    const int tid = threadIdx.x;
    const int KA = K + 1;
    const int E = K + K * (K + 1) / 2;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = min<int64_t>(rows, r0 + chunk);
    double acc[NE];
    int ia[NE], ja[NE];
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        acc[m] = 0.0;
        int e = tid + m * kThreads, i = 0, j = K;
        if (e < K) {
            i = e;
        } else if (e < E) {
            tri_index(e - K, i, j);
        }
        ia[m] = i;
        ja[m] = j;
    }
    for (int64_t base = r0; base < r1; base += tile_rows) {
        const int cnt = (int)min<int64_t>(tile_rows, r1 - base);
        for (int q = tid; q < cnt * KA; q += kThreads) {
            const int rr = q / KA, k = q - rr * KA;
            tileX[q] = k < K ? as_f64(X[(size_t)(base + rr) * ld + k]) : 1.0;
        }
        __syncthreads();
        for (int rr = 0; rr < cnt; ++rr) {
            const double *x = tileX + rr * KA;
#pragma unroll
            for (int m = 0; m < NE; ++m) acc[m] += x[ia[m]] * x[ja[m]];
        }
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        const int e = tid + m * kThreads;
        if (e < E) part[(size_t)blockIdx.x * E + e] = acc[m];
    }
}

// The same block sums on the FP64 matrix cores (nb = ceil(K/16) <= 7): one
// wavefront per block of rows, four rows per v_mfma_f64_16x16x4f64 step --
// lane l holds component 16*bi + (l % 16) of row 4g + l / 16 as an FP64
// value (FP32 factors convert exactly), which is both the A operand of block
// row bi and the B operand of block column bj, so only the nb(nb+1)/2 lower
// 16x16 blocks of X^T X are accumulated; sum x on the VALU from the same
// registers.  (The FP64 instruction returns D[4 v + l / 16][l % 16] in value v
// of lane l, unlike the FP32 one.)  Products of FP32 values are exact in
// FP64, and every sum is in FP64 in a fixed order.
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <int NB, typename XT>
__global__ __launch_bounds__(64) void hyper_moments_mfma(int K, const XT *__restrict__ X, int ld,
                                                         int64_t rows, int64_t chunk,
                                                         double *__restrict__ part)
{
    constexpr int NBLK = NB * (NB + 1) / 2;
    const int lane = threadIdx.x;
    const int col = lane & 15, kq = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = min<int64_t>(rows, r0 + chunk);
    const int E = K + K * (K + 1) / 2;
    doublex4 acc[NBLK];
#pragma unroll
    for (int q = 0; q < NBLK; ++q) acc[q] = doublex4{0.0, 0.0, 0.0, 0.0};
    double sx[NB];
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) sx[bi] = 0.0;
    // rows of the next step are loaded while this step's products run
    auto load = [&](int64_t base, XT (&y)[NB]) {
        const int64_t r = base + kq;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            const int c = 16 * bi + col;
            y[bi] = (r < r1 && c < K) ? X[(size_t)r * ld + c] : XT(0);
        }
    };
    XT ycur[NB], ynext[NB];
    load(r0, ycur);
    for (int64_t base = r0; base < r1; base += 4) {
        load(base + 4, ynext);
        double y[NB];
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            y[bi] = as_f64(ycur[bi]);
            sx[bi] += y[bi];
        }
        int q = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int bj = 0; bj <= bi; ++bj) {
                acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(y[bi], y[bj], acc[q], 0, 0, 0);
                ++q;
            }
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) ycur[bi] = ynext[bi];
    }
    double *dst = part + (size_t)blockIdx.x * E;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
        double t = sx[bi];
        t += __shfl_xor(t, 16);
        t += __shfl_xor(t, 32);
        const int c = 16 * bi + col;
        if (kq == 0 && c < K) dst[c] = t;
    }
    int q = 0;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = 0; bj <= bi; ++bj) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // FP64 result layout: lane l, value v holds D[4 v + l / 16][l % 16]
                const int i = 16 * bi + 4 * v + kq, j = 16 * bj + col;
                if (i < K && j <= i) dst[K + pk(i, j)] = acc[q][v];
            }
            ++q;
        }
}

// stats[e] = sum over blocks of part[b][e], in a fixed order, in two passes
// of one-wave workgroups (which fit beside the row kernels of the other
// side): wave (w, g) of the first pass takes entries 64 w .. 64 w + 63 (lane
// l entry 64 w + l, so every load of a wave is 512 contiguous bytes) and
// sums blocks g, g + 16, g + 32, ...; the second pass adds the 16 sums of
// each entry in order of g.
constexpr int kRedGroups = 16;
__global__ __launch_bounds__(64) void hyper_reduce_groups(int E, int nblk, const double *__restrict__ part,
                                                         double *__restrict__ red)
{
    const int lane = threadIdx.x;
    const int e = blockIdx.x * 64 + lane;
    const int g = blockIdx.y;
    if (e >= E) return;
    double s = 0.0;
#pragma unroll 8
    for (int b = g; b < nblk; b += kRedGroups) s += part[(size_t)b * E + e];
    red[(size_t)g * E + e] = s;
}

__global__ __launch_bounds__(64) void hyper_reduce(int E, const double *__restrict__ red,
                                                   double *__restrict__ stats)
{
    const int e = blockIdx.x * 64 + threadIdx.x;
    if (e >= E) return;
    double t = 0.0;
#pragma unroll
    for (int g = 0; g < kRedGroups; ++g) t += red[(size_t)g * E + e];
    stats[e] = t;
}

// In-place Cholesky of a packed lower K x K matrix (K <= 128) by the whole
// workgroup, right-looking with the column scaling deferred: step k
// subtracts P[i][k] P[j][k] / P[k][k] from the trailing entries (i >= j > k),
// reading column k unscaled; at the end column k is divided by
// sqrt(P[k][k]) and the pivot replaced by the root.  Steps go in pairs, one
// barrier per pair: every thread forms column k + 1 after step k from
// columns k and k + 1 as they were (the same operations in the same order
// as one step after the other), applies both steps to its trailing entries
// (j >= k + 2), and the pair's own update of column k + 1 is written in the
// next phase, when nothing reads that column.  Clears *ok on a
// non-positive pivot (which is then taken as 1).
template <int NT>
__device__ void chol_packed(int K, double *P, int *ok)
{
    __shared__ double root[128];
    const int tid = threadIdx.x;
    const int ti = tid & 31, tj = tid >> 5;  // a 32 x (NT / 32) tiling of the trailing triangle
    auto inv_pivot = [&](int k) {
        const double d = P[pk(k, k)];
        return 1.0 / (d > 0.0 ? d : 1.0);
    };
    // column c's update by step c - 1 (the second column of the pair before)
    auto pending = [&](int c) {
        const double rd = inv_pivot(c - 1), p = P[pk(c, c - 1)];
        for (int i = c + tid; i < K; i += NT) P[pk(i, c)] -= (P[pk(i, c - 1)] * rd) * p;
    };
    int k = 0;
    for (; k + 2 <= K - 1; k += 2) {
        if (k >= 2) pending(k - 1);
        const double rd0 = inv_pivot(k);
        const double p10 = P[pk(k + 1, k)];
        double d1 = P[pk(k + 1, k + 1)] - (p10 * rd0) * p10;
        const double rd1 = 1.0 / (d1 > 0.0 ? d1 : 1.0);
        for (int i = k + 2 + ti; i < K; i += 32) {
            const double pi0 = P[pk(i, k)] * rd0;
            const double pi1 = (P[pk(i, k + 1)] - pi0 * p10) * rd1;
            for (int j = k + 2 + tj; j <= i; j += NT / 32) {
                const double aj = P[pk(j, k)];
                const double qj = P[pk(j, k + 1)] - (aj * rd0) * p10;
                double v = P[pk(i, j)];
                v -= pi0 * aj;
                v -= pi1 * qj;
                P[pk(i, j)] = v;
            }
        }
        __syncthreads();
    }
    if (k >= 2) pending(k - 1);
    if (k == K - 2) {  // one step left: column K - 2 onto the last pivot
        if (tid == 0) {
            const double pik = P[pk(K - 1, k)] * inv_pivot(k);
            P[pk(K - 1, K - 1)] -= pik * P[pk(K - 1, k)];
        }
    }
    __syncthreads();
    for (int kk = tid; kk < K; kk += NT) {
        const double d = P[pk(kk, kk)];
        if (!(d > 0.0)) *ok = 0;
        root[kk] = sqrt(d > 0.0 ? d : 1.0);
    }
    __syncthreads();
    const int KK2 = K * (K + 1) / 2;
    for (int e = tid; e < KK2; e += NT) {
        int i, j;
        tri_index(e, i, j);
        P[e] = i == j ? root[j] : P[e] / root[j];
    }
    __syncthreads();
}

// X = C^-1 for a packed lower C (X packed lower, distinct storage): forward
// substitution on the identity with the row scaling deferred: step k
// subtracts C[i][k] X[k][j] / C[k][k] from the rows i > k, X[k] still
// unscaled; every row i is divided by C[i][i] at the end.  Steps go in
// pairs, one barrier per pair, as in chol_packed: row k + 1 after step k is
// formed by every thread that needs it and written in the next phase.
template <int NT>
__device__ void tri_inverse_packed(int K, const double *C, double *Xp)
{
    const int tid = threadIdx.x;
    const int KK2 = K * (K + 1) / 2;
    for (int e = tid; e < KK2; e += NT) {
        int i, j;
        tri_index(e, i, j);
        Xp[e] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    const int ti = tid & 31, tj = tid >> 5;  // a 32 x (NT / 32) tiling of rows i > k, columns j <= k
    // row r's update by step r - 1 (the second row of the pair before)
    auto pending = [&](int r) {
        const double c = C[pk(r, r - 1)] * (1.0 / C[pk(r - 1, r - 1)]);  // as in the pair
        for (int j = tid; j <= r - 1; j += NT) Xp[pk(r, j)] -= c * Xp[pk(r - 1, j)];
    };
    int k = 0;
    for (; k + 2 <= K - 1; k += 2) {
        if (k >= 2) pending(k - 1);
        const double rck0 = 1.0 / C[pk(k, k)], rck1 = 1.0 / C[pk(k + 1, k + 1)];
        const double c10 = C[pk(k + 1, k)] * rck0;
        for (int i = k + 2 + ti; i < K; i += 32) {
            const double ci0 = C[pk(i, k)] * rck0, ci1 = C[pk(i, k + 1)] * rck1;
            for (int j = tj; j <= k + 1; j += NT / 32) {
                const double xk = j <= k ? Xp[pk(k, j)] : 0.0;
                const double xk1 = j <= k ? Xp[pk(k + 1, j)] - c10 * xk : Xp[pk(k + 1, j)];
                double v = Xp[pk(i, j)];
                if (j <= k) v -= ci0 * xk;
                v -= ci1 * xk1;
                Xp[pk(i, j)] = v;
            }
        }
        __syncthreads();
    }
    if (k >= 2) pending(k - 1);
    if (k == K - 2) {  // one step left: row K - 1 from row K - 2
        const double c = C[pk(K - 1, k)] * (1.0 / C[pk(k, k)]);
        for (int j = tid; j <= k; j += NT) Xp[pk(K - 1, j)] -= c * Xp[pk(k, j)];
    }
    __syncthreads();
    for (int e = tid; e < KK2; e += NT) {
        int i, j;
        tri_index(e, i, j);
        Xp[e] /= C[pk(i, i)];
    }
    __syncthreads();
}

// The lower 16 x 16 blocks of a K x K product D = X Y on the FP64 matrix
// cores (v_mfma_f64_16x16x4_f64), the workgroup's waves taking the blocks
// in turn: block (bi, bj), bi >= bj, sums k over [k0, k1) = krange(bi, bj)
// in steps of four, lane l feeding X[16 bi + l % 16][k + l / 16] as the A
// operand and Y[k + l / 16][16 bj + l % 16] as the B operand (xf and yf
// return 0 outside their matrices' triangles and past K); out(i, j, d)
// receives every D[i][j] with j <= i < K (value v of lane l is
// D[4 v + l / 16][l % 16] of the block).  Every wave runs uniform loops.
template <int NT, typename XF, typename YF, typename KR, typename OUT>
__device__ __forceinline__ void lower_product_mfma(int K, XF xf, YF yf, KR krange, OUT out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int nb = (K + 15) / 16;
    for (int q = wave; q < nb * (nb + 1) / 2; q += NT / 64) {
        int bi, bj;
        tri_index(q, bi, bj);
        int k0, k1;
        krange(bi, bj, k0, k1);
        doublex4 acc = doublex4{0.0, 0.0, 0.0, 0.0};
        for (int kk = k0; kk < k1; kk += 4) {
            const double a = xf(16 * bi + col, kk + kq);
            const double b = yf(kk + kq, 16 * bj + col);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * bi + 4 * v + kq, j = 16 * bj + col;
            if (i < K && j <= i) out(i, j, acc[v]);
        }
    }
}

template <int NT, typename T>
__global__ __launch_bounds__(NT) void hyper_draw(
    int K, int64_t n, const double *__restrict__ stats, const double *__restrict__ mu0,
    const double *__restrict__ W0inv, double beta0, double nu0, uint64_t seed, uint32_t stream,
    const uint32_t *__restrict__ ctr, uint32_t t_off, double *__restrict__ gbuf, int n_lds_bufs,
    double *__restrict__ mu_out, double *__restrict__ Lam_out, T *__restrict__ Lam_w,
    T *__restrict__ Lmu_w, T *__restrict__ Linv_w, T *__restrict__ Ltmu_w, int *__restrict__ status)
{
    extern __shared__ __align__(16) char smem_raw[];
    const int KK2 = K * (K + 1) / 2;
    double *vec = (double *)smem_raw;  // xbar, mu*, z, mu  (4K)
    double *xbar = vec, *mus = vec + K, *zv = vec + 2 * K, *mu = vec + 3 * K;
    double *buf[3];
    for (int q = 0; q < 3; ++q)
        buf[q] = q < n_lds_bufs ? vec + 4 * K + (size_t)q * KK2 : gbuf + (size_t)q * KK2;
    double *Cm = buf[0];  // reversed W*^-1, then its Cholesky factor C, then A
    double *Ci = buf[1];  // C^-1
    double *Bm = buf[2];  // B = L_W A
    __shared__ int ok;
    const int tid = threadIdx.x;
    const uint32_t t = ctr[0] + t_off;
    const double dn = (double)n;
    const double beta_s = beta0 + dn;
    const double nu_s = nu0 + dn;
    const double shrink = beta0 * dn / beta_s;
    if (tid == 0) ok = 1;
    for (int k = tid; k < K; k += NT) {
        xbar[k] = stats[k] / dn;
        mus[k] = (beta0 * mu0[k] + dn * xbar[k]) / beta_s;
    }
    __syncthreads();
    // J W*^-1 J, packed: entry (i, j), i >= j, is W*^-1[K-1-j][K-1-i]
    for (int e = tid; e < KK2; e += NT) {
        int a, b;
        tri_index(e, a, b);  // W*^-1 entry (a, b), a >= b
        const double S = stats[K + e] - dn * xbar[a] * xbar[b];
        const double w = W0inv[a * K + b] + S + shrink * (xbar[a] - mu0[a]) * (xbar[b] - mu0[b]);
        Cm[pk(K - 1 - b, K - 1 - a)] = w;
    }
    __syncthreads();
    chol_packed<NT>(K, Cm, &ok);
    tri_inverse_packed<NT>(K, Cm, Ci);
    // Bartlett factor A (reuses Cm)
    for (int e = tid; e < KK2; e += NT) Cm[e] = 0.0;
    __syncthreads();
    for (int k = tid; k < K; k += NT)
        Cm[pk(k, k)] = sqrt(chi_square(seed, stream, t, (uint32_t)k, nu_s - (double)k, &ok));
    const int n_low = K * (K - 1) / 2;
    for (int blk = tid; 4 * blk < n_low; blk += NT) {
        double z[4];
        normals_block(seed, (uint32_t)blk, t, stream, 1u, 0u, z);
        for (int l = 0; l < 4 && 4 * blk + l < n_low; ++l) {
            int r, c;
            tri_index(4 * blk + l, r, c);  // strict-lower row-major index = pk(r+1, c)
            Cm[pk(r + 1, c)] = z[l];
        }
    }
    __syncthreads();
    // B = L_W A, L_W[r][m] = C^-1[K-1-m][K-1-r] (lower), A lower: block
    // (bi, bj) sums m over blocks bj .. bi
    lower_product_mfma<NT>(
        K, [&](int r, int m) { return (r < K && m <= r) ? Ci[pk(K - 1 - m, K - 1 - r)] : 0.0; },
        [&](int m, int c) { return (m < K && c <= m) ? Cm[pk(m, c)] : 0.0; },
        [](int bi, int bj, int &k0, int &k1) {
            k0 = 16 * bj;
            k1 = 16 * bi + 16;
        },
        [&](int r, int c, double d) { Bm[pk(r, c)] = d; });
    __syncthreads();
    // Lambda = B B^T: block (bi, bj) sums m over blocks 0 .. bj
    lower_product_mfma<NT>(
        K, [&](int r, int m) { return (r < K && m <= r) ? Bm[pk(r, m)] : 0.0; },
        [&](int m, int c) { return (c < K && m <= c) ? Bm[pk(c, m)] : 0.0; },
        [](int bi, int bj, int &k0, int &k1) {
            k0 = 0;
            k1 = 16 * bj + 16;
        },
        [&](int r, int c, double d) {
            Lam_out[r * K + c] = d;
            Lam_out[c * K + r] = d;
            Lam_w[r * K + c] = (T)d;
            Lam_w[c * K + r] = (T)d;
        });
    for (int blk = tid; 4 * blk < K; blk += NT) {
        double z[4];
        normals_block(seed, (uint32_t)blk, t, stream, 2u, 0u, z);
        for (int l = 0; l < 4 && 4 * blk + l < K; ++l) zv[4 * blk + l] = z[l];
    }
    __syncthreads();
    if (Linv_w) {
        // the rank-one row path needs B^-1 anyway: x = B^-T z as a product
        tri_inverse_packed<NT>(K, Bm, Ci);
        for (int i = tid; i < K; i += NT) {
            double s = 0.0;
            for (int j = i; j < K; ++j) s += Ci[pk(j, i)] * zv[j];
            mu[i] = s;  // staged: zv is still being read
        }
        __syncthreads();
        for (int i = tid; i < K; i += NT) zv[i] = mu[i];
    } else {
        // x = B^-T z (column oriented, one barrier per step), in zv: step i
        // takes x_i = zv[i] / B[i][i] (zv[i] final) and updates zv[j], j < i;
        // the divisions are applied to zv at the end
        for (int i = K - 1; i > 0; --i) {
            const double xi = zv[i] / Bm[pk(i, i)];
            for (int j = tid; j < i; j += NT) zv[j] -= Bm[pk(i, j)] * xi;
            __syncthreads();
        }
        for (int i = tid; i < K; i += NT) zv[i] /= Bm[pk(i, i)];
    }
    __syncthreads();
    const double rs = 1.0 / sqrt(beta_s);
    for (int k = tid; k < K; k += NT) {
        mu[k] = mus[k] + zv[k] * rs;
        mu_out[k] = mu[k];
    }
    __syncthreads();
    // Lambda mu from the packed factor: Lambda mu = B (B^T mu)
    for (int i = tid; i < K; i += NT) {
        double s = 0.0;
        for (int j = i; j < K; ++j) s += Bm[pk(j, i)] * mu[j];
        zv[i] = s;  // B^T mu
    }
    __syncthreads();
    for (int i = tid; i < K; i += NT) {
        double s = 0.0;
        for (int j = 0; j <= i; ++j) s += Bm[pk(i, j)] * zv[j];
        Lmu_w[i] = (T)s;
    }
    if (Linv_w) {
        // for the rank-one row path: chol(Lambda)^-1 = B^-1 (in Ci since the
        // solve for mu) and B^T mu
        for (int i = tid; i < K; i += NT) Ltmu_w[i] = (T)zv[i];
        for (int e = tid; e < K * K; e += NT) {
            const int r = e / K, cc = e - (e / K) * K;
            Linv_w[e] = cc <= r ? (T)Ci[pk(r, cc)] : (T)0;
        }
    }
    if (tid == 0 && !ok) *status = 0;
}

// For the rank-one row path after (mu, Lambda) were set by the host:
// chol(Lambda)^-1 and chol(Lambda)^T mu, FP64 in one workgroup.
template <typename T>
__global__ __launch_bounds__(kDrawThreads) void prior_factor(int K, const double *__restrict__ mu,
                                                         const double *__restrict__ Lam,
                                                         T *__restrict__ Linv_w, T *__restrict__ Ltmu_w,
                                                         int *__restrict__ status)
{
    extern __shared__ __align__(16) char smem_raw[];
    const int KK2 = K * (K + 1) / 2;
    double *P = (double *)smem_raw;
    double *Ci = P + KK2;
    __shared__ int ok;
    const int tid = threadIdx.x;
    if (tid == 0) ok = 1;
    for (int e = tid; e < KK2; e += kDrawThreads) {
        int r, c;
        tri_index(e, r, c);
        P[e] = Lam[r * K + c];
    }
    __syncthreads();
    chol_packed<kDrawThreads>(K, P, &ok);
    tri_inverse_packed<kDrawThreads>(K, P, Ci);
    for (int e = tid; e < K * K; e += kDrawThreads) {
        const int r = e / K, cc = e - (e / K) * K;
        Linv_w[e] = cc <= r ? (T)Ci[pk(r, cc)] : (T)0;
    }
    for (int i = tid; i < K; i += kDrawThreads) {
        double s = 0.0;
        for (int j = i; j < K; ++j) s += P[pk(j, i)] * mu[j];
        Ltmu_w[i] = (T)s;
    }
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

template <int NE>
void launch_moments(bpmf_ctx *c, const Side &sd, double *part, int used, int64_t chunk, hipStream_t s)
{
    const int tile_rows = (int)std::min<size_t>(64, 49152 / (sizeof(double) * (c->K + 1)));
    const size_t lds = sizeof(double) * tile_rows * (c->K + 1);
    if (c->prec == 0)
        hipLaunchKernelGGL((hyper_moments<NE, double>), dim3(used), dim3(kThreads), lds, s, c->K,
                           (const double *)sd.X, c->ld, sd.rows, chunk, tile_rows, part);
    else
        hipLaunchKernelGGL((hyper_moments<NE, float>), dim3(used), dim3(kThreads), lds, s, c->K,
                           (const float *)sd.X, c->ld, sd.rows, chunk, tile_rows, part);
}

int lds_buffers(int K, int lds_max)
{
    const size_t KK2 = (size_t)K * (K + 1) / 2;
    const size_t base = sizeof(double) * 4 * (size_t)K;
    int nb = 3;
    while (nb > 0 && base + sizeof(double) * nb * KK2 > (size_t)lds_max) --nb;
    return nb;
}

size_t draw_lds(int K, int nb) { return sizeof(double) * (4 * (size_t)K + nb * (size_t)K * (K + 1) / 2); }

}  // namespace

hipError_t launch_hyper(bpmf_ctx *c, int side_id, hipStream_t s, uint32_t t_off)
{
    double *part = c->hyp_part[side_id], *stats = c->hyp_stats[side_id];
    double *scratch = c->hyp_scratch[side_id];
    Side &sd = c->side[side_id];
    const int K = c->K;
    const int E = K + K * (K + 1) / 2;
    const int64_t rows = sd.rows;
    const int nblk = c->hyp_blocks;
    int64_t chunk = (rows + nblk - 1) / nblk;
    if (chunk < 1) chunk = 1;
    int used = (int)((rows + chunk - 1) / chunk);
    if (used < 1) used = 1;
    const int nbk = (K + 15) / 16;
    if (nbk <= 7) {
        auto go = [&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            if (c->prec == 0)
                hipLaunchKernelGGL((hyper_moments_mfma<NB, double>), dim3(used), dim3(64), 0, s, K,
                                   (const double *)sd.X, c->ld, rows, chunk, part);
            else
                hipLaunchKernelGGL((hyper_moments_mfma<NB, float>), dim3(used), dim3(64), 0, s, K,
                                   (const float *)sd.X, c->ld, rows, chunk, part);
        };
        switch (nbk) {
        case 1: go(std::integral_constant<int, 1>{}); break;
        case 2: go(std::integral_constant<int, 2>{}); break;
        case 3: go(std::integral_constant<int, 3>{}); break;
        case 4: go(std::integral_constant<int, 4>{}); break;
        case 5: go(std::integral_constant<int, 5>{}); break;
        case 6: go(std::integral_constant<int, 6>{}); break;
        default: go(std::integral_constant<int, 7>{}); break;
        }
    } else {
        const int ne = (E + kThreads - 1) / kThreads;
        if (ne <= 3) launch_moments<3>(c, sd, part, used, chunk, s);
        else if (ne <= 9) launch_moments<9>(c, sd, part, used, chunk, s);
        else if (ne <= 21) launch_moments<21>(c, sd, part, used, chunk, s);
        else launch_moments<33>(c, sd, part, used, chunk, s);
    }
    double *red = c->hyp_red[side_id];
    hipLaunchKernelGGL(hyper_reduce_groups, dim3((E + 63) / 64, kRedGroups), dim3(64), 0, s, E, used, part, red);
    hipLaunchKernelGGL(hyper_reduce, dim3((E + 63) / 64), dim3(64), 0, s, E, (const double *)red, stats);
    const int nb = lds_buffers(K, c->hyp_lds_max);
    const size_t lds2 = draw_lds(K, nb);
    // K <= 64: 256 threads (four waves find room beside the other side's row
    // kernels, where a 1024-thread workgroup waits for a whole free CU; one
    // wave is slower again: the steps' work outweighs their barriers);
    // above, 1024 threads
    auto draw = [&](auto ntc) {
        constexpr int NT = decltype(ntc)::value;
        if (c->prec == 0)
            hipLaunchKernelGGL((hyper_draw<NT, double>), dim3(1), dim3(NT), lds2, s, K, rows, stats, c->d_mu0,
                               c->d_W0inv, c->beta0, c->nu0, c->seed, sd.stream_hyp, c->ctr, t_off, scratch, nb,
                               sd.mu, sd.Lam, (double *)sd.Lam_w, (double *)sd.Lmu_w, (double *)nullptr,
                               (double *)nullptr, c->hyp_status);
        else
            hipLaunchKernelGGL((hyper_draw<NT, float>), dim3(1), dim3(NT), lds2, s, K, rows, stats, c->d_mu0,
                               c->d_W0inv, c->beta0, c->nu0, c->seed, sd.stream_hyp, c->ctr, t_off, scratch, nb,
                               sd.mu, sd.Lam, (float *)sd.Lam_w, (float *)sd.Lmu_w,
                               sd.n_low ? (float *)sd.Linv_w : (float *)nullptr,
                               sd.n_low ? (float *)sd.Ltmu_w : (float *)nullptr, c->hyp_status);
    };
    if (K <= 64)
        draw(std::integral_constant<int, 256>{});
    else
        draw(std::integral_constant<int, kDrawThreads>{});
    return hipGetLastError();
}

hipError_t prepare_hyper(bpmf_ctx *c)
{
    int dev_max = 65536;
    hipError_t e = hipDeviceGetAttribute(&dev_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device);
    if (e != hipSuccess) return e;
    c->hyp_lds_max = dev_max;
    const size_t need = draw_lds(c->K, lds_buffers(c->K, dev_max));
    if (need > 65536) {  // only above K = 64, where the draw has 1024 threads
        e = hipFuncSetAttribute((const void *)hyper_draw<kDrawThreads, double>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)hyper_draw<kDrawThreads, float>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
        if (e != hipSuccess) {  // keep the draw within the default limit
            (void)hipGetLastError();
            c->hyp_lds_max = 65536;
        }
    }
    return hipSuccess;
}

hipError_t launch_prior_to_working(bpmf_ctx *c, int side_id, hipStream_t s)
{
    Side &sd = c->side[side_id];
    if (sd.n_low && c->prec == 1) {
        const size_t lds = sizeof(double) * (size_t)c->K * (c->K + 1);
        hipLaunchKernelGGL((prior_factor<float>), dim3(1), dim3(kDrawThreads), lds, s, c->K, sd.mu, sd.Lam,
                           (float *)sd.Linv_w, (float *)sd.Ltmu_w, c->hyp_status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (c->prec == 0)
        hipLaunchKernelGGL((prior_to_working<double>), dim3(1), dim3(256), 0, s, c->K, sd.mu,
                           sd.Lam, (double *)sd.Lam_w, (double *)sd.Lmu_w);
    else
        hipLaunchKernelGGL((prior_to_working<float>), dim3(1), dim3(256), 0, s, c->K, sd.mu,
                           sd.Lam, (float *)sd.Lam_w, (float *)sd.Lmu_w);
    return hipGetLastError();
}

}  // namespace bpmf
