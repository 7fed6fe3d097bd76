// foldin.hip -- scoring and top-n selection for fold-in requests.
//
// A new user's draws u_s (one per stored posterior sample s, made by the
// row-update machinery) score every movie j: p_sj = u_s . v_j^(s) + mean
// rating.  The predictive mean over the S samples and the variance
// 1/alpha + (1/S) sum_s (p_sj - mean_j)^2 (rating noise plus the spread of
// the samples) are formed per (request, movie); the top-n unrated movies by
// mean (descending, ties to the smaller movie id) are then selected exactly.
#include "internal.h"

namespace bpmf {
namespace {

constexpr int kScoreThreads = 128;
constexpr int kReqPerBlock = 8;
constexpr int kTopThreads = 256;

// grid (ceil(N / 128), ceil(n_req / 8)); thread = one movie, 8 requests.
// Mean and second central moment over samples by Welford's update.
__global__ __launch_bounds__(kScoreThreads) void foldin_score(
    int K, int ld, int N, int S, int n_req, const float *__restrict__ Vring, int64_t v_stride,
    const float *__restrict__ U, float rbar, float inv_alpha, float *__restrict__ mean,
    float *__restrict__ var)
{
    extern __shared__ float us[];  // [kReqPerBlock][S][ld]
    const int b0 = blockIdx.y * kReqPerBlock;
    const int nb = min(kReqPerBlock, n_req - b0);
    const int per_req = S * ld;
    for (int q = threadIdx.x; q < nb * per_req; q += kScoreThreads)
        us[q] = U[(size_t)b0 * per_req + q];
    __syncthreads();
    const int j = blockIdx.x * kScoreThreads + threadIdx.x;
    if (j >= N) return;
    float m[kReqPerBlock], m2[kReqPerBlock];
#pragma unroll
    for (int b = 0; b < kReqPerBlock; ++b) m[b] = m2[b] = 0.f;
    for (int s = 0; s < S; ++s) {
        const float *v = Vring + (size_t)s * v_stride + (size_t)j * ld;
        const float inv_n = 1.0f / (float)(s + 1);
#pragma unroll
        for (int b = 0; b < kReqPerBlock; ++b) {
            if (b >= nb) break;
            const float *u = us + b * per_req + s * ld;
            float p = 0.f;
            for (int k = 0; k < K; k += 4) {
                const float4 a = *reinterpret_cast<const float4 *>(u + k);
                const float4 w = *reinterpret_cast<const float4 *>(v + k);
                p += a.x * w.x + a.y * w.y + a.z * w.z + a.w * w.w;  // padding is 0
            }
            const float d = p - m[b];
            m[b] += d * inv_n;
            m2[b] += d * (p - m[b]);
        }
    }
    for (int b = 0; b < nb; ++b) {
        mean[(size_t)(b0 + b) * N + j] = m[b] + rbar;
        var[(size_t)(b0 + b) * N + j] = inv_alpha + m2[b] / (float)S;
    }
}

// Order-preserving map of a float to an unsigned key (larger float, larger key).
__device__ __forceinline__ uint32_t ord_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// One workgroup per request: exact top-n of the unrated movies by mean,
// ties to the smaller id.  Radix select of the n-th largest key (4 passes of
// 8 bits), then the keys above it plus the smallest-id ties, sorted by
// (key desc, id asc) with a bitonic network.
__global__ __launch_bounds__(kTopThreads) void foldin_topk(
    int N, const float *__restrict__ mean, const float *__restrict__ var,
    const int32_t *__restrict__ req_beg, const int32_t *__restrict__ nbr,
    const int32_t *__restrict__ top_n, int top_max, int32_t *__restrict__ out_ids,
    float *__restrict__ out_mean, float *__restrict__ out_var)
{
    extern __shared__ uint32_t sm[];
    const int words = (N + 31) / 32;
    uint32_t *rated = sm;                       // bitmap
    uint32_t *hist = rated + words;             // 256 bins
    uint32_t *scan = hist + 256;                // kTopThreads
    unsigned long long *sel = (unsigned long long *)(scan + kTopThreads + (words & 1));  // top_max (pow2)
    __shared__ uint32_t s_prefix, s_remaining, s_count;
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const float *mb = mean + (size_t)b * N;
    const float *vb = var + (size_t)b * N;
    for (int w = tid; w < words; w += kTopThreads) rated[w] = 0u;
    __syncthreads();
    const int beg = req_beg[b], end = req_beg[b + 1];
    for (int e = beg + tid; e < end; e += kTopThreads) {
        const int j = nbr[e];
        atomicOr(&rated[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
    int n_rated = 0;
    for (int w = 0; w < words; ++w) n_rated += __popc(rated[w]);
    const int want = min(min(top_n[b], top_max), N - n_rated);
    // key 0 marks a rated movie (every real key is > 0)
    auto key_of = [&](int j) -> uint32_t {
        return (rated[j >> 5] >> (j & 31)) & 1u ? 0u : ord_key(mb[j]);
    };
    if (tid == 0) {
        s_prefix = 0u;
        s_remaining = (uint32_t)max(want, 0);
    }
    __syncthreads();
    for (int shift = 24; shift >= 0 && want > 0; shift -= 8) {
        for (int q = tid; q < 256; q += kTopThreads) hist[q] = 0u;
        __syncthreads();
        const uint32_t prefix = s_prefix;
        const uint32_t hmask = shift == 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
        for (int j = tid; j < N; j += kTopThreads) {
            const uint32_t k = key_of(j);
            if (k != 0u && (k & hmask) == (prefix & hmask)) atomicAdd(&hist[(k >> shift) & 0xFFu], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t rem = s_remaining, bin = 255;
            for (int q = 255; q >= 0; --q) {
                if (hist[q] >= rem) {
                    bin = (uint32_t)q;
                    break;
                }
                rem -= hist[q];
            }
            s_prefix = prefix | (bin << shift);
            s_remaining = rem;  // how many keys equal to the final threshold to take
        }
        __syncthreads();
    }
    const uint32_t T = s_prefix;
    const uint32_t take_eq = s_remaining;
    // contiguous ranges per thread so that ties are taken in id order
    const int per = (N + kTopThreads - 1) / kTopThreads;
    const int j0 = tid * per, j1 = min(N, j0 + per);
    uint32_t eq_local = 0;
    if (want > 0)
        for (int j = j0; j < j1; ++j) eq_local += key_of(j) == T ? 1u : 0u;
    scan[tid] = eq_local;
    if (tid == 0) s_count = 0u;
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0;
        for (int q = 0; q < kTopThreads; ++q) {
            const uint32_t v = scan[q];
            scan[q] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int pow2 = 1;
    while (pow2 < want) pow2 <<= 1;
    for (int q = tid; q < pow2; q += kTopThreads) sel[q] = 0ull;
    __syncthreads();
    if (want > 0) {
        uint32_t eq_seen = scan[tid];
        for (int j = j0; j < j1; ++j) {
            const uint32_t k = key_of(j);
            bool pick = false;
            if (k > T) {
                pick = true;
            } else if (k == T) {
                pick = eq_seen < take_eq;
                ++eq_seen;
            }
            if (pick) {
                const uint32_t slot = atomicAdd(&s_count, 1u);
                if (slot < (uint32_t)pow2)
                    sel[slot] = ((unsigned long long)k << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)j);
            }
        }
    }
    __syncthreads();
    // bitonic sort, descending
    for (int size = 2; size <= pow2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int q = tid; q < pow2; q += kTopThreads) {
                const int p = q ^ stride;
                if (p > q) {
                    const bool desc = (q & size) == 0;
                    const unsigned long long a = sel[q], c = sel[p];
                    if (desc ? (a < c) : (a > c)) {
                        sel[q] = c;
                        sel[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int q = tid; q < top_max; q += kTopThreads) {
        const size_t o = (size_t)b * top_max + q;
        if (q < want) {
            const int j = (int)(0xFFFFFFFFu - (uint32_t)(sel[q] & 0xFFFFFFFFull));
            out_ids[o] = j;
            out_mean[o] = mb[j];
            out_var[o] = vb[j];
        } else {
            out_ids[o] = -1;
            out_mean[o] = 0.f;
            out_var[o] = 0.f;
        }
    }
}

}  // namespace

hipError_t launch_foldin_score(const bpmf_ctx *c, int n_req, int S, const float *Vring,
                               const float *U, float *mean, float *var, hipStream_t s)
{
    if (n_req == 0) return hipSuccess;
    const int64_t v_stride = c->N * (int64_t)c->ld;
    dim3 grid((unsigned)((c->N + kScoreThreads - 1) / kScoreThreads),
              (unsigned)((n_req + kReqPerBlock - 1) / kReqPerBlock));
    const size_t lds = sizeof(float) * kReqPerBlock * S * c->ld;
    hipLaunchKernelGGL(foldin_score, grid, dim3(kScoreThreads), lds, s, c->K, c->ld, (int)c->N, S,
                       n_req, Vring, v_stride, U, (float)c->rbar, (float)(1.0 / c->alpha), mean, var);
    return hipGetLastError();
}

size_t foldin_topk_lds(int N, int top_max)
{
    const int words = (N + 31) / 32;
    return sizeof(uint32_t) * (words + 256 + kTopThreads + 1) + sizeof(unsigned long long) * top_max + 16;
}

hipError_t launch_foldin_topk(const bpmf_ctx *c, int n_req, const float *mean, const float *var,
                              const int32_t *req_beg, const int32_t *nbr, const int32_t *top_n,
                              int top_max, int32_t *out_ids, float *out_mean, float *out_var,
                              hipStream_t s)
{
    if (n_req == 0) return hipSuccess;
    hipLaunchKernelGGL(foldin_topk, dim3((unsigned)n_req), dim3(kTopThreads),
                       foldin_topk_lds((int)c->N, top_max), s, (int)c->N, mean, var, req_beg, nbr,
                       top_n, top_max, out_ids, out_mean, out_var);
    return hipGetLastError();
}

}  // namespace bpmf
