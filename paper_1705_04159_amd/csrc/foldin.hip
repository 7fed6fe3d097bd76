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

typedef float score4 __attribute__((ext_vector_type(4)));  // one MFMA result per lane

constexpr int kScoreWaves = 4;  // waves per score workgroup, one 16-movie tile each
constexpr int kTopThreads = 1024;
constexpr int kTopWaves = kTopThreads / 64;

// Block (request group rg, movie block m) of the score grid.  Workgroups are
// dealt to the eight XCDs round-robin by their linear id, so the request
// groups of one movie block are given ids 8 apart: they land on the same XCD
// and read that block of the stored V samples from its L2 once.
__device__ __forceinline__ bool score_block(int n_blocks, int n_rg, int &rg, int &m)
{
    const int L = blockIdx.x;
    const int r = L >> 3;
    rg = r % n_rg;
    m = (r / n_rg) * 8 + (L & 7);
    return m < n_blocks;
}

// The scores of one sample are a matrix product, P_s = U_s V_s^T (requests x
// movies, over the K components), on the FP32 matrix cores: one wave takes 16
// requests x 16 movies, ld / 4 steps of v_mfma_f32_16x16x4_f32 per sample.
// Lane (g, c) holds components KQ g .. KQ g + KQ - 1 (KQ = ld / 4) of request
// c (A operand) and of movie c (B operand) and feeds component KQ g + t in
// step t, so both operands are contiguous loads; the operands of the next
// 2-8 samples (as registers allow) are in flight during each sample's
// products, which hides the load latency when a batch is a single request.
// The result D[4 g + v][c] (request 4 g + v, movie c) is folded into its
// running mean and second central moment by Welford's update.  Each output
// depends on its own request's row only (rows past the batch are zero), so
// it is the same in any batch.
template <int KQ>
__global__ __launch_bounds__(64 * kScoreWaves) void foldin_score(
    int N, int S, int n_req, const float *__restrict__ Vring, int64_t v_stride,
    const float *__restrict__ U, float rbar, float inv_alpha, float *__restrict__ mean,
    float *__restrict__ var)
{
    constexpr int LD = 4 * KQ;
    const int n_tiles = (N + 15) / 16;
    const int n_blocks = (n_tiles + kScoreWaves - 1) / kScoreWaves;
    const int n_rg = (n_req + 15) / 16;
    int rg, mb;
    if (!score_block(n_blocks, n_rg, rg, mb)) return;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    const int tile = mb * kScoreWaves + (threadIdx.x >> 6);
    if (tile >= n_tiles) return;  // wave-uniform
    const int req = rg * 16 + c;     // request of this lane's A row
    const int mov = tile * 16 + c;   // movie of this lane's B column
    const bool ra = req < n_req, mv = mov < N;
    const float *up = U + (size_t)(ra ? req : 0) * S * LD + KQ * g;
    const float *vp = Vring + (size_t)(mv ? mov : 0) * LD + KQ * g;
    // a ring of PF samples' operands in flight (slot q holds sample s0 + q)
    constexpr int PF = KQ <= 4 ? 8 : (KQ <= 8 ? 4 : 2);
    float a[PF][KQ], b[PF][KQ];
    auto load = [&](int q, int s) {
        const float *ua = up + (size_t)s * LD, *vb = vp + (size_t)s * v_stride;
        if constexpr (KQ % 4 == 0) {  // 16-byte runs: float4 loads
#pragma unroll
            for (int t = 0; t < KQ; t += 4) {
                const float4 x = ra ? *reinterpret_cast<const float4 *>(ua + t) : float4{0.f, 0.f, 0.f, 0.f};
                const float4 y = mv ? *reinterpret_cast<const float4 *>(vb + t) : float4{0.f, 0.f, 0.f, 0.f};
                a[q][t] = x.x, a[q][t + 1] = x.y, a[q][t + 2] = x.z, a[q][t + 3] = x.w;
                b[q][t] = y.x, b[q][t + 1] = y.y, b[q][t + 2] = y.z, b[q][t + 3] = y.w;
            }
        } else {
#pragma unroll
            for (int t = 0; t < KQ; ++t) {
                a[q][t] = ra ? ua[t] : 0.f;
                b[q][t] = mv ? vb[t] : 0.f;
            }
        }
    };
    float m[4] = {0.f, 0.f, 0.f, 0.f}, m2[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < PF; ++q)
        if (q < S) load(q, q);
    for (int s0 = 0; s0 < S; s0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int s = s0 + q;
            if (s >= S) break;  // uniform
            float ca[KQ], cb[KQ];
#pragma unroll
            for (int t = 0; t < KQ; ++t) {
                ca[t] = a[q][t];
                cb[t] = b[q][t];
            }
            if (s + PF < S) load(q, s + PF);
            score4 p = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < KQ; ++t) p = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[t], cb[t], p, 0, 0, 0);
            const float inv_n = 1.0f / (float)(s + 1);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float d = p[v] - m[v];
                m[v] += d * inv_n;
                m2[v] += d * (p[v] - m[v]);
            }
        }
    }
    if (!mv) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = rg * 16 + 4 * g + v;
        if (r < n_req) {
            mean[(size_t)r * N + mov] = m[v] + rbar;
            var[(size_t)r * N + mov] = inv_alpha + m2[v] / (float)S;
        }
    }
}

// Order-preserving map of a float to an unsigned key (larger float, larger key).
__device__ __forceinline__ uint32_t ord_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Inclusive prefix sum over the 64 lanes of a wave (lane order), and the
// same from the last lane down (suffix sum).
__device__ __forceinline__ uint32_t wave_prefix(uint32_t x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_suffix(uint32_t x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_down(x, off, 64);
        if (lane + off < 64) x += y;
    }
    return x;
}

// Exclusive prefix sum of one value per thread over the workgroup (thread
// order); wsum holds kTopWaves words of LDS.
__device__ __forceinline__ uint32_t block_excl_prefix(uint32_t x, uint32_t *wsum)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t inc = wave_prefix(x);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        const uint32_t v = lane < kTopWaves ? wsum[lane] : 0u;
        const uint32_t vi = wave_prefix(v);
        if (lane < kTopWaves) wsum[lane] = vi - v;
    }
    __syncthreads();
    const uint32_t r = wsum[w] + inc - x;
    __syncthreads();  // wsum may be reused right after
    return r;
}

// One workgroup per request: exact top-n of the unrated movies by mean,
// ties to the smaller id.  Keys: order-preserving images of the means, 0 for
// rated movies.  The n-th largest key T is found by radix selection over
// 8-bit digits, starting below the highest bit in which the smallest and
// largest candidate keys differ (the bits above it are common to all); then
// the keys above T and the smallest-id keys equal to T are gathered and
// sorted by (key desc, id asc) with a bitonic network.
__global__ __launch_bounds__(kTopThreads) void foldin_topk(
    int N, const float *__restrict__ mean, const float *__restrict__ var,
    const int32_t *__restrict__ req_beg, const int32_t *__restrict__ nbr,
    const int32_t *__restrict__ top_n, int top_max, int32_t *__restrict__ out_ids,
    float *__restrict__ out_mean, float *__restrict__ out_var)
{
    extern __shared__ uint32_t sm[];
    const int words = (N + 31) / 32;
    uint32_t *rated = sm;                    // bitmap of rated movies
    uint32_t *hist = rated + words;          // 256 bins
    uint32_t *wsum = hist + 256;             // kTopWaves
    unsigned long long *sel = (unsigned long long *)(wsum + kTopWaves + (words & 1));  // top_max (pow2)
    __shared__ uint32_t s_prefix, s_remaining, s_count, s_kmin, s_kmax;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int b = blockIdx.x;
    const float *mb = mean + (size_t)b * N;
    const float *vb = var + (size_t)b * N;
    for (int q = tid; q < words; q += kTopThreads) rated[q] = 0u;
    if (tid == 0) {
        s_kmin = 0xFFFFFFFFu;
        s_kmax = 0u;
        s_count = 0u;
    }
    __syncthreads();
    const int beg = req_beg[b], end = req_beg[b + 1];
    for (int e = beg + tid; e < end; e += kTopThreads) {
        const int j = nbr[e];
        atomicOr(&rated[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
    // the request's movies are distinct (checked at submission)
    const int want = min(min(top_n[b], top_max), N - (end - beg));
    auto key_of = [&](int j) -> uint32_t {
        return (rated[j >> 5] >> (j & 31)) & 1u ? 0u : ord_key(mb[j]);
    };
    // smallest and largest candidate key
    {
        uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
        for (int j = tid; j < N; j += kTopThreads) {
            const uint32_t k = key_of(j);
            if (k) {
                kmin = min(kmin, k);
                kmax = max(kmax, k);
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            kmin = min(kmin, (uint32_t)__shfl_xor(kmin, off, 64));
            kmax = max(kmax, (uint32_t)__shfl_xor(kmax, off, 64));
        }
        if (lane == 0) {
            atomicMin(&s_kmin, kmin);
            atomicMax(&s_kmax, kmax);
        }
    }
    __syncthreads();
    const uint32_t kmin = s_kmin, kmax = s_kmax;
    // bits above position p: p = 31 -> none
    auto above = [](int p) -> uint32_t { return p >= 31 ? 0u : (0xFFFFFFFFu << (p + 1)); };
    const int hb = want > 0 && kmin != kmax ? 31 - __clz(kmin ^ kmax) : -1;
    uint32_t prefix = kmax & above(hb);
    uint32_t rem = (uint32_t)max(want, 0);
    for (int hi = hb; hi >= 0; hi -= 8) {
        const int lo = max(hi - 7, 0);
        const uint32_t dmask = (1u << (hi - lo + 1)) - 1u;
        const uint32_t hmask = above(hi);
        for (int q = tid; q < 256; q += kTopThreads) hist[q] = 0u;
        __syncthreads();
        for (int j = tid; j < N; j += kTopThreads) {
            const uint32_t k = key_of(j);
            if (k != 0u && (k & hmask) == prefix) atomicAdd(&hist[(k >> lo) & dmask], 1u);
        }
        __syncthreads();
        if (w == 0) {
            // lane l holds bins 4l .. 4l+3; the bin where the count from the
            // top reaches rem holds the rem-th largest key
            uint32_t h[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) h[q] = hist[4 * lane + q];
            const uint32_t tot = h[0] + h[1] + h[2] + h[3];
            uint32_t acc = wave_suffix(tot) - tot;  // keys in the bins above this lane's
#pragma unroll
            for (int q = 3; q >= 0; --q) {
                if (acc < rem && acc + h[q] >= rem) {
                    s_prefix = prefix | ((uint32_t)(4 * lane + q) << lo);
                    s_remaining = rem - acc;
                }
                acc += h[q];
            }
        }
        __syncthreads();
        prefix = s_prefix;
        rem = s_remaining;
    }
    const uint32_t T = prefix;     // the want-th largest key
    const uint32_t take_eq = rem;  // keys equal to T to take (smallest ids)
    // contiguous id ranges per thread, so that ties are taken in id order
    const int per = (N + kTopThreads - 1) / kTopThreads;
    const int j0 = min(N, tid * per), j1 = min(N, j0 + per);
    uint32_t eq_local = 0;
    if (want > 0)
        for (int j = j0; j < j1; ++j) eq_local += key_of(j) == T ? 1u : 0u;
    uint32_t eq_seen = block_excl_prefix(eq_local, wsum);
    int pow2 = 1;
    while (pow2 < want) pow2 <<= 1;
    for (int q = tid; q < pow2; q += kTopThreads) sel[q] = 0ull;
    __syncthreads();
    if (want > 0) {
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
    const int n_tiles = (int)((c->N + 15) / 16);
    const int n_blocks = (n_tiles + kScoreWaves - 1) / kScoreWaves;
    const int n_rg = (n_req + 15) / 16;
    const unsigned grid = (unsigned)((n_blocks + 7) / 8 * 8 * n_rg);
    auto go = [&](auto kq) {
        constexpr int KQ = decltype(kq)::value;
        hipLaunchKernelGGL((foldin_score<KQ>), dim3(grid), dim3(64 * kScoreWaves), 0, s, (int)c->N, S,
                           n_req, Vring, v_stride, U, (float)c->rbar, (float)(1.0 / c->alpha), mean, var);
    };
    switch (c->ld / 4) {  // fold-in runs with K <= 64
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    case 5: go(std::integral_constant<int, 5>{}); break;
    case 6: go(std::integral_constant<int, 6>{}); break;
    case 7: go(std::integral_constant<int, 7>{}); break;
    case 8: go(std::integral_constant<int, 8>{}); break;
    case 9: go(std::integral_constant<int, 9>{}); break;
    case 10: go(std::integral_constant<int, 10>{}); break;
    case 11: go(std::integral_constant<int, 11>{}); break;
    case 12: go(std::integral_constant<int, 12>{}); break;
    case 13: go(std::integral_constant<int, 13>{}); break;
    case 14: go(std::integral_constant<int, 14>{}); break;
    case 15: go(std::integral_constant<int, 15>{}); break;
    case 16: go(std::integral_constant<int, 16>{}); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t foldin_topk_lds(int N, int top_max)
{
    const int words = (N + 31) / 32;
    return sizeof(uint32_t) * (words + 256 + kTopWaves + 1) + sizeof(unsigned long long) * top_max + 16;
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
