// row_lowrank.hip -- row update for rows with few ratings (d <= DMAX), FP32
// factors, K <= 64: the Cholesky factor of P is built from chol(Lambda) by
// rank-one updates instead of being factorised from scratch.
//
// The paper's shared-memory sampler uses a cheaper serial method for items
// with few ratings and a full Cholesky for the others (Sec. III, Fig. 2).
// Here: with L_Lam = chol(Lambda) (from the FP64 hyper draw) and
// a_j = sqrt(alpha) L_Lam^-1 y_j,
//   P = Lambda + alpha sum_j y_j y_j^T = L_Lam (I + sum_j a_j a_j^T) L_Lam^T,
// and chol(I + sum_j a_j a_j^T) = R_1 R_2 ... R_d with
//   R_j = chol(I + w_j w_j^T),  w_j = (R_1 ... R_{j-1})^-1 a_j,
// so chol(P) = L_Lam R_1 ... R_d is the same unique factor the oracle forms,
// and the draw x = L^-T (L^-1 b + z) is the same sample.  Each R = chol(I +
// w w^T) has a closed form in t_k = 1 + sum_{m<=k} w_m^2: R_kk =
// sqrt(t_k / t_{k-1}) and R_ik = w_i w_k / sqrt(t_{k-1} t_k) (i > k), and
// with q_k = sqrt(t_{k-1}/t_k), s_k = q_k / t_{k-1} its two solves are
//   R^-1 v:   y_k = q_k v_k - w_k s_k sum_{m<k} w_m v_m,
//   R^-T v:   x_k = q_k v_k - w_k sum_{i>k} w_i s_i v_i,
// i.e. one prefix (or suffix) sum each.  L_Lam^-1 b = L_Lam^T mu +
// alpha sum_j r'_j L_Lam^-1 y_j needs the gathered rows only through
// L_Lam^-1 y_j, which a small kernel precomputes for the whole gathered
// factor (transform_rows); x = L_Lam^-T (R_1^-T ... R_d^-T (L^-1 b + z)).
//
// Layout: four rows per wavefront, one 16-lane row of the wave per row of
// the factor; lane l holds components C l .. C l + C - 1 (C = K_pad / 16),
// prefix and suffix sums run within the lane and then across the 16 lanes
// by DPP row shifts.  Cost per row O(d^2 K + K^2 / 16) instructions instead
// of the K^3 / 3 of a factorisation.
#include "internal.h"
#include "rng_device.h"
#include "row_common.h"

namespace bpmf {
namespace {

template <int N>
__device__ __forceinline__ float dpp_shr(float x)  // lane l16 reads l16 - N of its row (0 below)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x110 + N, 0xf, 0xf, true));
}

template <int N>
__device__ __forceinline__ float dpp_shl(float x)  // lane l16 reads l16 + N of its row (0 above)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x100 + N, 0xf, 0xf, true));
}

// Exclusive prefix / suffix sums of x over the 16 lanes of each row.
__device__ __forceinline__ float row_excl_prefix(float x)
{
    float s = x;
    s += dpp_shr<1>(s);
    s += dpp_shr<2>(s);
    s += dpp_shr<4>(s);
    s += dpp_shr<8>(s);
    return s - x;
}

__device__ __forceinline__ float row_excl_suffix(float x)
{
    float s = x;
    s += dpp_shl<1>(s);
    s += dpp_shl<2>(s);
    s += dpp_shl<4>(s);
    s += dpp_shl<8>(s);
    return s - x;
}

// One rank-one factor R = chol(I + w w^T) in the form the solves use.
template <int C>
struct Factor {
    float w[C], q[C], ws[C];
};

// Factor parameters from w (the transformed update vector).
template <int C>
__device__ __forceinline__ void make_factor(const float (&w)[C], Factor<C> &f)
{
    float sq[C], run = 0.f;
#pragma unroll
    for (int e = 0; e < C; ++e) {
        sq[e] = run;  // exclusive within the lane
        run += w[e] * w[e];
    }
    const float base = 1.f + row_excl_prefix(run);
#pragma unroll
    for (int e = 0; e < C; ++e) {
        const float t_prev = base + sq[e];           // t_{k-1}
        const float t_k = t_prev + w[e] * w[e];      // t_k
        const float q = __builtin_sqrtf(t_prev / t_k);
        f.w[e] = w[e];
        f.q[e] = q;
        f.ws[e] = w[e] * (q / t_prev);
    }
}

// v <- R^-1 v
template <int C>
__device__ __forceinline__ void solve_fwd(const Factor<C> &f, float (&v)[C])
{
    float pre[C], run = 0.f;
#pragma unroll
    for (int e = 0; e < C; ++e) {
        pre[e] = run;
        run += f.w[e] * v[e];
    }
    const float base = row_excl_prefix(run);
#pragma unroll
    for (int e = 0; e < C; ++e) v[e] = f.q[e] * v[e] - f.ws[e] * (base + pre[e]);
}

// v <- R^-T v
template <int C>
__device__ __forceinline__ void solve_bwd(const Factor<C> &f, float (&v)[C])
{
    float suf[C], run = 0.f;
#pragma unroll
    for (int e = C - 1; e >= 0; --e) {
        suf[e] = run;
        run += f.ws[e] * v[e];
    }
    const float base = row_excl_suffix(run);
#pragma unroll
    for (int e = 0; e < C; ++e) v[e] = f.q[e] * v[e] - f.w[e] * (base + suf[e]);
}

// Yt[j] = L_Lam^-1 Y[j] for every row j of the gathered factor (padding 0).
template <int KP>
__global__ __launch_bounds__(256) void transform_rows(int K, const float *__restrict__ Y, int ld,
                                                      int64_t rows, const float *__restrict__ Linv,
                                                      float *__restrict__ Yt)
{
    __shared__ float Ls[KP * KP];
    for (int q = threadIdx.x; q < KP * KP; q += 256) {
        const int r = q / KP, c = q % KP;
        Ls[q] = (r < K && c <= r) ? Linv[r * K + c] : 0.f;
    }
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = g / KP;
    const int c = (int)(g % KP);
    if (j >= rows || c >= ld) return;
    float s = 0.f;
    if (c < K) {
        const float *y = Y + (size_t)j * ld;
        for (int m = 0; m <= c; ++m) s += Ls[c * KP + m] * y[m];
    }
    Yt[(size_t)j * ld + c] = s;
}

constexpr int kLowWPB = 4;  // waves per workgroup; four rows per wave

template <int C, int DMAX>
__global__ __launch_bounds__(64 * kLowWPB) void row_lowrank(
    int K, float alpha, const RowItem *__restrict__ items, int64_t item0, int64_t n_items,
    const int32_t *__restrict__ nbr, const float *__restrict__ rc, const float *__restrict__ Yt,
    int ld, const float *__restrict__ Linv, const float *__restrict__ Ltmu, float *__restrict__ X,
    int ldx, uint64_t seed, uint32_t stream, const uint32_t *__restrict__ ctr)
{
    constexpr int KP = 16 * C;
    __shared__ float Ms[KP * KP];  // Ms[m][c] = L_Lam^-1[m][c] (lower), padding 0
    __shared__ float Vs[kLowWPB * 4 * KP];
    for (int q = threadIdx.x; q < KP * KP; q += 64 * kLowWPB) {
        const int m = q / KP, c = q % KP;
        Ms[q] = (m < K && c <= m) ? Linv[m * K + c] : 0.f;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = lane >> 4, l16 = lane & 15;
    const int64_t first = item0 + ((int64_t)blockIdx.x * kLowWPB + wave) * 4;
    if (first >= n_items) return;
    const int64_t id = first + grp;
    const bool live = id < n_items;
    RowItem it{-1, -1, 0, 0};
    if (live) it = items[id];
    const int d = (int)(it.end - it.beg);
    // the wave's largest degree (items are in descending degree order)
    const int dw = __builtin_amdgcn_readfirstlane((int)(items[first].end - items[first].beg));
    const float sa = __builtin_sqrtf(alpha);

    float vb[C];
#pragma unroll
    for (int e = 0; e < C; ++e) {
        const int c = C * l16 + e;
        vb[e] = c < K ? Ltmu[c] : 0.f;
    }
    Factor<C> F[DMAX];
    // Up to 8 factors: every neighbour's id, rating and transformed row are
    // loaded before the factors are built (two round trips to memory in
    // all, not two per neighbour); the 16-factor instance has no registers
    // to spare and loads them as it goes.
    constexpr bool kPrefetch = DMAX <= 8;
    float pa[kPrefetch ? DMAX : 1][C], pr[kPrefetch ? DMAX : 1];
    if constexpr (kPrefetch) {
        int pc[DMAX];
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            pc[j] = j < d ? nbr[it.beg + j] : -1;
            pr[j] = j < d ? rc[it.beg + j] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
#pragma unroll
            for (int e = 0; e < C; ++e) {
                const int c = C * l16 + e;
                pa[j][e] = (pc[j] >= 0 && c < K) ? sa * Yt[(size_t)pc[j] * ld + c] : 0.f;  // 0: identity factor
            }
    }
    static_for<0, DMAX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j >= dw) return;  // uniform
        float a[C];
        float r = 0.f;
        if constexpr (kPrefetch) {
            r = pr[j];
#pragma unroll
            for (int e = 0; e < C; ++e) a[e] = pa[j][e];
        } else if (j < d) {
            const int col = nbr[it.beg + j];
            r = rc[it.beg + j];
#pragma unroll
            for (int e = 0; e < C; ++e) {
                const int c = C * l16 + e;
                a[e] = c < K ? sa * Yt[(size_t)col * ld + c] : 0.f;
            }
        } else {
#pragma unroll
            for (int e = 0; e < C; ++e) a[e] = 0.f;  // identity factor
        }
        // b: alpha r' L^-1 y = sqrt(alpha) r' a
#pragma unroll
        for (int e = 0; e < C; ++e) vb[e] += sa * r * a[e];
        static_for<0, j>([&](auto ic) { solve_fwd<C>(F[decltype(ic)::value], a); });
        make_factor<C>(a, F[j]);
    });
    // y = L^-1 b, then + z
    static_for<0, DMAX>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if (i < dw) solve_fwd<C>(F[i], vb);
    });
    const uint32_t row = live ? (uint32_t)it.row : 0u;
    if constexpr (C == 4) {
        // components 4 l16 .. 4 l16 + 3: the four normals of Philox block l16
        if (4 * l16 < K) {
            const Block4 bl = philox4x32_10(row, ctr[0], (stream << 24) | (uint32_t)l16, 0u, seed);
            float z[4];
            bm_normal4_f32(bl, z);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (4 * l16 + e < K) vb[e] += z[e];
        }
    } else if constexpr (C == 2) {
        // components 2 l16, 2 l16 + 1: one Box-Muller pair of block l16 / 2
        if (2 * l16 < K) {
            const Block4 bl = philox4x32_10(row, ctr[0], (stream << 24) | (uint32_t)(l16 >> 1), 0u, seed);
            const bool hi = (l16 & 1) != 0;
            float zc, zs;
            bm_pair_f32(hi ? bl.w2 : bl.w0, hi ? bl.w3 : bl.w1, zc, zs);
            vb[0] += zc;
            if (2 * l16 + 1 < K) vb[1] += zs;
        }
    } else {
#pragma unroll
        for (int e = 0; e < C; ++e) {
            const int c = C * l16 + e;
            if (c < K) {
                const Block4 bl = philox4x32_10(row, ctr[0], (stream << 24) | (uint32_t)(c >> 2), 0u, seed);
                const int m = c & 3;
                vb[e] += bm_normal_f32(m < 2 ? bl.w0 : bl.w2, m < 2 ? bl.w1 : bl.w3, (m & 1) != 0);
            }
        }
    }
    // R_d^-T ... R_1^-T
    static_for<0, DMAX>([&](auto qc) {
        constexpr int i = DMAX - 1 - decltype(qc)::value;
        if (i < dw) solve_bwd<C>(F[i], vb);
    });
    // x = L_Lam^-T v: x_c = sum_m Linv[m][c] v_m, with v through LDS and a
    // rolled loop over m (an unrolled one keeps all K_pad x C matrix reads
    // in flight at once)
    float *vs = Vs + (wave * 4 + grp) * KP;
#pragma unroll
    for (int e = 0; e < C; ++e) vs[C * l16 + e] = vb[e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float x[C];
#pragma unroll
    for (int e = 0; e < C; ++e) x[e] = 0.f;
#pragma unroll 4
    for (int m = 0; m < KP; ++m) {
        const float vm = vs[m];
        const float *mrow = Ms + m * KP + C * l16;
#pragma unroll
        for (int e = 0; e < C; ++e) x[e] = fmaf(mrow[e], vm, x[e]);
    }
    if (live)
#pragma unroll
        for (int e = 0; e < C; ++e) {
            const int c = C * l16 + e;
            if (c < K) X[(size_t)it.row * ldx + c] = x[e];
        }
}

}  // namespace

// The low-rank path: FP32 factors, K <= 64, and the buffer-offset and row-id
// limits of the matrix-core kernels (the same as the column-per-lane
// kernel's), so that the factorisation kernels that run beside it stop at
// the rank-one rows: the generic kernel would draw every row.
bool lowrank_available(const bpmf_ctx *c) { return c->prec == 1 && c->K <= 64 && fast_path_available(c); }

// The rows stage of a side with low-rank rows: transform the gathered
// factor, then the rows [n_items - n_low, n_items).  Degrees descend along
// the suffix, so it splits into tiers by the instance whose register
// footprint fits: rows with 9..16 ratings take the 16-factor instance, 5..8
// the 8-factor one and at most 4 the 4-factor one (76 VGPRs at K = 64, six
// waves per SIMD against four for the 8-factor one's 124).  A row's draw
// does not depend on its tier: a wave runs as many factors as its largest
// degree, and the extra ones of its other rows are exact identities.
hipError_t launch_row_lowrank(bpmf_ctx *c, int side_id, hipStream_t s)
{
    Side &sd = c->side[side_id];
    Side &ot = c->side[1 - side_id];
    if (sd.n_low == 0) return hipSuccess;
    const int nb = (c->K + 15) / 16;
    const int64_t item0 = sd.n_items - sd.n_low;
    const int64_t item_small = sd.n_items - sd.n_low_small;
    // the rows with at most 4 ratings: the last ones of the plan, whose whole
    // rows are the last items in the same order
    int64_t lo = sd.rows - sd.n_low, hi = sd.rows;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        const int32_t r = sd.perm[mid];
        if (sd.hptr[r + 1] - sd.hptr[r] <= 4)
            hi = mid;
        else
            lo = mid + 1;
    }
    const int64_t item_tiny = sd.n_items - (sd.rows - lo);
    auto go = [&](auto cc) {
        constexpr int C = decltype(cc)::value;
        constexpr int KP = 16 * C;
        const int64_t tot = ot.rows * (int64_t)KP;
        hipLaunchKernelGGL((transform_rows<KP>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                           c->K, (const float *)ot.X, c->ld, ot.rows, (const float *)sd.Linv_w, sd.Yt);
        auto rows = [&](auto dc, int64_t beg, int64_t end) {
            constexpr int D = decltype(dc)::value;
            if (end <= beg) return;
            const int64_t per_block = 4 * kLowWPB;
            const unsigned grid = (unsigned)((end - beg + per_block - 1) / per_block);
            hipLaunchKernelGGL((row_lowrank<C, D>), dim3(grid), dim3(64 * kLowWPB), 0, s, c->K,
                               (float)c->alpha, sd.items, beg, end, sd.nbr, (const float *)sd.rc,
                               (const float *)sd.Yt, c->ld, (const float *)sd.Linv_w,
                               (const float *)sd.Ltmu_w, (float *)sd.X, c->ld, c->seed, sd.stream_row,
                               c->ctr);
        };
        using D4 = std::integral_constant<int, 4>;
        using D8 = std::integral_constant<int, 8>;
        using D16 = std::integral_constant<int, 16>;
        if (c->low_dmax > 8) {
            rows(D16{}, item0, item_small);
            rows(D8{}, item_small, item_tiny);
            rows(D4{}, item_tiny, sd.n_items);
        } else if (c->low_dmax > 4) {
            rows(D8{}, item0, item_tiny);
            rows(D4{}, item_tiny, sd.n_items);
        } else {
            rows(D4{}, item0, sd.n_items);
        }
    };
    switch (nb) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    default: go(std::integral_constant<int, 4>{}); break;
    }
    return hipGetLastError();
}

}  // namespace bpmf
