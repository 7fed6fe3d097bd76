// row_fast.hip -- matrix-core row update for FP32 factors, K <= 64 (sweeps
// take it up to K = 32, fold-in draws up to 64).
//
// Per row (Algorithm 1's item body with BPMF's conditional):
//   P = Lambda + alpha sum_j y_j y_j^T,  b = Lambda mu + alpha sum_j r'_j y_j,
//   P = L L^T,  y = L^-1 b,  x = L^-T (y + z).
//
// Work items are whole rows or segments of split rows; a wavefront takes
// RPW consecutive items (RPW = 64 / padded K: 4 for K <= 16, 2 for K <= 32,
// 1 above).
//
// Gram: the neighbour rows are gathered straight from HBM/L2 into the
// operand registers of v_mfma_f32_16x16x4_f32 -- lane l holds component
// 16*bi + (l % 16) of the neighbour row of rating 4g + l / 16, which is at
// once the A operand of block row bi and the B operand of block column bj --
// so only the nb(nb+1)/2 lower 16x16 blocks of P are accumulated (nb =
// ceil(K/16)), four ratings per instruction; the rhs accumulates on the VALU
// from the same registers.  Loads are buffer loads with 32-bit offsets:
// out-of-range offsets return 0, which masks the ragged tail and the padded
// components without branches.  The gather is software-pipelined: ids of
// chunk c+2 and rows of chunk c+1 are in flight while chunk c is multiplied.
//
// Cholesky: the accumulators go through LDS (packed lower triangle) into a
// column-per-lane layout
// (lane c of a row's lane group holds column c of P, plus b as an extra row).
// Right-looking elimination without square roots: at step k every column
// c > k subtracts its multiple of pivot column k, broadcast from lane k
// (v_readlane with one row per wave, ds_swizzle within 32- or 16-lane groups
// with several), so finished columns never need rescaling; the extra row
// carries b through the elimination, which is the forward solve L^-1 b.
// Each lane finally scales its column by 1/sqrt(d_c); the back solve runs
// row by row with one broadcast per row.
//
// Noise: lane c draws normal c of its row (Philox4x32-10 block c/4) with a
// Box-Muller evaluated in FP32 (the log of u close to 1 is taken as
// log1p(-(1-u)) so that no bits are lost).
#include <type_traits>

#include "internal.h"
#include "rng_device.h"
#include "row_common.h"

namespace bpmf {

hipError_t prepare_hyper(bpmf_ctx *c);

namespace {

// FP32 Gram and rhs of one work item (whole wave) on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16).  Each gathered FP32 entry y is split into
// three BF16 parts y = h + m + l (split3).  Block (bi, bj) of sum y y^T
// takes the six part products hh, hm, mh, hl, lh, mm, each exact, summed in
// FP32 by the matrix cores; the three left out (ml, lm, ll) are below
// 2^-22 |y_i y_j| together (FP32 rounding of the product itself: 2^-24).
// The rhs sum_j r'_j y_j uses the same instruction with the rating parts as
// the A operand: rows 0, 1, 2 of that tile hold the hi, mid and lo parts of
// r' (three planes, rc3), the other rows zero, and B runs over the three
// parts of y, so rows 0..2 of the result are sum_k part_p(r'_k) y_k and
// their sum is the rhs with all nine products.  Lane l holds, for the
// ratings 8 (l / 16) + e, e = 0..7, of a chunk of 32, the parts of
// component 16 bi + (l % 16): the A operand of block row bi and the B
// operand of block column bj at once.  Components >= K read whatever
// follows in the row (the caller ignores those entries); ratings past the
// end of the item read 0 (buffer range check on the last chunk).
template <int NB>
__device__ __forceinline__ void gram_item_p3(const RowItem &it, const int32_t *__restrict__ nbr,
                                             const uint16_t *__restrict__ rc3, uint32_t plane,
                                             __amdgpu_buffer_rsrc_t ysrc, uint32_t ldy4, int kq, int col,
                                             floatx4 (&acc)[NB * (NB + 1) / 2], floatx4 (&racc)[NB])
{
    const uint32_t cnt = (uint32_t)(it.end - it.beg);
    const __amdgpu_buffer_rsrc_t jsrc = make_rsrc(nbr + it.beg, cnt * 4u);
    const __amdgpu_buffer_rsrc_t psrc = make_rsrc(rc3 + it.beg, (uint32_t)(3u * plane - (uint32_t)it.beg) * 2u);
    const uint32_t poff = col < 3 ? 2u * ((uint32_t)col * plane + 8u * kq) : kOOB;
    const uint32_t coff = 4u * col;
    const uint32_t nchunk = (cnt + 31) / 32;
    // software pipeline: the next chunk's rows and rating parts, and the ids
    // of the chunk after it, are in flight during a chunk's products
    uint32_t jb[8];
    float yv[NB][8];
    u32x4 rp;
    auto load_ids = [&](uint32_t ch) {
#pragma unroll
        for (int e = 0; e < 8; ++e) jb[e] = buf_u32_stream(jsrc, (ch * 32 + 8 * kq + e) * 4u);
    };
    auto load_rows_t = [&](uint32_t ch, auto checkc) {
        constexpr bool CHECK = decltype(checkc)::value;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t t = ch * 32 + 8 * kq + e;
            uint32_t base = __umul24(jb[e], ldy4) + coff;  // fewer than 2^24 rows
            if constexpr (CHECK) base = t < cnt ? base : kOOB;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) yv[bi][e] = buf_f32(ysrc, base + 64u * bi);
        }
        rp = __builtin_amdgcn_raw_buffer_load_b128(psrc, poff + ch * 64u, 0, kStreamPolicy);
    };
    // only the last chunk (or chunk 0 of an empty item) runs past the end
    auto load_rows = [&](uint32_t ch) {
        if (ch + 1 < nchunk)
            load_rows_t(ch, std::integral_constant<bool, false>{});
        else
            load_rows_t(ch, std::integral_constant<bool, true>{});
    };
    bf16x8 H[NB], Md[NB], L[NB], R;
    auto convert = [&]() {
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            u32x4 h, m, l;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                uint32_t a, b, c;
                split3(yv[bi][2 * p], yv[bi][2 * p + 1], a, b, c);
                h[p] = a;
                m[p] = b;
                l[p] = c;
            }
            H[bi] = __builtin_bit_cast(bf16x8, h);
            Md[bi] = __builtin_bit_cast(bf16x8, m);
            L[bi] = __builtin_bit_cast(bf16x8, l);
        }
        R = __builtin_bit_cast(bf16x8, rp);
    };
    auto products = [&](auto firstc) {
        constexpr bool FIRST = decltype(firstc)::value;
        const floatx4 zero = floatx4{0.f, 0.f, 0.f, 0.f};
        // the small products first, block by block interleaved
        int q = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int bj = 0; bj <= bi; ++bj, ++q)
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Md[bi], Md[bj], FIRST ? zero : acc[q], 0, 0, 0);
#pragma unroll
        for (int bj = 0; bj < NB; ++bj)
            racc[bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(R, L[bj], FIRST ? zero : racc[bj], 0, 0, 0);
        q = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int bj = 0; bj <= bi; ++bj, ++q) {
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(L[bi], H[bj], acc[q], 0, 0, 0);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(H[bi], L[bj], acc[q], 0, 0, 0);
            }
#pragma unroll
        for (int bj = 0; bj < NB; ++bj)
            racc[bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(R, Md[bj], racc[bj], 0, 0, 0);
        q = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int bj = 0; bj <= bi; ++bj, ++q) {
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Md[bi], H[bj], acc[q], 0, 0, 0);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(H[bi], Md[bj], acc[q], 0, 0, 0);
            }
#pragma unroll
        for (int bj = 0; bj < NB; ++bj)
            racc[bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(R, H[bj], racc[bj], 0, 0, 0);
        q = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int bj = 0; bj <= bi; ++bj, ++q)
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(H[bi], H[bj], acc[q], 0, 0, 0);
    };
    // chunk ch: its rows are in registers, the ids of chunk ch + 1 in jb;
    // the next chunk's rows are issued before this chunk's products, then
    // the ids of the chunk after it
    auto step = [&](uint32_t ch, auto firstc) {
        convert();
        if (ch + 1 < nchunk) load_rows(ch + 1);
        if (ch + 2 < nchunk) load_ids(ch + 2);
        products(firstc);
    };
    // chunk 0 even for an empty item: every row it loads is 0 (out of range)
    load_ids(0);
    load_rows(0);
    if (nchunk > 1) load_ids(1);
    step(0u, std::integral_constant<bool, true>{});
    for (uint32_t ch = 1; ch < nchunk; ++ch) step(ch, std::integral_constant<bool, false>{});
}

// Factor and sample one row held column-per-lane: lane c of the group has
// v[r] = P[r][c] for r < KP (identity outside the leading K x K block) and
// v[KP] = b_c.  The normals come from Philox counters (c0, c1, stream<<24 |
// block, c3).  Returns x_c (meaningful for c < K).  A live lane whose pivot
// is not positive (P lost definiteness in FP32) clears *status.
template <int KP, int RPW>
__device__ __forceinline__ float chol_sample_column(float (&v)[KP + 1], int K, int c, uint32_t c0,
                                                    uint32_t c1, uint32_t c3, uint64_t seed,
                                                    uint32_t stream, bool live,
                                                    int *__restrict__ status)
{
    float mydiag = 1.f;
    static_for<0, KP>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const float dk = bcast<RPW, k>(v[k]);
        if (c == k) mydiag = dk;
        // lanes c <= k hold finished columns: multiplier 0 leaves them unchanged
        const float f = c > k ? v[k] * __builtin_amdgcn_rcpf(dk) : 0.f;
        float prk[KP + 1];
        static_for<k + 1, KP + 1>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            prk[r] = bcast<RPW, k>(v[r]);
        });
        static_for<k + 1, KP + 1>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            v[r] -= f * prk[r];
        });
    });
    if (live && !(mydiag > 0.f) && status) *status = 0;
    const float inv_s = __builtin_amdgcn_rsqf(mydiag);
#pragma unroll
    for (int r = 0; r < KP; ++r) v[r] *= inv_s;  // column c of L (rows > c)

    // w = L^-1 b + z
    float w = v[KP] * inv_s;
    {
        const uint32_t blk = (uint32_t)(c >> 2);
        const Block4 bl = philox4x32_10(c0, c1, (stream << 24) | blk, c3, seed);
        const int m = c & 3;
        const uint32_t wr = m < 2 ? bl.w0 : bl.w2;
        const uint32_t wa = m < 2 ? bl.w1 : bl.w3;
        if (c < K) w += bm_normal_f32(wr, wa, (m & 1) != 0);
    }
    // x = L^-T w, rows from the last (padded rows carry w = 0, x = 0)
    float accx = 0.f, myx = 0.f;
    static_for<0, KP>([&](auto qc) {
        constexpr int r = KP - 1 - decltype(qc)::value;
        const float xr = bcast<RPW, r>((w - accx) * inv_s);
        if (c == r) myx = xr;
        if (c < r) accx += v[r] * xr;
    });
    return myx;
}

// Lambda packed like the kernel's LDS copy of P: entry r (r + 1) / 2 + c,
// c <= r < KP, is Lambda[r][c] inside the leading K x K block, else 0.
__global__ __launch_bounds__(256) void prior_packed(int K, int KP, const float *__restrict__ Lam,
                                                    float *__restrict__ LamPk)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= KP * (KP + 1) / 2) return;
    int r = (int)((sqrtf(8.f * (float)e + 1.f) - 1.f) * 0.5f);
    while ((r + 1) * (r + 2) / 2 <= e) ++r;
    while (r * (r + 1) / 2 > e) --r;
    const int cc = e - r * (r + 1) / 2;
    LamPk[e] = (r < K && cc < K) ? Lam[r * K + cc] : 0.f;
}

// At least six waves per SIMD asked of the register allocator (K = 32: 71
// registers, so seven fit), which hides more of the gather latency than
// the unrestricted allocation's extra unrolling.  With P3 the Gram runs on
// the BF16 matrix cores from three-part splits of the FP32 rows and the
// rating planes rc3 (gram_item_p3); otherwise on the FP32 ones.
template <int NB, int RPW, int WPB, bool P3>
__global__ __launch_bounds__(64 * WPB, P3 ? 5 : 6) void row_fast_f32(
    int K, float alpha, const RowItem *__restrict__ items, int64_t item0, int64_t n_items,
    const int32_t *__restrict__ nbr, const float *__restrict__ rc, const uint16_t *__restrict__ rc3,
    uint32_t plane, const void *__restrict__ Y,
    int ldy, uint32_t y_bytes, const float *__restrict__ LamPk, const float *__restrict__ Lmu,
    float *__restrict__ X, int ldx, float *__restrict__ part, uint64_t seed, uint32_t stream,
    const uint32_t *__restrict__ ctr, int *__restrict__ status)
{
    constexpr int KP = 16 * NB;
    constexpr int NBLK = NB * (NB + 1) / 2;
    constexpr int LPR = 64 / RPW;  // lanes per row in the factorisation
    constexpr int REGION = KP * (KP + 1) / 2 + KP;  // packed lower triangle, then b
    extern __shared__ float smem_f[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int64_t first = item0 + ((int64_t)blockIdx.x * WPB + wave) * RPW;
    if (first >= n_items) return;
    float *Ps = smem_f + wave * RPW * REGION;
    const int col = lane & 15;
    const int kq = lane >> 4;
    const __amdgpu_buffer_rsrc_t ysrc = make_rsrc(Y, y_bytes);
    const uint32_t ldy4 = (uint32_t)ldy * 4u;
    uint32_t lane_off[NB];
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) lane_off[bi] = 16 * bi + col < K ? (16 * bi + col) * 4u : kOOB;
    const int KK2 = K * (K + 1) / 2;

    // The prior Lambda, packed like P (LamPk), into each row region of this
    // wave by direct global-to-LDS loads (no registers; they complete while
    // the gather runs): the Gram is later added onto it.
    {
        constexpr int NE = KP * (KP + 1) / 2;
        static_for<0, (NE + 63) / 64>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if (64 * i + lane < NE) {
#pragma unroll
                for (int h = 0; h < RPW; ++h)
                    __builtin_amdgcn_global_load_lds(
                        (const void __attribute__((address_space(1))) *)(LamPk + 64 * i + lane),
                        (void __attribute__((address_space(3))) *)(Ps + h * REGION + 64 * i), 4, 0, 0);
            }
        });
    }

    int row_of[RPW];
    static_for<0, RPW>([&](auto hc) {
        constexpr int h = decltype(hc)::value;
        row_of[h] = -1;
        const int64_t id = first + h;
        if (id >= n_items) return;
        const RowItem it = items[id];
        floatx4 acc[NBLK];
#pragma unroll
        for (int q = 0; q < NBLK; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
        float bacc[NB];
        if constexpr (P3) {
            floatx4 racc[NB];
            gram_item_p3<NB>(it, nbr, rc3, plane, ysrc, ldy4, kq, col, acc, racc);
            // rows 0..2 of the rhs tile (lanes 0..15: kq = 0), the three rating parts
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) bacc[bi] = (racc[bi][0] + racc[bi][1]) + racc[bi][2];
        } else {
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) bacc[bi] = 0.f;
            gram_item<NB, true>(it, nbr, rc, ysrc, ldy4, lane_off, kq, acc, bacc);
            // sum the rhs over the four rating slots of each 16-lane column
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) {
                bacc[bi] += __shfl_xor(bacc[bi], 16);
                bacc[bi] += __shfl_xor(bacc[bi], 32);
            }
        }
        if (it.slot >= 0) {  // segment of a split row: raw partial sums
            float *dst = part + (size_t)it.slot * (KK2 + K);
            int q = 0;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
                for (int bj = 0; bj <= bi; ++bj) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * bi + 4 * kq + v, c = 16 * bj + col;
                        if (r < K && c <= r) dst[pk(r, c)] = acc[q][v];
                    }
                    ++q;
                }
                const int c = 16 * bi + col;
                if (kq == 0 && c < K) dst[KK2 + c] = bacc[bi];
            }
            return;
        }
        float *P = Ps + h * REGION;
        int q = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
            for (int bj = 0; bj <= bi; ++bj) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * bi + 4 * kq + v, c = 16 * bj + col;
                    if (c <= r) P[pk(r, c)] = alpha * acc[q][v] + P[pk(r, c)];  // Lambda + alpha G
                }
                ++q;
            }
            if (kq == 0) P[KP * (KP + 1) / 2 + 16 * bi + col] = bacc[bi];
        }
        row_of[h] = it.row;
    });
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // column-per-lane within each lane group; groups without a full row
    // factor the identity and write nothing
    const int grp = lane / LPR;
    const int c = lane & (LPR - 1);
    int my_row = row_of[0];
#pragma unroll
    for (int h = 1; h < RPW; ++h)
        if (grp == h) my_row = row_of[h];
    const bool live = my_row >= 0 && c < K;
    const float *P = Ps + grp * REGION;
    const int cc = c < KP ? c : 0;
    float v[KP + 1];
#pragma unroll
    for (int r = 0; r < KP; ++r) v[r] = (live && r < K) ? P[r >= cc ? pk(r, cc) : pk(cc, r)] : (r == c ? 1.f : 0.f);
    v[KP] = live ? alpha * P[KP * (KP + 1) / 2 + cc] + Lmu[c] : 0.f;
    const float x = chol_sample_column<KP, RPW>(v, K, c, (uint32_t)my_row, ctr[0], 0u, seed, stream,
                                                live, status);
    if (live) X[(size_t)my_row * ldx + c] = x;
}

// Fold-in draws: item q is (request, stored sample s); its neighbour list is
// the request's rated movies, the gathered factor is V of sample s and the
// prior is (mu_U, Lambda_U) of sample s; the noise counter is
// (lo32(req id), s, stream<<24 | block, hi32(req id)).  Output row q of U.
template <int NB, int RPW, int WPB>
__global__ __launch_bounds__(64 * WPB) void foldin_draw_f32(
    int K, float alpha, const FoldItem *__restrict__ items, int64_t n_items,
    const int32_t *__restrict__ nbr, const float *__restrict__ rc, const float *__restrict__ Vring,
    int64_t v_stride, int ldy, uint32_t y_bytes, const float *__restrict__ Lam_ring,
    const float *__restrict__ Lmu_ring, const uint64_t *__restrict__ req_ids, int n_samples,
    float *__restrict__ U, int ldu, uint64_t seed, uint32_t stream, int *__restrict__ status)
{
    constexpr int KP = 16 * NB;
    constexpr int LDP = KP + 1;
    constexpr int NBLK = NB * (NB + 1) / 2;
    constexpr int LPR = 64 / RPW;
    constexpr int REGION = KP * LDP + KP;
    extern __shared__ float smem_f[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int64_t first = ((int64_t)blockIdx.x * WPB + wave) * RPW;
    if (first >= n_items) return;
    float *Ps = smem_f + wave * RPW * REGION;
    const int col = lane & 15;
    const int kq = lane >> 4;
    const uint32_t ldy4 = (uint32_t)ldy * 4u;
    uint32_t lane_off[NB];
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) lane_off[bi] = 16 * bi + col < K ? (16 * bi + col) * 4u : kOOB;
    int s_of[RPW], req_of[RPW];
    static_for<0, RPW>([&](auto hc) {
        constexpr int h = decltype(hc)::value;
        req_of[h] = -1;
        s_of[h] = 0;
        const int64_t id = first + h;
        if (id >= n_items) return;
        const FoldItem f = items[id];
        const RowItem it{f.req, -1, f.beg, f.end};
        const __amdgpu_buffer_rsrc_t ysrc = make_rsrc(Vring + (size_t)f.s * v_stride, y_bytes);
        floatx4 acc[NBLK];
#pragma unroll
        for (int q = 0; q < NBLK; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
        float bacc[NB];
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) bacc[bi] = 0.f;
        gram_item<NB, true>(it, nbr, rc, ysrc, ldy4, lane_off, kq, acc, bacc);
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            bacc[bi] += __shfl_xor(bacc[bi], 16);
            bacc[bi] += __shfl_xor(bacc[bi], 32);
        }
        float *P = Ps + h * REGION;
        int q = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
            for (int bj = 0; bj <= bi; ++bj) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * bi + 4 * kq + v, c = 16 * bj + col;
                    if (c <= r) P[pk(r, c)] = acc[q][v];
                }
                ++q;
            }
            if (kq == 0) P[KP * (KP + 1) / 2 + 16 * bi + col] = bacc[bi];
        }
        req_of[h] = f.req;
        s_of[h] = f.s;
    });
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int grp = lane / LPR;
    const int c = lane & (LPR - 1);
    int my_req = req_of[0], my_s = s_of[0];
#pragma unroll
    for (int h = 1; h < RPW; ++h)
        if (grp == h) {
            my_req = req_of[h];
            my_s = s_of[h];
        }
    const bool live = my_req >= 0 && c < K;
    const float *P = Ps + grp * REGION;
    const float *Lam = Lam_ring + (size_t)my_s * K * K;
    const float *Lmu = Lmu_ring + (size_t)my_s * K;
    const int cc = c < KP ? c : 0;
    float v[KP + 1];
#pragma unroll
    for (int r = 0; r < KP; ++r)
        v[r] = (live && r < K) ? alpha * P[r >= cc ? pk(r, cc) : pk(cc, r)] + Lam[r * K + c]
                               : (r == c ? 1.f : 0.f);
    v[KP] = live ? alpha * P[KP * (KP + 1) / 2 + cc] + Lmu[c] : 0.f;
    const uint64_t key = my_req >= 0 ? req_ids[my_req] : 0ull;
    const float x = chol_sample_column<KP, RPW>(v, K, c, (uint32_t)key, (uint32_t)my_s,
                                                (uint32_t)(key >> 32), seed, stream, live, status);
    const int64_t out_row = (int64_t)my_req * n_samples + my_s;
    if (live) U[(size_t)out_row * ldu + c] = x;
}

// Sum the partial slots of every split row into its first slot, in slot
// order (one thread per (row, entry)); eight slots' loads in flight at a
// time, added in order.
__global__ __launch_bounds__(256) void part_reduce(const FinishItem *__restrict__ fin, int E,
                                                   float *__restrict__ part)
{
    const FinishItem f = fin[blockIdx.x];
    const int e = blockIdx.y * 256 + threadIdx.x;
    if (e >= E || f.count <= 1) return;
    float *base = part + (size_t)f.first * E + e;
    float s = 0.f;
    int q = 0;
    for (; q + 8 <= f.count; q += 8) {
        float x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = base[(size_t)(q + u) * E];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += x[u];
    }
    for (; q < f.count; ++q) s += base[(size_t)q * E];
    base[0] = s;
}

// Split rows: lane c reads column c of the row's summed partial Gram (and
// b_c), adds the prior, then factors and samples as in the row kernel.  One
// wavefront per split row.
template <int NB, int WPB>
__global__ __launch_bounds__(64 * WPB) void row_finish_fast(
    int K, float alpha, const FinishItem *__restrict__ fin, int64_t n_fin,
    const float *__restrict__ part, const float *__restrict__ Lam, const float *__restrict__ Lmu,
    float *__restrict__ X, int ldx, uint64_t seed, uint32_t stream,
    const uint32_t *__restrict__ ctr, int *__restrict__ status)
{
    constexpr int KP = 16 * NB;
    const int c = threadIdx.x & 63;
    const int64_t fid = (int64_t)blockIdx.x * WPB + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (fid >= n_fin) return;
    const FinishItem f = fin[fid];
    const int KK2 = K * (K + 1) / 2;
    const bool live = c < K;
    const float *src = part + (size_t)f.first * (KK2 + K);
    float v[KP + 1];
#pragma unroll
    for (int r = 0; r < KP; ++r)
        v[r] = (live && r < K) ? alpha * src[r >= c ? pk(r, c) : pk(c, r)] + Lam[r * K + c]
                               : (r == c ? 1.f : 0.f);
    v[KP] = live ? alpha * src[KK2 + c] + Lmu[c] : 0.f;
    const float x = chol_sample_column<KP, 1>(v, K, c, (uint32_t)f.row, ctr[0], 0u, seed, stream,
                                              live, status);
    if (live) X[(size_t)f.row * ldx + c] = x;
}

template <int NB, int WPB>
hipError_t launch_finish_f32(bpmf_ctx *c, Side &sd, hipStream_t s)
{
    if (sd.n_fin == 0) return hipSuccess;
    hipError_t e = launch_part_reduce(c, sd, s, (int64_t)c->K * (c->K + 1) / 2 + c->K);
    if (e != hipSuccess) return e;
    const unsigned grid = (unsigned)((sd.n_fin + WPB - 1) / WPB);
    hipLaunchKernelGGL((row_finish_fast<NB, WPB>), dim3(grid), dim3(64 * WPB), 0, s, c->K,
                       (float)c->alpha, sd.fin, sd.n_fin, (const float *)c->part,
                       (const float *)sd.Lam_w, (const float *)sd.Lmu_w, (float *)sd.X, c->ld,
                       c->seed, sd.stream_row, c->ctr, c->hyp_status + 1);
    return hipGetLastError();
}

// Work items [item0, item_end): the segments of split rows are [0, n_slots),
// the whole rows follow, the rank-one path takes the last n_low.
template <int NB, int RPW, int WPB>
hipError_t launch_f32(bpmf_ctx *c, Side &sd, Side &ot, hipStream_t s, int64_t item0, int64_t item_end)
{
    constexpr int KP = 16 * NB;
    const size_t lds = sizeof(float) * WPB * RPW * (KP * (KP + 1) / 2 + KP);
    const int64_t count = item_end - item0;
    const int64_t per_block = (int64_t)WPB * RPW;
    const unsigned grid = (unsigned)((count + per_block - 1) / per_block);
    if (count <= 0) return hipSuccess;
    auto go = [&](auto kern, const void *Y, uint32_t y_bytes) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WPB), lds, s, c->K, (float)c->alpha, sd.items, item0,
                           item_end, sd.nbr, (const float *)sd.rc, (const uint16_t *)sd.rc3,
                           (uint32_t)(c->nnz + 32), Y, c->ld, y_bytes, (const float *)sd.Lam_pk,
                           (const float *)sd.Lmu_w, (float *)sd.X, c->ld, (float *)c->part, c->seed,
                           sd.stream_row, c->ctr, c->hyp_status + 1);
    };
    const uint32_t y_bytes = (uint32_t)(ot.rows * c->ld * sizeof(float));
    if constexpr (NB <= 2) {
        if (sd.rc3) {
            go(row_fast_f32<NB, RPW, WPB, true>, ot.X, y_bytes);
            return hipGetLastError();
        }
    }
    go(row_fast_f32<NB, RPW, WPB, false>, ot.X, y_bytes);
    return hipGetLastError();
}

}  // namespace

// Sum each split row's FP32 partial slots into its first slot.
hipError_t launch_part_reduce(bpmf_ctx *c, Side &sd, hipStream_t s, int64_t E)
{
    if (sd.n_fin == 0) return hipSuccess;
    hipLaunchKernelGGL(part_reduce, dim3((unsigned)sd.n_fin, (unsigned)((E + 255) / 256)), dim3(256),
                       0, s, sd.fin, (int)E, (float *)c->part);
    return hipGetLastError();
}

hipError_t launch_foldin_draw(const bpmf_ctx *c, const FoldItem *items, int64_t n_items,
                              const int32_t *nbr, const float *rc, const float *Vring,
                              const float *Lam_ring, const float *Lmu_ring, const uint64_t *req_ids,
                              int n_samples, float *U, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    const int nb = (c->K + 15) / 16;
    const int64_t v_stride = c->N * (int64_t)c->ld;
    const uint32_t y_bytes = (uint32_t)(v_stride * sizeof(float));
    auto go = [&](auto nbc, auto rpwc, auto wpbc) {
        constexpr int NB = decltype(nbc)::value, RPW = decltype(rpwc)::value, WPB = decltype(wpbc)::value;
        constexpr int KP = 16 * NB;
        const size_t lds = sizeof(float) * WPB * RPW * (KP * (KP + 1) + KP);
        const int64_t per_block = (int64_t)WPB * RPW;
        const unsigned grid = (unsigned)((n_items + per_block - 1) / per_block);
        hipLaunchKernelGGL((foldin_draw_f32<NB, RPW, WPB>), dim3(grid), dim3(64 * WPB), lds, s, c->K,
                           (float)c->alpha, items, n_items, nbr, rc, Vring, v_stride, c->ld, y_bytes,
                           Lam_ring, Lmu_ring, req_ids, n_samples, U, c->ld, c->seed, 7u,
                           (int *)nullptr);
    };
    using I = std::integral_constant<int, 1>;
    using II = std::integral_constant<int, 2>;
    using III = std::integral_constant<int, 3>;
    using IV = std::integral_constant<int, 4>;
    switch (nb) {
    case 1: go(I{}, IV{}, IV{}); break;
    case 2: go(II{}, II{}, IV{}); break;
    case 3: go(III{}, I{}, II{}); break;
    default: go(IV{}, I{}, II{}); break;
    }
    return hipGetLastError();
}

// The matrix-core path needs FP32 factors, K <= 64, and 32-bit buffer
// offsets for the gathered factor and every work item.
bool fast_path_available(const bpmf_ctx *c)
{
    if (c->prec != 1 || c->K > 64) return false;
    for (int s = 0; s < 2; ++s)
        if ((uint64_t)c->side[s].rows * c->ld * sizeof(float) >= kOOB || c->side[s].rows >= (1 << 24))
            return false;  // 32-bit buffer offsets, 24-bit row ids in the gather
    return (uint64_t)c->split_threshold * 4u < kOOB;
}

// FP32 factors with K <= 128: the matrix-core kernels form the Gram from
// three-part BF16 splits and take the rhs from the rating planes (the
// column-per-lane kernel always, the blocked one when its last block has
// room for the parts), read at 32-bit buffer offsets.
bool parts_gram_wanted(const bpmf_ctx *c)
{
    return c->prec == 1 && c->K <= 128 && 6u * ((uint64_t)c->nnz + 32u) < kOOB;
}

hipError_t launch_row_fast(bpmf_ctx *c, int side_id, hipStream_t s, int stage, bool *handled)
{
    *handled = false;
    // Sweeps use this kernel up to K = fast_kmax (32 by default: above it the
    // blocked factorisation of the K <= 128 kernel is faster; the autotuner
    // may raise it to 64).  Fold-in keeps it to K = 64.
    if (!fast_path_available(c) || c->K > c->fast_kmax) return hipSuccess;
    *handled = true;
    Side &sd = c->side[side_id];
    Side &ot = c->side[1 - side_id];
    const int nb = (c->K + 15) / 16;
    switch (stage) {
    case kStagePrior: {
        const int KP = 16 * nb;
        hipLaunchKernelGGL(prior_packed, dim3((KP * (KP + 1) / 2 + 255) / 256), dim3(256), 0, s, c->K, KP,
                           (const float *)sd.Lam_w, sd.Lam_pk);
        return hipGetLastError();
    }
    case kStageFinish:
        switch (nb) {
        case 1: return launch_finish_f32<1, 4>(c, sd, s);
        case 2: return launch_finish_f32<2, 4>(c, sd, s);
        case 3: return launch_finish_f32<3, 2>(c, sd, s);
        default: return launch_finish_f32<4, 2>(c, sd, s);
        }
    case kStageSegments: {
        // segments and whole rows in one launch: the heavy segments start
        // first and the whole rows fill in behind them, which balances the
        // load better than two launches (measured); the rank-one path (whole
        // rows stage) still runs beside it
        const int64_t e = sd.n_items - sd.n_low;
        switch (nb) {
        case 1: return launch_f32<1, 4, 4>(c, sd, ot, s, 0, e);
        case 2: return launch_f32<2, 2, 1>(c, sd, ot, s, 0, e);  // one-wave blocks: measured best
        case 3: return launch_f32<3, 1, 2>(c, sd, ot, s, 0, e);
        default: return launch_f32<4, 1, 2>(c, sd, ot, s, 0, e);
        }
    }
    default: return hipSuccess;
    }
}

hipError_t prepare_kernels(bpmf_ctx *c) { return prepare_hyper(c); }

}  // namespace bpmf
