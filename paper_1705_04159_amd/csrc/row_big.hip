// row_big.hip -- matrix-core row update with a blocked factorisation: FP32
// factors with 32 < K <= 128, and every K <= 128 in the BF16-Gram mode.
//
// Per row (Algorithm 1's item body with BPMF's conditional):
//   P = Lambda + alpha sum_j y_j y_j^T,  b = Lambda mu + alpha sum_j r'_j y_j,
//   P = L L^T,  y = L^-1 b,  x = L^-T (y + z).
// One wavefront per work item.
//
// Gram: FP32 rows on v_mfma_f32_16x16x4_f32 (as for K <= 32), or -- in the
// BF16-Gram mode -- BF16 copies of the neighbour rows on
// v_mfma_f32_16x16x32_bf16, where lane l supplies component 16*bi + (l % 16)
// of the 8 ratings 8*(l / 16) .. +7 of a 32-rating chunk; both accumulate in
// FP32 and only the nb(nb+1)/2 lower 16x16 blocks of P are formed.
//
// Storage: the accumulators hold the upper 16 x 16 blocks of the symmetric
// matrix -- block (i, j), i >= j, keeps T[16 j + r][16 i + c] (block row j,
// block column i) in the MFMA result layout, lane (g, c) rows r = 4g .. 4g+3
// of column c -- which the Gram forms directly by taking the block-column
// operand first.  In that storage both operands of every product the
// factorisation needs come straight from the registers.
//
// Factorisation: blocked right-looking Cholesky P = L L^T with 16 x 16
// blocks, by block rows of R = L^T.  For each block row kb:
//   - the diagonal block: column c of it is copied to every 16-lane row of
//     lanes (through LDS) and eliminated column by column without square
//     roots (column c > k takes -f_c times column k, f_c = P[k][c] / P[k][k],
//     column k's entry in the lane's own row coming from lane k of the row
//     by a DPP broadcast); the same column operations on the identity give
//     G = L_unit^-T (row r of G takes over row r's register once row r has
//     served as pivot row), so X = L_kk^-1 = D^-1/2 G^T is at hand, each lane
//     holding the A operand X[c][4g + v] of the products below; b's segment
//     rides along as one more row and yields y_kb = L_kk^-1 b_kb;
//   - the rest of the block row: R_kb,i = X T_kb,i on the matrix cores
//     (v_mfma_f32_16x16x4_f32, T_kb,i as the B operand straight from the
//     accumulators), and b_i -= L_i,kb y_kb;
//   - the trailing blocks: T_j,i -= R_kb,j^T R_kb,i on the matrix cores, both
//     operands straight from the accumulators (the first negated).
// Back solve x = L^-T w by block rows from the last, as products with the
// stored R and X and 16-lane reductions: no serial chain.
//
// Noise as in the other row kernels: Philox4x32-10 normal c of the row from
// block c/4 of counter (row, t, stream<<24 | block, 0), Box-Muller in FP32.
#include "internal.h"
#include "rng_device.h"
#include "row_common.h"

namespace bpmf {


namespace {


constexpr int kBigWPB = 1;     // waves per workgroup (independent; one-wave groups measured best)
constexpr int kPS = 17;        // panel row stride (floats)

// Waves per SIMD the register allocation must allow (left alone, the
// compiler trades occupancy for unrolled loads and drops to one wave).
template <int NB>
constexpr int big_waves()
{
    return NB <= 3 ? 4 : (NB == 4 ? 3 : 2);
}

// Per-wave LDS (floats): X = L_kk^-1 of every block row in the A-operand
// layout (one float4 per lane); the rhs b (becomes y), w and x.
template <int NB>
struct BigLds {
    static constexpr int XS = NB * 256;
    static constexpr int VEC = 16 * NB;
    static constexpr int BV = XS;  // offset of b
    static constexpr int TOTAL = XS + 3 * VEC;
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t buf_u16(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
}

// Gram and rhs of one work item from BF16 rows (whole wave).  Chunks of 32
// ratings; lane l takes ratings 8*(l/16) + e, e = 0..7, of each chunk, and
// loads component 16 bi + l % 16 of their rows for every block bi at
// immediate offsets from one address (components >= K of the last block
// then hold whatever follows the row and are replaced below).  The blocks
// are accumulated as upper blocks (block (bi, bj) holds (bj, bi)).  With
// AUG (kr = K - 16 (NB - 1) <= 13) lanes kr, kr + 1, kr + 2 of each row
// take the three BF16 parts of the ratings (hi + mid + lo == r', exactly)
// as components K, K + 1, K + 2, whose Gram rows then sum to the rhs
// sum_j r'_j y_j -- BF16 x BF16 products are exact in the FP32
// accumulation; the other components >= K are 0.  Without AUG they are
// all 0 and the rhs is summed into bacc on the vector units.  acc and bacc
// are written, not accumulated into.
template <int NB, bool AUG>
__device__ __forceinline__ void gram_item_bf16(const RowItem &it, const int32_t *__restrict__ nbr,
                                               const float *__restrict__ rc,
                                               const uint16_t *__restrict__ rc3, uint32_t plane, int kr,
                                               __amdgpu_buffer_rsrc_t ysrc, uint32_t ldy2, int kq, int col,
                                               floatx4 (&acc)[NB * (NB + 1) / 2],
                                               float (&bacc)[NB])
{
    const uint32_t cnt = (uint32_t)(it.end - it.beg);
    const __amdgpu_buffer_rsrc_t jsrc = make_rsrc(nbr + it.beg, cnt * 4u);
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(rc + it.beg, AUG ? 0u : cnt * 4u);
    // the three planes from this item on, one descriptor; lane part p reads
    // plane p, the other lanes read nothing
    const int p = col - kr;
    const bool part_lane = p >= 0 && p < 3;
    const __amdgpu_buffer_rsrc_t psrc =
        make_rsrc(rc3 + it.beg, AUG ? (uint32_t)(3u * plane - (uint32_t)it.beg) * 2u : 0u);
    const uint32_t poff = (AUG && part_lane) ? 2u * ((uint32_t)p * plane + 8u * kq) : kOOB;
    const bool pad_lane = col >= kr;  // components >= K of the last block
    const uint32_t coff = 2u * col;
    const uint32_t nchunk = (cnt + 31) / 32;
    // the first chunk starts the accumulators from zero (no separate clear)
    auto chunk = [&](uint32_t ch, auto firstc) {
        constexpr bool FIRST = decltype(firstc)::value;
        uint32_t base[8];
        float r[8];
        const bool last = ch + 1 >= nchunk;  // only the last chunk (or chunk 0 of an empty item) runs past the end
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t t = ch * 32 + 8 * kq + e;
            const uint32_t j = buf_u32_stream(jsrc, t * 4u);
            if constexpr (!AUG) r[e] = buf_f32_stream(rsrc, t * 4u);
            base[e] = __umul24(j, ldy2) + coff;  // fewer than 2^24 rows
            if (last) base[e] = t < cnt ? base[e] : kOOB;
        }
        u32x4 rp = u32x4{0u, 0u, 0u, 0u};
        if constexpr (AUG) rp = __builtin_amdgcn_raw_buffer_load_b128(psrc, poff + ch * 64u, 0, 0);
        // raw BF16 bits; pairs packed into dwords form the MFMA operand
        uint32_t yr[NB][8];
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int e = 0; e < 8; ++e) yr[bi][e] = buf_u16(ysrc, base[e] + 32u * bi) & 0xFFFFu;
        bf16x8 y[NB];
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            u32x4 w;
#pragma unroll
            for (int h = 0; h < 4; ++h) w[h] = yr[bi][2 * h] | (yr[bi][2 * h + 1] << 16);
            if (bi == NB - 1)
#pragma unroll
                for (int h = 0; h < 4; ++h) w[h] = pad_lane ? rp[h] : w[h];
            y[bi] = __builtin_bit_cast(bf16x8, w);
        }
        const floatx4 zero = floatx4{0.f, 0.f, 0.f, 0.f};
        int q = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
            for (int bj = 0; bj <= bi; ++bj) {
                // upper block (bj, bi)
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(y[bj], y[bi], FIRST ? zero : acc[q], 0, 0, 0);
                ++q;
            }
            if constexpr (!AUG) {
                float s = 0.f;
#pragma unroll
                for (int e = 0; e < 8; ++e) s += r[e] * __uint_as_float(yr[bi][e] << 16);  // c >= K: ignored
                bacc[bi] = FIRST ? s : bacc[bi] + s;
            }
        }
    };
    // chunk 0 even for an empty item: every row it loads is 0 (out of range)
    chunk(0u, std::integral_constant<bool, true>{});
    for (uint32_t ch = 1; ch < nchunk; ++ch) chunk(ch, std::integral_constant<bool, false>{});
}

// The FP32 Gram and rhs of one work item (whole wave) on the BF16 matrix
// cores, from three-part splits of the gathered FP32 rows (split3: y = h +
// m + l exactly; each block takes the six part products hh, hm, mh, hl, lh,
// mm, FP32 accumulation; the three left out are below 2^-22 |y_i y_j|),
// accumulated transposed like gram_item_bf16: block (bi, bj), bi >= bj,
// holds the upper block (bj, bi) in the MFMA result layout.  Chunks of 32
// ratings; lane l holds the parts of component 16 bi + l % 16 of the
// neighbour rows of ratings 8 (l / 16) + e, e = 0..7.  With AUG the last
// block's padding components kr, kr + 1, kr + 2 carry the centred rating's
// three BF16 parts (exact; the planes rc3) as their high part and zero mid
// and low parts, so that the Gram rows of those components hold the rhs
// with every part product (aug_rhs); otherwise the rhs is summed on the
// vector units from the FP32 rows.  Components >= K read whatever follows
// in the row (clear_padding drops them); ratings past the end of the item
// read 0 (buffer range check on the last chunk).
template <int NB, bool AUG>
__device__ __forceinline__ void gram_item_p3t(const RowItem &it, const int32_t *__restrict__ nbr,
                                              const float *__restrict__ rc,
                                              const uint16_t *__restrict__ rc3, uint32_t plane, int kr,
                                              __amdgpu_buffer_rsrc_t ysrc, uint32_t ldy4, int kq, int col,
                                              floatx4 (&acc)[NB * (NB + 1) / 2], float (&bacc)[NB])
{
    const uint32_t cnt = (uint32_t)(it.end - it.beg);
    const __amdgpu_buffer_rsrc_t jsrc = make_rsrc(nbr + it.beg, cnt * 4u);
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(rc + it.beg, AUG ? 0u : cnt * 4u);
    const int p = col - kr;
    const bool part_lane = p >= 0 && p < 3;
    const __amdgpu_buffer_rsrc_t psrc =
        make_rsrc(rc3 + it.beg, AUG ? (uint32_t)(3u * plane - (uint32_t)it.beg) * 2u : 0u);
    const uint32_t poff = (AUG && part_lane) ? 2u * ((uint32_t)p * plane + 8u * kq) : kOOB;
    const bool pad_lane = col >= kr;  // components >= K of the last block
    const uint32_t coff = 4u * col;
    const uint32_t nchunk = (cnt + 31) / 32;
    auto chunk = [&](uint32_t ch, auto firstc) {
        constexpr bool FIRST = decltype(firstc)::value;
        uint32_t base[8];
        float r[8];
        const bool last = ch + 1 >= nchunk;  // only the last chunk (or chunk 0 of an empty item) runs past the end
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t t = ch * 32 + 8 * kq + e;
            const uint32_t j = buf_u32_stream(jsrc, t * 4u);
            if constexpr (!AUG) r[e] = buf_f32_stream(rsrc, t * 4u);
            base[e] = __umul24(j, ldy4) + coff;  // fewer than 2^24 rows
            if (last) base[e] = t < cnt ? base[e] : kOOB;
        }
        u32x4 rp = u32x4{0u, 0u, 0u, 0u};
        if constexpr (AUG) rp = __builtin_amdgcn_raw_buffer_load_b128(psrc, poff + ch * 64u, 0, kStreamPolicy);
        bf16x8 H[NB], M[NB], L[NB];
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            float yv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) yv[e] = buf_f32(ysrc, base[e] + 64u * bi);
            if constexpr (!AUG) {
                float s = 0.f;
#pragma unroll
                for (int e = 0; e < 8; ++e) s += r[e] * yv[e];  // c >= K: dropped with the padding
                bacc[bi] = FIRST ? s : bacc[bi] + s;
            }
            u32x4 h, m, l;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t a, b, c;
                split3(yv[2 * q], yv[2 * q + 1], a, b, c);
                h[q] = a;
                m[q] = b;
                l[q] = c;
            }
            if (AUG && bi == NB - 1)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    h[q] = pad_lane ? rp[q] : h[q];
                    m[q] = pad_lane ? 0u : m[q];
                    l[q] = pad_lane ? 0u : l[q];
                }
            H[bi] = __builtin_bit_cast(bf16x8, h);
            M[bi] = __builtin_bit_cast(bf16x8, m);
            L[bi] = __builtin_bit_cast(bf16x8, l);
        }
        const floatx4 zero = floatx4{0.f, 0.f, 0.f, 0.f};
        // upper block (bj, bi): the small products first
        int q = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int bj = 0; bj <= bi; ++bj, ++q) {
                floatx4 a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(M[bj], M[bi], FIRST ? zero : acc[q], 0, 0, 0);
                a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(L[bj], H[bi], a, 0, 0, 0);
                a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(H[bj], L[bi], a, 0, 0, 0);
                a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(M[bj], H[bi], a, 0, 0, 0);
                a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(H[bj], M[bi], a, 0, 0, 0);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(H[bj], H[bi], a, 0, 0, 0);
            }
    };
    // chunk 0 even for an empty item: every row it loads is 0 (out of range)
    chunk(0u, std::integral_constant<bool, true>{});
    for (uint32_t ch = 1; ch < nchunk; ++ch) chunk(ch, std::integral_constant<bool, false>{});
}

// The rhs of an AUG Gram: component 16 bj + 4 g + v of sum_j r'_j y_j is
// value v of block (bj, NB - 1) summed over lanes kr .. kr + NP - 1 of row
// g (NP parts of the rating); left in lane kr of each row.
template <int NB, int NP>
__device__ __forceinline__ void aug_rhs(const floatx4 (&acc)[NB * (NB + 1) / 2], floatx4 (&rh)[NB])
{
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) {
        constexpr int q0 = (NB - 1) * NB / 2;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float x = acc[q0 + bj][v];
            if constexpr (NP == 3) {
                // row_shl:1 and row_shl:2: lane i + 1 and i + 2 of the row
                const float x1 = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x101, 0xf, 0xf, true));
                const float x2 = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x102, 0xf, 0xf, true));
                x += x1 + x2;
            }
            rh[bj][v] = x;
        }
    }
}

// Clear the Gram entries of components >= K (kr = K - 16 (NB - 1) < 16):
// columns kr.. of the blocks (bj, NB - 1), and rows kr.. of the last
// diagonal block.
template <int NB>
__device__ __forceinline__ void clear_padding(floatx4 (&acc)[NB * (NB + 1) / 2], int kr, int kq, int col)
{
    constexpr int q0 = (NB - 1) * NB / 2;
#pragma unroll
    for (int bj = 0; bj < NB; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const bool pad = col >= kr || (bj == NB - 1 && 4 * kq + v >= kr);
            acc[q0 + bj][v] = pad ? 0.f : acc[q0 + bj][v];
        }
}

// Sum over the 16 lanes of each 16-lane row, left in lane 15 of the row
// (inclusive prefix sums by DPP row shifts with zero fill).
__device__ __forceinline__ float row_sum16(float x)
{
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x111, 0xf, 0xf, true));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x112, 0xf, 0xf, true));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x114, 0xf, 0xf, true));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x118, 0xf, 0xf, true));
    return x;
}

// x from 16-lane row R of the wave, for every row (same lane within the
// row): v_permlane16_swap of x with itself leaves the even rows in the
// first result and the odd rows in the second (each twice), and
// v_permlane32_swap of that with itself leaves rows 0 and 1 of it in the
// first result and rows 2 and 3 in the second (each on all four rows).
template <int R>
__device__ __forceinline__ float bcast_row(float x)
{
    const uint32_t xi = __float_as_uint(x);
    const auto p = __builtin_amdgcn_permlane16_swap(xi, xi, false, false);
    const uint32_t y = (R & 1) ? p[1] : p[0];
    const auto q = __builtin_amdgcn_permlane32_swap(y, y, false, false);
    return __uint_as_float((R & 2) ? q[1] : q[0]);
}

// Blocked factorisation and draw for one row held in the accumulators (raw
// Gram, upper blocks) and b in LDS (b = alpha * rhs + Lambda mu already).
// Writes x_c.  A non-positive pivot of a real column clears *status.
template <int NB>
__device__ __forceinline__ void blocked_chol_sample(floatx4 (&acc)[NB * (NB + 1) / 2], float *lds,
                                                    int K, float alpha,
                                                    const floatx4 *__restrict__ img, uint32_t row,
                                                    uint32_t t, uint64_t seed, uint32_t stream,
                                                    float *__restrict__ xrow, int *__restrict__ status)
{
    using L = BigLds<NB>;
    float *xs = lds;              // X of block row kb: float4 per lane at kb * 256 + 4 lane
    float *bv = lds + L::BV;      // b, overwritten by y block by block
    float *wv = bv + L::VEC;
    float *xv = wv + L::VEC;
    const int lane = threadIdx.x & 63;
    const int col = lane & 15;
    const int kq = lane >> 4;

    // The accumulators hold the negated trailing matrix -(Lambda + alpha G -
    // sum R^T R), so that every product below takes positive operands (the
    // prior from its image in the same upper-block layout, identity on the
    // padding)
#pragma unroll
    for (int q = 0; q < NB * (NB + 1) / 2; ++q) {
        const floatx4 p = img[q * 64 + lane];
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[q][v] = -alpha * acc[q][v] - p[v];
    }

    // Diagonal block kb (already brought up to date): (1) lane (g, c) holds
    // rows 4g .. 4g + 3 of column c -- the accumulator layout itself (the
    // block is symmetric and stored whole); (2) eliminate columns k of the
    // real part: column c > k takes -f_c times column k (rows > k of d,
    // rows <= k of G -- the nonzero part of G's column k -- and b's row).
    // Each 16-lane group updates its own four rows; the pivot row comes from
    // the group that holds it.  Every block column but the last has 16 real
    // columns (the kernel is instantiated with NB = ceil(K / 16)).  (3)
    // pivots, y_kb, and X = L_kk^-1: lane (g, c) holds X[c][4g + v] =
    // G[4g + v][c] / sqrt(pivot_c), the A operand of step v, also kept in
    // LDS for the back solve.
    float xa[4];
    auto eliminate = [&](auto kbc) {
        constexpr int kb = decltype(kbc)::value;
        constexpr int qd = kb * (kb + 1) / 2 + kb;
        float u[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) u[v] = -acc[qd][v];
        float bc = bv[16 * kb + col];
        float mydiag = 1.f;
        const int kreal = K - 16 * kb;
        static_for<0, 16>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            constexpr int gk = k >> 2, vk = k & 3;
            if (kb + 1 < NB || k < kreal) {
                const float pr = bcast_row<gk>(u[vk]);  // row k of column col
                const float dk = bcast16<k>(pr);
                if (col == k) mydiag = dk;
                const float nf = col > k ? -pr * __builtin_amdgcn_rcpf(dk) : 0.f;
                if (kq == gk) u[vk] = col == k ? 1.f : 0.f;  // row k leaves d for G
                fmac_bc4<k>(u[0], u[1], u[2], u[3], nf);
                fmac_bc1<k>(bc, nf);
            }
        });
        if (kb + 1 == NB && kreal < 16)  // rows of the padding: G is the identity there
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (4 * kq + v >= kreal) u[v] = col == 4 * kq + v ? 1.f : 0.f;
        if (kq == 0 && col < kreal && !(mydiag > 0.f)) *status = 0;  // P not positive definite in FP32
        const float inv_s = __builtin_amdgcn_rsqf(mydiag);
#pragma unroll
        for (int v = 0; v < 4; ++v) xa[v] = u[v] * inv_s;
        *reinterpret_cast<float4 *>(xs + kb * 256 + 4 * lane) = float4{xa[0], xa[1], xa[2], xa[3]};
        if (kq == 0) bv[16 * kb + col] = bc * inv_s;  // y_kb
    };

    eliminate(std::integral_constant<int, 0>{});
    static_for<0, NB - 1>([&](auto kbc) {
        constexpr int kb = decltype(kbc)::value;
        constexpr int kn = kb + 1;
        __builtin_amdgcn_sched_barrier(0);
        // (4) R_kb,i = X T_kb,i = (-X)(-T_kb,i) on the matrix cores
        float nxa[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) nxa[v] = -xa[v];
        static_for<kb + 1, NB>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int q = i * (i + 1) / 2 + kb;
            floatx4 r = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) r = __builtin_amdgcn_mfma_f32_16x16x4f32(nxa[v], acc[q][v], r, 0, 0, 0);
            acc[q] = r;
        });
        wave_sync();  // y_kb visible to every lane
        // (5) b_i -= L_i,kb y_kb: (L_i,kb y)[c] = sum_m R_kb,i[m][c] y_m
        const float4 y4 = *reinterpret_cast<const float4 *>(bv + 16 * kb + 4 * kq);
        static_for<kb + 1, NB>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int q = i * (i + 1) / 2 + kb;
            float p = acc[q][0] * y4.x + acc[q][1] * y4.y + acc[q][2] * y4.z + acc[q][3] * y4.w;
            p += __shfl_xor(p, 16);
            p += __shfl_xor(p, 32);
            if (kq == 0) bv[16 * i + col] -= p;
        });
        wave_sync();  // b_kn visible to every lane
        // (6) trailing blocks T_j,i -= R_kb,j^T R_kb,i, kb < j <= i (the
        // negated T takes + R_kb,j^T R_kb,i): the next diagonal block first,
        // whose elimination then overlaps the other blocks' products
        auto trail = [&](auto jc, auto ic) {
            constexpr int j = decltype(jc)::value, i = decltype(ic)::value;
            constexpr int qi = i * (i + 1) / 2 + kb, qj = j * (j + 1) / 2 + kb;
            constexpr int q = i * (i + 1) / 2 + j;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(acc[qj][v], acc[qi][v], acc[q], 0, 0, 0);
        };
        trail(std::integral_constant<int, kn>{}, std::integral_constant<int, kn>{});
        static_for<kn, NB>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            static_for<kn, i + 1>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                if constexpr (!(i == kn && j == kn)) trail(jc, ic);
            });
        });
        eliminate(std::integral_constant<int, kn>{});
    });
    wave_sync();

    // w = y + z: lanes l and l + 32 (l < 4 NB) take components 4l, 4l + 1
    // and 4l + 2, 4l + 3, whose normals are the Box-Muller pairs (w0, w1) and
    // (w2, w3) of Philox block l
    {
        const int blk = lane & 31, hf = lane >> 5;
        const int c0 = 4 * blk + 2 * hf;
        if (blk < 4 * NB) {
            float2 w = *reinterpret_cast<const float2 *>(bv + c0);
            if (c0 < K) {
                const Block4 bl = philox4x32_10(row, t, (stream << 24) | (uint32_t)blk, 0u, seed);
                float zc, zs;
                bm_pair_f32(hf ? bl.w2 : bl.w0, hf ? bl.w3 : bl.w1, zc, zs);
                w.x += zc;
                if (c0 + 1 < K) w.y += zs;
            }
            *reinterpret_cast<float2 *>(wv + c0) = w;
        }
    }
    wave_sync();
    // x = L^-T w by block rows from the last:
    //   x_kb = X^T (w_kb - sum_{i > kb} R_kb,i x_i),
    // (R_kb,i x_i)[m] = sum_c R_kb,i[m][c] x_i[c] and (X^T w')[m] =
    // sum_c X[c][m] w'_c, both as 16-lane sums of per-lane products
    static_for<0, NB>([&](auto qc) {
        constexpr int kb = NB - 1 - decltype(qc)::value;
        float s[4] = {0.f, 0.f, 0.f, 0.f};
        static_for<kb + 1, NB>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int q = i * (i + 1) / 2 + kb;
            const float xc = xv[16 * i + col];
#pragma unroll
            for (int v = 0; v < 4; ++v) s[v] += acc[q][v] * xc;
        });
        if constexpr (kb + 1 < NB) {
#pragma unroll
            for (int v = 0; v < 4; ++v) s[v] = row_sum16(s[v]);
            if (col == 15) {
                float4 *p = reinterpret_cast<float4 *>(wv + 16 * kb + 4 * kq);
                float4 o = *p;
                o.x -= s[0];
                o.y -= s[1];
                o.z -= s[2];
                o.w -= s[3];
                *p = o;
            }
            wave_sync();
        }
        const float4 xa = *reinterpret_cast<const float4 *>(xs + kb * 256 + 4 * lane);
        const float wc = wv[16 * kb + col];
        float o[4] = {xa.x * wc, xa.y * wc, xa.z * wc, xa.w * wc};
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = row_sum16(o[v]);
        if (col == 15) *reinterpret_cast<float4 *>(xv + 16 * kb + 4 * kq) = float4{o[0], o[1], o[2], o[3]};
        wave_sync();
    });
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int cc = lane + 64 * h;
        if (cc < K) xrow[cc] = xv[cc];
    }
}

// Partial sums of a segment of a split row: the accumulator image (block q,
// lane l, value v at (64 q + l) 4 + v; zero on the padding) followed by the
// rhs (component c at 64 nb(nb+1)/2 ... + c), so stores and loads are whole
// float4 per lane.
template <int NB>
constexpr int64_t big_slot_elems()
{
    return (int64_t)NB * (NB + 1) / 2 * 256 + 16 * NB;
}


// SEG: the work items are segments of split rows and only their partial
// sums are written; otherwise they are whole rows, factored and sampled.
// (Two instantiations keep the partial path's registers out of the
// factorisation's budget.)  AUG (BF16 rows with K - 16 (NB - 1) <= 13): the
// rhs comes out of the Gram, the rating parts being padding components;
// otherwise it is summed on the vector units.
template <int NB, bool BF16, bool SEG, bool AUG>
__global__ __launch_bounds__(64 * kBigWPB, big_waves<NB>()) void row_big(
    int K, float alpha, const RowItem *__restrict__ items, int64_t item0, int64_t n_items,
    const int32_t *__restrict__ nbr, const float *__restrict__ rc, const uint16_t *__restrict__ rc3,
    uint32_t plane, const void *__restrict__ Y, int ldy, uint32_t y_bytes, const floatx4 *__restrict__ img,
    const float *__restrict__ Lmu, float *__restrict__ X, int ldx, float *__restrict__ part, uint64_t seed,
    uint32_t stream, const uint32_t *__restrict__ ctr, int *__restrict__ status)
{
    constexpr int NBLK = NB * (NB + 1) / 2;
    extern __shared__ float smem_f[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int64_t id = item0 + (int64_t)blockIdx.x * kBigWPB + wave;
    if (id >= n_items) return;
    const int col = lane & 15;
    const int kq = lane >> 4;
    const int kr = K - 16 * (NB - 1);  // real components of the last block
    const RowItem it = items[id];
    const __amdgpu_buffer_rsrc_t ysrc = make_rsrc(Y, y_bytes);
    floatx4 acc[NBLK];
    float bacc[NB];
    if constexpr (BF16)
        gram_item_bf16<NB, AUG>(it, nbr, rc, rc3, plane, kr, ysrc, (uint32_t)ldy * 2u, kq, col, acc, bacc);
    else  // FP32 rows: the Gram from their three-part BF16 splits
        gram_item_p3t<NB, AUG>(it, nbr, rc, rc3, plane, kr, ysrc, (uint32_t)ldy * 4u, kq, col, acc, bacc);
    float *lds = smem_f + wave * BigLds<NB>::TOTAL;
    float *bv = lds + BigLds<NB>::BV;
    float *rdst = SEG ? part + (size_t)it.slot * big_slot_elems<NB>() + NBLK * 256 : bv;
    if constexpr (AUG) {
        floatx4 rh[NB];
        aug_rhs<NB, 3>(acc, rh);
        clear_padding<NB>(acc, kr, kq, col);
        if (col == kr)
#pragma unroll
            for (int bj = 0; bj < NB; ++bj) *reinterpret_cast<floatx4 *>(rdst + 16 * bj + 4 * kq) = rh[bj];
    } else {
        clear_padding<NB>(acc, kr, kq, col);  // rows loaded past K (none if kr == 16)
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            bacc[bi] += __shfl_xor(bacc[bi], 16);
            bacc[bi] += __shfl_xor(bacc[bi], 32);
        }
        if (kq == 0)
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) rdst[16 * bi + col] = bacc[bi];
    }
    if constexpr (SEG) {
        float *dst = part + (size_t)it.slot * big_slot_elems<NB>();
#pragma unroll
        for (int q = 0; q < NBLK; ++q) reinterpret_cast<floatx4 *>(dst)[q * 64 + lane] = acc[q];
    } else {
        wave_sync();  // the rhs in bv
        if (kq == 0)
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) {
                const int c = 16 * bi + col;
                bv[c] = c < K ? alpha * bv[c] + Lmu[c] : 0.f;
            }
        wave_sync();
        blocked_chol_sample<NB>(acc, lds, K, alpha, img, (uint32_t)it.row, ctr[0], seed, stream,
                                X + (size_t)it.row * ldx, status);
    }
}

// Split rows: the partial Gram slots of the row, summed in slot order into
// the accumulators, then the same factorisation.
template <int NB>
__global__ __launch_bounds__(64 * kBigWPB, big_waves<NB>()) void row_finish_big(
    int K, float alpha, const FinishItem *__restrict__ fin, int64_t n_fin,
    const float *__restrict__ part, const floatx4 *__restrict__ img, const float *__restrict__ Lmu,
    float *__restrict__ X, int ldx, uint64_t seed, uint32_t stream,
    const uint32_t *__restrict__ ctr, int *__restrict__ status, int summed)
{
    constexpr int NBLK = NB * (NB + 1) / 2;
    extern __shared__ float smem_f[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int64_t fid = (int64_t)blockIdx.x * kBigWPB + wave;
    if (fid >= n_fin) return;
    float *lds = smem_f + wave * BigLds<NB>::TOTAL;
    const int col = lane & 15;
    const int kq = lane >> 4;
    const FinishItem f = fin[fid];
    // the row's partial slots summed in slot order (with `summed`, already
    // summed into the first by part_reduce, in the same order)
    const float *src = part + (size_t)f.first * big_slot_elems<NB>();
    const int count = summed ? 1 : f.count;
    floatx4 acc[NBLK];
#pragma unroll
    for (int q = 0; q < NBLK; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    float bs[2] = {0.f, 0.f};
    for (int sl = 0; sl < count; ++sl) {
        const float *sq = src + (size_t)sl * big_slot_elems<NB>();
#pragma unroll
        for (int q = 0; q < NBLK; ++q) acc[q] += reinterpret_cast<const floatx4 *>(sq)[q * 64 + lane];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = lane + 64 * h;
            if (c < 16 * NB) bs[h] += sq[NBLK * 256 + c];
        }
    }
    float *bv = lds + BigLds<NB>::BV;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = lane + 64 * h;
        if (c < 16 * NB) bv[c] = c < K ? alpha * bs[h] + Lmu[c] : 0.f;
    }
    wave_sync();
    blocked_chol_sample<NB>(acc, lds, K, alpha, img, (uint32_t)f.row, ctr[0], seed, stream,
                            X + (size_t)f.row * ldx, status);
}

// The prior Lambda (identity on the padding) in the accumulator layout of
// the upper blocks: block q = i (i + 1) / 2 + j (i >= j), lane l, value v
// holds Lambda[16 j + 4 (l / 16) + v][16 i + l % 16].
template <int NB>
__global__ __launch_bounds__(256) void prior_image(int K, const float *__restrict__ Lam, float *__restrict__ img)
{
    const int e = blockIdx.x * 256 + threadIdx.x;  // ((q * 64) + l) * 4 + v
    if (e >= NB * (NB + 1) / 2 * 256) return;
    const int v = e & 3, l = (e >> 2) & 63, q = e >> 8;
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= q) ++i;
    const int j = q - i * (i + 1) / 2;
    const int r = 16 * j + 4 * (l >> 4) + v, cc = 16 * i + (l & 15);
    img[e] = (r < K && cc < K) ? Lam[r * K + cc] : (r == cc ? 1.f : 0.f);
}

template <int NB>
hipError_t launch_big(bpmf_ctx *c, Side &sd, Side &ot, hipStream_t s, int stage)
{
    const size_t lds = sizeof(float) * kBigWPB * BigLds<NB>::TOTAL;
    const floatx4 *img = (const floatx4 *)sd.Lam_img;
    if (stage == kStagePrior) {
        // the prior image of this sweep (read by the whole rows and the finishing)
        hipLaunchKernelGGL((prior_image<NB>), dim3((NB * (NB + 1) / 2 * 256 + 255) / 256), dim3(256), 0, s,
                           c->K, (const float *)sd.Lam_w, sd.Lam_img);
        return hipGetLastError();
    }
    if (stage == kStageFinish) {
        if (sd.n_fin == 0) return hipSuccess;
        // up to K = 64 the slots are summed first by one thread per entry and
        // row (the same order as the finishing's own sum), so that a row with
        // many segments does not leave one wavefront streaming all its slots;
        // above, the finishing's own float4 sum measured faster
        constexpr bool summed = NB <= 4;
        if constexpr (summed) {
            const hipError_t e = launch_part_reduce(c, sd, s, big_slot_elems<NB>());
            if (e != hipSuccess) return e;
        }
        const unsigned grid = (unsigned)((sd.n_fin + kBigWPB - 1) / kBigWPB);
        hipLaunchKernelGGL((row_finish_big<NB>), dim3(grid), dim3(64 * kBigWPB), lds, s, c->K,
                           (float)c->alpha, sd.fin, sd.n_fin, (const float *)c->part, img,
                           (const float *)sd.Lmu_w, (float *)sd.X, c->ld, c->seed, sd.stream_row,
                           c->ctr, c->hyp_status + 1, summed ? 1 : 0);
        return hipGetLastError();
    }
    if (stage != kStageSegments && stage != kStageRows) return hipSuccess;
    // segments of split rows are items [0, n_slots), whole rows follow
    const int64_t n_seg = sd.n_slots, n_rows = sd.n_items - sd.n_slots - sd.n_low;
    const bool bf = c->prec == 2;
    const void *ysrc = bf ? (const void *)ot.Xbf : (const void *)ot.X;
    const uint32_t y_bytes = (uint32_t)(ot.rows * c->ld * (bf ? 2 : 4));
    // the rhs from the Gram where the padding has room for the rating
    const int kr = c->K - 16 * (NB - 1);
    const bool aug = kr <= 13 && sd.rc3 != nullptr;
    auto go = [&](auto kern, int64_t item0, int64_t count, size_t lds_bytes) {
        if (count <= 0) return;
        const unsigned grid = (unsigned)((count + kBigWPB - 1) / kBigWPB);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * kBigWPB), lds_bytes, s, c->K,
                           (float)c->alpha, sd.items, item0, item0 + count, sd.nbr,
                           (const float *)sd.rc, (const uint16_t *)sd.rc3, (uint32_t)(c->nnz + 32), ysrc,
                           c->ld, y_bytes, img, (const float *)sd.Lmu_w, (float *)sd.X, c->ld,
                           (float *)c->part, c->seed, sd.stream_row, c->ctr, c->hyp_status + 1);
    };
    auto pick = [&](auto segc) {
        constexpr bool SEG = decltype(segc)::value;
        const int64_t item0 = SEG ? 0 : n_seg, count = SEG ? n_seg : n_rows;
        const size_t bytes = SEG ? 0 : lds;
        if (bf) {
            if (aug)
                go(row_big<NB, true, SEG, true>, item0, count, bytes);
            else
                go(row_big<NB, true, SEG, false>, item0, count, bytes);
        } else {
            if (aug)
                go(row_big<NB, false, SEG, true>, item0, count, bytes);
            else
                go(row_big<NB, false, SEG, false>, item0, count, bytes);
        }
    };
    if (stage == kStageSegments)
        pick(std::integral_constant<bool, true>{});
    else
        pick(std::integral_constant<bool, false>{});
    return hipGetLastError();
}

}  // namespace

// FP32 factors with 32 < K <= 128 or BF16-Gram factors with K <= 128, and
// 32-bit buffer offsets.
bool big_path_available(const bpmf_ctx *c)
{
    if (c->prec == 0 || c->K > 128) return false;
    if (c->prec == 1 && c->K <= c->fast_kmax && c->K <= 64) return false;  // column-per-lane kernel
    for (int s = 0; s < 2; ++s)
        if ((uint64_t)c->side[s].rows * c->ld * sizeof(float) >= kOOB || c->side[s].rows >= (1 << 24))
            return false;  // 32-bit buffer offsets, 24-bit row ids in the gather
    return (uint64_t)c->split_threshold * 4u < kOOB;
}

int64_t part_slot_elems(const bpmf_ctx *c)
{
    if (big_path_available(c)) {
        const int64_t nb = (c->K + 15) / 16;
        return nb * (nb + 1) / 2 * 256 + 16 * nb;
    }
    return (int64_t)c->K * (c->K + 1) / 2 + c->K;
}

hipError_t launch_row_big(bpmf_ctx *c, int side_id, hipStream_t s, int stage, bool *handled)
{
    *handled = false;
    if (!big_path_available(c)) return hipSuccess;
    *handled = true;
    Side &sd = c->side[side_id];
    Side &ot = c->side[1 - side_id];
    switch ((c->K + 15) / 16) {
    case 1: return launch_big<1>(c, sd, ot, s, stage);
    case 2: return launch_big<2>(c, sd, ot, s, stage);
    case 3: return launch_big<3>(c, sd, ot, s, stage);
    case 4: return launch_big<4>(c, sd, ot, s, stage);
    case 5: return launch_big<5>(c, sd, ot, s, stage);
    case 6: return launch_big<6>(c, sd, ot, s, stage);
    case 7: return launch_big<7>(c, sd, ot, s, stage);
    default: return launch_big<8>(c, sd, ot, s, stage);
    }
}

}  // namespace bpmf
