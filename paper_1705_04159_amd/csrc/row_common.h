// row_common.h -- device helpers shared by the matrix-core row kernels.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>


#include "internal.h"
#include "rng_device.h"

namespace bpmf {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kOOB = 0x40000000u;  // offset beyond every buffer read here

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Two FP32 values as three BF16 parts each, x = h + m + l exactly (round to
// nearest even at every step: h keeps the top 8 significant bits, m the
// next 8 of the remainder, and the remainder after that has at most 8, so
// l holds it exactly): |m| <= 2^-8 |x| (1 + 2^-8), |l| <= 2^-15 |x|.  The
// parts of the pair come back packed as the two halves of h, m and l.
__device__ __forceinline__ void split3(float x0, float x1, uint32_t &h, uint32_t &m, uint32_t &l)
{
    const floatx2 x = floatx2{x0, x1};
    const bf16x2 hb = __builtin_convertvector(x, bf16x2);
    const floatx2 r = x - __builtin_convertvector(hb, floatx2);
    const bf16x2 mb = __builtin_convertvector(r, bf16x2);
    const floatx2 t = r - __builtin_convertvector(mb, floatx2);
    const bf16x2 lb = __builtin_convertvector(t, bf16x2);
    h = __builtin_bit_cast(uint32_t, hb);
    m = __builtin_bit_cast(uint32_t, mb);
    l = __builtin_bit_cast(uint32_t, lb);
}


template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }

__device__ __forceinline__ float readlane_f(float x, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}

// x from lane k of the caller's lane group (the whole wave for RPW = 1,
// 32 lanes for RPW = 2, 16 lanes for RPW = 4).
template <int RPW, int k>
__device__ __forceinline__ float bcast(float x)
{
    if constexpr (RPW == 1)
        return readlane_f(x, k);
    else if constexpr (RPW == 2)
        return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), k << 5));
    else
        return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x10 | (k << 5)));
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ uint32_t buf_u32(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
}

__device__ __forceinline__ float buf_f32(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __uint_as_float(buf_u32(r, off));
}

// Loads of data read once per sweep (neighbour ids, ratings), marked
// non-temporal (cache policy NT) so that they do not push the gathered
// factor rows, which every row re-reads, out of the L2.
constexpr int kStreamPolicy = 2;
__device__ __forceinline__ uint32_t buf_u32_stream(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, kStreamPolicy);
}

__device__ __forceinline__ float buf_f32_stream(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __uint_as_float(buf_u32_stream(r, off));
}

// x += f * (x of lane L of the same 16-lane row), one fused DPP multiply-add
// per value (v_fmac_f32 with row_newbcast:L on its first source).  The
// compiler does not fold its own DPP moves into v_fmac, so these are written
// out; each group starts with two wait states, which covers the VALU-write
// -> DPP-read hazard of a value written just before, and the values of a
// group are distinct registers, so none is read through DPP right after
// being written inside the group.
#define BPMF_FMAC_BC(i) "v_fmac_f32_dpp %" #i ", %" #i ", %[f] row_newbcast:%[l] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
template <int L>
__device__ __forceinline__ void fmac_bc1(float &a, float f)
{
    asm("s_nop 1\n\t" BPMF_FMAC_BC(0) : "+v"(a) : [f] "v"(f), [l] "n"(L));
}
template <int L>
__device__ __forceinline__ void fmac_bc2(float &a, float &b, float f)
{
    asm("s_nop 1\n\t" BPMF_FMAC_BC(0) BPMF_FMAC_BC(1) : "+v"(a), "+v"(b) : [f] "v"(f), [l] "n"(L));
}
template <int L>
__device__ __forceinline__ void fmac_bc3(float &a, float &b, float &c, float f)
{
    asm("s_nop 1\n\t" BPMF_FMAC_BC(0) BPMF_FMAC_BC(1) BPMF_FMAC_BC(2)
        : "+v"(a), "+v"(b), "+v"(c) : [f] "v"(f), [l] "n"(L));
}
template <int L>
__device__ __forceinline__ void fmac_bc4(float &a, float &b, float &c, float &d, float f)
{
    asm("s_nop 1\n\t" BPMF_FMAC_BC(0) BPMF_FMAC_BC(1) BPMF_FMAC_BC(2) BPMF_FMAC_BC(3)
        : "+v"(a), "+v"(b), "+v"(c), "+v"(d) : [f] "v"(f), [l] "n"(L));
}
#undef BPMF_FMAC_BC

// fmac_bc over x[B], x[B+1], ..., x[E-1] in groups of four.
template <int L, int B, int E, int N>
__device__ __forceinline__ void fmac_bc_range(float (&x)[N], float f)
{
    if constexpr (E - B >= 4) {
        fmac_bc4<L>(x[B], x[B + 1], x[B + 2], x[B + 3], f);
        fmac_bc_range<L, B + 4, E>(x, f);
    } else if constexpr (E - B == 3) {
        fmac_bc3<L>(x[B], x[B + 1], x[B + 2], f);
    } else if constexpr (E - B == 2) {
        fmac_bc2<L>(x[B], x[B + 1], f);
    } else if constexpr (E - B == 1) {
        fmac_bc1<L>(x[B], f);
    }
}

// Broadcast lane L of each 16-lane row to the whole row (DPP row_newbcast:
// a VALU move, no scalar round trip).
template <int L>
__device__ __forceinline__ float bcast16(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x150 + L, 0xf, 0xf, true));
}

// Box-Muller on Philox words: the pair (wr, wa) gives radius and angle, and
// both normals of the pair (cosine and sine branch).  FP32 evaluation.
__device__ __forceinline__ void bm_pair_f32(uint32_t wr, uint32_t wa, float &zc, float &zs)
{
    float lnu;
    if (wr < 0x80000000u) {
        const float u = ((float)wr + 0.5f) * 2.3283064365386963e-10f;
        lnu = logf(u);
    } else {
        const float v = ((float)(0xFFFFFFFFu - wr) + 0.5f) * 2.3283064365386963e-10f;  // 1 - u
        lnu = log1pf(-v);
    }
    const float rho = sqrtf(-2.0f * lnu);
    const float ua = ((float)wa + 0.5f) * 2.3283064365386963e-10f;
    float sv, cv;
    sincospif(2.0f * ua, &sv, &cv);
    zc = rho * cv;
    zs = rho * sv;
}

// One standard normal: `sine` picks the branch.
__device__ __forceinline__ float bm_normal_f32(uint32_t wr, uint32_t wa, bool sine)
{
    float zc, zs;
    bm_pair_f32(wr, wa, zc, zs);
    return sine ? zs : zc;
}

// The four normals of one Philox block: components 4 blk + m take the
// cosine (m even) and sine (m odd) of the pairs (w0, w1) for m < 2 and
// (w2, w3) otherwise -- the same values as bm_normal_f32 per component.
__device__ __forceinline__ void bm_normal4_f32(const Block4 &bl, float (&z)[4])
{
    bm_pair_f32(bl.w0, bl.w1, z[0], z[1]);
    bm_pair_f32(bl.w2, bl.w3, z[2], z[3]);
}

// Gram and rhs of one work item (whole wave), FP32 rows on
// v_mfma_f32_16x16x4_f32, with ids and rows loaded per group of four
// ratings: lane l holds component 16*bi + (l % 16)
// of the neighbour row of rating 4g + l / 16, which is both the A operand of
// block row bi and the B operand of block column bj.  Software-pipelined:
// ids of chunk c+2 and rows of chunk c+1 are in flight while chunk c is
// multiplied.  Ratings past the end read as 0 (buffer range check); only the
// last chunk of an item checks for them.  Row offsets use the full-rate
// 24-bit multiply (the gathered factor has fewer than 2^24 rows).  With
// PADOK the caller ignores every Gram and rhs entry outside the leading
// K x K block, so all blocks load at immediate offsets from one address
// (components >= K then hold whatever follows the row); otherwise
// components >= K read as 0 through lane_off.  With TRANS the blocks are
// accumulated transposed: block (bi, bj), bi >= bj, holds the upper block
// (bj, bi) of the Gram in the MFMA result layout.
template <int NB, int kUnroll, bool PADOK, bool TRANS = false>
__device__ __forceinline__ void gram_item_pipe(const RowItem &it, const int32_t *__restrict__ nbr,
                                          const float *__restrict__ rc,
                                          __amdgpu_buffer_rsrc_t ysrc, uint32_t ldy4,
                                          const uint32_t (&lane_off)[NB], int kq,
                                          floatx4 (&acc)[NB * (NB + 1) / 2], float (&bacc)[NB])
{
    const uint32_t cnt = (uint32_t)(it.end - it.beg);
    const __amdgpu_buffer_rsrc_t jsrc = make_rsrc(nbr + it.beg, cnt * 4u);
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(rc + it.beg, cnt * 4u);
    constexpr int kChunk = 4 * kUnroll;
    const uint32_t nchunk = (cnt + kChunk - 1) / kChunk;
    uint32_t jb[2][kUnroll];
    float yb[2][kUnroll][NB];
    float rb[2][kUnroll];
    auto load_ids = [&](int buf, uint32_t ch) {
#pragma unroll
        for (int g = 0; g < kUnroll; ++g) jb[buf][g] = buf_u32_stream(jsrc, (ch * kChunk + 4 * g + kq) * 4u);
    };
    auto load_rows_t = [&](int buf, uint32_t ch, auto checkc) {
        constexpr bool CHECK = decltype(checkc)::value;
#pragma unroll
        for (int g = 0; g < kUnroll; ++g) {
            const uint32_t t = ch * kChunk + 4 * g + kq;
            rb[buf][g] = buf_f32_stream(rsrc, t * 4u);  // 0 past the end
            uint32_t base = __umul24(jb[buf][g], ldy4);
            if constexpr (CHECK) base = t < cnt ? base : kOOB;
            if constexpr (PADOK) {
                const uint32_t a = base + lane_off[0];
#pragma unroll
                for (int bi = 0; bi < NB; ++bi) yb[buf][g][bi] = buf_f32(ysrc, a + 64u * bi);
            } else {
#pragma unroll
                for (int bi = 0; bi < NB; ++bi) yb[buf][g][bi] = buf_f32(ysrc, base + lane_off[bi]);
            }
        }
    };
    // only the last chunk (and the prefetch past it) can hold ratings past the end
    auto load_rows = [&](int buf, uint32_t ch) {
        if (ch + 1 < nchunk)
            load_rows_t(buf, ch, std::integral_constant<bool, false>{});
        else
            load_rows_t(buf, ch, std::integral_constant<bool, true>{});
    };
    auto compute = [&](int buf) {
#pragma unroll
        for (int g = 0; g < kUnroll; ++g) {
            int q = 0;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
                for (int bj = 0; bj <= bi; ++bj) {
                    if constexpr (TRANS)
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(yb[buf][g][bj], yb[buf][g][bi], acc[q], 0, 0, 0);
                    else
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(yb[buf][g][bi], yb[buf][g][bj], acc[q], 0, 0, 0);
                    ++q;
                }
                bacc[bi] += rb[buf][g] * yb[buf][g][bi];
            }
        }
    };
    if (nchunk == 0) return;
    load_ids(0, 0);
    load_ids(1, 1);
    load_rows(0, 0);
    for (uint32_t ch = 0; ch < nchunk; ch += 2) {
        load_ids(0, ch + 2);
        load_rows(1, ch + 1);
        compute(0);
        if (ch + 1 >= nchunk) break;
        load_ids(1, ch + 3);
        load_rows(0, ch + 2);
        compute(1);
    }
}

// Gram and rhs of one work item into the accumulators (whole wave): the
// pipelined per-group form, four groups (16 ratings) per stage for rows of
// up to 32 components and two for wider rows (register budget).
template <int NB, bool PADOK = false, bool TRANS = false>
__device__ __forceinline__ void gram_item(const RowItem &it, const int32_t *__restrict__ nbr,
                                          const float *__restrict__ rc,
                                          __amdgpu_buffer_rsrc_t ysrc, uint32_t ldy4,
                                          const uint32_t (&lane_off)[NB], int kq,
                                          floatx4 (&acc)[NB * (NB + 1) / 2], float (&bacc)[NB])
{
    gram_item_pipe<NB, (NB <= 2 ? 4 : 2), PADOK, TRANS>(it, nbr, rc, ysrc, ldy4, lane_off, kq, acc, bacc);
}

}  // namespace
}  // namespace bpmf
