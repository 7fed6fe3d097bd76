// row_fast.hip -- matrix-core row update for FP32 factors, K <= 64.
//
// One wavefront per work item (a whole row, or a segment of a split row).
// Per row (Algorithm 1's item body with BPMF's conditional):
//   P = Lambda + alpha sum_j y_j y_j^T,  b = Lambda mu + alpha sum_j r'_j y_j,
//   P = L L^T,  y = L^-1 b,  x = L^-T (y + z).
//
// Gram: the neighbour rows are gathered straight from HBM/L2 into the
// operand registers of v_mfma_f32_16x16x4_f32 -- lane l holds component
// 16*bi + (l % 16) of the neighbour row of rating 4g + l / 16, which is at
// once the A operand of block row bi and the B operand of block column bj --
// so only the nb(nb+1)/2 lower 16x16 blocks of P are accumulated (nb =
// ceil(K/16)), four ratings per instruction.  The rhs accumulates on the
// VALU from the same registers.
//
// Cholesky: the accumulators go through LDS into a column-per-lane layout
// (lane c holds column c of P, plus b as an extra row).  Right-looking
// elimination without the square roots: at step k every lane c > k updates
// its column with the pivot column broadcast by v_readlane, so the pivot
// row/column never needs rescaling; the extra row carries b through the
// elimination, which is the forward solve L^-1 b.  Each lane finally scales
// its column by 1/sqrt(d_c); the back solve runs row by row with one
// readlane per row.
//
// Noise: lane c draws normal c of the row (Philox4x32-10 block c/4) with a
// Box-Muller evaluated in FP32 (the log of u close to 1 is taken as
// log1p(-(1-u)) so that no bits are lost).
#include "internal.h"
#include "rng_device.h"

namespace bpmf {

hipError_t prepare_hyper(bpmf_ctx *c);
hipError_t launch_row_generic(bpmf_ctx *c, int side_id, hipStream_t s, int stage);

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kUnroll = 8;  // groups of 4 ratings in flight per wave

__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }

// Value of x in lane `src` (a compile-time constant), bit-exact.
__device__ __forceinline__ float readlane_f(float x, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}

// Standard normal from Philox words: the pair (wr, wa) gives radius and
// angle; `sine` picks the sine branch.  FP32 evaluation.
__device__ __forceinline__ float bm_normal_f32(uint32_t wr, uint32_t wa, bool sine)
{
    float lnu;
    if (wr < 0x80000000u) {
        float u = ((float)wr + 0.5f) * 2.3283064365386963e-10f;
        lnu = logf(u);
    } else {
        float v = ((float)(0xFFFFFFFFu - wr) + 0.5f) * 2.3283064365386963e-10f;  // 1 - u
        lnu = log1pf(-v);
    }
    float rho = sqrtf(-2.0f * lnu);
    float ua = ((float)wa + 0.5f) * 2.3283064365386963e-10f;
    float sv, cv;
    sincospif(2.0f * ua, &sv, &cv);
    return rho * (sine ? sv : cv);
}

template <int NB, int WPB>
__global__ __launch_bounds__(64 * WPB) void row_fast_f32(
    int K, float alpha, const RowItem *__restrict__ items, int64_t n_items,
    const int32_t *__restrict__ nbr, const float *__restrict__ rc, const float *__restrict__ Y,
    int ldy, const float *__restrict__ Lam, const float *__restrict__ Lmu, float *__restrict__ X,
    int ldx, float *__restrict__ part, uint64_t seed, uint32_t stream,
    const uint32_t *__restrict__ ctr)
{
    constexpr int KP = 16 * NB;
    constexpr int LDP = KP + 1;
    constexpr int NBLK = NB * (NB + 1) / 2;
    extern __shared__ float smem_f[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t item_id = (int64_t)blockIdx.x * WPB + wave;
    if (item_id >= n_items) return;
    float *Ps = smem_f + wave * (KP * LDP + KP);
    float *bs = Ps + KP * LDP;
    const RowItem it = items[item_id];
    const int col = lane & 15;
    const int kq = lane >> 4;

    floatx4 acc[NBLK];
#pragma unroll
    for (int q = 0; q < NBLK; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    float bacc[NB];
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) bacc[bi] = 0.f;

    for (int64_t base = it.beg; base < it.end; base += 4 * kUnroll) {
        float yv[kUnroll][NB];
        float rv[kUnroll];
#pragma unroll
        for (int g = 0; g < kUnroll; ++g) {
            const int64_t t = base + 4 * g + kq;
            const bool ok = t < it.end;
            const int j = ok ? nbr[t] : 0;
            rv[g] = ok ? rc[t] : 0.f;
            const float *yrow = Y + (size_t)j * ldy;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) {
                const int comp = 16 * bi + col;
                yv[g][bi] = (ok && comp < K) ? yrow[comp] : 0.f;
            }
        }
#pragma unroll
        for (int g = 0; g < kUnroll; ++g) {
            int q = 0;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
                for (int bj = 0; bj <= bi; ++bj) {
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(yv[g][bi], yv[g][bj], acc[q], 0, 0, 0);
                    ++q;
                }
                bacc[bi] += rv[g] * yv[g][bi];
            }
        }
    }
    // sum the rhs over the four rating slots of each 16-lane column
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
        bacc[bi] += __shfl_xor(bacc[bi], 16);
        bacc[bi] += __shfl_xor(bacc[bi], 32);
    }

    const int KK2 = K * (K + 1) / 2;
    if (it.slot >= 0) {  // segment of a split row: write the raw partial sums
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

    // accumulators -> symmetric P in this wave's LDS
    {
        int q = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
            for (int bj = 0; bj <= bi; ++bj) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * bi + 4 * kq + v, c = 16 * bj + col;
                    Ps[r * LDP + c] = acc[q][v];
                    if (bi != bj) Ps[c * LDP + r] = acc[q][v];
                }
                ++q;
            }
            if (kq == 0) bs[16 * bi + col] = bacc[bi];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // column-per-lane: v[r] = P[r][c] (r < KP), v[KP] = b_c; padding is identity
    const int c = lane;
    const bool live = c < K;
    float v[KP + 1];
#pragma unroll
    for (int r = 0; r < KP; ++r) {
        float p = (c < KP) ? Ps[r * LDP + (c < KP ? c : 0)] : 0.f;
        v[r] = (live && r < K) ? alpha * p + Lam[r * K + c] : (r == c ? 1.f : 0.f);
    }
    v[KP] = live ? alpha * bs[c] + Lmu[c] : 0.f;

    float mydiag = 1.f;
#pragma unroll
    for (int k = 0; k < KP; ++k) {  // padded columns are identity: their steps change nothing
        const float dk = readlane_f(v[k], k);
        if (c == k) mydiag = dk;
        const float f = v[k] * __builtin_amdgcn_rcpf(dk);
        const bool upd = c > k;
#pragma unroll
        for (int r = k + 1; r <= KP; ++r) {
            const float prk = readlane_f(v[r], k);
            if (upd) v[r] -= f * prk;
        }
    }
    const float inv_s = __builtin_amdgcn_rsqf(mydiag);
#pragma unroll
    for (int r = 0; r < KP; ++r) v[r] *= inv_s;  // column c of L (rows > c)

    // w = L^-1 b + z
    float w = v[KP] * inv_s;
    {
        const uint32_t t = ctr[0];
        const uint32_t blk = (uint32_t)(c >> 2);
        const Block4 bl = philox4x32_10((uint32_t)it.row, t, (stream << 24) | blk, 0u, seed);
        const int m = c & 3;
        const uint32_t wr = m < 2 ? bl.w0 : bl.w2;
        const uint32_t wa = m < 2 ? bl.w1 : bl.w3;
        if (live) w += bm_normal_f32(wr, wa, (m & 1) != 0);
    }
    // x = L^-T w, rows from the last
    float accx = 0.f, myx = 0.f;
#pragma unroll
    for (int r = KP - 1; r >= 0; --r) {  // padded rows carry w = 0, x = 0
        const float xr_all = (w - accx) * inv_s;
        const float xr = readlane_f(xr_all, r);
        if (c == r) myx = xr;
        if (c < r) accx += v[r] * xr;
    }
    if (live) X[(size_t)it.row * ldx + c] = myx;
}

template <int NB, int WPB>
hipError_t launch_f32(bpmf_ctx *c, Side &sd, Side &ot, hipStream_t s)
{
    constexpr int KP = 16 * NB;
    const size_t lds = sizeof(float) * WPB * (KP * (KP + 1) + KP);
    const unsigned grid = (unsigned)((sd.n_items + WPB - 1) / WPB);
    hipLaunchKernelGGL((row_fast_f32<NB, WPB>), dim3(grid), dim3(64 * WPB), lds, s, c->K,
                       (float)c->alpha, sd.items, sd.n_items, sd.nbr, (const float *)sd.rc,
                       (const float *)ot.X, c->ld, (const float *)sd.Lam_w,
                       (const float *)sd.Lmu_w, (float *)sd.X, c->ld, (float *)c->part, c->seed,
                       sd.stream_row, c->ctr);
    return hipGetLastError();
}

}  // namespace

bool fast_path_available(const bpmf_ctx *c) { return c->prec == 1 && c->K <= 64; }

hipError_t launch_row_fast(bpmf_ctx *c, int side_id, hipStream_t s, int stage, bool *handled)
{
    *handled = false;
    if (!fast_path_available(c)) return hipSuccess;
    *handled = true;
    Side &sd = c->side[side_id];
    Side &ot = c->side[1 - side_id];
    if (stage == 1) return launch_row_generic(c, side_id, s, 1);  // split-row finish
    if (sd.n_items == 0) return hipSuccess;
    const int nb = (c->K + 15) / 16;
    switch (nb) {
    case 1: return launch_f32<1, 4>(c, sd, ot, s);
    case 2: return launch_f32<2, 4>(c, sd, ot, s);
    case 3: return launch_f32<3, 2>(c, sd, ot, s);
    default: return launch_f32<4, 2>(c, sd, ot, s);
    }
}

hipError_t prepare_kernels(bpmf_ctx *c) { return prepare_hyper(c); }

}  // namespace bpmf
