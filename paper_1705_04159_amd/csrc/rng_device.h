// rng_device.h -- counter-based noise for the device kernels.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64-bit multiplications
// by 0xD2511F53 / 0xCD9E8D57 with XOR mixing; the 64-bit key is bumped by
// the Weyl constants 0x9E3779B9 / 0xBB67AE85 between rounds.  Normals come
// from the Box-Muller transform of (w + 1/2) 2^-32, evaluated in FP64;
// chi-square variates from Marsaglia & Tsang's gamma method (ACM TOMS 2000).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bpmf {

// Philox stream ids (counter word 2 = stream << 24 | sub-block).
enum : uint32_t {
    kStreamRowU = 1,
    kStreamRowV = 2,
    kStreamHypU = 3,
    kStreamHypV = 4,
    kStreamInitU = 5,
    kStreamInitV = 6,
    kStreamFoldin = 7,
};

struct Block4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Block4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint64_t seed)
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a = 0xD2511F53u, b = 0xCD9E8D57u;
        uint32_t hi_a = __umulhi(a, c0), lo_a = a * c0;
        uint32_t hi_b = __umulhi(b, c2), lo_b = b * c2;
        uint32_t n0 = hi_b ^ c1 ^ k0;
        uint32_t n2 = hi_a ^ c3 ^ k1;
        c0 = n0;
        c1 = lo_b;
        c2 = n2;
        c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Block4{c0, c1, c2, c3};
}

__device__ __forceinline__ double open_unit(uint32_t w)
{
    return ((double)w + 0.5) * 2.3283064365386962890625e-10;  // 2^-32
}

// Four standard normals from one block: (w0, w1) -> (cos, sin) pair,
// (w2, w3) -> (cos, sin) pair.
__device__ __forceinline__ void box_muller(const Block4 &b, double z[4])
{
    const double two_pi = 6.283185307179586476925286766559;
    double ra = sqrt(-2.0 * log(open_unit(b.w0)));
    double rb = sqrt(-2.0 * log(open_unit(b.w2)));
    double sa, ca, sb, cb;
    sincos(two_pi * open_unit(b.w1), &sa, &ca);
    sincos(two_pi * open_unit(b.w3), &sb, &cb);
    z[0] = ra * ca;
    z[1] = ra * sa;
    z[2] = rb * cb;
    z[3] = rb * sb;
}

// Normal k of the sequence keyed by (c0, c1, stream, c3): block k/4, lane k%4.
__device__ __forceinline__ void normals_block(uint64_t seed, uint32_t c0, uint32_t c1,
                                              uint32_t stream, uint32_t blk, uint32_t c3,
                                              double z[4])
{
    Block4 b = philox4x32_10(c0, c1, (stream << 24) | blk, c3, seed);
    box_muller(b, z);
}

// Chi-square(dof) = 2 Gamma(dof/2, 1) by Marsaglia-Tsang; attempt j uses the
// block with counter (index, t, stream<<24 | 0, j): normal from the cosine
// branch of (w0, w1), uniform from w2.  Shapes here are >= 1.  The loop is
// capped; `ok` is cleared if the cap is reached (acceptance is > 95% per
// attempt, so the cap is never reached in practice).
__device__ inline double chi_square(uint64_t seed, uint32_t stream, uint32_t t, uint32_t index,
                                    double dof, int *ok)
{
    const double two_pi = 6.283185307179586476925286766559;
    double d = 0.5 * dof - 1.0 / 3.0;
    double c = 1.0 / sqrt(9.0 * d);
    for (uint32_t attempt = 0; attempt < 4096u; ++attempt) {
        Block4 b = philox4x32_10(index, t, (stream << 24) | 0u, attempt, seed);
        double x = sqrt(-2.0 * log(open_unit(b.w0))) * cos(two_pi * open_unit(b.w1));
        double u = open_unit(b.w2);
        double v = 1.0 + c * x;
        if (v <= 0.0) continue;
        v = v * v * v;
        if (log(u) < 0.5 * x * x + d - d * v + d * log(v)) return 2.0 * d * v;
    }
    *ok = 0;
    return dof;
}

}  // namespace bpmf
