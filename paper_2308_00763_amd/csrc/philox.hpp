// Counter-based random numbers for the particle filter: Philox4x32-10
// (Salmon, Moraes, Dror, Shaw, SC'11) and the Box-Muller transform.
//
// The paper draws its normals in double and converts them to the working
// precision (Sec. 4, after Eq. (2)); the same seed is used by every precision
// (Sec. 5).  Here every particle k at step t owns the counter
// (k, t, stream_id, 0) and the step's resampling offset owns
// (0, t, stream_id, 1), so each draw is a pure function of its counter and
// no generator state is stored.  The double mode builds two 53-bit uniforms
// from the four words; the reduced modes take the top 24 bits of the same
// words, so every precision sees the same random stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pf {

struct u32x4 {
    uint32_t v0, v1, v2, v3;
};

// Three-way exclusive or in one gfx950 instruction (v_bitop3_b32 with the
// truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Ten rounds; each multiplies two counter words by the Philox constants,
// swaps the halves and mixes in the round key, which advances by the Weyl
// increments (0x9E3779B9, 0xBB67AE85) between rounds.  The key words are
// uniform across the wave, so their updates stay scalar; per round and lane
// the work is two 32x32->64 multiplies and two three-way exclusive ors.
__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n1 = (uint32_t)p1;
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        const uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return u32x4{c0, c1, c2, c3};
}

// 53-bit uniform in [0, 1) from (hi, lo): hi's 32 bits then lo's top 21.
__device__ __forceinline__ double uniform53(uint32_t hi, uint32_t lo)
{
    const uint64_t bits = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
    return (double)bits * 0x1.0p-53;
}

// Box-Muller in double (Box & Muller 1958): rho = sqrt(-2 ln(1 - u_a)),
// (z_x, z_y) = rho (cos 2 pi u_b, sin 2 pi u_b).  Written operation by
// operation; the library is compiled without contraction so each product
// and sum rounds separately.
__device__ __forceinline__ void normal_pair_f64(const u32x4& w, double& zx, double& zy)
{
    const double ua = uniform53(w.v0, w.v1);
    const double ub = uniform53(w.v2, w.v3);
    const double rho = sqrt(-2.0 * log(1.0 - ua));
    const double ang = 6.283185307179586 * ub;
    double s, c;
    sincos(ang, &s, &c);
    zx = rho * c;
    zy = rho * s;
}

// Box-Muller in float from the top 24 bits of the same words.  Uses the
// hardware transcendental instructions: log2, square root, and sine/cosine
// whose argument is in revolutions (so sin(2 pi u) is sin_rev(u) with no
// multiply by 2 pi).  1 - u_a lies in [2^-24, 1], so the logarithm is finite.
__device__ __forceinline__ void normal_pair_f32(const u32x4& w, float& zx, float& zy)
{
    const float ua = (float)(w.v0 >> 8) * 0x1.0p-24f;
    const float ub = (float)(w.v2 >> 8) * 0x1.0p-24f;
    // -2 ln(1 - u) = -2 ln(2) log2(1 - u)
    const float l2 = __builtin_amdgcn_logf(1.0f - ua);
    const float rho = __builtin_amdgcn_sqrtf(-1.3862943611198906f * l2);
    zx = rho * __builtin_amdgcn_cosf(ub);
    zy = rho * __builtin_amdgcn_sinf(ub);
}

}  // namespace pf
