// Stochastic rounding of the 16-bit storage formats: the rounding itself and
// the counter-based random bytes it uses.  Host and device share this code
// (the library's diagnostics call it on the host).
//
// Rounding to nearest stores a slowly varying value with the same error step
// after step; on fine grids the change of a DF per step falls below half an
// FP16 unit in the last place, and these errors add up to a bias of the heat
// flux that grows with the grid.  The 16-bit rows are therefore rounded
// stochastically, with one random byte per stored value drawn from a hash of
// the node's column and row, the step counter and the value's index among
// the format's 16-bit rows (FP16S: f rows 0-8, g rows 9-17; FP32 f + FP16 g:
// g rows 0-8).  The bytes depend on nothing else, so every launch
// configuration, graph replays and the copies of a column store the same
// bits.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

// FP32 value rounded stochastically to the FP16 grid, u a uniform random
// byte.  Adding (u + 1/2)/256 of an FP16 unit in the last place to the
// magnitude and cutting the FP32 mantissa to FP16's 10 bits rounds up with
// probability equal to the cut fraction (to 1/512), so the stored value is
// unbiased; the result is exact in FP16 and converts without a second
// rounding (FP16 subnormals, below 6.1e-5, round to nearest once more).
__host__ __device__ inline float round_stochastic_half(float v, unsigned u)
{
    const unsigned b = __builtin_bit_cast(unsigned, v);
    return __builtin_bit_cast(float, (b + (u << 5) + 16u) & 0xFFFFE000u);
}

namespace sr {
__host__ __device__ inline unsigned seed_x(int x) { return unsigned(x) * 0x9E3779B1u; }
__host__ __device__ inline unsigned seed_yt(int y, unsigned t) { return unsigned(y) * 0x85EBCA77u ^ t * 0xC2B2AE3Du; }
// integer finaliser (xor-shift / multiply rounds) of the combined seed
__host__ __device__ inline unsigned mix(unsigned h)
{
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    return h;
}
// Marsaglia's xorshift32 step (13, 17, 5)
__host__ __device__ inline unsigned xorshift(unsigned w)
{
    w ^= w << 13;
    w ^= w >> 17;
    w ^= w << 5;
    return w;
}
// random byte i of a node with mixed seed h: byte i % 4 of word i / 4, where
// word 0 is h and word k + 1 the xorshift32 step of word k (every byte of
// every word is uniform)
__host__ __device__ inline unsigned byte(unsigned h, int i)
{
    for (int k = 0; k < (i >> 2); ++k) h = xorshift(h);
    return (h >> (8 * (i & 3))) & 0xFFu;
}
// random byte i of the node (x, y) (wrapped on a periodic axis) in step t
__host__ __device__ inline unsigned byte_at(int x, int y, unsigned t, int i)
{
    return byte(mix(seed_x(x) ^ seed_yt(y, t)), i);
}
}  // namespace sr

}  // namespace lbm
