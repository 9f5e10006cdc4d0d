// Stochastic rounding of the 16-bit storage formats: the counter-based
// random operands and a host model of the rounding.  Host and device share
// the random-number code (the library's diagnostics call it on the host).
//
// Rounding to nearest stores a slowly varying value with the same error step
// after step; on fine grids the change of a DF per step falls below half an
// FP16 unit in the last place, and these errors add up to a bias of the heat
// flux that grows with the grid.  The 16-bit rows are therefore rounded
// stochastically: gfx950's v_cvt_sr_f16_f32 adds a 32-bit random operand to
// the discarded part of the FP32 value, aligned to the operand's top bit, and
// rounds the magnitude up on a carry, so the stored value is unbiased when
// the operand's top bits are uniform.  The operand of a value comes from a
// hash of its node's column and row, the step counter and the value's index
// among the format's 16-bit rows (FP16S: f rows 0-8, g rows 9-17; FP32 f +
// FP16 g: g rows 0-8), and from nothing else, so every launch configuration,
// graph replays and repeated runs store the same bits.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace lbm {

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
__host__ __device__ inline unsigned rotl(unsigned w, int s) { return s == 0 ? w : (w << s) | (w >> (32 - s)); }
// Random operand i of a node with mixed seed h: word i / 3 rotated left by
// 10 (i % 3) bits, where word 0 is h and word k + 1 the xorshift32 step of
// word k.  The rounding of a value depends on the top bits of its operand;
// the three operands of a word have disjoint top 10-bit fields (bits 31-22,
// 21-12, 11-2 of the word), so the roundings of a node's values are
// independent to 2^-10 of an FP16 unit in the last place.
constexpr int kOperandsPerWord = 3, kOperandShift = 10;
__host__ __device__ inline unsigned operand(unsigned h, int i)
{
    for (int k = 0; k < i / kOperandsPerWord; ++k) h = xorshift(h);
    return rotl(h, kOperandShift * (i % kOperandsPerWord));
}
// random operand i of the node (x, y) (wrapped on a periodic axis) in step t
__host__ __device__ inline unsigned operand_at(int x, int y, unsigned t, int i)
{
    return operand(mix(seed_x(x) ^ seed_yt(y, t)), i);
}
}  // namespace sr

// Host model of v_cvt_sr_f16_f32 for |v| < 65504: the magnitude is cut to
// the FP16 grid (spacing 2^(e - 10) for 2^e <= |v|, 2^-24 below 2^-14) and
// rounded up when the discarded fraction, scaled to 2^32, plus r reaches
// 2^32.  Returns the FP16 value as a double.
inline double round_half_stochastic_model(float v, unsigned r)
{
    const double a = std::fabs(double(v));
    if (a == 0.0) return double(v);
    int e;
    (void)std::frexp(a, &e);           // a = m 2^e, m in [0.5, 1)
    const double spacing = std::ldexp(1.0, std::max(e - 11, -24));
    const double q = a / spacing, lo = std::floor(q);
    const double frac32 = std::floor(std::ldexp(q - lo, 32));   // discarded bits past 32 are dropped
    const double up = frac32 + double(r) >= 4294967296.0 ? 1.0 : 0.0;
    const double res = (lo + up) * spacing;
    return v < 0 ? -res : res;
}

}  // namespace lbm
