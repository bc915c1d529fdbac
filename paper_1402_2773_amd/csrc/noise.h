// noise.h -- the decoder's Gaussian source on gfx950 (device code).
//
// Sec. III-C draws q_k ~ N(0, eta^2 N0/2) independently for every bit and
// round.  The paper leaves the generator open; this library fixes it so
// that any implementation can reproduce the draws bit for bit:
//
//   words  = Philox4x32-10(counter = (k >> 2, t, frame lo, frame hi),
//                          key = (seed lo, seed hi))        [Salmon et al. SC'11]
//   pair p of the quad uses words (2p, 2p+1) = (a, b):
//     u1  = ((a >> 8) + 1) * 2^-24          in (0, 1]
//     phi = 2 pi (b >> 8) 2^-24             in [0, 2 pi)
//     z   = sqrt(-2 ln u1) * (cos phi, sin phi)
//   bit 4j + 2p + 0 takes the cosine branch, 4j + 2p + 1 the sine branch.
//
// ln, sin and cos are fixed binary32 operation sequences (below); sqrt and
// the one division are IEEE correctly rounded (computed by short hardware
// sequences whose results equal IEEE's on every input they receive); every fma
// is explicit and the file is compiled with -ffp-contract=off.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ngdbf {

// Philox-4x32 round multipliers and key (Weyl) increments, as published.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

struct Words4 {
  uint32_t w0, w1, w2, w3;
};

// a ^ b ^ k in one VALU instruction: gfx950's three-input bitwise operation
// with truth table 0x96 (odd parity); k is wave-uniform (a scalar operand)
__device__ __forceinline__ uint32_t xor3_sk(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

// Ten Philox-4x32 rounds.  The key schedule depends only on the seed, so it
// stays in scalar registers when the key is wave-uniform.
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
    const uint32_t n0 = xor3_sk((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3_sk((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return Words4{c0, c1, c2, c3};
}

// The same ten rounds for a counter (j, t, c2, c3) whose c2, c3 and key are
// fixed for a whole frame and whose t is wave-uniform: rounds 0 and 1 and half
// of round 2 then depend on j only through four per-lane words computed once
// per frame (PhiloxLane) and on t only through wave-uniform words computed
// once per round (PhiloxRound).  philox_split(philox_lane(j, ...),
// philox_round(t, ...), ...) equals philox4x32_10(j, t, c2, c3, k0, k1).
struct PhiloxLane {
  uint32_t B;    // c3 after round 0: lo(M0 j)
  uint32_t E;    // c1 after round 1: lo(M1 A), A = hi(M0 j) ^ c3 ^ k1
  uint32_t H0c;  // hi(M0 C) of round 2, C = hi(M1 A) ^ lo(M1 c2) ^ (k0 + W0)
  uint32_t L0c;  // lo(M0 C): c3 after round 2
};
struct PhiloxRound {
  uint32_t dp;  // hi(M0 U) ^ (k1 + W1), U = hi(M1 c2) ^ t ^ k0: with B gives c2 after round 1
  uint32_t vk;  // lo(M0 U) ^ (k1 + 2 W1): with H0c gives c2 after round 2
};

__device__ __forceinline__ PhiloxLane philox_lane(uint32_t j, uint32_t c2, uint32_t c3, uint32_t k0,
                                                  uint32_t k1) {
  const uint64_t p0 = (uint64_t)kPhiloxM0 * j;
  const uint32_t A = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
  const uint64_t p1 = (uint64_t)kPhiloxM1 * A;
  const uint32_t L1a = (uint32_t)((uint64_t)kPhiloxM1 * c2);
  const uint32_t C = (uint32_t)(p1 >> 32) ^ L1a ^ (k0 + kPhiloxW0);
  const uint64_t p2 = (uint64_t)kPhiloxM0 * C;
  return PhiloxLane{(uint32_t)p0, (uint32_t)p1, (uint32_t)(p2 >> 32), (uint32_t)p2};
}

__device__ __forceinline__ PhiloxRound philox_round(uint32_t t, uint32_t c2, uint32_t k0,
                                                    uint32_t k1) {
  const uint32_t U = (uint32_t)(((uint64_t)kPhiloxM1 * c2) >> 32) ^ t ^ k0;
  const uint64_t p = (uint64_t)kPhiloxM0 * U;
  return PhiloxRound{(uint32_t)(p >> 32) ^ (k1 + kPhiloxW1),
                     (uint32_t)p ^ (k1 + 2u * kPhiloxW1)};
}

__device__ __forceinline__ Words4 philox_split(const PhiloxLane &pl, const PhiloxRound &pr,
                                               uint32_t k0, uint32_t k1) {
  // round 2 (rounds 0 and 1 are in pl and pr)
  const uint32_t D = pl.B ^ pr.dp;  // c2 after round 1
  const uint64_t p1 = (uint64_t)kPhiloxM1 * D;
  uint32_t c0 = xor3_sk((uint32_t)(p1 >> 32), pl.E, k0 + 2u * kPhiloxW0);
  uint32_t c1 = (uint32_t)p1;
  uint32_t c2 = pl.H0c ^ pr.vk;
  uint32_t c3 = pl.L0c;
  k0 += 3u * kPhiloxW0;
  k1 += 3u * kPhiloxW1;
#pragma unroll
  for (int r = 3; r < 10; ++r) {
    const uint64_t q0 = (uint64_t)kPhiloxM0 * c0;
    const uint64_t q1 = (uint64_t)kPhiloxM1 * c2;
    const uint32_t n0 = xor3_sk((uint32_t)(q1 >> 32), c1, k0);
    const uint32_t n2 = xor3_sk((uint32_t)(q0 >> 32), c3, k1);
    c1 = (uint32_t)q1;
    c3 = (uint32_t)q0;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return Words4{c0, c1, c2, c3};
}

// binary32 constants, written as exact hex literals
constexpr float kSqrt2 = 0x1.6a09e6p+0f;      // fl(sqrt 2)
constexpr float kTwoLn2 = 0x1.62e430p+0f;     // fl(2 ln 2)
constexpr float kTwoPiM24 = 0x1.921fb6p-22f;  // fl(2 pi) * 2^-24
// 2 atanh(s) = 2 s (1 + s^2/3 + s^4/5 + ... + s^10/11)
constexpr float kA3 = 0x1.555556p-2f, kA5 = 0x1.99999ap-3f, kA7 = 0x1.24924ap-3f,
                kA9 = 0x1.c71c72p-4f, kA11 = 0x1.745d18p-4f;
// sin a = a + a^3 (-1/3! + a^2 (1/5! + a^2 (-1/7! + a^2 / 9!)))
constexpr float kS3 = -0x1.555556p-3f, kS5 = 0x1.111112p-7f, kS7 = -0x1.a01a02p-13f,
                kS9 = 0x1.71de3ap-19f;
// cos a = 1 + a^2 (-1/2! + a^2 (1/4! + a^2 (-1/6! + a^2 (1/8! - a^2/10!))))
constexpr float kC2 = -0.5f, kC4 = 0x1.555556p-5f, kC6 = -0x1.6c16c2p-10f,
                kC8 = 0x1.a01a02p-16f, kC10 = -0x1.27e4fcp-22f;

// (f - 1) / (f + 1) for f in [1/sqrt2, sqrt2), correctly rounded: the
// hardware reciprocal refined once, then one quotient correction by the exact
// fma residual (Markstein).  Its equality with IEEE division for every f the
// radius takes is part of the exhaustive radius comparison over all 2^24 m.
__device__ __forceinline__ float div_near1(float n, float d) {
  const float y0 = __builtin_amdgcn_rcpf(d);
  const float y1 = __builtin_fmaf(__builtin_fmaf(-d, y0, 1.0f), y0, y0);
  const float q0 = n * y1;
  const float r = __builtin_fmaf(-q0, d, n);
  return __builtin_fmaf(r, y1, q0);
}

// sqrt(x) correctly rounded for x = 0 or x in [2^-24, 2^6): the hardware root,
// moved to a neighbour when the exact fma residuals say so.  No scaling is
// needed in this range; checked exhaustively like the division above.
__device__ __forceinline__ float sqrt_radius(float x) {
  const float s = __builtin_amdgcn_sqrtf(x);
  const float sd = __uint_as_float(__float_as_uint(s) - 1u);
  const float su = __uint_as_float(__float_as_uint(s) + 1u);
  const float rd = __builtin_fmaf(-sd, s, x);
  const float ru = __builtin_fmaf(-su, s, x);
  float r = (rd <= 0.0f) ? sd : s;
  r = (ru > 0.0f) ? su : r;
  return r;
}

// Box-Muller radius for u1 = m 2^-24, m in [1, 2^24]:
// m = f 2^e with f in [1/sqrt2, sqrt2); ln u1 = (e - 24) ln 2 + 2 atanh((f-1)/(f+1)).
__device__ __forceinline__ float bm_radius(uint32_t m) {
  int e = 31 - __builtin_clz(m);
  float f = ldexpf((float)m, -e);
  if (f > kSqrt2) {
    f = f * 0.5f;
    e = e + 1;
  }
  const float s = div_near1(f - 1.0f, f + 1.0f);
  const float s2 = s * s;
  float p = __builtin_fmaf(s2, kA11, kA9);
  p = __builtin_fmaf(s2, p, kA7);
  p = __builtin_fmaf(s2, p, kA5);
  p = __builtin_fmaf(s2, p, kA3);
  p = __builtin_fmaf(s2, p, 1.0f);
  const float base = (float)(24 - e) * kTwoLn2;
  return sqrt_radius(__builtin_fmaf(-4.0f * s, p, base));
}

// cos and sin of the angle 2 pi i 2^-24, i in [0, 2^24): exact quadrant and
// octant reduction on the integer, then the series on [0, pi/4].
__device__ __forceinline__ void bm_turn(uint32_t i, float &co, float &si) {
  const uint32_t q = (i >> 22) & 3u;
  const uint32_t r = i & 0x3FFFFFu;
  const bool refl = r > 0x200000u;
  const uint32_t rr = refl ? (0x400000u - r) : r;
  const float a = (float)rr * kTwoPiM24;
  const float a2 = a * a;
  float ps = __builtin_fmaf(a2, kS9, kS7);
  ps = __builtin_fmaf(a2, ps, kS5);
  ps = __builtin_fmaf(a2, ps, kS3);
  float sn = __builtin_fmaf(a * a2, ps, a);
  float pc = __builtin_fmaf(a2, kC10, kC8);
  pc = __builtin_fmaf(a2, pc, kC6);
  pc = __builtin_fmaf(a2, pc, kC4);
  pc = __builtin_fmaf(a2, pc, kC2);
  float cs = __builtin_fmaf(a2, pc, 1.0f);
  if (refl) {
    const float t = sn;
    sn = cs;
    cs = t;
  }
  // quarter turns: (c, s) -> (-s, c)
  const bool swap = (q & 1u) != 0;
  const float c1 = swap ? sn : cs;
  const float s1 = swap ? cs : sn;
  co = (q == 1u || q == 2u) ? -c1 : c1;
  si = (q >= 2u) ? -s1 : s1;
}

__device__ __forceinline__ void bm_pair(uint32_t a, uint32_t b, float &z0, float &z1) {
  const float rho = bm_radius((a >> 8) + 1u);
  float c, s;
  bm_turn(b >> 8, c, s);
  z0 = rho * c;
  z1 = rho * s;
}

// The four draws of bit quad j (bits 4j .. 4j+3) of a frame at round t.
struct Draw4 {
  float z[4];
};

__device__ __forceinline__ Draw4 draw_quad(uint32_t j, uint32_t t, uint64_t frame,
                                           uint32_t k0, uint32_t k1) {
  const Words4 w = philox4x32_10(j, t, (uint32_t)frame, (uint32_t)(frame >> 32), k0, k1);
  Draw4 d;
  bm_pair(w.w0, w.w1, d.z[0], d.z[1]);
  bm_pair(w.w2, w.w3, d.z[2], d.z[3]);
  return d;
}

}  // namespace ngdbf
